"""The speculative end of step (DTSPH_OPT_SPECULATE): dtsph_step with the
corrector and the next rate pass queued behind the device gate gives the same
bits as without, whether the gate opens (converged sims, valid candidate
lists) or stays closed (tiny skin, loops needing more chunks), for single
sims, batches, steady, moving and shifting sims, with timing on."""
import numpy as np
import pytest

from paper_1904_00861_amd import dtsph as D
from paper_1904_00861_amd import inputs as I

from gpu_helpers import banner

pytestmark = pytest.mark.gpu


def _with(prob, **kw):
    prob = prob.copy()
    prob.params = dict(prob.params, **kw)
    return prob


CASES = {
    "tgv2d_30": lambda: I.tgv2d(30, seed=5),
    "batch_4": lambda: [I.tgv2d(20, seed=1), I.cavity(14), I.tgv2d(26, seed=2), I.cavity(10)],
    "cavity_steady_16": lambda: I.cavity(16, steady=True),
    "tgv2d_30_move2": lambda: _with(I.tgv2d(30, seed=7), move=2),
    "dam_0.05": lambda: I.dam_break(0.05),
    "tgv3d_8": lambda: I.tgv3d(8, seed=3),
    "tgv2d_30_shift": lambda: _with(I.tgv2d(30, seed=6, jitter=0.1), shift=1),
    "dam_0.05_shift": lambda: _with(I.dam_break(0.05), shift=1),
}


def run(prob, prec, spec, steps, opts=None):
    sim = D.Sim(prob, precision=prec)
    try:
        sim.set_option(D.OPT_SPECULATE, spec)
        for k, v in (opts or {}).items():
            sim.set_option(k, v)
        st, reps = sim.step(steps)
        st2, reps2 = sim.step(2)  # a second call starts from a booked state
        return sim.get_state(), reps + reps2, st
    finally:
        sim.close()


@pytest.mark.parametrize("prec", [D.FP32, D.FP64])
@pytest.mark.parametrize("case", list(CASES))
def test_speculation_gives_the_same_bits(case, prec):
    banner(f"speculative end of step {case} precision {prec}")
    a, ra, sa = run(CASES[case](), prec, 1, 6)
    b, rb, sb = run(CASES[case](), prec, 0, 6)
    assert sa == sb and ra == rb
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_closed_gate_and_timing():
    banner("speculation with a tiny skin (gate closed) and sampled timing")
    prob = CASES["batch_4"]()
    a, ra, _ = run(prob, D.FP32, 1, 5, {D.OPT_SKIN: 1, D.OPT_TIMING: 2})
    b, rb, _ = run(prob, D.FP32, 0, 5, {D.OPT_SKIN: 1, D.OPT_TIMING: 2})
    assert ra == rb
    for k in a:
        assert np.array_equal(a[k], b[k]), k
