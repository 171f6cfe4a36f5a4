"""The entry point that allocates nothing (dtsph_create_static): a context whose
device arrays live in the library's static scratch gives the same results as a
dtsph_create context, bit for bit, on two static contexts in a row (the second
smaller, on scratch that still holds the first one's data); a second static
context while one lives is refused, a context larger than the scratch is
refused, and so are the options that would allocate."""
import numpy as np
import pytest

from paper_1904_00861_amd import dtsph as D
from paper_1904_00861_amd import inputs as I

from gpu_helpers import banner

pytestmark = pytest.mark.gpu

PREC = {"fp64": D.FP64, "fp32": D.FP32}


def _run(prob, prec, static, steps):
    sim = D.Sim(prob, precision=PREC[prec], static=static)
    try:
        st, reps = sim.step(steps)
        return sim.get_state(), reps, st
    finally:
        sim.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_static_context_matches_regular_two_calls(prec):
    # first a 40 x 40 vortex with shifting, then a smaller walled cavity
    first = I.tgv2d(40, seed=3)
    first.params = dict(first.params, shift=1)
    for prob, steps in ((first, 4), (I.cavity(14), 3)):
        banner(f"static context {prob.name} n={prob.n} {prec}")
        g_ref, r_ref, st_ref = _run(prob, prec, False, steps)
        g, r, st = _run(prob, prec, True, steps)
        assert st == st_ref
        assert r == r_ref
        for k in g_ref:
            assert np.array_equal(g[k], g_ref[k]), (prob.name, k)


def test_static_context_limits():
    banner("static context limits")
    a = D.Sim(I.tgv2d(20, seed=1), precision=D.FP32, static=True)
    try:
        with pytest.raises(D.DtsphError) as e:  # one static context per GPU
            D.Sim(I.tgv2d(16, seed=2), precision=D.FP32, static=True)
        assert e.value.status == D.EINVAL
        for opt in (D.OPT_PAIR_CACHE, D.OPT_GRAPHS, D.OPT_TIMING):
            with pytest.raises(D.DtsphError) as e:
                a.set_option(opt, 1)
            assert e.value.status == D.EINVAL
        with pytest.raises(D.DtsphError):
            a.autotune()
        a.step(1)  # still usable
    finally:
        a.close()
    # the scratch is free again, but too small for C1's 160k particles
    with pytest.raises(D.DtsphError) as e:
        D.Sim(I.config("C1"), precision=D.FP64, static=True)
    assert e.value.status == D.ENOMEM
    b = D.Sim(I.tgv2d(12, seed=4), precision=D.FP64, static=True)  # released after the failure
    b.step(1)
    b.close()
