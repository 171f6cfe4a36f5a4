"""Every lanes-per-particle count of the pair pass (the autotuner may pick any):
one real step at a fixed iteration count matches the oracle for each pass
variant the workloads use — 2D and 3D periodic, walls with and without
artificial viscosity, the steady solve (convective sum) and particles moving in
pseudo-time — in FP64 and FP32, with the bars of the step tests. The lanes of
a particle take entries sub, sub + L, ... and combine their sums by butterfly
shuffles, so every L sums in its own order (within rounding of the others)."""
import numpy as np
import pytest

from paper_1904_00861_amd import dtsph as D
from paper_1904_00861_amd import inputs as I

from gpu_helpers import Bars, banner, oracle_steps, rel_l2

pytestmark = pytest.mark.gpu

PREC = {"fp64": D.FP64, "fp32": D.FP32}
TOL = {"fp64": dict(v=1e-10, p=1e-11, x=1e-12), "fp32": dict(v=1e-5, p=1e-4, x=1e-7)}


def _with(prob, **kw):
    prob = prob.copy()
    prob.params = dict(prob.params, **kw)
    return prob


CASES = {
    "tgv2d_30": lambda: I.tgv2d(30, seed=5),
    "tgv3d_8": lambda: I.tgv3d(8, seed=3),
    "dam_0.05": lambda: I.dam_break(0.05),
    "cavity_16": lambda: I.cavity(16),
    "cavity_steady_16": lambda: I.cavity(16, steady=True),
    "tgv2d_24_move": lambda: _with(I.tgv2d(24, seed=6), move=1),
}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("lanes", [1, 2, 4, 8])
@pytest.mark.parametrize("case", list(CASES))
def test_pass_lanes_match_oracle(case, lanes, prec):
    prob = CASES[case]()
    fixed = 5
    banner(f"pair pass lanes {lanes} {case} {prec}, 1 step of {fixed} iterations")
    nf = prob.n_fluid
    sim = D.Sim(prob, precision=PREC[prec])
    try:
        sim.set_option(D.OPT_LANES, lanes)
        sim.predict()
        _, reps = sim.pseudo_iterate(fixed)
        sim.correct()
        g = sim.get_state()
    finally:
        sim.close()
    x, v, vp, p, oreps, _ = oracle_steps(prob, 1, fixed)
    assert reps[0]["iters"] == oreps[0]["iters"] == fixed
    t = TOL[prec]
    # the dam break's momentum right side is a cancellation of grad p / rho and g:
    # its velocity is compared on the |g| dt scale of those terms (zero without g)
    vfl = float(np.linalg.norm(prob.params["g"])) * prob.params["dt"] * np.sqrt(nf)
    b = Bars(f"pass lanes {lanes} {case} {prec}")
    b.absmax("x", g["x"], x, t["x"])
    b.rel("V", g["v"][:nf], v[:nf], t["v"], vfl)
    b.rel("p", g["p"][:nf], p[:nf], t["p"])
    b.done()
    if prob.params["steady"]:
        assert np.array_equal(g["x"], prob.x)
