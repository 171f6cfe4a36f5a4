"""GPU parity of the steady-state solve (sections 2.3 and 3.3) against the
oracle: segments of fixed iteration counts and free-running segments with the
stop test, on channel, cavity and periodic vortex cases in 2D and 3D; the
Poiseuille profile reached on the GPU; fixed particles and exact lists;
steady and time-accurate sims sharing one context."""
import numpy as np
import pytest

import oracle as O
from paper_1904_00861_amd import dtsph as D
from paper_1904_00861_amd import inputs as I

from gpu_helpers import Bars, banner, oracle_steps, oracle_steps_at, rel_l2

pytestmark = pytest.mark.gpu

PREC = {"fp64": D.FP64, "fp32": D.FP32}
# FP32 sums on a contracting iteration: the error settles at the size of one
# iteration's rounding relative to the field, it does not accumulate
TOL = {"fp64": dict(v=1e-10, p=1e-11), "fp32": dict(v=1e-5, p=1e-4)}


def _steady(prob):
    prob = prob.copy()
    prob.params = dict(prob.params, steady=1)
    return prob


CASES = {
    "poiseuille_10": lambda: I.poiseuille(ny=10),
    "cavity_steady_16": lambda: I.cavity(16, steady=True),
    "tgv2d_steady_24": lambda: _steady(I.tgv2d(24, seed=3)),
    "tgv3d_steady_8": lambda: _steady(I.tgv3d(8, seed=4)),
}


def gpu_fixed_segments(prob, n_seg, iters, precision):
    sim = D.Sim(prob, precision=precision)
    try:
        reps = []
        for _ in range(n_seg):
            sim.predict()
            reps.append(sim.pseudo_iterate(iters)[1])
            sim.correct()
        return sim.get_state(), reps
    finally:
        sim.close()


def p_floor(prm, nf):
    """Pressure scale rho c V_ref (per particle, L2) for the channel, whose pressure
    vanishes identically (it is zero up to round-off); other cases compare p
    on its own norm."""
    if prm["periodic"][0] and not prm["periodic"][1] and prm["g"][0] != 0.0:
        return prm["rho0"] * prm["beta"] * prm["vref"] ** 2 * np.sqrt(nf)
    return 0.0


def _compare(g, x, v, vp, p, nf, t, what, prm):
    assert np.array_equal(g["x"], x), f"{what}: particles moved"
    b = Bars(what)
    b.rel("V", g["v"][:nf], v[:nf], t["v"])
    b.rel("V_prev", g["v_prev"][:nf], vp[:nf], t["v"])
    b.rel("p", g["p"][:nf], p[:nf], t["p"], p_floor(prm, nf))
    b.done()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case,n_seg,iters", [("poiseuille_10", 3, 40), ("cavity_steady_16", 2, 50),
                                              ("tgv2d_steady_24", 2, 30), ("tgv3d_steady_8", 2, 10)])
def test_fixed_segments_match_oracle(case, n_seg, iters, prec):
    prob = CASES[case]()
    banner(f"steady segments {case} {n_seg}x{iters} {prec}")
    nf = prob.n_fluid
    x, v, vp, p, oreps, _ = oracle_steps(prob, n_seg, iters)
    g, greps = gpu_fixed_segments(prob, n_seg, iters, PREC[prec])
    assert [r[0]["iters"] for r in greps] == [r["iters"] for r in oreps]
    assert [r[0]["pairs"] for r in greps] == [r["pairs"] for r in oreps]
    _compare(g, x, v, vp, p, nf, TOL[prec], f"steady {case} {n_seg}x{iters} {prec}", prob.params)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_free_running_segments_match_oracle(prec):
    prob = CASES["cavity_steady_16"]()
    prob.params = dict(prob.params, tol=1e-3)
    banner(f"steady free-running cavity_steady_16 {prec}")
    nf = prob.n_fluid
    _, _, _, _, oreps, _ = oracle_steps(prob, 4)
    sim = D.Sim(prob, precision=PREC[prec])
    st, greps = sim.step(4)
    g = sim.get_state()
    sim.close()
    gi, oi = [r[0]["iters"] for r in greps], [r["iters"] for r in oreps]
    if prec == "fp64":
        assert gi == oi
    else:  # a stop decision may move by one iteration in FP32
        assert all(abs(a - b) <= 1 for a, b in zip(gi, oi))
    x, v, vp, p, _ = oracle_steps_at(prob, gi)
    _compare(g, x, v, vp, p, nf, TOL[prec], f"steady free running {prec} iters {gi} oracle {oi}", prob.params)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_poiseuille_profile_on_gpu(prec):
    prob = CASES["poiseuille_10"]()
    banner(f"steady Poiseuille profile {prec}")
    nf = prob.n_fluid
    g, _ = gpu_fixed_segments(prob, 1, 3000, PREC[prec])
    y, u = g["x"][:nf, 1], g["v"][:nf, 0]
    exact = prob.params["g"][0] * y * (1.0 - y) / (2.0 * prob.params["nu"])
    assert np.abs(u - exact).max() / exact.max() < 0.03  # the oracle's first-order wall error
    assert np.abs(g["v"][:nf, 1]).max() < (1e-12 if prec == "fp64" else 1e-5)


def test_lists_stay_exact_and_particles_fixed():
    prob = CASES["cavity_steady_16"]()
    banner("steady lists and positions")
    sim = D.Sim(prob, precision=D.FP64)
    sim.step(3)
    g = sim.get_state()
    off, idx = sim.neighbor_list()
    sim.close()
    assert np.array_equal(g["x"], prob.x)
    ob, ib = O.neighbors(prob.params, prob.n_fluid, prob.n_wall, prob.x, "brute")
    assert np.array_equal(off, ob) and np.array_equal(idx, ib)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_steady_and_time_accurate_sims_share_a_context(prec):
    probs = [CASES["cavity_steady_16"](), I.tgv2d(20, seed=8), I.cavity(12), CASES["poiseuille_10"]()]
    banner(f"mixed steady / time-accurate batch {prec}")
    sim = D.Sim(probs, precision=PREC[prec])
    reps = []
    for _ in range(2):
        sim.predict()
        reps.append(sim.pseudo_iterate(6)[1])
        sim.correct()
    gb = sim.get_state()
    sl = sim.sim_slices()
    sim.close()
    t = TOL[prec]
    for s, prob in enumerate(probs):
        x, v, vp, p, oreps, _ = oracle_steps(prob, 2, 6)
        nf = prob.n_fluid
        sub = {k: gb[k][sl[s]] for k in gb}
        if prob.params["steady"]:
            assert np.array_equal(sub["x"], prob.x)
        else:
            assert np.abs(sub["x"] - x).max() <= (1e-12 if prec == "fp64" else 1e-7)
        b = Bars(f"mixed batch member {s} {prec}")
        b.rel("V", sub["v"][:nf], v[:nf], t["v"])
        b.rel("p", sub["p"][:nf], p[:nf], t["p"], p_floor(prob.params, nf))
        b.done()
        if prec == "fp64" or prob.params["steady"]:
            # FP32 predicted positions of a moving sim may put a pair on the other
            # side of the support radius than FP64 ones do
            assert [r[s]["pairs"] for r in reps] == [r["pairs"] for r in oreps]


def test_steady_rejects_shifting():
    prob = CASES["cavity_steady_16"]()
    prob.params = dict(prob.params, shift=1)
    banner("steady with shifting is rejected")
    with pytest.raises(D.DtsphError):
        D.Sim(prob, precision=D.FP64)
