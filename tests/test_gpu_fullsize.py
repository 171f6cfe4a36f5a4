"""Full-size workloads (C1 2D TGV 400^2, C2 3D TGV 64^3, C3 dam break ~518k, C4
batch of 64 sims, 2.57M particles) in the benchmark's launch configuration
(FP32 sums, autotuned shape, XCD-aware tile order):

* neighbour lists bit-exact against the oracle's binned search, every particle
  of every config (each C4 sim against its own oracle lists), from the
  autotuned kernel and from the staged-tile kernel of the 2D configs;
* one real step at a fixed count of 4 pseudo-iterations over the whole
  workload, FP32 and FP64, every particle against the oracle's step (each C4
  sim against its own oracle run);
* outputs at sampled particles of the predictor and of one pseudo-iteration
  from a perturbed in-loop state, against the oracle evaluated row by row.

Bars (relative L2, every measured value printed): FP64 step V, p <= 1e-11,
positions <= 1e-12; FP32 step V <= 1e-5, p <= 1e-4, positions <= 1e-7; sampled
rows V <= 1e-6, p <= 1e-5, except the dam break's predicted velocity (a
hydrostatic cancellation of grad p / rho and g, compared on the |g| dt scale of
those terms: 1.5e-4); the FP32 pressure rate <= 1e-4 for the 3D vortex and
1e-3 for the 2D workloads, whose finer resolution leaves a nearly solenoidal
velocity field: its divergence sum cancels to ~1e-3 of its terms, and float32
rounding of the terms appears magnified (measured 1.8e-4 C1, 3.3e-4 C3, 2.5e-4
C4, 1.8e-5 C2)."""
import numpy as np
import pytest

import oracle as O
from paper_1904_00861_amd import dtsph as D
from paper_1904_00861_amd import inputs as I

from gpu_helpers import Bars, banner, oracle_steps, rel_l2

pytestmark = pytest.mark.gpu

PREC = {"fp64": D.FP64, "fp32": D.FP32}
TOL_STEP = {"fp64": dict(v=1e-11, p=1e-11, x=1e-12), "fp32": dict(v=1e-5, p=1e-4, x=1e-7)}
DTAU_ROWS = {"C1": 1e-3, "C2": 1e-4, "C3": 1e-3, "C4": 1e-3}
V0_ROWS = {"C1": 1e-6, "C2": 1e-6, "C3": 1.5e-4}
FIXED = 4


def _rows(prob, k=48, seed=0):
    nf = prob.n_fluid
    rng = np.random.default_rng(seed)
    r = np.unique(np.concatenate([np.linspace(0, nf - 1, k // 2).astype(int),
                                  rng.integers(0, nf, k // 2), [0, nf - 1]]))
    return r


def v_floor(prm, n):
    """|g| dt per particle (L2): with gravity the momentum rate is the small
    difference of grad p / rho and g, terms of size |g| each; 0 without it."""
    return float(np.linalg.norm(prm["g"])) * prm["dt"] * np.sqrt(n)


def _problems(cfg):
    prob = I.config(cfg)
    return prob if isinstance(prob, list) else [prob]


_ORACLE = {}


def _oracle_step(cfg, s, prob):
    key = (cfg, s)
    if key not in _ORACLE:
        x, v, vp, p, reps, st = oracle_steps(prob, 1, FIXED)
        _ORACLE[key] = (x, v, vp, p, reps)
    return _ORACLE[key]


def _pair_band(prob, rel):
    """Fluid-row pair counts at the oracle's predicted positions r^(0) with the
    support radius scaled by (1 - rel) and (1 + rel): the lists of any r^(0)
    within rounding of the oracle's lie between the two (pairs at exactly kappa h,
    where W and grad W vanish, may fall on either side)."""
    pr = O.predict(prob.params, prob.n_fluid, prob.n_wall, prob.x, prob.v, prob.p)
    out = []
    for f in (1.0 - rel, 1.0 + rel):
        prm = dict(prob.params, kappa=prob.params["kappa"] * f)
        off, _ = O.neighbors(prm, prob.n_fluid, prob.n_wall, pr["x_iter"], "bins")
        out.append(int(off[prob.n_fluid]))
    return out


_LISTS = {}


def _oracle_lists(cfg, s, prob):
    if (cfg, s) not in _LISTS:
        _LISTS[(cfg, s)] = O.neighbors(prob.params, prob.n_fluid, prob.n_wall, prob.x, "bins")
    return _LISTS[(cfg, s)]


@pytest.mark.parametrize("cfg", ["C1", "C2", "C3", "C4"])
def test_fullsize_neighbour_lists_match_binned_oracle(cfg):
    probs = _problems(cfg)
    banner(f"full-size neighbour lists {cfg}: {len(probs)} sims, {sum(p.n for p in probs)} particles")
    sim = D.Sim(probs, precision=D.FP32)
    sim.autotune()
    for s, prob in enumerate(probs):
        off, idx = sim.neighbor_list(s)
        ob, ib = _oracle_lists(cfg, s, prob)
        assert np.array_equal(off, ob) and np.array_equal(idx, ib), (cfg, s)
    sim.close()


@pytest.mark.parametrize("div", [2, 3])
@pytest.mark.parametrize("cfg", ["C1", "C3", "C4"])
def test_fullsize_staged_tile_lists_match_binned_oracle(cfg, div):
    # the staged-tile kernel (2D) at full size, whichever kernel the autotuner
    # would pick
    probs = _problems(cfg)
    banner(f"full-size staged-tile neighbour lists {cfg} cell subdivision {div}")
    sim = D.Sim(probs, precision=D.FP32)
    sim.set_option(D.OPT_CELL_DIV, div)
    sim.set_option(D.OPT_NBR_TILES, 1)
    for s, prob in enumerate(probs):
        off, idx = sim.neighbor_list(s)
        ob, ib = _oracle_lists(cfg, s, prob)
        assert np.array_equal(off, ob) and np.array_equal(idx, ib), (cfg, s)
    sim.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("cfg", ["C2", "C3", "C4"])
def test_fullsize_step_fixed_iterations(cfg, prec):
    probs = _problems(cfg)
    banner(f"full-size step {cfg} {prec}: 1 step of {FIXED} iterations, "
           f"{len(probs)} sims, {sum(p.n for p in probs)} particles")
    sim = D.Sim(probs, precision=PREC[prec])
    sim.autotune()
    sim.predict()
    st, reps = sim.pseudo_iterate(FIXED)
    sim.correct()
    g = sim.get_state()
    sl = sim.sim_slices()
    sim.close()
    t = TOL_STEP[prec]
    b = Bars(f"full-size step {cfg} {prec}")
    for s, prob in enumerate(probs):
        x, v, vp, p, oreps = _oracle_step(cfg, s, prob)
        nf = prob.n_fluid
        sub = {k: g[k][sl[s]] for k in g}
        assert reps[s]["iters"] == FIXED
        # the lists at r^(0) are each side's exact lists at its own predicted
        # positions, which differ by rounding: on perfect lattices (cavity, dam
        # break) many pairs sit exactly at kappa h and may fall on either side
        if reps[s]["pairs"] != oreps[0]["pairs"]:
            lo, hi = _pair_band(prob, 1e-12 if prec == "fp64" else 1e-6)
            print(f"[gpu-err] {cfg} {prec} sim{s} pairs gpu {reps[s]['pairs']} oracle {oreps[0]['pairs']} "
                  f"band [{lo}, {hi}]", flush=True)
            assert lo <= reps[s]["pairs"] <= hi, (cfg, prec, s)
        tag = f"sim{s} " if len(probs) > 1 else ""
        b.absmax(tag + "x", sub["x"], x, t["x"])
        b.rel(tag + "V", sub["v"][:nf], v[:nf], t["v"], v_floor(prob.params, nf))
        b.rel(tag + "V_prev", sub["v_prev"][:nf], vp[:nf], t["v"], v_floor(prob.params, nf))
        b.rel(tag + "p", sub["p"][:nf], p[:nf], t["p"])
    b.done()


@pytest.mark.parametrize("cfg", ["C1", "C2", "C3"])
def test_fullsize_predict_sampled(cfg):
    prob = I.config(cfg)
    banner(f"full-size predict {cfg} n={prob.n}")
    nf, nw = prob.n_fluid, prob.n_wall
    sim = D.Sim(prob, precision=D.FP32)
    sim.autotune()
    sim.predict()
    g = sim.get_state(loop=True)
    sim.close()
    rows = _rows(prob)
    vo, po, do = O.rows(prob.params, nf, nw, 0, rows, prob.x, prob.v, prob.p)
    b = Bars(f"full-size predict {cfg}")
    b.rel("V(0)", g["v_iter"][rows], vo, V0_ROWS[cfg], v_floor(prob.params, len(rows)))
    b.rel("dp/dtau", g["dpdtau"][rows], do, DTAU_ROWS[cfg])
    b.done()
    if nw == 0 and not any(prob.params["g"]):
        # periodic, no body force: pairwise antisymmetry conserves momentum
        dv = g["v_iter"][:nf] - prob.v[:nf]
        assert np.abs(dv.sum(axis=0)).max() <= 1e-5 * np.abs(dv).sum()


@pytest.mark.parametrize("cfg", ["C1", "C2", "C3"])
def test_fullsize_first_iteration_sampled(cfg):
    prob = I.config(cfg)
    banner(f"full-size first pseudo-iteration {cfg}")
    nf, nw = prob.n_fluid, prob.n_wall
    ls = I.loop_state_from(prob)
    sim = D.Sim(prob, precision=D.FP32)
    sim.autotune()
    sim.set_state_from_problems(loop=ls)
    st, reps = sim.pseudo_iterate(1)
    g = sim.get_state(loop=True)
    sim.close()
    rows = _rows(prob, seed=1)
    vo, po, do = O.rows(prob.params, nf, nw, 1, rows, ls["x_iter"], ls["v_iter"], ls["p_iter"],
                        ls["dpdtau"], prob.v, prob.v_prev)
    b = Bars(f"full-size first iteration {cfg}")
    b.rel("V1", g["v_iter"][rows], vo, 1e-6)
    b.rel("p1", g["p_iter"][rows], po, 1e-5)
    b.rel("dp/dtau", g["dpdtau"][rows], do, DTAU_ROWS[cfg])
    b.done()
    assert reps[0]["iters"] == 1


def test_fullsize_batch_sampled():
    probs = I.config("C4")
    banner(f"full-size batch of {len(probs)}: predictor at sampled rows of every 8th sim")
    sim = D.Sim(probs, precision=D.FP32)
    sim.autotune()
    sim.predict()
    g = sim.get_state(loop=True)
    sl = sim.sim_slices()
    sim.close()
    b = Bars("full-size batch predict")
    for s, prob in enumerate(probs):
        if s % 8:
            continue
        rows = _rows(prob, k=16, seed=s)
        vo, po, do = O.rows(prob.params, prob.n_fluid, prob.n_wall, 0, rows, prob.x, prob.v, prob.p)
        b.rel(f"sim{s} V(0)", g["v_iter"][sl[s]][rows], vo, 1e-6)
        b.rel(f"sim{s} dp/dtau", g["dpdtau"][sl[s]][rows], do, DTAU_ROWS["C4"])
    b.done()
