"""Shared helpers of the GPU tests (comparison metrics and runners)."""
import numpy as np

import oracle as O
from paper_1904_00861_amd import dtsph as D


def rel_l2(a, b, floor=0.0):
    """||a - b|| / max(||b||, floor)."""
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b))) / max(nb, floor, 1e-300)


def rate_floor(prob):
    """L2 scale of a pressure rate: rho c^2 V_ref / h per particle (the size of one
    divergence term), so that a field that vanishes by symmetry is compared on
    the scale of its terms rather than on its round-off."""
    p = prob.params
    c = p["beta"] * p["vref"]
    return p["rho0"] * c * c * p["vref"] / p["h"] * np.sqrt(prob.n_fluid)


def oracle_steps(prob, n_steps, fixed_iters=0):
    return O.step(prob.params, prob.n_fluid, prob.n_wall, prob.x, prob.v, prob.v_prev, prob.p,
                  n_steps, fixed_iters)


def gpu_steps(prob, n_steps, precision):
    sim = D.Sim(prob, precision=precision)
    try:
        st, reps = sim.step(n_steps)
        return sim.get_state(), reps, st
    finally:
        sim.close()


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)
