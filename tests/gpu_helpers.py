"""Shared helpers of the GPU tests (comparison metrics and runners)."""
import numpy as np

import oracle as O
from paper_1904_00861_amd import dtsph as D


def rel_l2(a, b, floor=0.0):
    """||a - b|| / max(||b||, floor)."""
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b))) / max(nb, floor, 1e-300)


class Bars:
    """Collects field comparisons of one test, prints every measured error (so a
    run's log states the per-field errors) and fails at the end with all
    comparisons that exceeded their bars."""

    def __init__(self, case: str):
        self.case = case
        self.fails = []

    def rel(self, field, got, ref, bar, floor=0.0):
        e = rel_l2(got, ref, floor)
        self._book(field, "rel L2", e, bar)
        return e

    def absmax(self, field, got, ref, bar):
        e = float(np.abs(np.asarray(got) - np.asarray(ref)).max()) if np.size(ref) else 0.0
        self._book(field, "max abs", e, bar)
        return e

    def _book(self, field, kind, e, bar):
        print(f"[gpu-err] {self.case} {field} {kind} {e:.3e} bar {bar:.1e}", flush=True)
        if not e <= bar:
            self.fails.append(f"{field} {kind} {e:.3e} > {bar:.1e}")

    def done(self):
        assert not self.fails, f"{self.case}: " + "; ".join(self.fails)


def oracle_steps(prob, n_steps, fixed_iters=0):
    return O.step(prob.params, prob.n_fluid, prob.n_wall, prob.x, prob.v, prob.v_prev, prob.p,
                  n_steps, fixed_iters)


def oracle_steps_at(prob, iters):
    """Oracle real steps, step s running exactly iters[s] pseudo-iterations: the
    reference for a free-running GPU run whose per-step counts may differ from the
    oracle's own by one (float32 residuals near the tolerance)."""
    x, v, vp, p = prob.x, prob.v, prob.v_prev, prob.p
    reps = []
    for k in iters:
        x, v, vp, p, r, st = O.step(prob.params, prob.n_fluid, prob.n_wall, x, v, vp, p, 1, int(k))
        reps += r
    return x, v, vp, p, reps


def gpu_steps(prob, n_steps, precision):
    sim = D.Sim(prob, precision=precision)
    try:
        st, reps = sim.step(n_steps)
        return sim.get_state(), reps, st
    finally:
        sim.close()


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)
