"""Pins of the oracle's pseudo-time loop control and pressure integrator.

Parts pinned here, each against a closed form derived from the paper's
statements rather than against the oracle's own code:

* the stop test (section 3.4: eq. conv and the stall rule after it) on
  hand-made residual histories with known outcomes: below tolerance, a spread
  under 5% over the last four values (relative to their maximum), the iteration
  cap, non-finite values, the max norm;
* the stop reason and iteration count of free-running loops whose residual
  series are geometric in closed form (isolated particles, section 3.4's
  analysis of the frozen update, eq. dv_dtau_exact): stalls at exactly the
  window length when the spread 1 - rho^3 is under 5%, never when it is over,
  the cap when it is lower;
* the max norm on two isolated particles with different initial errors;
* the two pressure half steps of eqs. pkstar_frozen and pkp1_frozen and the
  residual scale dt / (rho c^2) of eq. conv: on a perfect periodic lattice a
  Fourier mode of p is an eigenvector of the EDAC diffusion sum
  (eq. dp-dtau-frozen-edac), with an eigenvalue computed here from the kernel
  by a lattice sum, so p after K iterations and the residuals follow in closed
  form. A full step instead of two half steps, a stage 1 that ignores the stored
  rate, or a residual without the 1/rho or the dt fails these.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1904_00861_amd import inputs as I


def _prm(**kw):
    p = dict(I.BASE_PARAMS)
    p.update(dim=2, h=0.01, mass=1e-4, dt=0.0025, lo=(0, 0, 0), hi=(1, 1, 1), periodic=(0, 0, 0))
    p.update(kw)
    return p


# ----------------------------------------------------------------------------- stop test

def test_stop_rule_on_given_histories():
    prm = _prm(tol=1e-3, stall_window=4, stall_rel=0.05, max_iter=1000)
    st = lambda rp, rv, **kw: O.stop_test(dict(prm, **kw), rp, rv)
    # below the tolerance in both series after one iteration: converged
    assert st([5e-4], [9e-4]) == "converged"
    # one series above: continue
    assert st([2e-3], [5e-4]) == "continue"
    assert st([5e-4], [1e-3]) == "continue"  # strict "<"
    # non-finite
    assert st([float("nan")], [1.0]) == "nonfinite"
    assert st([1.0], [float("inf")]) == "nonfinite"
    # pressure stalled (spread 0.03 of the max over the last four), velocity below
    assert st([1.0, 0.99, 0.98, 0.97], [1e-4] * 4) == "stalled"
    # both stalled
    assert st([1.0, 0.99, 0.98, 0.97], [2.0, 1.99, 1.98, 1.97]) == "stalled"
    # only three values: the window of four is not full yet
    assert st([1.0, 0.999, 0.998], [1e-4] * 3) == "continue"
    # the last four values count, not the first four
    assert st([10.0, 1.0, 0.99, 0.98, 0.97], [1e-4] * 5) == "stalled"
    assert st([1.0, 0.99, 0.98, 0.97, 0.5], [1e-4] * 5) == "continue"
    # 5% threshold, relative to the maximum of the window: spread 0.048 of 1.0 is
    # under 5% (it would be 5.04% of the minimum 0.952)
    assert st([1.0, 0.952, 0.952, 0.952], [1e-4] * 4) == "stalled"
    assert st([1.0, 0.94, 0.96, 0.97], [1e-4] * 4) == "continue"
    # a stalled pressure does not stop the loop while the velocity still moves
    assert st([1.0, 0.99, 0.98, 0.97], [1.0, 0.5, 0.25, 0.125]) == "continue"
    # window length and threshold are parameters
    assert st([1.0, 0.99, 0.98], [1e-4] * 3, stall_window=3) == "stalled"
    assert st([1.0, 0.97, 0.96, 0.955], [1e-4] * 4, stall_rel=0.04) == "continue"
    assert st([1.0, 0.99, 0.98, 0.97], [1e-4] * 4, stall_window=0) == "continue"
    # the iteration cap
    h = [1.0, 0.5, 0.25, 0.125, 0.0625]
    assert st(h[:4], h[:4], max_iter=5) == "continue"
    assert st(h, h, max_iter=5) == "max_iter"
    # settled at the cap: the settled reason is reported
    assert st([1e-4] * 5, [1e-4] * 5, max_iter=5) == "converged"


# ----------------------------------------------------------------------------- isolated particles

def _isolated_run(beta, vref=2.5, **kw):
    """One particle with no neighbours: D = 0 and R = g, so V^k approaches
    V* = (4V^n - V^{n-1} + 2 dt g)/3 with the error ratio rho = 2 dt/(2 dt + 3 dtau)
    = 2 beta/(2 beta + 3) per iteration; |Vtilde^k| = beta (1 - rho) rho^(k-1) |e0|."""
    prm = _prm(beta=beta, vref=vref, g=(0.0, -2.0, 0.0), **kw)
    x = np.array([[0.5, 0.5, 0.0]])
    vn = np.array([[0.3, -0.1, 0.0]])
    vnm1 = np.array([[0.25, 0.05, 0.0]])
    v0 = vn + prm["dt"] * np.array(prm["g"])
    vk, pk, dk, rep = O.pseudo_loop(prm, 1, 0, x, vn, vnm1, v0, np.array([0.7]), np.array([0.0]))
    vstar = (4 * vn - vnm1 + 2 * prm["dt"] * np.array(prm["g"])) / 3.0
    e0 = np.linalg.norm(v0 - vstar)
    rho = 2.0 * beta / (2.0 * beta + 3.0)
    return rep, e0, rho, prm


def test_isolated_particle_stalls_at_the_window_length():
    # beta = 100: rho = 200/203, the spread of four consecutive values of a
    # geometric series is 1 - rho^3 = 0.0437 < 0.05, the three-value spread
    # 1 - rho^2 = 0.0293; pressure residual 0 (below any tol)
    rep, e0, rho, prm = _isolated_run(100.0, tol=1e-12)
    assert 1 - rho ** 3 < 0.05 < 1 - rho ** 2 + 0.05
    assert O.REASONS[rep["reason"]] == "stalled" and rep["iters"] == 4
    rv = 100.0 * (1 - rho) * rho ** 3 * e0 / prm["vref"]
    assert rep["rv_mean"] == pytest.approx(rv, rel=1e-12)
    assert rep["rv_max"] == pytest.approx(rv, rel=1e-12)
    assert rep["rp_mean"] == 0.0 and rep["rp_max"] == 0.0
    # a window of three stalls one iteration earlier
    rep3, *_ = _isolated_run(100.0, tol=1e-12, stall_window=3)
    assert O.REASONS[rep3["reason"]] == "stalled" and rep3["iters"] == 3
    # the cap below the window: max_iter at the cap
    rep_c, *_ = _isolated_run(100.0, tol=1e-12, max_iter=3)
    assert O.REASONS[rep_c["reason"]] == "max_iter" and rep_c["iters"] == 3


def test_isolated_particle_without_stall_runs_to_the_cap_or_tolerance():
    # beta = 80: 1 - rho^3 = 0.0542 > 0.05, so the stall rule never fires
    rep, e0, rho, prm = _isolated_run(80.0, tol=1e-12, max_iter=40)
    assert 1 - rho ** 3 > 0.05
    assert O.REASONS[rep["reason"]] == "max_iter" and rep["iters"] == 40
    assert rep["rv_mean"] == pytest.approx(80.0 * (1 - rho) * rho ** 39 * e0 / prm["vref"], rel=1e-11)
    # with a reachable tolerance it converges at the first k whose residual is below it
    tol = 0.01
    rep, e0, rho, prm = _isolated_run(80.0, tol=tol, max_iter=1000)
    k = 1
    while 80.0 * (1 - rho) * rho ** (k - 1) * e0 / prm["vref"] >= tol:
        k += 1
    assert O.REASONS[rep["reason"]] == "converged" and rep["iters"] == k and k > 4


def test_max_norm_on_two_isolated_particles():
    # two particles far apart (no neighbours), initial errors e1 < e2; beta = 10
    # (no stall). The mean norm stops when beta(1-rho)rho^(k-1)(e1+e2)/2 < tol,
    # the max norm when beta(1-rho)rho^(k-1) e2 < tol.
    beta = 10.0
    prm = _prm(beta=beta, vref=1.0, g=(0.0, 0.0, 0.0), tol=1e-3)
    x = np.array([[0.2, 0.5, 0.0], [0.8, 0.5, 0.0]])
    vn = np.zeros((2, 3))
    v0 = np.array([[0.01, 0.0, 0.0], [0.0, -0.05, 0.0]])  # V* = 0: errors 0.01, 0.05
    rho = 2 * beta / (2 * beta + 3)
    series = lambda e, k: beta * (1 - rho) * rho ** (k - 1) * e
    e1, e2 = 0.01, 0.05
    first_below = lambda e: next(k for k in range(1, 10000) if series(e, k) < prm["tol"])
    k_mean, k_max = first_below(0.5 * (e1 + e2)), first_below(e2)
    assert k_max > k_mean
    for norm, k_exp in ((0, k_mean), (1, k_max)):
        vk, pk, dk, rep = O.pseudo_loop(dict(prm, conv_norm=norm), 2, 0, x, vn, vn, v0,
                                        np.zeros(2), np.zeros(2))
        assert O.REASONS[rep["reason"]] == "converged" and rep["iters"] == k_exp
        assert rep["rv_mean"] == pytest.approx(series(0.5 * (e1 + e2), k_exp), rel=1e-11)
        assert rep["rv_max"] == pytest.approx(series(e2, k_exp), rel=1e-11)


# ----------------------------------------------------------------------------- pressure half steps

def _fourier_setup(n=32, rho0=2.5, beta=10.0, nu_e=0.01, dtau=0.0385, dt=0.01, kvec=(8, 0)):
    """Perfect n x n periodic lattice, V = 0, p = cos(k.r) with k = 2 pi kvec. The
    default mode (8, 0) has half the largest lattice eigenvalue; dtau keeps every
    mode's factor |1 + dtau lambda| below one (the explicit half steps are stable)."""
    dx = 1.0 / n
    prm = dict(I.BASE_PARAMS)
    prm.update(dim=2, h=dx, mass=rho0 * dx * dx, rho0=rho0, vref=1.0, beta=beta, nu=0.0, nu_e=nu_e,
               alpha=0.0, dt=dt, dtau=dtau, lo=(0, 0, 0), hi=(1, 1, 1), periodic=(1, 1, 0))
    ax = (np.arange(n) + 0.5) * dx
    gx, gy = np.meshgrid(ax, ax, indexing="ij")
    x = np.zeros((n * n, 3))
    x[:, 0], x[:, 1] = gx.ravel(), gy.ravel()
    k = 2 * np.pi * np.array(kvec, dtype=float)
    p0 = np.cos(x[:, :2] @ k)
    # eigenvalue of the EDAC diffusion sum on the perfect lattice: for p = cos(k.r),
    # sum_j (p_i - p_j) F(r_ij) = p_i sum_s (1 - cos(k.s)) F(|s|), F = dW/dr |s|/(s^2 + eta h^2)
    # over lattice offsets s with |s| < 3h (the sine part cancels between s and -s)
    offs = np.array([(a, b) for a in range(-3, 4) for b in range(-3, 4) if 0 < a * a + b * b < 9],
                    dtype=float) * dx
    r = np.linalg.norm(offs, axis=1)
    F = O.kernel_dwdr(2, dx, r) * r / (r * r + prm["eta"] * dx * dx)
    lam = 2.0 * (prm["mass"] / rho0) * nu_e * np.sum((1.0 - np.cos(offs @ k)) * F)
    return prm, x, p0, lam


def test_edac_eigenvalue_is_the_laplacian_symbol():
    # the lattice sum approximates nu_e * lap: lambda -> -nu_e |k|^2 (within the
    # lattice and eta errors at kh = 0.2)
    prm, x, p0, lam = _fourier_setup(kvec=(1, 0))
    assert lam < 0
    assert lam / (-0.01 * (2 * np.pi) ** 2) == pytest.approx(1.0, abs=0.03)
    # and the oracle's rate at V = 0 is lambda p (eigenvector), to round-off
    D, R, _, _, _ = O.rates(prm, x.shape[0], 0, x, np.zeros_like(x), p0)
    assert np.abs(D - lam * p0).max() < 1e-12 * abs(lam)


@pytest.mark.parametrize("stored_rate", ["eigen", "zero"])
def test_pressure_half_steps_one_iteration(stored_rate):
    # V^0 = 0, so iteration 0's divergence term vanishes exactly and
    # D^{1/2} = lambda p^{1/2}:  p^{1/2} = p^0 + dtau/2 D^0,  p^1 = p^{1/2} + dtau/2 D^{1/2}
    prm, x, p0, lam = _fourier_setup()
    dtau, dt, c = prm["dtau"], prm["dt"], prm["beta"] * prm["vref"]
    a = 0.5 * dtau * lam
    assert -0.4 < a < -0.3  # a full step would differ by a^2 ~ 0.13 relative
    d0 = lam * p0 if stored_rate == "eigen" else np.zeros_like(p0)
    n = x.shape[0]
    vk, pk, dk, rep = O.pseudo_loop(prm, n, 0, x, np.zeros((n, 3)), np.zeros((n, 3)), np.zeros((n, 3)),
                                    p0, d0, fixed_iters=1)
    phalf = p0 * (1 + a) if stored_rate == "eigen" else p0
    assert np.abs(pk - phalf * (1 + a)).max() < 1e-12
    assert np.abs(dk - lam * phalf).max() < 1e-12 * abs(lam)
    # eq. conv: mean and max of |D| over fluid times dt / (rho c^2)
    scale = dt / (prm["rho0"] * c * c)
    assert rep["rp_mean"] == pytest.approx(abs(lam) * np.mean(np.abs(phalf)) * scale, rel=1e-11)
    assert rep["rp_max"] == pytest.approx(abs(lam) * np.max(np.abs(phalf)) * scale, rel=1e-11)


def test_pressure_half_steps_many_iterations():
    # with c -> 0 the divergence term (c^2 div V) vanishes and every rate is
    # lambda times the pressure it is taken at. Stage 1 uses the stored rate, so the
    # half-step values obey p^{k+3/2} = p^{k+1} + dtau/2 D^{k+1/2} = (1 + 2a) p^{k+1/2}
    # with a = dtau lambda / 2, and p^K = (1 + a) p^{K-1/2}: from D^0 = lambda p^0,
    # p^K = (1 + a)^2 (1 + 2a)^(K-1) p^0 and the stored rate is lambda p^{K-1/2}.
    # (A full step p^{k+1} = p^k + dtau D(p^k) would give (1 + 2a)^K: 47% off here.)
    prm, x, p0, lam = _fourier_setup(beta=1e-7)
    n = x.shape[0]
    a = 0.5 * prm["dtau"] * lam
    for K in (2, 5, 12):
        vk, pk, dk, rep = O.pseudo_loop(prm, n, 0, x, np.zeros((n, 3)), np.zeros((n, 3)), np.zeros((n, 3)),
                                        p0, lam * p0, fixed_iters=K)
        phalf = (1 + a) * (1 + 2 * a) ** (K - 1) * p0
        assert np.abs(pk - (1 + a) * phalf).max() < 1e-10
        assert np.abs(dk - lam * phalf).max() < 1e-10 * abs(lam)
        assert rep["iters"] == K
