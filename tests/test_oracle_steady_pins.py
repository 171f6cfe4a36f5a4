"""Pins of the oracle's steady-state solve (sections 2.3 and 3.3: pressure rate
eq. dp-dtau-frozen, momentum eq. mom-steady, particles fixed) against what the
mathematics fixes:

* plane Poiseuille flow between Adami walls converges to the analytic parabola
  u = g y (1 - y) / (2 nu), with the first-order error of the wall treatment
  (it halves when the spacing halves), no cross-flow and no pressure;
* the convective sum of eq. mom-steady reproduces (V . grad) V of a linear field
  on a lattice, and the steady pressure rate is -rho c^2 div V;
* the steady pressure rate has no EDAC diffusion term;
* a steady step never moves a particle and rotates the velocity history.
"""
import numpy as np
import pytest

import oracle as O
from paper_1904_00861_amd import inputs as I


def _poiseuille_error(ny, iters):
    prob = I.poiseuille(ny=ny)
    nf = prob.n_fluid
    x, v, vp, p, reps, st = O.step(prob.params, nf, prob.n_wall, prob.x, prob.v, prob.v_prev, prob.p, 1, iters)
    y, u = x[:nf, 1], v[:nf, 0]
    exact = prob.params["g"][0] * y * (1.0 - y) / (2.0 * prob.params["nu"])
    return prob, x, v, vp, p, np.abs(u - exact).max() / exact.max()


def test_poiseuille_converges_to_the_parabola_at_first_order():
    # pseudo time 0.75 (ny=10) and 0.5 (ny=20) in units of H^2/nu: the slowest
    # transient mode has decayed by exp(-pi^2 tau) < 1e-2 of the centre speed
    prob10, x10, v10, _, p10, e10 = _poiseuille_error(10, 3000)
    prob20, x20, v20, _, p20, e20 = _poiseuille_error(20, 8000)
    assert e10 < 0.03 and e20 < 0.015          # within the wall treatment's O(dx) error
    assert 1.6 < e10 / e20 < 2.5                # first-order convergence to the parabola
    for prob, x, v, p in ((prob10, x10, v10, p10), (prob20, x20, v20, p20)):
        nf = prob.n_fluid
        assert np.array_equal(x, prob.x)        # particles never move
        assert np.abs(v[:nf, 1]).max() < 1e-12  # no cross-flow
        assert np.abs(p[:nf]).max() < 1e-10     # div V = 0: no pressure builds up


def _lattice_box(n):
    dx = 1.0 / n
    ax = (np.arange(n) + 0.5) * dx
    X, Y = np.meshgrid(ax, ax, indexing="ij")
    x = np.zeros((X.size, 3))
    x[:, 0], x[:, 1] = X.ravel(), Y.ravel()
    kh = 3.0 * dx
    prm = I._params(dim=2, h=dx, rho0=1.0, mass=dx * dx, vref=1.0, beta=10.0, nu=0.0, dt=0.25 * dx,
                    lo=(-kh, -kh, 0.0), hi=(1.0 + kh, 1.0 + kh, 1.0), periodic=(0, 0, 0), steady=1)
    inner = np.all((x[:, :2] > 3.5 * dx) & (x[:, :2] < 1.0 - 3.5 * dx), axis=1)
    return x, prm, inner


def test_convective_sum_of_a_linear_field():
    x, prm, inner = _lattice_box(24)
    a, b = 1.0, 0.5  # V = (a x', b y') about the centre; div V = a + b
    xc = x[:, :2] - 0.5
    v = np.zeros_like(x)
    v[:, 0], v[:, 1] = a * xc[:, 0], b * xc[:, 1]
    p = np.zeros(x.shape[0])
    D, R, _, _, _ = O.rates(prm, x.shape[0], 0, x, v, p)
    # (V . grad) V = (a^2 x', b^2 y'); with p = 0, nu = 0, no AV and no g the
    # steady momentum rate is its negative
    want = -np.stack([a * a * xc[:, 0], b * b * xc[:, 1]], axis=1)
    err = np.abs(R[inner, :2] - want[inner]).max() / np.abs(want[inner]).max()
    assert err < 1e-2
    # a transposed reading (V_j . gradW) or the other sign would miss by O(1)
    c = prm["beta"] * prm["vref"]
    assert np.allclose(D[inner], -prm["rho0"] * c * c * (a + b), rtol=1e-2)


def test_steady_pressure_rate_has_no_edac_term():
    x, prm, inner = _lattice_box(16)
    v = np.zeros_like(x)
    p = x[:, 0] ** 2 + x[:, 1] ** 2
    D_steady, _, _, _, _ = O.rates(prm, x.shape[0], 0, x, v, p)
    D_unsteady, _, _, _, _ = O.rates(dict(prm, steady=0), x.shape[0], 0, x, v, p)
    assert np.all(D_steady == 0.0)
    assert np.abs(D_unsteady[inner]).min() > 0.0  # the EDAC term sees the Laplacian of p


def test_steady_step_history_and_fixed_positions():
    prob = I.cavity(12, steady=True)
    nf, nw = prob.n_fluid, prob.n_wall
    x1, v1, vp1, p1, r1, _ = O.step(prob.params, nf, nw, prob.x, prob.v, prob.v_prev, prob.p, 1, 5)
    x2, v2, vp2, p2, r2, _ = O.step(prob.params, nf, nw, x1, v1, vp1, p1, 1, 5)
    assert np.array_equal(x1, prob.x) and np.array_equal(x2, prob.x)
    assert np.array_equal(vp2[:nf], v1[:nf])    # V^{n-1} <- V^n
    assert np.abs(v2[:nf] - v1[:nf]).max() > 0  # the lid drives the flow
    assert r1[0]["iters"] == 5 and r2[0]["iters"] == 5


def test_fluid_at_rest_is_a_steady_state():
    prob = I.poiseuille(ny=10, g=0.0, nu=1.0)
    nf, nw = prob.n_fluid, prob.n_wall
    x, v, vp, p, reps, _ = O.step(prob.params, nf, nw, prob.x, prob.v, prob.v_prev, prob.p, 1, 20)
    assert np.all(v == 0.0) and np.all(p == 0.0)
