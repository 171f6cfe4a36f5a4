"""Pins of the oracle's moving-particle variant (sections 2.1 and 3.1,
Algorithm 1) against what the mathematics and the paper fix:

* with Vtilde^0 = 0 the first pseudo-iteration is the frozen scheme's, bit for bit;
* the advective pressure term is Vtilde . grad(p) (checked at rho != 1, where
  the printed sum alone would give Vtilde . grad(p) / rho);
* the advective momentum term is (Vtilde . grad) V of a linear field;
* the Taylor-Green vortex decays as with frozen particles (the paper finds no
  noticeable difference) and the two neighbour modes agree.
"""
import math

import numpy as np

import oracle as O
from paper_1904_00861_amd import inputs as I


def _lattice_box(n, rho=1.0):
    dx = 1.0 / n
    ax = (np.arange(n) + 0.5) * dx
    X, Y = np.meshgrid(ax, ax, indexing="ij")
    x = np.zeros((X.size, 3))
    x[:, 0], x[:, 1] = X.ravel(), Y.ravel()
    kh = 3.0 * dx
    prm = I._params(dim=2, h=dx, rho0=rho, mass=rho * dx * dx, vref=1.0, beta=10.0, nu=0.0, dt=0.25 * dx,
                    lo=(-kh, -kh, 0.0), hi=(1.0 + kh, 1.0 + kh, 1.0), periodic=(0, 0, 0), move=1)
    inner = np.all((x[:, :2] > 3.5 * dx) & (x[:, :2] < 1.0 - 3.5 * dx), axis=1)
    return x, prm, inner


def test_first_iteration_equals_the_frozen_one():
    prob = I.tgv2d(30, seed=5)
    for move in (1, 2):
        a = O.step(dict(prob.params, move=move), prob.n, 0, prob.x, prob.v, prob.v_prev, prob.p, 1, 1)
        b = O.step(dict(prob.params, move=0), prob.n, 0, prob.x, prob.v, prob.v_prev, prob.p, 1, 1)
        for k in range(4):
            assert np.array_equal(a[k], b[k])


def test_advective_pressure_term_is_vtilde_dot_grad_p():
    x, prm, inner = _lattice_box(24, rho=2.0)
    n = x.shape[0]
    a = np.array([1.0, 0.5])
    p = x[:, 0] * a[0] + x[:, 1] * a[1]
    v = np.zeros_like(x)
    vt = np.zeros_like(x)
    b = np.array([0.3, -0.2])
    vt[:, 0], vt[:, 1] = b
    D1, _, _, _, _ = O.rates(prm, n, 0, x, v, p, vt=vt)
    D0, _, _, _, _ = O.rates(prm, n, 0, x, v, p)
    assert np.allclose(D1[inner] - D0[inner], b @ a, rtol=1e-2)


def test_advective_momentum_term_of_a_linear_field():
    x, prm, inner = _lattice_box(24)
    n = x.shape[0]
    A = np.array([[1.0, 0.4], [-0.3, 0.5]])
    xc = x[:, :2] - 0.5
    v = np.zeros_like(x)
    v[:, :2] = xc @ A.T
    vt = np.zeros_like(x)
    b = np.array([0.3, -0.2])
    vt[:, 0], vt[:, 1] = b
    p = np.zeros(n)
    _, R1, _, _, _ = O.rates(prm, n, 0, x, v, p, vt=vt)
    _, R0, _, _, _ = O.rates(prm, n, 0, x, v, p)
    want = A @ b  # (Vtilde . grad) V for V = A x
    err = np.abs(R1[inner, :2] - R0[inner, :2] - want).max() / np.abs(want).max()
    assert err < 1e-2


def test_tgv_decay_with_moving_particles():
    prob = I.config("C0")
    t = 10 * prob.params["dt"]
    exact = math.exp(-8 * math.pi ** 2 * t / 100.0)
    out = {}
    for move in (1, 2):
        x, v, vp, p, reps, st = O.step(dict(prob.params, move=move), prob.n, 0, prob.x, prob.v, prob.v_prev,
                                       prob.p, 10)
        assert st == 0
        ratio = np.linalg.norm(v, axis=1).max() / np.linalg.norm(prob.v, axis=1).max()
        assert abs(ratio - exact) / exact < 0.01
        out[move] = v
    fx, fv, _, _, _, _ = O.step(prob.params, prob.n, 0, prob.x, prob.v, prob.v_prev, prob.p, 10)
    scale = np.abs(fv).max()
    # neighbour updates change only pairs at the edge of the support, where the
    # kernel and its gradient vanish to fifth order
    assert np.abs(out[2] - out[1]).max() < 1e-9 * scale
    # moving and frozen particles agree to the size of the pseudo-time motion
    assert np.abs(out[1] - fv).max() < 1e-2 * scale
