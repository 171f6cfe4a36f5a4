"""CPU checks of the seeded synthetic workloads (paper_1904_00861_amd/inputs.py):
they are reproducible, have the documented sizes and parameters, keep
periodic positions inside their box, jitter within 0.01 dx of the lattice, and
start the Taylor-Green vortex from its analytic field (section 4 set-ups)."""
import math

import numpy as np
import pytest

from paper_1904_00861_amd import inputs as I


@pytest.mark.parametrize("name", ["C0", "C1", "C3"])
def test_workloads_are_reproducible(name):
    a, b = I.config(name), I.config(name)
    for f in ("x", "v", "v_prev", "p"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
    assert a.params == b.params


def test_seeds_change_only_the_jitter():
    a, b = I.tgv2d(20, seed=1), I.tgv2d(20, seed=2)
    assert not np.array_equal(a.x, b.x)
    dx = 1.0 / 20
    assert np.abs(a.x - b.x).max() <= 2 * 0.01 * dx + 1e-15


@pytest.mark.parametrize("name,n_fluid,n_wall", [("C0", 2500, 0), ("C1", 160000, 0), ("C2", 262144, 0),
                                                 ("C3", 500000, 18018)])
def test_documented_sizes(name, n_fluid, n_wall):
    prob = I.config(name)
    assert (prob.n_fluid, prob.n_wall) == (n_fluid, n_wall)
    assert prob.x.shape == (prob.n, 3) and prob.v.shape == (prob.n, 3) and prob.p.shape == (prob.n,)


def test_batch_workload():
    probs = I.config("C4")
    assert len(probs) == 64
    assert sum(p.n for p in probs) == 2574722
    for s, p in enumerate(probs):
        # fluid counts log-uniform in [2.5k, 160k] (rounded to square lattices),
        # Re = V_ref L / nu uniform in [100, 1000] on unit boxes
        assert 2500 * 0.97 <= p.n_fluid <= 160000 * 1.03
        assert 100.0 * (1 - 1e-12) <= p.params["vref"] / p.params["nu"] <= 1000.0 * (1 + 1e-12)
        if s % 2 == 0:
            assert p.n_wall == 0 and all(p.params["periodic"][:2])   # Taylor-Green vortex
        else:
            assert p.n_wall > 0 and not any(p.params["periodic"][:2])  # lid-driven cavity


@pytest.mark.parametrize("name", ["C0", "C1", "C2"])
def test_periodic_positions_inside_the_box_and_near_the_lattice(name):
    prob = I.config(name)
    prm = prob.params
    dim = prm["dim"]
    lo, hi = np.array(prm["lo"][:dim]), np.array(prm["hi"][:dim])
    x = prob.x[:, :dim]
    assert np.all(x >= lo) and np.all(x < hi)
    dx = prm["h"]  # h = dx on these lattices
    n = round((hi[0] - lo[0]) / dx)
    frac = (x - lo) / dx - 0.5
    assert np.abs(frac - np.round(frac)).max() <= 0.01 + 1e-9
    assert n ** dim == prob.n_fluid


@pytest.mark.parametrize("name", ["C0", "C1", "C2", "C3"])
def test_kernel_support_and_time_step(name):
    prob = I.config(name)
    prm = prob.params
    assert prm["kappa"] == 3.0
    # dt = C h / V_ref with C = 0.25
    assert math.isclose(prm["dt"], I.CFL * prm["h"] / prm["vref"], rel_tol=1e-12)
    assert I.CFL == 0.25


def test_tgv_starts_from_the_analytic_field():
    prob = I.config("C0")
    X, Y = prob.x[:, 0], prob.x[:, 1]
    assert np.allclose(prob.v[:, 0], -np.cos(2 * np.pi * X) * np.sin(2 * np.pi * Y), atol=1e-15)
    assert np.allclose(prob.v[:, 1], np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y), atol=1e-15)
    assert np.allclose(prob.p, -(np.cos(4 * np.pi * X) + np.cos(4 * np.pi * Y)) / 4.0, atol=1e-15)
    # V^{n-1}: the same field one step back, amplitude exp(8 pi^2 nu dt) larger
    ratio = prob.v_prev[:, :2] / np.where(prob.v[:, :2] == 0.0, 1.0, prob.v[:, :2])
    growth = math.exp(8 * math.pi ** 2 * prob.params["nu"] * prob.params["dt"])
    assert np.allclose(ratio[prob.v[:, :2] != 0.0], growth, rtol=1e-12)
