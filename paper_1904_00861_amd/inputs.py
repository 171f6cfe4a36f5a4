"""Seeded synthetic workloads shaped like the paper's test problems.

This module only lays out particles and assigns the initial and boundary data of
each problem. It holds none of the solver's arithmetic (no kernel, no rate, no
integrator), so that the GPU library and the CPU oracle can both be driven from
the same inputs without sharing any code.

Problems (paper, section "Results and discussion"):
  * 2D Taylor-Green vortex on the periodic unit square; initial field from the
    exact solution (eq. tgv_sol), positions jittered with a fixed seed
    (subsection "Perturbation in initial positions").
  * 3D Taylor-Green vortex on the periodic unit cube (single-mode textbook field,
    since the paper has no 3D case).
  * Lid-driven cavity in the unit box, lid speed 1, three wall layers
    (subsection "The lid-driven-cavity problem").
  * 2D dam break: a 1 x 2 water column in a 4 x 4 tank with three wall layers and
    hydrostatic initial pressure (subsection "Dam-break in 2 dimensions").
  * A batch of uneven TGV / cavity instances with seeded sizes and Reynolds numbers.

Every problem is a :class:`Problem`: a parameter dictionary with physical inputs
(the solver derives c, nu_e and the pseudo step from them) and float64 arrays in
caller order: each simulation lists its fluid particles first, then its walls.
Positions are always stored with three components (unused ones are zero).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List

import numpy as np

#: Default parameters shared by every problem (the paper's section 3.4 choices and
#: the Morris regulariser value); the problem builders override what they set.
BASE_PARAMS = dict(
    dim=2,
    h=0.0,
    kappa=3.0,          # quintic spline support radius in units of h
    rho0=1.0,
    mass=0.0,
    vref=1.0,
    beta=10.0,
    nu=0.0,
    nu_e=0.0,           # 0 -> solver default h*c/16
    alpha=0.0,
    eps_av=0.01,
    eta=0.01,
    g=(0.0, 0.0, 0.0),
    dt=0.0,
    dtau=0.0,           # 0 -> solver default dt/beta
    tol=1e-3,
    max_iter=1000,
    stall_window=4,
    stall_rel=0.05,
    conv_norm=0,        # 0: mean residual norm, 1: max norm
    lo=(0.0, 0.0, 0.0),
    hi=(1.0, 1.0, 1.0),
    periodic=(1, 1, 1),
    edac_reg_literal=0,
    edac_rho_literal=0,
    max_neighbors=0,    # 0 -> library estimate
    shift=0,            # particle shifting after the corrector (section 3.5): 0 off, 1 on
    shift_r=1.0,        # shifting coefficient 1 + shift_r * (W / W(dx))^shift_n,
    shift_n=1,          # dx = h; the printed form is R = n = 1
    steady=0,           # 1: steady-state solve (sections 2.3, 3.3), particles never move
    move=0,             # particles in pseudo-time (Algorithm 1): 0 frozen, 1 moving with the
                        # lists of r^(0), 2 moving with the lists recomputed every iteration
)

CFL = 0.25  # dt * V_ref = C * h with C = 0.25


@dataclasses.dataclass
class Problem:
    name: str
    params: dict
    x: np.ndarray        # (n, 3) float64
    v: np.ndarray        # (n, 3) V^n for fluid; prescribed velocity for walls
    v_prev: np.ndarray   # (n, 3) V^{n-1} for fluid; zero for walls
    p: np.ndarray        # (n,)   p^n for fluid; zero for walls
    n_fluid: int
    n_wall: int

    @property
    def n(self) -> int:
        return self.n_fluid + self.n_wall

    def copy(self) -> "Problem":
        return Problem(self.name, dict(self.params), self.x.copy(), self.v.copy(),
                       self.v_prev.copy(), self.p.copy(), self.n_fluid, self.n_wall)


def _params(**kw) -> dict:
    p = dict(BASE_PARAMS)
    p.update(kw)
    for k in ("g", "lo", "hi", "periodic"):
        p[k] = tuple(p[k])
    return p


def _lattice(n_per_axis, dx, dim, origin=0.0):
    axes = [origin + (np.arange(n_per_axis) + 0.5) * dx for _ in range(dim)]
    grids = np.meshgrid(*axes, indexing="ij")
    pts = np.zeros((grids[0].size, 3))
    for a in range(dim):
        pts[:, a] = grids[a].ravel()
    return pts


def _jitter(x, dim, amp, rng):
    x = x.copy()
    x[:, :dim] += rng.uniform(-amp, amp, size=(x.shape[0], dim))
    return x


def tgv2d(n: int = 50, re: float = 100.0, seed: int = 1904, jitter: float = 0.01,
          U: float = 1.0, rho: float = 1.0, beta: float = 10.0, tol: float = 1e-3,
          name: str = None) -> Problem:
    """2D Taylor-Green vortex, n x n particles on the periodic unit square."""
    dx = 1.0 / n
    h = dx
    rng = np.random.default_rng(seed)
    x = _jitter(_lattice(n, dx, 2), 2, jitter * dx, rng)
    X, Y = x[:, 0], x[:, 1]
    v = np.zeros_like(x)
    v[:, 0] = -U * np.cos(2 * np.pi * X) * np.sin(2 * np.pi * Y)
    v[:, 1] = U * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y)
    p = -rho * U * U * (np.cos(4 * np.pi * X) + np.cos(4 * np.pi * Y)) / 4.0
    nu = U * 1.0 / re
    dt = CFL * h / U
    # exact solution one step back in time: amplitude grows by exp(8 pi^2 nu dt)
    v_prev = v * math.exp(8.0 * math.pi ** 2 * nu * dt)
    prm = _params(dim=2, h=h, rho0=rho, mass=rho * dx * dx, vref=U, beta=beta, nu=nu,
                  dt=dt, tol=tol, lo=(0, 0, 0), hi=(1, 1, 1), periodic=(1, 1, 1))
    return Problem(name or f"tgv2d_{n}", prm, x, v, v_prev, p, x.shape[0], 0)


def tgv3d(n: int = 64, re: float = 1600.0, seed: int = 1906, jitter: float = 0.01,
          U: float = 1.0, rho: float = 1.0, beta: float = 10.0, tol: float = 1e-3,
          name: str = None) -> Problem:
    """3D Taylor-Green vortex, n^3 particles on the periodic unit cube."""
    dx = 1.0 / n
    h = dx
    rng = np.random.default_rng(seed)
    x = _jitter(_lattice(n, dx, 3), 3, jitter * dx, rng)
    k = 2 * np.pi
    X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
    v = np.zeros_like(x)
    v[:, 0] = U * np.sin(k * X) * np.cos(k * Y) * np.cos(k * Z)
    v[:, 1] = -U * np.cos(k * X) * np.sin(k * Y) * np.cos(k * Z)
    p = rho * U * U / 16.0 * (np.cos(2 * k * X) + np.cos(2 * k * Y)) * (np.cos(2 * k * Z) + 2.0)
    nu = U * 1.0 / re
    dt = CFL * h / U
    # the single-mode field decays like exp(-3 k^2 nu t) at early times
    v_prev = v * math.exp(3.0 * k * k * nu * dt)
    prm = _params(dim=3, h=h, rho0=rho, mass=rho * dx ** 3, vref=U, beta=beta, nu=nu,
                  dt=dt, tol=tol, lo=(0, 0, 0), hi=(1, 1, 1), periodic=(1, 1, 1))
    return Problem(name or f"tgv3d_{n}", prm, x, v, v_prev, p, x.shape[0], 0)


def _wall_box(nx, ny, dx, layers, x_ext, y_ext, open_top):
    """Wall particles around the rectangle [0, nx*dx] x [0, ny*dx] (layers thick).

    x_ext/y_ext: number of lattice rows of the wall columns along x / y.
    """
    pts = []
    for i in range(-layers, x_ext + layers):
        for j in range(-layers, y_ext + (0 if open_top else layers)):
            inside_x = 0 <= i < x_ext
            inside_y = 0 <= j < y_ext
            if inside_x and inside_y:
                continue
            if open_top and j >= y_ext:
                continue
            pts.append(((i + 0.5) * dx, (j + 0.5) * dx, 0.0))
    return np.asarray(pts, dtype=np.float64).reshape(-1, 3)


def cavity(n: int = 50, re: float = 100.0, lid: float = 1.0, beta: float = 10.0,
           tol: float = 1e-4, layers: int = 3, name: str = None, steady: bool = False) -> Problem:
    """Lid-driven cavity: n x n fluid in the unit box, wall layers all around.

    The top wall layers (full width, corners included) move at u = lid. With
    steady=True the sim is solved for its steady state (particles fixed).
    """
    dx = 1.0 / n
    h = dx
    fluid = _lattice(n, dx, 2)
    walls = _wall_box(n, n, dx, layers, n, n, open_top=False)
    x = np.concatenate([fluid, walls])
    nf, nw = fluid.shape[0], walls.shape[0]
    v = np.zeros_like(x)
    v[nf:, 0] = np.where(walls[:, 1] > 1.0, lid, 0.0)
    p = np.zeros(x.shape[0])
    nu = lid * 1.0 / re
    dt = CFL * h / lid
    kh = 3.0 * h
    lo = (-layers * dx - kh, -layers * dx - kh, 0.0)
    hi = (1 + layers * dx + kh, 1 + layers * dx + kh, 1.0)
    prm = _params(dim=2, h=h, rho0=1.0, mass=dx * dx, vref=lid, beta=beta, nu=nu, dt=dt,
                  tol=tol, lo=lo, hi=hi, periodic=(0, 0, 0), steady=1 if steady else 0)
    return Problem(name or f"cavity{'_steady' if steady else ''}_{n}", prm, x, v, np.zeros_like(x), p, nf, nw)


def poiseuille(ny: int = 20, nx: int = 8, nu: float = 1.0, g: float = 1.0, beta: float = 10.0,
               layers: int = 3, steady: bool = True, dtau: float = None, name: str = None) -> Problem:
    """Plane channel of height 1 between two walls (y < 0 and y > 1), periodic in
    x over nx columns, driven by a body force g along x, fluid at rest. Its
    steady state is u(y) = g y (1 - y) / (2 nu). The pseudo step defaults to a
    tenth of the viscous limit h^2 / nu."""
    dx = 1.0 / ny
    h = dx
    xs = (np.arange(nx) + 0.5) * dx
    ys = (np.arange(-layers, ny + layers) + 0.5) * dx
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    pts = np.zeros((X.size, 3))
    pts[:, 0], pts[:, 1] = X.ravel(), Y.ravel()
    is_fluid = (pts[:, 1] > 0.0) & (pts[:, 1] < 1.0)
    fluid, walls = pts[is_fluid], pts[~is_fluid]
    x = np.concatenate([fluid, walls])
    nf, nw = fluid.shape[0], walls.shape[0]
    vref = g / (8.0 * nu) if g > 0 else 1.0  # centre-line speed
    dt = CFL * h / vref
    kh = 3.0 * h
    lo = (0.0, -layers * dx - kh, 0.0)
    hi = (nx * dx, 1.0 + layers * dx + kh, 1.0)
    prm = _params(dim=2, h=h, rho0=1.0, mass=dx * dx, vref=vref, beta=beta, nu=nu, dt=dt,
                  dtau=dtau if dtau is not None else 0.1 * h * h / nu, g=(g, 0.0, 0.0),
                  tol=1e-8, lo=lo, hi=hi, periodic=(1, 0, 0), steady=1 if steady else 0)
    z = np.zeros_like(x)
    return Problem(name or f"poiseuille_{ny}", prm, x, z.copy(), z.copy(), np.zeros(x.shape[0]), nf, nw)


def dam_break(dx: float = 0.002, width: float = 1.0, height: float = 2.0, tank: float = 4.0,
              rho: float = 1000.0, g: float = 9.81, alpha: float = 0.1, beta: float = 10.0,
              tol: float = 1e-4, layers: int = 3, name: str = None) -> Problem:
    """2D dam break: width x height column in a tank x tank box, open top."""
    h = dx
    nx, ny = int(round(width / dx)), int(round(height / dx))
    nt = int(round(tank / dx))
    axes_x = (np.arange(nx) + 0.5) * dx
    axes_y = (np.arange(ny) + 0.5) * dx
    X, Y = np.meshgrid(axes_x, axes_y, indexing="ij")
    fluid = np.zeros((X.size, 3))
    fluid[:, 0], fluid[:, 1] = X.ravel(), Y.ravel()
    walls = _wall_box(nt, nt, dx, layers, nt, nt, open_top=True)
    x = np.concatenate([fluid, walls])
    nf, nw = fluid.shape[0], walls.shape[0]
    v = np.zeros_like(x)
    p = np.zeros(x.shape[0])
    p[:nf] = rho * g * (height - fluid[:, 1])
    vref = math.sqrt(2.0 * g * height)
    dt = CFL * h / vref
    kh = 3.0 * h
    lo = (-layers * dx - kh, -layers * dx - kh, 0.0)
    hi = (tank + layers * dx + kh, tank + kh, 1.0)
    prm = _params(dim=2, h=h, rho0=rho, mass=rho * dx * dx, vref=vref, beta=beta, nu=0.0,
                  alpha=alpha, g=(0.0, -g, 0.0), dt=dt, tol=tol, lo=lo, hi=hi,
                  periodic=(0, 0, 0))
    return Problem(name or f"dam_break_{dx:g}", prm, x, v, np.zeros_like(x), p, nf, nw)


def hydrostatic_tank(n: int = 10, depth_cells: int = None, rho: float = 1.0, g: float = 1.0,
                     beta: float = 10.0, tol: float = 1e-6, layers: int = 3,
                     name: str = None) -> Problem:
    """Fluid at rest in a closed-bottom open-top tank, starting from p = 0."""
    depth_cells = depth_cells or n
    dx = 1.0 / n
    h = dx
    fluid = _lattice(n, dx, 2)[: n * n]
    fluid = fluid[fluid[:, 1] < depth_cells * dx]
    walls = _wall_box(n, depth_cells + 4, dx, layers, n, depth_cells + 4, open_top=True)
    x = np.concatenate([fluid, walls])
    nf, nw = fluid.shape[0], walls.shape[0]
    H = depth_cells * dx
    vref = math.sqrt(2.0 * g * H)
    dt = CFL * h / vref
    kh = 3.0 * h
    lo = (-layers * dx - kh, -layers * dx - kh, 0.0)
    hi = (1 + layers * dx + kh, (depth_cells + 4) * dx + kh, 1.0)
    prm = _params(dim=2, h=h, rho0=rho, mass=rho * dx * dx, vref=vref, beta=beta, nu=0.0,
                  alpha=0.1, g=(0.0, -g, 0.0), dt=dt, tol=tol, lo=lo, hi=hi,
                  periodic=(0, 0, 0))
    z = np.zeros_like(x)
    return Problem(name or f"tank_{n}", prm, x, z.copy(), z.copy(), np.zeros(x.shape[0]), nf, nw)


def batch(n_sims: int = 64, seed: int = 1904, n_min: float = 2500.0, n_max: float = 160000.0,
          re_lo: float = 100.0, re_hi: float = 1000.0) -> List[Problem]:
    """Uneven batch: even index -> periodic TGV, odd index -> lid-driven cavity.

    Fluid counts are log-uniform in [n_min, n_max], Re uniform in [re_lo, re_hi].
    """
    rng = np.random.default_rng(seed)
    counts = np.exp(rng.uniform(math.log(n_min), math.log(n_max), size=n_sims))
    res = rng.uniform(re_lo, re_hi, size=n_sims)
    out = []
    for s in range(n_sims):
        n = int(round(math.sqrt(counts[s])))
        if s % 2 == 0:
            out.append(tgv2d(n, re=float(res[s]), seed=1904000 + s, name=f"b{s}_tgv{n}"))
        else:
            out.append(cavity(n, re=float(res[s]), name=f"b{s}_cav{n}"))
    return out


# -- named workloads -------------------------------------------------------------

def config(name: str):
    """The five named workloads of the performance study.

    C0: 2D TGV 50^2, FP64, 10 steps      C1: 2D TGV 400^2, 200 steps
    C2: 3D TGV 64^3, 50 steps            C3: 2D dam break dx=0.002, 100 steps
    C4: batch of 64 TGV/cavity instances, 50 steps each

    C2 and C3 switch on the paper's particle shifting (section 3.5, used there
    for every test case): without it the 3D vortex turns unstable after about
    30 steps and the dam break after about 58, the same in any implementation of
    the step (the oracle and the library follow the same trajectory).
    """
    if name == "C0":
        return tgv2d(50, seed=1904)
    if name == "C1":
        return tgv2d(400, seed=1905)
    if name == "C2":
        prob = tgv3d(64, seed=1906)
        prob.params = dict(prob.params, shift=1)
        return prob
    if name == "C3":
        prob = dam_break(0.002)
        prob.params = dict(prob.params, shift=1)
        return prob
    if name == "C4":
        return batch(64)
    raise KeyError(name)


CONFIG_STEPS = {"C0": 10, "C1": 200, "C2": 50, "C3": 100, "C4": 50}


def loop_state_from(prob: Problem, seed: int = 7, amp_v: float = 0.05, amp_d: float = 1.0):
    """An in-loop state for testing the pseudo-time iteration in isolation.

    Frozen positions are the problem's positions; V^k and (dp/dtau)^k are the
    problem's fields plus seeded noise, p^k the problem's pressure, and V^n,
    V^{n-1} the problem's v and v_prev. Returns a dict of float64 arrays.
    """
    rng = np.random.default_rng(seed)
    n, nf = prob.n, prob.n_fluid
    vk = prob.v.copy()
    dim = prob.params["dim"]
    vk[:nf, :dim] += amp_v * prob.params["vref"] * rng.standard_normal((nf, dim))
    d = np.zeros(n)
    d[:nf] = amp_d * rng.standard_normal(nf)
    return dict(x_iter=prob.x.copy(), v_iter=vk, p_iter=prob.p.copy(), dpdtau=d)
