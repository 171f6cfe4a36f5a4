"""FP64 CPU oracle of the frozen-particle dual-time EDAC SPH step (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: the independent reference that the GPU library is
checked against. Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import it. It shares no code with the GPU library; the
two are driven from the same seeded inputs (``paper_1904_00861_amd.inputs``).

The C source (``dtsph_oracle.c``) cites the paper passage each function follows.
Functions here take and return float64 numpy arrays in caller order (fluid
particles first, then walls; vectors with three components per particle).

Parity status: every function is pinned by the CPU tests in
``tests/test_oracle_pins.py`` except the free-running iteration counts, for which
the paper gives only a qualitative bound (parity unpinned, see that file).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dtsph_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

REASONS = {1: "converged", 2: "stalled", 3: "max_iter", 4: "nonfinite", 5: "fixed"}


class Params(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("pad0", C.c_int32),
        ("h", C.c_double), ("kappa", C.c_double),
        ("rho0", C.c_double), ("mass", C.c_double),
        ("vref", C.c_double), ("beta", C.c_double),
        ("nu", C.c_double), ("nu_e", C.c_double),
        ("alpha", C.c_double), ("eps_av", C.c_double), ("eta", C.c_double),
        ("g", C.c_double * 3),
        ("dt", C.c_double), ("dtau", C.c_double),
        ("tol", C.c_double),
        ("max_iter", C.c_int32), ("stall_window", C.c_int32),
        ("stall_rel", C.c_double),
        ("conv_norm", C.c_int32), ("pad1", C.c_int32),
        ("lo", C.c_double * 3), ("hi", C.c_double * 3),
        ("periodic", C.c_int32 * 3),
        ("edac_reg_literal", C.c_int32), ("edac_rho_literal", C.c_int32),
        ("pad2", C.c_int32),
        ("shift", C.c_int32), ("shift_n", C.c_int32),
        ("shift_r", C.c_double),
        ("steady", C.c_int32), ("move", C.c_int32),
    ]


class Report(C.Structure):
    _fields_ = [
        ("iters", C.c_int32), ("reason", C.c_int32),
        ("rp_mean", C.c_double), ("rv_mean", C.c_double),
        ("rp_max", C.c_double), ("rv_max", C.c_double),
        ("pairs", C.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fno-fast-math", "-ffp-contract=off",
               "-fopenmp", "-shared", "-fPIC", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        P = C.POINTER
        d = P(C.c_double)
        L.or_sigma.restype = C.c_double
        L.or_sigma.argtypes = [C.c_int, C.c_double]
        L.or_w.restype = C.c_double
        L.or_w.argtypes = [C.c_int, C.c_double, C.c_double]
        L.or_dwdr.restype = C.c_double
        L.or_dwdr.argtypes = [C.c_int, C.c_double, C.c_double]
        L.or_neighbors.restype = C.c_int64
        L.or_neighbors.argtypes = [P(Params), C.c_int, C.c_int, d, C.c_int, P(C.c_int64),
                                   P(C.c_int32), C.c_int64]
        L.or_rates.restype = C.c_int64
        L.or_rates.argtypes = [P(Params), C.c_int, C.c_int, d, d, d, C.c_int, d, d, d, d]
        L.or_rates_vt.restype = C.c_int64
        L.or_rates_vt.argtypes = [P(Params), C.c_int, C.c_int, d, d, d, d, C.c_int, d, d, d, d]
        L.or_predict.restype = C.c_int64
        L.or_predict.argtypes = [P(Params), C.c_int, C.c_int, d, d, d, d, d, d, d, d]
        L.or_pseudo_loop.restype = C.c_int
        L.or_pseudo_loop.argtypes = [P(Params), C.c_int, C.c_int, d, d, d, d, d, d, C.c_int,
                                     C.c_int, P(Report)]
        L.or_correct.restype = None
        L.or_correct.argtypes = [P(Params), C.c_int, C.c_int, d, d, d, d, d, d]
        L.or_step.restype = C.c_int
        L.or_step.argtypes = [P(Params), C.c_int, C.c_int, d, d, d, d, C.c_int, C.c_int,
                              P(Report)]
        L.or_rows.restype = None
        L.or_rows.argtypes = [P(Params), C.c_int, C.c_int, C.c_int, d, d, d, d, d, d, C.c_int,
                              P(C.c_int32), d, d, d]
        L.or_shift.restype = None
        L.or_shift.argtypes = [P(Params), C.c_int, C.c_int, d, d, d, d, P(C.c_int32)]
        L.or_stop_test.restype = C.c_int
        L.or_stop_test.argtypes = [P(Params), d, d, C.c_int]
        L.or_num_threads.restype = C.c_int
        L.or_set_num_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def params(p: dict) -> Params:
    s = Params()
    for name, _ in Params._fields_:
        if name.startswith("pad"):
            continue
        val = p[name]
        if name in ("g", "lo", "hi"):
            getattr(s, name)[:] = [float(t) for t in val]
        elif name == "periodic":
            getattr(s, name)[:] = [int(t) for t in val]
        elif name in ("dim", "max_iter", "stall_window", "conv_norm", "edac_reg_literal",
                      "edac_rho_literal", "shift", "shift_n", "steady", "move"):
            setattr(s, name, int(val))
        else:
            setattr(s, name, float(val))
    return s


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, shape):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a.reshape(shape)


def sigma(dim, h):
    return lib().or_sigma(dim, h)


def kernel_w(dim, h, r):
    return np.array([lib().or_w(dim, h, float(t)) for t in np.ravel(r)]).reshape(np.shape(r))


def kernel_dwdr(dim, h, r):
    return np.array([lib().or_dwdr(dim, h, float(t)) for t in np.ravel(r)]).reshape(np.shape(r))


def neighbors(prm: dict, nf: int, nw: int, x, method: str = "bins"):
    """Neighbour lists as CSR (offsets[n+1], idx) with rows in ascending id."""
    n = nf + nw
    x = _f64(x, (n, 3))
    P = params(prm)
    m = 0 if method == "brute" else 1
    off = np.zeros(n + 1, dtype=np.int64)
    total = lib().or_neighbors(C.byref(P), nf, nw, _d(x), m,
                               off.ctypes.data_as(C.POINTER(C.c_int64)), None, 0)
    idx = np.zeros(max(total, 1), dtype=np.int32)
    lib().or_neighbors(C.byref(P), nf, nw, _d(x), m, off.ctypes.data_as(C.POINTER(C.c_int64)),
                       idx.ctypes.data_as(C.POINTER(C.c_int32)), total)
    return off, idx[:total]


def rates(prm: dict, nf: int, nw: int, x, v, p, method: str = "bins", vt=None):
    """D (pressure rate) and R (momentum right side incl. g) of every fluid particle
    at (x, v, p), walls set by the wall pass first; with vt (pseudo-time velocity
    Vtilde per particle, (n, 3)) the advective terms of the moving-particle
    scheme are included. Returns D[nf], R[nf,3], p_w[n], ghost velocity[n,3] and
    the number of fluid-row pairs."""
    n = nf + nw
    x, v, p = _f64(x, (n, 3)), _f64(v, (n, 3)), _f64(p, (n,))
    vt_arr = None if vt is None else _f64(vt, (n, 3))
    vtp = None if vt_arr is None else _d(vt_arr)
    D = np.zeros(n + 1)
    R = np.zeros((n + 1, 3))
    pw = np.zeros(n + 1)
    vg = np.zeros((n + 1, 3))
    P = params(prm)
    pairs = lib().or_rates_vt(C.byref(P), nf, nw, _d(x), _d(v), _d(p), vtp, 0 if method == "brute" else 1,
                              _d(D), _d(R), _d(pw), _d(vg))
    return D[:nf], R[:nf], pw[:n], vg[:n], pairs


def predict(prm: dict, nf: int, nw: int, x, v, p):
    """Predictor: returns dict(x_iter, v_iter, p_iter, dpdtau, acc, pairs)."""
    n = nf + nw
    x, v, p = _f64(x, (n, 3)), _f64(v, (n, 3)), _f64(p, (n,))
    x0, v0, acc = np.zeros((n, 3)), np.zeros((n, 3)), np.zeros((n, 3))
    p0, d0 = np.zeros(n), np.zeros(n)
    P = params(prm)
    pairs = lib().or_predict(C.byref(P), nf, nw, _d(x), _d(v), _d(p), _d(x0), _d(v0), _d(p0),
                             _d(d0), _d(acc))
    return dict(x_iter=x0, v_iter=v0, p_iter=p0, dpdtau=d0, acc=acc, pairs=pairs)


def pseudo_loop(prm: dict, nf: int, nw: int, x_iter, v_n, v_nm1, v_iter, p_iter, dpdtau,
                fixed_iters: int = 0):
    """Pseudo-time loop from an in-loop state. Returns (v_iter, p_iter, dpdtau, report)."""
    n = nf + nw
    x0 = _f64(x_iter, (n, 3))
    vn, vnm1 = _f64(v_n, (n, 3)), _f64(v_nm1, (n, 3))
    vk = _f64(v_iter, (n, 3)).copy()
    pk = _f64(p_iter, (n,)).copy()
    dk = _f64(dpdtau, (n,)).copy()
    rep = Report()
    P = params(prm)
    st = lib().or_pseudo_loop(C.byref(P), nf, nw, _d(x0), _d(vn), _d(vnm1), _d(vk), _d(pk), _d(dk),
                              int(fixed_iters), 1, C.byref(rep))
    r = rep.as_dict()
    r["status"] = st
    return vk, pk, dk, r


def correct(prm: dict, nf: int, nw: int, x, v, v_prev, p, v_iter, p_iter):
    n = nf + nw
    x, v = _f64(x, (n, 3)).copy(), _f64(v, (n, 3)).copy()
    vp, p = _f64(v_prev, (n, 3)).copy(), _f64(p, (n,)).copy()
    P = params(prm)
    lib().or_correct(C.byref(P), nf, nw, _d(x), _d(v), _d(vp), _d(p),
                     _d(_f64(v_iter, (n, 3))), _d(_f64(p_iter, (n,))))
    return x, v, vp, p


def step(prm: dict, nf: int, nw: int, x, v, v_prev, p, n_steps: int = 1, fixed_iters: int = 0):
    """Advance n_steps real steps (Algorithm 2; particle shifting after each
    corrector when prm["shift"] is 1). With prm["steady"] = 1 each step is one
    run of the steady-state pseudo-time loop from the current state (sections
    2.3 and 3.3), particles fixed. Returns (x, v, v_prev, p, reports, status)."""
    n = nf + nw
    x, v = _f64(x, (n, 3)).copy(), _f64(v, (n, 3)).copy()
    vp, p = _f64(v_prev, (n, 3)).copy(), _f64(p, (n,)).copy()
    reps = (Report * max(n_steps, 1))()
    P = params(prm)
    st = lib().or_step(C.byref(P), nf, nw, _d(x), _d(v), _d(vp), _d(p), int(n_steps),
                       int(fixed_iters), reps)
    return x, v, vp, p, [reps[s].as_dict() for s in range(n_steps)], st


def shift(prm: dict, nf: int, nw: int, x, v, p):
    """Particle shifting with Taylor correction (section 3.5). Returns new
    (x, v, p), the shift vectors of the fluid (nf, 3) and the free-surface flags."""
    n = nf + nw
    x = _f64(x, (n, 3)).copy()
    v = _f64(v, (n, 3)).copy()
    p = _f64(p, (n,)).copy()
    dr = np.zeros((max(nf, 1), 3))
    fs = np.zeros(max(nf, 1), dtype=np.int32)
    lib().or_shift(C.byref(params(prm)), nf, nw, _d(x), _d(v), _d(p), _d(dr),
                   fs.ctypes.data_as(C.POINTER(C.c_int32)))
    return x, v, p, dr[:nf], fs[:nf].astype(bool)


def rows(prm: dict, nf: int, nw: int, mode: int, rows_idx, x, vk, pk, dk=None, vn=None,
         vnm1=None):
    """Sampled rows, brute-force neighbours (large inputs). mode 0: predictor
    (returns V^(0), p^(0), D^n); mode 1: one pseudo-iteration from the in-loop
    state (returns V^1, p^1, D^{1/2})."""
    n = nf + nw
    rows_idx = np.ascontiguousarray(rows_idx, dtype=np.int32)
    m = rows_idx.size
    x, vk, pk = _f64(x, (n, 3)), _f64(vk, (n, 3)), _f64(pk, (n,))
    dk = _f64(dk if dk is not None else np.zeros(n), (n,))
    vn = _f64(vn if vn is not None else np.zeros((n, 3)), (n, 3))
    vnm1 = _f64(vnm1 if vnm1 is not None else np.zeros((n, 3)), (n, 3))
    vo, po, do = np.zeros((m, 3)), np.zeros(m), np.zeros(m)
    P = params(prm)
    lib().or_rows(C.byref(P), nf, nw, int(mode), _d(x), _d(vk), _d(pk), _d(dk), _d(vn), _d(vnm1),
                  m, rows_idx.ctypes.data_as(C.POINTER(C.c_int32)), _d(vo), _d(po), _d(do))
    return vo, po, do


def stop_test(prm: dict, rp, rv) -> str:
    """The stop test (eq. conv and the stall rule) applied to residual histories
    rp, rv (one value per iteration run so far). Returns the reason name, or
    "continue"."""
    rp = np.ascontiguousarray(rp, dtype=np.float64)
    rv = np.ascontiguousarray(rv, dtype=np.float64)
    assert rp.shape == rv.shape and rp.ndim == 1
    r = lib().or_stop_test(C.byref(params(prm)), _d(rp), _d(rv), int(rp.size))
    return REASONS.get(r, "continue")


def num_threads() -> int:
    return lib().or_num_threads()


def set_num_threads(n: int) -> None:
    lib().or_set_num_threads(int(n))
