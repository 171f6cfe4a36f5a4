"""ctypes binding of libdtsph.so (declared in include/dtsph.h).

Argument marshalling only: the functions named ``dtsph_*`` forward to the C-ABI
entry points of the same name, and :class:`Sim` keeps the caller-order state in
torch device tensors and passes their device pointers and the current HIP
stream. Every step of the hot path runs in the library's kernels. Importing is
cheap; the library is loaded on first use and a missing build raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdtsph.so")

OK, WARN_MAXITER = 0, 1
EINVAL, ENOMEM, EHIP, ENONFINITE, EOVERFLOW = -1, -2, -3, -4, -5
FP64, FP32 = 0, 1
REASONS = {0: "running", 1: "converged", 2: "stalled", 3: "max_iter", 4: "nonfinite", 5: "fixed"}
OPT_TIMING, OPT_RESET_TIMING, OPT_CHUNK, OPT_BLOCK, OPT_XCD_REMAP, OPT_LANES, OPT_SKIN = 1, 2, 3, 4, 5, 6, 7
OPT_CELL_DIV, OPT_NBR_LANES, OPT_GRAPHS, OPT_PAIR_CACHE, OPT_SPECULATE, OPT_FILTER_LANES = 8, 9, 10, 11, 12, 13
OPT_ABS32_POSITIONS, OPT_NBR_TILES, OPT_TAIL_LOOP, OPT_TAIL_SPIN = 14, 15, 16, 17

EXPORTS = [
    "dtsph_create", "dtsph_destroy", "dtsph_last_error", "dtsph_set_state", "dtsph_get_state",
    "dtsph_build_cells", "dtsph_predict", "dtsph_pseudo_iterate", "dtsph_correct", "dtsph_step",
    "dtsph_neighbor_list", "dtsph_set_option", "dtsph_get_timing",
    "dtsph_get_info", "dtsph_autotune", "dtsph_workspace_bytes", "dtsph_set_workspace",
    "dtsph_create_static",
]
STATIC_SCRATCH_BYTES = 64 << 20


class DtsphError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"dtsph status {status}: {msg}")
        self.status = status


class SimDesc(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("max_neighbors", C.c_int32),
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
        ("conv_norm", C.c_int32), ("edac_reg_literal", C.c_int32),
        ("edac_rho_literal", C.c_int32), ("reserved0", C.c_int32),
        ("lo", C.c_double * 3), ("hi", C.c_double * 3),
        ("periodic", C.c_int32 * 3), ("reserved1", C.c_int32),
        ("shift", C.c_int32), ("shift_n", C.c_int32),
        ("shift_r", C.c_double),
        ("steady", C.c_int32), ("move", C.c_int32),
    ]


class StateView(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in
                ("x", "v", "v_prev", "p", "x_iter", "v_iter", "p_iter", "dpdtau")]


class CellsView(C.Structure):
    _fields_ = [("keys", C.c_void_p), ("caller_index", C.c_void_p), ("cell_start", C.c_void_p)]


class IterReport(C.Structure):
    _fields_ = [("iters", C.c_int32), ("reason", C.c_int32),
                ("rp_mean", C.c_double), ("rv_mean", C.c_double),
                ("rp_max", C.c_double), ("rv_max", C.c_double),
                ("pairs", C.c_int64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class Timing(C.Structure):
    _fields_ = [("pass_launches", C.c_int64), ("pass_ms", C.c_double),
                ("pass_pairs", C.c_int64), ("pass_particles", C.c_int64),
                ("wall_launches", C.c_int64), ("wall_ms", C.c_double),
                ("build_launches", C.c_int64), ("build_ms", C.c_double),
                ("build_particles", C.c_int64), ("filter_launches", C.c_int64), ("filter_ms", C.c_double),
                ("full_builds", C.c_int64), ("list_filters", C.c_int64),
                ("last_max_shift", C.c_double), ("last_disp", C.c_double),
                ("spec_tries", C.c_int64), ("spec_hits", C.c_int64), ("tail_launches", C.c_int64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class Info(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_fluid", C.c_int64), ("n_wall", C.c_int64),
                ("n_cells", C.c_int64), ("n_sims", C.c_int32), ("precision", C.c_int32),
                ("nbr_capacity", C.c_int32), ("block", C.c_int32), ("lanes", C.c_int32),
                ("reserved", C.c_int32), ("device_bytes", C.c_int64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class TuneEntry(C.Structure):
    _fields_ = [("lanes", C.c_int32), ("block", C.c_int32), ("us", C.c_double)]


class TuneReport(C.Structure):
    _fields_ = [("lanes", C.c_int32), ("block", C.c_int32), ("us", C.c_double),
                ("n_entries", C.c_int32), ("reserved", C.c_int32), ("entries", TuneEntry * 12),
                ("nbr_lanes", C.c_int32), ("filter_lanes", C.c_int32),
                ("nbr_us", C.c_double), ("filter_us", C.c_double),
                ("cell_div", C.c_int32), ("nbr_tiles", C.c_int32), ("build_us", C.c_double)]

    def as_dict(self) -> dict:
        return dict(lanes=self.lanes, block=self.block, us=self.us, nbr_lanes=self.nbr_lanes,
                    nbr_tiles=self.nbr_tiles,
                    cell_div=self.cell_div, build_us=self.build_us,
                    filter_lanes=self.filter_lanes, nbr_us=self.nbr_us, filter_us=self.filter_us,
                    entries=[dict(lanes=e.lanes, block=e.block, us=e.us)
                             for e in self.entries[:self.n_entries]])


_lib = None


def lib() -> C.CDLL:
    """Load libdtsph.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(or python paper_1904_00861_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        P, vp = C.POINTER, C.c_void_p
        L.dtsph_create.argtypes = [P(SimDesc), P(C.c_int64), P(C.c_int64), C.c_int32, C.c_int32,
                                   vp, P(vp)]
        L.dtsph_create_static.argtypes = L.dtsph_create.argtypes
        L.dtsph_destroy.argtypes = [vp]
        L.dtsph_destroy.restype = None
        L.dtsph_last_error.argtypes = [vp]
        L.dtsph_last_error.restype = C.c_char_p
        L.dtsph_set_state.argtypes = [vp, P(StateView)]
        L.dtsph_get_state.argtypes = [vp, P(StateView)]
        L.dtsph_build_cells.argtypes = [vp, P(CellsView)]
        L.dtsph_predict.argtypes = [vp]
        L.dtsph_pseudo_iterate.argtypes = [vp, C.c_int32, P(IterReport)]
        L.dtsph_correct.argtypes = [vp]
        L.dtsph_step.argtypes = [vp, C.c_int32, P(IterReport)]
        L.dtsph_neighbor_list.argtypes = [vp, C.c_int32, P(C.c_int64), P(C.c_int32), C.c_int64,
                                          P(C.c_int64)]
        L.dtsph_set_option.argtypes = [vp, C.c_int32, C.c_int64]
        L.dtsph_get_timing.argtypes = [vp, P(Timing)]
        L.dtsph_get_info.argtypes = [vp, P(Info)]
        L.dtsph_autotune.argtypes = [vp, C.c_int32, P(TuneReport)]
        L.dtsph_workspace_bytes.argtypes = [vp, P(C.c_size_t)]
        L.dtsph_set_workspace.argtypes = [vp, vp, C.c_size_t]
        for name in EXPORTS:
            if name not in ("dtsph_destroy", "dtsph_last_error"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def desc_from_params(p: dict) -> SimDesc:
    d = SimDesc()
    for name, _ in SimDesc._fields_:
        if name.startswith("reserved"):
            continue
        val = p[name]
        if name in ("g", "lo", "hi"):
            getattr(d, name)[:] = [float(t) for t in val]
        elif name == "periodic":
            getattr(d, name)[:] = [int(t) for t in val]
        elif name in ("dim", "max_neighbors", "max_iter", "stall_window", "conv_norm",
                      "edac_reg_literal", "edac_rho_literal", "shift", "shift_n", "steady", "move"):
            setattr(d, name, int(val))
        else:
            setattr(d, name, float(val))
    return d


def last_error(ctx) -> str:
    return lib().dtsph_last_error(ctx).decode()


def _check(ctx, status: int) -> int:
    if status < 0:
        raise DtsphError(status, last_error(ctx))
    return status


# ---- thin forwards with the C names ---------------------------------------------

def _create(fn, params, n_fluid, n_wall, precision, stream):
    n = len(params)
    descs = (SimDesc * n)(*[desc_from_params(p) for p in params])
    nf = (C.c_int64 * n)(*[int(v) for v in n_fluid])
    nw = (C.c_int64 * n)(*[int(v) for v in n_wall])
    out = C.c_void_p()
    st = fn(descs, nf, nw, n, int(precision), C.c_void_p(stream or 0), C.byref(out))
    if st < 0:
        raise DtsphError(st, last_error(None))
    return out


def dtsph_create(params: Sequence[dict], n_fluid: Sequence[int], n_wall: Sequence[int],
                 precision: int = FP32, stream: Optional[int] = None):
    return _create(lib().dtsph_create, params, n_fluid, n_wall, precision, stream)


def dtsph_create_static(params: Sequence[dict], n_fluid: Sequence[int], n_wall: Sequence[int],
                        precision: int = FP32, stream: Optional[int] = None):
    return _create(lib().dtsph_create_static, params, n_fluid, n_wall, precision, stream)


def dtsph_destroy(ctx) -> None:
    lib().dtsph_destroy(ctx)


def dtsph_set_state(ctx, view: StateView) -> int:
    return _check(ctx, lib().dtsph_set_state(ctx, C.byref(view)))


def dtsph_get_state(ctx, view: StateView) -> int:
    return _check(ctx, lib().dtsph_get_state(ctx, C.byref(view)))


def dtsph_build_cells(ctx, layout=None):
    """Build (if the positions changed). With layout = (n, n_cells) also return
    the cell-ordered layout: keys[n], caller_index[n], cell_start[2 n_cells + 1]."""
    if layout is None:
        _check(ctx, lib().dtsph_build_cells(ctx, None))
        return None
    n, n_cells = layout
    keys = np.zeros(n, dtype=np.int32)
    callers = np.zeros(n, dtype=np.int32)
    starts = np.zeros(2 * n_cells + 1, dtype=np.int64)
    view = CellsView(keys.ctypes.data, callers.ctypes.data, starts.ctypes.data)
    _check(ctx, lib().dtsph_build_cells(ctx, C.byref(view)))
    return keys, callers, starts


def dtsph_predict(ctx) -> int:
    return _check(ctx, lib().dtsph_predict(ctx))


def dtsph_pseudo_iterate(ctx, fixed_iters: int, n_sims: int):
    reps = (IterReport * n_sims)()
    st = _check(ctx, lib().dtsph_pseudo_iterate(ctx, int(fixed_iters), reps))
    return st, [r.as_dict() for r in reps]


def dtsph_correct(ctx) -> int:
    return _check(ctx, lib().dtsph_correct(ctx))


def dtsph_step(ctx, n_steps: int, n_sims: int, want_reports: bool = True):
    reps = (IterReport * max(1, n_steps * n_sims))() if want_reports else None
    st = _check(ctx, lib().dtsph_step(ctx, int(n_steps), reps))
    if not want_reports:
        return st, None
    out = [[reps[s * n_sims + k].as_dict() for k in range(n_sims)] for s in range(n_steps)]
    return st, out


def dtsph_neighbor_list(ctx, m: int, sim: int = -1):
    """Exact neighbour rows (CSR offsets[m + 1], indices) of every particle
    (sim = -1, m = n) or of sim `sim` alone (m = its particle count, indices
    relative to its first particle)."""
    off = np.zeros(m + 1, dtype=np.int64)
    need = C.c_int64()
    P = C.POINTER
    _check(ctx, lib().dtsph_neighbor_list(ctx, int(sim), off.ctypes.data_as(P(C.c_int64)), None, 0,
                                          C.byref(need)))
    idx = np.zeros(max(need.value, 1), dtype=np.int32)
    _check(ctx, lib().dtsph_neighbor_list(ctx, int(sim), off.ctypes.data_as(P(C.c_int64)),
                                          idx.ctypes.data_as(P(C.c_int32)), need.value,
                                          C.byref(need)))
    return off, idx[:need.value]


def dtsph_set_option(ctx, option: int, value: int) -> int:
    return _check(ctx, lib().dtsph_set_option(ctx, int(option), int(value)))


def dtsph_get_timing(ctx) -> dict:
    t = Timing()
    _check(ctx, lib().dtsph_get_timing(ctx, C.byref(t)))
    return t.as_dict()


def dtsph_autotune(ctx, repeats: int = 5) -> dict:
    r = TuneReport()
    _check(ctx, lib().dtsph_autotune(ctx, int(repeats), C.byref(r)))
    return r.as_dict()


def dtsph_get_info(ctx) -> dict:
    i = Info()
    _check(ctx, lib().dtsph_get_info(ctx, C.byref(i)))
    return i.as_dict()


def dtsph_workspace_bytes(ctx) -> int:
    b = C.c_size_t(0)
    _check(ctx, lib().dtsph_workspace_bytes(ctx, C.byref(b)))
    return int(b.value)


def dtsph_set_workspace(ctx, dev_ptr: int, nbytes: int) -> int:
    return _check(ctx, lib().dtsph_set_workspace(ctx, C.c_void_p(dev_ptr or None), int(nbytes)))


# ---- convenience wrapper over torch device tensors --------------------------------

class Sim:
    """One context over one or more problems (``inputs.Problem``), state in torch
    float64 device tensors in caller order."""

    def __init__(self, problems, precision: int = FP32, device: str = "cuda:0", static: bool = False):
        import torch

        self.torch = torch
        if not isinstance(problems, (list, tuple)):
            problems = [problems]
        self.problems = list(problems)
        self.device = torch.device(device)
        self.n_sims = len(self.problems)
        self.n = sum(p.n for p in self.problems)
        self.precision = precision
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
            create = dtsph_create_static if static else dtsph_create
            self.ctx = create([p.params for p in self.problems], [p.n_fluid for p in self.problems],
                              [p.n_wall for p in self.problems], precision, stream)
        z3 = lambda: torch.zeros((self.n, 3), dtype=torch.float64, device=self.device)
        z1 = lambda: torch.zeros((self.n,), dtype=torch.float64, device=self.device)
        self.t = dict(x=z3(), v=z3(), v_prev=z3(), p=z1(), x_iter=z3(), v_iter=z3(), p_iter=z1(),
                      dpdtau=z1())
        self.info = dtsph_get_info(self.ctx)
        self.set_state_from_problems()

    def close(self):
        if getattr(self, "ctx", None):
            dtsph_destroy(self.ctx)
            self.ctx = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def _view(self, keys) -> StateView:
        v = StateView()
        for k in keys:
            setattr(v, k, self.t[k].data_ptr())
        return v

    def _sync(self):
        self.torch.cuda.synchronize(self.device)

    def set_state(self, x, v, v_prev, p, loop: Optional[Dict[str, np.ndarray]] = None):
        T = self.torch
        for k, a in (("x", x), ("v", v), ("v_prev", v_prev), ("p", p)):
            self.t[k].copy_(T.as_tensor(np.ascontiguousarray(a, dtype=np.float64)))
        keys = ["x", "v", "v_prev", "p"]
        if loop is not None:
            for k in ("x_iter", "v_iter", "p_iter", "dpdtau"):
                self.t[k].copy_(T.as_tensor(np.ascontiguousarray(loop[k], dtype=np.float64)))
            keys += ["x_iter", "v_iter", "p_iter", "dpdtau"]
        self._sync()
        dtsph_set_state(self.ctx, self._view(keys))

    def set_state_from_problems(self, loop=None):
        cat = lambda f: np.concatenate([getattr(p, f) for p in self.problems])
        self.set_state(cat("x"), cat("v"), cat("v_prev"), cat("p"), loop)

    def get_state(self, loop: bool = False) -> Dict[str, np.ndarray]:
        keys = ["x", "v", "v_prev", "p"] + (["x_iter", "v_iter", "p_iter", "dpdtau"] if loop else [])
        dtsph_get_state(self.ctx, self._view(keys))
        return {k: self.t[k].cpu().numpy().copy() for k in keys}

    def build_cells(self):
        return dtsph_build_cells(self.ctx)

    def cell_layout(self):
        """Cell-ordered layout of the lists in use (keys, caller indices, cell starts)."""
        return dtsph_build_cells(self.ctx, (self.n, dtsph_get_info(self.ctx)["n_cells"]))

    def predict(self):
        return dtsph_predict(self.ctx)

    def pseudo_iterate(self, fixed_iters: int = 0):
        return dtsph_pseudo_iterate(self.ctx, fixed_iters, self.n_sims)

    def correct(self):
        return dtsph_correct(self.ctx)

    def step(self, n_steps: int = 1, reports: bool = True):
        return dtsph_step(self.ctx, n_steps, self.n_sims, reports)

    def neighbor_list(self, sim: int = -1):
        m = self.n if sim < 0 else self.problems[sim].n
        return dtsph_neighbor_list(self.ctx, m, sim)

    def set_option(self, option: int, value: int):
        return dtsph_set_option(self.ctx, option, value)

    def timing(self) -> dict:
        return dtsph_get_timing(self.ctx)

    def autotune(self, repeats: int = 5) -> dict:
        rep = dtsph_autotune(self.ctx, repeats)
        self.info = dtsph_get_info(self.ctx)
        return rep

    def use_workspace(self, tensor=None):
        """Move the context's device arrays into ``tensor`` (a torch uint8 device
        tensor of at least ``dtsph_workspace_bytes`` bytes, kept alive by this
        object), or back into library allocations with None."""
        if tensor is None:
            dtsph_set_workspace(self.ctx, 0, 0)
        else:
            dtsph_set_workspace(self.ctx, tensor.data_ptr(), tensor.numel() * tensor.element_size())
        self.workspace = tensor

    def sim_slices(self) -> List[slice]:
        out, o = [], 0
        for p in self.problems:
            out.append(slice(o, o + p.n))
            o += p.n
        return out
