"""Thin ctypes binding of the C ABI in include/csph.h (libcsph.so).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  The functions carry the C names; ``Solver`` is a small convenience
wrapper over them.  Arrays may be numpy arrays (host) or torch tensors on the
GPU (device pointers, ordered on the solver's stream).  If the library is not
built this module raises at import time: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

# torch ships its own HIP runtime (same soname as the system one).  Loading
# torch first makes the dynamic loader bind this library to that runtime, so
# the process holds one HIP runtime and torch streams/pointers are valid here.
try:
    import torch  # noqa: F401
except ImportError:  # a plain C/numpy user gets the system runtime
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcsph.so")

SW_OK = 0
SW_ERR_ARG, SW_ERR_HIP, SW_ERR_NONFINITE, SW_ERR_DT_UNDERFLOW, SW_ERR_STATE, SW_ERR_CFL = (
    -1, -2, -3, -4, -5, -6)
ERROR_NAMES = {-1: "SW_ERR_ARG", -2: "SW_ERR_HIP", -3: "SW_ERR_NONFINITE",
               -4: "SW_ERR_DT_UNDERFLOW", -5: "SW_ERR_STATE", -6: "SW_ERR_CFL"}
SW_BC_WALL, SW_BC_OPEN = 0, 1
SW_SED_NONE, SW_SED_GRASS, SW_SED_EQ4 = 0, 1, 2
SW_PTR_HOST, SW_PTR_DEVICE = 0, 1
SW_FLAG_HGS, SW_FLAG_UNFUSED, SW_FLAG_NO_GRAPH, SW_FLAG_FORCE2 = 1, 2, 4, 8
SW_LIM_MINMOD, SW_LIM_MC, SW_LIM_SUPERBEE = 0, 1, 2
SW_HLL_DAVIS, SW_HLL_TWO_RAREFACTION = 0, 1


class sw_grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("dx", C.c_double), ("bc", C.c_int32 * 4)]


class sw_params(C.Structure):
    _fields_ = [("g", C.c_double), ("cfl", C.c_double), ("eps_dry", C.c_double),
                ("h_sed", C.c_double), ("dt_max", C.c_double), ("dt_min", C.c_double),
                ("s_rel", C.c_double), ("C_J", C.c_double), ("C_Sh", C.c_double),
                ("A_G", C.c_double), ("m_exp", C.c_double), ("sed_law", C.c_int32),
                ("flags", C.c_uint32), ("limiter", C.c_int32), ("hll_speeds", C.c_int32)]


SW_STEP_LOG = 1024


class sw_step_record(C.Structure):
    _fields_ = [("step", C.c_int64), ("t", C.c_double), ("dt", C.c_double), ("vp", C.c_double),
                ("vs", C.c_double), ("D", C.c_double), ("inflow", C.c_double),
                ("binding", C.c_int32), ("reserved", C.c_int32)]


class sw_sums(C.Structure):
    _fields_ = [("t", C.c_double), ("last_dt", C.c_double), ("water_volume", C.c_double),
                ("sediment_volume", C.c_double), ("water_boundary_out", C.c_double),
                ("water_source_in", C.c_double), ("sed_boundary_out", C.c_double),
                ("sed_source_in", C.c_double), ("vp", C.c_double), ("vs", C.c_double),
                ("D", C.c_double), ("step", C.c_int64), ("wet_cells", C.c_int64),
                ("active_tiles", C.c_int64), ("cells_lagrange", C.c_int64),
                ("cells_euler", C.c_int64), ("binding_term", C.c_int32), ("error", C.c_int32),
                ("graph_builds", C.c_int64), ("water_rain_in", C.c_double),
                ("water_absorbed", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_fp = C.POINTER(C.c_float)
_ctxp = C.c_void_p

# (name, restype, argtypes) of every exported entry point
SIGNATURES = [
    ("sw_default_params", None, [C.POINTER(sw_params)]),
    ("sw_create", C.c_int, [C.POINTER(sw_grid), C.POINTER(sw_params), C.c_void_p, C.POINTER(C.c_void_p)]),
    ("sw_destroy", C.c_int, [_ctxp]),
    ("sw_set_bed", C.c_int, [_ctxp, C.c_void_p, C.c_int]),
    ("sw_set_soil", C.c_int, [_ctxp, C.c_void_p, C.c_float, C.c_void_p, C.c_float, C.c_void_p,
                              C.c_float, C.c_int]),
    ("sw_set_state", C.c_int, [_ctxp, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    ("sw_set_inflow", C.c_int, [_ctxp, C.c_void_p, C.c_void_p, C.c_int32, C.c_double, C.c_double,
                                C.c_double, C.c_double]),
    ("sw_set_sed_sources", C.c_int, [_ctxp, C.c_void_p, C.c_void_p, C.c_int]),
    ("sw_set_time", C.c_int, [_ctxp, C.c_double, C.c_int64]),
    ("sw_set_forcing", C.c_int, [_ctxp, C.c_double, C.c_void_p, C.c_float, C.c_double, C.c_double,
                                 C.c_double, C.c_double, C.c_int]),
    ("sw_advance", C.c_int, [_ctxp, C.c_int32]),
    ("sw_advance_fixed_dt", C.c_int, [_ctxp, C.c_int32, C.c_double]),
    ("sw_advance_profiled", C.c_int, [_ctxp, C.c_int32, C.POINTER(C.c_double)]),
    ("sw_set_tile_shape", C.c_int, [_ctxp, C.c_int32, C.c_int32]),
    ("sw_autotune", C.c_int, [_ctxp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    ("sw_sync", C.c_int, [_ctxp]),
    ("sw_get_fields", C.c_int, [_ctxp, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    ("sw_get_sums", C.c_int, [_ctxp, C.POINTER(sw_sums)]),
    ("sw_step_bound", C.c_int, [_ctxp, C.POINTER(C.c_double)]),
    ("sw_get_step_log", C.c_int, [_ctxp, C.c_int32, C.POINTER(sw_step_record), C.POINTER(C.c_int32)]),
    ("sw_last_error", C.c_char_p, [_ctxp]),
    ("sw_save_begin", C.c_int, [_ctxp]),
    ("sw_save_wait", C.c_int, [_ctxp, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    ("sw_checkpoint_size", C.c_int, [_ctxp, C.POINTER(C.c_int64)]),
    ("sw_checkpoint_save", C.c_int, [_ctxp, C.c_void_p, C.c_int64]),
    ("sw_checkpoint_load", C.c_int, [_ctxp, C.c_void_p, C.c_int64]),
    ("swb_create", C.c_int, [C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p)]),
    ("swb_destroy", C.c_int, [C.c_void_p]),
    ("swb_set_tile_shape", C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    ("swb_advance", C.c_int, [C.c_void_p, C.c_int32]),
    ("swb_sync", C.c_int, [C.c_void_p]),
    ("swb_last_error", C.c_char_p, [C.c_void_p]),
    ("swb_autotune", C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    ("swb_get_fields", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_int]),
    ("swb_get_sums", C.c_int, [C.c_void_p, C.c_int32, C.POINTER(sw_sums)]),
    ("swb_set_state", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                C.c_int]),
    ("swb_set_bed", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int]),
    ("swb_set_soil", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_float, C.c_void_p,
                               C.c_float, C.c_void_p, C.c_float, C.c_int]),
    ("swb_set_inflow", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32,
                                 C.c_double, C.c_double, C.c_double, C.c_double]),
    ("swb_set_sed_sources", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int]),
    ("sw_replace_state", C.c_int, [_ctxp, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_double, C.c_int64]),
    ("sw_get_grid", C.c_int, [_ctxp, C.POINTER(sw_grid)]),
    ("sw_advance_noalloc", C.c_int, [C.POINTER(sw_grid), C.POINTER(sw_params), C.c_float, C.c_float,
                                     C.c_float, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_int32, C.c_double, C.c_double, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_char_p, C.c_int32]),
    ("sws_create", C.c_int, [C.POINTER(C.c_int32), C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)]),
    ("sws_destroy", C.c_int, [C.c_void_p]),
    ("sws_param_count", C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    ("sws_set_params", C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    ("sws_get_params", C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    ("sws_set_scales", C.c_int, [C.c_void_p, C.POINTER(C.c_float), C.POINTER(C.c_float)]),
    ("sws_forward", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                              C.c_int]),
    ("sws_train_step", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                 C.c_int32, C.c_float, C.POINTER(C.c_double), C.c_int]),
    ("sws_grad", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                           C.c_void_p, C.POINTER(C.c_double), C.c_int]),
    ("sws_advance", C.c_int, [C.c_void_p, _ctxp, C.c_int32, C.c_double, C.c_double,
                              C.POINTER(C.c_int32)]),
    ("sws_train", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                            C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    ("sws_advance_K", C.c_int, [C.c_void_p, _ctxp, C.c_int32, C.c_int32, C.c_double, C.c_double,
                                C.c_int32, C.c_double, C.c_void_p]),
    ("sws_last_error", C.c_char_p, [C.c_void_p]),
]


def load_library(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is not built (run __graft_entry__.build())")
    lib = C.CDLL(path)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = load_library()


class SwError(RuntimeError):
    def __init__(self, code, msg=""):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


def _check(ctx, rc):
    if rc != SW_OK:
        msg = lib.sw_last_error(ctx).decode() if ctx else ""
        raise SwError(rc, msg)


def default_params(**over) -> sw_params:
    p = sw_params()
    lib.sw_default_params(C.byref(p))
    for k, v in over.items():
        setattr(p, k, v)
    return p


def make_grid(nx, ny, dx, bc=(0, 0, 0, 0)) -> sw_grid:
    g = sw_grid()
    g.nx, g.ny, g.dx = int(nx), int(ny), float(dx)
    for k in range(4):
        g.bc[k] = int(bc[k])
    return g


def _ptr(a, n):
    """(pointer, ptr_kind, keep-alive) of a host numpy array or a CUDA torch tensor."""
    if a is None:
        return None, SW_PTR_HOST, None
    if hasattr(a, "data_ptr") and hasattr(a, "is_cuda"):
        if a.is_cuda:
            import torch
            assert a.dtype == torch.float32 and a.is_contiguous() and a.numel() == n
            return C.c_void_p(a.data_ptr()), SW_PTR_DEVICE, a
        a = a.numpy()
    arr = np.ascontiguousarray(a, dtype=np.float32).reshape(-1)
    assert arr.size == n, (arr.size, n)
    return arr.ctypes.data_as(C.c_void_p), SW_PTR_HOST, arr


class Solver:
    """Owns one sw_ctx; methods map one-to-one onto the C entry points."""

    def __init__(self, nx, ny, dx, bc=(0, 0, 0, 0), stream=None, **params):
        self.nx, self.ny = int(nx), int(ny)
        self.grid = make_grid(nx, ny, dx, bc)
        self.params = default_params(**params)
        h = C.c_void_p()
        s = C.c_void_p(stream) if stream is not None else None
        _check(None, lib.sw_create(C.byref(self.grid), C.byref(self.params), s, C.byref(h)))
        self.ctx = h

    def close(self):
        if self.ctx:
            lib.sw_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def n(self):
        return self.nx * self.ny

    def set_bed(self, b):
        p, kind, keep = _ptr(b, self.n)
        _check(self.ctx, lib.sw_set_bed(self.ctx, p, kind))

    def set_soil(self, manning=0.0, d50=5e-4, psi=0.4):
        args, kinds, keep = [], set(), []
        for v in (manning, d50, psi):
            if np.isscalar(v):
                args += [None, float(v)]
            else:
                p, kind, k = _ptr(v, self.n)
                args += [p, 0.0]
                kinds.add(kind)
                keep.append(k)
        assert len(kinds) <= 1, "mix of host and device soil arrays"
        kind = kinds.pop() if kinds else SW_PTR_HOST
        _check(self.ctx, lib.sw_set_soil(self.ctx, *args, kind))

    def set_state(self, h, hu, hv):
        (ph, kind, k1), (pu, _, k2), (pv, _, k3) = (_ptr(x, self.n) for x in (h, hu, hv))
        _check(self.ctx, lib.sw_set_state(self.ctx, ph, pu, pv, kind))

    def set_inflow(self, cells, weights, q_base, q_peak, t_peak, t_sigma):
        if cells is None or len(cells) == 0:
            _check(self.ctx, lib.sw_set_inflow(self.ctx, None, None, 0, 0.0, 0.0, 0.0, 1.0))
            return
        idx = np.ascontiguousarray(cells, dtype=np.int32)
        w = np.ascontiguousarray(weights, dtype=np.float32)
        _check(self.ctx, lib.sw_set_inflow(self.ctx, idx.ctypes.data_as(C.c_void_p),
                                           w.ctypes.data_as(C.c_void_p), int(idx.size),
                                           float(q_base), float(q_peak), float(t_peak),
                                           float(t_sigma)))

    def set_sed_sources(self, qb_plus=None, qb_minus=None):
        (pp, k1, a), (pm, k2, b) = _ptr(qb_plus, self.n), _ptr(qb_minus, self.n)
        kind = k1 if qb_plus is not None else k2
        _check(self.ctx, lib.sw_set_sed_sources(self.ctx, pp, pm, kind))

    def set_forcing(self, rain=0.0, beta=0.0, coriolis=0.0, wind_x=0.0, wind_y=0.0, wind_coef=0.0):
        """Rainfall (m/s), absorption coefficient beta (1/s, scalar or per-cell
        array), Coriolis parameter (1/s), wind (m/s) and its stress coefficient."""
        if np.isscalar(beta):
            pb, kind, keep = None, SW_PTR_HOST, None
            bs = float(beta)
        else:
            pb, kind, keep = _ptr(beta, self.n)
            bs = 0.0
        _check(self.ctx, lib.sw_set_forcing(self.ctx, float(rain), pb, bs, float(coriolis),
                                            float(wind_x), float(wind_y), float(wind_coef), kind))

    def set_time(self, t, step=0):
        _check(self.ctx, lib.sw_set_time(self.ctx, float(t), int(step)))

    def advance(self, nsteps, dt=None):
        if dt is None:
            _check(self.ctx, lib.sw_advance(self.ctx, int(nsteps)))
        else:
            _check(self.ctx, lib.sw_advance_fixed_dt(self.ctx, int(nsteps), float(dt)))

    def advance_profiled(self, nsteps):
        """Advance with per-kernel HIP events; returns (lagrange_ms, euler_ms) averages."""
        out = (C.c_double * 2)()
        _check(self.ctx, lib.sw_advance_profiled(self.ctx, int(nsteps), out))
        return out[0], out[1]

    def set_tile_shape(self, tx, ty):
        _check(self.ctx, lib.sw_set_tile_shape(self.ctx, int(tx), int(ty)))

    def autotune(self, nsteps=20):
        """Pick the fastest tile shape on the current state; returns (tile_x, tile_y)."""
        tx, ty = C.c_int32(), C.c_int32()
        _check(self.ctx, lib.sw_autotune(self.ctx, int(nsteps), C.byref(tx), C.byref(ty)))
        return tx.value, ty.value

    def sync(self):
        _check(self.ctx, lib.sw_sync(self.ctx))

    def get_fields(self, out=None):
        """Return (h, hu, hv, b) as float32 numpy arrays [ny, nx] (or fill torch tensors)."""
        if out is not None:
            ptrs = [_ptr(t, self.n) for t in out]
            _check(self.ctx, lib.sw_get_fields(self.ctx, *[p for p, _, _ in ptrs], SW_PTR_DEVICE))
            return out
        arrs = [np.empty((self.ny, self.nx), dtype=np.float32) for _ in range(4)]
        _check(self.ctx, lib.sw_get_fields(self.ctx, *[a.ctypes.data_as(C.c_void_p) for a in arrs],
                                           SW_PTR_HOST))
        return tuple(arrs)

    def get_sums(self) -> dict:
        s = sw_sums()
        _check(self.ctx, lib.sw_get_sums(self.ctx, C.byref(s)))
        return s.as_dict()

    def step_log(self, n=SW_STEP_LOG) -> list:
        """The records of the last min(n, steps since the state was set,
        SW_STEP_LOG) steps, oldest first (sw_get_step_log), as dicts."""
        buf = (sw_step_record * max(int(n), 1))()
        cnt = C.c_int32()
        _check(self.ctx, lib.sw_get_step_log(self.ctx, int(n), buf, C.byref(cnt)))
        return [{k: getattr(buf[q], k) for k, _ in sw_step_record._fields_ if k != "reserved"}
                for q in range(cnt.value)]

    def step_bound(self) -> float:
        """The Eq. 7 step bound of the current fields (sw_step_bound)."""
        dt = C.c_double()
        _check(self.ctx, lib.sw_step_bound(self.ctx, C.byref(dt)))
        return dt.value

    def save_begin(self):
        """Start copying the current state to the host on a second stream."""
        _check(self.ctx, lib.sw_save_begin(self.ctx))

    def save_wait(self):
        """(h, hu, hv, b, t, step) of the snapshot sw_save_begin took."""
        arrs = [np.empty((self.ny, self.nx), dtype=np.float32) for _ in range(4)]
        t, step = C.c_double(), C.c_int64()
        _check(self.ctx, lib.sw_save_wait(self.ctx, *[a.ctypes.data_as(C.c_void_p) for a in arrs],
                                          C.byref(t), C.byref(step)))
        return (*arrs, t.value, step.value)

    def checkpoint(self) -> np.ndarray:
        """The solver's whole state as a host blob (uint8 array) for a later restore."""
        n = C.c_int64()
        _check(self.ctx, lib.sw_checkpoint_size(self.ctx, C.byref(n)))
        buf = np.empty(n.value, np.uint8)
        _check(self.ctx, lib.sw_checkpoint_save(self.ctx, buf.ctypes.data, n.value))
        return buf

    def restore(self, blob) -> None:
        """Continue from a blob written by checkpoint() (same grid and inputs)."""
        a = np.ascontiguousarray(blob, dtype=np.uint8)
        _check(self.ctx, lib.sw_checkpoint_load(self.ctx, a.ctypes.data, a.size))

    def reset(self, w):
        """Restart from workload ``w``'s initial bed and state (time back to 0).
        The library's set-up of the new state (its Eq. 7 maxima and wet-tile
        flags) runs here too, so the next advance launches steps only."""
        self.set_bed(w.b)
        self.set_state(w.H, w.qx, w.qy)
        self.advance(0)

    def load_workload(self, w):
        """Upload a paper_2103_15196_amd.workloads.Workload (bed, soil, state, sources)."""
        self.set_bed(w.b)
        self.set_soil(w.nM, w.d50, w.psi)
        if w.qb is not None:
            self.set_sed_sources(np.maximum(w.qb, 0), np.maximum(-np.asarray(w.qb), 0))
        if w.inflow_idx is not None:
            self.set_inflow(w.inflow_idx, w.inflow_w, w.Q_base, w.Q_peak, w.t_peak, w.t_sigma)
        self.set_state(w.H, w.qx, w.qy)


def solver_for(w, stream=None, **params) -> Solver:
    """A Solver loaded with workload ``w`` (its grid, boundary kinds, CFL and law)."""
    kw = dict(cfl=w.cfl, sed_law=w.sed_law)
    kw.update(params)
    s = Solver(w.nx, w.ny, w.dx, w.bc, stream=stream, **kw)
    s.load_workload(w)
    return s


SW_NOALLOC_SCRATCH_BYTES = 72 << 20


def advance_noalloc(grid, params, manning, d50, psi, h, hu, hv, b, nsteps, dt_fixed=0.0, t0=0.0,
                    t_out=None, err_out=None, stream=None):
    """sw_advance_noalloc on device tensors h, hu, hv, b ([ny, nx] float32,
    updated in place); t_out (float64) and err_out (int32) are optional
    one-element device tensors.  Raises SwError on a non-zero return."""
    ptrs = []
    for a in (h, hu, hv, b):
        if a is None:
            ptrs.append(None)
            continue
        assert a.is_cuda and a.is_contiguous() and a.numel() == grid.nx * grid.ny
        ptrs.append(C.c_void_p(a.data_ptr()))
    tp = C.c_void_p(t_out.data_ptr()) if t_out is not None else None
    ep = C.c_void_p(err_out.data_ptr()) if err_out is not None else None
    msg = C.create_string_buffer(256)
    rc = lib.sw_advance_noalloc(C.byref(grid), C.byref(params), float(manning), float(d50),
                                float(psi), *ptrs, int(nsteps), float(dt_fixed), float(t0), tp, ep,
                                C.c_void_p(stream) if stream is not None else None, msg, 256)
    if rc != SW_OK:
        raise SwError(rc, msg.value.decode())


def _bcheck(b, rc):
    if rc != SW_OK:
        msg = lib.swb_last_error(b).decode() if b else ""
        raise SwError(rc, msg)


class Batch:
    """Owns one swb_ctx over existing Solver members (which it keeps alive)."""

    def __init__(self, members):
        self.members = list(members)
        arr = (C.c_void_p * len(self.members))(*[m.ctx for m in self.members])
        h = C.c_void_p()
        _bcheck(None, lib.swb_create(len(self.members), arr, C.byref(h)))
        self.ctx = h

    def close(self):
        if self.ctx:
            lib.swb_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tile_shape(self, tx, ty):
        _bcheck(self.ctx, lib.swb_set_tile_shape(self.ctx, int(tx), int(ty)))

    def advance(self, nsteps):
        _bcheck(self.ctx, lib.swb_advance(self.ctx, int(nsteps)))

    def sync(self):
        _bcheck(self.ctx, lib.swb_sync(self.ctx))

    def autotune(self, nsteps=10):
        """Pick the fastest tile shape for the batch from the current states."""
        tx, ty = C.c_int32(), C.c_int32()
        _bcheck(self.ctx, lib.swb_autotune(self.ctx, int(nsteps), C.byref(tx), C.byref(ty)))
        return tx.value, ty.value

    def get_fields(self, m):
        """Member m's (h, hu, hv, b) as float32 numpy arrays [ny, nx]."""
        s = self.members[m]
        arrs = [np.empty((s.ny, s.nx), dtype=np.float32) for _ in range(4)]
        _bcheck(self.ctx, lib.swb_get_fields(self.ctx, int(m),
                                             *[a.ctypes.data_as(C.c_void_p) for a in arrs],
                                             SW_PTR_HOST))
        return tuple(arrs)

    def get_sums(self, m) -> dict:
        out = sw_sums()
        _bcheck(self.ctx, lib.swb_get_sums(self.ctx, int(m), C.byref(out)))
        return out.as_dict()

    def set_state(self, m, h, hu, hv):
        n = self.members[m].n
        (ph, kind, k1), (pu, _, k2), (pv, _, k3) = (_ptr(x, n) for x in (h, hu, hv))
        _bcheck(self.ctx, lib.swb_set_state(self.ctx, int(m), ph, pu, pv, kind))

    def set_bed(self, m, b):
        p, kind, keep = _ptr(b, self.members[m].n)
        _bcheck(self.ctx, lib.swb_set_bed(self.ctx, int(m), p, kind))


def _scheck(h, rc):
    if rc != SW_OK:
        msg = lib.sws_last_error(h).decode() if h else ""
        raise SwError(rc, msg)


class sws_train_cfg(C.Structure):
    _fields_ = [("steps", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float), ("seed", C.c_uint64)]


class sws_train_report(C.Structure):
    _fields_ = [("first_loss", C.c_double), ("final_loss", C.c_double), ("steps", C.c_int32)]


class sws_stats(C.Structure):
    _fields_ = [("calls", C.c_int32), ("kept", C.c_int32), ("fallbacks_volume", C.c_int32),
                ("fallbacks_residual", C.c_int32), ("checks", C.c_int32),
                ("max_volume_drift", C.c_double), ("max_residual", C.c_double),
                ("fallbacks_stability", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Surrogate:
    """The convolutional surrogate (BF16 matrix-core convolutions): widths
    `channels` (5 inputs ... 4 outputs); parameters as one FP32 vector (per
    layer W[c_out][c_in][3][3] then b[c_out])."""

    def __init__(self, channels, stream=None):
        self.channels = [int(c) for c in channels]
        arr = (C.c_int32 * len(self.channels))(*self.channels)
        h = C.c_void_p()
        _scheck(None, lib.sws_create(arr, len(self.channels) - 1, stream, C.byref(h)))
        self.ctx = h
        n = C.c_int64()
        _scheck(self.ctx, lib.sws_param_count(self.ctx, C.byref(n)))
        self.nparam = n.value

    def close(self):
        if self.ctx:
            lib.sws_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, p):
        a = np.ascontiguousarray(p, dtype=np.float32).reshape(-1)
        assert a.size == self.nparam
        _scheck(self.ctx, lib.sws_set_params(self.ctx, a.ctypes.data, SW_PTR_HOST))

    def get_params(self):
        a = np.empty(self.nparam, np.float32)
        _scheck(self.ctx, lib.sws_get_params(self.ctx, a.ctypes.data, SW_PTR_HOST))
        return a

    def set_scales(self, in_scale, out_scale):
        i = (C.c_float * 5)(*[float(v) for v in in_scale])
        o = (C.c_float * 4)(*[float(v) for v in out_scale])
        _scheck(self.ctx, lib.sws_set_scales(self.ctx, i, o))

    def forward(self, x):
        """x: [nimg, 5, ny, nx] -> [nimg, 4, ny, nx] (host arrays)."""
        x = np.ascontiguousarray(x, dtype=np.float32)
        nimg, c, ny, nx = x.shape
        assert c == 5
        y = np.empty((nimg, 4, ny, nx), np.float32)
        _scheck(self.ctx, lib.sws_forward(self.ctx, x.ctypes.data, y.ctypes.data, nimg, nx, ny,
                                          SW_PTR_HOST))
        return y

    def grad(self, x, target):
        """(gradient vector, loss) without an update."""
        x = np.ascontiguousarray(x, dtype=np.float32)
        t = np.ascontiguousarray(target, dtype=np.float32)
        nimg, _, ny, nx = x.shape
        g = np.empty(self.nparam, np.float32)
        loss = C.c_double()
        _scheck(self.ctx, lib.sws_grad(self.ctx, x.ctypes.data, t.ctypes.data, nimg, nx, ny,
                                       g.ctypes.data, C.byref(loss), SW_PTR_HOST))
        return g, loss.value

    def train_step(self, x, target, lr):
        x = np.ascontiguousarray(x, dtype=np.float32)
        t = np.ascontiguousarray(target, dtype=np.float32)
        nimg, _, ny, nx = x.shape
        loss = C.c_double()
        _scheck(self.ctx, lib.sws_train_step(self.ctx, x.ctypes.data, t.ctypes.data, nimg, nx, ny,
                                             float(lr), C.byref(loss), SW_PTR_HOST))
        return loss.value

    def train(self, x, target, steps, batch, lr, seed=0, keep_losses=False):
        """sws_train on scaled pairs x [n, 5, ny, nx], target [n, 4, ny, nx]:
        returns (report dict, per-step losses or None)."""
        x = np.ascontiguousarray(x, dtype=np.float32)
        t = np.ascontiguousarray(target, dtype=np.float32)
        npairs, _, ny, nx = x.shape
        cfg = sws_train_cfg(int(steps), int(batch), float(lr), int(seed))
        rep = sws_train_report()
        losses = np.empty(int(steps), np.float32) if keep_losses else None
        _scheck(self.ctx, lib.sws_train(self.ctx, x.ctypes.data, t.ctypes.data, npairs, nx, ny,
                                        C.byref(cfg), C.byref(rep),
                                        losses.ctypes.data if losses is not None else None,
                                        SW_PTR_HOST))
        return {"first_loss": rep.first_loss, "final_loss": rep.final_loss, "steps": rep.steps}, losses

    def advance_k(self, solver, n_calls, k, dt, max_drift=1e-5, check_every=0, max_err=5e-3):
        """sws_advance_K: n_calls surrogate calls with the conservation and
        residual checks; returns the stats dict."""
        st = sws_stats()
        _scheck(self.ctx, lib.sws_advance_K(self.ctx, solver.ctx, int(n_calls), int(k), float(dt),
                                            float(max_drift), int(check_every), float(max_err),
                                            C.byref(st)))
        return st.as_dict()

    def advance(self, solver, k, dt, max_drift=1e-5):
        """k steps of `solver` by the surrogate (or by the solver if the water
        volume would change by more than max_drift); returns True if the
        surrogate's prediction was kept."""
        used = C.c_int32()
        _scheck(self.ctx, lib.sws_advance(self.ctx, solver.ctx, int(k), float(dt), float(max_drift),
                                          C.byref(used)))
        return bool(used.value)
