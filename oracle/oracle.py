"""FP64 CPU oracle of the CSPH-TVD step (Khrapov & Khoperskov 2020) -- ctypes wrapper.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark call this module; the product path (the HIP library and its
Python binding) never imports it, and this module imports nothing from it.

The arithmetic lives in ``csph_oracle.c`` next to this file (plain C, FP64,
each stage a whole-grid loop); this wrapper only marshals numpy arrays.
Parity unpinned: the authors' own CSPH-TVD program, the intended exponent of
Eq. 4 and Eq. 7 without C_J (see the header of ``csph_oracle.c``).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csph_oracle.c")
_LIB = os.environ.get("CSPH_ORACLE_LIB") or os.path.join(_HERE, "libcsph_oracle.so")

SED_NONE, SED_GRASS, SED_EQ4 = 0, 1, 2
LIM_MINMOD, LIM_MC, LIM_SUPERBEE = 0, 1, 2
SPEEDS_DAVIS, SPEEDS_TWO_RAREFACTION = 0, 1
BC_WALL, BC_OPEN = 0, 1
BINDING_NAMES = ("h/(2vp)", "h/vs", "h^2/(2D)", "dt_max", "fixed")


# -O3 for the generic x86-64 AVX2/FMA level rather than -march=native: the
# library is built on one machine and may run on another host; contraction
# into FMA stays off, so each operation is rounded as the source writes it.
CFLAGS = ["-O3", "-march=x86-64-v3", "-ffp-contract=off", "-std=c11", "-fopenmp", "-fPIC",
          "-shared", "-Wall", "-Wno-unknown-pragmas"]


def compile_source(src: str, out: str) -> str:
    """Compile one oracle source file with gcc (CFLAGS: -O3, C11, OpenMP) into ``out``."""
    tmp = out + ".tmp"
    subprocess.check_call(["gcc"] + CFLAGS + [src, "-o", tmp, "-lm"])
    os.replace(tmp, out)
    return out


_SRC_F32 = os.path.join(_HERE, "csph_oracle_f32.c")
_LIB_F32 = os.path.join(_HERE, "libcsph_oracle_f32.so")


def build_f32(force: bool = True) -> str:
    """Compile the float32 evaluation of the oracle (csph_oracle_f32.c: the
    same source, every literal and operation in float32).  It only measures
    how far float32 rounding moves the FP64 answer; it is never a reference."""
    newest = max(os.path.getmtime(_SRC), os.path.getmtime(_SRC_F32))
    if force or not os.path.exists(_LIB_F32) or os.path.getmtime(_LIB_F32) < newest:
        tmp = _LIB_F32 + ".tmp"
        subprocess.check_call(["gcc"] + CFLAGS + ["-fsingle-precision-constant", _SRC_F32, "-o", tmp,
                                                  "-lm"])
        os.replace(tmp, _LIB_F32)
    return _LIB_F32


def build(force: bool = True) -> str:
    """Compile the oracle.  Returns the library path."""
    if os.environ.get("CSPH_ORACLE_LIB"):
        return _LIB
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        compile_source(_SRC, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("dx", C.c_double),
                ("bc", C.c_int32 * 4), ("g", C.c_double), ("cfl", C.c_double),
                ("eps", C.c_double), ("h_sed", C.c_double), ("dt_max", C.c_double),
                ("dt_min", C.c_double), ("s_rel", C.c_double), ("C_J", C.c_double),
                ("C_Sh", C.c_double), ("A_G", C.c_double), ("m_exp", C.c_double),
                ("sed_law", C.c_int32), ("limiter", C.c_int32), ("hll_speeds", C.c_int32),
                ("rain", C.c_double), ("coriolis", C.c_double), ("wind_x", C.c_double),
                ("wind_y", C.c_double), ("wind_coef", C.c_double), ("force_order", C.c_int32)]


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class _Inputs(C.Structure):
    _fields_ = [("nM", _dp), ("d50", _dp), ("psi", _dp), ("qb", _dp),
                ("n_inflow", C.c_int32), ("inflow_idx", _ip), ("inflow_w", _dp),
                ("Q_base", C.c_double), ("Q_peak", C.c_double), ("t_peak", C.c_double),
                ("t_sigma", C.c_double), ("beta", _dp)]


class _Info(C.Structure):
    _fields_ = [("dt", C.c_double), ("vp", C.c_double), ("vs", C.c_double), ("D", C.c_double),
                ("binding", C.c_int32), ("out_w", C.c_double), ("in_w", C.c_double),
                ("out_s", C.c_double), ("in_s", C.c_double), ("rain_in", C.c_double),
                ("absorbed", C.c_double)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = C.CDLL(_LIB)
        lib.orc_w.restype = C.c_double
        lib.orc_w.argtypes = [C.c_double, C.c_double]
        lib.orc_minmod.restype = C.c_double
        lib.orc_minmod.argtypes = [C.c_double, C.c_double]
        lib.orc_j0.restype = None
        lib.orc_j0.argtypes = [C.POINTER(_Params), C.c_double, C.c_double, C.c_double,
                               C.c_double, C.c_double, _dp, _dp]
        lib.orc_hll.restype = None
        lib.orc_hll.argtypes = [C.c_double] + [C.c_double] * 8 + [_dp]
        lib.orc_hll_v.restype = None
        lib.orc_hll_v.argtypes = [C.c_int, C.c_double] + [C.c_double] * 8 + [_dp]
        lib.orc_limiter.restype = C.c_double
        lib.orc_limiter.argtypes = [C.c_int, C.c_double, C.c_double]
        lib.orc_wave_speeds.restype = None
        lib.orc_wave_speeds.argtypes = [C.c_int, C.c_double] + [C.c_double] * 4 + [_dp, _dp]
        lib.orc_trr_star.restype = None
        lib.orc_trr_star.argtypes = [C.c_double] + [C.c_double] * 4 + [_dp, _dp]
        lib.orc_force.restype = C.c_int
        lib.orc_force.argtypes = [C.POINTER(_Params), _dp, _dp, _dp, _dp]
        lib.orc_hydrograph.restype = C.c_double
        lib.orc_hydrograph.argtypes = [C.POINTER(_Inputs), C.c_double]
        lib.orc_cfl.restype = C.c_int
        lib.orc_cfl.argtypes = [C.POINTER(_Params), C.POINTER(_Inputs), _dp, _dp, _dp,
                                _dp, _dp, _dp, _dp, _ip]
        lib.orc_step.restype = C.c_int
        lib.orc_step.argtypes = [C.POINTER(_Params), C.POINTER(_Inputs), _dp, _dp, _dp, _dp,
                                 C.c_double, C.c_double, C.POINTER(_Info)]
        lib.orc_threads.restype = C.c_int
        lib.orc_threads.argtypes = []
        lib.orc_set_threads.restype = None
        lib.orc_set_threads.argtypes = [C.c_int]
        lib.orc_volumes.restype = None
        lib.orc_volumes.argtypes = [C.POINTER(_Params), C.POINTER(_Inputs), _dp, _dp, _dp, _dp]
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code: int):
        names = {-1: "ERR_ARG", -3: "ERR_NONFINITE", -4: "ERR_DT_UNDERFLOW", -6: "ERR_CFL"}
        super().__init__(f"oracle step failed: {names.get(code, code)}")
        self.code = code


@dataclass
class Params:
    """Grid, boundary conditions and model constants (SI units)."""
    nx: int
    ny: int
    dx: float
    bc: tuple = (BC_WALL, BC_WALL, BC_WALL, BC_WALL)  # W, E, S, N
    g: float = 9.81
    cfl: float = 0.3
    eps: float = 1e-5
    h_sed: float = 1e-2
    dt_max: float = 1.0
    dt_min: float = 1e-9
    s_rel: float = 2.65
    C_J: float = 2.0
    C_Sh: float = 5.0
    A_G: float = 1e-3
    m_exp: float = 2.0
    sed_law: int = SED_EQ4
    limiter: int = LIM_MINMOD
    hll_speeds: int = SPEEDS_DAVIS
    rain: float = 0.0        # m/s
    coriolis: float = 0.0    # 1/s
    wind_x: float = 0.0      # m/s
    wind_y: float = 0.0
    wind_coef: float = 0.0   # (rho_air / rho_water) C_D
    force_order: int = 1     # Lagrangian force on cell values (1) or reconstructed states (2)

    def _c(self) -> _Params:
        p = _Params()
        p.nx, p.ny, p.dx = self.nx, self.ny, self.dx
        for k in range(4):
            p.bc[k] = int(self.bc[k])
        for name in ("g", "cfl", "eps", "h_sed", "dt_max", "dt_min", "s_rel", "C_J", "C_Sh",
                     "A_G", "m_exp", "rain", "coriolis", "wind_x", "wind_y", "wind_coef"):
            setattr(p, name, float(getattr(self, name)))
        p.sed_law = int(self.sed_law)
        p.limiter = int(self.limiter)
        p.hll_speeds = int(self.hll_speeds)
        p.force_order = int(self.force_order)
        return p


@dataclass
class Inputs:
    """Per-cell soil fields (scalars are broadcast), bed sources and inflow."""
    nM: object = 0.0
    d50: object = 5e-4
    psi: object = 0.4
    qb: object = None              # q_b^+ - q_b^- per cell (m/s) or None
    inflow_idx: object = None      # flat cell indices
    inflow_w: object = None        # weights, sum 1
    Q_base: float = 0.0
    Q_peak: float = 0.0
    t_peak: float = 0.0
    t_sigma: float = 1.0
    beta: object = None            # absorption coefficient per cell (1/s), scalar, or None
    _keep: list = field(default_factory=list, repr=False)

    def _c(self, n: int) -> _Inputs:
        def full(x):
            a = np.asarray(x, dtype=np.float64)
            a = np.full(n, float(a)) if a.ndim == 0 else np.array(a, dtype=np.float64).reshape(n)
            self._keep.append(a)
            return a.ctypes.data_as(_dp)
        ci = _Inputs()
        ci.nM, ci.d50, ci.psi = full(self.nM), full(self.d50), full(self.psi)
        ci.qb = full(self.qb) if self.qb is not None else _dp()
        ci.beta = full(self.beta) if self.beta is not None else _dp()
        if self.inflow_idx is not None and len(self.inflow_idx) > 0:
            idx = np.ascontiguousarray(self.inflow_idx, dtype=np.int32).reshape(-1)
            w = np.ascontiguousarray(self.inflow_w, dtype=np.float64).reshape(-1)
            self._keep += [idx, w]
            ci.n_inflow = idx.size
            ci.inflow_idx = idx.ctypes.data_as(_ip)
            ci.inflow_w = w.ctypes.data_as(_dp)
        else:
            ci.n_inflow = 0
        ci.Q_base, ci.Q_peak = float(self.Q_base), float(self.Q_peak)
        ci.t_peak, ci.t_sigma = float(self.t_peak), float(self.t_sigma)
        return ci


def _arr(a, n):
    a = np.ascontiguousarray(a, dtype=np.float64)
    assert a.size == n
    return a


class State:
    """FP64 state H, qx, qy, b (each [ny, nx]) plus time and accumulated balances."""

    def __init__(self, H, qx, qy, b, t: float = 0.0):
        self.H = np.array(H, dtype=np.float64, copy=True)
        self.qx = np.array(qx, dtype=np.float64, copy=True)
        self.qy = np.array(qy, dtype=np.float64, copy=True)
        self.b = np.array(b, dtype=np.float64, copy=True)
        self.t = float(t)
        self.step = 0
        self.out_w = self.in_w = self.out_s = self.in_s = 0.0
        self.rain_in = self.absorbed = 0.0
        self.last = None

    def copy(self) -> "State":
        s = State(self.H, self.qx, self.qy, self.b, self.t)
        s.step = self.step
        s.out_w, s.in_w, s.out_s, s.in_s = self.out_w, self.in_w, self.out_s, self.in_s
        s.rain_in, s.absorbed = self.rain_in, self.absorbed
        return s


def step(p: Params, inp: Inputs, s: State, dt_fixed: float = 0.0) -> dict:
    """Advance ``s`` by one CSPH-TVD step in place; returns the step record."""
    lib = _load()
    n = p.nx * p.ny
    cp, ci = p._c(), inp._c(n)
    info = _Info()
    for name in ("H", "qx", "qy", "b"):
        setattr(s, name, _arr(getattr(s, name), n).reshape(p.ny, p.nx))
    rc = lib.orc_step(C.byref(cp), C.byref(ci), s.H.ctypes.data_as(_dp),
                      s.qx.ctypes.data_as(_dp), s.qy.ctypes.data_as(_dp),
                      s.b.ctypes.data_as(_dp), s.t, float(dt_fixed), C.byref(info))
    inp._keep.clear()
    if rc != 0:
        raise OracleError(rc)
    s.t += info.dt
    s.step += 1
    s.out_w += info.out_w
    s.in_w += info.in_w
    s.out_s += info.out_s
    s.in_s += info.in_s
    s.rain_in += info.rain_in
    s.absorbed += info.absorbed
    rec = {k: getattr(info, k) for k, _ in _Info._fields_}
    s.last = rec
    return rec


def run(p: Params, inp: Inputs, s: State, nsteps: int, dt_fixed: float = 0.0) -> State:
    for _ in range(nsteps):
        step(p, inp, s, dt_fixed)
    return s


_lib_f32 = None


def run_f32(p: Params, inp: Inputs, s: State, nsteps: int, dt_fixed: float = 0.0) -> State:
    """``nsteps`` steps of the oracle evaluated in float32 arithmetic (see
    build_f32): the state is rounded to float32 before each step.  For
    measuring the conditioning of a problem only."""
    global _lib_f32
    if _lib_f32 is None:
        lib = C.CDLL(build_f32(force=False))
        lib.orcf_step.restype = C.c_int
        lib.orcf_step.argtypes = [C.POINTER(_Params), C.POINTER(_Inputs), _dp, _dp, _dp, _dp,
                                  C.c_double, C.c_double, C.POINTER(_Info)]
        lib.orcf_set_threads.restype = None
        lib.orcf_set_threads.argtypes = [C.c_int]
        _lib_f32 = lib
    _lib_f32.orcf_set_threads(threads())
    n = p.nx * p.ny
    for _ in range(nsteps):
        cp, ci = p._c(), inp._c(n)
        info = _Info()
        for name in ("H", "qx", "qy", "b"):
            setattr(s, name, _arr(getattr(s, name), n).reshape(p.ny, p.nx))
        rc = _lib_f32.orcf_step(C.byref(cp), C.byref(ci), s.H.ctypes.data_as(_dp),
                                s.qx.ctypes.data_as(_dp), s.qy.ctypes.data_as(_dp),
                                s.b.ctypes.data_as(_dp), s.t, float(dt_fixed), C.byref(info))
        inp._keep.clear()
        if rc != 0:
            raise OracleError(rc)
        s.t += info.dt
        s.step += 1
    return s


def cfl(p: Params, inp: Inputs, s: State) -> dict:
    """Eq. 7 time step and its three maxima for the state ``s``."""
    lib = _load()
    n = p.nx * p.ny
    cp, ci = p._c(), inp._c(n)
    dt, vp, vs, D = C.c_double(), C.c_double(), C.c_double(), C.c_double()
    bnd = C.c_int32()
    H, qx, qy = (_arr(a, n) for a in (s.H, s.qx, s.qy))
    rc = lib.orc_cfl(C.byref(cp), C.byref(ci), H.ctypes.data_as(_dp), qx.ctypes.data_as(_dp),
                     qy.ctypes.data_as(_dp), C.byref(dt), C.byref(vp), C.byref(vs),
                     C.byref(D), C.byref(bnd))
    inp._keep.clear()
    if rc != 0:
        raise OracleError(rc)
    return {"dt": dt.value, "vp": vp.value, "vs": vs.value, "D": D.value, "binding": bnd.value}


def volumes(p: Params, inp: Inputs, s: State):
    """(water volume, sediment volume) = (sum H dx^2, sum (1-psi) b dx^2)."""
    lib = _load()
    n = p.nx * p.ny
    cp, ci = p._c(), inp._c(n)
    vw, vs = C.c_double(), C.c_double()
    H, b = _arr(s.H, n), _arr(s.b, n)
    lib.orc_volumes(C.byref(cp), C.byref(ci), H.ctypes.data_as(_dp), b.ctypes.data_as(_dp),
                    C.byref(vw), C.byref(vs))
    inp._keep.clear()
    return vw.value, vs.value


def w(H: float, eps: float = 1e-5) -> float:
    return _load().orc_w(float(H), float(eps))


def minmod(a: float, b: float) -> float:
    return _load().orc_minmod(float(a), float(b))


def j0(p: Params, H, u, v, nM, d50):
    jx, jy = C.c_double(), C.c_double()
    cp = p._c()
    _load().orc_j0(C.byref(cp), float(H), float(u), float(v), float(nM), float(d50),
                   C.byref(jx), C.byref(jy))
    return jx.value, jy.value


def hll(g, HsL, uLnL, uLtL, unL, HsR, uLnR, uLtR, unR):
    f = (C.c_double * 3)()
    _load().orc_hll(float(g), float(HsL), float(uLnL), float(uLtL), float(unL), float(HsR),
                    float(uLnR), float(uLtR), float(unR), f)
    return tuple(f)


def force(p: Params, Hd, b):
    """The Lagrangian force per unit area (Sx, Sy) of depth Hd over bed b
    ([ny, nx] arrays), in the first- or second-order form of p."""
    Hd = np.ascontiguousarray(Hd, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    assert Hd.shape == (p.ny, p.nx) and b.shape == Hd.shape
    Sx = np.empty_like(Hd)
    Sy = np.empty_like(Hd)
    pc = p._c()
    rc = _load().orc_force(C.byref(pc), Hd.ctypes.data_as(_dp), b.ctypes.data_as(_dp),
                           Sx.ctypes.data_as(_dp), Sy.ctypes.data_as(_dp))
    if rc != 0:
        raise OracleError(rc)
    return Sx, Sy


def limiter(kind: int, a: float, b: float) -> float:
    return _load().orc_limiter(int(kind), float(a), float(b))


def hll_v(speeds, g, HsL, uLnL, uLtL, unL, HsR, uLnR, uLtR, unR):
    f = (C.c_double * 3)()
    _load().orc_hll_v(int(speeds), float(g), float(HsL), float(uLnL), float(uLtL), float(unL),
                      float(HsR), float(uLnR), float(uLtR), float(unR), f)
    return tuple(f)


def wave_speeds(kind, g, HsL, unL, HsR, unR):
    a, b = C.c_double(), C.c_double()
    _load().orc_wave_speeds(int(kind), float(g), float(HsL), float(unL), float(HsR), float(unR),
                            C.byref(a), C.byref(b))
    return a.value, b.value


def trr_star(g, HsL, unL, HsR, unR):
    u, c = C.c_double(), C.c_double()
    _load().orc_trr_star(float(g), float(HsL), float(unL), float(HsR), float(unR), C.byref(u),
                         C.byref(c))
    return u.value, c.value


def hydrograph(inp: Inputs, t: float) -> float:
    ci = _Inputs()
    ci.Q_base, ci.Q_peak = float(inp.Q_base), float(inp.Q_peak)
    ci.t_peak, ci.t_sigma = float(inp.t_peak), float(inp.t_sigma)
    return _load().orc_hydrograph(C.byref(ci), float(t))


def threads() -> int:
    """OpenMP threads the oracle's loops use."""
    return int(_load().orc_threads())


def set_threads(n: int) -> None:
    """Run the oracle's loops on n OpenMP threads from now on."""
    _load().orc_set_threads(int(n))
