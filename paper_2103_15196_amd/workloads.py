"""Seeded synthetic workloads for the CSPH-TVD step.

This module only draws inputs: terrains, initial water, soil fields, inflow
cells and hydrographs.  It holds none of the method's arithmetic, and both the
HIP path and the CPU reference take their inputs from it.  Every generator is
deterministic in its seed (numpy PCG64).

The paper's own workload, the Volga-Akhtuba floodplain (Section 3: 1024^2 to
4096^2 grids, a mostly dry floodplain with river channels, a spring flood),
is a dataset that is not available; these terrains stand in for its shape.

Fields are float64 arrays of shape [ny, nx] (x fastest).  Sides are indexed
W=0, E=1, S=2, N=3; boundary kinds WALL=0, OPEN=1; sediment laws NONE=0,
GRASS=1, EQ4=2.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

WALL, OPEN = 0, 1
SED_NONE, SED_GRASS, SED_EQ4 = 0, 1, 2


@dataclass
class Workload:
    """One scenario: grid, boundary kinds, model constants and initial fields."""
    name: str
    nx: int
    ny: int
    dx: float
    bc: tuple
    H: np.ndarray
    qx: np.ndarray
    qy: np.ndarray
    b: np.ndarray
    nM: object          # scalar or [ny, nx]
    d50: object         # scalar or [ny, nx]
    psi: object         # scalar or [ny, nx]
    steps: int
    cfl: float = 0.3
    sed_law: int = SED_EQ4
    qb: Optional[np.ndarray] = None
    inflow_idx: Optional[np.ndarray] = None
    inflow_w: Optional[np.ndarray] = None
    Q_base: float = 0.0
    Q_peak: float = 0.0
    t_peak: float = 0.0
    t_sigma: float = 1.0
    extra: dict = field(default_factory=dict)

    @property
    def cells(self) -> int:
        return self.nx * self.ny

    def as_float32(self) -> "Workload":
        """Same scenario with every field rounded to float32 (then held as
        float64), so an FP32 and an FP64 solver start from identical values."""
        def r(a):
            if a is None or np.isscalar(a):
                return None if a is None else float(np.float32(a))
            return np.asarray(a, dtype=np.float32).astype(np.float64)
        w = Workload(**{k: getattr(self, k) for k in self.__dataclass_fields__})
        for k in ("H", "qx", "qy", "b", "nM", "d50", "psi", "qb", "inflow_w"):
            setattr(w, k, r(getattr(self, k)))
        w.dx = float(np.float32(self.dx))
        return w


def fractal_surface(nx: int, ny: int, seed: int, relief: float) -> np.ndarray:
    """Gaussian random surface with power spectrum ~ |k|^-2 (amplitude ~ |k|^-1),
    the k = 0 mode removed, rescaled so that max - min = relief and min = 0."""
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal((ny, nx))
    F = np.fft.rfft2(noise)
    ky = np.fft.fftfreq(ny)[:, None]
    kx = np.fft.rfftfreq(nx)[None, :]
    k = np.sqrt(kx * kx + ky * ky)
    amp = np.zeros_like(k)
    amp[k > 0] = 1.0 / k[k > 0]
    surf = np.fft.irfft2(F * amp, s=(ny, nx))
    surf -= surf.min()
    span = surf.max()
    return surf * (relief / span) if span > 0 else surf


def dam_break_1d(nx: int = 256, ny: int = 64, dx: float = 1.0, h_left: float = 2.0,
                 h_right: float = 0.5, x_dam: int = 128, manning: float = 0.02,
                 sediment: bool = True, bc=(WALL, WALL, WALL, WALL), steps: int = 200,
                 cfl: float = 0.3) -> Workload:
    """Dam break on a flat erodible bed: depth h_left for cells i < x_dam and
    h_right beyond, still water, psi = 0.4, d50 = 0.5 mm (the 256 x 64 case)."""
    H = np.full((ny, nx), h_right, dtype=np.float64)
    H[:, :x_dam] = h_left
    z = np.zeros((ny, nx))
    return Workload(name=f"dam_break_{nx}x{ny}", nx=nx, ny=ny, dx=dx, bc=tuple(bc), H=H,
                    qx=z.copy(), qy=z.copy(), b=z.copy(), nM=manning, d50=5e-4, psi=0.4,
                    steps=steps, cfl=cfl, sed_law=SED_EQ4 if sediment else SED_NONE)


def dam_break_fractal(n: int = 2048, dx: float = 2.0, seed: int = 2, relief: float = 10.0,
                      dam_height: float = 1.0, depth: float = 8.0, manning: float = 0.03,
                      d50: float = 5e-4, psi: float = 0.4, steps: int = 1000,
                      cfl: float = 0.3, ny: Optional[int] = None,
                      sed_law: int = SED_GRASS) -> Workload:
    """2-D dam break over a seeded fractal bed (spectral slope -2): a dam line
    `dam_height` above the terrain on column n/4, a reservoir upstream whose
    flat surface sits `depth` above the mean upstream bed, dry downstream,
    open boundaries on all sides.  No grain size is part of this scenario, so
    the bedload is the Grass law (A_G = 0.001, m = 2); d50 only sets the
    Shamov critical speed."""
    nx = n
    ny = n if ny is None else ny
    b = fractal_surface(nx, ny, seed, relief)
    i_dam = nx // 4
    b[:, i_dam] += dam_height
    zeta_r = b[:, :i_dam].mean() + depth
    H = np.zeros((ny, nx))
    H[:, :i_dam] = np.maximum(0.0, zeta_r - b[:, :i_dam])
    z = np.zeros((ny, nx))
    return Workload(name=f"dam_break_fractal_{nx}x{ny}", nx=nx, ny=ny, dx=dx,
                    bc=(OPEN, OPEN, OPEN, OPEN), H=H, qx=z.copy(), qy=z.copy(), b=b,
                    nM=manning, d50=d50, psi=psi, steps=steps, cfl=cfl, sed_law=sed_law,
                    extra={"seed": seed, "i_dam": i_dam, "zeta_r": zeta_r})


def river_valley(n: int = 8192, dx: float = 5.0, seed: int = 3, relief: float = 20.0,
                 slope: float = 1e-3, amplitude: float = 600.0, wavelength: float = 6000.0,
                 depth: float = 5.0, width: float = 200.0, manning: float = 0.03,
                 Q_base: float = 100.0, Q_peak: float = 2000.0, t_peak: float = 120.0,
                 t_sigma: float = 40.0, steps: int = 2000, cfl: float = 0.3,
                 ny: Optional[int] = None) -> Workload:
    """River valley: fractal terrain (relief `relief`) on a regional slope
    falling along x, a meandering parabolic channel carved along
    y_c(x) = Ly/2 + amplitude sin(2 pi x / wavelength), per-cell d50 ~ U[0.2, 2] mm
    and psi ~ U[0.3, 0.45], an inflow hydrograph on the x = 0 channel cells
    (Q_base + Q_peak exp(-(t-t_peak)^2 / (2 t_sigma^2)) m^3/s), open at x = max,
    walls elsewhere, initially dry."""
    nx = n
    ny = n if ny is None else ny
    b = fractal_surface(nx, ny, seed, relief)
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dx
    b += slope * (x.max() - x)[None, :]
    yc = 0.5 * ny * dx + amplitude * np.sin(2.0 * np.pi * x / wavelength)
    dist = np.abs(y[:, None] - yc[None, :])
    half = 0.5 * width
    carve = np.where(dist < half, depth * (1.0 - (dist / half) ** 2), 0.0)
    b -= carve
    rng = np.random.default_rng(seed + 7919)
    d50 = rng.uniform(0.2e-3, 2.0e-3, size=(ny, nx))
    psi = rng.uniform(0.30, 0.45, size=(ny, nx))
    rows = np.nonzero(dist[:, 0] < half)[0]
    inflow_idx = (rows * nx + 0).astype(np.int32)
    wts = carve[rows, 0]
    wts = wts / wts.sum()
    z = np.zeros((ny, nx))
    return Workload(name=f"river_valley_{nx}x{ny}", nx=nx, ny=ny, dx=dx,
                    bc=(WALL, OPEN, WALL, WALL), H=z.copy(), qx=z.copy(), qy=z.copy(), b=b,
                    nM=manning, d50=d50, psi=psi, steps=steps, cfl=cfl, sed_law=SED_EQ4,
                    inflow_idx=inflow_idx, inflow_w=wts, Q_base=Q_base, Q_peak=Q_peak,
                    t_peak=t_peak, t_sigma=t_sigma, extra={"seed": seed})


def ensemble(count: int = 64, seed0: int = 1000, n_min: int = 256, n_max: int = 1536,
             steps: int = 1000, size_step: int = 1) -> list:
    """Ensemble of uneven dam-break scenarios: member k uses seed seed0 + k, a
    square side drawn uniformly from [n_min, n_max] (multiples of size_step),
    its own fractal bed (10 m relief), reservoir depth U[1, 10] m and Manning n
    U[0.015, 0.05]."""
    members = []
    for k in range(count):
        rng = np.random.default_rng(seed0 + k)
        n = int(rng.integers(n_min // size_step, n_max // size_step + 1)) * size_step
        depth = float(rng.uniform(1.0, 10.0))
        manning = float(rng.uniform(0.015, 0.05))
        w = dam_break_fractal(n=n, dx=2.0, seed=seed0 + k, relief=10.0, dam_height=1.0,
                              depth=depth, manning=manning, steps=steps)
        w.name = f"ensemble_{k}_{n}"
        w.extra.update({"member": k, "depth": depth})
        members.append(w)
    return members


def lake_at_rest(nx: int, ny: int, dx: float = 1.0, seed: int = 11, relief: float = 3.0,
                 level: float = 2.0, bc=(WALL, WALL, WALL, WALL)) -> Workload:
    """Still water with a flat surface `level` over a fractal bed whose highest
    parts emerge as dry islands."""
    b = fractal_surface(nx, ny, seed, relief)
    H = np.maximum(0.0, level - b)
    z = np.zeros((ny, nx))
    return Workload(name=f"lake_{nx}x{ny}", nx=nx, ny=ny, dx=dx, bc=tuple(bc), H=H,
                    qx=z.copy(), qy=z.copy(), b=b, nM=0.03, d50=5e-4, psi=0.4, steps=100)
