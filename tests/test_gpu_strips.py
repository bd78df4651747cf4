"""The strip kernels (one wavefront per 58-column tile, rows marched in
registers, x neighbours by lane shifts) against the LDS tile kernels: every
strip height gives exactly the bits of the 64 x 8 tiles on walls, open sides,
per-cell soil, inflow and bed sources, ragged edges, grids narrower than one
strip, graph replay and eager launches, dry-tile skipping on and off."""
import copy

import numpy as np
import pytest

from paper_2103_15196_amd import workloads as W
from tests.gpu_common import run_gpu, say

pytestmark = pytest.mark.gpu

STRIPS = [(58, 8), (58, 16), (58, 32)]


def _same(a, b, what):
    (fa, sa), (fb, sb) = a, b
    for x, y, name in zip(fa, fb, ("h", "hu", "hv", "b")):
        assert np.array_equal(x, y), f"{what}: {name} differs"
    assert sa["t"] == sb["t"] and sa["step"] == sb["step"], what
    for k in ("water_volume", "water_boundary_out", "sed_boundary_out"):
        assert sa[k] == sb[k], f"{what}: {k}"


def _river():
    w = W.river_valley(n=200, ny=136, dx=5.0, amplitude=60.0, wavelength=500.0, width=40.0,
                       Q_base=20.0, Q_peak=200.0, t_peak=40.0, t_sigma=15.0)
    w.qb = np.zeros((w.ny, w.nx))
    w.qb[60:70, 100:110] = 2e-6
    return w.as_float32()


def _mixed_bc():
    f = W.dam_break_fractal(n=130, ny=98, dx=2.0, seed=9, relief=5.0, depth=4.0).as_float32()
    f.bc = (0, 1, 1, 0)
    return f


CASES = {
    "fractal_open_300x236": (lambda: W.dam_break_fractal(n=300, ny=236, dx=2.0, seed=7, relief=10.0,
                                                         depth=8.0).as_float32(), 200),
    "dam_break_walls_eq4_256x64": (lambda: W.dam_break_1d().as_float32(), 200),
    "river_inflow_soil_sources_200x136": (_river, 300),
    "fractal_mixed_bc_130x98": (_mixed_bc, 150),
    "narrow_40x90": (lambda: W.dam_break_fractal(n=40, ny=90, dx=1.0, seed=3, relief=2.0,
                                                 depth=2.0).as_float32(), 120),
    "one_row_96x1": (lambda: W.dam_break_1d(nx=96, ny=1, x_dam=40).as_float32(), 80),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_gpu_strips_equal_tiles(case):
    make, steps = CASES[case]
    w = make()
    ref = run_gpu(w, steps)
    for shape in STRIPS:
        say(f"strip {shape} on {case} ({w.nx}x{w.ny}, {steps} steps)")
        _same(run_gpu(w, steps, shape=shape), ref, f"{case} {shape}")


def test_gpu_strips_variants():
    """Dry-tile skipping off and eager launches give the same bits on strips."""
    from paper_2103_15196_amd import csph
    w = W.dam_break_fractal(n=400, ny=200, dx=2.0, seed=11, relief=10.0, depth=6.0).as_float32()
    w.bc = (0, 1, 1, 0)
    ref = run_gpu(w, 151)
    for flags in (0, csph.SW_FLAG_HGS | csph.SW_FLAG_NO_GRAPH, csph.SW_FLAG_HGS):
        say(f"strip (58, 16) flags {flags}")
        _same(run_gpu(w, 151, flags=flags, shape=(58, 16)), ref, f"flags {flags}")


@pytest.mark.parametrize("bc", [(0, 0, 0, 0), (1, 1, 1, 1)])
def test_gpu_strips_lake_at_rest_is_exact(bc):
    w = W.lake_at_rest(200, 130, dx=1.0, relief=3.0, level=2.0, bc=bc).as_float32()
    (h, hu, hv, b), _ = run_gpu(w, 300, shape=(58, 16))
    assert np.array_equal(h, w.H.astype(np.float32))
    assert np.all(hu == 0) and np.all(hv == 0)
    assert np.array_equal(b, w.b.astype(np.float32))


def test_gpu_strips_tiny_grids():
    """Grids of 1-3 cells per side (every lane but a few is halo)."""
    for nx, ny in ((3, 1), (2, 1), (3, 3), (1, 5)):
        H = np.zeros((ny, nx))
        H.flat[0] = 1.0
        z = np.zeros((ny, nx))
        w = W.Workload(name="t", nx=nx, ny=ny, dx=1.0, bc=(0, 0, 0, 0), H=H, qx=z, qy=z, b=z,
                       nM=0.0, d50=5e-4, psi=0.4, steps=1, cfl=0.9, sed_law=0)
        ref = run_gpu(w, 5, dt=0.05)
        for shape in STRIPS:
            _same(run_gpu(w, 5, dt=0.05, shape=shape), ref, f"{nx}x{ny} {shape}")


def test_gpu_strips_long_lists_take_several_passes():
    """8192 x 2048 cells: 58 x 8 strips make 36352 tiles.  With dry tiles
    skipped and every tile wet that is more than the stage grid's 8192
    workgroups of 4 wavefronts hold, so the Lagrangian and Euler kernels take
    their lists in two passes; a shorter list (the dam break's own dry
    regions, or one small wet block) fits one pass, and the Lagrangian stage
    then puts two wavefronts on each listed tile; with every tile listed (no
    skipping) one grid covers them all; 58 x 32 strips (4544 tiles) take one
    pass either way.  All give the bits of the 64 x 8 tiles."""
    from paper_2103_15196_amd import csph
    w = W.dam_break_fractal(n=8192, ny=2048, dx=2.0, seed=5, relief=10.0, depth=6.0).as_float32()
    wet = copy.deepcopy(w)
    wet.H = (w.H + 0.5).astype(np.float32).astype(np.float64)
    block = copy.deepcopy(w)
    block.H = np.zeros_like(w.H)
    block.H[1000:1100, 4000:4200] = w.H[1000:1100, 4000:4200] + 1.0
    block.H = block.H.astype(np.float32).astype(np.float64)
    for name, case, flags in (("all tiles", w, 0), ("all wet", wet, csph.SW_FLAG_HGS),
                              ("dry tiles skipped", w, csph.SW_FLAG_HGS),
                              ("one wet block", block, csph.SW_FLAG_HGS)):
        ref = run_gpu(case, 30, flags=flags, shape=(64, 8))
        for shape in ((58, 8), (58, 32)):
            say(f"strip {shape}, {name}, 8192x2048, 30 steps")
            _same(run_gpu(case, 30, flags=flags, shape=shape), ref, f"{name} {shape}")


def test_gpu_strips_pass_kernels_with_per_cell_soil_vs_tiles_and_oracle():
    """The kernels the 8192^2 river valley runs: 58 x 8 strips on more than
    32 Ki tiles (here 8192 x 2048: 36352 tiles; one grid of them with every
    tile listed, two passes with dry tiles skipped) with per-cell soil planes
    (Manning n, d50, psi), bed sources and an inflow hydrograph.  Both give
    the bits of the 64 x 8 LDS tiles; after 20 steps of an all-wet start
    every cell of h, hu, hv, b agrees with the FP64 oracle within the
    precision bounds."""
    from paper_2103_15196_amd import csph
    from oracle import oracle as O
    from tests.gpu_common import field_check, run_oracle
    O.build(force=False)
    w = W.river_valley(n=8192, ny=2048, dx=5.0, wavelength=3000.0, amplitude=300.0)
    rng = np.random.default_rng(17)
    w.nM = rng.uniform(0.02, 0.04, size=(w.ny, w.nx))
    w.qb = np.zeros((w.ny, w.nx))
    w.qb[900:940, 3000:3100] = 5e-6
    w.qb[100:110, 7000:7010] = -1e-6
    w.H = np.full((w.ny, w.nx), 0.5)
    w = w.as_float32()
    steps = 20
    say("river valley 8192x2048 per-cell soil: 64x8 tiles")
    ref = run_gpu(w, steps, shape=(64, 8))
    for flags in (csph.SW_FLAG_HGS, 0):
        say(f"  58x8 strips, flags {flags}")
        _same(run_gpu(w, steps, flags=flags), ref, f"flags {flags}")
    say("  oracle")
    p, inp, st = run_oracle(O, w, steps)
    f = field_check(ref[0], st, None, O.cfl(p, inp, st)["vs"])
    for name, r in f.items():
        say(f"  {name}: err {r['err']:.3e} (bound {r['bound']:.3e}) at {r['worst']}")
        assert r["err"] <= r["bound"], name
    assert abs(ref[1]["t"] - st.t) <= 1e-5 * st.t
