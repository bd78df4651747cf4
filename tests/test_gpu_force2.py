"""The second-order Lagrangian force on the GPU (SW_FLAG_FORCE2: hydrostatic
faces on states reconstructed with the TVD limiter, plus the centred
bed-slope term; a reading of the Lagrangian stage of Section 3) against the
FP64 oracle run with force_order = 2, and its structure: every strip height,
one grid and passes, dry-tile skipping on and off give the same bits, the
lake at rest stays still, a batch member equals the member alone, and the
shapes and paths the flag is not built into are refused."""
import copy

import numpy as np
import pytest

from paper_2103_15196_amd import workloads as W
from tests.gpu_common import compare, run_gpu, run_oracle, say, torch_stream
from tests.test_gpu_parity import _check

pytestmark = pytest.mark.gpu


def _f2(hgs=True):
    from paper_2103_15196_amd import csph
    return csph.SW_FLAG_FORCE2 | (csph.SW_FLAG_HGS if hgs else 0)


@pytest.fixture(scope="module")
def O():
    from oracle import oracle as O
    O.build(force=False)
    return O


@pytest.mark.parametrize("limiter", [0, 1])
def test_gpu_force2_dam_break_256x64(O, limiter):
    """The 256 x 64 dam break (walls, Eq. 4 bedload), 200 steps: every cell
    at the flat bounds, with minmod and with MC reconstructions."""
    w = W.dam_break_1d().as_float32()
    say(f"case force2 limiter {limiter}: dam break 256x64 200 steps")
    res = compare(O, w, run_gpu(w, 200, flags=_f2(), limiter=limiter),
                  run_oracle(O, w, 200, force_order=2, limiter=limiter))
    _check(res)


def test_gpu_force2_fractal_dam_break_ragged(O):
    """Fractal bed, open sides, wet/dry fronts, ragged 300 x 236 grid, 500
    steps; cells ill-conditioned at float32 precision are counted apart."""
    w = W.dam_break_fractal(n=300, ny=236, dx=2.0, seed=7, relief=10.0, depth=8.0).as_float32()
    say("case force2: fractal dam break 300x236 500 steps")
    over = dict(force_order=2)
    res = compare(O, w, run_gpu(w, 500, flags=_f2()), run_oracle(O, w, 500, **over), spread=True,
                  steps=500, over=over)
    _check(res)


def test_gpu_force2_river_valley(O):
    """Inflow hydrograph, per-cell d50 and psi, walls + one open side, bed
    sources (the per-cell-soil kernels), 600 steps."""
    w = W.river_valley(n=200, ny=136, dx=5.0, amplitude=60.0, wavelength=500.0, width=40.0,
                       Q_base=20.0, Q_peak=200.0, t_peak=40.0, t_sigma=15.0)
    w.qb = np.zeros((w.ny, w.nx))
    w.qb[60:70, 100:110] = 2e-6
    w = w.as_float32()
    say("case force2: river valley 200x136 600 steps")
    over = dict(force_order=2)
    gpu = run_gpu(w, 600, flags=_f2())
    res = compare(O, w, gpu, run_oracle(O, w, 600, **over), spread=True, steps=600, over=over)
    _check(res)
    assert gpu[1]["wet_cells"] > 100


def test_gpu_force2_strips_skipping_and_rest_are_bitwise():
    """58 x 8, 16 and 32 strips and dry-tile skipping off give the bits of
    58 x 8 with skipping; the force differs from the first-order one; a lake
    at rest over an uneven bed with islands stays bit for bit still."""
    w = W.dam_break_fractal(n=130, ny=98, dx=2.0, seed=3, relief=6.0, depth=5.0).as_float32()
    w.bc = (0, 1, 1, 0)
    say("case force2 structure: fractal 130x98 150 steps")
    ref, rs = run_gpu(w, 150, flags=_f2())
    for shape, hgs in (((58, 16), True), ((58, 32), True), ((58, 8), False)):
        f, s = run_gpu(w, 150, flags=_f2(hgs), shape=shape)
        for a, b in zip(f, ref):
            assert np.array_equal(a, b), (shape, hgs)
        assert s["t"] == rs["t"]
    first, _ = run_gpu(w, 150)
    assert not np.array_equal(first[0], ref[0])
    lake = W.lake_at_rest(120, 70).as_float32()
    (h, hu, hv, b), _ = run_gpu(lake, 300, flags=_f2())
    assert np.array_equal(h, np.asarray(lake.H, np.float32))
    assert not hu.any() and not hv.any()


def test_gpu_force2_one_grid_and_passes():
    """8192 x 2048 cells (36352 strip tiles of 58 x 8): with skipping the
    stage kernels take their lists in passes, without it one grid; 58 x 32
    strips (4544 tiles) one pass.  All give the same bits, on an all-wet
    fractal dam break."""
    w = W.dam_break_fractal(n=8192, ny=2048, dx=2.0, seed=5, relief=10.0, depth=6.0).as_float32()
    w.H = (w.H + 0.5).astype(np.float32).astype(np.float64)
    say("case force2: 8192x2048 all wet 30 steps, passes")
    ref, _ = run_gpu(w, 30, flags=_f2())
    for shape, hgs in (((58, 8), False), ((58, 32), True)):
        say(f"  {shape} skipping {hgs}")
        f, _ = run_gpu(w, 30, flags=_f2(hgs), shape=shape)
        for a, b in zip(f, ref):
            assert np.array_equal(a, b), (shape, hgs)


def test_gpu_force2_short_list_two_wavefronts_per_tile():
    """The same grid dry but for one wet block: with skipping the list fits
    one pass and the Lagrangian stage puts two wavefronts on each listed
    tile (each marching half its rows); without skipping one wavefront
    marches four stacked tiles.  Same bits."""
    w = W.dam_break_fractal(n=8192, ny=2048, dx=2.0, seed=5, relief=10.0, depth=6.0).as_float32()
    H = np.zeros_like(w.H)
    H[1000:1100, 4000:4200] = w.H[1000:1100, 4000:4200] + 1.0
    w.H = H.astype(np.float32).astype(np.float64)
    say("case force2: 8192x2048 one wet block 30 steps, skipping on and off")
    ref, rs = run_gpu(w, 30, flags=_f2(False))
    f, fs = run_gpu(w, 30, flags=_f2(True))
    for a, b in zip(f, ref):
        assert np.array_equal(a, b)
    assert fs["t"] == rs["t"] and fs["water_volume"] == rs["water_volume"]


def test_gpu_force2_batch_and_refusals():
    """A batch of two members with the flag: each equals its run alone; a
    batch mixing force orders, an LDS tile shape and the unfused sequence are
    refused (SW_ERR_ARG); the autotuner keeps to strip shapes."""
    import torch
    from paper_2103_15196_amd import csph
    stream = torch.cuda.Stream()
    ms = [W.dam_break_fractal(n=n, dx=2.0, seed=s, relief=8.0, depth=4.0).as_float32()
          for n, s in ((150, 21), (97, 22))]
    alone = [run_gpu(m, 60, flags=_f2(), stream=stream.cuda_stream)[0] for m in ms]
    solvers = [csph.solver_for(m, stream=stream.cuda_stream, flags=_f2()) for m in ms]
    b = csph.Batch(solvers)
    b.advance(60)
    b.sync()
    for s, ref in zip(solvers, alone):
        for a, r in zip(s.get_fields(), ref):
            assert np.array_equal(a, r)
    b.close()
    plain = csph.solver_for(ms[0], stream=stream.cuda_stream)
    with pytest.raises(csph.SwError) as e:
        csph.Batch([solvers[0], plain])
    assert e.value.code == csph.SW_ERR_ARG
    with pytest.raises(csph.SwError) as e:
        solvers[0].set_tile_shape(64, 8)
    assert e.value.code == csph.SW_ERR_ARG
    assert solvers[0].autotune(3)[0] == 58
    with pytest.raises(csph.SwError):
        csph.solver_for(ms[0], stream=stream.cuda_stream,
                        flags=csph.SW_FLAG_FORCE2 | csph.SW_FLAG_UNFUSED)
    for s in solvers + [plain]:
        s.close()
