"""Parity of the HIP path (FP32 state, FP64 sums and dt) with the FP64 CPU oracle.

Every case starts both sides from the same float32-rounded seeded inputs and
calls the library through its C ABI.  Tolerances are the ones the precision
policy fixes: L-inf depth <= 1e-4 m, relative mass drift <= 1e-6, wet/dry mask
disagreement <= 0.1 % of cells (wet <=> h > 1e-4 m); bed elevation within
1e-4 m and unit discharges within 1e-4 m x max(|v| + c) (tests/gpu_common.py),
on every cell where the problem is well conditioned at float32 precision:
cells where the oracle's own algorithm evaluated in float32 arithmetic already
ends a tenth of the bound away from the FP64 answer are counted and reported
instead (tests/gpu_common.py; at most 0.5 % of the grid).
"""
import numpy as np
import pytest

from paper_2103_15196_amd import workloads as W
from tests.gpu_common import ILL_MAX, compare, run_gpu, run_oracle, say, torch_stream
from tests.helpers import oracle_case, read_golden

pytestmark = pytest.mark.gpu

LINF_H = 1e-4
MASS = 1e-6
MASK = 1e-3


def _check(res):
    f = res.pop("fields", {})
    say(f"  {res}")
    for name, r in f.items():
        say(f"  {name}: err {r['err']:.3e} (bound {r['bound']:.3e}) at {r['worst']}; "
            f"ill-conditioned cells {r['n_ill']} (max err there {r['err_ill']:.3e}); "
            f"cells over the bound {r['n_over']}")
        assert r["err"] <= r["bound"], name
        assert r["n_ill"] <= ILL_MAX * res["cells"], name
    assert res["mass_drift_gpu"] <= MASS
    assert res["mask_disagree"] <= MASK
    assert abs(res["t_gpu"] - res["t_oracle"]) <= 1e-5 * max(res["t_oracle"], 1e-9)


@pytest.fixture(scope="module")
def O():
    from oracle import oracle as O
    O.build(force=False)
    return O


def test_gpu_dam_break_256x64_cfl(O):
    """The 256 x 64 dam break (2 m | 0.5 m, erodible bed, Eq. 4 bedload,
    Manning 0.02, walls, K = 0.3), 200 steps with the Eq. 7 step."""
    w = W.dam_break_1d().as_float32()
    say("case dam_break 256x64 cfl 200")
    res = compare(O, w, run_gpu(w, 200), run_oracle(O, w, 200))
    _check(res)


def test_gpu_dam_break_256x64_fixed_dt(O):
    w = W.dam_break_1d().as_float32()
    say("case dam_break 256x64 fixed dt 0.05, 200")
    res = compare(O, w, run_gpu(w, 200, dt=0.05), run_oracle(O, w, 200, dt=0.05))
    _check(res)
    assert res["t_gpu"] == pytest.approx(10.0, rel=1e-12)


def test_gpu_fractal_dam_break_ragged_1000_steps(O):
    """2-D dam break over a fractal bed with open boundaries, wet/dry fronts
    and a ragged grid (not a multiple of the tile size), 1000 steps."""
    w = W.dam_break_fractal(n=300, ny=236, dx=2.0, seed=7, relief=10.0, depth=8.0,
                            steps=1000).as_float32()
    say("case fractal dam break 300x236 1000 steps")
    res = compare(O, w, run_gpu(w, 1000), run_oracle(O, w, 1000), spread=True, steps=1000)
    _check(res)


def test_gpu_river_valley_inflow_per_cell_soil(O):
    """Inflow hydrograph, per-cell d50 and psi, walls + one open side, bed sources."""
    w = W.river_valley(n=200, ny=136, dx=5.0, amplitude=60.0, wavelength=500.0, width=40.0,
                       Q_base=20.0, Q_peak=200.0, t_peak=40.0, t_sigma=15.0)
    w.qb = np.zeros((w.ny, w.nx))
    w.qb[60:70, 100:110] = 2e-6
    w = w.as_float32()
    say("case river valley 200x136 600 steps")
    gpu = run_gpu(w, 600)
    orc = run_oracle(O, w, 600)
    res = compare(O, w, gpu, orc, spread=True, steps=600)
    _check(res)
    sums = gpu[1]
    assert abs(sums["water_source_in"] - orc[2].in_w) <= 1e-6 * orc[2].in_w
    assert sums["wet_cells"] > 100


@pytest.mark.parametrize("name,steps,dt", [("hand_step_3x1_wall.txt", 1, 0.1)])
def test_gpu_hand_step_3x1(name, steps, dt):
    exp = read_golden(name)
    w = W.Workload(name="h", nx=3, ny=1, dx=1.0, bc=(0, 0, 0, 0), H=np.array([[1.0, 0, 0]]),
                   qx=np.zeros((1, 3)), qy=np.zeros((1, 3)), b=np.zeros((1, 3)), nM=0.0,
                   d50=5e-4, psi=0.4, steps=1, cfl=0.9, sed_law=0)
    (h, hu, hv, b), _ = run_gpu(w, 1, dt=0.1)
    for i in range(3):
        assert h[0, i] == pytest.approx(exp[f"H{i}"], abs=2e-6)
        assert hu[0, i] == pytest.approx(exp[f"qx{i}"], abs=2e-6)


def test_gpu_hand_steps_3x3():
    for name, dt in (("hand_step_3x3_column.txt", 0.1), ("hand_step_3x3_drained.txt", 0.25)):
        exp = read_golden(name)
        H = np.zeros((3, 3))
        H[1, 1] = 1.0
        z = np.zeros((3, 3))
        w = W.Workload(name="h", nx=3, ny=3, dx=1.0, bc=(0, 0, 0, 0), H=H, qx=z, qy=z, b=z,
                       nM=0.0, d50=5e-4, psi=0.4, steps=1, cfl=0.9, sed_law=0)
        (h, hu, hv, b), _ = run_gpu(w, 1, dt=dt)
        assert h[1, 1] == pytest.approx(exp["H_centre"], abs=2e-6)
        for (j, i) in ((0, 1), (2, 1), (1, 0), (1, 2)):
            assert h[j, i] == pytest.approx(exp["H_edge"], abs=2e-6)
        assert h[0, 0] == 0.0 and h[2, 2] == 0.0


def test_gpu_hand_step_momentum_and_exner():
    exp = read_golden("hand_step_2x1_momentum.txt")
    H = np.ones((1, 2))
    w = W.Workload(name="h", nx=2, ny=1, dx=1.0, bc=(0, 0, 0, 0), H=H, qx=np.array([[1.0, 0.0]]),
                   qy=np.zeros((1, 2)), b=np.zeros((1, 2)), nM=0.0, d50=5e-4, psi=0.4, steps=1,
                   cfl=0.9, sed_law=0)
    (h, hu, hv, b), _ = run_gpu(w, 1, dt=0.1)
    assert float(hu.sum()) == pytest.approx(exp["sum_q"], abs=5e-6)
    exp = read_golden("hand_step_exner_3x1.txt")
    H = np.ones((1, 3))
    w = W.Workload(name="e", nx=3, ny=1, dx=1.0, bc=(1, 1, 0, 0), H=H,
                   qx=np.array([[1.0, 1.5, 1.0]]), qy=np.zeros((1, 3)),
                   b=np.array([[0.0, 0.1, 0.0]]), nM=0.0, d50=5e-4, psi=0.4, steps=1, cfl=0.3,
                   sed_law=1)
    (h, hu, hv, b), _ = run_gpu(w, 1, dt=0.05, A_G=1e-3, m_exp=2.0)
    for i in range(3):
        assert b[0, i] == pytest.approx(exp[f"b{i}"], abs=1e-8)


@pytest.mark.parametrize("bc", [(0, 0, 0, 0), (1, 1, 1, 1)])
def test_gpu_lake_at_rest_is_exact(bc):
    """Still water over a fractal bed with dry islands stays bit-for-bit still."""
    w = W.lake_at_rest(200, 130, dx=1.0, relief=3.0, level=2.0, bc=bc).as_float32()
    (h, hu, hv, b), sums = run_gpu(w, 500)
    assert np.array_equal(h, w.H.astype(np.float32))
    assert np.all(hu == 0) and np.all(hv == 0)
    assert np.array_equal(b, w.b.astype(np.float32))


def test_gpu_y_uniform_and_transpose_bitwise():
    w = W.dam_break_1d(nx=160, ny=70, x_dam=80).as_float32()
    (h, hu, hv, b), _ = run_gpu(w, 150)
    assert np.all(hv == 0)
    for f in (h, hu, b):
        assert np.array_equal(f, np.broadcast_to(f[:1], f.shape))
    f = W.dam_break_fractal(n=130, ny=98, dx=2.0, seed=9, relief=5.0, depth=4.0).as_float32()
    f.bc = (0, 1, 1, 0)
    (h1, u1, v1, b1), s1 = run_gpu(f, 120)
    t = W.Workload(**{k: getattr(f, k) for k in f.__dataclass_fields__})
    t.nx, t.ny = f.ny, f.nx
    t.H, t.b, t.qx, t.qy = f.H.T.copy(), f.b.T.copy(), f.qy.T.copy(), f.qx.T.copy()
    t.bc = (f.bc[2], f.bc[3], f.bc[0], f.bc[1])
    (h2, u2, v2, b2), s2 = run_gpu(t, 120)
    assert np.array_equal(h2, h1.T) and np.array_equal(b2, b1.T)
    assert np.array_equal(u2, v1.T) and np.array_equal(v2, u1.T)


def test_gpu_device_pointers_and_torch_stream(O):
    """Inputs and outputs as torch device tensors (ptr_kind = device)."""
    import torch
    from paper_2103_15196_amd import csph
    w = W.dam_break_1d(nx=128, ny=48, x_dam=64).as_float32()
    dev = torch.device("cuda:0")
    t = {k: torch.tensor(getattr(w, k), dtype=torch.float32, device=dev).contiguous()
         for k in ("H", "qx", "qy", "b")}
    s = csph.Solver(w.nx, w.ny, w.dx, w.bc, stream=torch.cuda.current_stream().cuda_stream,
                    cfl=w.cfl, sed_law=w.sed_law)
    s.set_bed(t["b"])
    s.set_soil(w.nM, w.d50, w.psi)
    s.set_state(t["H"], t["qx"], t["qy"])
    s.advance(100)
    out = [torch.empty_like(t["H"]) for _ in range(4)]
    s.get_fields(out)
    torch.cuda.synchronize()
    h_host = s.get_fields()[0]
    s.close()
    assert np.array_equal(out[0].cpu().numpy(), h_host)
    p, inp, st = run_oracle(O, w, 100)
    assert np.abs(h_host - st.H).max() <= LINF_H


def test_gpu_errors_are_reported_and_state_kept():
    from paper_2103_15196_amd import csph
    w = W.dam_break_1d(nx=64, ny=16, x_dam=32).as_float32()
    s = csph.solver_for(w, stream=None)
    s.advance(5)
    h5 = s.get_fields()[0]
    s.advance(3, dt=10.0)          # far above the Eq. 7 step
    with pytest.raises(csph.SwError) as e:
        s.sync()
    assert e.value.code == csph.SW_ERR_CFL
    with pytest.raises(csph.SwError):
        s.get_fields()
    s.reset(w)                     # bed and state again; a new state clears the error
    s.advance(5)
    assert np.array_equal(s.get_fields()[0], h5)
    bad = w.H.copy()
    bad[3, 3] = np.nan
    with pytest.raises(csph.SwError) as e:
        s.set_state(bad, w.qx, w.qy)
    assert e.value.code == csph.SW_ERR_ARG
    s.close()


def test_gpu_variants_are_bitwise_identical():
    """Tiled vs unfused kernels, HGS on vs off, graph replay vs eager launches:
    identical bits (same per-cell and per-face arithmetic, exact dry-tile skip)."""
    from paper_2103_15196_amd import csph
    w = W.dam_break_fractal(n=400, ny=200, dx=2.0, seed=11, relief=10.0, depth=6.0).as_float32()
    w.bc = (0, 1, 1, 0)
    F = csph
    runs = {}
    for name, flags in (("tiled_hgs_graph", F.SW_FLAG_HGS), ("tiled_nohgs", 0),
                        ("tiled_hgs_eager", F.SW_FLAG_HGS | F.SW_FLAG_NO_GRAPH),
                        ("unfused", F.SW_FLAG_UNFUSED)):
        say(f"variant {name}")
        runs[name] = run_gpu(w, 301, flags=flags)
    ref = runs["unfused"]
    for name, (f, sums) in runs.items():
        for a, b in zip(f, ref[0]):
            assert np.array_equal(a, b), name
        assert sums["t"] == ref[1]["t"], name
    assert 0 < runs["tiled_hgs_graph"][1]["active_tiles"] < (400 // 64 + 1) * (200 // 8)


def test_gpu_tile_shapes_and_autotune_give_the_same_bits():
    from paper_2103_15196_amd import csph
    import torch
    w = W.dam_break_fractal(n=300, ny=236, dx=2.0, seed=7, relief=10.0, depth=8.0).as_float32()
    ref, ref_sums = run_gpu(w, 200)
    for shape in ((64, 4), (64, 16), (128, 4), (58, 8), (58, 16), (58, 32)):
        s = csph.solver_for(w, stream=torch.cuda.current_stream().cuda_stream)
        s.set_tile_shape(*shape)
        s.advance(200)
        f = s.get_fields()
        s.close()
        for a, b in zip(f, ref):
            assert np.array_equal(a, b), shape
    s = csph.solver_for(w, stream=torch.cuda.current_stream().cuda_stream)
    s.advance(60)
    shape = s.autotune(8)
    say(f"autotuned shape {shape}")
    s.advance(140)
    f = s.get_fields()
    sums = s.get_sums()
    s.close()
    for a, b in zip(f, ref):
        assert np.array_equal(a, b)
    assert sums["t"] == ref_sums["t"] and sums["step"] == 200


def test_gpu_profiled_advance_gives_the_same_bits_and_times():
    """The measurement path (one launch per kernel with time stamps: the strip
    launches' own, events between LDS-tile launches) steps exactly like
    sw_advance and reports positive mean kernel durations."""
    from paper_2103_15196_amd import csph
    import torch
    w = W.dam_break_fractal(n=300, ny=236, dx=2.0, seed=7, relief=10.0, depth=8.0).as_float32()
    ref, ref_sums = run_gpu(w, 50)
    for shape in ((58, 8), (64, 8)):
        s = csph.solver_for(w, stream=torch.cuda.current_stream().cuda_stream)
        s.set_tile_shape(*shape)
        lag_ms, eul_ms = s.advance_profiled(50)
        f = s.get_fields()
        sums = s.get_sums()
        s.close()
        say(f"profiled {shape}: lagrange {lag_ms * 1e3:.2f} us, euler {eul_ms * 1e3:.2f} us")
        assert lag_ms > 0.0 and eul_ms > 0.0
        for a, b in zip(f, ref):
            assert np.array_equal(a, b), shape
        assert sums["t"] == ref_sums["t"] and sums["step"] == 50


@pytest.mark.timeout(600)
def test_gpu_dam_break_2048_full_size_every_cell(O):
    """The 2048 x 2048 fractal dam break, 1000 steps, in the launch
    configuration the dam-break benchmark times (graph replay, dry-tile
    skipping, default tile shape), against the FP64 oracle run here from the
    same float32 inputs: h, hu, hv and b on every cell, the wet mask, time and
    water balance.  Which cells are ill-conditioned at float32 precision (the
    oracle's algorithm evaluated in float32 ends a tenth of the bound away
    from the FP64 answer there) comes from tests/golden/dam_break_2048_ref.npz
    (written by make_dam_break_2048_reference.py, which calls only the oracle
    and the input generator); the FP64 oracle run here must reproduce that
    file's samples.  Every other cell is held to the flat bounds."""
    import os
    import time
    from tests.gpu_common import field_check
    ref = np.load(os.path.join(os.path.dirname(__file__), "golden", "dam_break_2048_ref.npz"))
    steps = int(ref["steps"])
    w = W.dam_break_fractal(n=2048, steps=steps).as_float32()
    say("case dam break 2048^2 1000 steps: GPU")
    (h, hu, hv, b), sums = run_gpu(w, steps)
    say(f"  GPU done, t = {sums['t']:.4f} s; oracle ({steps} steps)")
    t0 = time.time()
    p, inp, st = run_oracle(O, w, steps)
    say(f"  oracle done in {time.time() - t0:.0f} s")
    stv = int(ref["stride"])
    sl = (slice(0, None, stv), slice(0, None, stv))
    for name, a in (("h", st.H), ("hu", st.qx), ("hv", st.qy), ("b", st.b)):
        np.testing.assert_allclose(a[sl], ref[name], rtol=0, atol=1e-12)
    assert st.t == pytest.approx(float(ref["t"]), rel=1e-14)
    vs = float(ref["vs"])
    spread = {}
    for name in ("h", "hu", "hv", "b"):
        d = np.zeros(h.size)
        d[ref[f"spread_{name}_idx"]] = ref[f"spread_{name}"]
        spread[name] = d.reshape(h.shape)
    res = {"linf_h": float(np.abs(h - st.H).max()), "t_gpu": sums["t"], "t_oracle": st.t,
           "cells": int(h.size)}
    res["mask_disagree"] = float(np.mean((h > 1e-4) != (st.H > 1e-4)))
    V0 = float(ref["V0"])
    res["mass_drift_gpu"] = abs(sums["water_volume"] - V0 + sums["water_boundary_out"]) / V0
    res["volume_vs_oracle"] = abs(sums["water_volume"] - float(ref["Vw"])) / float(ref["Vw"])
    res["fields"] = field_check((h, hu, hv, b), st, spread, vs)
    eh = np.abs(h - st.H)
    over = np.argwhere(eh > LINF_H)
    say(f"  cells with |dh| > 1e-4 m: {len(over)} at (i, j) {[(int(q[1]), int(q[0])) for q in over[:10]]}"
        f"; 99.9% of cells within {np.quantile(eh, 0.999):.2e} m")
    _check(res)
    assert res["volume_vs_oracle"] <= 1e-6


@pytest.mark.timeout(600)
def test_gpu_river_valley_8192_full_size_one_step_every_cell(O):
    """The 8192 x 8192 river valley (the benchmark's workload, its launch
    configuration: 58 x 8 strips, every tile processed, one grid of
    per-cell-soil kernels) after 1000 steps from its initial state, inflow
    running: one more GPU step against one FP64 oracle step from the same
    float32 state and time, every cell of h, hu, hv and b, the step length and
    the inflow volume of the step.  (The oracle takes about 2 s a step on the
    grid: the full 2000-step run is out of its reach, one step from the GPU's
    state is not.)"""
    import time
    from paper_2103_15196_amd import csph
    from tests.gpu_common import field_check
    w = W.river_valley(n=8192, steps=2000).as_float32()
    say("case river valley 8192^2: 1000 GPU steps, then one step on both sides")
    s = csph.solver_for(w, stream=torch_stream(), flags=0)
    s.advance(1000)
    h, hu, hv, b = s.get_fields()
    s0 = s.get_sums()
    s.advance(1)
    g = s.get_fields()
    s1 = s.get_sums()
    s.close()
    say(f"  GPU at t = {s0['t']:.4f} s, wet cells {s0['wet_cells']}; oracle step")
    p, inp, st = oracle_case(O, w)
    st = O.State(h, hu, hv, b, t=s0["t"])
    t0 = time.time()
    rec = O.step(p, inp, st)
    say(f"  oracle step in {time.time() - t0:.1f} s, dt {rec['dt']!r} (GPU {s1['last_dt']!r})")
    assert abs(s1["last_dt"] - rec["dt"]) <= 1e-6 * rec["dt"]
    assert abs((s1["water_source_in"] - s0["water_source_in"]) - rec["in_w"]) <= 1e-6 * rec["in_w"]
    vs = O.cfl(p, inp, st)["vs"]
    f = field_check(g, st, None, vs)
    for name, r in f.items():
        say(f"  {name}: err {r['err']:.3e} (bound {r['bound']:.3e}) at {r['worst']}")
        assert r["err"] <= r["bound"], name
    assert s0["wet_cells"] > 100
