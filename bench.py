"""Benchmark of the CSPH-TVD step on one MI355X.

Workload (N=1): the 8192 x 8192 river valley (67.1 M cells, dx = 5 m): seeded
fractal terrain (20 m relief) on a 1e-3 regional slope, a meandering
parabolic channel 5 m deep and 200 m wide, per-cell grain size d50 ~ U[0.2, 2]
mm and porosity psi ~ U[0.3, 0.45], Manning n = 0.03, Eq. 4 bedload, an inflow
hydrograph Q = 100 + 2000 exp(-(t - 120)^2 / (2 40^2)) m^3/s on the x = 0
channel cells, open at x = max, walls elsewhere, initially dry, K = 0.3,
2000 steps.  One "step" is one CSPH-TVD time step over the whole grid (the
work-list pass with the Eq. 7 step, the Lagrangian stage, the fused Euler
stage), replayed from HIP graphs.  ``value`` processes every tile of the grid
(dry-tile skipping off): it is the rate of the kernels on the whole grid; the
rate of the same run with dry tiles skipped (the hierarchical grid system of
Section 3) and its wet fraction are reported beside it.  Inputs are resident
on the GPU, the state's set-up pass and the graph capture finish before the
timed region starts.

Prints one JSON line: value = grid cells x steps / wall time (Gcell-steps/s),
a roofline object for the dominant kernel (the strip Euler kernel, timed live
with its own launch time stamps on the solver's stream, against 8 TB/s with
the 40 B of state and soil each cell-step must move: h, hu, hv, b read and
written, d50 and psi read; HBM traffic per launch from the committed rocprofv3
counter summary while it matches the kernel sources), the CPU oracle timed
on a bounded sample of the same workload (all host threads and one thread),
and side measurements (the 2048^2 dam break, the 64-member ensemble, the
learned surrogate trained on river-valley basins).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
# FP32 FMA issue rate without packed math: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# (a wave64 FMA every 4 cycles per SIMD; independent FMA chains reach 0.94-0.97
# of it).  Some other vector instruction kinds issue faster, so it bounds the
# FP32 arithmetic of a kernel, not every instruction it counts.
VALU_PEAK_TLANE = 256 * 4 * 16 * 2.4e9 / 1e12
# the Euler kernel the river valley's launch selects: 58 x 8 strips, per-cell
# soil, every tile listed in one grid, minmod limiter and Davis speeds
EULER_KERNEL = "k_euler_sl<8,true,1,false>"
KERNEL_SOURCES = ("paper_2103_15196_amd/csrc/csph.hip", "paper_2103_15196_amd/csrc/csph_device.h")
PROFILE = "profiles/k_euler_sl_river_valley_8192_counters.md"
# algorithmic bytes per cell-step of the river valley: h, hu, hv, b read and
# written (16 + 16 B) and the per-cell soil d50, psi read (8 B); halo
# re-reads, the Lagrangian momentum and scratch planes are not counted
STEP_BYTES = 40


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profiled_counters():
    """Per-launch HBM bytes and VALU instructions of the dominant kernel from
    the committed rocprofv3 summary, if it was taken on the current kernel
    sources (else None: the counters no longer describe this kernel)."""
    path = os.path.join(ROOT, PROFILE)
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if line.startswith("<!-- bench:"):
            for kv in line.strip()[len("<!-- bench:"):-3].split():
                k, v = kv.split("=", 1)
                rec[k] = v
    if rec.get("src_sha256") != kernel_source_hash():
        return None
    return rec


def timed_advance(s, stream, steps, torch):
    """ms of s.advance(steps) between two events on the solver's stream."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    s.advance(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=8192, help="grid side of the river valley")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-hgs", action="store_true", help="skip the dry-tile-skipping run")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target seconds of each oracle sample (all threads, one thread)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a 1 GiB in / 1 GiB out torch mul (HBM counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: the solver has no multi-GPU path "
              "(row-strip sharding is described in the design notes only).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2103_15196_amd import csph, workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    # a real (non-null) stream: the solver orders its kernels on it and the
    # timing events are recorded on it
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)

    if args.calibrate_copy:
        # a plain streaming kernel of known size (1 GiB read, 1 GiB written,
        # larger than the 256 MB Infinity Cache) to scale the HBM counters
        src = torch.ones(256 * 1024 * 1024, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        log("[bench] counter calibration: 3 x (1073741824 bytes read + written) by the mul kernel")
        del src, dst

    log(f"[bench] building workload river_valley n={args.n}")
    w = W.river_valley(n=args.n, steps=args.steps).as_float32()
    cells = w.nx * w.ny
    assert stream.cuda_stream != 0
    s = csph.solver_for(w, stream=stream.cuda_stream, flags=0)
    log(f"[bench] warmup {args.warmup} steps")
    if args.warmup:
        s.advance(args.warmup)
        s.sync()
    s.reset(w)  # timed steps start from the initial bed and state (set-up done here)
    s.sync()
    builds0 = s.get_sums()["graph_builds"]
    log(f"[bench] timing {args.steps} steps (every tile processed)")
    t0 = time.perf_counter()
    ms = timed_advance(s, stream, args.steps, torch)
    wall = time.perf_counter() - t0
    sums = s.get_sums()
    assert sums["graph_builds"] == builds0, "a step graph was captured inside the timed region"
    value = cells * args.steps / (ms * 1e-3) / 1e9
    log(f"[bench] {ms:.2f} ms ({wall*1e3:.2f} ms wall) -> {value:.2f} Gcell-steps/s, "
        f"t={sums['t']:.3f} s, wet={sums['wet_cells']}")

    # per-kernel durations: each strip launch records its own start and end on
    # the solver's stream, the same steps again
    s.reset(w)
    lag_ms, eul_ms = s.advance_profiled(args.steps)
    ps = s.get_sums()
    eul_cells = ps["cells_euler"] / args.steps
    lag_cells = ps["cells_lagrange"] / args.steps
    achieved = eul_cells * STEP_BYTES / (eul_ms * 1e-3) / 1e9
    prof = profiled_counters()
    log(f"[bench] kernels: lagrange {lag_ms*1e3:.1f} us ({lag_cells:.0f} cells), "
        f"euler {eul_ms*1e3:.1f} us ({eul_cells:.0f} cells) -> {achieved:.0f} GB/s")
    s.close()

    out = {
        "metric": "Gcell-steps/s",
        "value": round(value, 3),
        "unit": "Gcell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"river_valley_{w.nx}x{w.ny}", "grid": [w.nx, w.ny], "dx_m": w.dx,
                   "relief_m": 20.0, "channel": "meandering, 5 m deep, 200 m wide",
                   "soil": "per-cell d50 U[0.2,2] mm, psi U[0.3,0.45]", "manning": 0.03,
                   "inflow_peak_m3s": 2000.0, "bc": "walls, open at x = max", "cfl": w.cfl,
                   "sed_law": "eq4", "skip_dry_tiles": False, "graph": True,
                   "parallelism": "single-gpu"},
        "hbm_frac_step": round(value * STEP_BYTES / HBM_PEAK_GBS, 4),
        # the dominant kernel against the HBM roof with the method's own bytes
        "roofline": {"kernel": EULER_KERNEL, "bound": "hbm", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": (int(float(prof["traffic_bytes"])) if prof else None),
                     "bytes_per_cell": STEP_BYTES, "cells_per_launch": round(eul_cells),
                     "avg_launch_us": round(eul_ms * 1e3, 2),
                     "lagrange_avg_launch_us": round(lag_ms * 1e3, 2)},
        "time_s_model": sums["t"],
        "wet_fraction_end": round(sums["wet_cells"] / cells, 6),
    }
    if prof:
        # executed vector work of the same kernel (counters on these sources):
        # every issued lane-instruction against the non-packed FP32 FMA rate
        lane_ops = float(prof["valu_insts"]) * 64
        ach = lane_ops / (eul_ms * 1e-3) / 1e12
        out["roofline"]["valu"] = {"achieved": round(ach, 2), "unit": "Tlane-op/s",
                                   "fp32_fma_rate": round(VALU_PEAK_TLANE, 2),
                                   "frac_of_fma_rate": round(ach / VALU_PEAK_TLANE, 4),
                                   "lane_ops_per_cell": round(lane_ops / eul_cells, 1)}
        # HBM bytes the counters saw per launch, at the launch time measured here
        out["roofline"]["traffic_gbs"] = round(float(prof["traffic_bytes"]) / (eul_ms * 1e-3) / 1e9, 1)
        out["roofline"]["traffic_frac"] = round(out["roofline"]["traffic_gbs"] / HBM_PEAK_GBS, 4)

    if not args.no_hgs:
        out["hgs"] = hgs_rate(csph, w, torch, stream, args.steps, value)
    if not args.no_extras:
        out["save_overlap"] = save_overlap(csph, w, torch, stream)
    if not args.no_extras:
        out["dam_break_2048"] = dam_break_rate(csph, W, torch, stream)
        out["surrogate"] = surrogate_rates(csph, torch)
        out["ensemble"] = ensemble_rates(csph, W, torch)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def hgs_rate(csph, w, torch, stream, steps, full_rate):
    """The same run with dry tiles skipped (HGS): rate, wet fraction, gain."""
    log(f"[bench] river valley {w.nx}^2 x {steps} steps, dry tiles skipped")
    s = csph.solver_for(w, stream=stream.cuda_stream, flags=csph.SW_FLAG_HGS)
    s.advance(20)
    s.reset(w)
    s.sync()
    ms = timed_advance(s, stream, steps, torch)
    sums = s.get_sums()
    s.close()
    rate = w.nx * w.ny * steps / (ms * 1e-3) / 1e9
    res = {"gcell_steps_s": round(rate, 3), "ms_per_step": round(ms / steps, 4),
           "wet_fraction_end": round(sums["wet_cells"] / (w.nx * w.ny), 6),
           "active_tiles_end": sums["active_tiles"],
           "cells_euler_per_step": round(sums["cells_euler"] / steps),
           "gain_vs_every_tile": round(rate / full_rate, 2)}
    log(f"[bench]   hgs: {res}")
    return res


def save_overlap(csph, w, torch, stream, steps=400, every=100):
    """The state read back every `every` steps (the Save block of Section 3):
    synchronously (sw_get_fields between the advances) and asynchronously
    (sw_save_begin, then sw_save_wait one interval later, the copy running on a
    second stream), against the same steps without readback."""
    log(f"[bench] readback every {every} steps on {w.nx}^2, {steps} steps")
    s = csph.solver_for(w, stream=stream.cuda_stream, flags=0)
    s.advance(2)
    s.save_begin()
    s.save_wait()

    def run(mode):
        s.reset(w)
        s.sync()
        t0 = time.perf_counter()
        pending = False
        for _ in range(steps // every):
            s.advance(every)
            if mode == "sync":
                s.get_fields()
            elif mode == "async":
                if pending:
                    s.save_wait()
                s.save_begin()
                pending = True
        if pending:
            s.save_wait()
        s.sync()
        return (time.perf_counter() - t0) * 1e3 / steps

    plain, sync, asyn = run("none"), run("sync"), run("async")
    s.close()
    res = {"grid": [w.nx, w.ny], "steps": steps, "every": every,
           "ms_per_step_no_readback": round(plain, 4), "ms_per_step_sync": round(sync, 4),
           "ms_per_step_async": round(asyn, 4),
           "async_gain_vs_sync": round(sync / asyn - 1.0, 4)}
    log(f"[bench]   readback: {res}")
    return res


def dam_break_rate(csph, W, torch, stream, n=2048, steps=1000):
    """The 2048^2 fractal dam break (state in the Infinity Cache), skipping on."""
    log(f"[bench] dam break {n}^2 x {steps} steps")
    w = W.dam_break_fractal(n=n, steps=steps).as_float32()
    s = csph.solver_for(w, stream=stream.cuda_stream)
    s.advance(20)
    s.reset(w)
    s.sync()
    ms = timed_advance(s, stream, steps, torch)
    sums = s.get_sums()
    s.close()
    res = {"gcell_steps_s": round(w.nx * w.ny * steps / (ms * 1e-3) / 1e9, 3),
           "ms_per_step": round(ms / steps, 5), "skip_dry_tiles": True,
           "wet_fraction_end": round(sums["wet_cells"] / (w.nx * w.ny), 4)}
    log(f"[bench]   dam break: {res}")
    return res


def surrogate_rates(csph, torch, train_steps=8000, trajectories=200, heldout=20):
    """The learned surrogate (6 BF16 matrix-core 3x3 convolutions, widths 5,
    48 x 5, 4; k = 8 fixed steps of 0.02 s per call) trained here with the
    library's training loop on 200 trajectories of 1024^2 closed basins on the
    river valley's terrain (a reservoir released down the meandering channel,
    per-cell soil, a random spin-up each; 12 consecutive pairs per trajectory,
    each kept as a 256^2 window around a wet cell; a seed whose flow outruns
    the fixed step is replaced by the next); held out: 20 basins of 1024^2
    (seeds from 6000, 4 pairs each, whole grids).  Reported: the held-out
    depth error of one call against the 5e-3 m gate, beside the error of
    predicting no change, and the effective rate of the surrogate step on a
    1024^2 basin (conservation, stability and residual checks, fall backs
    included) next to the plain solver's 8 fixed steps."""
    import numpy as np
    from paper_2103_15196_amd import surrogate as SG
    st = torch.cuda.current_stream().cuda_stream
    t0 = time.perf_counter()
    tr, drop_tr = SG.collect_valley(range(5000, 5000 + 2 * trajectories), 1024, 96, 8, stream=st,
                                    depth_range=(1.5, 3.0), crop=256, count=trajectories)
    ho, drop_ho = SG.collect_valley(range(6000, 6000 + 5 * heldout), 1024, 32, 8, stream=st,
                                    depth_range=(1.5, 3.0), count=heldout)
    t_data = time.perf_counter() - t0
    ins, outs = SG.scales(tr)
    net = csph.Surrogate(SG.DESIGN_CHANNELS, stream=st)
    net.set_params(SG.he_init(SG.DESIGN_CHANNELS, 1))
    t1 = time.perf_counter()
    losses = SG.train(net, tr, ins, outs, steps=train_steps, batch=8, lr=1e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    err, drift = SG.evaluate(net, ho, ins, outs)
    zero = np.abs(ho.d[:, 0]).max(axis=(1, 2))
    w = SG.valley_basin(1024, 7100, 2.5)
    gain = SG.measure_gain(net, w, SG.VALLEY_DT, calls=20, k=8, stream=st)
    net.close()
    enabled = bool(err.max() <= 5e-3)
    res = {"train_trajectories": trajectories, "trajectory_grid": [1024, 1024],
           "train_window": [256, 256], "dropped_seeds": drop_tr + drop_ho,
           "train_pairs": int(len(tr.x)), "train_steps": train_steps, "batch": 8,
           "first_loss": round(float(losses[0]), 5),
           "final_loss": round(float(np.mean(losses[-50:])), 5),
           "heldout_seeds": heldout, "heldout_pairs": int(len(ho.x)),
           "heldout_linf_dh_m": round(float(err.max()), 5),
           "heldout_median_linf_dh_m": round(float(np.median(err)), 5),
           "no_change_linf_dh_m": round(float(zero.max()), 5),
           "no_change_median_linf_dh_m": round(float(np.median(zero)), 5),
           "gate_m": 5e-3, "enabled": enabled,
           "heldout_median_volume_drift": float(np.median(drift)), **gain,
           "data_seconds": round(t_data, 1), "train_seconds": round(t_train, 1),
           "seconds": round(time.perf_counter() - t0, 1)}
    log(f"[bench]   surrogate: {res}")
    return res


def ensemble_rates(csph, W, torch, count=64, steps=1000):
    """64 dam-break members of uneven size (sides U{256..1536}, own terrain,
    depth, Manning n and Eq. 7 step), 1000 steps each: one batch (one launch
    per stage over all members' tiles, graph replay, tile shape from the
    batch autotuner) against the members advanced one after another (each
    with its set-up pass and step graphs done before the timing); both rates
    are all members' cell-steps over the wall time, from the same initial
    states."""
    log(f"[bench] ensemble of {count} x {steps} steps")
    ms = [m.as_float32() for m in W.ensemble(count=count, seed0=1000, n_min=256, n_max=1536,
                                             steps=steps)]
    cells = sum(m.nx * m.ny for m in ms)
    stream = torch.cuda.current_stream()
    solvers = [csph.solver_for(m, stream=stream.cuda_stream) for m in ms]
    b = csph.Batch(solvers)
    shape = b.autotune(10)  # the batch's tile shape, chosen from the initial states
    b.advance(2)
    b.sync()
    for s, m in zip(solvers, ms):
        s.reset(m)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.advance(steps)
    b.sync()
    t_batch = time.perf_counter() - t0
    b.close()
    for s, m in zip(solvers, ms):
        s.advance(2)
        s.reset(m)
    torch.cuda.synchronize()
    t_seq = 0.0
    for s in solvers:
        t0 = time.perf_counter()
        s.advance(steps)
        s.sync()
        t_seq += time.perf_counter() - t0
    for s in solvers:
        s.close()
    res = {"members": count, "cells": cells, "steps": steps, "batch_tile_shape": list(shape),
           "batched_gcell_steps_s": round(cells * steps / t_batch / 1e9, 3),
           "sequential_gcell_steps_s": round(cells * steps / t_seq / 1e9, 3),
           "speedup": round(t_seq / t_batch, 3)}
    log(f"[bench]   ensemble: {res}")
    return res


def cpu_baseline(w, seconds):
    """The FP64 CPU oracle on the same grid: a bounded number of steps with all
    host threads, then with one thread (the paper's serial reference point)."""
    from oracle import oracle as O
    O.build(force=False)
    from tests.helpers import oracle_case
    res = {}
    n_all = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    for label, nthr in (("all", n_all), ("one", 1)):
        O.set_threads(nthr)
        p, inp, st = oracle_case(O, w)
        t0 = time.perf_counter()
        O.step(p, inp, st)  # one step, timed, also sizes the sample
        one = time.perf_counter() - t0
        steps = max(1, min(600, int(seconds / max(one, 1e-3))))
        log(f"[bench] cpu oracle ({label}): {steps} + 1 steps on {w.nx}x{w.ny}, {O.threads()} threads")
        t0 = time.perf_counter()
        O.run(p, inp, st, steps)
        dt = time.perf_counter() - t0
        res[label] = {"value": round(w.nx * w.ny * steps / dt / 1e9, 6), "cores": O.threads(),
                      "steps": steps, "seconds": round(dt, 2)}
    O.set_threads(n_all)
    a, b = res["all"], res["one"]
    return {"value": a["value"], "unit": "Gcell-steps/s", "cores": a["cores"], "kind": "oracle",
            "sample": f"{a['steps']} steps (after 1 timed set-up step) of the {w.nx}x{w.ny} river "
                      f"valley from its initial state, FP64, {a['seconds']} s on {a['cores']} threads",
            "one_thread": {"value": b["value"], "cores": 1,
                           "sample": f"{b['steps']} steps (after 1) of the same run, {b['seconds']} s"}}


if __name__ == "__main__":
    main()
