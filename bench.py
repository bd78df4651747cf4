"""Benchmark of the CSPH-TVD step on one MI355X.

Workload (N=1): the 2-D dam break over a seeded fractal bed, 2048 x 2048 cells,
dx = 2 m, 1 m dam line, 8 m reservoir, dry downstream, open boundaries,
psi = 0.4, Manning n = 0.03, Grass bedload (A_G = 0.001, m = 2; d50 = 0.5 mm
for the Shamov critical speed), K = 0.3.  One "step"
is one CSPH-TVD time step over the whole grid (Lagrangian stage with the Eq. 7
step, then the fused Euler stage), replayed from a HIP graph with dry tiles
skipped.  Inputs are resident on the GPU before the timed region starts.

Prints one JSON line: value = grid cells x steps / wall time (Gcell-steps/s),
a roofline object for the dominant kernel (the strip Euler kernel, timed live
with HIP events on the solver's stream; it is bound by VALU issue, so the
roof is the non-packed FP32 VALU rate against the kernel's algorithmic
operations, with its HBM figures beside it; HBM traffic and executed VALU work
per launch come from the committed rocprofv3 counter summary when it was taken
on the current kernel sources), the CPU oracle timed on a bounded sample of the same
workload, and side measurements (the river-valley grid with dry-tile skipping
on and off; the learned surrogate's accuracy and effective rate).
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
# FP32 VALU issue peak without packed math: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_PEAK_TLANE = 256 * 4 * 16 * 2.4e9 / 1e12
KERNEL_SOURCES = ("paper_2103_15196_amd/csrc/csph.hip", "paper_2103_15196_amd/csrc/csph_device.h")
PROFILE = "profiles/k_euler_sl_dam_break_2048_counters.md"
# algorithmic bytes per cell of one launch (float32 planes read + written)
EULER_BYTES = {"scalar_soil": 40, "per_cell_soil": 52}    # h,hu,hv,b,QLx,QLy in; h,hu,hv,b out (+nM,d50,psi)
# (per processed cell of one Euler launch: the strip kernel reads each of these once
# from HBM when halo rows and columns are served from cache)
LAGRANGE_BYTES = {"scalar_soil": 24, "per_cell_soil": 28}  # h,hu,hv,b in; QLx,QLy out (+nM)
STEP_BYTES = 32  # per cell-step: state read once + written once
# algorithmic FP32 operations per processed cell of one Euler launch (each
# add, sub, mul, fma, min, max, compare, div, sqrt, exp2, log2 counted once;
# selects and data movement not counted), one evaluation per cell and per
# face: remap inputs 11, minmod reconstruction along x and y 64, two HLL faces
# with hydrostatic depths 92, two bedload faces 20, draining limiter 12, K8
# update 44, Eq. 7 maxima and J0 of the new state 32
EULER_OPS = 275


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=2048, help="grid side of the dam-break workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=0, help="oracle steps (0: auto, ~10-30 s)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a 1 GiB in / 1 GiB out torch mul (HBM counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: the solver has no multi-GPU path "
              "(row-strip sharding is described in the design notes only).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
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

    log(f"[bench] building workload dam_break_fractal n={args.n}")
    w = W.dam_break_fractal(n=args.n, steps=args.steps).as_float32()
    cells = w.nx * w.ny
    assert stream.cuda_stream != 0
    s = csph.solver_for(w, stream=stream.cuda_stream)
    log(f"[bench] warmup {args.warmup} steps")
    if args.warmup:
        s.advance(args.warmup)
        s.sync()
    s.reset(w)  # timed steps start from the initial bed and state
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} steps")
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    s.advance(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    s.sync()
    sums = s.get_sums()
    value = cells * args.steps / (ms * 1e-3) / 1e9
    log(f"[bench] {ms:.2f} ms ({wall*1e3:.2f} ms wall) -> {value:.2f} Gcell-steps/s, "
        f"t={sums['t']:.3f} s, wet={sums['wet_cells']}")

    # per-kernel durations (HIP events on the solver's stream), same steps again
    s.reset(w)
    lag_ms, eul_ms = s.advance_profiled(args.steps)
    ps = s.get_sums()
    eul_cells = ps["cells_euler"] / args.steps
    lag_cells = ps["cells_lagrange"] / args.steps
    soil = "scalar_soil"
    eul_bytes = eul_cells * EULER_BYTES[soil]
    achieved = eul_bytes / (eul_ms * 1e-3) / 1e9
    alu_ach = eul_cells * EULER_OPS / (eul_ms * 1e-3) / 1e12
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
        "config": {"workload": f"dam_break_fractal_{w.nx}x{w.ny}", "grid": [w.nx, w.ny],
                   "dx_m": w.dx, "reservoir_m": 8.0, "dam_m": 1.0, "relief_m": 10.0,
                   "bc": "open", "cfl": w.cfl, "sed_law": "grass", "skip_dry_tiles": True,
                   "graph": True, "parallelism": "single-gpu"},
        "hbm_frac_algorithmic": round(value * STEP_BYTES / HBM_PEAK_GBS, 4),
        # the strip Euler kernel is bound by VALU issue: its roofline is the
        # non-packed FP32 VALU rate, against the algorithmic operations it must do
        "roofline": {"kernel": "k_euler_sl<8,false,1>", "bound": "alu", "achieved": round(alu_ach, 3),
                     "peak": round(VALU_PEAK_TLANE, 2), "unit": "Top/s",
                     "frac": round(alu_ach / VALU_PEAK_TLANE, 4),
                     "traffic": (int(float(prof["traffic_bytes"])) if prof else None),
                     "avg_launch_us": round(eul_ms * 1e3, 2), "ops_per_cell": EULER_OPS,
                     "cells_per_launch": round(eul_cells),
                     "hbm": {"achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(achieved / HBM_PEAK_GBS, 4),
                             "bytes_per_cell": EULER_BYTES[soil]},
                     "lagrange_avg_launch_us": round(lag_ms * 1e3, 2)},
        "time_s_model": sums["t"],
    }
    if prof:
        # executed VALU work of the same kernel (profiled on these sources):
        # every issued lane-operation, overhead included, against the same peak
        lane_ops = float(prof["valu_insts"]) * 64
        ach = lane_ops / (eul_ms * 1e-3) / 1e12
        out["roofline"]["executed"] = {"achieved": round(ach, 2), "unit": "Top/s",
                                       "frac": round(ach / VALU_PEAK_TLANE, 4),
                                       "valu_lane_ops_per_launch": int(lane_ops)}

    if not args.no_extras:
        out["river_valley"] = river_valley_rates(csph, W, torch)
        out["surrogate"] = surrogate_rates(csph, torch)
        out["ensemble"] = ensemble_rates(csph, W, torch)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_steps)
    print(json.dumps(out), flush=True)


def river_valley_rates(csph, W, torch, n=8192, steps=2000):
    """The 8192^2 river valley (meandering channel, per-cell soil, inflow
    hydrograph, initially dry): whole-grid rate with dry-tile skipping on and off."""
    log(f"[bench] river valley {n}^2 x {steps} steps")
    w = W.river_valley(n=n, steps=steps).as_float32()
    res = {"grid": [w.nx, w.ny], "steps": steps}
    stream = torch.cuda.current_stream()
    for name, flags in (("skip_on", csph.SW_FLAG_HGS), ("skip_off", 0)):
        s = csph.solver_for(w, stream=stream.cuda_stream, flags=flags)
        s.advance(20)
        s.reset(w)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        s.advance(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        sums = s.get_sums()
        res[name] = {"gcell_steps_s": round(w.nx * w.ny * steps / (ms * 1e-3) / 1e9, 3),
                     "ms_per_step": round(ms / steps, 4),
                     "wet_fraction": round(sums["wet_cells"] / (w.nx * w.ny), 5),
                     "t_model_s": round(sums["t"], 3)}
        log(f"[bench]   {name}: {res[name]}")
        s.close()
    return res


def surrogate_rates(csph, torch, train_steps=1500):
    """The learned surrogate (6 BF16 matrix-core 3x3 convolutions, widths 5, 48 x 5, 4)
    trained here on 24 closed-basin trajectories of 128^2 (k = 8 fixed steps per
    call): held-out depth error against the 5e-3 m gate, and the effective rate
    of the surrogate step on a 1024^2 basin (fall backs included) next to the
    plain solver's 8 fixed steps."""
    import numpy as np
    from paper_2103_15196_amd import surrogate as SG
    st = torch.cuda.current_stream().cuda_stream
    t0 = time.perf_counter()
    tr = SG.collect(range(5000, 5024), 128, 160, 8, stream=st)
    ho = SG.collect(range(6000, 6004), 128, 160, 8, stream=st)
    ins, outs = SG.scales(tr)
    net = csph.Surrogate(SG.DESIGN_CHANNELS, stream=st)
    net.set_params(SG.he_init(SG.DESIGN_CHANNELS, 1))
    losses = SG.train(net, tr, ins, outs, steps=train_steps, batch=8, lr=1e-3)
    err, drift = SG.evaluate(net, ho, ins, outs)
    w = SG.basin(1024, 6100, 5.0)
    gain = SG.measure_gain(net, w, SG.fixed_dt(w), calls=20, k=8, stream=st)
    net.close()
    enabled = bool(err.max() <= 5e-3)
    res = {"train_pairs": int(len(tr.x)), "train_steps": train_steps,
           "final_loss": round(float(np.mean(losses[-50:])), 5),
           "heldout_linf_dh_m": round(float(err.max()), 5), "gate_m": 5e-3, "enabled": enabled,
           "heldout_median_volume_drift": float(np.median(drift)), **gain,
           "seconds": round(time.perf_counter() - t0, 1)}
    log(f"[bench]   surrogate: {res}")
    return res


def ensemble_rates(csph, W, torch, count=64, steps=1000):
    """64 dam-break members of uneven size (sides U{256..1536}, own terrain,
    depth, Manning n and Eq. 7 step), 1000 steps each: one batch (one launch
    per stage over all members' tiles, graph replay) against the members
    advanced one after another; both rates are all members' cell-steps over
    the wall time, from the same initial states."""
    log(f"[bench] ensemble of {count} x {steps} steps")
    ms = [m.as_float32() for m in W.ensemble(count=count, seed0=1000, n_min=256, n_max=1536,
                                             steps=steps)]
    cells = sum(m.nx * m.ny for m in ms)
    stream = torch.cuda.current_stream()
    solvers = [csph.solver_for(m, stream=stream.cuda_stream) for m in ms]
    b = csph.Batch(solvers)
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
    res = {"members": count, "cells": cells, "steps": steps,
           "batched_gcell_steps_s": round(cells * steps / t_batch / 1e9, 3),
           "sequential_gcell_steps_s": round(cells * steps / t_seq / 1e9, 3),
           "speedup": round(t_seq / t_batch, 3)}
    log(f"[bench]   ensemble: {res}")
    return res


def cpu_baseline(w, steps):
    """The FP64 CPU oracle on the same grid, a bounded number of steps."""
    from oracle import oracle as O
    O.build(force=False)
    from tests.helpers import oracle_case
    p, inp, st = oracle_case(O, w)
    O.step(p, inp, st)  # first step untimed (allocation, page faults)
    if steps <= 0:
        t0 = time.perf_counter()
        O.step(p, inp, st)
        one = time.perf_counter() - t0
        steps = max(2, min(600, int(15.0 / max(one, 1e-3))))
    log(f"[bench] cpu oracle: {steps} steps on {w.nx}x{w.ny}, {O.threads()} threads")
    t0 = time.perf_counter()
    O.run(p, inp, st, steps)
    dt = time.perf_counter() - t0
    return {"value": round(w.nx * w.ny * steps / dt / 1e9, 5), "unit": "Gcell-steps/s",
            "cores": O.threads(), "kind": "oracle",
            "sample": f"{steps} steps (after 1 untimed) of the {w.nx}x{w.ny} dam break, FP64, "
                      f"{dt:.1f} s"}


if __name__ == "__main__":
    main()
