"""Training and evaluation of the convolutional surrogate on solver trajectories.

Everything numerical runs in the library: the trajectories come from the
solver (fixed step), training from `sws_train` (forward, backward and Adam
kernels), the surrogate step with its checks from `sws_advance_K`.  This
module only assembles arrays (sampling pairs, per-channel scales).

A training pair is (state at step n, change of (h, hu, hv, b) over the next k
steps).  Network inputs are x = in_scale * (h, hu, hv, b, wet mask); its
targets the changes divided by out_scale.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np

from . import csph
from . import workloads as W

DESIGN_CHANNELS = (5, 48, 48, 48, 48, 48, 4)
G = 9.81


@dataclass
class Pairs:
    x: np.ndarray       # [n, 5, ny, nx] raw inputs (h, hu, hv, b, mask)
    d: np.ndarray       # [n, 4, ny, nx] changes over k steps
    k: int
    dt: np.ndarray      # [n] step of each pair's trajectory


def basin(n, seed, depth, relief=10.0, dx=2.0):
    """A closed fractal basin with a dam-break reservoir (walls on every side,
    Grass bedload): the water volume cannot change."""
    w = W.dam_break_fractal(n=n, dx=dx, seed=seed, relief=relief, depth=depth).as_float32()
    w.bc = (0, 0, 0, 0)
    return w


def valley_basin(n, seed, depth, dx=5.0):
    """A closed basin on the terrain of the large river valley (fractal relief
    on a regional slope, a meandering carved channel, per-cell d50 and psi,
    Eq. 4 bedload; meander amplitude min(600 m, a quarter of the side)),
    walls on every side and no inflow: the upstream quarter holds a reservoir
    whose flat surface lies `depth` above the lowest twentieth of its bed (the
    channel), released at t = 0 down the channel and over its banks.  The
    water volume cannot change."""
    side = n * dx
    w = W.river_valley(n=n, dx=dx, seed=seed, amplitude=min(600.0, 0.25 * side))
    w.bc = (W.WALL, W.WALL, W.WALL, W.WALL)
    w.inflow_idx, w.inflow_w, w.Q_base, w.Q_peak = None, None, 0.0, 0.0
    q = n // 4
    level = float(np.quantile(w.b[:, :q], 0.05)) + depth
    H = np.zeros_like(w.b)
    H[:, :q] = np.maximum(0.0, level - w.b[:, :q])
    w.H = H
    w.name = f"valley_basin_{n}_{seed}"
    return w.as_float32()


# fixed step of the valley basins (dx = 5 m, depths up to about 11 m): below
# their Eq. 7 bound (K = 0.3) while |v| < 3 sqrt(g H_max), which the flood
# waves running down the 1024^2 valleys' slopes approach
VALLEY_DT = 0.02


def collect_valley(seeds, n, steps, k, stream=None, depth_range=(1.5, 4.0), spinup=(0, 600),
                   crop=None, count=None):
    """Pairs from valley basins of side n: each seed draws its reservoir depth
    and a spin-up of fixed steps (so the pairs cover the flood wave at
    different stages), then records steps // k consecutive pairs.  With crop,
    each pair keeps a crop x crop window around a wet cell drawn from the
    seed's generator (the basin is mostly dry).  A trajectory whose flow
    outruns the fixed step (SW_ERR_CFL from the solver) is dropped; with
    count, seeds are taken until that many trajectories are complete.
    Returns the pairs and the list of dropped seeds."""
    xs, ds, dts, dropped, done = [], [], [], [], 0
    for sd in seeds:
        if count is not None and done >= count:
            break
        rng = np.random.default_rng(sd)
        w = valley_basin(n, sd, float(rng.uniform(*depth_range)))
        s = csph.solver_for(w, stream=stream)
        tx, td = [], []
        try:
            n0 = int(rng.integers(spinup[0], spinup[1] + 1))
            if n0:
                s.advance(n0, dt=VALLEY_DT)
            f0 = s.get_fields()
            for _ in range(steps // k):
                s.advance(k, dt=VALLEY_DT)
                f1 = s.get_fields()
                h, hu, hv, b = f0
                x = np.stack([h, hu, hv, b, (h > 0).astype(np.float32)])
                d = np.stack([a1 - a0 for a1, a0 in zip(f1, f0)])
                if crop:
                    wet = np.flatnonzero(h > 0)
                    c = int(wet[rng.integers(len(wet))]) if len(wet) else int(rng.integers(h.size))
                    y0 = min(max(c // w.nx - crop // 2, 0), w.ny - crop)
                    x0 = min(max(c % w.nx - crop // 2, 0), w.nx - crop)
                    x = x[:, y0:y0 + crop, x0:x0 + crop].copy()
                    d = d[:, y0:y0 + crop, x0:x0 + crop].copy()
                tx.append(x)
                td.append(d)
                f0 = f1
        except csph.SwError as e:
            if e.code != csph.SW_ERR_CFL:
                raise
            dropped.append(sd)
            continue
        finally:
            s.close()
        xs += tx
        ds += td
        dts += [VALLEY_DT] * len(tx)
        done += 1
    if not xs:
        raise RuntimeError(f"no valley trajectory completed (dropped seeds {dropped})")
    return Pairs(np.stack(xs), np.stack(ds), k, np.array(dts)), dropped


def fixed_dt(w, factor=0.08):
    """dt = factor dx / sqrt(g H_max) of the trajectory's initial state; 0.08
    keeps it under the Eq. 7 step (K = 0.3) while |v| + c stays below about
    3.7 sqrt(g H_max), which covers the dam-break flows."""
    return factor * w.dx / math.sqrt(G * max(float(w.H.max()), 1e-3))


def trajectory_pairs(w, steps, k, dt, stream=None):
    """Run the solver for `steps` fixed steps and return the (state, change
    over k steps) pairs at every k-th step."""
    s = csph.solver_for(w, stream=stream)
    xs, ds = [], []
    f0 = s.get_fields()
    for _ in range(steps // k):
        s.advance(k, dt=dt)
        f1 = s.get_fields()
        h, hu, hv, b = f0
        xs.append(np.stack([h, hu, hv, b, (h > 0).astype(np.float32)]))
        ds.append(np.stack([a1 - a0 for a1, a0 in zip(f1, f0)]))
        f0 = f1
    s.close()
    return xs, ds


def collect(seeds, n, steps, k, stream=None, depth_range=(2.0, 8.0)):
    xs, ds, dts = [], [], []
    for sd in seeds:
        rng = np.random.default_rng(sd)
        w = basin(n, sd, float(rng.uniform(*depth_range)))
        dt = fixed_dt(w)
        x, d = trajectory_pairs(w, steps, k, dt, stream)
        xs += x
        ds += d
        dts += [dt] * len(x)
    return Pairs(np.stack(xs), np.stack(ds), k, np.array(dts))


def scales(p: Pairs):
    ins = [1.0 / max(float(np.abs(p.x[:, c]).max()), 1e-6) for c in range(4)] + [1.0]
    outs = [max(float(p.d[:, c].std()), 1e-9) for c in range(4)]
    return np.array(ins, np.float32), np.array(outs, np.float32)


def he_init(channels, seed):
    rng = np.random.default_rng(seed)
    parts = []
    for cin, cout in zip(channels[:-1], channels[1:]):
        bound = math.sqrt(6.0 / (9 * cin))
        parts.append(rng.uniform(-bound, bound, cout * cin * 9))
        parts.append(np.zeros(cout))
    return np.concatenate(parts).astype(np.float32)


def train(net, p: Pairs, in_s, out_s, steps, batch, lr, seed=0, log=None):
    """Scale the pairs and run the library's training loop (sws_train: Adam,
    cosine learning-rate decay, minibatches drawn on the host side of the
    library).  Returns the per-step losses."""
    net.set_scales(in_s, out_s)
    x = p.x * in_s[None, :, None, None]
    t = p.d / out_s[None, :, None, None]
    rep, losses = net.train(x, t, steps, batch, lr, seed=seed, keep_losses=True)
    if log:
        log(f"trained {steps} steps: loss {rep['first_loss']:.4e} -> {rep['final_loss']:.4e}")
    return list(losses)


def evaluate(net, p: Pairs, in_s, out_s):
    """Largest depth error of one surrogate call over the pairs, and the
    relative volume change each prediction would make."""
    y = net.forward(p.x * in_s[None, :, None, None])
    dh = y[:, 0] * out_s[0]
    err = np.abs(dh - p.d[:, 0]).max(axis=(1, 2))
    vol = p.x[:, 0].sum(axis=(1, 2)).astype(np.float64)
    h_new = np.maximum(p.x[:, 0] + dh, 0.0)
    drift = np.abs(h_new.sum(axis=(1, 2)) - vol) / np.maximum(vol, 1e-30)
    return err, drift


def measure_gain(net, w, dt, calls, k=8, max_drift=1e-5, check_every=4, max_err=5e-3,
                 stream=None):
    """Effective rate of the surrogate step (sws_advance_K: k steps per call,
    the conservation and stability checks every call and the plain step
    judging every check_every-th call, fall backs included) against the plain solver's k
    fixed steps over the same model time, both in grid cells x steps per
    second, from the same initial state; graphs and set-up are done before
    either timing."""
    import torch
    s = csph.solver_for(w, stream=stream)
    s.advance(k, dt=dt)  # the step graphs are built here
    s.reset(w)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = net.advance_k(s, calls, k, dt, max_drift, check_every, max_err)
    torch.cuda.synchronize()
    t_sur = time.perf_counter() - t0
    s.reset(w)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.advance(calls * k, dt=dt)
    s.sync()
    t_plain = time.perf_counter() - t0
    s.close()
    cells = w.nx * w.ny * k * calls
    return {"grid": [w.nx, w.ny], "k": k, "calls": calls, "max_drift": max_drift,
            "check_every": check_every, "max_err_m": max_err,
            "surrogate_gcell_steps_s": round(cells / t_sur / 1e9, 3),
            "plain_gcell_steps_s": round(cells / t_plain / 1e9, 3),
            "kept": stats["kept"], "fallbacks_volume": stats["fallbacks_volume"],
            "fallbacks_residual": stats["fallbacks_residual"],
            "fallbacks_stability": stats["fallbacks_stability"], "checks": stats["checks"],
            "max_residual_m": round(stats["max_residual"], 6),
            "fallback_rate": round(1.0 - stats["kept"] / calls, 4)}
