"""Helpers shared by the GPU tests: run a workload through the C ABI and through
the FP64 oracle from the same float32-rounded inputs, and compare them."""
from __future__ import annotations

import sys

import numpy as np

from tests.helpers import oracle_case


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def torch_stream():
    import torch
    assert torch.cuda.is_available()
    return torch.cuda.current_stream().cuda_stream


def run_gpu(w, steps, dt=None, flags=None, stream=None, shape=None, **params):
    """Run workload ``w`` for ``steps`` steps on the GPU (tile shape ``shape``
    if given); returns (fields, sums)."""
    from paper_2103_15196_amd import csph
    if flags is not None:
        params["flags"] = flags
    s = csph.solver_for(w, stream=stream if stream is not None else torch_stream(), **params)
    try:
        if shape is not None:
            s.set_tile_shape(*shape)
        if steps:
            s.advance(steps, dt)
        f = s.get_fields()
        sums = s.get_sums()
    finally:
        s.close()
    return f, sums


def run_oracle(O, w, steps, dt=None, **over):
    p, inp, st = oracle_case(O, w, **over)
    O.run(p, inp, st, steps, dt_fixed=dt or 0.0)
    return p, inp, st


# Precision target: L-inf depth error 1e-4 m against the FP64 oracle.  The bed
# elevation is held to the same 1e-4 m; the unit discharges to 1e-4 m times
# the largest wave speed max(|v| + c) of the oracle's final state (a depth
# error dh carried by a wave moves the discharge by (u +- c) dh).
LINF_H = 1e-4
# A cell counts as ill-conditioned when the oracle's own answer moves by more
# than COND times the field's bound when its inputs move by their float32
# rounding (oracle on the float64 inputs vs on the float32-rounded ones): no
# float32 path can be held to the bound there.  Such cells are counted and
# reported, and may make up at most ILL_MAX of the grid.
COND = 0.1
ILL_MAX = 1e-3


def field_check(fields, st, spread, vs):
    """Per-field errors of the FP32 GPU fields against the oracle state st,
    split by the oracle's input-rounding spread (None: no spread, every cell
    well conditioned).  Returns {field: dict(bound, err, n_ill, err_ill, worst)}."""
    out = {}
    for name, g, o, bound in (("h", fields[0], st.H, LINF_H), ("hu", fields[1], st.qx, LINF_H * vs),
                              ("hv", fields[2], st.qy, LINF_H * vs), ("b", fields[3], st.b, LINF_H)):
        e = np.abs(np.asarray(g, np.float64) - o)
        ill = (spread[name] >= COND * bound) if spread is not None else np.zeros(e.shape, bool)
        well = ~ill
        j = np.unravel_index(int(np.argmax(np.where(well, e, -1.0))), e.shape)
        out[name] = {"bound": bound, "err": float(e[well].max()) if well.any() else 0.0,
                     "n_ill": int(ill.sum()), "err_ill": float(e[ill].max()) if ill.any() else 0.0,
                     "n_over": int((e > bound).sum()), "worst": (int(j[1]), int(j[0]))}
    return out


def oracle_spread(O, w64, st, steps, dt=None, **over):
    """|oracle(float64 inputs) - oracle(float32 inputs)| per field: how far
    the FP64 answer itself moves under the float32 rounding of the inputs."""
    _, _, s64 = run_oracle(O, w64, steps, dt, **over)
    return {"h": np.abs(s64.H - st.H), "hu": np.abs(s64.qx - st.qx),
            "hv": np.abs(s64.qy - st.qy), "b": np.abs(s64.b - st.b)}


def compare(O, w, gpu, orc, wet_h=1e-4, w64=None, steps=None, dt=None):
    """Per-field errors of the FP32 GPU result against the FP64 oracle; with
    w64 (the scenario before float32 rounding) also the oracle's own spread."""
    (h, hu, hv, b), sums = gpu
    p, inp, st = orc
    dx2 = w.dx * w.dx
    V0 = float(np.sum(w.H)) * dx2
    Vg = sums["water_volume"]
    Vo = O.volumes(p, inp, st)[0]
    mask_g = h > wet_h
    mask_o = st.H > wet_h
    res = {
        "linf_h": float(np.abs(h - st.H).max()),
        "linf_hu": float(np.abs(hu - st.qx).max()),
        "linf_hv": float(np.abs(hv - st.qy).max()),
        "linf_b": float(np.abs(b - st.b).max()),
        "mass_drift_gpu": abs(Vg - V0 + sums["water_boundary_out"] - sums["water_source_in"])
        / max(V0 + sums["water_source_in"], 1e-300),
        "mass_gpu_vs_oracle": abs(Vg - Vo) / max(Vo, 1e-300),
        "mask_disagree": float(np.mean(mask_g != mask_o)),
        "t_gpu": sums["t"],
        "t_oracle": st.t,
    }
    vs = O.cfl(p, inp, st)["vs"]
    spread = oracle_spread(O, w64, st, steps, dt) if w64 is not None else None
    res["fields"] = field_check((h, hu, hv, b), st, spread, vs)
    res["cells"] = int(h.size)
    return res
