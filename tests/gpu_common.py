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


def compare(O, w, gpu, orc, wet_h=1e-4):
    """Per-field errors of the FP32 GPU result against the FP64 oracle."""
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
    return res
