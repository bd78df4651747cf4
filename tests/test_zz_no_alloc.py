"""The allocation-free advance (sw_advance_noalloc) against the solver's own
path (sw_create + sw_set_* + sw_advance + sw_get_fields) on the same inputs:
identical bits, two calls in a row on the one scratch array, the second on a
smaller grid."""
import numpy as np
import pytest

from paper_2103_15196_amd import workloads as W
from tests.gpu_common import run_gpu, say

pytestmark = pytest.mark.gpu


def _noalloc(w, steps, dt_fixed=0.0, flags=None):
    import torch
    from paper_2103_15196_amd import csph
    dev = torch.device("cuda")
    f = [torch.tensor(np.asarray(a, np.float32), device=dev).contiguous()
         for a in (w.H, w.qx, w.qy, w.b)]
    t_out = torch.full((1,), -1.0, dtype=torch.float64, device=dev)
    err_out = torch.full((1,), 99, dtype=torch.int32, device=dev)
    kw = dict(cfl=w.cfl, sed_law=w.sed_law)
    if flags is not None:
        kw["flags"] = flags
    params = csph.default_params(**kw)
    grid = csph.make_grid(w.nx, w.ny, w.dx, w.bc)
    stream = torch.cuda.current_stream().cuda_stream
    csph.advance_noalloc(grid, params, w.nM, w.d50, w.psi, *f, steps, dt_fixed=dt_fixed,
                         t_out=t_out, err_out=err_out, stream=stream)
    torch.cuda.synchronize()
    return [a.cpu().numpy() for a in f], float(t_out.item()), int(err_out.item())


def _same(w, steps, dt_fixed=0.0, flags=None):
    say(f"no-alloc case {w.name} {w.nx}x{w.ny}, {steps} steps, dt_fixed={dt_fixed}, flags={flags}")
    fields, t, err = _noalloc(w, steps, dt_fixed, flags)
    ref, sums = run_gpu(w, steps, dt=dt_fixed or None, flags=flags)
    assert err == 0
    assert t == sums["t"]
    for name, a, r in zip(("h", "hu", "hv", "b"), fields, ref):
        assert np.array_equal(a, r), (name, float(np.abs(a - r).max()))
    return fields


def test_gpu_noalloc_matches_the_solver_on_two_calls_in_a_row():
    big = W.dam_break_fractal(n=300, ny=236, dx=2.0, seed=7, relief=10.0, depth=8.0).as_float32()
    small = W.dam_break_1d(nx=130, ny=40, x_dam=60, steps=80).as_float32()
    f1 = _same(big, 150)
    assert float(np.abs(f1[1]).max()) > 0.1  # the flow moved
    _same(small, 80)
    # and once more at the large size, skipping off, fixed step
    _same(big, 40, dt_fixed=0.02, flags=0)


def test_gpu_noalloc_rejects_a_negative_depth_on_the_device():
    w = W.dam_break_1d(nx=64, ny=16, x_dam=32, steps=5).as_float32()
    w.H = w.H.copy()
    w.H[3, 7] = -1.0
    fields, t, err = _noalloc(w, 5)
    from paper_2103_15196_amd import csph
    assert err == csph.SW_ERR_ARG
    assert t == 0.0
    # no step ran: the caller's arrays hold the input again
    for a, r in zip(fields, (w.H, w.qx, w.qy, w.b)):
        assert np.array_equal(a, np.asarray(r, np.float32))
