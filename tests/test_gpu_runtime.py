"""Runtime behaviour of the C ABI on the GPU: graphs kept across a new state,
resume from saved fields (bitwise), and errors raised on the device
(non-finite state, Eq. 7 step below dt_min) returned through the ABI."""
import numpy as np
import pytest

from paper_2103_15196_amd import workloads as W
from tests.gpu_common import say, torch_stream

pytestmark = pytest.mark.gpu


def _small_valley():
    w = W.river_valley(n=200, ny=136, dx=5.0, amplitude=60.0, wavelength=500.0, width=40.0,
                       Q_base=20.0, Q_peak=200.0, t_peak=40.0, t_sigma=15.0)
    return w.as_float32()


def test_gpu_new_state_keeps_the_step_graphs():
    """A new state, bed or time lands in the same device planes: the captured
    step graphs are kept (no capture inside a timed advance after a reset);
    changing a kernel argument (soil) rebuilds them."""
    from paper_2103_15196_amd import csph
    w = W.dam_break_fractal(n=300, ny=236, dx=2.0, seed=7, relief=10.0, depth=8.0).as_float32()
    s = csph.solver_for(w, stream=torch_stream())
    s.advance(40)
    a = s.get_fields()
    assert s.get_sums()["graph_builds"] == 1
    s.reset(w)
    s.advance(40)
    b = s.get_fields()
    assert s.get_sums()["graph_builds"] == 1
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    s.set_soil(w.nM, w.d50, w.psi)
    s.reset(w)
    s.advance(40)
    assert s.get_sums()["graph_builds"] == 2
    for x, y in zip(a, s.get_fields()):
        assert np.array_equal(x, y)
    s.close()


def test_gpu_resume_from_saved_fields_is_bitwise():
    """Save mid-run (fields, time, step), restore them into a fresh solver and
    continue: identical bits to the uninterrupted run, inflow hydrograph
    included (the step depends only on the state, the bed and the time)."""
    from paper_2103_15196_amd import csph
    w = _small_valley()
    st = torch_stream()
    ref = csph.solver_for(w, stream=st)
    ref.advance(300)
    f_ref, s_ref = ref.get_fields(), ref.get_sums()
    ref.close()
    a = csph.solver_for(w, stream=st)
    a.advance(170)
    h, hu, hv, b = a.get_fields()
    sa = a.get_sums()
    a.close()
    say(f"saved at step {sa['step']}, t = {sa['t']:.6f} s")
    r = csph.solver_for(w, stream=st)
    r.set_bed(b)
    r.set_state(h, hu, hv)
    r.set_time(sa["t"], sa["step"])
    r.advance(130)
    f, s = r.get_fields(), r.get_sums()
    r.close()
    for x, y in zip(f, f_ref):
        assert np.array_equal(x, y)
    assert s["t"] == s_ref["t"] and s["step"] == s_ref["step"] == 300


def test_gpu_nonfinite_state_is_raised_by_the_device():
    """A NaN installed through sw_replace_state (no host check on that path)
    is found by the device's Eq. 7 pass: SW_ERR_NONFINITE through sw_sync,
    later steps do not run, and a new state clears the error."""
    import torch
    from paper_2103_15196_amd import csph
    w = W.dam_break_1d(nx=128, ny=48, x_dam=64).as_float32()
    s = csph.solver_for(w, stream=torch_stream())
    s.advance(10)
    dev = torch.device("cuda:0")
    t = [torch.tensor(x, dtype=torch.float32, device=dev).contiguous()
         for x in s.get_fields()]
    t[1][20, 30] = float("nan")
    rc = csph.lib.sw_replace_state(s.ctx, t[0].data_ptr(), t[1].data_ptr(), t[2].data_ptr(),
                                   t[3].data_ptr(), 1.0, 10)
    assert rc == csph.SW_OK
    s.advance(5)
    with pytest.raises(csph.SwError) as e:
        s.sync()
    assert e.value.code == csph.SW_ERR_NONFINITE
    st = csph.sw_sums()
    assert csph.lib.sw_get_sums(s.ctx, st) == csph.SW_OK
    assert st.error == csph.SW_ERR_NONFINITE and st.step == 10
    s.reset(w)
    s.advance(3)
    s.sync()
    s.close()


def test_gpu_dt_underflow_is_raised_by_the_device():
    """dt_min above the Eq. 7 step: SW_ERR_DT_UNDERFLOW raised on the device at
    the first step, state left at the start of that step."""
    from paper_2103_15196_amd import csph
    w = W.dam_break_1d(nx=128, ny=48, x_dam=64).as_float32()
    # first step of this dam break: 0.3 dx / sqrt(g 2 m) = 0.0677 s
    s = csph.solver_for(w, stream=torch_stream(), dt_min=0.1)
    s.advance(4)
    with pytest.raises(csph.SwError) as e:
        s.sync()
    assert e.value.code == csph.SW_ERR_DT_UNDERFLOW
    st = csph.sw_sums()
    assert csph.lib.sw_get_sums(s.ctx, st) == csph.SW_OK
    assert st.error == csph.SW_ERR_DT_UNDERFLOW and st.step == 0
    s.close()
    ok = csph.solver_for(w, stream=torch_stream(), dt_min=0.05)
    ok.advance(1)
    ok.sync()
    assert ok.get_sums()["last_dt"] == pytest.approx(0.3 / np.sqrt(9.81 * 2.0), rel=1e-6)
    ok.close()
