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


def test_gpu_resume_from_a_checkpoint_is_bitwise():
    """Checkpoint mid-run, load the blob into a fresh solver and continue:
    identical fields, time, step and balances to the uninterrupted run
    (inflow hydrograph, per-cell soil, bed sources, open boundary)."""
    from paper_2103_15196_amd import csph
    w = _small_valley()
    w.qb = np.zeros((w.ny, w.nx))
    w.qb[60:70, 100:110] = 2e-6
    st = torch_stream()
    ref = csph.solver_for(w, stream=st)
    ref.advance(300)
    f_ref, s_ref = ref.get_fields(), ref.get_sums()
    ref.close()
    a = csph.solver_for(w, stream=st)
    a.advance(171)
    blob = a.checkpoint()
    sa = a.get_sums()
    a.close()
    say(f"checkpoint at step {sa['step']}, t = {sa['t']:.6f} s, {blob.size} bytes")
    r = csph.solver_for(w, stream=st)
    r.advance(7)                   # whatever it held before is replaced
    r.restore(blob)
    assert r.get_sums()["step"] == 171
    r.advance(129)
    f, s = r.get_fields(), r.get_sums()
    for x, y in zip(f, f_ref):
        assert np.array_equal(x, y)
    for k in ("t", "step", "water_volume", "sediment_volume", "water_boundary_out",
              "water_source_in", "sed_boundary_out", "sed_source_in"):
        assert s[k] == s_ref[k], k
    other = csph.Solver(w.nx + 1, w.ny, w.dx, w.bc, stream=st)
    with pytest.raises(csph.SwError) as e:
        other.restore(blob)
    assert e.value.code == csph.SW_ERR_ARG
    other.close()
    r.close()


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


def test_gpu_async_save_snapshots_the_state_while_steps_go_on():
    """sw_save_begin takes the state after the queued steps and copies it on
    a second stream while later steps run: the snapshot equals the state a
    plain run reads at that step, the run itself is unchanged, and out-of-order
    calls are SW_ERR_STATE."""
    from paper_2103_15196_amd import csph
    import torch
    w = W.dam_break_fractal(n=200, ny=150, dx=2.0, seed=21, relief=8.0, depth=5.0).as_float32()
    stream = torch.cuda.Stream().cuda_stream
    a = csph.solver_for(w, stream=stream)
    with pytest.raises(csph.SwError) as e:
        a.save_wait()
    assert e.value.code == csph.SW_ERR_STATE
    a.advance(30)
    a.save_begin()
    with pytest.raises(csph.SwError) as e:
        a.save_begin()
    assert e.value.code == csph.SW_ERR_STATE
    a.advance(30)
    h, hu, hv, b, t, step = a.save_wait()
    end = a.get_fields()
    ref = csph.solver_for(w, stream=stream)
    ref.advance(30)
    r30, s30 = ref.get_fields(), ref.get_sums()
    ref.advance(30)
    r60 = ref.get_fields()
    for x, y in zip((h, hu, hv, b), r30):
        assert np.array_equal(x, y)
    assert t == s30["t"] and step == 30
    for x, y in zip(end, r60):
        assert np.array_equal(x, y)
    a.close()
    ref.close()


def test_gpu_step_bound_is_the_next_steps_eq7_step():
    """sw_step_bound takes the Eq. 7 maxima over the current fields as the
    next step's K3 takes them: on a fresh all-wet river valley and again 60
    steps later it equals the step the solver then takes; a fixed step equal
    to it runs, one a millionth above it raises SW_ERR_CFL on the device; a
    NaN in the fields is SW_ERR_NONFINITE."""
    import torch
    from paper_2103_15196_amd import csph
    w = _small_valley()
    w.H = np.full((w.ny, w.nx), 0.5)
    w = w.as_float32()
    s = csph.solver_for(w, stream=torch_stream())
    for n in (0, 60):
        if n:
            s.advance(n)
        bound = s.step_bound()
        s.advance(1)
        last = s.get_sums()["last_dt"]
        say(f"after {n} steps: bound {bound!r}, step taken {last!r}")
        assert last == bound
    bound = s.step_bound()
    s.advance(1, dt=bound)
    s.sync()
    bound = s.step_bound()
    s.advance(1, dt=bound * (1.0 + 1e-6))
    with pytest.raises(csph.SwError) as e:
        s.sync()
    assert e.value.code == csph.SW_ERR_CFL
    s.reset(w)
    dev = torch.device("cuda:0")
    t = [torch.tensor(x, dtype=torch.float32, device=dev).contiguous() for x in s.get_fields()]
    t[2][10, 12] = float("nan")
    assert csph.lib.sw_replace_state(s.ctx, t[0].data_ptr(), t[1].data_ptr(), t[2].data_ptr(),
                                     t[3].data_ptr(), 0.0, 0) == csph.SW_OK
    with pytest.raises(csph.SwError) as e:
        s.step_bound()
    assert e.value.code == csph.SW_ERR_NONFINITE
    s.close()


def test_gpu_step_log_records_each_step():
    """The step log (the Screen block's record) holds one record per step:
    the times chain exactly (t + dt is the next record's t), the last record
    is what sw_get_sums reports (step length, Eq. 7 maxima, binding term),
    the inflow is the hydrograph at t + dt/2; fixed steps record binding 4;
    past SW_STEP_LOG steps only the last ones remain, consecutive; a new
    state clears it."""
    import math
    from paper_2103_15196_amd import csph
    w = _small_valley()
    s = csph.solver_for(w, stream=torch_stream())
    s.advance(50)
    log = s.step_log()
    assert [r["step"] for r in log] == list(range(50))
    for a, b in zip(log, log[1:]):
        assert b["t"] == a["t"] + a["dt"]
    sums = s.get_sums()
    last = log[-1]
    assert last["dt"] == sums["last_dt"] and last["binding"] == sums["binding_term"]
    assert (last["vp"], last["vs"], last["D"]) == (sums["vp"], sums["vs"], sums["D"])
    assert sums["t"] == last["t"] + last["dt"]
    for r in log:
        d = r["t"] + 0.5 * r["dt"] - w.t_peak
        q = w.Q_base + w.Q_peak * math.exp(-d * d / (2.0 * w.t_sigma ** 2))
        assert abs(r["inflow"] - q) <= 1e-12 * q
    s.advance(1100, dt=0.05)
    log = s.step_log()
    assert len(log) == csph.SW_STEP_LOG
    assert [r["step"] for r in log] == list(range(1150 - csph.SW_STEP_LOG, 1150))
    assert all(r["binding"] == 4 and r["dt"] == 0.05 for r in log)
    assert len(s.step_log(10)) == 10 and s.step_log(10)[-1]["step"] == 1149
    s.reset(w)
    assert s.step_log() == []
    s.close()
