"""The surrogate's kernels (BF16 matrix-core convolutions and weight
gradients, FP32 Adam) against the FP64 oracle of the network, its training
loop, and its solver step (conservation and residual checks, plain fall
back) against the solver itself."""
import numpy as np
import pytest

from oracle import surrogate_oracle as S
from paper_2103_15196_amd import workloads as W
from tests.gpu_common import say

pytestmark = pytest.mark.gpu

DESIGN = (5, 48, 48, 48, 48, 48, 4)


def _flat(Ws, bs):
    return np.concatenate([np.concatenate([w.reshape(-1), b]) for w, b in zip(Ws, bs)])


def _unflat(p, chans):
    Ws, bs, o = [], [], 0
    for cin, cout in zip(chans[:-1], chans[1:]):
        n = cout * cin * 9
        Ws.append(p[o:o + n].reshape(cout, cin, 3, 3))
        o += n
        bs.append(p[o:o + cout])
        o += cout
    return Ws, bs


def _net(chans, seed):
    from paper_2103_15196_amd import csph
    import torch
    Ws, bs = S.init_weights(chans, seed)
    rng = np.random.default_rng(seed + 1)
    bs = [rng.uniform(-0.1, 0.1, b.shape) for b in bs]
    p = _flat(Ws, bs).astype(np.float32)
    net = csph.Surrogate(chans, stream=torch.cuda.current_stream().cuda_stream)
    net.set_params(p)
    Ws, bs = _unflat(p.astype(np.float64), chans)
    return net, Ws, bs


@pytest.mark.parametrize("chans", [DESIGN, (5, 8, 4), (5, 16, 11, 4)])
def test_gpu_surrogate_forward_matches_oracle(chans):
    net, Ws, bs = _net(chans, seed=10)
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 5, 23, 37)).astype(np.float32)
    y = net.forward(x)
    for i in range(2):
        ref, _ = S.forward(x[i].astype(np.float64), Ws, bs, bf16=True)
        err = np.abs(y[i] - ref).max()
        say(f"forward {chans} image {i}: max |gpu - oracle| {err:.3e}, max |oracle| {np.abs(ref).max():.3e}")
        assert err <= 5e-3 * np.abs(ref).max() + 1e-4
    net.close()


def test_gpu_surrogate_forward_spans_several_tiles():
    """An image wider than two 64-pixel strips and taller than two 32-row
    segments, with ragged tails in both directions."""
    net, Ws, bs = _net(DESIGN, seed=12)
    rng = np.random.default_rng(7)
    x = rng.standard_normal((1, 5, 71, 150)).astype(np.float32)
    y = net.forward(x)
    ref, _ = S.forward(x[0].astype(np.float64), Ws, bs, bf16=True)
    err = np.abs(y[0] - ref).max()
    say(f"forward 71x150: max |gpu - oracle| {err:.3e}, max |oracle| {np.abs(ref).max():.3e}")
    assert err <= 5e-3 * np.abs(ref).max() + 1e-4
    net.close()


# (1101, 70): the weight-gradient kernel's work items span several rows (its
# ring of staged input rows is reused) and the last item of a strip is
# shorter; (3, 16640): more 64-pixel strips than workgroups, so workgroups
# take several items
@pytest.mark.parametrize("chans,hw", [((5, 16, 11, 4), (19, 41)), (DESIGN, (19, 41)),
                                     (DESIGN, (45, 133)), (DESIGN, (1101, 70)),
                                     (DESIGN, (3, 16640))])
def test_gpu_surrogate_gradients_match_oracle(chans, hw):
    net, Ws, bs = _net(chans, seed=20)
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2, 5) + hw).astype(np.float32)
    t = rng.standard_normal((2, 4) + hw).astype(np.float32)
    g, loss = net.grad(x, t)
    gW = [np.zeros_like(w) for w in Ws]
    gb = [np.zeros_like(b) for b in bs]
    lref = 0.0
    for i in range(2):
        out, cache = S.forward(x[i].astype(np.float64), Ws, bs, bf16=True)
        d = out - t[i]
        lref += float(np.sum(d * d))
        dW, db = S.backward(Ws, cache, 2.0 * d / t.size, bf16=True)
        for l in range(len(Ws)):
            gW[l] += dW[l]
            gb[l] += db[l]
    lref /= t.size
    assert loss == pytest.approx(lref, rel=2e-3)
    ref = _flat(gW, gb)
    o = 0
    for l, (w, b) in enumerate(zip(gW, gb)):
        n = w.size + b.size
        err = np.abs(g[o:o + n] - ref[o:o + n]).max()
        scale = np.abs(ref[o:o + n]).max()
        say(f"grad {chans} {hw} layer {l}: max err {err:.3e} of max {scale:.3e}")
        assert err <= 3e-2 * scale + 1e-7
        # the direction of the layer gradient agrees closely
        cos = float(np.dot(g[o:o + n], ref[o:o + n]) /
                    (np.linalg.norm(g[o:o + n]) * np.linalg.norm(ref[o:o + n]) + 1e-30))
        assert cos > 0.999
        o += n
    net.close()


def test_gpu_surrogate_adam_step_matches_oracle():
    chans = (5, 16, 4)
    net, Ws, bs = _net(chans, seed=30)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((1, 5, 16, 32)).astype(np.float32)
    t = rng.standard_normal((1, 4, 16, 32)).astype(np.float32)
    p0 = net.get_params().astype(np.float64)
    g, _ = net.grad(x, t)
    net.train_step(x, t, lr=1e-3)
    p1 = net.get_params()
    ref = [p0.copy()]
    S.adam_step(ref, [g.astype(np.float64)], [np.zeros_like(p0)], [np.zeros_like(p0)], t=1, lr=1e-3)
    assert np.abs(p1 - ref[0]).max() <= 1e-6
    net.close()


def test_gpu_surrogate_training_reduces_loss():
    chans = (5, 16, 4)
    net, _, _ = _net(chans, seed=40)
    rng = np.random.default_rng(6)
    x = rng.standard_normal((4, 5, 24, 24)).astype(np.float32)
    t = 0.5 * np.roll(x[:, :4], 1, axis=3)  # a shift the 3x3 stencil can represent
    losses = [net.train_step(x, t, lr=3e-3) for _ in range(150)]
    say(f"training loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert losses[-1] < 0.3 * losses[0]
    net.close()


def _closed_basin():
    w = W.dam_break_fractal(n=96, ny=64, dx=2.0, seed=5, relief=3.0, depth=3.0).as_float32()
    w.bc = (0, 0, 0, 0)
    return w


def test_gpu_surrogate_step_keeps_or_falls_back():
    from paper_2103_15196_amd import csph
    import torch
    st = torch.cuda.current_stream().cuda_stream
    w = _closed_basin()
    dt = 0.02
    # zero network: the predicted change is 0, the volume is kept, the state stays
    net = csph.Surrogate((5, 16, 4), stream=st)
    net.set_params(np.zeros(net.nparam, np.float32))
    s = csph.solver_for(w, stream=st)
    used = net.advance(s, 8, dt)
    assert used
    h, hu, hv, b = s.get_fields()
    assert np.array_equal(h, w.H.astype(np.float32)) and np.array_equal(b, w.b.astype(np.float32))
    sums = s.get_sums()
    assert sums["t"] == pytest.approx(8 * dt, rel=1e-12) and sums["step"] == 8
    # the solver continues from the replaced state
    s.advance(5, dt=dt)
    s.sync()
    s.close()
    # a wild network changes the volume: the solver takes the 8 fixed steps itself
    wild = csph.Surrogate((5, 16, 4), stream=st)
    wild.set_params(np.random.default_rng(7).uniform(-1, 1, wild.nparam).astype(np.float32))
    wild.set_scales([1, 1, 1, 1, 1], [1, 1, 1, 1])
    s = csph.solver_for(w, stream=st)
    used = wild.advance(s, 8, dt)
    assert not used
    f = s.get_fields()
    r = csph.solver_for(w, stream=st)
    r.advance(8, dt=dt)
    g = r.get_fields()
    for a, c in zip(f, g):
        assert np.array_equal(a, c)
    s.close()
    r.close()
    net.close()
    wild.close()


def test_gpu_surrogate_training_driver_end_to_end():
    """Trajectories from the solver, a short training run, held-out error and
    volume change, and the gain measurement (conservation and residual
    checks, fall backs included)."""
    import torch
    from paper_2103_15196_amd import csph, surrogate as SG
    st = torch.cuda.current_stream().cuda_stream
    tr = SG.collect([5000, 5001], n=48, steps=32, k=8, stream=st)
    ho = SG.collect([6000], n=48, steps=32, k=8, stream=st)
    assert tr.x.shape == (8, 5, 48, 48) and tr.d.shape == (8, 4, 48, 48)
    ins, outs = SG.scales(tr)
    net = csph.Surrogate((5, 16, 16, 4), stream=st)
    net.set_params(SG.he_init((5, 16, 16, 4), 1))
    xs = tr.x * ins[None, :, None, None]
    ts = tr.d / outs[None, :, None, None]
    net.set_scales(ins, outs)
    _, before = net.grad(xs, ts)
    losses = SG.train(net, tr, ins, outs, steps=200, batch=4, lr=3e-3)
    _, after = net.grad(xs, ts)
    assert after < 0.8 * before
    err, drift = SG.evaluate(net, ho, ins, outs)
    assert np.all(np.isfinite(err)) and np.all(np.isfinite(drift))
    w = SG.basin(64, 6100, 4.0)
    res = SG.measure_gain(net, w, SG.fixed_dt(w), calls=2, k=8, stream=st)
    say(f"end to end: training-set loss {before:.3f} -> {after:.3f}; held-out max err {err.max():.3e}; {res}")
    assert res["calls"] == 2 and 0.0 <= res["fallback_rate"] <= 1.0
    net.close()


def test_gpu_surrogate_plain_step_judges_the_prediction():
    """sws_advance_K with the residual check on every call: a network that
    predicts no change keeps a still lake (residual 0) but is overruled on a
    dam break, where the solver's own k steps are kept (the final state is the
    plain run's, bit for bit)."""
    from paper_2103_15196_amd import csph
    import torch
    st = torch.cuda.current_stream().cuda_stream
    net = csph.Surrogate((5, 16, 4), stream=st)
    net.set_params(np.zeros(net.nparam, np.float32))
    lake = W.lake_at_rest(64, 48, bc=(0, 0, 0, 0)).as_float32()
    s = csph.solver_for(lake, stream=st)
    stats = net.advance_k(s, 3, 8, 0.05, check_every=1, max_err=5e-3)
    say(f"lake: {stats}")
    assert stats["kept"] == 3 and stats["checks"] == 3 and stats["max_residual"] == 0.0
    assert np.array_equal(s.get_fields()[0], np.asarray(lake.H, np.float32))
    s.close()
    w = _closed_basin()
    dt = 0.02
    s = csph.solver_for(w, stream=st)
    stats = net.advance_k(s, 3, 8, dt, check_every=1, max_err=5e-3)
    say(f"dam break: {stats}")
    assert stats["kept"] == 0 and stats["fallbacks_residual"] == 3 and stats["max_residual"] > 5e-3
    r = csph.solver_for(w, stream=st)
    r.advance(24, dt=dt)
    for a, c in zip(s.get_fields(), r.get_fields()):
        assert np.array_equal(a, c)
    assert s.get_sums()["t"] == pytest.approx(24 * dt, rel=1e-12)
    s.close()
    r.close()
    net.close()


def test_gpu_surrogate_unstable_prediction_falls_back():
    """A prediction that keeps the water and bed volumes but carries momentum
    the solver's Eq. 7 step cannot take (+1000 m^2/s of hu on every cell) is
    not kept: the call's start is restored and the plain steps are taken, so
    the final state is the plain run's, bit for bit."""
    from paper_2103_15196_amd import csph
    import torch
    st = torch.cuda.current_stream().cuda_stream
    net = csph.Surrogate((5, 16, 4), stream=st)
    p = np.zeros(net.nparam, np.float32)
    p[16 * 5 * 9 + 16 + 4 * 16 * 9 + 1] = 1.0  # bias of the hu output
    net.set_params(p)
    net.set_scales(np.ones(5, np.float32), np.array([0.0, 1000.0, 0.0, 0.0], np.float32))
    lake = W.lake_at_rest(64, 48, bc=(0, 0, 0, 0)).as_float32()
    dt = 0.05
    s = csph.solver_for(lake, stream=st)
    stats = net.advance_k(s, 3, 8, dt, check_every=0)
    say(f"unstable: {stats}")
    assert stats["kept"] == 0 and stats["fallbacks_stability"] == 3
    assert stats["fallbacks_volume"] == 0 and stats["max_volume_drift"] == 0.0
    r = csph.solver_for(lake, stream=st)
    r.advance(24, dt=dt)
    for a, c in zip(s.get_fields(), r.get_fields()):
        assert np.array_equal(a, c)
    assert s.get_sums()["t"] == pytest.approx(24 * dt, rel=1e-12)
    s.close()
    r.close()
    net.close()


def test_gpu_surrogate_corrupt_weights_fall_back_to_the_plain_steps():
    """Weights that make every prediction NaN: every call falls back on the
    conservation check, and the final state is the plain run's, bit for bit."""
    from paper_2103_15196_amd import csph
    import torch
    st = torch.cuda.current_stream().cuda_stream
    net = csph.Surrogate((5, 16, 4), stream=st)
    net.set_params(np.full(net.nparam, np.nan, np.float32))
    w = _closed_basin()
    dt = 0.02
    s = csph.solver_for(w, stream=st)
    stats = net.advance_k(s, 3, 8, dt, check_every=0)
    say(f"corrupt: {stats}")
    assert stats["kept"] == 0 and stats["fallbacks_volume"] == 3
    r = csph.solver_for(w, stream=st)
    r.advance(24, dt=dt)
    for a, c in zip(s.get_fields(), r.get_fields()):
        assert np.array_equal(a, c)
    s.close()
    r.close()
    net.close()


def test_gpu_surrogate_training_loop_is_deterministic_and_learns():
    """sws_train (minibatches from a seed, cosine learning rate) lowers the
    loss, reports it, and repeats bit for bit from the same seed."""
    from paper_2103_15196_amd import csph, surrogate as SG
    import torch
    st = torch.cuda.current_stream().cuda_stream
    tr = SG.collect([5000, 5001, 5002], n=48, steps=32, k=8, stream=st)
    ins, outs = SG.scales(tr)
    x = tr.x * ins[None, :, None, None]
    t = tr.d / outs[None, :, None, None]
    params = []
    for _ in range(2):
        net = csph.Surrogate((5, 16, 16, 4), stream=st)
        net.set_params(SG.he_init((5, 16, 16, 4), 3))
        net.set_scales(ins, outs)
        rep, losses = net.train(x, t, 150, 4, 3e-3, seed=11, keep_losses=True)
        assert rep["final_loss"] < 0.8 * rep["first_loss"]
        assert rep["first_loss"] == pytest.approx(float(losses[0]), rel=1e-6)
        params.append(net.get_params())
        net.close()
    assert np.array_equal(params[0], params[1])


def test_gpu_valley_trajectories_windows_and_drops():
    """collect_valley on 1024^2-style valley basins (small here): consecutive
    pairs, windows around a wet cell, the change equal to the difference of
    the solver's states; a seed whose flow outruns the fixed step is dropped
    and the next taken (forced here with a step far above Eq. 7's)."""
    from paper_2103_15196_amd import csph, surrogate as SG
    import torch
    st = torch.cuda.current_stream().cuda_stream
    p, dropped = SG.collect_valley(range(5000, 5004), 128, 16, 8, stream=st, crop=64, count=2,
                                   spinup=(0, 50))
    assert dropped == [] and p.x.shape == (4, 5, 64, 64) and p.d.shape == (4, 4, 64, 64)
    assert all((x[0] > 0).any() for x in p.x)
    assert np.array_equal(p.x[:, 4], (p.x[:, 0] > 0).astype(np.float32))
    # pairs of one trajectory are consecutive: whole grids (no window) chain exactly
    q, _ = SG.collect_valley([5000], 128, 16, 8, stream=st, spinup=(0, 50))
    np.testing.assert_allclose(q.x[0, 0] + q.d[0, 0], q.x[1, 0], rtol=0, atol=1e-6)
    old = SG.VALLEY_DT
    try:
        SG.VALLEY_DT = 5.0
        with pytest.raises(RuntimeError) as e:
            SG.collect_valley(range(5000, 5003), 96, 8, 8, stream=st, count=1)
        assert "5000, 5001, 5002" in str(e.value)
    finally:
        SG.VALLEY_DT = old


def test_gpu_surrogate_training_rejects_rows_beyond_the_kernel_limit():
    """Training calls refuse images whose row of 48 BF16 channels would
    exceed a 31-bit byte count (the weight-gradient kernel's buffer
    resource spans one row) with SW_ERR_ARG and a message, before reading
    the inputs; the net keeps training at ordinary sizes afterwards."""
    import ctypes as C
    from paper_2103_15196_amd import csph
    net, _, _ = _net(DESIGN, seed=3)
    buf = np.zeros(16, np.float32)  # never read: the call is refused first
    nx = 2**31 // 96 + 1
    rc = csph.lib.sws_grad(net.ctx, buf.ctypes.data, buf.ctypes.data, 1, nx, 1, buf.ctypes.data,
                           None, csph.SW_PTR_HOST)
    assert rc == csph.SW_ERR_ARG
    assert b"nx" in csph.lib.sws_last_error(net.ctx)
    cfg = csph.sws_train_cfg(1, 1, 1e-3, 0)
    rep = csph.sws_train_report()
    rc = csph.lib.sws_train(net.ctx, buf.ctypes.data, buf.ctypes.data, 1, nx, 1, C.byref(cfg),
                            C.byref(rep), None, csph.SW_PTR_HOST)
    assert rc == csph.SW_ERR_ARG
    assert b"nx" in csph.lib.sws_last_error(net.ctx)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((1, 5, 9, 70)).astype(np.float32)
    t = rng.standard_normal((1, 4, 9, 70)).astype(np.float32)
    g, loss = net.grad(x, t)
    assert np.isfinite(loss) and np.all(np.isfinite(g))
    net.close()
