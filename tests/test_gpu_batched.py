"""The ensemble path: members of uneven sizes with their own terrain, soil,
inflow and Eq. 7 step advance together (one launch per stage per step) and
each produces exactly the bits it produces alone; one member is also checked
against the FP64 oracle."""
import numpy as np
import pytest

from paper_2103_15196_amd import workloads as W
from tests.gpu_common import compare, run_oracle, say

pytestmark = pytest.mark.gpu


def _members():
    ms = W.ensemble(count=5, seed0=1000, n_min=70, n_max=330, steps=150)
    ms = [m.as_float32() for m in ms]
    rv = W.river_valley(n=150, ny=97, dx=5.0, amplitude=40.0, wavelength=400.0, width=40.0,
                        Q_base=20.0, Q_peak=100.0, t_peak=20.0, t_sigma=8.0).as_float32()
    ms.append(rv)
    ms.append(W.dam_break_1d(nx=96, ny=17, x_dam=40).as_float32())
    return ms


def _solo(w, steps, stream):
    from paper_2103_15196_amd import csph
    s = csph.solver_for(w, stream=stream)
    s.advance(steps)
    f, sums = s.get_fields(), s.get_sums()
    s.close()
    return f, sums


@pytest.mark.parametrize("shape", [(64, 8), (64, 4), (58, 16)])
def test_gpu_batch_equals_members_alone(shape):
    import torch
    from paper_2103_15196_amd import csph
    stream = torch.cuda.Stream()
    ms = _members()
    steps = 151  # odd: exercises the eager step after the graph pairs
    solvers = [csph.solver_for(w, stream=stream.cuda_stream) for w in ms]
    b = csph.Batch(solvers)
    b.set_tile_shape(*shape)
    b.advance(steps)
    b.sync()
    for k, (w, s) in enumerate(zip(ms, solvers)):
        f, sums = s.get_fields(), s.get_sums()
        rf, rsums = _solo(w, steps, stream.cuda_stream)
        say(f"member {k} {w.nx}x{w.ny}: t={sums['t']:.4f} solo t={rsums['t']:.4f}")
        for a, r in zip(f, rf):
            assert np.array_equal(a, r), (k, w.name)
        assert sums["t"] == rsums["t"] and sums["step"] == steps
    ts = {round(s.get_sums()["t"], 6) for s in solvers}
    assert len(ts) > 3  # members really took their own time steps
    b.close()
    for s in solvers:
        s.close()


def test_gpu_batch_member_matches_oracle():
    import torch
    from oracle import oracle as O
    from paper_2103_15196_amd import csph
    O.build(force=False)
    stream = torch.cuda.Stream()
    ms = _members()
    solvers = [csph.solver_for(w, stream=stream.cuda_stream) for w in ms]
    b = csph.Batch(solvers)
    b.advance(200)
    b.sync()
    for k in (0, len(ms) - 2):
        w = ms[k]
        res = compare(O, w, (solvers[k].get_fields(), solvers[k].get_sums()), run_oracle(O, w, 200))
        say(f"member {k}: {res}")
        assert res["linf_h"] <= 1e-4 and res["mass_drift_gpu"] <= 1e-6
        assert res["mask_disagree"] <= 1e-3
    b.close()
    for s in solvers:
        s.close()


def test_gpu_batch_rejects_mixed_parity():
    import torch
    from paper_2103_15196_amd import csph
    stream = torch.cuda.Stream()
    ms = _members()[:2]
    solvers = [csph.solver_for(w, stream=stream.cuda_stream) for w in ms]
    solvers[0].advance(1)
    b = csph.Batch(solvers)
    with pytest.raises(csph.SwError) as e:
        b.advance(2)
    assert e.value.code == csph.SW_ERR_STATE
    solvers[1].advance(1)
    b.advance(2)
    b.sync()
    b.close()
    for s in solvers:
        s.close()


def test_gpu_batch_full_size_member_matches_oracle():
    """A member of the ensemble's full size (1024 x 1024, within the 256..1536
    range of the 64-member workload: own fractal bed, reservoir depth, Manning
    n) advanced in a batch beside small members, read through swb_get_fields
    / swb_get_sums, against the FP64 oracle on every cell (cells
    ill-conditioned at float32 precision counted apart)."""
    import torch
    from oracle import oracle as O
    from paper_2103_15196_amd import csph
    from tests.test_gpu_parity import _check
    O.build(force=False)
    stream = torch.cuda.Stream()
    big = W.dam_break_fractal(n=1024, dx=2.0, seed=1017, relief=10.0, dam_height=1.0, depth=6.5,
                              manning=0.027).as_float32()
    ms = [big] + _members()[:3]
    solvers = [csph.solver_for(w, stream=stream.cuda_stream) for w in ms]
    b = csph.Batch(solvers)
    steps = 160
    say(f"case batch member 1024x1024, {steps} steps")
    b.advance(steps)
    b.sync()
    f, sums = b.get_fields(0), b.get_sums(0)
    assert sums["step"] == steps
    res = compare(O, big, (f, sums), run_oracle(O, big, steps), spread=True, steps=steps)
    _check(res)
    b.close()
    for s in solvers:
        s.close()


def test_gpu_batch_autotune_keeps_states_and_bits():
    """swb_autotune times every tile shape from the members' states, puts the
    states back and keeps the fastest shape; the batch then still gives each
    member's bits alone."""
    import torch
    from paper_2103_15196_amd import csph
    stream = torch.cuda.Stream()
    ms = _members()[:4]
    solvers = [csph.solver_for(w, stream=stream.cuda_stream) for w in ms]
    b = csph.Batch(solvers)
    b.advance(10)
    b.sync()
    before = [b.get_fields(m) for m in range(len(ms))]
    shape = b.autotune(5)
    say(f"batch autotune chose {shape}")
    for m in range(len(ms)):
        for a, r in zip(b.get_fields(m), before[m]):
            assert np.array_equal(a, r)
        assert b.get_sums(m)["step"] == 10
    b.advance(60)
    b.sync()
    for k, (w, s) in enumerate(zip(ms, solvers)):
        rf, rsums = _solo(w, 70, stream.cuda_stream)
        for a, r in zip(b.get_fields(k), rf):
            assert np.array_equal(a, r), k
    with pytest.raises(csph.SwError) as e:
        b.get_sums(len(ms))  # member index out of range: checked in the library
    assert e.value.code == csph.SW_ERR_ARG
    b.close()
    for s in solvers:
        s.close()
