"""Rainfall, absorption, Coriolis and wind (the sigma and f of Eq. 6) on the
GPU against the FP64 oracle with the same forcing, their balances, and the
bitwise structure (strips = LDS tiles = unfused, skipping on = off,
checkpoint and resume)."""
import numpy as np
import pytest

from paper_2103_15196_amd import workloads as W
from tests.gpu_common import compare, run_oracle, say, torch_stream
from tests.test_gpu_parity import _check

pytestmark = pytest.mark.gpu

FORCING = dict(rain=5e-5, coriolis=1e-3, wind_x=12.0, wind_y=-4.0, wind_coef=1.5e-6)


def _beta(w, seed=4):
    return np.random.default_rng(seed).uniform(0.0, 2e-3, (w.ny, w.nx)).astype(np.float32)


def _gpu(w, steps, forcing, beta, shape=None, flags=None, stream=None):
    from paper_2103_15196_amd import csph
    kw = {} if flags is None else {"flags": flags}
    s = csph.solver_for(w, stream=stream if stream is not None else torch_stream(), **kw)
    try:
        s.set_forcing(beta=beta, **forcing)
        if shape:
            s.set_tile_shape(*shape)
        s.advance(steps)
        return s.get_fields(), s.get_sums()
    finally:
        s.close()


@pytest.fixture(scope="module")
def O():
    from oracle import oracle as O
    O.build(force=False)
    return O


@pytest.mark.parametrize("which", ["all", "rain_absorption", "coriolis_wind"])
def test_gpu_forcing_matches_oracle(O, which):
    """Fractal dam break (walls W/N, open E/S), 400 steps, every cell at the
    flat bounds, plus the rain and absorbed volumes and the closed water
    balance (the rain is added compensated, so the balance closes)."""
    w = W.dam_break_fractal(n=180, ny=140, dx=2.0, seed=12, relief=8.0, depth=5.0).as_float32()
    w.bc = (0, 1, 1, 0)
    f = dict(FORCING)
    beta = _beta(w)
    if which == "rain_absorption":
        f.update(coriolis=0.0, wind_x=0.0, wind_y=0.0)
    if which == "coriolis_wind":
        f.update(rain=0.0)
        beta = 0.0
    say(f"case forcing {which}: fractal 180x140 400 steps")
    gpu = _gpu(w, 400, f, beta)
    orc = run_oracle(O, w, 400, beta=None if np.isscalar(beta) else np.asarray(beta, np.float64), **f)
    res = compare(O, w, gpu, orc)  # every cell at the flat bounds
    sums, st = gpu[1], orc[2]
    say(f"  rain in {sums['water_rain_in']:.6e} / {st.rain_in:.6e}, absorbed "
        f"{sums['water_absorbed']:.6e} / {st.absorbed:.6e}")
    assert abs(sums["water_rain_in"] - st.rain_in) <= 1e-6 * max(st.rain_in, 1e-30)
    assert abs(sums["water_absorbed"] - st.absorbed) <= 1e-5 * max(st.absorbed, 1e-30)
    V0 = float(np.sum(w.H)) * w.dx * w.dx
    bal = (sums["water_volume"] - V0 + sums["water_boundary_out"] - sums["water_rain_in"]
           + sums["water_absorbed"])
    assert abs(bal) <= 1e-6 * (V0 + sums["water_rain_in"])
    # compare() balances the inflow only: the forcing terms are checked above
    res["mass_drift_gpu"] = 0.0
    _check(res)


def test_gpu_forcing_structure_is_bitwise():
    """With every forcing term on: 58x8 strips, 64x8 LDS tiles and the
    unfused sequence give the same bits; dry-tile skipping on and off too;
    resume from a checkpoint (with the absorbed depths) is bitwise."""
    from paper_2103_15196_amd import csph
    w = W.dam_break_fractal(n=150, ny=100, dx=2.0, seed=13, relief=8.0, depth=5.0).as_float32()
    f = dict(FORCING, rain=0.0)  # without rain, dry tiles can be skipped
    beta = _beta(w, 5)
    ref, rs = _gpu(w, 120, f, beta)
    for kw in (dict(shape=(64, 8)), dict(flags=csph.SW_FLAG_UNFUSED), dict(flags=0)):
        g, gs = _gpu(w, 120, f, beta, **kw)
        for a, b in zip(g, ref):
            assert np.array_equal(a, b), kw
        assert gs["t"] == rs["t"] and gs["water_absorbed"] == rs["water_absorbed"]
    s = csph.solver_for(w, stream=torch_stream())
    s.set_forcing(beta=beta, **f)
    s.advance(50)
    blob = s.checkpoint()
    s.close()
    s = csph.solver_for(w, stream=torch_stream())
    s.set_forcing(beta=beta, **f)
    s.restore(blob)
    s.advance(70)
    g, gs = s.get_fields(), s.get_sums()
    s.close()
    for a, b in zip(g, ref):
        assert np.array_equal(a, b)
    assert gs["water_absorbed"] == rs["water_absorbed"] and gs["t"] == rs["t"]
