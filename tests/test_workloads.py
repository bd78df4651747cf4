"""Host-side checks of the seeded workload generators (no GPU): the shapes,
value ranges and structure that the benchmark and the parity tests rely on."""
import numpy as np

from paper_2103_15196_amd import workloads as W


def test_generators_are_deterministic_in_their_seed():
    a = W.river_valley(n=128, seed=4)
    b = W.river_valley(n=128, seed=4)
    c = W.river_valley(n=128, seed=5)
    assert np.array_equal(a.b, b.b) and np.array_equal(a.d50, b.d50)
    assert not np.array_equal(a.b, c.b)


def test_fractal_surface_has_the_requested_relief():
    s = W.fractal_surface(96, 64, 3, 10.0)
    assert s.shape == (64, 96)
    assert s.min() == 0.0 and abs(s.max() - 10.0) < 1e-12


def test_river_valley_soil_and_inflow():
    w = W.river_valley(n=256, seed=3)
    assert 0.2e-3 <= w.d50.min() and w.d50.max() <= 2e-3
    assert 0.30 <= w.psi.min() and w.psi.max() <= 0.45
    assert w.bc == (W.WALL, W.OPEN, W.WALL, W.WALL)
    assert np.all(w.inflow_idx % w.nx == 0)            # on the x = 0 column
    assert abs(w.inflow_w.sum() - 1.0) < 1e-12 and np.all(w.inflow_w > 0)
    assert np.all(w.H == 0.0)                           # initially dry


def test_valley_basin_is_closed_with_an_upstream_reservoir():
    from paper_2103_15196_amd import surrogate as SG
    w = SG.valley_basin(256, 5000, 2.0)
    assert w.bc == (W.WALL, W.WALL, W.WALL, W.WALL) and w.inflow_idx is None
    q = w.nx // 4
    assert np.all(w.H[:, q:] == 0.0) and (w.H[:, :q] > 0).any()
    zeta = (w.H + w.b)[w.H > 0]
    assert np.ptp(zeta) < 1e-5 * max(1.0, abs(zeta).max())   # one flat surface
    assert w.H.dtype == np.float64 and np.array_equal(w.H, w.H.astype(np.float32))


def test_ensemble_sizes_depths_and_manning_are_in_range():
    ms = W.ensemble(count=6, seed0=10, n_min=64, n_max=96)
    for m in ms:
        assert 64 <= m.nx <= 96 and m.nx == m.ny
        assert 1.0 <= m.extra["depth"] <= 10.0
        assert 0.015 <= m.nM <= 0.05
