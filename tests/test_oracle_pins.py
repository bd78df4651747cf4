"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each checks a closed form, an
exact solution, an invariant the scheme must keep, or a hand-derived step
(tests/golden/).  Together they are chosen so that a dropped term, a flipped
sign, a wrong neighbour index or an x/y mix-up in any stage fails one of them.
"""
import math

import numpy as np
import pytest

from paper_2103_15196_amd import workloads as W
from tests.helpers import oracle_case, read_golden, ritter, stoker

G = 9.81


# ---------------------------------------------------------------- building blocks

def test_desingularised_velocity(oracle_mod):
    """O1: w(H) = 1/H above eps, continuous at eps, zero at H = 0."""
    O = oracle_mod
    eps = 1e-5
    assert O.w(2.0, eps) == 0.5
    assert O.w(0.0, eps) == 0.0
    below = O.w(eps * (1 - 1e-12), eps)
    assert abs(below - 1.0 / eps) / (1.0 / eps) < 1e-10
    # tends to H * sqrt(2)/eps^2 for H << eps
    assert abs(O.w(1e-9, eps) - 1e-9 * math.sqrt(2) / eps ** 2) < 1e-6 * O.w(1e-9, eps)


def test_minmod(oracle_mod):
    O = oracle_mod
    assert O.minmod(1.0, 2.0) == 1.0
    assert O.minmod(-3.0, -2.0) == -2.0
    assert O.minmod(1.0, -1.0) == 0.0
    assert O.minmod(0.0, 5.0) == 0.0


def test_hll_consistency_and_reflection(oracle_mod):
    """HLL: equal states give the physical flux; supersonic states upwind;
    mirroring the problem mirrors the flux."""
    O = oracle_mod
    H, uL, ut, un = 1.3, 0.7, -0.2, 0.6
    f = O.hll(G, H, uL, ut, un, H, uL, ut, un)
    np.testing.assert_allclose(f, (un * H, un * H * uL, un * H * ut), rtol=1e-14)
    # supersonic to the right: flux is the left physical flux
    f = O.hll(G, 0.01, 5.0, 1.0, 5.0, 0.02, 4.0, 0.0, 4.0)
    np.testing.assert_allclose(f, (5.0 * 0.01, 5.0 * 0.01 * 5.0, 5.0 * 0.01 * 1.0), rtol=1e-14)
    # reflection x -> -x: swap sides, negate normal velocities
    a = (1.1, 0.3, 0.2, 0.4)
    b = (0.6, -0.5, 0.1, -0.3)
    f = O.hll(G, *a, *b)
    g = O.hll(G, b[0], -b[1], b[2], -b[3], a[0], -a[1], a[2], -a[3])
    np.testing.assert_allclose(g, (-f[0], f[1], -f[2]), rtol=1e-13, atol=1e-15)


def test_bedload_shamov_cutoff_and_laws(oracle_mod):
    """Eqs. 3-5: critical speed v_k = C_Sh d50^(1/3) H^(1/6) (0.4455 m/s at
    d50 = 0.5 mm, H = 2 m); no bedload at or below it; above it the Grass law
    A_G |v|^m v, or Eq. 4's coefficient with m = 4."""
    O = oracle_mod
    vk = 5.0 * (5e-4) ** (1 / 3) * 2.0 ** (1 / 6)
    assert abs(vk - 0.4455) < 1e-4
    p = O.Params(nx=1, ny=1, dx=1.0, sed_law=O.SED_GRASS)
    assert O.j0(p, 2.0, 0.99 * vk, 0.0, 0.02, 5e-4) == (0.0, 0.0)
    jx, _ = O.j0(p, 2.0, 1.01 * vk, 0.0, 0.02, 5e-4)
    assert jx == pytest.approx(1e-3 * (1.01 * vk) ** 3)
    jx, jy = O.j0(p, 2.0, 0.6, 0.8, 0.02, 5e-4)          # |v| = 1
    assert jx == pytest.approx(1e-3 * 0.6) and jy == pytest.approx(1e-3 * 0.8)
    assert O.j0(p, 0.005, 3.0, 0.0, 0.02, 5e-4) == (0.0, 0.0)   # below h_sed
    p4 = O.Params(nx=1, ny=1, dx=1.0, sed_law=O.SED_EQ4)
    A = 0.05 * 0.02 ** 3 / (1.65 * math.sqrt(G * 2.0) * 5e-4)
    jx, jy = O.j0(p4, 2.0, 1.0, 0.0, 0.02, 5e-4)
    assert jx == pytest.approx(A * 1.0) and jy == 0.0
    jx, _ = O.j0(p4, 2.0, 2.0, 0.0, 0.02, 5e-4)
    assert jx == pytest.approx(A * 2.0 ** 5)            # |v|^4 v


def test_first_time_step_of_dam_break(oracle_mod):
    """Eq. 7 on the 256 x 64 dam break at rest: vp = 0 and D = 0 are infinite
    terms, vs = sqrt(2 g), so dt_0 = 0.3 dx / sqrt(2 g) = 0.067729 s."""
    O = oracle_mod
    p, inp, s = oracle_case(O, W.dam_break_1d())
    c = O.cfl(p, inp, s)
    assert c["vp"] == 0.0 and c["D"] == 0.0 and c["binding"] == 1
    assert abs(c["dt"] - 0.3 / math.sqrt(2 * G)) < 1e-15
    assert abs(c["dt"] - 0.067729) < 1e-6


def test_all_dry_step_is_dt_max(oracle_mod):
    O = oracle_mod
    z = np.zeros((4, 5))
    p = O.Params(nx=5, ny=4, dx=1.0)
    c = O.cfl(p, O.Inputs(nM=0.02), O.State(z, z, z, z))
    assert c["dt"] == p.dt_max and c["binding"] == 3


def test_eq7_each_term_binds(oracle_mod):
    """Eq. 7 on prescribed fields: a thin fast sheet makes h/(2 vp) bind, deep
    still water makes h/vs bind, strong bedload makes h^2/(2D) bind."""
    O = oracle_mod
    one = np.ones((2, 3))
    p = O.Params(nx=3, ny=2, dx=2.0, sed_law=O.SED_NONE)
    c = O.cfl(p, O.Inputs(nM=0.0), O.State(1e-4 * one, 3e-4 * one, 0 * one, 0 * one))
    assert c["binding"] == 0 and c["vp"] == pytest.approx(3.0)
    assert c["dt"] == pytest.approx(0.3 * 2.0 / (2 * 3.0), rel=1e-12)
    c = O.cfl(p, O.Inputs(nM=0.0), O.State(4.0 * one, 0 * one, 0 * one, 0 * one))
    assert c["binding"] == 1 and c["dt"] == pytest.approx(0.3 * 2.0 / math.sqrt(4 * G), rel=1e-12)
    pg = O.Params(nx=3, ny=2, dx=2.0, sed_law=O.SED_GRASS, A_G=10.0, m_exp=2.0)
    c = O.cfl(pg, O.Inputs(nM=0.0, d50=5e-4, psi=0.4), O.State(one, one, 0 * one, 0 * one))
    D = 10.0 / 0.6
    assert c["binding"] == 2 and c["D"] == pytest.approx(D, rel=1e-12)
    assert c["dt"] == pytest.approx(0.3 * 4.0 / (2 * D), rel=1e-12)


def test_manning_normal_flow_is_steady(oracle_mod):
    """Uniform flow down a plane of slope S0: the hydrostatic-face force on a
    linear bed is g H S0 (1 - S0 dx / (2 H)) and balances Manning friction
    g n^2 u^2 / H^(1/3) at u^2 = H^(4/3) S0 (1 - S0 dx/(2H)) / n^2, within
    0.3% of Manning's formula u = H^(2/3) S0^(1/2) / n.  Started there, the
    interior stays steady (predictor and corrector are both at equilibrium)."""
    O = oracle_mod
    nx, ny, dx, S0, n, H0 = 64, 3, 10.0, 1e-3, 0.03, 1.0
    u = math.sqrt(H0 ** (4 / 3) * S0 * (1 - S0 * dx / (2 * H0))) / n
    assert abs(u - H0 ** (2 / 3) * math.sqrt(S0) / n) / u < 3e-3
    x = (np.arange(nx) + 0.5) * dx
    b = np.broadcast_to(-S0 * x, (ny, nx)).copy()
    H = np.full((ny, nx), H0)
    p = O.Params(nx=nx, ny=ny, dx=dx, bc=(1, 1, 0, 0), sed_law=O.SED_NONE)
    s = O.State(H, H * u, np.zeros_like(H), b)
    O.run(p, O.Inputs(nM=n), s, 15)
    mid = slice(24, 40)
    assert np.abs(s.H[:, mid] - H0).max() < 1e-12
    assert np.abs(s.qx[:, mid] - H0 * u).max() < 1e-12
    assert np.abs(s.qx[:, :2] - H0 * u).max() > 1e-6   # the ends do feel the boundary


# ---------------------------------------------------------------- hand-stepped grids

def test_hand_step_3x1_wall(oracle_mod):
    O = oracle_mod
    exp = read_golden("hand_step_3x1_wall.txt")
    p = O.Params(nx=3, ny=1, dx=1.0, cfl=0.9, sed_law=O.SED_NONE)
    H = np.array([[1.0, 0.0, 0.0]])
    z = np.zeros_like(H)
    s = O.State(H, z, z, z)
    O.step(p, O.Inputs(nM=0.0), s, dt_fixed=0.1)
    for i in range(3):
        assert s.H[0, i] == pytest.approx(exp[f"H{i}"], abs=1e-14)
        assert s.qx[0, i] == pytest.approx(exp[f"qx{i}"], abs=1e-14)
    assert np.all(s.qy == 0.0) and np.all(s.b == 0.0)


def test_hand_step_3x3_column(oracle_mod):
    O = oracle_mod
    exp = read_golden("hand_step_3x3_column.txt")
    p = O.Params(nx=3, ny=3, dx=1.0, cfl=0.9, sed_law=O.SED_NONE)
    H = np.zeros((3, 3))
    H[1, 1] = 1.0
    z = np.zeros_like(H)
    s = O.State(H, z, z, z)
    O.step(p, O.Inputs(nM=0.0), s, dt_fixed=0.1)
    assert s.H[1, 1] == pytest.approx(exp["H_centre"], abs=1e-14)
    for (j, i) in ((0, 1), (2, 1), (1, 0), (1, 2)):
        assert s.H[j, i] == pytest.approx(exp["H_edge"], abs=1e-14)
    for (j, i) in ((0, 0), (0, 2), (2, 0), (2, 2)):
        assert s.H[j, i] == exp["H_corner"]
    assert np.all(s.qx == 0.0) and np.all(s.qy == 0.0)


def test_hand_step_exner_3x1(oracle_mod):
    O = oracle_mod
    exp = read_golden("hand_step_exner_3x1.txt")
    p = O.Params(nx=3, ny=1, dx=1.0, bc=(1, 1, 0, 0), sed_law=O.SED_GRASS, A_G=1e-3,
                 m_exp=2.0)
    H = np.ones((1, 3))
    b = np.array([[0.0, 0.1, 0.0]])
    s = O.State(H, np.array([[1.0, 1.5, 1.0]]), np.zeros_like(H), b)
    O.step(p, O.Inputs(nM=0.0, d50=5e-4, psi=0.4), s, dt_fixed=0.05)
    for i in range(3):
        assert s.b[0, i] == pytest.approx(exp[f"b{i}"], abs=1e-15)


def test_hand_step_2x1_momentum_budget(oracle_mod):
    O = oracle_mod
    exp = read_golden("hand_step_2x1_momentum.txt")
    p = O.Params(nx=2, ny=1, dx=1.0, cfl=0.9, sed_law=O.SED_NONE)
    H = np.ones((1, 2))
    s = O.State(H, np.array([[1.0, 0.0]]), np.zeros_like(H), np.zeros_like(H))
    O.step(p, O.Inputs(nM=0.0), s, dt_fixed=0.1)
    assert s.qx.sum() == pytest.approx(exp["sum_q"], abs=1e-14)
    assert s.H.sum() == pytest.approx(exp["sum_H"], abs=1e-14)


def test_hand_step_3x3_drained_column(oracle_mod):
    O = oracle_mod
    exp = read_golden("hand_step_3x3_drained.txt")
    p = O.Params(nx=3, ny=3, dx=1.0, cfl=0.9, sed_law=O.SED_NONE)
    H = np.zeros((3, 3))
    H[1, 1] = 1.0
    z = np.zeros_like(H)
    s = O.State(H, z, z, z)
    O.step(p, O.Inputs(nM=0.0), s, dt_fixed=0.25)
    assert s.H[1, 1] == pytest.approx(exp["H_centre"], abs=1e-14)
    for (j, i) in ((0, 1), (2, 1), (1, 0), (1, 2)):
        assert s.H[j, i] == pytest.approx(exp["H_edge"], abs=1e-14)
    for (j, i) in ((0, 0), (0, 2), (2, 0), (2, 2)):
        assert s.H[j, i] == exp["H_corner"]


# ---------------------------------------------------------------- invariants

@pytest.mark.parametrize("bc", [(0, 0, 0, 0), (1, 1, 1, 1), (0, 1, 1, 0)])
def test_lake_at_rest_with_islands(oracle_mod, bc):
    """Still water over a fractal bed with emerged dry islands stays still:
    forces and fluxes vanish exactly at rest (hydrostatic faces)."""
    O = oracle_mod
    w = W.lake_at_rest(48, 40, dx=1.0, relief=3.0, level=2.0, bc=bc)
    p, inp, s = oracle_case(O, w)
    assert (w.H == 0).mean() > 0.05 and (w.H > 0).mean() > 0.5   # islands and water
    zeta0 = w.H + w.b
    O.run(p, inp, s, 300)
    wet = w.H > 0
    assert np.abs((s.H + s.b) - zeta0)[wet].max() <= 1e-12
    assert np.all(s.H[~wet] == 0.0)
    assert np.abs(s.qx).max() <= 1e-12 and np.abs(s.qy).max() <= 1e-12
    assert np.array_equal(s.b, w.b)


def test_water_and_sediment_conservation_with_walls(oracle_mod):
    """Walls, no sources: sum H dx^2 and sum (1-psi) b dx^2 are constant
    (per-cell porosity exercises Eq. 1's (1-psi) outside the divergence)."""
    O = oracle_mod
    w = W.dam_break_1d(nx=96, ny=24, x_dam=48, h_left=2.0, h_right=0.0)
    rng = np.random.default_rng(5)
    w.psi = rng.uniform(0.3, 0.45, size=(w.ny, w.nx))
    w.b = 0.05 * rng.standard_normal((w.ny, w.nx))
    w.H = np.maximum(0.0, np.where(np.arange(w.nx)[None, :] < 48, 2.0, 0.0) - w.b)
    p, inp, s = oracle_case(O, w)
    V0 = O.volumes(p, inp, s)
    O.run(p, inp, s, 200)
    V1 = O.volumes(p, inp, s)
    assert abs(V1[0] - V0[0]) / V0[0] <= 1e-13
    assert abs(V1[1] - V0[1]) <= 1e-13 * np.abs((1 - w.psi) * w.b).sum()
    assert np.abs(s.b - w.b).max() > 1e-4      # the bed did move


def test_balance_with_open_boundaries_and_inflow(oracle_mod):
    """Open outflow boundary + hydrograph inflow + bed sources: the volume
    change equals inflow minus boundary outflow."""
    O = oracle_mod
    w = W.river_valley(n=128, ny=96, dx=5.0, amplitude=60.0, wavelength=400.0, width=40.0,
                       Q_base=20.0, Q_peak=200.0, t_peak=30.0, t_sigma=10.0)
    w.qb = np.zeros((w.ny, w.nx))
    w.qb[40:50, 60:70] = 1e-5
    w.qb[10:12, 10:12] = -2e-6
    w.H = np.where(w.b < np.percentile(w.b, 40), 1.0, 0.0)   # ponds, some at the outlet
    p, inp, s = oracle_case(O, w)
    V0 = O.volumes(p, inp, s)
    O.run(p, inp, s, 400)
    V1 = O.volumes(p, inp, s)
    assert s.in_w > 0 and abs(s.out_w) > 1.0    # zero-gradient boundary: flow both ways
    rw = V1[0] - V0[0] + s.out_w - s.in_w
    assert abs(rw) / V1[0] <= 1e-12
    rs = V1[1] - V0[1] + s.out_s - s.in_s
    assert abs(rs) <= 1e-12 * np.abs((1 - w.psi) * w.b).sum()


def test_y_uniform_problem_stays_uniform_bitwise(oracle_mod):
    O = oracle_mod
    w = W.dam_break_1d()
    p, inp, s = oracle_case(O, w)
    O.run(p, inp, s, 200)
    assert np.all(s.qy == 0.0)
    for f in (s.H, s.qx, s.b):
        assert np.array_equal(f, np.broadcast_to(f[:1], f.shape))


def _fractal_dam(n0=40, n1=28, bc=(0, 1, 0, 1)):
    w = W.dam_break_fractal(n=n0, ny=n1, dx=2.0, seed=21, relief=4.0, depth=3.0, steps=60)
    w.bc = bc
    rng = np.random.default_rng(4)
    w.psi = rng.uniform(0.3, 0.45, size=(w.ny, w.nx))
    w.d50 = rng.uniform(2e-4, 2e-3, size=(w.ny, w.nx))
    return w


def test_transpose_symmetry_bitwise(oracle_mod):
    """Swapping x and y (fields transposed, qx <-> qy, W/E <-> S/N) gives the
    transposed result bit for bit."""
    O = oracle_mod
    w = _fractal_dam()
    p, inp, s = oracle_case(O, w)
    O.run(p, inp, s, 60)
    t = W.Workload(**{k: getattr(w, k) for k in w.__dataclass_fields__})
    t.nx, t.ny = w.ny, w.nx
    t.H, t.b = w.H.T.copy(), w.b.T.copy()
    t.qx, t.qy = w.qy.T.copy(), w.qx.T.copy()
    t.psi, t.d50 = w.psi.T.copy(), w.d50.T.copy()
    t.bc = (w.bc[2], w.bc[3], w.bc[0], w.bc[1])
    pt, it, st = oracle_case(O, t)
    O.run(pt, it, st, 60)
    assert np.array_equal(st.H, s.H.T)
    assert np.array_equal(st.b, s.b.T)
    assert np.array_equal(st.qx, s.qy.T)
    assert np.array_equal(st.qy, s.qx.T)
    assert abs(st.t - s.t) == 0.0


def test_mirror_symmetry(oracle_mod):
    """Reflecting x (fields flipped, qx negated, W <-> E) reflects the result."""
    O = oracle_mod
    w = _fractal_dam(bc=(0, 1, 1, 0))
    p, inp, s = oracle_case(O, w)
    O.run(p, inp, s, 60)
    m = W.Workload(**{k: getattr(w, k) for k in w.__dataclass_fields__})
    m.H, m.b = w.H[:, ::-1].copy(), w.b[:, ::-1].copy()
    m.qx, m.qy = -w.qx[:, ::-1].copy(), w.qy[:, ::-1].copy()
    m.psi, m.d50 = w.psi[:, ::-1].copy(), w.d50[:, ::-1].copy()
    m.bc = (w.bc[1], w.bc[0], w.bc[2], w.bc[3])
    pm, im, sm = oracle_case(O, m)
    O.run(pm, im, sm, 60)
    np.testing.assert_allclose(sm.H, s.H[:, ::-1], rtol=0, atol=1e-12)
    np.testing.assert_allclose(sm.b, s.b[:, ::-1], rtol=0, atol=1e-12)
    np.testing.assert_allclose(sm.qx, -s.qx[:, ::-1], rtol=0, atol=1e-12)
    np.testing.assert_allclose(sm.qy, s.qy[:, ::-1], rtol=0, atol=1e-12)
    assert np.abs(s.qx).max() > 0.1


# ---------------------------------------------------------------- exact solutions

def _run_to(O, p, inp, s, T):
    binds = set()
    while s.t < T - 1e-12:
        c = O.cfl(p, inp, s)
        binds.add(c["binding"])
        O.step(p, inp, s, dt_fixed=min(c["dt"], T - s.t))
    return binds


def test_stoker_dam_break(oracle_mod):
    """Wet-bed dam break (2 m | 0.5 m, no friction, no sediment) against the exact
    Riemann solution: plateau depth and speed within 1%, shock within 2 cells,
    L1 error falling under refinement."""
    O = oracle_mod
    errs = []
    for nx, dx in ((256, 1.0), (512, 0.5)):
        w = W.dam_break_1d(nx=nx, ny=2, dx=dx, x_dam=nx // 2, manning=0.0, sediment=False)
        p, inp, s = oracle_case(O, w)
        _run_to(O, p, inp, s, 10.0)
        x = (np.arange(nx) + 0.5) * dx
        h, u, hm, um, sp = stoker(2.0, 0.5, x, s.t, 128.0)
        H = s.H[0]
        U = s.qx[0] / H
        errs.append(np.abs(H - h).sum() * dx)
        band = (x > 128 + 0.3 * um * 10) & (x < 128 + 0.8 * sp * 10)
        assert abs(H[band].mean() - hm) / hm < 0.01
        assert abs(U[band].mean() - um) / um < 0.01
        xs = x[np.argmax(H < 0.5 * (hm + 0.5))]
        assert abs(xs - (128 + sp * s.t)) <= 2 * dx
    assert abs(hm - 1.1035) < 1e-4 and abs(um - 2.2785) < 1e-4 and abs(sp - 4.1663) < 1e-4
    assert errs[1] < 0.6 * errs[0]


def test_ritter_dam_break(oracle_mod):
    """Dry-bed dam break (2 m | dry): L1 error against Ritter's solution falls
    under refinement; nothing is wet beyond the exact front; Eq. 7's h/(2 vp)
    term binds at some step."""
    O = oracle_mod
    errs = []
    for nx, dx in ((256, 1.0), (512, 0.5)):
        w = W.dam_break_1d(nx=nx, ny=2, dx=dx, x_dam=nx // 2, h_right=0.0, manning=0.0,
                           sediment=False)
        p, inp, s = oracle_case(O, w)
        binds = _run_to(O, p, inp, s, 8.0)
        x = (np.arange(nx) + 0.5) * dx
        h = ritter(2.0, x, s.t, 128.0)
        errs.append(np.abs(s.H[0] - h).sum() * dx)
        assert 0 in binds
        front = 128.0 + 2 * math.sqrt(2 * G) * s.t
        assert np.all(s.H[0][x > front + 2 * dx] == 0.0)
    assert errs[1] < 0.6 * errs[0]


def test_friction_decay_matches_ode(oracle_mod):
    """Uniform flow on a flat bed with open ends and Manning friction only: the
    Euler stage is inert, the velocity follows the semi-implicit
    predictor-corrector u_{n+1} = u_n / (1 + dt c u_p), u_p = u_n / (1 + dt c u_n / 2)
    with c = g n^2 / H^(4/3), and converges (first order in dt) to the ODE
    solution u(t) = u0 / (1 + c u0 t)."""
    O = oracle_mod
    H0, u0, n, T = 1.5, 2.0, 0.05, 4.0
    cf = G * n * n / H0 ** (4 / 3)
    ref = u0 / (1.0 + cf * u0 * T)
    errs = []
    for dt in (0.02, 0.01, 0.005):
        p = O.Params(nx=6, ny=3, dx=10.0, bc=(1, 1, 1, 1), sed_law=O.SED_NONE)
        H = np.full((3, 6), H0)
        s = O.State(H, H * u0, np.zeros_like(H), np.zeros_like(H))
        N = int(round(T / dt))
        O.run(p, O.Inputs(nM=n), s, N, dt_fixed=dt)
        assert np.all(s.H == H0)
        u = s.qx / s.H
        assert np.ptp(u) == 0.0
        un = u0
        for _ in range(N):
            up = un / (1.0 + 0.5 * dt * cf * un)
            un = un / (1.0 + dt * cf * up)
        assert abs(u[0, 0] - un) < 1e-13
        errs.append(abs(u[0, 0] - ref))
    assert errs[2] < 2e-4 * ref
    assert 0.4 < errs[1] / errs[0] < 0.6 and 0.4 < errs[2] / errs[1] < 0.6


def test_bed_slope_diffusion_decays_mode(oracle_mod):
    """Eq. 2's slope term makes Exner a diffusion of b with coefficient
    C_J |J0| / (1 - psi).  Under deep uniform flow (bedload uniform to
    1e-5) a cosine bed mode decays at the discrete rate
    (1 - D dt k2)^N, k2 = (2/dx^2)(1 - cos(k dx))."""
    O = oracle_mod
    nx, dx, Hd, u, lam, amp = 192, 1.0, 100.0, 5.0, 8.0, 1e-3
    x = (np.arange(nx) + 0.5) * dx
    k = 2 * math.pi / lam
    b = amp * np.cos(k * x)[None, :] * np.ones((2, 1))
    H = Hd - b
    p = O.Params(nx=nx, ny=2, dx=dx, bc=(1, 1, 0, 0), sed_law=O.SED_GRASS, A_G=1e-3,
                 m_exp=2.0, C_J=2.0, cfl=0.5)
    s = O.State(H, H * u, np.zeros_like(H), b)
    inp = O.Inputs(nM=0.0, d50=5e-4, psi=0.4)
    dt, N = 0.008, 600
    O.run(p, inp, s, N, dt_fixed=dt)
    D = 2.0 * 1e-3 * u ** 3 / 0.6
    k2 = (2.0 / dx ** 2) * (1.0 - math.cos(k * dx))
    expect = (1.0 - D * dt * k2) ** N
    sel = (x > 48) & (x < 144)
    bb = s.b[0, sel]
    xs = x[sel]
    c = 2 * np.mean(bb * np.cos(k * xs))
    sn = 2 * np.mean(bb * np.sin(k * xs))
    got = math.hypot(c, sn) / amp
    assert expect < 0.5                      # the mode really decays
    assert abs(got - expect) / expect < 0.03


# ---------------------------------------------------------------- error paths

def test_fixed_step_above_eq7_is_rejected(oracle_mod):
    O = oracle_mod
    p, inp, s = oracle_case(O, W.dam_break_1d(nx=16, ny=4, x_dam=8))
    with pytest.raises(O.OracleError) as e:
        O.step(p, inp, s, dt_fixed=1.0)
    assert e.value.code == -6


def test_nonfinite_state_is_rejected(oracle_mod):
    O = oracle_mod
    p, inp, s = oracle_case(O, W.dam_break_1d(nx=16, ny=4, x_dam=8))
    s.qx[2, 3] = np.nan
    with pytest.raises(O.OracleError) as e:
        O.step(p, inp, s)
    assert e.value.code == -3


def test_eq4_fractal_dam_break_is_ill_conditioned(oracle_mod):
    """Why the 2-D fractal dam breaks use the Grass law: with Eq. 4's
    coefficient (proportional to 1/sqrt(g h)) the bedload jumps from 0 to
    O(10) m^2/s where a fast thin front crosses h_sed, and a 1e-7 relative
    change of the initial depth (float32 rounding) moves the FP64 solution by
    more than the parity tolerance within 100 steps; with the Grass law the same change stays
    near rounding level (the parity tolerance on depth is 1e-4 m)."""
    O = oracle_mod
    base = W.dam_break_fractal(n=120, ny=96, dx=2.0, seed=7, relief=10.0, depth=8.0).as_float32()
    rng = np.random.default_rng(0)
    pert = base.H * (1 + 1e-7 * rng.standard_normal(base.H.shape))
    out = {}
    for law in (O.SED_EQ4, O.SED_GRASS):
        res = []
        for H in (base.H, pert):
            w = W.Workload(**{k: getattr(base, k) for k in base.__dataclass_fields__})
            w.H = H
            p, inp, s = oracle_case(O, w, sed_law=law)
            O.run(p, inp, s, 100)
            res.append(s.H)
        out[law] = float(np.abs(res[0] - res[1]).max())
    assert out[O.SED_EQ4] > 1e-4
    assert out[O.SED_GRASS] < 1e-5
    assert out[O.SED_EQ4] > 30 * out[O.SED_GRASS]


# ---------------------------------------------------------------- inflow hydrograph

def test_hydrograph_gaussian_pulse_values(oracle_mod):
    """O0: Q(t) = Q_base + Q_peak exp(-(t - t_p)^2 / (2 s^2)) through properties
    of the Gaussian pulse: Q_base + Q_peak at the peak, symmetric about it,
    Q_base + Q_peak / sqrt(e) one standard deviation away, Q_base + Q_peak / 2
    at the half-maximum points t_p +- s sqrt(2 ln 2), Q_base far away."""
    O = oracle_mod
    inp = O.Inputs(Q_base=100.0, Q_peak=2000.0, t_peak=120.0, t_sigma=40.0)
    assert O.hydrograph(inp, 120.0) == 2100.0
    for d in (3.0, 17.5, 40.0, 95.0):
        assert O.hydrograph(inp, 120.0 + d) == pytest.approx(O.hydrograph(inp, 120.0 - d),
                                                             rel=1e-15)
    assert O.hydrograph(inp, 160.0) == pytest.approx(100.0 + 2000.0 / math.sqrt(math.e), rel=1e-14)
    half = 40.0 * math.sqrt(2.0 * math.log(2.0))
    assert O.hydrograph(inp, 120.0 + half) == pytest.approx(1100.0, rel=1e-14)
    assert O.hydrograph(inp, 120.0 - half) == pytest.approx(1100.0, rel=1e-14)
    assert O.hydrograph(inp, 120.0 + 40.0 * 40.0) == 100.0


def test_inflow_volume_is_the_midpoint_rule_of_the_hydrograph(oracle_mod):
    """O8 / R26: the source of a step is Q(t_n + dt/2) dt.  Over the rising half
    of the pulse (t = 0 .. t_p in fixed steps) the accumulated inflow must
    match the closed-form integral Q_base t_p + Q_peak s sqrt(pi/2)
    erf(t_p / (s sqrt 2)) within the midpoint rule's error bound
    t_p dt^2 max|Q''| / 24 (max|Q''| = Q_peak / s^2); evaluating Q at t_n or
    t_n + dt would be off by about dt (Q(t_p) - Q(0)) / 2, 300 times that
    bound.  The closed basin then holds exactly that volume."""
    O = oracle_mod
    n, dx = 16, 50.0
    z = np.zeros((n, n))
    w = W.Workload(name="pulse", nx=n, ny=n, dx=dx, bc=(0, 0, 0, 0), H=z, qx=z, qy=z, b=z,
                   nM=0.0, d50=5e-4, psi=0.4, steps=240, cfl=0.3, sed_law=0,
                   inflow_idx=np.array([5 * n + 5, 5 * n + 6, 9 * n + 2], dtype=np.int32),
                   inflow_w=np.array([0.5, 0.3, 0.2]), Q_base=100.0, Q_peak=2000.0,
                   t_peak=120.0, t_sigma=40.0)
    p, inp, s = oracle_case(O, w)
    dt, tp, sg = 0.5, 120.0, 40.0
    O.run(p, inp, s, int(tp / dt), dt_fixed=dt)
    assert s.t == pytest.approx(tp, rel=1e-15)
    exact = 100.0 * tp + 2000.0 * sg * math.sqrt(math.pi / 2.0) * math.erf(tp / (sg * math.sqrt(2.0)))
    bound = tp * dt * dt * (2000.0 / sg ** 2) / 24.0
    assert abs(s.in_w - exact) <= bound
    assert 0.5 * dt * (2100.0 - O.hydrograph(inp, 0.0)) > 300 * bound
    V = O.volumes(p, inp, s)[0]
    assert V == pytest.approx(s.in_w, rel=1e-13)
