"""Pins of the oracle's forcing terms: rainfall and absorption in the water
source sigma of Eq. 6, Coriolis and wind stress in its force f (the paper
names them as model inputs without formulas; the readings are in the oracle
source).  Each check is a closed form, an exact fixed point or a symmetry."""
import math

import numpy as np

from paper_2103_15196_amd import workloads as W
from tests.helpers import oracle_case

G = 9.81


def _flat(nx=12, ny=10, H=1.0, u=0.0, v=0.0, bc=(1, 1, 1, 1), manning=0.0):
    w = W.dam_break_1d(nx=nx, ny=ny, dx=2.0, h_left=H, h_right=H, x_dam=nx // 2, manning=manning,
                       sediment=False, bc=bc)
    w.qx = np.full((ny, nx), H * u)
    w.qy = np.full((ny, nx), H * v)
    return w


def test_rain_raises_still_water_uniformly(oracle_mod):
    """Flat walled basin, still water: depth grows by r t exactly, nothing
    moves, and the balance reports r t A."""
    O = oracle_mod
    w = _flat(bc=(0, 0, 0, 0))
    r = 2e-4
    p, inp, s = oracle_case(O, w, rain=r)
    V0 = O.volumes(p, inp, s)[0]
    O.run(p, inp, s, 40, dt_fixed=0.05)
    assert np.allclose(s.H, 1.0 + r * s.t, rtol=0, atol=1e-13)
    assert np.abs(s.qx).max() == 0.0 and np.abs(s.qy).max() == 0.0
    A = w.nx * w.ny * w.dx ** 2
    assert abs(s.rain_in - r * s.t * A) <= 1e-12 * r * s.t * A
    assert abs(O.volumes(p, inp, s)[0] - V0 - s.rain_in) <= 1e-12 * V0


def test_absorption_is_the_implicit_decay_and_keeps_velocity(oracle_mod):
    """Uniform flow on a flat bed with open sides and absorption beta:
    H_n = H_0 / (1 + beta dt)^n, the velocity is unchanged, and the absorbed
    volume is what the depth lost; under refinement H tends to H_0 e^(-beta t)."""
    O = oracle_mod
    beta, dt = 0.02, 0.05
    w = _flat(H=1.5, u=0.4, v=-0.1)
    p, inp, s = oracle_case(O, w, beta=beta)
    O.run(p, inp, s, 60, dt_fixed=dt)
    Hn = 1.5 / (1 + beta * dt) ** 60
    assert np.allclose(s.H, Hn, rtol=1e-13, atol=0)
    assert np.allclose(s.qx / s.H, 0.4, rtol=1e-12) and np.allclose(s.qy / s.H, -0.1, rtol=1e-12)
    A = w.nx * w.ny * w.dx ** 2
    assert abs(s.absorbed - (1.5 - Hn) * A) <= 1e-12 * A
    errs = []
    for k in (1, 4):
        p, inp, s = oracle_case(O, w, beta=beta)
        O.run(p, inp, s, 20 * k, dt_fixed=0.1 / k)
        errs.append(abs(s.H[0, 0] - 1.5 * math.exp(-beta * s.t)))
    assert errs[1] < 0.3 * errs[0]


def test_rain_and_absorption_settle_at_r_over_beta(oracle_mod):
    """The fixed point of H = (H + r dt) / (1 + beta dt) is r / beta."""
    O = oracle_mod
    w = _flat(H=0.2, bc=(0, 0, 0, 0))
    r, beta = 3e-4, 0.05
    p, inp, s = oracle_case(O, w, rain=r, beta=beta)
    O.run(p, inp, s, 3000, dt_fixed=0.2)
    assert np.allclose(s.H, r / beta, rtol=1e-9)


def test_coriolis_turns_uniform_flow_in_an_inertial_circle(oracle_mod):
    """Uniform flow, no friction, open sides, Coriolis f: the velocity turns
    to the right at rate f, u = u0 cos(f t), v = -u0 sin(f t) (the midpoint
    predictor-corrector's phase error is O((f dt)^2 f t))."""
    O = oracle_mod
    f, u0 = 1e-2, 0.8
    w = _flat(H=2.0, u=u0)
    p, inp, s = oracle_case(O, w, coriolis=f)
    O.run(p, inp, s, 1, dt_fixed=0.1)
    assert s.qy[0, 0] < 0.0  # f > 0 turns the flow to the right
    O.run(p, inp, s, 999, dt_fixed=0.1)
    u, v = s.qx / s.H, s.qy / s.H
    assert np.allclose(u, u0 * math.cos(f * s.t), atol=1e-6)
    assert np.allclose(v, -u0 * math.sin(f * s.t), atol=1e-6)
    assert np.allclose(s.H, 2.0, rtol=0, atol=1e-12)


def test_wind_accelerates_still_water_at_the_stress_rate(oracle_mod):
    """Flat bed, no friction, open sides: q grows by C_w |W| W per second,
    scaled by min(1, H / h_sed) on a layer thinner than h_sed."""
    O = oracle_mod
    Cw, Wx, Wy = 1.5e-6, 10.0, 5.0
    Ws = Cw * math.hypot(Wx, Wy)
    for H, chi in ((1.0, 1.0), (2.5e-3, 0.25)):
        w = _flat(H=H)
        p, inp, s = oracle_case(O, w, wind_x=Wx, wind_y=Wy, wind_coef=Cw)
        O.run(p, inp, s, 50, dt_fixed=0.1)
        assert np.allclose(s.qx, chi * Ws * Wx * s.t, rtol=1e-11, atol=0)
        assert np.allclose(s.qy, chi * Ws * Wy * s.t, rtol=1e-11, atol=0)


def test_wind_against_manning_friction_reaches_the_steady_speed(oracle_mod):
    """Wind along x on uniform water of depth H with Manning n: the stress
    balances the friction g n^2 u^2 / H^(1/3) at u = sqrt(C_w |W| W H^(1/3) / (g n^2))."""
    O = oracle_mod
    Cw, Wx, n, H = 1e-4, 12.0, 0.1, 1.0
    w = _flat(H=H, manning=n)
    p, inp, s = oracle_case(O, w, wind_x=Wx, wind_coef=Cw)
    O.run(p, inp, s, 2000, dt_fixed=0.15)
    u_ss = math.sqrt(Cw * Wx * Wx * H ** (1.0 / 3.0) / (G * n * n))
    assert np.allclose(s.qx / s.H, u_ss, rtol=1e-6)
    assert np.abs(s.qy).max() == 0.0


def test_coriolis_keeps_the_lake_at_rest_and_mirrors_with_its_sign(oracle_mod):
    """A lake at rest under Coriolis stays exactly at rest; a dam break
    mirrored in x with f -> -f and W_x -> -W_x gives the mirrored answer."""
    O = oracle_mod
    lake = W.lake_at_rest(40, 30, bc=(0, 0, 0, 0))
    p, inp, s = oracle_case(O, lake, coriolis=1e-3)
    z0 = s.H + s.b
    O.run(p, inp, s, 100)
    assert np.abs((s.H + s.b) - z0)[s.H > 0].max() <= 1e-12 and np.abs(s.qx).max() <= 1e-12
    w = W.dam_break_fractal(n=36, ny=20, dx=2.0, seed=9, relief=5.0, depth=4.0)
    kw = dict(coriolis=2e-3, wind_x=8.0, wind_y=3.0, wind_coef=2e-6)
    p, inp, s = oracle_case(O, w, **kw)
    O.run(p, inp, s, 100)
    wm = W.dam_break_fractal(n=36, ny=20, dx=2.0, seed=9, relief=5.0, depth=4.0)
    wm.H, wm.b = wm.H[:, ::-1].copy(), wm.b[:, ::-1].copy()
    km = dict(coriolis=-2e-3, wind_x=-8.0, wind_y=3.0, wind_coef=2e-6)
    pm, im, sm = oracle_case(O, wm, **km)
    O.run(pm, im, sm, 100)
    np.testing.assert_allclose(sm.H[:, ::-1], s.H, atol=1e-11)
    np.testing.assert_allclose(-sm.qx[:, ::-1], s.qx, atol=1e-10)
    np.testing.assert_allclose(sm.qy[:, ::-1], s.qy, atol=1e-10)
