"""Pins of the oracle's limiter and wave-speed variants of the Euler stage
(Section 3 names TVD limiters and HLL without fixing either): MC and superbee
slopes, the two-rarefaction (Toro) HLL speeds; and of the second-order form of
the Lagrangian force (hydrostatic faces on reconstructed states).

As in test_oracle_pins.py, each check is against a hand-worked value, an exact
solution or an invariant, never the oracle against itself."""
import math
import os

import numpy as np
import pytest

from paper_2103_15196_amd import workloads as W
from tests.helpers import exact_riemann_star, oracle_case, ritter, stoker

G = 9.81
LIMITERS = {"minmod": 0, "mc": 1, "superbee": 2}
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "limiters.txt")


def test_limiters_match_hand_worked_values(oracle_mod):
    O = oracle_mod
    rows = [list(map(float, l.split())) for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) >= 8
    for a, b, *want in rows:
        for kind, w in zip((0, 1, 2), want):
            assert O.limiter(kind, a, b) == w, (kind, a, b)


def test_limiters_lie_in_the_tvd_region(oracle_mod):
    """Sweby's second-order TVD region: with r = b/a > 0 and phi = sigma/a,
    0 <= phi <= min(2r, 2), phi(1) = 1, phi symmetric (sigma(a,b) = sigma(b,a));
    minmod <= MC <= superbee."""
    O = oracle_mod
    for r in np.geomspace(1e-3, 1e3, 61):
        for a in (0.7, -1.3):
            b = a * r
            phis = [O.limiter(k, a, b) / a for k in (0, 1, 2)]
            for k, phi in enumerate(phis):
                assert -1e-15 <= phi <= min(2 * r, 2.0) + 1e-12, (k, r, phi)
                assert O.limiter(k, a, b) == O.limiter(k, b, a)
            assert phis[0] <= phis[1] + 1e-15 and phis[1] <= phis[2] + 1e-15
    for k in (0, 1, 2):
        assert O.limiter(k, 1.7, 1.7) == 1.7


def test_two_rarefaction_star_state_is_exact_for_two_rarefactions(oracle_mod):
    """When both waves are rarefactions the two-rarefaction star state is the
    exact one (exact Riemann solver of tests/helpers.py)."""
    O = oracle_mod
    for hl, ul, hr, ur in ((1.0, -0.5, 1.0, 0.5), (2.0, -1.0, 0.5, 4.0), (1.2, -0.4, 0.9, 1.5)):
        hs, us = exact_riemann_star(hl, ul, hr, ur)
        assert hs < min(hl, hr)  # both waves really are rarefactions
        u, c = O.trr_star(G, hl, ul, hr, ur)
        assert abs(c - math.sqrt(G * hs)) < 1e-12 and abs(u - us) < 1e-12


def test_two_rarefaction_speeds_bound_the_exact_waves(oracle_mod):
    """Equal states: u -+ c for both estimates.  Two rarefactions: the heads
    uL - cL and uR + cR.  Two shocks (colliding streams): the estimate lies
    outside the exact shock speeds, as HLL requires."""
    O = oracle_mod
    for kind in (0, 1):
        SL, SR = O.wave_speeds(kind, G, 1.3, 0.4, 1.3, 0.4)
        c = math.sqrt(G * 1.3)
        assert abs(SL - (0.4 - c)) < 1e-14 and abs(SR - (0.4 + c)) < 1e-14
    SL, SR = O.wave_speeds(1, G, 1.0, -0.5, 1.0, 0.5)
    assert abs(SL - (-0.5 - math.sqrt(G))) < 1e-14 and abs(SR - (0.5 + math.sqrt(G))) < 1e-14
    for hl, ul, hr, ur in ((1.0, 2.0, 1.0, -2.0), (1.0, 1.0, 2.0, -3.0), (0.5, 3.0, 0.8, 0.0)):
        hs, us = exact_riemann_star(hl, ul, hr, ur)
        assert hs > max(hl, hr)  # both waves are shocks
        sl = ul - math.sqrt(G * hl) * math.sqrt(0.5 * (hs + hl) * hs / hl ** 2)
        sr = ur + math.sqrt(G * hr) * math.sqrt(0.5 * (hs + hr) * hs / hr ** 2)
        SL, SR = O.wave_speeds(1, G, hl, ul, hr, ur)
        assert SL <= sl and SR >= sr, (SL, sl, SR, sr)


def test_hll_with_two_rarefaction_speeds_is_consistent_and_upwind(oracle_mod):
    O = oracle_mod
    H, uL, ut, un = 1.3, 0.7, -0.2, 0.6
    f = O.hll_v(1, G, H, uL, ut, un, H, uL, ut, un)
    np.testing.assert_allclose(f, (un * H, un * H * uL, un * H * ut), rtol=1e-14)
    f = O.hll_v(1, G, 0.01, 5.0, 1.0, 5.0, 0.02, 4.0, 0.0, 4.0)
    np.testing.assert_allclose(f, (5.0 * 0.01, 5.0 * 0.01 * 5.0, 5.0 * 0.01 * 1.0), rtol=1e-14)
    a, b = (1.1, 0.3, 0.2, 0.4), (0.6, -0.5, 0.1, -0.3)
    f = O.hll_v(1, G, *a, *b)
    g = O.hll_v(1, G, b[0], -b[1], b[2], -b[3], a[0], -a[1], a[2], -a[3])
    np.testing.assert_allclose(g, (-f[0], f[1], -f[2]), rtol=1e-13, atol=1e-15)


def _run_to(O, p, inp, s, T):
    while s.t < T - 1e-12:
        c = O.cfl(p, inp, s)
        O.step(p, inp, s, dt_fixed=min(c["dt"], T - s.t))


def _stoker_errors(O, **variant):
    errs = []
    for nx, dx in ((256, 1.0), (512, 0.5)):
        w = W.dam_break_1d(nx=nx, ny=2, dx=dx, x_dam=nx // 2, manning=0.0, sediment=False)
        p, inp, s = oracle_case(O, w, **variant)
        _run_to(O, p, inp, s, 10.0)
        x = (np.arange(nx) + 0.5) * dx
        h, u, hm, um, sp = stoker(2.0, 0.5, x, s.t, 128.0)
        H = s.H[0]
        U = s.qx[0] / H
        errs.append(np.abs(H - h).sum() * dx)
        band = (x > 128 + 0.3 * um * 10) & (x < 128 + 0.8 * sp * 10)
        assert abs(H[band].mean() - hm) / hm < 0.01, variant
        assert abs(U[band].mean() - um) / um < 0.01, variant
        xs = x[np.argmax(H < 0.5 * (hm + 0.5))]
        assert abs(xs - (128 + sp * s.t)) <= 2 * dx, variant
    assert errs[1] < 0.6 * errs[0], variant
    return errs


def test_stoker_with_every_limiter_and_speed_estimate(oracle_mod):
    """Each variant converges to the exact wet-bed dam break (plateau within 1%,
    shock within two cells, L1 falling under refinement); MC and superbee,
    the less diffusive limiters, are closer to it than minmod."""
    O = oracle_mod
    e = {name: _stoker_errors(O, limiter=k) for name, k in LIMITERS.items()}
    assert e["mc"][0] < e["minmod"][0] and e["superbee"][0] < e["minmod"][0]
    _stoker_errors(O, hll_speeds=1)
    _stoker_errors(O, limiter=2, hll_speeds=1)
    _stoker_errors(O, force_order=2)
    _stoker_errors(O, limiter=1, force_order=2)


def test_ritter_with_two_rarefaction_speeds(oracle_mod):
    """Dry-bed dam break with the two-rarefaction speeds: L1 falls under
    refinement and no water runs ahead of the exact front."""
    O = oracle_mod
    errs = []
    for nx, dx in ((256, 1.0), (512, 0.5)):
        w = W.dam_break_1d(nx=nx, ny=2, dx=dx, x_dam=nx // 2, h_right=0.0, manning=0.0,
                           sediment=False)
        p, inp, s = oracle_case(O, w, hll_speeds=1)
        _run_to(O, p, inp, s, 8.0)
        x = (np.arange(nx) + 0.5) * dx
        errs.append(np.abs(s.H[0] - ritter(2.0, x, s.t, 128.0)).sum() * dx)
        front = 128.0 + 2 * math.sqrt(2 * G) * s.t
        assert np.all(s.H[0][x > front + 2 * dx] == 0.0)
    assert errs[1] < 0.6 * errs[0]


@pytest.mark.parametrize("limiter,speeds,force_order",
                         [(1, 0, 1), (2, 0, 1), (0, 1, 1), (2, 1, 1), (0, 0, 2), (1, 0, 2),
                          (2, 1, 2)])
def test_variants_keep_the_lake_at_rest_and_conserve(oracle_mod, limiter, speeds, force_order):
    """Well-balanced and conservative with every variant: a lake over a seeded
    bed with emerged islands stays still (walls, then open sides), and a
    walled fractal dam break keeps its water and sediment volume."""
    O = oracle_mod
    for bc in ((0, 0, 0, 0), (1, 1, 1, 1)):
        w = W.lake_at_rest(48, 36, bc=bc)
        p, inp, s = oracle_case(O, w, limiter=limiter, hll_speeds=speeds,
                                force_order=force_order)
        z0 = s.H + s.b
        O.run(p, inp, s, 200)
        wet = s.H > 0
        assert np.abs((s.H + s.b) - z0)[wet].max() <= 1e-12
        assert np.abs(s.qx).max() <= 1e-12 and np.abs(s.qy).max() <= 1e-12
    w = W.dam_break_fractal(n=40, ny=28, dx=2.0, seed=5, relief=6.0, depth=4.0)
    w.bc = (0, 0, 0, 0)
    w.psi = np.random.default_rng(1).uniform(0.3, 0.45, (w.ny, w.nx))
    w.sed_law = W.SED_EQ4
    p, inp, s = oracle_case(O, w, limiter=limiter, hll_speeds=speeds, force_order=force_order)
    V0 = O.volumes(p, inp, s)
    O.run(p, inp, s, 300)
    V1 = O.volumes(p, inp, s)
    assert abs(V1[0] - V0[0]) / V0[0] < 1e-13
    assert abs(V1[1] - V0[1]) / V0[1] < 1e-13


@pytest.mark.parametrize("limiter,speeds,force_order", [(1, 1, 1), (2, 0, 1), (1, 0, 2)])
def test_variants_keep_mirror_symmetry(oracle_mod, limiter, speeds, force_order):
    """A problem mirrored in x gives the mirrored answer (walls on both x
    sides exercise the mirrored-ghost wall flux of each estimate)."""
    O = oracle_mod
    w = W.dam_break_fractal(n=36, ny=20, dx=2.0, seed=9, relief=5.0, depth=4.0)
    w.bc = (0, 0, 1, 1)
    p, inp, s = oracle_case(O, w, limiter=limiter, hll_speeds=speeds, force_order=force_order)
    O.run(p, inp, s, 120)
    wm = W.dam_break_fractal(n=36, ny=20, dx=2.0, seed=9, relief=5.0, depth=4.0)
    wm.bc = (0, 0, 1, 1)
    wm.H, wm.b = wm.H[:, ::-1].copy(), wm.b[:, ::-1].copy()
    wm.qx, wm.qy = -wm.qx[:, ::-1].copy(), wm.qy[:, ::-1].copy()
    pm, im, sm = oracle_case(O, wm, limiter=limiter, hll_speeds=speeds, force_order=force_order)
    O.run(pm, im, sm, 120)
    np.testing.assert_allclose(sm.H[:, ::-1], s.H, atol=1e-11)
    np.testing.assert_allclose(-sm.qx[:, ::-1], s.qx, atol=1e-10)
    np.testing.assert_allclose(sm.qy[:, ::-1], s.qy, atol=1e-10)


def _smooth_force_errors(O, limiter, force_order, sizes=(32, 64, 128, 256)):
    """L1 (mean) and L-inf error of the Lagrangian force against the exact
    -g H dzeta/dx at the cell centres, for a smooth surface
    zeta = 3 + 0.3 cos(pi x / L) (level at both walls) over a sloping, waving
    bed, uniform along y."""
    out = []
    for n in sizes:
        L = 100.0
        dx = L / n
        x = (np.arange(n) + 0.5) * dx
        zeta = 3.0 + 0.3 * np.cos(np.pi * x / L)
        b = 0.8 * np.sin(2 * np.pi * x / L) + 0.3 * x / L
        H = zeta - b
        p = O.Params(nx=n, ny=3, dx=dx, limiter=limiter, force_order=force_order)
        Sx, Sy = O.force(p, np.tile(H, (3, 1)), np.tile(b, (3, 1)))
        assert np.all(Sy == 0.0)
        exact = -G * H * (-0.3 * np.pi / L) * np.sin(np.pi * x / L)
        e = np.abs(Sx[1] - exact)
        out.append((e.mean(), e.max()))
    return np.array(out)


def test_second_order_force_converges_at_second_order(oracle_mod):
    """On a smooth state the hydrostatic-face force on cell values is a
    first-order approximation of -g H grad(zeta) (the face bed max(b_L, b_R)
    departs from the bed by O(dx) where it slopes); on limited reconstructed
    states with the centred term it is second order in L1 for every limiter
    (the limiters clip the slopes at the surface's extrema, so L-inf stays
    first order)."""
    O = oracle_mod
    e1 = _smooth_force_errors(O, 0, 1)
    o1 = np.log2(e1[:-1, 0] / e1[1:, 0])
    assert np.all((o1 > 0.95) & (o1 < 1.15)), o1
    for lim in (0, 1, 2):
        e2 = _smooth_force_errors(O, lim, 2)
        o2 = np.log2(e2[:-1, 0] / e2[1:, 0])
        assert np.all((o2 > 1.9) & (o2 < 2.1)), (lim, o2)
        assert e2[-1, 0] < e1[-1, 0] / 10
        oi = np.log2(e2[:-1, 1] / e2[1:, 1])
        assert np.all(oi > 0.9), (lim, oi)


def test_second_order_force_is_exact_at_rest_and_symmetric(oracle_mod):
    """At rest over a seeded bed with islands the second-order force vanishes
    on every wet cell up to FP64 rounding of g H^2 / (2 dx) (as the
    first-order one does), while a 1 mm bump of the surface is felt; the
    force of the transposed state is the transposed y force bit for bit, and
    the mirrored state's x force is the negated mirror (up to the order of a
    product's factors)."""
    O = oracle_mod
    w = W.lake_at_rest(40, 30, seed=12, relief=3.0, level=2.0)
    wet = w.H > 0
    for lim in (0, 1, 2):
        p = O.Params(nx=w.nx, ny=w.ny, dx=1.0, limiter=lim, force_order=2)
        Sx, Sy = O.force(p, w.H, w.b)
        assert np.abs(Sx[wet]).max() <= 1e-13 and np.abs(Sy[wet]).max() <= 1e-13, lim
        Hb = w.H.copy()
        Hb[wet & (np.arange(w.nx)[None, :] == 20)] += 1e-3
        Bx, _ = O.force(p, Hb, w.b)
        assert np.abs(Bx[wet]).max() > 1e-3, lim
    d = W.dam_break_fractal(n=30, ny=22, dx=2.0, seed=4, relief=5.0, depth=3.0)
    p = O.Params(nx=30, ny=22, dx=2.0, limiter=1, force_order=2)
    Sx, Sy = O.force(p, d.H, d.b)
    pt = O.Params(nx=22, ny=30, dx=2.0, limiter=1, force_order=2)
    Tx, Ty = O.force(pt, d.H.T, d.b.T)
    assert np.array_equal(Ty, Sx.T) and np.array_equal(Tx, Sy.T)
    Mx, My = O.force(p, d.H[:, ::-1], d.b[:, ::-1])
    np.testing.assert_allclose(Mx[:, ::-1], -Sx, rtol=0, atol=1e-12)
    np.testing.assert_allclose(My[:, ::-1], Sy, rtol=0, atol=1e-12)
    assert np.abs(Sx).max() > 0.1
