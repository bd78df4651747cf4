"""Shared test helpers: build oracle inputs from a seeded workload, read golden fixtures,
and the exact dam-break solutions used as pins."""
from __future__ import annotations

import math
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def oracle_case(O, w, **over):
    """(Params, Inputs, State) of the FP64 oracle for workload ``w``."""
    kw = dict(nx=w.nx, ny=w.ny, dx=w.dx, bc=tuple(w.bc), cfl=w.cfl, sed_law=w.sed_law)
    kw.update({k: v for k, v in over.items() if k in O.Params.__dataclass_fields__})
    p = O.Params(**kw)
    inp = O.Inputs(nM=w.nM, d50=w.d50, psi=w.psi, qb=w.qb, inflow_idx=w.inflow_idx,
                   inflow_w=w.inflow_w, Q_base=w.Q_base, Q_peak=w.Q_peak, t_peak=w.t_peak,
                   t_sigma=w.t_sigma, beta=over.get("beta"))
    s = O.State(w.H, w.qx, w.qy, w.b)
    return p, inp, s


def read_golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split()
            vals[k] = float(v)
    return vals


def stoker(hl, hr, x, t, x0, g=9.81):
    """Exact wet-bed dam break (rarefaction + shock; textbook Riemann problem).
    Returns h(x,t), u(x,t), h_m, u_m, shock speed."""
    from scipy.optimize import brentq
    cl = math.sqrt(g * hl)

    def f(hm):
        u_rar = 2.0 * (cl - math.sqrt(g * hm))
        u_sho = (hm - hr) * math.sqrt(0.5 * g * (hm + hr) / (hm * hr))
        return u_rar - u_sho

    hm = brentq(f, hr, hl, xtol=1e-15)
    um = 2.0 * (cl - math.sqrt(g * hm))
    cm = math.sqrt(g * hm)
    s = hm * um / (hm - hr)
    xi = (x - x0) / t
    h = np.where(xi < -cl, hl, np.where(xi < um - cm, (2 * cl - xi) ** 2 / (9 * g),
                                        np.where(xi < s, hm, hr)))
    u = np.where(xi < -cl, 0.0, np.where(xi < um - cm, (2.0 / 3.0) * (cl + xi),
                                         np.where(xi < s, um, 0.0)))
    return h, u, hm, um, s


def ritter(h0, x, t, x0, g=9.81):
    """Exact dry-bed dam break: h = (2 c0 - xi)^2 / (9 g) on -c0 < xi < 2 c0."""
    c0 = math.sqrt(g * h0)
    xi = (x - x0) / t
    return np.where(xi < -c0, h0, np.where(xi < 2 * c0, (2 * c0 - xi) ** 2 / (9 * g), 0.0))


def exact_riemann_star(hl, ul, hr, ur, g=9.81):
    """Star state (h*, u*) of the shallow-water Riemann problem with wet sides,
    from the exact wave relations (textbook: each side a rarefaction if h* <= h_K,
    else a shock; root of f_L(h) + f_R(h) + u_R - u_L)."""
    from scipy.optimize import brentq

    def f(h, hk):
        if h <= hk:
            return 2.0 * (math.sqrt(g * h) - math.sqrt(g * hk))
        return (h - hk) * math.sqrt(0.5 * g * (h + hk) / (h * hk))

    def phi(h):
        return f(h, hl) + f(h, hr) + ur - ul

    hs = brentq(phi, 1e-12, 100.0 * max(hl, hr) + 10.0, xtol=1e-15, rtol=1e-15, maxiter=500)
    us = 0.5 * (ul + ur) + 0.5 * (f(hs, hr) - f(hs, hl))
    return hs, us
