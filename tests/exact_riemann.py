"""Exact solution of the 1D Riemann problem for an ideal gas (test utility).

Written from the standard textbook construction (pressure function of the
left and right waves -- shock via Rankine-Hugoniot, rarefaction via the
isentropic Riemann invariant -- and a monotone root solve for the star
pressure; see E. F. Toro, Riemann Solvers and Numerical Methods for Fluid
Dynamics, ch. 4).  Independent of the oracle and of the HIP library.
"""
from __future__ import annotations

import math


def _wave(p, rho, pK, cK, g):
    """Pressure function f_K(p) and its derivative."""
    if p > pK:
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pK
        s = math.sqrt(A / (p + B))
        return (p - pK) * s, s * (1.0 - 0.5 * (p - pK) / (B + p))
    r = p / pK
    f = 2.0 * cK / (g - 1.0) * (r ** ((g - 1.0) / (2.0 * g)) - 1.0)
    df = 1.0 / (rho * cK) * r ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_pressure(rl, ul, pl, rr, ur, pr, g=1.4):
    """Star-region pressure p* (0 when the data generate vacuum)."""
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    du = ur - ul
    if 2.0 * (cl + cr) / (g - 1.0) <= du:
        return 0.0

    def F(p):
        a, da = _wave(p, rl, pl, cl, g)
        b, db = _wave(p, rr, pr, cr, g)
        return a + b + du, da + db

    # F is increasing in p; bracket the root, then bisect/Newton.
    lo, hi = 0.0, max(pl, pr)
    while F(hi)[0] < 0.0:
        lo, hi = hi, 2.0 * hi
    p = 0.5 * (lo + hi)
    for _ in range(400):
        f, df = F(p)
        if f == 0.0:
            return p
        if f < 0.0:
            lo = p
        else:
            hi = p
        pn = p - f / df if df > 0 else 0.5 * (lo + hi)
        if not (lo < pn < hi):
            pn = 0.5 * (lo + hi)
        if abs(pn - p) <= 1e-16 * max(p, 1e-300) or hi - lo <= 1e-16 * hi:
            return pn
        p = pn
    return p


def max_wave_speed(rl, ul, pl, rr, ur, pr, g=1.4):
    """max(-(left wave speed)_+, (right wave speed)_+) of the exact fan:
    shock speed for a shock, head speed for a rarefaction."""
    ps = star_pressure(rl, ul, pl, rr, ur, pr, g)
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    if ps > pl:
        sl = ul - cl * math.sqrt((g + 1.0) / (2.0 * g) * ps / pl + (g - 1.0) / (2.0 * g))
    else:
        sl = ul - cl
    if ps > pr:
        sr = ur + cr * math.sqrt((g + 1.0) / (2.0 * g) * ps / pr + (g - 1.0) / (2.0 * g))
    else:
        sr = ur + cr
    return max(max(-sl, 0.0), max(sr, 0.0)), ps


def sample(rl, ul, pl, rr, ur, pr, xi, g=1.4):
    """(rho, u, p) of the self-similar solution at xi = x/t (no vacuum)."""
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    ps = star_pressure(rl, ul, pl, rr, ur, pr, g)
    fl, _ = _wave(ps, rl, pl, cl, g)
    fr, _ = _wave(ps, rr, pr, cr, g)
    us = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    gm = (g - 1.0) / (g + 1.0)
    if xi <= us:  # left of contact
        if ps > pl:
            sl = ul - cl * math.sqrt((g + 1.0) / (2.0 * g) * ps / pl + (g - 1.0) / (2.0 * g))
            if xi <= sl:
                return rl, ul, pl
            r = rl * (ps / pl + gm) / (gm * ps / pl + 1.0)
            return r, us, ps
        shl = ul - cl
        if xi <= shl:
            return rl, ul, pl
        cs = cl * (ps / pl) ** ((g - 1.0) / (2.0 * g))
        stl = us - cs
        if xi > stl:
            return rl * (ps / pl) ** (1.0 / g), us, ps
        c = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * (ul - xi))
        u = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * ul + xi)
        r = rl * (c / cl) ** (2.0 / (g - 1.0))
        return r, u, pl * (c / cl) ** (2.0 * g / (g - 1.0))
    if ps > pr:
        sr = ur + cr * math.sqrt((g + 1.0) / (2.0 * g) * ps / pr + (g - 1.0) / (2.0 * g))
        if xi >= sr:
            return rr, ur, pr
        r = rr * (ps / pr + gm) / (gm * ps / pr + 1.0)
        return r, us, ps
    shr = ur + cr
    if xi >= shr:
        return rr, ur, pr
    cs = cr * (ps / pr) ** ((g - 1.0) / (2.0 * g))
    str_ = us + cs
    if xi < str_:
        return rr * (ps / pr) ** (1.0 / g), us, ps
    c = 2.0 / (g + 1.0) * (cr - 0.5 * (g - 1.0) * (ur - xi))
    u = 2.0 / (g + 1.0) * (-cr + 0.5 * (g - 1.0) * ur + xi)
    r = rr * (c / cr) ** (2.0 / (g - 1.0))
    return r, u, pr * (c / cr) ** (2.0 * g / (g - 1.0))
