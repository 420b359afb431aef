"""Exact solution of the 1-D Euler Riemann problem for an ideal gas.

Test pin for shock problems: the star pressure solves
f_L(p) + f_R(p) + (u_R - u_L) = 0, where f_K is the shock (Rankine-Hugoniot)
or rarefaction (isentropic) velocity jump across the wave of side K; the
solution is then sampled on rays x/t.  Written from the gas-dynamics
relations; shares nothing with the scheme under test.
"""
import math

import numpy as np


def _fk(p, rho, pk, ck, g):
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        s = math.sqrt(A / (p + B))
        f = (p - pk) * s
        df = s * (1.0 - 0.5 * (p - pk) / (B + p))
    else:  # rarefaction
        f = 2.0 * ck / (g - 1.0) * ((p / pk) ** ((g - 1.0) / (2.0 * g)) - 1.0)
        df = 1.0 / (rho * ck) * (p / pk) ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(left, right, g=1.4):
    rl, ul, pl = left
    rr, ur, pr = right
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    if 2.0 * (cl + cr) / (g - 1.0) <= ur - ul:
        raise ValueError("vacuum is generated")
    p = max(1e-12, 0.5 * (pl + pr) - 0.125 * (ur - ul) * (rl + rr) * (cl + cr))
    for _ in range(200):
        fl, dfl = _fk(p, rl, pl, cl, g)
        fr, dfr = _fk(p, rr, pr, cr, g)
        dp = (fl + fr + ur - ul) / (dfl + dfr)
        pn = max(1e-14, p - dp)
        if abs(pn - p) <= 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _fk(p, rl, pl, cl, g)
    fr, _ = _fk(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(left, right, s, g=1.4):
    """(rho, u, p) on the ray x/t = s (jump at x = 0, t > 0)."""
    rl, ul, pl = left
    rr, ur, pr = right
    ps, us = star_state(left, right, g)
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    if s <= us:  # left of the contact
        if ps > pl:
            sl = ul - cl * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
            if s <= sl:
                return rl, ul, pl
            r = rl * (ps / pl + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pl + 1)
            return r, us, ps
        csl = cl * (ps / pl) ** ((g - 1) / (2 * g))
        if s <= ul - cl:
            return rl, ul, pl
        if s >= us - csl:
            return rl * (ps / pl) ** (1 / g), us, ps
        u = 2 / (g + 1) * (cl + (g - 1) / 2 * ul + s)
        c = 2 / (g + 1) * (cl + (g - 1) / 2 * (ul - s))
        r = rl * (c / cl) ** (2 / (g - 1))
        return r, u, pl * (c / cl) ** (2 * g / (g - 1))
    if ps > pr:
        sr = ur + cr * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
        if s >= sr:
            return rr, ur, pr
        r = rr * (ps / pr + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pr + 1)
        return r, us, ps
    csr = cr * (ps / pr) ** ((g - 1) / (2 * g))
    if s >= ur + cr:
        return rr, ur, pr
    if s <= us + csr:
        return rr * (ps / pr) ** (1 / g), us, ps
    u = 2 / (g + 1) * (-cr + (g - 1) / 2 * ur + s)
    c = 2 / (g + 1) * (cr - (g - 1) / 2 * (ur - s))
    r = rr * (c / cr) ** (2 / (g - 1))
    return r, u, pr * (c / cr) ** (2 * g / (g - 1))


def cell_average_density(left, right, x0, t, xf, g=1.4, sub=64):
    """Exact cell averages of rho on cells with faces xf (midpoint rule on
    `sub` sub-cells per cell)."""
    out = np.empty(len(xf) - 1)
    for i in range(len(xf) - 1):
        xs = xf[i] + (np.arange(sub) + 0.5) * (xf[i + 1] - xf[i]) / sub
        out[i] = np.mean([sample(left, right, (x - x0) / t, g)[0] for x in xs])
    return out
