"""Exact solution of the Riemann problem for the 1D Euler equations of an
ideal gas -- TEST INFRASTRUCTURE ONLY (part of the oracle).

The FD-LB model is built to recover the Euler equations of Sec. 2, Eq. (e2),
with pressure P = rho T (R = 1) and energy density rho (b T + u^2) / 2, i.e.
an ideal gas of adiabatic index gamma = (b + 2) / b.  The paper validates the
model against exact solutions of shock-tube problems (Sec. 4 (1)); this is
that exact solution, written from the gas dynamics: the star-region pressure
solves f_L(p) + f_R(p) + (u_R - u_L) = 0, where f_K is the shock
(Rankine-Hugoniot) branch for p > p_K and the rarefaction (isentrope plus
Riemann invariant) branch otherwise; the solution is self-similar in
x / t and is sampled wave by wave.  Newton iteration from the
two-rarefaction estimate, then bisection safeguarding.
"""
from __future__ import annotations

import math

import numpy as np


def _fk(p, rho, pk, g):
    """Pressure function of one side and its derivative."""
    a = math.sqrt(g * pk / rho)
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        s = math.sqrt(A / (p + B))
        return (p - pk) * s, s * (1.0 - 0.5 * (p - pk) / (B + p))
    # rarefaction
    r = (p / pk) ** ((g - 1.0) / (2.0 * g))
    return 2.0 * a / (g - 1.0) * (r - 1.0), 1.0 / (rho * a) * (p / pk) ** (-(g + 1.0) / (2.0 * g))


def star_state(left, right, gamma):
    """(p*, u*) for left/right states (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    g = gamma
    al = math.sqrt(g * pl / rl)
    ar = math.sqrt(g * pr / rr)
    du = ur - ul
    if 2.0 * (al + ar) / (g - 1.0) <= du:
        raise ValueError("vacuum is generated; not handled")
    z = (g - 1.0) / (2.0 * g)
    p = ((al + ar - 0.5 * (g - 1.0) * du) / (al / pl ** z + ar / pr ** z)) ** (1.0 / z)
    p = max(p, 1e-12 * min(pl, pr))

    def F(pp):
        fl, dl = _fk(pp, rl, pl, g)
        fr, dr = _fk(pp, rr, pr, g)
        return fl + fr + du, dl + dr

    lo, hi = 0.0, max(pl, pr)
    while F(hi)[0] < 0.0:
        hi *= 2.0
    for _ in range(200):
        val, der = F(p)
        if val > 0.0:
            hi = min(hi, p)
        else:
            lo = max(lo, p)
        pn = p - val / der
        if not (lo < pn < hi):
            pn = 0.5 * (lo + hi)
        if abs(pn - p) <= 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _fk(p, rl, pl, g)
    fr, _ = _fk(p, rr, pr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(left, right, gamma, xi):
    """(rho, u, p) at similarity coordinates xi = (x - x0) / t (array)."""
    rl, ul, pl = left
    rr, ur, pr = right
    g = gamma
    ps, us = star_state(left, right, gamma)
    al = math.sqrt(g * pl / rl)
    ar = math.sqrt(g * pr / rr)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    gm = (g - 1.0) / (g + 1.0)
    for n, s in enumerate(xi.flat):
        if s <= us:  # left of contact
            if ps > pl:  # left shock
                rs = rl * (ps / pl + gm) / (gm * ps / pl + 1.0)
                S = ul - al * math.sqrt((g + 1.0) / (2.0 * g) * ps / pl + (g - 1.0) / (2.0 * g))
                st = (rl, ul, pl) if s <= S else (rs, us, ps)
            else:  # left rarefaction
                rs = rl * (ps / pl) ** (1.0 / g)
                ash = al * (ps / pl) ** ((g - 1.0) / (2.0 * g))
                head, tail = ul - al, us - ash
                if s <= head:
                    st = (rl, ul, pl)
                elif s >= tail:
                    st = (rs, us, ps)
                else:
                    c = 2.0 / (g + 1.0) + (g - 1.0) / ((g + 1.0) * al) * (ul - s)
                    st = (rl * c ** (2.0 / (g - 1.0)),
                          2.0 / (g + 1.0) * (al + 0.5 * (g - 1.0) * ul + s),
                          pl * c ** (2.0 * g / (g - 1.0)))
        else:  # right of contact
            if ps > pr:  # right shock
                rs = rr * (ps / pr + gm) / (gm * ps / pr + 1.0)
                S = ur + ar * math.sqrt((g + 1.0) / (2.0 * g) * ps / pr + (g - 1.0) / (2.0 * g))
                st = (rr, ur, pr) if s >= S else (rs, us, ps)
            else:  # right rarefaction
                rs = rr * (ps / pr) ** (1.0 / g)
                ash = ar * (ps / pr) ** ((g - 1.0) / (2.0 * g))
                head, tail = ur + ar, us + ash
                if s >= head:
                    st = (rr, ur, pr)
                elif s <= tail:
                    st = (rs, us, ps)
                else:
                    c = 2.0 / (g + 1.0) - (g - 1.0) / ((g + 1.0) * ar) * (ur - s)
                    st = (rr * c ** (2.0 / (g - 1.0)),
                          2.0 / (g + 1.0) * (-ar + 0.5 * (g - 1.0) * ur + s),
                          pr * c ** (2.0 * g / (g - 1.0)))
        rho.flat[n], u.flat[n], p.flat[n] = st
    return rho, u, p


def profile(left, right, gamma, x, x0, t):
    """Exact (rho, u, p) at positions x and time t > 0, discontinuity at x0."""
    return sample(left, right, gamma, (np.asarray(x, dtype=np.float64) - x0) / t)
