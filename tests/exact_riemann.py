"""Closed-form references for the oracle's pins (independent of the oracle).

Exact solution of the 1D shallow-water Riemann problem on a flat frictionless
bed, from the textbook construction (Toro, "Shock-capturing methods for
free-surface shallow flows", ch. 5): the star depth is the root of
f_L(h) + f_R(h) + u_R - u_L = 0, with f_K the rarefaction branch
2 (sqrt(g h) - sqrt(g h_K)) for h <= h_K and the shock branch
(h - h_K) sqrt(g (h + h_K) / (2 h h_K)) for h > h_K.  The paper's wet-bed dam
break (Sec. 6.3) is the Stoker case; the dry-bed case is Ritter's solution.
"""
from __future__ import annotations

import math

import numpy as np

G = 9.81


def _fK(h, hK, g=G):
    if h <= hK:
        return 2.0 * (math.sqrt(g * h) - math.sqrt(g * hK))
    return (h - hK) * math.sqrt(0.5 * g * (h + hK) / (h * hK))


def star_state(hL, uL, hR, uR, g=G):
    """(h*, u*) for a wet/wet problem, by bisection (robust, 200 halvings)."""
    def f(h):
        return _fK(h, hL, g) + _fK(h, hR, g) + uR - uL
    lo, hi = 1e-14, 10.0 * max(hL, hR) + (abs(uL) + abs(uR)) ** 2 / g
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid) > 0.0:
            hi = mid
        else:
            lo = mid
    hs = 0.5 * (lo + hi)
    us = 0.5 * (uL + uR) + 0.5 * (_fK(hs, hR, g) - _fK(hs, hL, g))
    return hs, us


def sample(xi, hL, uL, hR, uR, g=G):
    """Exact (h, u) at similarity coordinates xi = (x - x0)/t."""
    xi = np.asarray(xi, np.float64)
    h = np.empty_like(xi)
    u = np.empty_like(xi)
    aL, aR = math.sqrt(g * hL), math.sqrt(g * hR) if hR > 0 else 0.0
    if hR <= 0.0:  # Ritter: dry bed on the right
        head, front = uL - aL, uL + 2.0 * aL
        fan = (xi >= head) & (xi <= front)
        h[:] = 0.0
        u[:] = 0.0
        h[xi < head] = hL
        u[xi < head] = uL
        h[fan] = (uL + 2.0 * aL - xi[fan]) ** 2 / (9.0 * g)
        u[fan] = (uL + 2.0 * aL + 2.0 * xi[fan]) / 3.0
        return h, u
    hs, us = star_state(hL, uL, hR, uR, g)
    a_s = math.sqrt(g * hs)
    for i, x in enumerate(xi.ravel()):
        if x <= us:  # left of the contact
            if hs > hL:
                SL = uL - aL * math.sqrt(0.5 * (hs + hL) * hs / hL ** 2)
                h.flat[i], u.flat[i] = (hL, uL) if x < SL else (hs, us)
            else:
                head, tail = uL - aL, us - a_s
                if x < head:
                    h.flat[i], u.flat[i] = hL, uL
                elif x > tail:
                    h.flat[i], u.flat[i] = hs, us
                else:
                    h.flat[i] = (uL + 2.0 * aL - x) ** 2 / (9.0 * g)
                    u.flat[i] = (uL + 2.0 * aL + 2.0 * x) / 3.0
        else:
            if hs > hR:
                SR = uR + aR * math.sqrt(0.5 * (hs + hR) * hs / hR ** 2)
                h.flat[i], u.flat[i] = (hR, uR) if x > SR else (hs, us)
            else:
                head, tail = uR + aR, us + a_s
                if x > head:
                    h.flat[i], u.flat[i] = hR, uR
                elif x < tail:
                    h.flat[i], u.flat[i] = hs, us
                else:
                    h.flat[i] = (-uR + 2.0 * aR + x) ** 2 / (9.0 * g)
                    u.flat[i] = (uR - 2.0 * aR + 2.0 * x) / 3.0
    return h, u


def cell_average_h(x_c, x0, t, hL, uL, hR, uR, dx, nsub=16, g=G):
    """Exact h averaged over [x_c - dx/2, x_c + dx/2] (midpoint sub-sampling)."""
    off = (np.arange(nsub) + 0.5) / nsub - 0.5
    xs = (np.asarray(x_c)[:, None] + off[None, :] * dx)
    h, _ = sample((xs - x0) / t, hL, uL, hR, uR, g)
    return h.mean(axis=1)
