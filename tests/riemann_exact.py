"""Exact solution of the 1D shallow-water Riemann problem (flat bed, no friction).

Independent of both the oracle and the HIP path: it follows the textbook construction (Stoker
1957; Toro, "Shock-capturing methods for free-surface shallow flows", 2001, ch. 5): the star
depth solves f_L(h) + f_R(h) + u_R - u_L = 0 with rarefaction branches
2 (sqrt(g h) - sqrt(g h_K)) and shock branches (h - h_K) sqrt(g (h + h_K) / (2 h h_K)); the
solution at x/t is then sampled wave by wave.  Dry beds use Ritter's fans.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq


def _f(h, hk, g):
    if h <= hk:
        return 2.0 * (math.sqrt(g * h) - math.sqrt(g * hk))
    return (h - hk) * math.sqrt(0.5 * g * (h + hk) / (h * hk))


def star_state(hl, ul, hr, ur, g=9.81):
    """Star depth and velocity of a wet-wet Riemann problem (no vacuum)."""
    fun = lambda h: _f(h, hl, g) + _f(h, hr, g) + ur - ul
    hi = max(hl, hr)
    while fun(hi) < 0.0:
        hi *= 2.0
    hs = brentq(fun, 1e-14, hi, xtol=1e-15, rtol=1e-15, maxiter=500)
    us = 0.5 * (ul + ur) + 0.5 * (_f(hs, hr, g) - _f(hs, hl, g))
    return hs, us


def wave_speeds(hl, ul, hr, ur, g=9.81):
    """Slowest and fastest signal speeds of the exact solution."""
    cl, cr = math.sqrt(g * hl), math.sqrt(g * hr)
    if hr == 0.0:
        return ul - cl, ul + 2.0 * cl
    if hl == 0.0:
        return ur - 2.0 * cr, ur + cr
    if ur - ul >= 2.0 * (cl + cr):        # dry region opens in the middle
        return ul - cl, ur + cr
    hs, us = star_state(hl, ul, hr, ur, g)
    if hs > hl:
        s_left = ul - cl * math.sqrt(0.5 * (hs + hl) * hs / (hl * hl))
    else:
        s_left = ul - cl
    if hs > hr:
        s_right = ur + cr * math.sqrt(0.5 * (hs + hr) * hs / (hr * hr))
    else:
        s_right = ur + cr
    return s_left, s_right


def sample(xi, hl, ul, hr, ur, g=9.81):
    """Depth and velocity at x/t = xi (array) for the Riemann problem (hl, ul | hr, ur)."""
    xi = np.asarray(xi, dtype=np.float64)
    h = np.empty_like(xi)
    u = np.empty_like(xi)
    cl, cr = math.sqrt(g * hl), math.sqrt(g * hr)
    if hr == 0.0:                          # Ritter: left rarefaction into a dry bed
        head, front = ul - cl, ul + 2.0 * cl
        left = xi <= head
        fan = (xi > head) & (xi < front)
        a = (ul + 2.0 * cl - xi[fan]) / 3.0
        h[left], u[left] = hl, ul
        h[fan], u[fan] = a * a / g, xi[fan] + a
        h[xi >= front], u[xi >= front] = 0.0, 0.0
        return h, u
    hs, us = star_state(hl, ul, hr, ur, g)
    cs = math.sqrt(g * hs)
    for idx in np.ndindex(xi.shape):
        x = xi[idx]
        if x <= us:  # left of the contact
            if hs > hl:
                s = ul - cl * math.sqrt(0.5 * (hs + hl) * hs / (hl * hl))
                h[idx], u[idx] = (hl, ul) if x < s else (hs, us)
            else:
                head, tail = ul - cl, us - cs
                if x <= head:
                    h[idx], u[idx] = hl, ul
                elif x >= tail:
                    h[idx], u[idx] = hs, us
                else:
                    a = (ul + 2.0 * cl - x) / 3.0
                    h[idx], u[idx] = a * a / g, x + a
        else:
            if hs > hr:
                s = ur + cr * math.sqrt(0.5 * (hs + hr) * hs / (hr * hr))
                h[idx], u[idx] = (hr, ur) if x > s else (hs, us)
            else:
                head, tail = ur + cr, us + cs
                if x >= head:
                    h[idx], u[idx] = hr, ur
                elif x <= tail:
                    h[idx], u[idx] = hs, us
                else:
                    a = (-ur + 2.0 * cr + x) / 3.0
                    h[idx], u[idx] = a * a / g, x - a
    return h, u
