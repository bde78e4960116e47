"""Exact solution of the Riemann problem for the 1D Euler equations of an ideal
gas (test helper, not method arithmetic).

Written from the standard construction: the star-region pressure p* solves
f_L(p) + f_R(p) + u_R - u_L = 0, where f_K is the velocity change across the
left or right wave: across a shock (p > p_K), from the Rankine-Hugoniot
conditions, f_K = (p - p_K) sqrt(A_K / (p + B_K)) with A_K = 2 / ((gamma + 1)
rho_K) and B_K = (gamma - 1) / (gamma + 1) p_K; across a rarefaction (p <= p_K),
from the isentropic relation and the Riemann invariant,
f_K = 2 c_K / (gamma - 1) ((p / p_K)^((gamma - 1) / (2 gamma)) - 1).
Then u* = (u_L + u_R + f_R(p*) - f_L(p*)) / 2, and the self-similar solution is
sampled at xi = x / t.
"""
from __future__ import annotations

import math

import numpy as np


def _f(p, rho, pk, gamma):
    c = math.sqrt(gamma * pk / rho)
    if p > pk:
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pk
        return (p - pk) * math.sqrt(A / (p + B))
    return 2.0 * c / (gamma - 1.0) * ((p / pk) ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)


def star_state(left, right, gamma):
    """(p*, u*) of the Riemann problem left = (rho, u, p), right = (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    g = lambda p: _f(p, rl, pl, gamma) + _f(p, rr, pr, gamma) + ur - ul
    lo, hi = 1e-14, max(pl, pr)
    while g(hi) < 0.0:
        hi *= 2.0
    for _ in range(200):                  # bisection: g is increasing in p
        mid = 0.5 * (lo + hi)
        if g(mid) > 0.0:
            hi = mid
        else:
            lo = mid
    p = 0.5 * (lo + hi)
    u = 0.5 * (ul + ur + _f(p, rr, pr, gamma) - _f(p, rl, pl, gamma))
    return p, u


def _side(state, ps, us, gamma, xi, sign):
    """The solution on one side of the contact; sign = +1 for the left wave (the
    right wave is the left wave of the mirrored problem)."""
    rk, uk, pk = state
    uk, us_, xi = sign * uk, sign * us, sign * xi          # mirrored: the wave faces -xi
    ck = math.sqrt(gamma * pk / rk)
    gm = (gamma - 1.0) / (gamma + 1.0)
    rho = np.full(xi.shape, rk)
    u = np.full(xi.shape, uk)
    p = np.full(xi.shape, pk)
    if ps > pk:                                           # shock
        S = uk - ck * math.sqrt((gamma + 1.0) / (2.0 * gamma) * ps / pk + (gamma - 1.0) / (2.0 * gamma))
        star = xi > S
        rho[star] = rk * (ps / pk + gm) / (gm * ps / pk + 1.0)
        u[star], p[star] = us_, ps
    else:                                                 # rarefaction
        cs = ck * (ps / pk) ** ((gamma - 1.0) / (2.0 * gamma))
        fan = (xi > uk - ck) & (xi < us_ - cs)
        star = xi >= us_ - cs
        rho[star] = rk * (ps / pk) ** (1.0 / gamma)
        u[star], p[star] = us_, ps
        c = 2.0 / (gamma + 1.0) * (ck + (gamma - 1.0) / 2.0 * (uk - xi[fan]))
        u[fan] = 2.0 / (gamma + 1.0) * (ck + (gamma - 1.0) / 2.0 * uk + xi[fan])
        rho[fan] = rk * (c / ck) ** (2.0 / (gamma - 1.0))
        p[fan] = pk * (c / ck) ** (2.0 * gamma / (gamma - 1.0))
    return np.stack([rho, sign * u, p])


def sample(left, right, gamma, xi):
    """(rho, u, p) of the exact solution at similarity coordinates xi = x / t
    (interface at x = 0)."""
    ps, us = star_state(left, right, gamma)
    xi = np.atleast_1d(np.asarray(xi, dtype=np.float64))
    lo = xi <= us
    out = np.empty((3, xi.size))
    out[:, lo] = _side(left, ps, us, gamma, xi[lo], 1.0)
    out[:, ~lo] = _side(right, ps, us, gamma, xi[~lo], -1.0)
    return out


SOD_LEFT, SOD_RIGHT = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)   # section 6.2, gamma = 1.4


def sod_periodic_profile(s, t, gamma=1.4):
    """(rho, u_par, p) of the Sod problem on the period-2 line with the left state
    on [-1/2, 1/2] and the right state on (1/2, 3/2], at coordinate s and time t,
    while the waves of the two interfaces have not met (t <= 0.2 here: they stay
    within 0.26 < s < 0.85 and its mirror image).  On [0, 1] it is the Sod solution
    of the interface at 1/2; on (1, 2) the mirror image about s = 1 (velocity
    negated).  u_par is the velocity along s."""
    sm = np.mod(np.atleast_1d(np.asarray(s, dtype=np.float64)), 2.0)
    out = np.empty((3, sm.size))
    lo = sm <= 1.0
    if lo.any():
        out[:, lo] = sample(SOD_LEFT, SOD_RIGHT, gamma, (sm[lo] - 0.5) / t)
    if (~lo).any():
        w = sample(SOD_LEFT, SOD_RIGHT, gamma, (2.0 - sm[~lo] - 0.5) / t)
        w[1] = -w[1]
        out[:, ~lo] = w
    return out


def sod_exact_cell_averages(config, n, h, t, q=6):
    """Density cell averages [ny, nx] of the exact Sod solution at time t on the
    periodic grid of inputs.sod (q-point Gauss rule per axis), and the coordinate
    s of every cell centre."""
    from paper_2401_16543_amd import inputs
    nx, ny = n
    g, w = np.polynomial.legendre.leggauss(q)
    xc = (np.arange(nx) + 0.5) * h
    yc = (np.arange(ny) + 0.5) * h
    Y, X = np.meshgrid(yc, xc, indexing="ij")
    acc = np.zeros((ny, nx))
    for gy, wy in zip(g, w):
        for gx, wx in zip(g, w):
            s = inputs.sod_parallel_coordinate(config, X + 0.5 * gx * h, Y + 0.5 * gy * h)
            acc += 0.25 * wx * wy * sod_periodic_profile(s.ravel(), t)[0].reshape(s.shape)
    return acc, inputs.sod_parallel_coordinate(config, X, Y)


def sod_l1_error(rho, config, n, h, t):
    """(mean, max) |rho - exact| over the cells whose centre has s mod 2 in [0, 1]
    (the tube and its left and right states; the rest is its mirror image)."""
    ex, s = sod_exact_cell_averages(config, n, h, t)
    sel = np.mod(s, 2.0) <= 1.0
    d = np.abs(np.asarray(rho) - ex)[sel]
    return float(d.mean()), float(d.max())
