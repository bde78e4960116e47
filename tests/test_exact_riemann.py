"""Pins of the exact Riemann solver used as a reference by the Sod tests: the
jump conditions across each wave and the relations inside a rarefaction."""

import numpy as np
import pytest

import exact_riemann as ER


def _cons(w, gamma):
    rho, u, p = w
    return np.array([rho, rho * u, p / (gamma - 1.0) + 0.5 * rho * u * u])


def _flux(w, gamma):
    rho, u, p = w
    E = p / (gamma - 1.0) + 0.5 * rho * u * u
    return np.array([rho * u, rho * u * u + p, (E + p) * u])


@pytest.mark.parametrize("left,right,gamma", [(ER.SOD_LEFT, ER.SOD_RIGHT, 1.4),
                                               ((1.0, 0.0, 1000.0), (1.0, 0.0, 0.01), 1.4),
                                               ((1.0, -2.0, 0.4), (1.0, 2.0, 0.4), 1.4),
                                               ((5.99924, 19.5975, 460.894), (5.99242, -6.19633, 46.095), 5.0 / 3.0)])
def test_waves_satisfy_their_conditions(left, right, gamma):
    ps, us = ER.star_state(left, right, gamma)
    # the star pressure makes the two wave curves meet
    assert abs(ER._f(ps, left[0], left[2], gamma) + ER._f(ps, right[0], right[2], gamma) + right[1] - left[1]) \
        <= 1e-10 * (1.0 + abs(right[1] - left[1]))
    xi = np.linspace(-30.0, 30.0, 120001)
    W = ER.sample(left, right, gamma, xi)
    # contact: pressure and velocity continuous, density may jump
    k = np.searchsorted(xi, us)
    assert abs(W[2, k - 1] - W[2, k]) <= 1e-9 * ps and abs(W[1, k - 1] - W[1, k]) <= 1e-9 * (1 + abs(us))
    for side, ref in ((0, left), (1, right)):
        if ps > ref[2]:
            # shock: locate it, check Rankine-Hugoniot F(b) - F(a) = S (U(b) - U(a))
            seg = slice(0, k) if side == 0 else slice(k, None)
            rho = W[0, seg]
            jumps = np.flatnonzero(np.abs(np.diff(rho)) > 1e-12)
            j = jumps[0] if side == 0 else jumps[-1]
            a, b = W[:, seg][:, j], W[:, seg][:, j + 1]
            Ua, Ub = _cons(a, gamma), _cons(b, gamma)
            # the mass condition gives the shock speed; momentum and energy must agree
            S = (Ub[1] - Ua[1]) / (Ub[0] - Ua[0])
            assert abs(S - xi[seg][j]) <= 2 * (xi[1] - xi[0])
            res = _flux(b, gamma) - _flux(a, gamma) - S * (Ub - Ua)
            assert np.all(np.abs(res) <= 1e-9 * (np.abs(_flux(b, gamma)) + np.abs(S * Ub) + 1.0))
        else:
            # rarefaction: entropy p / rho^gamma and the Riemann invariant constant
            seg = slice(0, k) if side == 0 else slice(k, None)
            w = W[:, seg]
            ent = w[2] / w[0] ** gamma
            assert np.abs(ent / (ref[2] / ref[0] ** gamma) - 1.0).max() <= 1e-9
            c = np.sqrt(gamma * w[2] / w[0])
            inv = w[1] + (2.0 if side == 0 else -2.0) * c / (gamma - 1.0)
            assert np.abs(inv - inv[0]).max() <= 1e-9 * (1.0 + abs(inv[0]))


def test_sod_periodic_profile_mirrors():
    s = np.linspace(0.0, 1.0, 101)
    a = ER.sod_periodic_profile(s, 0.2)
    b = ER.sod_periodic_profile(2.0 - s, 0.2)
    assert np.allclose(a[[0, 2]], b[[0, 2]]) and np.allclose(a[1], -b[1])
    # undisturbed states at the ends of [0, 1]
    assert np.allclose(a[:, 0], [1.0, 0.0, 1.0]) and np.allclose(a[:, -1], [0.125, 0.0, 0.1])
