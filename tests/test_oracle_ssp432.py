"""Pins of the oracle's SSP(4,3,2) step (section 6: the four-stage third-order SSP
Runge-Kutta method with the embedded three-stage second-order SSP method): the
order of the main method, the order of the embedded error estimate, and a
constant state."""
import math

import numpy as np
import pytest

from paper_2401_16543_amd import inputs


def _U(n=16):
    return inputs.cell_averages(inputs.smooth(4, 2, 2), n, 1.4, rule="gauss", q=3).numpy()


def test_main_method_is_third_order(oracle_mod):
    """Integrate to T with dt, dt/2, dt/4 and compare to dt/64 on the same spatial
    discretisation: the error falls by ~8 per halving."""
    n = 16
    o = oracle_mod.Oracle(2, 2, (n, n))
    U0 = _U(n)
    T = 0.04

    def run(k):
        U = U0.copy()
        for _ in range(k):
            U, _ = o.step_ssp432(U, T / k)
        return U

    ref = run(64)
    errs = [np.abs(run(k) - ref).max() for k in (4, 8, 16)]
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) >= 2.7, (errs, rates)


def test_embedded_estimate_is_third_order_local(oracle_mod):
    """The estimate U+ - Uhat is the local error of the embedded second-order
    method: O(dt^3) for one step."""
    n = 16
    o = oracle_mod.Oracle(2, 2, (n, n))
    U0 = _U(n)
    e = [o.step_ssp432(U0, dt, atol=1e-3, rtol=0.0)[1] for dt in (0.01, 0.005, 0.0025)]
    rates = [math.log2(e[i] / e[i + 1]) for i in range(2)]
    assert all(2.7 <= r <= 3.3 for r in rates), (e, rates)


def test_constant_state(oracle_mod):
    n = 12
    U = np.empty((4, n, n))
    U[0], U[1], U[2], U[3] = 1.2, 0.3, -0.2, 2.9
    o = oracle_mod.Oracle(2, 2, (n, n))
    Up, err = o.step_ssp432(U, 0.01)
    assert np.abs(Up - U).max() <= 1e-13 and err <= 1e-9
