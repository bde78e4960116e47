"""The host step controller of the SSP(4,3,2) driver (`integrate.py`), run on
the CPU against a stand-in device whose error norm follows a known law:
err = (dt / h)^3, the local behaviour of a third-order embedded estimate.
The stand-in's step advances a clock held in the state, so the state tells
which attempts were kept."""
import pytest
import torch

from paper_2401_16543_amd.integrate import integrate


class Clock:
    def __init__(self, h, cfl=1e9, err_zero=False):
        self.h, self.cfl, self.err_zero = h, cfl, err_zero
        self.attempts = []

    def cfl_dt(self, U, cfl_max):
        return self.cfl * cfl_max

    def step_ssp432(self, U, out, dt, atol, rtol):
        self.attempts.append(dt)
        out.copy_(U + dt)
        return 0.0 if self.err_zero else (dt / self.h) ** 3


def _run(dev, t_end, **kw):
    U = torch.zeros(3, dtype=torch.float64)
    res = integrate(dev, U, t_end, **kw)
    return U, res


def test_reaches_the_end_time_exactly_with_kept_steps_only():
    dev = Clock(h=0.013)
    U, res = _run(dev, 1.0, dt0=0.05)
    assert res["t"] == pytest.approx(1.0, abs=1e-14)
    assert float(U[0]) == pytest.approx(1.0, abs=1e-12)          # rejected attempts left U alone
    assert sum(res["dts"]) == pytest.approx(1.0, abs=1e-12)
    assert len(res["dts"]) == res["accepted"]
    assert res["accepted"] + res["rejected"] == len(dev.attempts)
    assert res["rhs_evaluations"] == 4 * len(dev.attempts)
    assert all(dt <= dev.h * (1 + 1e-12) for dt in res["dts"])    # err <= 1 on every kept step


def test_settles_at_the_safety_fraction_of_the_largest_stable_step():
    dev = Clock(h=0.01)
    _, res = _run(dev, 0.5, dt0=0.01)
    # err = (dt/h)^3 and factor 0.9 err^(-1/3): every kept step after the first is 0.9 h
    inner = res["dts"][1:-1]
    assert inner and all(dt == pytest.approx(0.9 * dev.h, rel=1e-12) for dt in inner)
    assert res["rejected"] == 0


def test_rejections_shrink_by_at_most_five():
    dev = Clock(h=0.01)
    _, res = _run(dev, 1.0, dt0=0.1)
    # 0.1 -> err 1000, factor clipped to 0.2 -> 0.02 -> err 8, factor 0.45 -> 0.009 kept
    assert dev.attempts[:3] == pytest.approx([0.1, 0.02, 0.009], rel=1e-12)
    assert res["rejected"] == 2


def test_growth_is_capped_at_five_and_by_the_cfl_step():
    dev = Clock(h=1.0, err_zero=True)
    _, res = _run(dev, 10.0, dt0=1e-3, cfl_max=1.0)
    assert dev.attempts[:4] == pytest.approx([1e-3, 5e-3, 25e-3, 125e-3], rel=1e-12)
    dev = Clock(h=1.0, cfl=0.05, err_zero=True)
    _, res = _run(dev, 1.0, cfl_max=0.5)
    assert res["dts"][:-1] == pytest.approx([0.025] * (len(res["dts"]) - 1), rel=1e-12)
    assert res["accepted"] == 40


def test_max_steps_bounds_the_attempts():
    dev = Clock(h=1e-3)
    _, res = _run(dev, 1.0, dt0=1e-3, max_steps=7)
    assert len(dev.attempts) == 7 and res["t"] < 1.0


def test_on_step_sees_every_attempt():
    seen = []
    dev = Clock(h=0.01)
    _run(dev, 0.05, dt0=0.1, on_step=lambda t, a, r: seen.append((t, a, r)))
    assert len(seen) == len(dev.attempts)
    assert seen[0] == (0.0, 0, 1) and seen[-1][0] == pytest.approx(0.05, abs=1e-14)
