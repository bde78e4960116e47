"""Error-controlled time integration with SSP(4,3,2) (section 6) on the library.

The library computes each step and the norm of its embedded error estimate on
the GPU (kfvm_step_ssp432); this driver accepts or rejects the step and picks
the next step size: dt <- dt * clamp(0.9 * err^(-1/3), 0.2, 5) (the estimate is
the local error of the embedded second-order method, O(dt^3)), never above the
CFL limit cfl_max * dt_CFL.  The paper cites its controller; this elementary
one is the reading used here.
"""
from __future__ import annotations


def integrate(dev, U, t_end: float, atol: float = 1e-6, rtol: float = 1e-6, cfl_max: float = 1.0,
              dt0: float | None = None, max_steps: int = 10 ** 7, on_step=None) -> dict:
    """Advance U (a device tensor, updated in place) from 0 to t_end.  Returns the
    counts of accepted and rejected steps and of right-hand-side evaluations, and
    the accepted step sizes ("dts").  on_step(t, accepted, rejected), if given,
    is called after every attempt."""
    import torch
    out = torch.empty_like(U)
    t, accepted, rejected = 0.0, 0, 0
    dts = []
    dt = dt0 if dt0 is not None else dev.cfl_dt(U, cfl_max)
    while t < t_end - 1e-14 * max(1.0, t_end) and accepted + rejected < max_steps:
        dt = min(dt, dev.cfl_dt(U, cfl_max), t_end - t)
        err = dev.step_ssp432(U, out, dt, atol, rtol)
        if err <= 1.0:
            U.copy_(out)
            t += dt
            accepted += 1
            dts.append(dt)
        else:
            rejected += 1
        if on_step is not None:
            on_step(t, accepted, rejected)
        fac = 5.0 if err == 0.0 else min(5.0, max(0.2, 0.9 * err ** (-1.0 / 3.0)))
        dt *= fac
    return {"t": t, "accepted": accepted, "rejected": rejected, "rhs_evaluations": 4 * (accepted + rejected),
            "dts": dts}
