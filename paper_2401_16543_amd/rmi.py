"""The Richtmyer-Meshkov run of section 6.3 on one GPU through the library.

    python -m paper_2401_16543_amd.rmi [--R 2] [--cells-per-unit 512] [--t-end 3.33]
                                       [--integrator ssp3|ssp432] [--cfl 0.5] [--cfl-form sum]
                                       [--tol 1e-3] [--no-indicator] [--flattener K1]
                                       [--precision fp64] [--compare-fp64]

Domain [-1/2, 11/2] x [0, 1] at spacing 1/512 (3072 x 512 cells), Mach-3 shock
into an oblique density jump (rho_D = 2), fixed inflow at x = -1/2, outflow at
x = 11/2, reflecting walls in y; any precision path, with or without the KXRCF
two-pass reconstruction (m = 3/2) and the limiter's flattener.  Time stepping:
SSP-RK3 at a fixed CFL number, or the paper's choice for this run, SSP(4,3,2)
with error-based step control (atol = rtol = 1e-3, CFL at most 1).  Prints a
progress line every few hundred steps and one JSON summary: right-hand-side
evaluations, wall time per evaluation, device time per kernel class, and the
fraction of cells the indicator flags at the end.
"""
from __future__ import annotations

import argparse
import json
import sys
import time


def run(R: int = 2, cells_per_unit: int = 512, t_end: float = 3.33, cfl: float = 0.5, indicator: bool = True,
        report_every: int = 500, max_steps: int | None = None, precision: str = "fp64", keep_state: bool = False,
        dts=None, integrator: str = "ssp3", tol: float = 1e-3, flattener: float | None = None,
        cfl_form: str = "sum") -> dict:
    """One run; `dts` replays a recorded sequence of SSP-RK3 step sizes (the
    summary's "dts" when keep_state is set: the step sizes taken, accepted ones
    for ssp432) so that two runs can be compared state for state.  integrator
    "ssp432" takes atol = rtol = tol and cfl as the largest CFL number."""
    import torch

    from . import inputs, kfvm
    U, m = inputs.rmi(R, cells_per_unit, device="cuda")
    U = U.contiguous()
    nx, ny = m["n"]
    dev = kfvm.KFVM(2, (nx, ny), dx=[m["dx"]] * 2, order=2 * R + 1, gamma=inputs.RMI_GAMMA)
    dev.set_boundary(0, "inflow", "outflow", lower_state=m["inflow"])
    dev.set_boundary(1, "reflecting", "reflecting")
    dev.set_precision(precision)
    if indicator:
        dev.set_indicator("kxrcf", 1.5)
    if flattener:
        dev.set_flattener(flattener)
    dev.set_cfl_form(cfl_form)
    dev.set_timing(True)
    dev.kernel_times()
    torch.cuda.synchronize()
    t, steps = 0.0, 0
    totals = {}

    def collect():
        # the recorded events are summed and released at every report
        for k, (ms, _) in dev.kernel_times().items():
            totals[k] = totals.get(k, 0.0) + ms

    taken = []
    t0 = time.perf_counter()
    if integrator == "ssp432":
        from .integrate import integrate

        def on_step(tt, acc, rej):
            if (acc + rej) % report_every == 0:
                collect()
                print(f"# attempt {acc + rej} ({rej} rejected) t={tt:.4f} wall {time.perf_counter() - t0:.1f} s",
                      file=sys.stderr, flush=True)

        res = integrate(dev, U, t_end, atol=tol, rtol=tol, cfl_max=cfl,
                        max_steps=max_steps if max_steps is not None else 10 ** 7, on_step=on_step)
        t, steps = res["t"], res["accepted"] + res["rejected"]
        taken = res["dts"]
    while integrator == "ssp3" and t < t_end - 1e-12 and (max_steps is None or steps < max_steps):
        if dts is not None:
            if steps >= len(dts):
                break
            dt = dts[steps]
        else:
            dt = min(dev.cfl_dt(U, cfl), t_end - t)
        taken.append(dt)
        dev.step(U, dt)
        t += dt
        steps += 1
        if steps % report_every == 0:
            collect()
            print(f"# step {steps} t={t:.4f} wall {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    status = dev.status()
    collect()
    flagged = float(dev.get_flags()[0].float().mean()) if indicator else 1.0
    nrhs = (4 if integrator == "ssp432" else 3) * steps
    out = {"problem": "Richtmyer-Meshkov, Ma 3, rho_D 2", "R": R, "grid": [nx, ny], "t": t, "steps": steps,
            "precision": precision, "integrator": integrator, "flattener_k1": flattener, "cfl_form": cfl_form,
            "rhs_evaluations": nrhs, "cfl": cfl, "indicator": "KXRCF m=3/2" if indicator else "none (WENO-AO everywhere)",
            "wall_s": wall, "wall_ms_per_rhs": wall / nrhs * 1e3,
            "device_ms_total": totals,
            "flagged_fraction_final": flagged, "status": status,
            "rho_range": [float(U[0].min()), float(U[0].max())]}
    if integrator == "ssp432":
        out.update(tol=tol, accepted=res["accepted"], rejected=res["rejected"])
    if keep_state:
        out["U"] = U
        out["dts"] = taken
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--R", type=int, default=2)
    ap.add_argument("--cells-per-unit", type=int, default=512)
    ap.add_argument("--t-end", type=float, default=3.33)
    ap.add_argument("--integrator", default="ssp3", choices=["ssp3", "ssp432"])
    ap.add_argument("--cfl", type=float, default=None, help="CFL number (ssp3, default 0.5) or its cap (ssp432, default 1)")
    ap.add_argument("--tol", type=float, default=1e-3, help="ssp432: atol = rtol")
    ap.add_argument("--cfl-form", default="sum", choices=["sum", "max_axis"],
                    help="CFL step from the sum over axes of (|u|+c)/dx (default) or its largest term")
    ap.add_argument("--flattener", type=float, default=None, help="the limiter flattener's onset k1 (default off)")
    ap.add_argument("--no-indicator", action="store_true")
    ap.add_argument("--max-steps", type=int, default=None)
    ap.add_argument("--precision", default="fp64", help="fp64, split_f16 or split_bf16")
    ap.add_argument("--compare-fp64", action="store_true",
                    help="also run the FP64 path with the same step sizes and report the L1 density difference")
    a = ap.parse_args()
    cfl = a.cfl if a.cfl is not None else (1.0 if a.integrator == "ssp432" else 0.5)
    if a.compare_fp64 and a.integrator != "ssp3":
        ap.error("--compare-fp64 replays SSP-RK3 step sizes: use --integrator ssp3")
    out = run(a.R, a.cells_per_unit, a.t_end, cfl, not a.no_indicator, max_steps=a.max_steps,
              precision=a.precision, keep_state=a.compare_fp64, integrator=a.integrator, tol=a.tol,
              flattener=a.flattener, cfl_form=a.cfl_form)
    if a.compare_fp64:
        ref = run(a.R, a.cells_per_unit, a.t_end, cfl, not a.no_indicator, precision="fp64", keep_state=True,
                  dts=out["dts"], flattener=a.flattener, cfl_form=a.cfl_form)
        out["l1_rho_vs_fp64"] = float((out["U"][0] - ref["U"][0]).abs().mean())
        out["fp64_wall_ms_per_rhs"] = ref["wall_ms_per_rhs"]
        out.pop("U")
        out.pop("dts")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
