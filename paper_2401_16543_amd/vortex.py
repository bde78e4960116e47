"""The isentropic vortex convergence study of section 6.1 (Table 1) on one GPU.

    python -m paper_2401_16543_amd.vortex [--R 2] [--n 32 64 128 256]
                                          [--scheme linear|weno|kxrcf|gate] [--tol 1e-9]
                                          [--precision fp64|split_f16|split_bf16] [--ell 5]

The vortex on the periodic [-10, 10]^2 returns to its initial position at
t = 20; the L1 density error is the mean |rho(20) - rho(0)| over the cell
averages.  Time steps: SSP(4,3,2) with error-based control (atol = rtol = tol)
and the CFL number capped at 1.  The scheme: the linear S0 reconstruction
everywhere (as the paper's table), WENO-AO everywhere, the KXRCF two-pass
reconstruction, or the learned troubled-cell gate (split precision only; the
committed 2D network).  Prints one JSON line with the errors, the observed
orders and, for the indicator and the gate, the fraction of (cell, variable)
pairs the last reconstruction sent to WENO-AO.
"""
from __future__ import annotations

import argparse
import json
import math
import time


def run(R: int = 2, ns=(32, 64, 128, 256), scheme: str = "linear", tol: float = 1e-9,
        precision: str = "fp64", ell_hat: float = 5.0, periods: int = 1) -> dict:
    """The study at each n in ns; `periods` vortex periods (t = 20 each), the
    error taken against the initial state, which every period returns to."""
    import torch

    from . import inputs, kfvm
    from .integrate import integrate
    gamma = 1.4
    spec = inputs.isentropic_vortex(gamma)
    rows = []
    for n in ns:
        U0 = inputs.cell_averages(spec, n, gamma, rule="gauss", q=4).cuda()
        dev = kfvm.KFVM(2, (n, n), dx=[20.0 / n] * 2, order=2 * R + 1, gamma=gamma, ell_hat=ell_hat)
        dev.set_precision(precision)
        if scheme == "linear":
            dev.set_flags(torch.zeros((4, n * n), dtype=torch.uint8, device="cuda"))
        elif scheme == "kxrcf":
            dev.set_indicator("kxrcf", 1.5)
        elif scheme == "gate":
            if precision == "fp64":
                raise ValueError("the learned gate runs on the split-precision paths")
            from . import gate
            params, thr, _ = gate.load(2)
            dev.set_gate(torch.from_numpy(params).cuda(), thr)
        U = U0.clone()
        t0 = time.perf_counter()
        res = integrate(dev, U, 20.0 * periods, atol=tol, rtol=tol, cfl_max=1.0)
        torch.cuda.synchronize()
        err = float((U[0] - U0[0]).abs().mean())
        row = dict(n=n, l1_rho=err, accepted=res["accepted"], rejected=res["rejected"],
                   wall_s=time.perf_counter() - t0)
        if scheme in ("kxrcf", "gate"):
            st = dev.stats()
            row["weno_fraction"] = st["weno_cell_vars"] / st["cell_vars"]
        rows.append(row)
        dev.close()
    for a, b in zip(rows, rows[1:]):
        b["eoc"] = math.log(a["l1_rho"] / b["l1_rho"], 2)
    return {"problem": f"isentropic vortex, t = {20 * periods}", "R": R, "scheme": scheme, "tol": tol,
            "precision": precision, "ell_hat": ell_hat, "results": rows}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--R", type=int, default=2)
    ap.add_argument("--n", type=int, nargs="+", default=[32, 64, 128, 256])
    ap.add_argument("--scheme", default="linear", choices=["linear", "weno", "kxrcf", "gate"])
    ap.add_argument("--tol", type=float, default=1e-9)
    ap.add_argument("--precision", default=None, choices=["fp64", "split_f16", "split_bf16"],
                    help="default fp64, split_f16 for the gate")
    ap.add_argument("--ell", type=float, default=5.0, help="kernel length scale in cells (the paper's 5)")
    a = ap.parse_args()
    precision = a.precision or ("split_f16" if a.scheme == "gate" else "fp64")
    print(json.dumps(run(a.R, a.n, a.scheme, a.tol, precision, a.ell)), flush=True)


if __name__ == "__main__":
    main()
