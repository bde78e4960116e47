#!/usr/bin/env python3
"""Throughput of the KFVM-WENO right-hand side on one MI355X.

A step is one SSP-RK3 step (three right-hand-side evaluations, each the
reconstruction, face-flux and update kernels) over the whole grid of the
workload, with the state already resident in HBM.  The metric is cell-updates
per second per Runge-Kutta stage: cells * 3 * steps / elapsed.

Prints one JSON line.  The headline `value` is the split-precision path with
the learned gate; the plain FP64 path, the ungated split path and the FP64 path
driven by the paper's KXRCF indicator (the two-pass reconstruction) are timed
beside it on the same state and step.  `roofline` covers the dominant kernel of
each: algorithmic bytes (or FP64 flops) per launch over its average launch time,
measured with HIP events on the library's stream over the timed steps.
`cpu_baseline` times the FP64 CPU oracle on a bounded periodic sub-box of the
same initial state (rank 0, N = 1).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

METRIC = "cell-updates/sec per RK stage, plain FP64 vs mixed+learned at stated L1 error"
FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 vector peak
HBM_PEAK_GBS = 8000.0
MFMA_F16_PEAK_TFLOPS = 2500.0   # MI355X dense fp16 / bf16 matrix-core peak
VALU_ISSUE_PEAK_G = 256 * 4 * 2.4 / 4   # wave64 VALU instructions per ns: 256 CUs x 4 SIMDs, one per 4 cycles

# (sum of N_q over the stencils, face points, derivative rows, stencils, |S0|)
_SHAPES = {(2, 2): (38, 8, 5, 6, 13), (2, 3): (82, 12, 9, 6, 29),
           (3, 2): (106, 24, 9, 8, 33), (3, 3): (348, 54, 19, 8, 123)}


def recon_flops_per_cell(d: int, R: int) -> int:
    """Algorithmic FP64 flops of the reconstruction kernel per cell (FMA = 2):
    per variable the dot products of every stencil row with its gathered values,
    the squared-derivative sums, the nonlinear weights and the WENO-AO blend;
    plus the linearised-primitive transform of the S0 values."""
    sn, npts, nder, nst, n0 = _SHAPES[(d, R)]
    nv = d + 2
    per_var = 2 * (npts + nder) * sn + 2 * nder * nst + 5 * nst + 2 * npts * nst
    return nv * per_var + n0 * (5 * d + 3)


def state_bytes_per_cell(d: int) -> int:
    """Algorithmic HBM bytes per cell and Runge-Kutta stage: the minimum state
    traffic of a stage, the stage's input average and the step's initial average
    read and the new average written, float64 each.  Face states, limiter
    factors, face fluxes and halo re-reads are implementation traffic."""
    return 3 * 8 * (d + 2)


def contraction_flops_per_cell(d: int, R: int) -> int:
    """Algorithmic flops of the weight-apply and smoothness-indicator contraction
    per cell (FMA = 2): every row (face points and derivatives) of every stencil
    against that stencil's gathered values, per variable."""
    sn, npts, nder, _, _ = _SHAPES[(d, R)]
    return 2 * sn * (npts + nder) * (d + 2)


# sources a kernel is built from: a profile's counters stand only while these are unchanged
_KERNEL_SOURCES = {
    "k_recon_mixed": ["rhs_mixed.hip", "device_common.hpp", "stencil.hpp", "kernels.hpp"],
    "k_recon": ["rhs_fp64.hip", "device_common.hpp", "stencil.hpp", "kernels.hpp"],
    "k_kxrcf_jump": ["kxrcf.hip", "device_common.hpp", "stencil.hpp", "kernels.hpp"],
}


def sources_digest(kernel: str) -> str:
    import hashlib
    h = hashlib.sha256()
    base = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2401_16543_amd", "csrc")
    for f in _KERNEL_SOURCES[kernel]:
        with open(os.path.join(base, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary of this
    kernel and workload, or None when there is none or its sources changed since."""
    import re
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", f"{kernel}_{workload}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    dg = re.search(r"sources digest: `([0-9a-f]+)`", text)
    tb = re.search(r"traffic bytes per launch: `([0-9.eE+]+)`", text)
    if not dg or not tb or dg.group(1) != sources_digest(kernel):
        return None
    return float(tb.group(1))


def profiled_figure(kernel: str, workload: str, label: str):
    """A per-launch figure ("VALU instructions per wave", "waves per launch") from
    the committed rocprofv3 summary of this kernel and workload, or None when
    there is none or its sources changed since."""
    import re
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", f"{kernel}_{workload}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    dg = re.search(r"sources digest: `([0-9a-f]+)`", text)
    m = re.search(re.escape(label) + r": `([0-9.eE+]+)`", text)
    if not dg or not m or dg.group(1) != sources_digest(kernel):
        return None
    return float(m.group(1))


def cpu_baseline(U_host, cfg, budget_s: float):
    """Time the oracle's whole-grid RHS on a periodic sub-box of the same state."""
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from oracle import core
    d, R, gamma = cfg["d"], cfg["R"], cfg["gamma"]
    core.build()
    threads = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))

    def run(m):
        sl = (slice(None),) + (slice(0, m),) * d
        Us = U_host[sl].copy()
        o = core.Oracle(d, R, (m,) * d, dx=[1.0 / cfg["n"]] * d, gamma=gamma)
        t = time.perf_counter()
        o.rhs(Us)
        return time.perf_counter() - t

    m = 16 if d == 3 else 64
    t = run(m)
    # grow the box until one RHS takes about a third of the budget
    while t < budget_s / 3 and m < cfg["n"]:
        grow = min(2.0, max(1.2, (budget_s / 3 / max(t, 1e-3)) ** (1.0 / d)))
        m = min(cfg["n"], int(m * grow))
        t = run(m)
    cells = m ** d
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": cells / t, "unit": "cell-updates/s", "cores": threads, "kind": "oracle", "cpu_model": model,
            "sample": f"one whole-grid RHS (one RK stage) of the FP64 oracle on the periodic "
                      f"{'x'.join([str(m)] * d)} corner sub-box of the {cfg['n']}^{d} initial state, "
                      f"{t:.2f} s"}


def kxrcf_flops_per_cell(d: int, R: int) -> int:
    """Algorithmic FP64 flops of the KXRCF jump kernel per cell (FMA = 2): per axis
    the unlimited states of both sides of the upper face at its Gauss points, one
    dot product of length |S0| per (side, point, variable).  The entropies (a few
    dozen flops per point) are not counted."""
    _, npts, _, _, n0 = _SHAPES[(d, R)]
    return 2 * npts * (d + 2) * n0        # 2 D sides x points per face = n_pts dot products per variable


def _time_path(dev, U0, dt, steps, warmup, mode, kfvm, torch, gate=None, indicator=None):
    """Warm up on a scratch copy, then time `steps` SSP-RK3 steps from U0."""
    dev.set_precision(mode)
    if gate is None:
        dev.set_gate(None)
    else:
        dev.set_gate(torch.from_numpy(gate[0]).cuda(), gate[1])
    dev.set_indicator(indicator)
    Uw = U0.clone()
    for _ in range(warmup):
        dev.step(Uw, dt)
    del Uw
    torch.cuda.synchronize()
    if dev.status() != kfvm.KFVM_OK:
        raise SystemExit(f"non-physical state during warm-up ({mode})")
    U = U0.clone()
    dev.set_timing(True)
    dev.kernel_times()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        dev.step(U, dt)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kt = dev.kernel_times()
    dev.set_timing(False)
    if dev.status() != kfvm.KFVM_OK:
        raise SystemExit(f"non-physical state during the timed steps ({mode})")
    return U, elapsed, kt


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="3d_smooth_256")
    ap.add_argument("--mixed", default="split_f16", help="split_f16 or split_bf16")
    ap.add_argument("--cpu-seconds", type=float, default=30.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run one device copy of 1 GiB (read 1 GiB, write 1 GiB) to scale HBM counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported "
              f"(the path would shard by spatial domain; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2401_16543_amd import inputs, kfvm

    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = src.clone()
        torch.cuda.synchronize()
        print("# copy calibration: 1073741824 bytes read, 1073741824 bytes written", file=sys.stderr, flush=True)
        del src, dst
    U0, cfg = inputs.config_state(args.workload, device="cuda")
    d, n, R, gamma = cfg["d"], cfg["n"], cfg["R"], cfg["gamma"]
    ncell = n ** d
    print(f"# workload {args.workload}: {n}^{d} cells, R={R}, gamma={gamma:.4f}", file=sys.stderr, flush=True)
    dev = kfvm.KFVM(d, (n,) * d, order=2 * R + 1, gamma=gamma)
    dt = dev.cfl_dt(U0, cfg["cfl"])
    stages = 3 * args.steps

    U_plain, t_plain, kt_plain = _time_path(dev, U0, dt, args.steps, args.warmup, "fp64", kfvm, torch)
    print(f"# plain fp64: {t_plain / args.steps * 1e3:.2f} ms/step", file=sys.stderr, flush=True)
    U_kx, t_kx, kt_kx = _time_path(dev, U0, dt, args.steps, args.warmup, "fp64", kfvm, torch, indicator="kxrcf")
    kx_flagged = float(dev.get_flags().float().mean())
    print(f"# fp64 + KXRCF two-pass: {t_kx / args.steps * 1e3:.2f} ms/step, flagged {kx_flagged:.4f}",
          file=sys.stderr, flush=True)
    l1_kx = float((U_kx[0] - U_plain[0]).abs().mean())
    del U_kx
    U_ung, t_ung, kt_ung = _time_path(dev, U0, dt, args.steps, args.warmup, args.mixed, kfvm, torch)
    print(f"# {args.mixed}: {t_ung / args.steps * 1e3:.2f} ms/step", file=sys.stderr, flush=True)
    l1_ung = float((U_ung[0] - U_plain[0]).abs().mean())
    del U_ung
    from paper_2401_16543_amd import gate as gate_mod
    gp, thr, gmeta = gate_mod.load(d)
    U_mix, t_mix, kt_mix = _time_path(dev, U0, dt, args.steps, args.warmup, args.mixed, kfvm, torch, (gp, thr))
    flagged = float(dev.get_flags().float().mean())
    print(f"# {args.mixed} + learned gate: {t_mix / args.steps * 1e3:.2f} ms/step, flagged {flagged:.4f}",
          file=sys.stderr, flush=True)
    l1 = float((U_mix[0] - U_plain[0]).abs().mean())
    # misclassification of the gate's decisions on the final state against the
    # WENO-AO labels of the FP64 reconstruction (troubled iff 1 - omega_0/gamma_0 > cut)
    dev.rhs(U_mix)
    dec = dev.get_flags().bool()
    _, ratio = dev.gate_samples(U_mix, inputs=False)
    troubled = (1.0 - ratio) > gate_mod.LABEL_CUT
    n_tr = int(troubled.sum())
    mis = {"false_smooth": float((troubled & ~dec).sum()) / max(1, n_tr),
           "false_troubled": float((~troubled & dec).sum()) / max(1, int((~troubled).sum())),
           "labelled_troubled": n_tr / troubled.numel(), "flagged": float(dec.float().mean()),
           "note": f"decisions of the gated run's last state against the labels of its FP64 WENO-AO "
                   f"reconstruction (troubled iff 1 - omega_0/gamma_0 > {gate_mod.LABEL_CUT})"}
    del dec, ratio, troubled
    # the same decisions replayed on the FP64 path: the precision part of l1
    from paper_2401_16543_amd.accuracy import replay_l1
    plain = kfvm.KFVM(d, (n,) * d, order=2 * R + 1, gamma=gamma)
    l1_same, _ = replay_l1(dev, plain, U0, [dt] * args.steps)
    plain.close()
    print(f"# gated, same decisions replayed in FP64: L1 rho {l1_same:.3e}", file=sys.stderr, flush=True)

    def roof(kt):
        ms, nl = kt["recon"]
        avg = ms / nl / 1e3
        ach = recon_flops_per_cell(d, R) * ncell / avg / 1e12
        tr = profiled_traffic("k_recon", args.workload)
        return {"kernel": "k_recon", "bound": "alu", "achieved": ach, "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": ach / FP64_PEAK_TFLOPS, "traffic": tr,
                "traffic_ratio": tr / (sbytes * ncell) if tr else None,
                "flops_per_cell": recon_flops_per_cell(d, R), "alg_bytes_per_cell": sbytes,
                "hbm_achieved_gbs": sbytes * ncell / avg / 1e9,
                "hbm_frac": sbytes * ncell / avg / 1e9 / HBM_PEAK_GBS, "avg_launch_ms": avg * 1e3}

    def kx_roof(kt):
        ms, nl = kt["indicator"]
        avg = ms / nl / 1e3
        ach = kxrcf_flops_per_cell(d, R) * ncell / avg / 1e12
        return {"kernel": "k_kxrcf_jump (+ k_kxrcf_flags)", "bound": "alu", "achieved": ach,
                "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": ach / FP64_PEAK_TFLOPS,
                "traffic": profiled_traffic("k_kxrcf_jump", args.workload),
                "flops_per_cell": kxrcf_flops_per_cell(d, R), "avg_launch_ms": avg * 1e3}

    per_launch = lambda kt: {k: (v[0] / v[1] if v[1] else None) for k, v in kt.items()}
    mix_ms, mix_n = kt_mix["recon"]
    mix_avg = mix_ms / mix_n / 1e3
    sbytes = state_bytes_per_cell(d)
    cflops = contraction_flops_per_cell(d, R)
    mix_traffic = profiled_traffic("k_recon_mixed", args.workload)
    # VALU issue of the headline kernel, the unit that bounds it: counter
    # figures (rocprofv3 SQ_INSTS_VALU per wave, SQ_WAVES) over the live launch
    # time, against one wave64 VALU instruction per 4 cycles per SIMD (16 lanes
    # a cycle) on 1,024 SIMDs at 2.4 GHz
    vpw = profiled_figure("k_recon_mixed", args.workload, "VALU instructions per wave")
    wpl = profiled_figure("k_recon_mixed", args.workload, "waves per launch")
    valu = None
    if vpw and wpl:
        got = vpw * wpl / mix_avg / 1e9
        valu = {"achieved": got, "peak": VALU_ISSUE_PEAK_G, "unit": "G wave-instructions/s",
                "frac": got / VALU_ISSUE_PEAK_G, "valu_per_wave": vpw, "waves_per_launch": wpl}
    out = {
        "metric": METRIC, "value": ncell * stages / t_mix, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": t_mix / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": ("f16" if args.mixed == "split_f16" else "bf16") + " hi/lo MFMA, f32 acc, f64 epilogue; bf16 gate",
        "data": "synthetic",
        "config": {"workload": args.workload, "grid": [n] * d, "R": R, "order": 2 * R + 1,
                   "gamma": gamma, "cfl": cfg["cfl"], "dt": dt, "path": args.mixed, "riemann": "hllc",
                   "limiter": "on, kappa=0.5",
                   "gate": f"learned ({gmeta['samples']} training samples, threshold {thr:.4f}, "
                           f"held-out false-smooth {gmeta['val_false_smooth']:.4f})"},
        "gate_flagged_fraction": flagged,
        "gate_misclassification": mis,
        "l1_rho_vs_fp64": l1,
        "l1_rho_vs_fp64_ungated": l1_ung,
        "l1_rho_vs_fp64_same_decisions": l1_same,
        "l1_note": f"mean |rho - rho_fp64| after {args.steps} steps from the same state and dt (the FP64 GPU "
                   f"path matches the CPU oracle to ~1e-15); ungated = split precision with WENO-AO everywhere; "
                   f"same_decisions = the gated run against the FP64 path replaying its decisions at every "
                   f"stage (the precision error alone); l1_rho_vs_fp64 - that = the gate-induced difference",
        "roofline": {"kernel": "k_recon_mixed", "bound": "mfma", "achieved": cflops * ncell / mix_avg / 1e12,
                     "peak": MFMA_F16_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": cflops * ncell / mix_avg / 1e12 / MFMA_F16_PEAK_TFLOPS,
                     "traffic": mix_traffic,
                     "traffic_ratio": mix_traffic / (sbytes * ncell) if mix_traffic else None,
                     "flops_per_cell": cflops, "alg_bytes_per_cell": sbytes, "avg_launch_ms": mix_avg * 1e3,
                     "valu_issue": valu,
                     "hbm_achieved_gbs": sbytes * ncell / mix_avg / 1e9,
                     "hbm_frac": sbytes * ncell / mix_avg / 1e9 / HBM_PEAK_GBS,
                     "note": "achieved = the sparse weight-apply and smoothness-indicator contraction (every "
                             "stencil row, every variable, no hi/lo split) per launch over the mean launch time, "
                             "against the dense fp16 matrix-core peak; hbm_* = the stage's state traffic "
                             "(3 float64 averages per variable) over the same time; traffic = measured HBM bytes "
                             "per launch (rocprofv3 counters), traffic_ratio = traffic / state bytes; "
                             "valu_issue = VALU wave-instructions issued per second (SQ_INSTS_VALU per wave x "
                             "waves per launch from the same counter summary, over the mean launch time) against "
                             "1,024 SIMDs issuing one every 4 cycles at 2.4 GHz: the unit that bounds this kernel"},
        "kernels_ms_per_launch": per_launch(kt_mix),
        "plain_fp64": {"value": ncell * stages / t_plain, "ms_per_step": t_plain / args.steps * 1e3,
                       "dtype": "f64", "roofline": roof(kt_plain), "kernels_ms_per_launch": per_launch(kt_plain)},
        "mixed_ungated": {"value": ncell * stages / t_ung, "ms_per_step": t_ung / args.steps * 1e3,
                          "kernels_ms_per_launch": per_launch(kt_ung)},
        "fp64_kxrcf": {"value": ncell * stages / t_kx, "ms_per_step": t_kx / args.steps * 1e3, "dtype": "f64",
                       "indicator": "KXRCF two-pass, m = 3/2", "flagged_fraction": kx_flagged,
                       "l1_rho_vs_fp64_weno_everywhere": l1_kx,
                       "roofline": kx_roof(kt_kx), "kernels_ms_per_launch": per_launch(kt_kx)},
        "speedup_vs_plain_fp64": t_plain / t_mix,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(U0.cpu().numpy(), cfg, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
