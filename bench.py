#!/usr/bin/env python3
"""Benchmark of the Fourier-domain slice pipeline on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Prints one JSON line.  The headline workload is prox_tnn with the full
per-slice SVD (Algorithm 3) on Y = P*Q + S + E, 200 x 200 x 50,
tau = 1/sqrt(200*50); a step is one tp_prox_tnn call on that tensor (FFT,
Jacobi SVD, shrinkage, two reconstruction products, inverse FFT), with the
input resident in HBM.  value = n1*n2*n3 / time per call, in Melem/s.

The same line reports tprod on the precision workload (A 512x512x128,
B 512x256x128) in FP32, split-BF16 (BF16X3) and BF16, in algorithmic
TFLOP/s (8 n1 n2 l flops per complex slice product, 2 n1 n2 l per real one).

Per-kernel times come from HIP events the library records around each of its
launches on the launch stream (tp_trace_enable), over the timed region.
The cpu_baseline leg times the FP64 oracle on the host cores and compares
the GPU results with it.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "prox_tnn Melem/s learned-rank vs full-SVD @rel.err≤1e-4; tprod TFLOP/s"
PEAK = {"hbm_GBs": 8000.0, "fp32_mfma_TF": 157.3, "bf16_mfma_TF": 2500.0, "valu_TF": 78.6}
KNAMES = {0: "rfft", 1: "irfft", 2: "cgemm", 3: "jacobi", 4: "shrink", 5: "tnn_reduce"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def tprod_flops(n1, n2, l, n3):
    h = n3 // 2 + 1
    nreal = 2 if n3 % 2 == 0 else 1
    return (8 * (h - nreal) + 2 * nreal) * n1 * n2 * l


def jacobi_sweep_flops(R, P, real):
    """Flops of one sweep of one-sided Jacobi over an R x P slice: per pair and
    row, alpha, beta and gamma (4 + 4 + 8 flops complex) and the two column
    updates (2 x 10); real slices 2 + 2 + 2 and 2 x 4."""
    per = 14 if real else 36
    return per * R * P * (P - 1) // 2


def collect(lib, cap=1 << 16):
    import ctypes
    ids = (ctypes.c_int * cap)()
    ms = (ctypes.c_float * cap)()
    n = lib.tp_trace_collect(ids, ms, cap)
    if n < 0:
        raise RuntimeError("tp_trace_collect failed")
    n = min(n, cap)
    out = {}
    for i in range(n):
        out.setdefault(KNAMES.get(ids[i], str(ids[i])), []).append(ms[i])
    return out


def timed(fn, steps, warmup, lib):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    collect(lib)
    lib.tp_trace_enable(1)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(steps):
        fn()
    stop.record()
    torch.cuda.synchronize()
    lib.tp_trace_enable(0)
    per_kernel = collect(lib)
    return start.elapsed_time(stop) / steps, per_kernel


def per_launch_ms(per_kernel, name, launches_per_step, steps):
    v = per_kernel.get(name, [])
    if not v:
        return None
    return float(np.sum(v)) / (steps * launches_per_step)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--tprod-steps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(this build has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1806_07247_amd as tp
    from paper_1806_07247_amd import _lib, inputs

    lib = _lib.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    # ---------------------------------------------------- prox full SVD --
    parts = inputs.prox_full_parts(seed=0)
    n1, n2, n3 = parts["S"].shape
    tau = float(parts["tau"])
    P = torch.from_numpy(parts["P"]).to(dev)
    Q = torch.from_numpy(parts["Q"]).to(dev)
    Y = (tp.tp_tprod(P, Q) + torch.from_numpy(parts["S"]).to(dev) + torch.from_numpy(parts["E"]).to(dev)).contiguous()
    h = n3 // 2 + 1
    X = torch.empty_like(Y)
    info = torch.zeros(h, dtype=torch.int32, device=dev)
    rank = torch.zeros(h, dtype=torch.int32, device=dev)
    ws = torch.empty(tp.tp_prox_tnn_workspace_size(n1, n2, n3), dtype=torch.uint8, device=dev)

    def prox_step():
        tp.tp_prox_tnn(Y, tau, out=X, info=info, rank=rank, workspace=ws)

    log(f"prox_tnn {n1}x{n2}x{n3} tau={tau:.4g}: warmup {args.warmup}, steps {args.steps}")
    ms, pk = timed(prox_step, args.steps, args.warmup, lib)
    sweeps = info.cpu().numpy()
    value = n1 * n2 * n3 / (ms * 1e-3) / 1e6
    R, Pc = max(n1, n2), min(n1, n2)
    jflops = sum(abs(int(s)) * jacobi_sweep_flops(R, Pc, k == 0 or (n3 % 2 == 0 and k == h - 1))
                 for k, s in enumerate(sweeps))
    jms = per_launch_ms(pk, "jacobi", 1, args.steps)
    stages = {}
    fft_in = n1 * n2 * n3 * 4
    fft_out = h * n1 * n2 * 8
    for name, nl, byts in (("rfft", 1, fft_in + fft_out), ("irfft", 1, fft_in + fft_out),
                           ("shrink", 1, 2 * h * n1 * n2 * 8 + h * Pc * 8)):
        t = per_launch_ms(pk, name, nl, args.steps)
        if t:
            stages[name] = {"ms": round(t, 5), "GB_s": round(byts / (t * 1e-3) / 1e9, 1),
                            "frac_hbm": round(byts / (t * 1e-3) / 1e9 / PEAK["hbm_GBs"], 4)}
    gemm_ms = per_launch_ms(pk, "cgemm", 2, args.steps)
    recon_flops = 2 * tprod_flops(n1, Pc, n2, n3) // 1  # two products, each ~ 8 n1 p n2 per complex slice
    if gemm_ms:
        stages["cgemm"] = {"ms_per_launch": round(gemm_ms, 5),
                           "TFLOP_s": round(recon_flops / 2 / (gemm_ms * 1e-3) / 1e12, 2)}
    stages["jacobi"] = {"ms": round(jms, 4), "sweeps": [int(s) for s in sweeps],
                        "GFLOP": round(jflops / 1e9, 3),
                        "TFLOP_s": round(jflops / (jms * 1e-3) / 1e12, 3)}
    roofline = {"kernel": "jacobi", "bound": "alu", "achieved": round(jflops / (jms * 1e-3) / 1e12, 3),
                "peak": PEAK["valu_TF"], "unit": "TFLOP/s",
                "frac": round(jflops / (jms * 1e-3) / 1e12 / PEAK["valu_TF"], 4), "traffic": None}
    log(f"  {ms:.4f} ms/step, {value:.1f} Melem/s, stages {json.dumps(stages)}")

    # --------------------------------------------------- tprod precision --
    A_np, B_np = inputs.tprod_precision(seed=0)
    A, B = torch.from_numpy(A_np).to(dev), torch.from_numpy(B_np).to(dev)
    tn1, tn2, tl, tn3 = A_np.shape[0], A_np.shape[1], B_np.shape[1], A_np.shape[2]
    flops = tprod_flops(tn1, tn2, tl, tn3)
    tws = torch.empty(tp.tp_tprod_workspace_size(tn1, tn2, tl, tn3), dtype=torch.uint8, device=dev)
    C = torch.empty((tn1, tl, tn3), dtype=torch.float32, device=dev)
    tprod = {"workload": f"A {tn1}x{tn2}x{tn3} * B {tn2}x{tl}x{tn3}, N(0,1)", "GFLOP": round(flops / 1e9, 3)}
    outs = {}
    for prec in ("fp32", "bf16x3", "bf16"):
        def tstep():
            tp.tp_tprod(A, B, prec=prec, out=C, workspace=tws)
        log(f"tprod {prec}")
        tms, tpk = timed(tstep, args.tprod_steps, 2, lib)
        g = per_launch_ms(tpk, "cgemm", 1, args.tprod_steps)
        peak = PEAK["fp32_mfma_TF"] if prec == "fp32" else PEAK["bf16_mfma_TF"]
        rf = per_launch_ms(tpk, "rfft", 2, args.tprod_steps)
        irf = per_launch_ms(tpk, "irfft", 1, args.tprod_steps)
        th = tn3 // 2 + 1
        rfft_bytes = ((tn1 * tn2 + tn2 * tl) * tn3 * 4 + th * (tn1 * tn2 + tn2 * tl) * 8) / 2
        irfft_bytes = tn1 * tl * tn3 * 4 + th * tn1 * tl * 8
        tprod[prec] = {"ms": round(tms, 4), "TFLOP_s": round(flops / (tms * 1e-3) / 1e12, 2),
                       "cgemm_ms": round(g, 4), "cgemm_TFLOP_s": round(flops / (g * 1e-3) / 1e12, 2),
                       "cgemm_frac_peak": round(flops / (g * 1e-3) / 1e12 / peak, 4),
                       "rfft_GB_s": round(rfft_bytes / (rf * 1e-3) / 1e9, 1),
                       "irfft_GB_s": round(irfft_bytes / (irf * 1e-3) / 1e9, 1)}
        outs[prec] = C.cpu().numpy()
        log(f"  {json.dumps(tprod[prec])}")

    # ------------------------------------------------------ cpu baseline --
    cpu = None
    parity = {}
    if not args.no_cpu_baseline:
        import oracle
        nthr = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or min(16, os.cpu_count() or 1)
        oracle.set_threads(nthr)
        Ln = oracle.tprod(parts["P"], parts["Q"])
        Yn = (Ln + parts["S"] + parts["E"]).astype(np.float32)
        calls, t0 = 0, time.perf_counter()
        while True:
            Xref = oracle.prox_tnn(Yn, np.float32(tau))
            calls += 1
            el = time.perf_counter() - t0
            if el >= args.cpu_seconds or calls >= 20:
                break
        cpu = {"value": round(n1 * n2 * n3 * calls / el / 1e6, 4), "unit": "Melem/s",
               "cores": oracle.get_threads(), "kind": "oracle",
               "sample": f"{calls} full prox_tnn call(s) on the same {n1}x{n2}x{n3} workload (FP64, "
                         f"Y composed by the oracle's t-product), {el:.1f} s"}
        # parity at full size: the GPU input Y was composed on the GPU; the
        # comparison uses the GPU prox of the oracle-composed Y
        Xg = tp.tp_prox_tnn(torch.from_numpy(Yn).to(dev), tau).cpu().numpy()
        parity["prox_full_rel_err"] = float(np.linalg.norm(Xg - Xref) / np.linalg.norm(Xref))
        rng = np.random.default_rng(1)
        idx = rng.choice(tn1 * tl * tn3, size=4000, replace=False)
        ref = oracle.tprod_entries(A_np, B_np, idx)
        for prec, Cn in outs.items():
            parity[f"tprod_{prec}_sampled_rel_err"] = float(
                np.linalg.norm(Cn.reshape(-1)[idx] - ref) / np.linalg.norm(ref))
        log(f"cpu baseline {cpu}, parity {parity}")

    line = {
        "metric": METRIC, "value": round(value, 3), "unit": "Melem/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"prox_tnn full-SVD, Y = P*Q + S + E {n1}x{n2}x{n3}, tau = 1/sqrt({n1}*{n3})",
                   "n1": n1, "n2": n2, "n3": n3, "tau": tau, "parallelism": "single GPU"},
        "roofline": roofline, "cpu_baseline": cpu, "stages": stages, "tprod": tprod, "parity": parity,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
