"""Benchmark: received symbols/s of the demapping path on one MI355X.

Workload (the metric's configuration): 8D constellation with M = 2048 Gaussian
points (unit energy per 2D, binary-index labels), N = 1e7 received symbols per SNR
point, 11 SNR points 4..14 dB.  One step is one pass of the whole path over that
sweep: for every SNR point awgn_sample (channel draw into resident HBM buffers),
llr_exact (label-order prep + fused score/exp/subset-sum kernel + fallback) and
gmi_reduce.  value = 11 * N received symbols per step / step time.

Prints one JSON line.  Extra objects:
  roofline      the dominant kernel (the llr_exact launch) against the
                transcendental (exp) throughput of the chip, timed with HIP events
                on the stream the kernels run on;
  cpu_baseline  the FP64 oracle on a bounded sample of the same workload, timed on
                this host's cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "received symbols/s for exact LLR+GMI (8D, M=2048) and learned-vs-exact at ≤0.01b"
# Transcendental issue rate: 256 CUs x 2.4 GHz x 32 exp lanes per clock per CU
# (a quarter of the 128 FP32 VALU lanes per clock per CU).
EXP_PEAK = 256 * 2.4e9 * 32


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=10_000_000, help="received symbols per SNR point")
    ap.add_argument("--prec", default="fp32", choices=["fp32", "bf16"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target duration of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain device copy of known size (HBM counter calibration)")
    return ap.parse_args()


def cpu_baseline(X, labels, snr_db, seconds):
    import numpy as np
    import oracle
    import synth
    s2 = synth.sigma2_from_snr_db(X, snr_db)

    def run(n):
        tx, y = oracle.awgn(X, 99, 0, n, math.sqrt(s2))
        t0 = time.perf_counter()
        L = oracle.llr_exact(X, labels, y, s2)
        oracle.gmi(L, tx, labels)
        return time.perf_counter() - t0

    n0 = 2000
    dt0 = run(n0)
    n = int(min(2_000_000, max(n0, n0 * seconds / max(dt0, 1e-6))))
    dt = run(n)
    return {"value": n / dt, "unit": "symbols/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{n} symbols of the 8D M=2048 workload at {snr_db:g} dB (exact LLR + GMI, FP64, "
                      f"{dt:.1f} s)"}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the demapping path is measured on a single MI355X "
              "(multi-GPU sharding is a design note, not part of this build)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2104_06311_amd as md
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    wl = synth.workload_8d2048(N=args.n)
    X = torch.from_numpy(wl.X).to(dev)
    labels = torch.from_numpy(wl.labels.astype(np.int32)).to(dev)
    N, M, D, m = wl.N, wl.M, wl.D, wl.m
    snrs = wl.snr_db
    sig2 = [wl.sigma2(s) for s in snrs]
    tx = torch.empty(N, dtype=torch.int32, device=dev)
    y = torch.empty((N, D), dtype=torch.float32, device=dev)
    llr = torch.empty((N, m), dtype=torch.float32, device=dev)
    gmis = torch.zeros(len(snrs), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in snrs]
    llr_ms = []

    def step(record):
        for i, s2 in enumerate(sig2):
            md.awgn_sample(X, wl.seed, i * N, N, math.sqrt(s2), tx=tx, y=y)
            if record:
                ev[i][0].record(stream)
            md.llr_exact(X, labels, y, s2, prec=args.prec, out=llr)
            if record:
                ev[i][1].record(stream)
            g, _, _ = md.gmi_reduce(llr, tx, labels, per_bit=False, se=False)
            gmis[i:i + 1].copy_(g)

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
        torch.cuda.synchronize()
        llr_ms.extend(a.elapsed_time(b) for a, b in ev)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = 1e3 * dt / args.steps
    sym_per_step = len(snrs) * N
    value = sym_per_step / (dt / args.steps)

    llr_avg_ms = float(np.mean(llr_ms))
    pairs = N * M
    achieved = pairs / (llr_avg_ms * 1e-3)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": EXP_PEAK / 1e12, "unit": "Texp/s",
                "frac": achieved / EXP_PEAK, "traffic": None,
                "kernel": "llr_exact (llr_fast_kernel<1,16,false> + prep + fallback)",
                "per_launch": f"{pairs:.3e} exp2 (N*M pairs)", "avg_launch_ms": llr_avg_ms}

    if args.copy_probe:
        a = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device=dev)   # 256 MiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()

    out = {
        "metric": METRIC, "value": value, "unit": "symbols/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if args.prec == "fp32" else "bf16", "data": "synthetic",
        "config": {"workload": "8d_m2048_gauss_sweep", "M": M, "D": D, "N_per_snr": N,
                   "snr_db": snrs, "prec": args.prec,
                   "step": "awgn_sample + llr_exact + gmi_reduce per SNR point"},
        "roofline": roofline,
        "detail": {"gmi_bits": {f"{s:g}": round(float(g), 6) for s, g in zip(snrs, gmis.cpu().tolist())},
                   "llr_symbols_per_s": N / (llr_avg_ms * 1e-3)},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl.X, wl.labels, 9.0, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
