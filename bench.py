#!/usr/bin/env python3
"""Benchmark of the REDO propagator path on one MI355X.

Headline workload: the noisy-drive freezing simulation of a 10-qubit Ising
chain (d = 1024) with 4096 seeded noise realisations batched in one launch.
One benchmark step advances every realisation by one time segment: coarse
graining of its amplitude, the table products of its step, the chain product,
the magnetisation observable, and the Newton-Schulz re-projection whenever the
global step index reaches a multiple of 64.  value = realisation-steps/s.

Also reported: GRAPE iterations/s (fidelity + adjoint gradient) of a
10-qubit NMR chain (d = 1024, N = 500), the plain per-step exponential on the
same GPU when the library provides it, the roofline fraction of the dominant
kernel (batched complex GEMM, timed with HIP events on its stream), and the
FP64 oracle timed on the host cores on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def count_products(codes: np.ndarray, base: int, digits: int) -> int:
    """Number of dense table-factor products a set of codes asks for (one per
    non-zero digit)."""
    a = np.abs(codes.astype(np.int64))
    n = 0
    for _ in range(digits):
        n += int(np.count_nonzero(a % base))
        a //= base
    return n


def bench_freezing(args, redo, W, torch):
    B, K, Wm = args.realisations, args.steps, args.warmup
    N = Wm + K
    log(f"[bench] building the Ising workload: B={B} d=1024 steps={N}")
    p = W.ising_freezing(n=10, B=B, N=N)
    t0 = time.time()
    table = redo.RedoTable.from_problem(p)
    torch.cuda.synchronize()
    t_table = time.time() - t0
    log(f"[bench] table built in {t_table:.2f}s ({table.device_bytes / 2**30:.2f} GiB)")
    u = torch.tensor(p.u, device="cuda")
    cols, vals = W.observable_ell(p.M)
    obs = (torch.tensor(cols, device="cuda"), torch.tensor(vals, device="cuda", dtype=torch.complex64))
    U = torch.empty((B, p.d, p.d), dtype=torch.complex64, device="cuda")
    mag = torch.empty((B, N), dtype=torch.float64, device="cuda")

    def step(n, first=False):
        Un, _, m = table.chain(u[:, n:n + 1].contiguous(), X0=None if first else U, out=U, step_offset=n,
                               reproject_every=args.reproject, observable=obs)
        mag[:, n:n + 1] = m

    for n in range(Wm):
        step(n, first=(n == 0))
        torch.cuda.synchronize()
        log(f"[bench] warmup step {n + 1}/{Wm}")
    redo.profile_enable(True)
    redo.profile_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for n in range(Wm, N):
        step(n, first=(n == 0))
        if (n - Wm) % 2 == 1:
            log(f"[bench] timed step {n - Wm + 1}/{K}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    gemm_ms, launches = redo.profile_read(reset=True)
    redo.profile_enable(False)
    codes, _ = table.quantise(u[:, Wm:N].contiguous())
    products = count_products(codes.cpu().numpy(), p.base, p.digits)
    flops = 8.0 * p.d ** 3 * products
    achieved = flops / (gemm_ms * 1e-3) / 1e12
    m = mag.cpu().numpy()
    res = dict(value=B * K / elapsed, ms_per_step=1e3 * elapsed / K, table_build_s=t_table,
               gemm_ms=gemm_ms, gemm_launches=launches, products=products, achieved=achieved,
               flops_per_launch=flops / max(launches, 1), avg_launch_ms=gemm_ms / max(launches, 1),
               mag_first=float(m[:, 0].mean()), mag_last=float(m[:, -1].mean()))
    del table
    return res, p


def bench_grape(args, redo, W, torch):
    p = W.c6_grape_1024(B=1, N=500)
    table = redo.RedoTable.from_problem(p)
    u = torch.tensor(p.u, device="cuda")
    Uf = torch.tensor(p.U_target, device="cuda")
    for i in range(1):
        table.grape(u, Uf)
    torch.cuda.synchronize()
    log("[bench] grape warmup done")
    t0 = time.perf_counter()
    for i in range(args.grape_iters):
        F, _, g = table.grape(u, Uf)
        # projected gradient ascent update (the accepted step of an iteration)
        u = torch.clamp(u + 1e3 * g, -p.u_scale, p.u_scale)
        torch.cuda.synchronize()
        log(f"[bench] grape iteration {i + 1}/{args.grape_iters}")
    elapsed = time.perf_counter() - t0
    del table
    return dict(iters_per_s=args.grape_iters / elapsed, ms_per_iter=1e3 * elapsed / args.grape_iters,
                fidelity=float(F.item()))


def cpu_baseline(args, W):
    """The FP64 oracle on the host: REDO steps of one realisation of the same
    workload, with the magnetisation at every step."""
    import oracle as O
    threads = None
    try:
        from threadpoolctl import threadpool_info
        threads = max(i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas")
    except Exception:
        threads = os.cpu_count()
    n = args.cpu_steps
    p = W.ising_freezing(n=10, B=1, N=n)
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    t0 = time.perf_counter()
    steps = O.compose_all_redo(p, tab, 0)
    O.magnetisation_series(steps, p.M)
    el = time.perf_counter() - t0
    return dict(value=n / el, unit="realisation-steps/s", cores=int(threads), kind="oracle",
                sample=f"1 realisation x {n} steps of the d=1024 Ising workload (REDO products, chain and "
                       f"magnetisation in FP64 numpy), {el:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--realisations", type=int, default=4096)
    ap.add_argument("--reproject", type=int, default=64)
    ap.add_argument("--grape-iters", type=int, default=3)
    ap.add_argument("--cpu-steps", type=int, default=60)
    ap.add_argument("--no-grape", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(sharding over realisations or time blocks is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1707_02162_amd import redo
    from paper_1707_02162_amd import workloads as W
    torch.cuda.init()
    free, total = torch.cuda.mem_get_info()
    log(f"[bench] device {torch.cuda.get_device_name(0)}, {free / 2**30:.0f}/{total / 2**30:.0f} GiB free")

    fr, p = bench_freezing(args, redo, W, torch)
    torch.cuda.empty_cache()
    gr = None if args.no_grape else bench_grape(args, redo, W, torch)
    torch.cuda.empty_cache()
    cpu = None if args.no_cpu else cpu_baseline(args, W)
    out = {
        "metric": "propagator steps/s + GRAPE iters/s at d=1024, REDO vs plain expm, same GPU",
        "value": fr["value"],
        "unit": "propagator steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fr["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 (fp32 complex, 4 real MFMA products per complex product)",
        "data": "synthetic (seeded noise realisations)",
        "config": {"workload": "noisy-drive freezing, 10-qubit Ising chain, d=1024, 4096 realisations, "
                               "REDO b=100 P=2, one step = one time segment for all realisations, "
                               "magnetisation every step, re-projection every 64 steps",
                   "realisations": args.realisations, "d": 1024, "base": p.base, "digits": p.digits},
        "grape_iters_per_s": None if gr is None else gr["iters_per_s"],
        "grape": None if gr is None else {"workload": "10-qubit NMR chain d=1024, N=500, b=32 P=2, "
                                                      "fidelity + adjoint gradient + update", **gr},
        "expm_baseline": None,
        "table_build_s": fr["table_build_s"],
        "roofline": {"bound": "mfma", "kernel": "cgemm_kernel<128,128,4M>",
                     "achieved": fr["achieved"], "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                     "frac": fr["achieved"] / PEAK_FP32_MFMA_TFLOPS, "traffic": None,
                     "flops_per_launch": fr["flops_per_launch"], "avg_launch_ms": fr["avg_launch_ms"],
                     "launches": fr["gemm_launches"]},
        "cpu_baseline": cpu,
        "magnetisation_mean": {"first_step": fr["mag_first"], "last_step": fr["mag_last"]},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
