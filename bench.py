#!/usr/bin/env python3
"""Benchmark of the REDO propagator path on one MI355X.

Headline workload: the noisy-drive freezing simulation of a 10-qubit Ising
chain (d = 1024) with 4096 seeded noise realisations batched in one launch.
One benchmark step advances every realisation by one time segment: coarse
graining of its amplitude, the table products of its step, the chain product,
the magnetisation observable, and the Newton-Schulz re-projection whenever the
global step index reaches a multiple of 64.  Steps are issued --chunk at a
time per library call.  value = realisation-steps/s.

Also reported: GRAPE iterations/s (fidelity + adjoint gradient) of a
10-qubit NMR chain (d = 1024, N = 500), the plain per-step exponential on the
same GPU when the library provides it, the roofline fraction of the dominant
kernel (batched complex GEMM, timed with HIP events on its stream), and the
FP64 oracle timed on the host cores on a bounded sample: realisation 0 of the
headline workload over the steps the GPU ran, whose REDO chain and EXACT chain
(unsplit, unquantised) give the error of every GPU line and REDO's method error.
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
PEAK_FP32_VECTOR_TFLOPS = 78.6   # non-packed FP32 FMA rate: 256 CUs x 4 SIMDs x 16 lanes x 2 x 2.4 GHz

# HBM bytes per launch of the headline GEMM (three-product FP32 form, 4096
# products at d = 1024), from two rocprofv3 --pmc runs (FETCH_SIZE, then
# WRITE_SIZE) of this script with --calibrate, each counter scaled by what it
# reads for the plain 1 GiB device copy of that run.  The figure belongs to
# the kernel sources it was measured on (the FP32 GEMM and the header it shares
# with the split-BF16 one; SHA-256 of the two files in this order) and is
# reported only while they are unchanged.
GEMM_TRAFFIC = {
    "sources": ["paper_1707_02162_amd/csrc/cgemm.hip", "paper_1707_02162_amd/csrc/cgemm_common.h"],
    "sha256": "c2cf851026c68510a799a340f1c26fb3e1ed4088297da34a758cdb5b79a6c199",
    # FETCH_SIZE 83,909,700 KiB per launch (mean of 64, six digits) x 1.99993 (a 1 GiB copy reads
    # as about 524,305 KiB)
    "fetch_bytes": 171841050953,
    # WRITE_SIZE 33,554,432 KiB per launch x 1.0000 (a 1 GiB copy writes 1,048,576 KiB)
    "write_bytes": 34359738368,
}


def gemm_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for src in GEMM_TRAFFIC["sources"]:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def gemm_traffic(realisations, cache):
    t = GEMM_TRAFFIC
    if t["sha256"] is None or realisations != 4096 or not cache:
        return None
    if gemm_sources_sha256() != t["sha256"]:
        return None
    return t["fetch_bytes"] + t["write_bytes"]


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


def window_warmup(warmup: int, steps: int, reproject: int) -> int:
    """Smallest warm-up length >= warmup whose timed window of `steps` steps
    contains a re-projection step (global step count a multiple of `reproject`):
    with steps >= reproject any window holds one per `reproject` steps; a
    shorter window then holds one, more often than the run does."""
    if reproject <= 0:
        return warmup
    w = warmup
    while (w + steps) // reproject == w // reproject:
        w += 1
    return w


def bench_freezing(args, redo, W, torch):
    """REDO chain (FP32 headline, split BF16) and the plain per-step exponential
    on the same 4096-realisation workload, one table."""
    B, K = args.realisations, args.steps
    Wr = window_warmup(args.warmup, K, args.reproject)
    N = max(Wr + K, args.warmup + args.expm_steps)
    log(f"[bench] building the Ising workload: B={B} d=1024 steps={N} (warm-up {Wr}, timed {K})")
    p = W.ising_freezing(n=10, B=B, N=N)
    t0 = time.time()
    table = redo.RedoTable.from_problem(p)
    torch.cuda.synchronize()
    t_table = time.time() - t0
    log(f"[bench] table built in {t_table:.2f}s ({table.device_bytes / 2**30:.2f} GiB)")
    t_cache = 0.0
    if args.cache:
        t0 = time.time()
        table.cache_levels()
        torch.cuda.synchronize()
        t_cache = time.time() - t0
        log(f"[bench] every level composed once in {t_cache:.2f}s (table + cache {table.device_bytes / 2**30:.1f} GiB)")
    u = torch.tensor(p.u, device="cuda")
    cols, vals = W.observable_ell(p.M)
    obs = (torch.tensor(cols, device="cuda"), torch.tensor(vals, device="cuda", dtype=torch.complex64))
    # M = sum_q I_x^(q) is diagonal in the Walsh basis: the states are carried as W = X H / sqrt(d)
    spec = redo.walsh_observable(cols, vals)
    U = torch.empty((B, p.d, p.d), dtype=torch.complex64, device="cuda")
    mag = torch.empty((B, N), dtype=torch.float64, device="cuda")

    def run(kind, precision, steps, warm, walsh=True):
        wf = spec if walsh else None
        ob = None if walsh else obs

        def advance(n0, n1):
            un = u[:, n0:n1].contiguous()
            X0 = None if n0 == 0 else U
            if kind == "redo":
                _, _, m = table.chain(un, X0=X0, out=U, step_offset=n0, reproject_every=args.reproject,
                                      observable=ob, precision=precision, walsh=wf)
            elif kind == "kron":
                _, m = table.kron_chain(un, X0=X0, out=U, step_offset=n0, reproject_every=args.reproject,
                                        observable=ob, walsh=wf)
            elif kind == "expm_split":
                _, m = table.expm_split_chain(un, X0=X0, out=U, step_offset=n0, reproject_every=args.reproject,
                                              precision=precision, walsh=wf)
            else:
                _, m = table.expm_chain(un, X0=X0, out=U, step_offset=n0, reproject_every=args.reproject,
                                        observable=ob, precision=precision, walsh=wf)
            mag[:, n0:n1] = m

        for n0 in range(0, warm, args.chunk):
            advance(n0, min(warm, n0 + args.chunk))
        torch.cuda.synchronize()
        redo.profile_enable(True)
        redo.profile_read(reset=True)
        t0 = time.perf_counter()
        for n0 in range(warm, warm + steps, args.chunk):
            n1 = min(warm + steps, n0 + args.chunk)
            advance(n0, n1)
            log(f"[bench] {kind} p{precision} timed steps {n1 - warm}/{steps}")
        if wf is not None:
            redo.walsh_right(U)   # the final states back in the computational basis
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        gemm_ms, launches = redo.profile_read(reset=True)                # step products
        kron_ms, kron_launches = redo.profile_read(reset=True, kind=1)
        rp_ms, rp_launches = redo.profile_read(reset=True, kind=2)       # re-projection products
        redo.profile_enable(False)
        m = mag[:, :warm + steps].cpu().numpy()
        common = dict(value=B * steps / elapsed, ms_per_step=1e3 * elapsed / steps, steps=steps, warmup_run=warm,
                      reprojections_timed=(warm + steps) // args.reproject - warm // args.reproject
                      if args.reproject > 0 else 0,
                      mag_last=m[:, -1].copy(), mag0=m[0].copy(), x0=U[0].cpu().numpy().astype(np.complex128))
        if kind == "kron":
            # one launch per step reads and writes every realisation's state once (algorithmic bytes)
            kbytes = 2.0 * 8 * p.d * p.d * B
            return dict(common, avg_launch_ms=kron_ms / max(kron_launches, 1), launches=kron_launches,
                        bytes_per_launch=kbytes,
                        achieved_gbs=kbytes / (kron_ms / max(kron_launches, 1) * 1e-3) / 1e9 if kron_launches else None)
        codes, _ = table.quantise(u[:, warm:warm + steps].contiguous())
        cn = codes.cpu().numpy()
        products = int(np.count_nonzero(cn)) if args.cache else count_products(cn, p.base, p.digits)
        # the product form's own real flops: 8 d^3 (four real products), 6 d^3 (Gauss, three)
        per_product = (6.0 if precision == 1 else 8.0) * p.d ** 3
        flops = per_product * products
        # every re-projection step adds two products per realisation, timed apart: the Gram
        # product X^dag X (Hermitian: only the tiles that meet the upper triangle run) at the
        # chain's precision, then the correction X E as a split-BF16 product; with two
        # arithmetics and a partial tile set no single peak applies, so the time is reported
        rp = None
        if kind == "redo" and rp_launches:
            nrp = common["reprojections_timed"]
            rp = dict(launches=rp_launches, avg_launch_ms=rp_ms / rp_launches, products=2 * B * nrp,
                      ms_per_reprojection=rp_ms / nrp if nrp else None,
                      form="Gram product at the chain's precision (upper tiles) + split-BF16 correction X E")
        return dict(common, gemm_ms=gemm_ms, gemm_launches=launches, products=products,
                    achieved=(flops / (gemm_ms * 1e-3) / 1e12) if kind == "redo" else None, reproject_gemm=rp,
                    flops_per_launch=flops / max(launches, 1), avg_launch_ms=gemm_ms / max(launches, 1))

    fp32 = run("redo", 1, K, Wr)
    lists = None if args.no_lists else run("redo", 1, K, Wr, walsh=False)
    bf = None
    if not args.no_bf16:
        t_split = None
        if args.cache:
            # the cached levels as pre-split BF16 panels: only the state is split as it is loaded
            t0 = time.time()
            table.cache_split_bf16()
            torch.cuda.synchronize()
            t_split = time.time() - t0
            log(f"[bench] cached levels pre-split to BF16 in {t_split:.2f}s")
        bf = run("redo", 2, K, Wr)
        bf["presplit_build_s"] = t_split
        if args.cache:
            table.cache_split_bf16(False)
    g4 = None if args.no_4m else run("redo", 0, K, Wr)
    ex = None if args.no_expm else run("expm", 1, args.expm_steps, args.warmup)
    exs = None if args.no_expm else run("expm_split", 1, args.expm_steps, args.warmup)
    kr = None if args.no_kron else run("kron", 0, K, Wr)
    out = dict(fp32=fp32, lists=lists, bf16x3=bf, f32_4m=g4, expm=ex, expm_split=exs, kron=kr, table_build_s=t_table,
               cache_build_s=t_cache)
    del table
    return out, p


def bench_grape(args, redo, W, torch):
    p = W.c6_grape_1024(B=1, N=500)
    table = redo.RedoTable.from_problem(p)
    if args.cache:
        table.cache_levels()
    u = torch.tensor(p.u, device="cuda")
    Uf = torch.tensor(p.U_target, device="cuda")
    res = {}
    first = {}
    for kind in ("redo", "expm"):
        if kind == "expm" and args.no_expm:
            continue
        # both methods on the three-product FP32 GEMM, as the headline
        fn0 = table.grape if kind == "redo" else table.expm_grape
        fn = lambda uu_, Uf_: fn0(uu_, Uf_, precision=1)
        uu = u.clone()
        # one whole untimed iteration, update included (the first use of each
        # kernel loads its code object); its F and gradient at the start point
        # compare the two methods
        F, _, g = fn(uu, Uf)
        first[kind] = (float(F.item()), g.double().cpu().numpy())
        redo.ascent_step(uu, g, 1e3, -p.u_scale, p.u_scale)
        torch.cuda.synchronize()
        uu = u.clone()
        log(f"[bench] {kind} grape warmup done")
        t0 = time.perf_counter()
        for i in range(args.grape_iters):
            F, _, g = fn(uu, Uf)
            # projected gradient ascent update (the accepted step of an iteration), in the library
            redo.ascent_step(uu, g, 1e3, -p.u_scale, p.u_scale)
            torch.cuda.synchronize()
            log(f"[bench] {kind} grape iteration {i + 1}/{args.grape_iters}")
        elapsed = time.perf_counter() - t0
        res[kind] = dict(iters_per_s=args.grape_iters / elapsed, ms_per_iter=1e3 * elapsed / args.grape_iters,
                         fidelity=float(F.item()))
    if "expm" in first:
        gr, ge = first["redo"][1], first["expm"][1]
        res["method"] = {
            "point": "the workload's start pulse (Haar target, F ~ 1/d^2)",
            "fidelity_redo": first["redo"][0], "fidelity_expm": first["expm"][0],
            "grad_rel_l2_redo_vs_expm": float(np.linalg.norm(gr - ge) / np.linalg.norm(ge)),
            "note": "REDO: quantised split steps, exact straight-through gradient; expm: unquantised unsplit "
                    "steps, first-order GRAPE gradient"}
    del table
    return res


def bench_next(args, redo, W, torch):
    """The NEXT rows measured on d = 1024 workloads: the Strang splitting on the
    headline workload (4096 realisations, observable every step, three-product
    GEMMs) and state-transfer GRAPE on the GRAPE workload (target: the state the
    Haar target unitary makes of |0>)."""
    out = {}
    B, K = args.realisations, args.steps
    Wm = window_warmup(args.warmup, K, args.reproject)
    p = W.ising_freezing(n=10, B=B, N=Wm + K)
    p.splitting = "strang"
    table = redo.RedoTable.from_problem(p)
    if args.cache:
        table.cache_levels()
    u = torch.tensor(p.u, device="cuda")
    cols, vals = W.observable_ell(p.M)
    spec = redo.walsh_observable(cols, vals)
    U = torch.empty((B, p.d, p.d), dtype=torch.complex64, device="cuda")
    def advance(n0, n1):
        table.chain(u[:, n0:n1].contiguous(), X0=None if n0 == 0 else U, out=U, step_offset=n0,
                    reproject_every=args.reproject, precision=1, walsh=spec)

    for n0 in range(0, Wm, args.chunk):
        advance(n0, min(Wm, n0 + args.chunk))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for n0 in range(Wm, Wm + K, args.chunk):
        advance(n0, min(Wm + K, n0 + args.chunk))
    redo.walsh_right(U)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out["strang"] = {"workload": "headline workload with the Strang splitting V(dt/2) C_n V(dt/2)",
                     "value": B * K / el, "unit": "propagator steps/s", "ms_per_step": 1e3 * el / K}
    log(f"[bench] Strang headline: {B * K / el:.4g} steps/s")
    del table, U
    torch.cuda.empty_cache()
    q = W.c6_grape_1024(B=1, N=500)
    table = redo.RedoTable.from_problem(q)
    if args.cache:
        table.cache_levels()
    uq = torch.tensor(q.u, device="cuda")
    psi0 = np.zeros((1, q.d), np.complex128)
    psi0[0, 0] = 1.0
    psif = q.U_target[:, :, 0].copy()
    # warm-up: one whole iteration, the update included (torch loads its kernels on first use)
    _, _, g = table.state_grape(uq, psi0, psif)
    redo.ascent_step(uq, g, 1e3, -q.u_scale, q.u_scale)
    torch.cuda.synchronize()
    iters = 20
    t0 = time.perf_counter()
    for _ in range(iters):
        F, _, g = table.state_grape(uq, psi0, psif)
        redo.ascent_step(uq, g, 1e3, -q.u_scale, q.u_scale)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / iters
    # each step applies its one composed factor (8 d^2 bytes read) to the forward and the backward vector
    gbs = 2 * q.N * 8 * q.d * q.d / el / 1e9
    out["state_grape"] = {"workload": "10-qubit NMR chain d=1024, N=500, F_S = |<psi_f|U|0>|^2, gradient + update",
                          "iters_per_s": 1.0 / el, "ms_per_iter": 1e3 * el,
                          "factor_read_GBs": gbs, "frac_of_hbm": gbs / PEAK_HBM_GBS}
    log(f"[bench] state GRAPE d=1024: {1.0 / el:.4g} it/s ({gbs:.0f} GB/s of factor reads)")
    del table
    return out


def bench_c2(args, redo, W, torch):
    """Secondary comparison at d = 64 (6-qubit chain, 256 replicas x 2000 steps):
    the fused small-d REDO chain against the plain per-step exponential on the
    batched GEMMs, both chaining every step of every replica."""
    p = W.c2_six_qubit(B=256, N=2000)
    table = redo.RedoTable.from_problem(p)
    if args.cache:
        table.cache_levels()
    u = torch.tensor(p.u, device="cuda")
    res = {}
    for kind in ("redo", "expm"):
        if kind == "expm" and args.no_expm:
            continue
        fn = table.chain if kind == "redo" else table.expm_chain
        fn(u)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 3
        for _ in range(reps):
            fn(u)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / reps
        res[kind] = dict(value=p.B * p.N / el, unit="propagator steps/s", ms_per_call=1e3 * el)
        log(f"[bench] d=64 {kind} chain: {p.B * p.N / el:.3g} steps/s")
    del table
    out = {"workload": "6-qubit NMR chain d=64, 256 replicas x 2000 steps, b=32 P=2, chain only",
           "redo": res["redo"]}
    if "expm" in res:
        out["expm"] = res["expm"]
        out["speedup_vs_expm"] = res["redo"]["value"] / res["expm"]["value"]
    return out


def bench_small(args, redo, W, torch):
    """The small-d configurations: two spins (d = 4, 65,536 seeded replicas x 200
    steps, two phased channels, 8-bit levels, every level cached): chain steps/s and
    GRAPE iterations/s (fidelity + adjoint gradient + update); batched ragged GRAPE of
    64 five-qubit systems (d = 32, N_b ~ U{500..3000}, five phased channels, each its
    own drift and target): iterations/s.  Algorithmic work: 8 d^3 real flops per
    table-factor product (one per non-zero code with every level cached), the
    VALU-bound kernels' roofline against the non-packed FP32 vector peak."""
    out = {}
    p = W.c1_two_spin(B=args.c1_replicas, N=200)
    table = redo.RedoTable.from_problem(p)
    table.cache_levels()
    u = torch.tensor(p.u, device="cuda")
    Uf = torch.tensor(p.U_target, device="cuda")
    codes, _ = table.quantise(u)
    nnz = int(torch.count_nonzero(codes).item())
    table.chain(u)
    torch.cuda.synchronize()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        table.chain(u)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    steps = p.B * p.N
    flops = 8.0 * p.d ** 3 * nnz
    chain = {"value": steps / el, "unit": "propagator steps/s", "ms_per_call": 1e3 * el,
             "achieved_tflops": flops / el / 1e12, "peak_tflops": PEAK_FP32_VECTOR_TFLOPS,
             "frac": flops / el / 1e12 / PEAK_FP32_VECTOR_TFLOPS}
    F, _, g = table.grape(u, Uf)
    redo.ascent_step(u, g, 1e3, -p.u_scale, p.u_scale)
    torch.cuda.synchronize()
    iters = 5
    t0 = time.perf_counter()
    for _ in range(iters):
        F, _, g = table.grape(u, Uf)
        redo.ascent_step(u, g, 1e3, -p.u_scale, p.u_scale)
    torch.cuda.synchronize()
    elg = (time.perf_counter() - t0) / iters
    # forward, recomputed segment and backward scan apply every factor once each, plus Y = X L per step
    gflops = 8.0 * p.d ** 3 * (3 * nnz + steps)
    out["c1_two_spin"] = {
        "workload": "2 spins (d=4), 65,536 replicas x 200 steps of 5 us, 2 phased channels, b=16 P=2 "
                    "(every level cached), Haar targets",
        "chain": chain,
        "grape": {"iters_per_s": 1.0 / elg, "ms_per_iter": 1e3 * elg, "replica_steps_per_s": steps / elg,
                  "achieved_tflops": gflops / elg / 1e12, "frac": gflops / elg / 1e12 / PEAK_FP32_VECTOR_TFLOPS}}
    log(f"[bench] d=4 chain {steps / el:.3g} steps/s, GRAPE {1.0 / elg:.3g} it/s")
    del table, u, Uf
    torch.cuda.empty_cache()
    q = W.c4_batched_grape(B=64)
    table = redo.RedoTable.from_problem(q)
    table.cache_levels()
    u = torch.tensor(q.u, device="cuda")
    Uf = torch.tensor(q.U_target, device="cuda")
    ns = torch.tensor(q.n_steps, device="cuda")
    codes, _ = table.quantise(u)
    live = (torch.arange(q.N, device="cuda")[None, :] < ns[:, None]).unsqueeze(-1)
    nnz = int(torch.count_nonzero(codes * live).item())
    F, _, g = table.grape(u, Uf, n_steps=ns)
    redo.ascent_step(u, g, 1e3, -q.u_scale, q.u_scale)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(iters):
        F, _, g = table.grape(u, Uf, n_steps=ns)
        redo.ascent_step(u, g, 1e3, -q.u_scale, q.u_scale)
    torch.cuda.synchronize()
    elc = (time.perf_counter() - t0) / iters
    total = int(q.n_steps.sum())
    cflops = 8.0 * q.d ** 3 * (3 * nnz + total)
    out["c4_batched_grape"] = {
        "workload": "64 five-qubit systems (d=32), ragged N_b ~ U{500..3000} (sum %d), 5 phased channels, "
                    "b=32 P=2 (every level cached), own drift and Haar target each, checkpoints every "
                    "ceil(sqrt N) steps" % total,
        "iters_per_s": 1.0 / elc, "ms_per_iter": 1e3 * elc, "system_steps_per_s": total / elc,
        "achieved_tflops": cflops / elc / 1e12, "frac": cflops / elc / 1e12 / PEAK_FP32_VECTOR_TFLOPS,
        "note": "step propagators composed first (all system-steps in parallel), then one workgroup per system "
                "scans them: 64 workgroups on 256 compute units, latency-bound"}
    log(f"[bench] d=32 batched GRAPE {1.0 / elc:.3g} it/s")
    del table
    return out


def bench_sweep(args):
    """The paper's own experiment (Sec. IV): the noisy-drive freezing sweep of
    a 3-spin chain (d = 8), 10,000 time points per (omega, lambda) instance,
    order parameter Q = time average of the magnetisation response.  Timed
    on the first `--sweep-instances` instances of the 500 x 1000 grid."""
    from paper_1707_02162_amd import freezing
    freezing.sweep(500, 1000, N=10000, first=0, count=min(512, args.sweep_instances))   # warm-up
    Q, secs, steps = freezing.sweep(500, 1000, N=10000, first=0, count=args.sweep_instances)
    log(f"[bench] freezing sweep: {steps / secs:.3g} steps/s")
    return {"workload": "noisy-drive freezing sweep (3-spin chain, d=8), 10,000 time points per (omega, lambda) "
                        "instance, b=100 P=2, observable every time point, first instances of the 500 x 1000 grid",
            "instances": args.sweep_instances, "steps": steps, "seconds": secs, "value": steps / secs,
            "unit": "propagator steps/s", "full_grid_seconds_estimate": 5e9 / (steps / secs)}


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max(i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas")
    except Exception:
        return os.cpu_count()


def oracle_accuracy(args, W, p, fr):
    """The FP64 oracle on the host for realisation 0 of the headline workload,
    over the steps the GPU ran: its REDO chain (Sec. II processes 1-2 with the
    split step of Sec. III; timed, this is the CPU baseline) and its EXACT chain
    (Sec. III, Eq. propUn: unsplit, unquantised), and the error of every GPU
    line against them."""
    import oracle as O
    f32 = fr["fp32"]
    n_r = f32["warmup_run"] + f32["steps"]
    q = p.subset([0])
    tab = O.DiscreteTable(q.S, q.dt, q.eps, q.base, q.digits)
    t0 = time.perf_counter()
    redo_steps = O.compose_all_redo(q, tab, 0, n_steps=n_r)
    m_redo, X_redo = O.magnetisation_series(redo_steps, q.M)
    el = time.perf_counter() - t0
    cpu = dict(value=n_r / el, unit="realisation-steps/s", cores=int(blas_threads()), kind="oracle",
               sample=f"realisation 0 x {n_r} steps of the d=1024 Ising workload (REDO products, chain and "
                      f"magnetisation in FP64 numpy), {el:.1f} s")
    log(f"[bench] oracle REDO chain: {n_r} steps in {el:.1f} s")

    def err(line, m_ref, X_ref):
        n = len(m_ref)
        return {"max_abs_dm": float(np.abs(line["mag0"][:n] - m_ref).max()),
                "nfrob": None if X_ref is None else float(np.linalg.norm(line["x0"] - X_ref) / np.sqrt(p.d))}

    acc = {"realisation": 0, "steps": n_r,
           "bound_note": "FP32 products at K = 1024: ||dX||_F/sqrt(d) random-walks as ~1.6e-6 sqrt(products); "
                         "the magnetisation gate is |dm| <= 1e-5"}
    names = {"fp32": "headline", "lists": "row_list", "bf16x3": "bf16x3", "f32_4m": "f32_4m",
             "kron": "structure_aware"}
    for key, name in names.items():
        if fr.get(key) is not None:
            acc[name + "_vs_oracle"] = err(fr[key], m_redo, X_redo)
    exs = fr.get("expm_split")
    if exs is not None:
        n_s = exs["warmup_run"] + exs["steps"]
        acc["expm_equal_result_vs_oracle"] = dict(err(exs, m_redo[:n_s], O.chain(redo_steps[:n_s])), steps=n_s)
    del redo_steps
    if not args.no_exact:
        H0m = np.diag(q.H0[0]).astype(np.complex128)
        t0 = time.perf_counter()
        ex_steps = [O.step_exact(H0m, q.S, None, q.u[0, n].astype(np.float64), q.dt) for n in range(n_r)]
        m_ex, X_ex = O.magnetisation_series(ex_steps, q.M)
        el_x = time.perf_counter() - t0
        log(f"[bench] oracle EXACT chain: {n_r} steps in {el_x:.1f} s")
        acc["method_error_vs_exact"] = {
            "steps": n_r,
            "redo_oracle": {"max_abs_dm": float(np.abs(m_redo - m_ex).max()),
                            "nfrob": float(np.linalg.norm(X_redo - X_ex) / np.sqrt(p.d))},
            "headline_gpu": err(f32, m_ex, X_ex),
            "exact_oracle_seconds": el_x}
        ex = fr.get("expm")
        if ex is not None:
            n_e = ex["warmup_run"] + ex["steps"]
            X_e = O.chain(ex_steps[:n_e])
            acc["expm_vs_exact"] = dict(err(ex, m_ex[:n_e], X_e), steps=n_e,
                                        headline_same_steps_max_abs_dm=float(np.abs(f32["mag0"][:n_e] - m_ex[:n_e]).max()))
    return cpu, acc


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--realisations", type=int, default=4096)
    ap.add_argument("--reproject", type=int, default=64)
    ap.add_argument("--grape-iters", type=int, default=5)
    ap.add_argument("--no-exact", action="store_true",
                    help="skip the oracle's EXACT chain (the method-error comparison)")
    ap.add_argument("--no-grape", action="store_true")
    ap.add_argument("--no-bf16", action="store_true")
    ap.add_argument("--no-4m", action="store_true", help="skip the four-product FP32 line")
    ap.add_argument("--no-lists", action="store_true",
                    help="skip the line with the two-pass row-list observable (computational basis)")
    ap.add_argument("--no-expm", action="store_true")
    ap.add_argument("--no-kron", action="store_true", help="skip the structure-aware chain on the headline workload")
    ap.add_argument("--no-next", action="store_true", help="skip the Strang and state-GRAPE lines")
    ap.add_argument("--expm-steps", type=int, default=4)
    ap.add_argument("--chunk", type=int, default=4, help="time segments advanced per library call")
    ap.add_argument("--calibrate", action="store_true",
                    help="first run a plain 1 GiB device copy (reference for hardware byte counters)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-c2", action="store_true", help="skip the d=64 REDO vs expm chain comparison")
    ap.add_argument("--no-sweep", action="store_true", help="skip the d=8 freezing sweep")
    ap.add_argument("--no-freezing", action="store_true",
                    help="skip the headline workload (profiling runs of the others; prints no headline value)")
    ap.add_argument("--sweep-instances", type=int, default=16384)
    ap.add_argument("--c1-replicas", type=int, default=65536)
    ap.add_argument("--no-small", action="store_true", help="skip the d=4 and d=32 lines")
    ap.add_argument("--no-cache", dest="cache", action="store_false",
                    help="apply one product per non-zero digit instead of the composed level of each amplitude")
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

    if args.calibrate:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("[bench] calibration copy: 3 x 1 GiB read + 1 GiB write")
    fr, p = (None, None) if args.no_freezing else bench_freezing(args, redo, W, torch)
    torch.cuda.empty_cache()
    gr = None if args.no_grape else bench_grape(args, redo, W, torch)
    torch.cuda.empty_cache()
    c2 = None if args.no_c2 else bench_c2(args, redo, W, torch)
    torch.cuda.empty_cache()
    nx = None if (args.no_next or args.no_freezing) else bench_next(args, redo, W, torch)
    torch.cuda.empty_cache()
    sw = None if args.no_sweep else bench_sweep(args)
    torch.cuda.empty_cache()
    sm = None if args.no_small else bench_small(args, redo, W, torch)
    torch.cuda.empty_cache()
    cpu, acc = (None, None) if (args.no_cpu or fr is None) else oracle_accuracy(args, W, p, fr)
    rg = None if gr is None else gr.get("redo")
    eg = None if gr is None else gr.get("expm")
    if fr is None:
        # profiling runs of the secondary workloads only: no headline figure
        print(json.dumps({"metric": "propagator steps/s + GRAPE iters/s at d=1024, REDO vs plain expm, same GPU",
                          "value": None, "note": "headline workload skipped (--no-freezing)",
                          "grape_iters_per_s": None if rg is None else rg["iters_per_s"],
                          "grape_expm_iters_per_s": None if eg is None else eg["iters_per_s"],
                          "d64_chain": c2, "paper_freezing_sweep_d8": sw, "small_d": sm}), flush=True)
        return
    f32, bf, ex, kr, g4, ls = fr["fp32"], fr["bf16x3"], fr["expm"], fr["kron"], fr["f32_4m"], fr["lists"]
    out = {
        "metric": "propagator steps/s + GRAPE iters/s at d=1024, REDO vs plain expm, same GPU",
        "value": f32["value"],
        "unit": "propagator steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f32["ms_per_step"],
        "timed_window": {"first_step": f32["warmup_run"] + 1, "last_step": f32["warmup_run"] + f32["steps"],
                         "reprojections": f32["reprojections_timed"],
                         "note": "untimed warm-up extended from --warmup so that the timed window holds a "
                                 "re-projection step (one per 64 steps when --steps >= 64, else one in the window)"},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 (fp32 complex; 3 real MFMA products per complex product, Gauss)",
        "data": "synthetic (seeded noise realisations)",
        "config": {"workload": "noisy-drive freezing, 10-qubit Ising chain, d=1024, 4096 realisations, "
                               "REDO b=100 P=2" + (" with every level composed once (process 3)" if args.cache else "") +
                               ", one step = one time segment for all realisations, "
                               "magnetisation every step, re-projection every 64 steps; states carried in the "
                               "right Walsh frame (M diagonal there: one-pass magnetisation), back-transformed "
                               "once at the end inside the timed region",
                   "realisations": args.realisations, "d": 1024, "base": p.base, "digits": p.digits},
        "expm_baseline": None if ex is None else {
            "value": ex["value"], "unit": "propagator steps/s", "ms_per_step": ex["ms_per_step"],
            "steps": args.expm_steps, "method": "per-step exp(-i dt H_n), scaling-and-squaring Taylor "
                                                 "(Paterson-Stockmeyer), same batched FP32 MFMA GEMM (three real products), "
                                                 "same Walsh-frame magnetisation"},
        "speedup_vs_expm": None if ex is None else f32["value"] / ex["value"],
        "expm_equal_result": None if fr.get("expm_split") is None else {
            "value": fr["expm_split"]["value"], "unit": "propagator steps/s",
            "ms_per_step": fr["expm_split"]["ms_per_step"], "steps": args.expm_steps,
            "method": "the same split, coarse-grained steps as REDO with each control factor "
                      "exp(-i dt q eps S) by the same Taylor / Paterson-Stockmeyer evaluation and GEMMs, "
                      "drift phases in the chain product: equal to REDO's result up to FP32 rounding",
            "error_vs_redo_oracle": None if acc is None else acc.get("expm_equal_result_vs_oracle")},
        "speedup_vs_expm_equal_result": None if fr.get("expm_split") is None else
            f32["value"] / fr["expm_split"]["value"],
        "max_abs_dm_vs_oracle": None if acc is None else acc["headline_vs_oracle"]["max_abs_dm"],
        "nfrob_vs_oracle": None if acc is None else acc["headline_vs_oracle"]["nfrob"],
        "method_error_vs_exact": None if acc is None else acc.get("method_error_vs_exact"),
        "expm_error_vs_exact": None if acc is None else acc.get("expm_vs_exact"),
        "row_list_observable": None if ls is None else {
            "value": ls["value"], "unit": "propagator steps/s", "ms_per_step": ls["ms_per_step"],
            "method": "same chain in the computational basis, magnetisation from the row lists in two passes "
                      "(T = M X written, then a dot pass)",
            "max_abs_dm_vs_headline_last_step": float(np.abs(ls["mag_last"] - f32["mag_last"]).max())},
        "bf16x3": None if bf is None else {"value": bf["value"], "unit": "propagator steps/s",
                                          "ms_per_step": bf["ms_per_step"],
                                          "achieved_algorithmic_tflops": bf["achieved"],
                                          "executed_bf16_tflops": 3 * bf["achieved"],
                                          "frac_of_bf16_peak": 3 * bf["achieved"] / 2500.0,
                                          "avg_launch_ms": bf["avg_launch_ms"],
                                          "reproject_gemm": bf["reproject_gemm"],
                                          "presplit_levels": bf["presplit_build_s"] is not None,
                                          "presplit_build_s": bf["presplit_build_s"],
                                          "max_abs_dm_vs_fp32_last_step": float(np.abs(bf["mag_last"] - f32["mag_last"]).max())},
        "f32_4m": None if g4 is None else {
            "value": g4["value"], "unit": "propagator steps/s", "ms_per_step": g4["ms_per_step"],
            "method": "FP32, four real MFMA products per complex product",
            "avg_launch_ms": g4["avg_launch_ms"], "achieved_tflops": g4["achieved"],
            "frac_of_fp32_peak": g4["achieved"] / PEAK_FP32_MFMA_TFLOPS,
            "max_abs_dm_vs_headline_last_step": float(np.abs(g4["mag_last"] - f32["mag_last"]).max())},
        "structure_aware": None if kr is None else {
            "value": kr["value"], "unit": "propagator steps/s", "ms_per_step": kr["ms_per_step"],
            "method": "same quantised steps with spin-factorised control blocks (one 2x2 per spin, O(n d^2)); "
                      "a competitor of the dense REDO factors, not the paper's method",
            "speedup_vs_redo": kr["value"] / f32["value"],
            "step_kernel": {"bound": "hbm", "avg_launch_ms": kr["avg_launch_ms"], "launches": kr["launches"],
                            "bytes_per_launch": kr["bytes_per_launch"], "achieved_GBs": kr["achieved_gbs"],
                            "peak_GBs": PEAK_HBM_GBS,
                            "frac": None if kr["achieved_gbs"] is None else kr["achieved_gbs"] / PEAK_HBM_GBS},
            "max_abs_dm_vs_redo_last_step": float(np.abs(kr["mag_last"] - f32["mag_last"]).max())},
        "grape_iters_per_s": None if rg is None else rg["iters_per_s"],
        "grape": None if rg is None else {"workload": "10-qubit NMR chain d=1024, N=500, b=32 P=2, "
                                                      "fidelity + adjoint gradient + update, FP32 three-product GEMMs",
                                          **rg},
        "grape_expm_iters_per_s": None if eg is None else eg["iters_per_s"],
        "grape_speedup_vs_expm": None if (rg is None or eg is None) else rg["iters_per_s"] / eg["iters_per_s"],
        "grape_method_comparison": None if gr is None else gr.get("method"),
        "d64_chain": c2,
        "paper_freezing_sweep_d8": sw,
        "small_d": sm,
        "strang": None if nx is None else nx["strang"],
        "state_grape": None if nx is None else nx["state_grape"],
        "table_build_s": fr["table_build_s"],
        "level_cache_build_s": fr["cache_build_s"],
        "roofline": {"bound": "mfma", "kernel": "cgemm_kernel<128,64,3M> (batched complex GEMM, FP32, three real products)",
                     "achieved": f32["achieved"], "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                     "frac": f32["achieved"] / PEAK_FP32_MFMA_TFLOPS,
                     "traffic": gemm_traffic(args.realisations, args.cache), "traffic_unit": "HBM bytes per launch",
                     "flops_per_launch": f32["flops_per_launch"], "avg_launch_ms": f32["avg_launch_ms"],
                     "launches": f32["gemm_launches"],
                     "flops_note": "6 d^3 real flops per complex product (the Gauss form's own count; the "
                                   "four-product form would be 8 d^3) over the step products of the timed "
                                   "window, one launch per step (4096 products); the re-projection products "
                                   "run as separate instantiations (the Gram product role 4, the split-BF16 "
                                   "correction role 2) and are reported apart",
                     "reproject_gemm": f32["reproject_gemm"]},
        "cpu_baseline": cpu,
        "accuracy_vs_oracle": acc,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
