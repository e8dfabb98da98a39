"""The benchmarked configurations end to end against the FP64 oracle.

Chain: the noisy-drive freezing simulation of Sec. IV at d = 1024 with 4096
realisations in one launch, every level composed once (process 3 of Sec. II),
three-product FP32 (or split-BF16) GEMMs, states carried in the right Walsh
frame with the one-pass magnetisation, Newton-Schulz re-projection every 64
steps, advanced a few steps per call as the benchmark does, over 130 steps
(two re-projections); two sampled realisations against the oracle's REDO
chain at every step (magnetisation) and every 10 steps (state).  The split-BF16
run reads the cached levels as pre-split panels, as the benchmark does.

GRAPE: the d = 1024 NMR workload of the GRAPE benchmark (one collective phased
channel, every level cached, every state kept, three-product GEMMs) against
the oracle's straight-through REDO gradient (Sec. III).

Bounds:
  * magnetisation |dm_n| <= 1e-5 at every step (the observable gate of the
    long d = 1024 chain);
  * state ||dX||_F / sqrt(d) <= 1e-5 at every tenth step.  It grows as a random
    walk of the FP32 accumulation error of the products (about 6e-7 sqrt(g) after
    g products at K = 1024, less the non-unitary part each re-projection removes),
    so this bound holds for a few hundred steps, not for the whole 5000-step run;
  * split BF16: ||dX||_F / sqrt(d) <= 1e-3 and |dm_n| <= 1e-3;
  * GRAPE: |dF| <= 1e-6, |dg| <= 1e-5, gradient relative L2 <= 1e-4.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_1707_02162_amd import workloads as W

pytestmark = pytest.mark.gpu

N_STEPS = 130
CHUNK = 10
REPROJECT = 64
SAMPLES = (0, 4095)
OBS_TOL = 1e-5
FROB_TOL = 1e-5
BF_TOL = 1e-3


def R():
    from paper_1707_02162_amd import redo
    return redo


def nfrob(A, B):
    return float(np.linalg.norm(np.asarray(A, np.complex128) - B) / math.sqrt(B.shape[-1]))


@pytest.fixture(scope="module")
def headline():
    """The workload, and the oracle's magnetisation series and states at the
    chunk ends for the sampled realisations."""
    p = W.ising_freezing(n=10, B=4096, N=N_STEPS)
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    ref = {}
    for b in SAMPLES:
        xs = O.chain(O.compose_all_redo(p, tab, b), keep=True)
        m = np.array([O.magnetisation(X, p.M) for X in xs[1:]])
        ref[b] = (m, {n: xs[n] for n in range(CHUNK, N_STEPS + 1, CHUNK)} | {N_STEPS: xs[N_STEPS]})
        del xs
    return p, ref


def run_headline(p, precision):
    redo = R()
    t = redo.RedoTable.from_problem(p)
    t.cache_levels()
    if precision == 2:
        t.cache_split_bf16()   # as benchmarked: the cached levels read as pre-split BF16 panels
    cols, vals = W.observable_ell(p.M)
    D = redo.walsh_observable(cols, vals)
    assert D is not None
    u = torch.tensor(p.u).cuda()
    Wt = torch.empty((p.B, p.d, p.d), dtype=torch.complex64, device="cuda")
    mag = torch.empty((p.B, p.N), dtype=torch.float64, device="cuda")
    snaps = {}
    for n0 in range(0, p.N, CHUNK):
        n1 = min(p.N, n0 + CHUNK)
        _, _, m = t.chain(u[:, n0:n1].contiguous(), X0=None if n0 == 0 else Wt, out=Wt, step_offset=n0,
                          reproject_every=REPROJECT, precision=precision, walsh=D)
        mag[:, n0:n1] = m
        snaps[n1] = torch.stack([Wt[b] for b in SAMPLES])
    st, _ = t.device_status()
    assert st in (0, 100)
    out = {}
    for n, s in snaps.items():
        out[n] = redo.walsh_right(s.contiguous()).cpu().numpy()
    return mag.cpu().numpy(), out


def test_headline_chain_3m_cached_walsh_reprojected_vs_oracle(headline):
    p, ref = headline
    mag, snaps = run_headline(p, precision=1)
    for i, b in enumerate(SAMPLES):
        mo, xs = ref[b]
        dm = np.abs(mag[b] - mo)
        errs = {n: nfrob(snaps[n][i], xs[n]) for n in sorted(xs)}
        print(f"\n[headline 3M] realisation {b}: max|dm| {dm.max():.3e} (step {int(dm.argmax()) + 1}); "
              + " ".join(f"{n}:{e:.2e}" for n, e in errs.items()))
        assert dm.max() <= OBS_TOL
        for n, e in errs.items():
            assert e <= FROB_TOL, (b, n, e)


def test_headline_chain_split_bf16_cached_walsh_reprojected_vs_oracle(headline):
    p, ref = headline
    mag, snaps = run_headline(p, precision=2)
    for i, b in enumerate(SAMPLES):
        mo, xs = ref[b]
        dm = np.abs(mag[b] - mo)
        errs = {n: nfrob(snaps[n][i], xs[n]) for n in sorted(xs)}
        print(f"\n[headline split BF16] realisation {b}: max|dm| {dm.max():.3e}; "
              + " ".join(f"{n}:{e:.2e}" for n, e in errs.items()))
        assert dm.max() <= BF_TOL
        assert max(errs.values()) <= BF_TOL


@pytest.mark.parametrize("target", ["haar", "reachable"])
def test_grape_d1024_benchmark_shape_vs_oracle(target):
    """One system of the d = 1024 GRAPE workload (8 steps), every level cached and
    every state kept as in the benchmark.  A Haar target gives F ~ 1/d^2, so a
    second target, the oracle's REDO chain of the pulse at half amplitude, puts F
    at O(1) with a gradient of generic size (close to a maximum of F the gradient
    vanishes and a relative bound on it measures cancellation, not the adjoint)."""
    p = W.c6_grape_1024(B=1, N=8)
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    if target == "reachable":
        q = W.c6_grape_1024(B=1, N=8)
        q.u = (q.u * np.float32(0.5)).astype(np.float32)
        p.U_target = O.chain(O.compose_all_redo(q, tab, 0))[None]
    redo = R()
    t = redo.RedoTable.from_problem(p)
    t.cache_levels()
    F, ov, grad = t.grape(torch.tensor(p.u).cuda(), torch.tensor(p.U_target).cuda(), checkpoint_every=1,
                          precision=1)
    F, ov, grad = F.cpu().numpy(), ov.cpu().numpy(), grad.cpu().numpy()
    Fo, go, gro = O.fidelity_and_gradient(p, 0, model="redo", table=tab)
    rel = np.linalg.norm(grad[0] - gro) / np.linalg.norm(gro)
    print(f"\n[grape d=1024 {target}] F {F[0]:.9f} vs {Fo:.9f} (|dF| {abs(F[0] - Fo):.2e}), "
          f"|dg| {abs(ov[0] - go):.2e}, grad rel L2 {rel:.2e}")
    assert abs(F[0] - Fo) <= 1e-6
    assert abs(ov[0] - go) <= 1e-5
    assert rel <= 1e-4
