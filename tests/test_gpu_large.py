"""GPU parity of the large-d path (d >= 128: batched MFMA complex GEMMs)
against the FP64 oracle.  Tolerances as for the small path:
||dU||_F / sqrt(d) <= 1e-5 (FP32), |dF| <= 1e-6, gradient relative L2 <= 1e-4."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_1707_02162_amd import workloads as W

pytestmark = pytest.mark.gpu

FROB_TOL = 1e-5
FID_TOL = 1e-6
GRAD_TOL = 1e-4


def R():
    from paper_1707_02162_amd import redo
    return redo


def nfrob(A, B):
    return float(np.linalg.norm(np.asarray(A, np.complex128) - B) / math.sqrt(B.shape[-1]))


def generic_problem(d, B, N, seed, phased=False, K=1):
    """Random Hermitian generators and diagonal drift at a dimension that is
    not a power of two (exercises 64-wide tiles and ragged tile counts)."""
    rng = np.random.default_rng(seed)
    S = []
    for _ in range(K):
        A = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
        S.append((A + A.conj().T) / (2 * math.sqrt(d)))
    S = np.stack(S)
    H0 = rng.uniform(-2e4, 2e4, (1, d))
    dt = 1e-6
    scale = 3e4
    if phased:
        raise NotImplementedError
    u = (rng.uniform(-1, 1, (B, N, K)) * scale).astype(np.float32)
    eps = scale / (32 * 32 - 1)
    return W.Problem("generic", d, K, False, H0, True, S, None, dt, eps, 32, 2, u, None, None, None, u_scale=scale)


def test_compose_d128_vs_oracle():
    p = W.nmr_chain(7, 2, 12, 2e-6, 32, 2, 201)
    t = R().RedoTable.from_problem(p)
    U = t.compose(torch.tensor(p.u).cuda()).cpu().numpy()
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    for b in range(p.B):
        steps = O.compose_all_redo(p, tab, b)
        for n in range(p.N):
            assert nfrob(U[b, n], steps[n]) < FROB_TOL


@pytest.mark.parametrize("prec", [0, 1])
def test_chain_d128_ragged_vs_oracle(prec):
    lens = np.array([40, 17, 33], np.int32)
    p = W.nmr_chain(7, 3, 40, 2e-6, 32, 2, 202, lengths=lens, n_drift=2)
    t = R().RedoTable.from_problem(p)
    U, _, _ = t.chain(torch.tensor(p.u).cuda(), n_steps=torch.tensor(lens), precision=prec)
    U = U.cpu().numpy()
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    for b in range(p.B):
        X = O.chain(O.compose_all_redo(p, tab, b))
        assert nfrob(U[b], X) < FROB_TOL, (b, nfrob(U[b], X))


def test_chain_generic_d192_signed_vs_oracle():
    p = generic_problem(192, 3, 30, 203)
    t = R().RedoTable.from_problem(p)
    U, _, _ = t.chain(torch.tensor(p.u).cuda(), reproject_every=8)
    U = U.cpu().numpy()
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    for b in range(p.B):
        X = O.chain(O.compose_all_redo(p, tab, b))
        assert nfrob(U[b], X) < FROB_TOL


def test_chain_generic_two_channels_dense_drift_vs_oracle():
    p = generic_problem(128, 2, 20, 204, K=2)
    rng = np.random.default_rng(5)
    A = rng.normal(size=(128, 128)) + 1j * rng.normal(size=(128, 128))
    p.H0 = ((A + A.conj().T) * 1e3)[None]
    p.drift_is_diag = False
    t = R().RedoTable.from_problem(p)
    U, _, _ = t.chain(torch.tensor(p.u).cuda())
    U = U.cpu().numpy()
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    for b in range(p.B):
        assert nfrob(U[b], O.chain(O.compose_all_redo(p, tab, b))) < FROB_TOL


def test_ising_d128_observable_vs_oracle():
    p = W.ising_freezing(n=7, B=3, N=70)
    t = R().RedoTable.from_problem(p)
    cols, vals = W.observable_ell(p.M)
    U, _, m = t.chain(torch.tensor(p.u).cuda(), observable=(cols, vals), reproject_every=64)
    U, m = U.cpu().numpy(), m.cpu().numpy()
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    for b in range(p.B):
        mo, X = O.magnetisation_series(O.compose_all_redo(p, tab, b), p.M)
        assert nfrob(U[b], X) < FROB_TOL
        assert np.abs(m[b] - mo).max() < 1e-5


def test_chunked_chain_equals_one_call_d128():
    p = W.ising_freezing(n=7, B=2, N=40)
    t = R().RedoTable.from_problem(p)
    u = torch.tensor(p.u).cuda()
    U_all, _, _ = t.chain(u, reproject_every=8)
    U_a, _, _ = t.chain(u[:, :24].contiguous(), reproject_every=8)
    U_b, _, _ = t.chain(u[:, 24:].contiguous(), X0=U_a, reproject_every=8, step_offset=24)
    assert torch.equal(U_all, U_b)


@pytest.mark.parametrize("prec", [0, 1])
def test_grape_d128_phased_vs_oracle(prec):
    """Default schedule at d = 128 (every state kept, traces from the sparse
    pattern of the collective generators), four- and three-product GEMMs;
    every fifth step has zero amplitude, so the q = 0 (Cartesian) derivative
    is exercised too."""
    p = W.nmr_chain(7, 2, 30, 2e-6, 32, 2, 205)
    p.u[:, ::5] = 0.0
    t = R().RedoTable.from_problem(p)
    F, ov, grad = t.grape(torch.tensor(p.u).cuda(), torch.tensor(p.U_target).cuda(), precision=prec)
    F, ov, grad = F.cpu().numpy(), ov.cpu().numpy(), grad.cpu().numpy()
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    for b in range(p.B):
        Fo, go, gro = O.fidelity_and_gradient(p, b, model="redo", table=tab)
        assert abs(F[b] - Fo) < FID_TOL
        assert abs(ov[b] - go) < 1e-5
        assert np.linalg.norm(grad[b] - gro) <= GRAD_TOL * np.linalg.norm(gro)


def test_grape_d512_phased_ragged_vs_oracle():
    """d = 512 (9-spin chain: 9 pattern entries per row and the diagonal, 12 slots of the
    per-step trace kernel), ragged lengths, every state kept."""
    p = W.nmr_chain(9, 2, 6, 2e-6, 32, 2, 206)
    p.n_steps = np.array([6, 4], np.int32)
    p.u[:, ::3] = 0.0
    t = R().RedoTable.from_problem(p)
    F, ov, grad = t.grape(torch.tensor(p.u).cuda(), torch.tensor(p.U_target).cuda(),
                          n_steps=torch.tensor(p.n_steps), checkpoint_every=1)
    F, ov, grad = F.cpu().numpy(), ov.cpu().numpy(), grad.cpu().numpy()
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    for b in range(p.B):
        Fo, go, gro = O.fidelity_and_gradient(p, b, model="redo", table=tab)
        nb = int(p.n_steps[b])
        assert abs(F[b] - Fo) < FID_TOL
        assert abs(ov[b] - go) < 1e-5
        assert np.linalg.norm(grad[b, :nb] - gro) <= GRAD_TOL * np.linalg.norm(gro)
        assert np.all(grad[b, nb:] == 0)


def test_grape_d128_signed_ragged_vs_oracle():
    p = W.ising_freezing(n=7, B=2, N=25)
    p.n_steps = np.array([25, 14], np.int32)
    p.U_target = np.stack([W.haar_unitary(128, W.rng(33, 2, b)) for b in range(2)])
    t = R().RedoTable.from_problem(p)
    F, ov, grad = t.grape(torch.tensor(p.u).cuda(), torch.tensor(p.U_target).cuda(),
                          n_steps=torch.tensor(p.n_steps), checkpoint_every=4)
    F, grad = F.cpu().numpy(), grad.cpu().numpy()
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    for b in range(p.B):
        Fo, go, gro = O.fidelity_and_gradient(p, b, model="redo", table=tab)
        nb = int(p.n_steps[b])
        assert abs(F[b] - Fo) < FID_TOL
        assert np.linalg.norm(grad[b, :nb] - gro) <= GRAD_TOL * np.linalg.norm(gro)
        assert np.all(grad[b, nb:] == 0)


def test_grape_memory_schedules_agree():
    """The same 7-qubit problem with every state kept (checkpoint 1: the two
    scans side by side, FP64 traces at the generators' pattern) and with
    checkpoints every 6 or 4 steps (recomputed segments, traces of the FP32
    product Y): the forward chain is the same sequence of products, so F is
    bitwise equal; recomputation is exact, so the two checkpointed runs agree
    bitwise; the two trace routes differ by FP32 rounding of Y."""
    p = W.nmr_chain(7, 2, 20, 2e-6, 32, 2, 206)
    p.n_steps = np.array([20, 13], np.int32)
    t = R().RedoTable.from_problem(p)
    u, Uf, ns = torch.tensor(p.u).cuda(), torch.tensor(p.U_target).cuda(), torch.tensor(p.n_steps)
    F1, _, g1 = t.grape(u, Uf, n_steps=ns, checkpoint_every=1)
    F2, _, g2 = t.grape(u, Uf, n_steps=ns, checkpoint_every=6)
    F3, _, g3 = t.grape(u, Uf, n_steps=ns, checkpoint_every=4)
    assert torch.equal(F1, F2) and torch.equal(F2, F3)
    assert torch.equal(g2, g3)
    assert float((g1 - g2).norm() / g2.norm()) < 1e-5
    assert torch.all(g1[1, 13:] == 0)


def test_grape_d128_dense_generator_full_storage_vs_oracle():
    """Dense random generator (no sparse pattern): with every state kept the
    traces come from batched products Y = X L^dag."""
    p = generic_problem(128, 2, 12, 215)
    p.U_target = np.stack([W.haar_unitary(128, W.rng(215, 2, b)) for b in range(2)])
    t = R().RedoTable.from_problem(p)
    F, ov, grad = t.grape(torch.tensor(p.u).cuda(), torch.tensor(p.U_target).cuda(), checkpoint_every=1)
    F, grad = F.cpu().numpy(), grad.cpu().numpy()
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    for b in range(p.B):
        Fo, go, gro = O.fidelity_and_gradient(p, b, model="redo", table=tab)
        assert abs(F[b] - Fo) < FID_TOL
        assert np.linalg.norm(grad[b] - gro) <= GRAD_TOL * np.linalg.norm(gro)


@pytest.mark.parametrize("width", [1, 13])
def test_grape_d128_pattern_widths_vs_oracle(width):
    """Generators with 1 entry per row (spin 0 alone: the per-step trace kernel with 4
    slots) and with 13 (collective X plus nearest-neighbour XX terms: 16 slots, the
    row-block trace kernel), every state kept."""
    n, d = 7, 128
    S = W.collective(n, [0], "x")
    if width == 13:
        S = W.collective(n, range(n), "x")
        for q in range(n - 1):
            S = S + W.collective(n, [q], "x") @ W.collective(n, [q + 1], "x")
    assert int((np.abs(S) > 0).sum(1).max()) == width
    p = generic_problem(d, 2, 10, 216 + width)
    p.S = S[None]
    p.U_target = np.stack([W.haar_unitary(d, W.rng(216, 3, b)) for b in range(2)])
    t = R().RedoTable.from_problem(p)
    F, ov, grad = t.grape(torch.tensor(p.u).cuda(), torch.tensor(p.U_target).cuda(), checkpoint_every=1)
    F, grad = F.cpu().numpy(), grad.cpu().numpy()
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    for b in range(p.B):
        Fo, go, gro = O.fidelity_and_gradient(p, b, model="redo", table=tab)
        assert abs(F[b] - Fo) < FID_TOL
        assert np.linalg.norm(grad[b] - gro) <= GRAD_TOL * np.linalg.norm(gro)


# ---------------------------------------------------------------- full size
def test_ising_d1024_special_cases_full_dimension():
    """At d = 1024: without coupling the magnetisation stays 1 for any noisy
    drive; without drive it follows [2 cos Jt + (n-2) cos^2 Jt]/n.  Bound:
    each FP32 product with K = 1024 carries ~u sqrt(2d) ~ 3e-6 relative error,
    48 of them random-walk to ~2e-5 in ||dX||_F / sqrt(d), and |dm| <~ 2 of
    that, so 1e-4."""
    p = W.ising_freezing(n=10, B=2, N=24, J=0.0)
    t = R().RedoTable.from_problem(p)
    cols, vals = W.observable_ell(p.M)
    _, _, m = t.chain(torch.tensor(p.u).cuda(), observable=(cols, vals))
    assert np.abs(m.cpu().numpy() - 1.0).max() < 1e-4
    q = W.ising_freezing(n=10, B=1, N=24)
    q.u[:] = 0.0
    t2 = R().RedoTable.from_problem(q)
    _, _, m2 = t2.chain(torch.tensor(q.u).cuda(), observable=(cols, vals))
    J = q.meta["J"]
    tt = np.arange(1, 25) * q.dt
    want = (2 * np.cos(J * tt) + 8 * np.cos(J * tt) ** 2) / 10
    assert np.abs(m2.cpu().numpy()[0] - want).max() < 1e-4


@pytest.mark.parametrize("prec", [0, 1])
def test_ising_d1024_full_batch_sampled_vs_oracle(prec):
    """The benchmark's launch shape (4096 realisations x d = 1024, one call
    per step window) on its first steps, four- and three-product GEMMs;
    sampled realisations against the oracle."""
    n_steps = 3
    p = W.ising_freezing(n=10, B=4096, N=n_steps)
    t = R().RedoTable.from_problem(p)
    cols, vals = W.observable_ell(p.M)
    U, _, m = t.chain(torch.tensor(p.u).cuda(), observable=(cols, vals), precision=prec)
    torch.cuda.synchronize()
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    for b in (0, 4095):
        mo, X = O.magnetisation_series(O.compose_all_redo(p, tab, b), p.M)
        assert nfrob(U[b].cpu().numpy(), X) < FROB_TOL
        assert np.abs(m[b].cpu().numpy() - mo).max() < 1e-5


# ---------------------------------------------------------------- level cache (process 3)
def test_level_cache_full_range_chain_vs_oracle():
    lens = np.array([30, 11], np.int32)
    p = W.ising_freezing(n=7, B=2, N=30)
    t = R().RedoTable.from_problem(p)
    t.cache_levels()
    cols, vals = W.observable_ell(p.M)
    U, _, m = t.chain(torch.tensor(p.u).cuda(), n_steps=torch.tensor(lens), observable=(cols, vals),
                      reproject_every=7)
    U, m = U.cpu().numpy(), m.cpu().numpy()
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    for b in range(p.B):
        mo, X = O.magnetisation_series(O.compose_all_redo(p, tab, b, n_steps=int(lens[b])), p.M)
        assert nfrob(U[b], X) < FROB_TOL
        assert np.abs(m[b, :lens[b]] - mo).max() < 1e-5


def test_level_cache_partial_range_phased_vs_oracle():
    """Levels inside the cached range use one composed factor, the others the
    digit products; both mixed within one step batch."""
    p = W.nmr_chain(7, 3, 25, 2e-6, 32, 2, 207, n_drift=2)
    t = R().RedoTable.from_problem(p)
    t.cache_levels(200, 700)
    U, _, _ = t.chain(torch.tensor(p.u).cuda())
    Uc = t.compose(torch.tensor(p.u[:, :6]).cuda()).cpu().numpy()
    U = U.cpu().numpy()
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    for b in range(p.B):
        steps = O.compose_all_redo(p, tab, b)
        assert nfrob(U[b], O.chain(steps)) < FROB_TOL
        for n in range(6):
            # one FP32 rounding of the composed level and of each phase factor
            assert nfrob(Uc[b, n], steps[n]) < 1e-6


def test_level_cache_grape_vs_oracle():
    p = W.nmr_chain(7, 1, 24, 2e-6, 32, 2, 208)
    t = R().RedoTable.from_problem(p)
    t.cache_levels()
    F, ov, grad = t.grape(torch.tensor(p.u).cuda(), torch.tensor(p.U_target).cuda())
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    Fo, go, gro = O.fidelity_and_gradient(p, 0, model="redo", table=tab)
    assert abs(F[0].item() - Fo) < FID_TOL
    g = grad[0].cpu().numpy()
    assert np.linalg.norm(g - gro) <= GRAD_TOL * np.linalg.norm(gro)


def test_level_cache_d1024_special_case_and_sampled():
    p = W.ising_freezing(n=10, B=64, N=24, J=0.0)
    t = R().RedoTable.from_problem(p)
    t.cache_levels()
    cols, vals = W.observable_ell(p.M)
    _, _, m = t.chain(torch.tensor(p.u).cuda(), observable=(cols, vals))
    # FP32 products with K = 1024: ~u sqrt(2d) relative error each, random-walking over
    # 24 steps, and |dm| <~ 2 ||dX||_F / sqrt(d): bound 1e-4
    assert np.abs(m.cpu().numpy() - 1.0).max() < 1e-4


# ---------------------------------------------------------------- plain per-step exponential (comparison point)
def _exact_steps(p, b):
    V, H0m = O.drift_propagator(p.H0[b % p.n_drift], p.dt, p.drift_is_diag), (
        np.diag(p.H0[b % p.n_drift]).astype(complex) if p.drift_is_diag else p.H0[b % p.n_drift])
    g = p.g if p.phased else None
    return [O.step_exact(H0m, p.S, g, p.u[b, n].astype(np.float64), p.dt) for n in range(int(p.lengths()[b]))]


def test_expm_chain_phased_d128_vs_oracle_exact():
    lens = np.array([20, 9], np.int32)
    p = W.nmr_chain(7, 2, 20, 2e-6, 32, 2, 209, lengths=lens, n_drift=2)
    t = R().RedoTable.from_problem(p)
    U, _ = t.expm_chain(torch.tensor(p.u).cuda(), n_steps=torch.tensor(lens))
    U = U.cpu().numpy()
    for b in range(p.B):
        assert nfrob(U[b], O.chain(_exact_steps(p, b))) < FROB_TOL


def test_expm_chain_signed_observable_d128_vs_oracle_exact():
    p = W.ising_freezing(n=7, B=2, N=30)
    t = R().RedoTable.from_problem(p)
    cols, vals = W.observable_ell(p.M)
    U, m = t.expm_chain(torch.tensor(p.u).cuda(), observable=(cols, vals), reproject_every=16)
    U, m = U.cpu().numpy(), m.cpu().numpy()
    for b in range(p.B):
        mo, X = O.magnetisation_series(_exact_steps(p, b), p.M)
        assert nfrob(U[b], X) < FROB_TOL
        assert np.abs(m[b] - mo).max() < 1e-5


def test_expm_grape_d128_vs_oracle_first_order():
    p = W.nmr_chain(7, 1, 16, 2e-6, 32, 2, 210)
    t = R().RedoTable.from_problem(p)
    F, ov, grad = t.expm_grape(torch.tensor(p.u).cuda(), torch.tensor(p.U_target).cuda())
    Fo, go, gro = O.fidelity_and_gradient(p, 0, model="exact_first_order")
    assert abs(F[0].item() - Fo) < FID_TOL
    g = grad[0].cpu().numpy()
    assert np.linalg.norm(g - gro) <= GRAD_TOL * np.linalg.norm(gro)


# ---------------------------------------------------------------- split-BF16 products
BF_TOL = 1e-3   # split-BF16 chain including its periodic re-projection, ||dU||_F / sqrt(d)


def test_bf16x3_compose_and_chain_d128_vs_oracle():
    p = W.nmr_chain(7, 2, 64, 2e-6, 32, 2, 211)
    t = R().RedoTable.from_problem(p)
    u = torch.tensor(p.u).cuda()
    Uc = t.compose(u[:, :4].contiguous(), precision=2).cpu().numpy()
    U, _, _ = t.chain(u, precision=2, reproject_every=16)
    U = U.cpu().numpy()
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    for b in range(p.B):
        steps = O.compose_all_redo(p, tab, b)
        for n in range(4):
            # one split product: the dropped lo*lo term and the lo rounding, ~2^-16 relative
            assert nfrob(Uc[b, n], steps[n]) < 5e-5
        assert nfrob(U[b], O.chain(steps)) < BF_TOL


def test_bf16x3_ising_d1024_sampled_vs_oracle():
    p = W.ising_freezing(n=10, B=16, N=40)
    t = R().RedoTable.from_problem(p)
    t.cache_levels()
    cols, vals = W.observable_ell(p.M)
    U, _, m = t.chain(torch.tensor(p.u).cuda(), precision=2, reproject_every=16, observable=(cols, vals))
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    mo, X = O.magnetisation_series(O.compose_all_redo(p, tab, 5), p.M)
    assert nfrob(U[5].cpu().numpy(), X) < BF_TOL
    assert np.abs(m[5].cpu().numpy() - mo).max() < BF_TOL


def test_large_batch_and_single_calls_bitwise_equal():
    """A batch of instances gives bitwise the results of one call per instance."""
    p = W.nmr_chain(7, 3, 12, 2e-6, 32, 2, 212)
    t = R().RedoTable.from_problem(p)
    u = torch.tensor(p.u).cuda()
    U_all, _, _ = t.chain(u, reproject_every=5)
    for b in range(p.B):
        U1, _, _ = t.chain(u[b:b + 1].contiguous(), reproject_every=5)
        assert torch.equal(U1[0], U_all[b])


# ---------------------------------------------------------------- Strang splitting (NEXT row f1)
def _strang(p):
    return W.Problem(**{**p.__dict__, "splitting": "strang"})


@pytest.mark.parametrize("cache", [False, True])
def test_strang_chain_d128_vs_oracle(cache):
    p = _strang(W.nmr_chain(7, 2, 24, 2e-6, 32, 2, 221))
    t = R().RedoTable.from_problem(p)
    if cache:
        t.cache_levels()
    U, _, _ = t.chain(torch.tensor(p.u).cuda())
    U = U.cpu().numpy()
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    for b in range(p.B):
        assert nfrob(U[b], O.chain(O.compose_all_redo(p, tab, b))) < FROB_TOL


@pytest.mark.parametrize("checkpoint", [1, 5])
def test_strang_grape_d128_vs_oracle(checkpoint):
    """Stored states with sparse FP64 traces (1) and recomputed segments with
    dense traces (5): the traces see V(dt/2) S V(dt/2)^dag."""
    p = W.nmr_chain(7, 2, 20, 2e-6, 32, 2, 222)
    p.u[:, ::6] = 0.0
    p.n_steps = np.array([20, 13], np.int32)
    p = _strang(p)
    t = R().RedoTable.from_problem(p)
    F, ov, grad = t.grape(torch.tensor(p.u).cuda(), torch.tensor(p.U_target).cuda(),
                          n_steps=torch.tensor(p.n_steps), checkpoint_every=checkpoint)
    F, grad = F.cpu().numpy(), grad.cpu().numpy()
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    for b in range(p.B):
        Fo, go, gro = O.fidelity_and_gradient(p, b, model="redo", table=tab)
        nb = int(p.n_steps[b])
        assert abs(F[b] - Fo) < FID_TOL
        assert np.linalg.norm(grad[b, :nb] - gro) <= GRAD_TOL * np.linalg.norm(gro)


def test_strang_signed_grape_d128_vs_oracle():
    p = W.ising_freezing(n=7, B=1, N=16)
    p.U_target = W.haar_unitary(128, W.rng(34, 2, 0))[None]
    p = _strang(p)
    t = R().RedoTable.from_problem(p)
    F, ov, grad = t.grape(torch.tensor(p.u).cuda(), torch.tensor(p.U_target).cuda())
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    Fo, go, gro = O.fidelity_and_gradient(p, 0, model="redo", table=tab)
    assert abs(F[0].item() - Fo) < FID_TOL
    g = grad[0].cpu().numpy()
    assert np.linalg.norm(g - gro) <= GRAD_TOL * np.linalg.norm(gro)


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_chain_large_batch_tiles_d128_vs_oracle(prec):
    """Enough instances for the 128 x 64 tiles (4M, 3M and split BF16) with a
    ragged length and the observable; sampled instances against the oracle."""
    B, N = 300, 12
    lens = np.full(B, N, np.int32)
    lens[7] = 5
    p = W.ising_freezing(n=7, B=B, N=N)
    t = R().RedoTable.from_problem(p)
    cols, vals = W.observable_ell(p.M)
    U, _, m = t.chain(torch.tensor(p.u).cuda(), n_steps=torch.tensor(lens), observable=(cols, vals), precision=prec)
    U, m = U.cpu().numpy(), m.cpu().numpy()
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    for b in (0, 7, B - 1):
        mo, X = O.magnetisation_series(O.compose_all_redo(p, tab, b, n_steps=int(lens[b])), p.M)
        tol = BF_TOL if prec == 2 else FROB_TOL
        assert nfrob(U[b], X) < tol
        assert np.abs(m[b, :lens[b]] - mo).max() < (BF_TOL if prec == 2 else 1e-5)


# ---------------------------------------------------------------- Newton-Schulz re-projection
def _perturbed_unitaries(d, B, delta, seed):
    """Haar unitaries times (I + delta G), G Hermitian with ||G||_F / sqrt(d) = 1:
    ||X^dag X - I||_F / sqrt(d) ~ 2 delta."""
    gen = np.random.default_rng(seed)
    X = np.empty((B, d, d), np.complex128)
    for b in range(B):
        A = gen.normal(size=(d, d)) + 1j * gen.normal(size=(d, d))
        G = (A + A.conj().T) / 2
        G *= math.sqrt(d) / np.linalg.norm(G)
        X[b] = W.haar_unitary(d, gen) @ (np.eye(d) + delta * G)
    return X


def _unitarity(X):
    d = X.shape[-1]
    X = np.asarray(X, np.complex128)
    return float(np.linalg.norm(X.conj().T @ X - np.eye(d)) / math.sqrt(d))


# small batches run the Gram product X^dag X on 64 x 64 tiles, B = 64 at d = 256 on 128 x 64
REPROJ_CASES = [("chain", 7, 3, 0), ("chain", 7, 3, 1), ("chain", 7, 3, 2), ("chain", 8, 64, 0),
                ("chain", 8, 64, 1), ("chain", 8, 64, 2), ("chain", 10, 2, 1), ("kron", 8, 64, 1),
                ("expm", 7, 3, 1)]


@pytest.mark.parametrize("kind, n, B, prec", REPROJ_CASES)
def test_reprojection_step_vs_newton_schulz(kind, n, B, prec):
    """One step from states about 4e-4 off unitarity, re-projected after it, against
    the Newton-Schulz polar step Y (3I - Y^dag Y) / 2 of Y = U_1 X0 in FP64 (U_1 the
    oracle's step; the exact exponential for the comparison-point chain).  The step
    must also take the state back to unitarity (FP32: below 1e-5; split BF16, whose
    Gram product carries its own ~1e-5 error: below 1e-4)."""
    p = W.ising_freezing(n=n, B=B, N=1)
    d = p.d
    X0 = _perturbed_unitaries(d, B, 2e-4, 700 + n).astype(np.complex64)
    t = R().RedoTable.from_problem(p)
    u = torch.tensor(p.u).cuda()
    X0t = torch.tensor(X0).cuda()
    if kind == "chain":
        U, _, _ = t.chain(u, precision=prec, X0=X0t, reproject_every=1)
    elif kind == "kron":
        U, _ = t.kron_chain(u, X0=X0t, reproject_every=1)
    else:
        U, _ = t.expm_chain(u, precision=prec, X0=X0t, reproject_every=1)
    U = U.cpu().numpy()
    tab = None if kind == "expm" else O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    tol, unit_tol = (1e-3, 1e-4) if prec == 2 else (FROB_TOL, 1e-5)
    for b in sorted({0, B // 2, B - 1}):
        step = _exact_steps(p, b)[0] if kind == "expm" else O.compose_all_redo(p, tab, b)[0]
        Y = step @ X0[b].astype(np.complex128)
        Xe = Y @ (3 * np.eye(d) - Y.conj().T @ Y) / 2
        assert _unitarity(Y) > 3e-4
        assert nfrob(U[b], Xe) < tol, (b, nfrob(U[b], Xe))
        assert _unitarity(U[b]) < unit_tol, (b, _unitarity(U[b]))


@pytest.mark.parametrize("prec", [1, 2])
def test_reprojection_skips_finished_instances(prec):
    """Ragged lengths: an instance whose chain has ended (length 0 here) is neither
    stepped nor re-projected, so it keeps its X0 bit for bit; its neighbours in the
    same Gram and correction launches are re-projected (B = 64 at d = 256: 128 x 64
    tiles)."""
    p = W.ising_freezing(n=8, B=64, N=1)
    X0 = _perturbed_unitaries(p.d, p.B, 2e-4, 731).astype(np.complex64)
    lens = np.ones(p.B, np.int32)
    lens[1::3] = 0
    t = R().RedoTable.from_problem(p)
    U, _, _ = t.chain(torch.tensor(p.u).cuda(), n_steps=torch.tensor(lens), precision=prec,
                      X0=torch.tensor(X0).cuda(), reproject_every=1)
    U = U.cpu().numpy()
    for b in range(p.B):
        if lens[b] == 0:
            assert np.array_equal(U[b], X0[b]), b
        else:
            assert _unitarity(U[b]) < (1e-4 if prec == 2 else 1e-5), (b, _unitarity(U[b]))
