"""The right Walsh frame through the C ABI: the transform against numpy's
Hadamard products, and the REDO and structure-aware chains carried as W = X Hn
with the one-pass observable against the FP64 oracle and against the same
chains in the computational basis.  Tolerances as for the chains:
||dU||_F / sqrt(d) <= 1e-5 (U recovered from W by the transform), |dm| <= 1e-5."""
import math

import numpy as np
import pytest
import torch
from scipy.linalg import hadamard

import oracle as O
from paper_1707_02162_amd import workloads as W

pytestmark = pytest.mark.gpu

FROB_TOL = 1e-5
OBS_TOL = 1e-5


def R():
    from paper_1707_02162_amd import redo
    return redo


def nfrob(A, B):
    return float(np.linalg.norm(np.asarray(A, np.complex128) - B) / math.sqrt(B.shape[-1]))


def to_x(Wt):
    """W -> X (the transform is its own inverse), on a copy."""
    return R().walsh_right(Wt.clone()).cpu().numpy()


@pytest.mark.parametrize("d", [128, 1024, 4096])
def test_walsh_right_matches_hadamard_and_is_an_involution(d):
    rng = np.random.default_rng(d)
    B = 2 if d < 4096 else 1
    X = (rng.normal(size=(B, d, d)) + 1j * rng.normal(size=(B, d, d))).astype(np.complex64)
    Hn = hadamard(d).astype(np.float64) / math.sqrt(d)
    Xt = torch.tensor(X).cuda()
    R().walsh_right(Xt)
    Y = Xt.cpu().numpy()
    for b in range(B):
        ref = X[b].astype(np.complex128) @ Hn
        assert np.abs(Y[b] - ref).max() <= 1e-5 * np.abs(ref).max()
    R().walsh_right(Xt)
    assert np.abs(Xt.cpu().numpy() - X).max() <= 1e-5 * np.abs(X).max()


def test_walsh_chain_ising_d128_vs_oracle():
    p = W.ising_freezing(n=7, B=3, N=70)
    t = R().RedoTable.from_problem(p)
    cols, vals = W.observable_ell(p.M)
    D = R().walsh_observable(cols, vals)
    assert D is not None
    Wt, _, m = t.chain(torch.tensor(p.u).cuda(), reproject_every=64, walsh=D)
    U, m = to_x(Wt), m.cpu().numpy()
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    for b in range(p.B):
        mo, X = O.magnetisation_series(O.compose_all_redo(p, tab, b), p.M)
        assert nfrob(U[b], X) < FROB_TOL
        assert np.abs(m[b] - mo).max() < OBS_TOL


def test_walsh_chain_equals_basis_chain_phased_ragged_strang_d256():
    """Phased channels, two drifts, ragged lengths and the Strang splitting: the Walsh
    frame gives the chain of the computational basis (up to FP32 rounding), and two
    calls with a carried state equal one call bit for bit."""
    lens = np.array([16, 9, 12], np.int32)
    p = W.nmr_chain(8, 3, 16, 2e-6, 32, 2, 311, lengths=lens, n_drift=2)
    p.splitting = "strang"
    t = R().RedoTable.from_problem(p)
    M = W.collective(8, range(8), "x")
    cols, vals = W.observable_ell(M)
    D = R().walsh_observable(cols, vals)
    u = torch.tensor(p.u).cuda()
    ns = torch.tensor(lens)
    Ub, _, mb = t.chain(u, n_steps=ns, observable=(cols, vals), reproject_every=8)
    Wt, _, mw = t.chain(u, n_steps=ns, reproject_every=8, walsh=D)
    assert nfrob(to_x(Wt), Ub.cpu().numpy().astype(np.complex128)) < FROB_TOL
    for b in range(p.B):
        assert np.abs(mw[b, :lens[b]].cpu().numpy() - mb[b, :lens[b]].cpu().numpy()).max() < OBS_TOL
    Wa, _, ma = t.chain(u[:, :10].contiguous(), n_steps=ns.clamp(max=10), reproject_every=8, walsh=D)
    Wb, _, mb2 = t.chain(u[:, 10:].contiguous(), n_steps=(ns - 10).clamp(min=0), X0=Wa,
                         reproject_every=8, step_offset=10, walsh=D)
    assert torch.equal(Wb, Wt)
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    for b in range(p.B):
        mo, X = O.magnetisation_series(O.compose_all_redo(p, tab, b), M)
        assert np.abs(mw[b, :lens[b]].cpu().numpy() - mo).max() < OBS_TOL


@pytest.mark.parametrize("quantised", [True, False])
def test_walsh_kron_chain_d256_vs_oracle(quantised):
    p = W.ising_freezing(n=8, B=2, N=20)
    t = R().RedoTable.from_problem(p)
    cols, vals = W.observable_ell(p.M)
    D = R().walsh_observable(cols, vals)
    u = torch.tensor(p.u).cuda()
    Wt, m = t.kron_chain(u, quantised=quantised, reproject_every=8, walsh=D)
    Uk, mk = t.kron_chain(u, quantised=quantised, observable=(cols, vals), reproject_every=8)
    U, m = to_x(Wt), m.cpu().numpy()
    assert nfrob(U, Uk.cpu().numpy().astype(np.complex128)) < FROB_TOL
    assert np.abs(m - mk.cpu().numpy()).max() < OBS_TOL
    if quantised:
        tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
        for b in range(p.B):
            mo, X = O.magnetisation_series(O.compose_all_redo(p, tab, b), p.M)
            assert nfrob(U[b], X) < FROB_TOL
            assert np.abs(m[b] - mo).max() < OBS_TOL


def test_walsh_chain_ising_d1024_full_batch_sampled_vs_oracle():
    """The benchmark's launch shape (4096 realisations x d = 1024), first steps, both
    chains; sampled realisations against the oracle."""
    p = W.ising_freezing(n=10, B=4096, N=3)
    t = R().RedoTable.from_problem(p)
    t.cache_levels()
    cols, vals = W.observable_ell(p.M)
    D = R().walsh_observable(cols, vals)
    u = torch.tensor(p.u).cuda()
    Wr, _, mr = t.chain(u, precision=1, walsh=D)
    Wk, mk = t.kron_chain(u, walsh=D)
    torch.cuda.synchronize()
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    for b in (0, 4095):
        mo, X = O.magnetisation_series(O.compose_all_redo(p, tab, b), p.M)
        for Wt, m in ((Wr, mr), (Wk, mk)):
            assert nfrob(to_x(Wt[b:b + 1])[0], X) < FROB_TOL
            assert np.abs(m[b].cpu().numpy() - mo).max() < OBS_TOL


def test_walsh_argument_errors():
    redo = R()
    p = W.ising_freezing(n=7, B=2, N=3)
    t = redo.RedoTable.from_problem(p)
    cols, vals = W.observable_ell(p.M)
    u = torch.tensor(p.u).cuda()
    U = torch.empty((2, p.d, p.d), dtype=torch.complex64, device="cuda")
    obs = torch.empty((2, 3), dtype=torch.float64, device="cuda")
    ws = t.workspace(redo.OP_CHAIN, 2, 3)
    P = redo._ptr
    # an observable series without an observable
    assert redo.lib().redo_chain_propagator_walsh(t._h, 0, P(u), None, 2, 3, 0, 0, None, P(U), None, P(obs),
                                                  P(ws), ws.numel(), None) == 1
    # an observable of another dimension
    q8 = W.ising_freezing(n=8, B=1, N=2)
    D8 = redo.walsh_observable(*W.observable_ell(q8.M))
    assert redo.lib().redo_chain_propagator_walsh(t._h, 0, P(u), None, 2, 3, 0, 0, None, P(U), D8._h, P(obs),
                                                  P(ws), ws.numel(), None) == 1
    with pytest.raises(ValueError):
        t.chain(u, walsh=D8)
    # a list observable beside a Walsh observable
    D7 = redo.walsh_observable(cols, vals)
    with pytest.raises(ValueError):
        t.chain(u, observable=(cols, vals), walsh=D7)
    # d = 64 and d = 4096 tables: outside the Walsh frame's range
    q = W.ising_freezing(n=6, B=1, N=2)
    with pytest.raises(redo.RedoError, match="2048"):
        redo.RedoTable.from_problem(q).chain(torch.tensor(q.u).cuda(), walsh=True)
    with pytest.raises(redo.RedoError, match="power of two"):
        redo.walsh_right(torch.empty((1, 192, 192), dtype=torch.complex64, device="cuda"))
    torch.cuda.synchronize()


def test_walsh_expm_chain_equals_basis_chain_d128():
    """The comparison point's chain in the Walsh frame: the same states and magnetisation
    as in the computational basis (up to FP32 rounding)."""
    p = W.ising_freezing(n=7, B=2, N=12)
    t = R().RedoTable.from_problem(p)
    cols, vals = W.observable_ell(p.M)
    D = R().walsh_observable(cols, vals)
    u = torch.tensor(p.u).cuda()
    Ub, mb = t.expm_chain(u, observable=(cols, vals), reproject_every=8)
    Wt, mw = t.expm_chain(u, reproject_every=8, walsh=D)
    assert nfrob(to_x(Wt), Ub.cpu().numpy().astype(np.complex128)) < FROB_TOL
    assert np.abs(mw.cpu().numpy() - mb.cpu().numpy()).max() < OBS_TOL


def test_walsh_chains_d2048_equal_basis_chains():
    """The largest Walsh-frame size (d = 2048: the 8-column strip is 128 KiB of LDS, eight
    rows per lane): REDO and structure-aware chains against their computational-basis
    runs (themselves checked against the oracle at smaller d)."""
    p = W.ising_freezing(n=11, B=2, N=3)
    t = R().RedoTable.from_problem(p)
    cols, vals = W.observable_ell(p.M)
    D = R().walsh_observable(cols, vals)
    u = torch.tensor(p.u).cuda()
    Ub, _, mb = t.chain(u, observable=(cols, vals), precision=1)
    Wt, _, mw = t.chain(u, precision=1, walsh=D)
    assert nfrob(to_x(Wt), Ub.cpu().numpy().astype(np.complex128)) < FROB_TOL
    assert np.abs(mw.cpu().numpy() - mb.cpu().numpy()).max() < OBS_TOL
    Uk, mk = t.kron_chain(u, observable=(cols, vals))
    Wk, mkw = t.kron_chain(u, walsh=D)
    assert nfrob(to_x(Wk), Uk.cpu().numpy().astype(np.complex128)) < FROB_TOL
    assert np.abs(mkw.cpu().numpy() - mk.cpu().numpy()).max() < OBS_TOL


def test_walsh_kron_d1024_fused_observable_with_reprojection_and_ragged():
    """At d = 1024 the structure-aware step carries the Walsh-frame observable in the same
    launch, except on re-projection steps (separate pass after the re-projection): both
    kinds of step, ragged lengths, against the computational-basis chain."""
    p = W.ising_freezing(n=10, B=3, N=9)
    lens = torch.tensor([9, 5, 8], dtype=torch.int32)
    t = R().RedoTable.from_problem(p)
    cols, vals = W.observable_ell(p.M)
    D = R().walsh_observable(cols, vals)
    u = torch.tensor(p.u).cuda()
    Uk, mk = t.kron_chain(u, n_steps=lens, observable=(cols, vals), reproject_every=4)
    Wk, mw = t.kron_chain(u, n_steps=lens, reproject_every=4, walsh=D)
    assert nfrob(to_x(Wk), Uk.cpu().numpy().astype(np.complex128)) < FROB_TOL
    for b in range(3):
        nb = int(lens[b])
        assert np.abs(mw[b, :nb].cpu().numpy() - mk[b, :nb].cpu().numpy()).max() < OBS_TOL
