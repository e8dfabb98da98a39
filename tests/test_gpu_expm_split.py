"""The equal-result comparison point (the REDO chain's split model with each control
factor an exponential at the coarse-grained amplitude, Sec. III split of Eq. propUn,
Sec. II Eq. cgrain) against the REDO chain and the oracle's REDO chain: the table
product equals the exponential at the quantised amplitude, so the two methods give the
same result to FP32 rounding (||dU||_F / sqrt(d) <= 1e-5, |dm| <= 1e-5)."""
import math

import numpy as np
import pytest
import torch

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


@pytest.mark.parametrize("prec", [0, 1])
def test_split_exponential_chain_equals_redo_d128(prec):
    lens = np.array([24, 11, 24], np.int32)
    p = W.ising_freezing(n=7, B=3, N=24)
    t = R().RedoTable.from_problem(p)
    u = torch.tensor(p.u).cuda()
    ns = torch.tensor(lens)
    Ue, _ = t.expm_split_chain(u, n_steps=ns, precision=prec, reproject_every=8)
    Ur, _, _ = t.chain(u, n_steps=ns, precision=prec, reproject_every=8)
    Ue, Ur = Ue.cpu().numpy(), Ur.cpu().numpy()
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    for b in range(p.B):
        X = O.chain(O.compose_all_redo(p, tab, b, n_steps=int(lens[b])))
        assert nfrob(Ue[b], X) < FROB_TOL
        assert nfrob(Ue[b], Ur[b].astype(np.complex128)) < FROB_TOL


def test_split_exponential_walsh_observable_d128():
    p = W.ising_freezing(n=7, B=2, N=30)
    t = R().RedoTable.from_problem(p)
    cols, vals = W.observable_ell(p.M)
    D = R().walsh_observable(cols, vals)
    u = torch.tensor(p.u).cuda()
    We, me = t.expm_split_chain(u, reproject_every=16, walsh=D)
    me = me.cpu().numpy()
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    for b in range(p.B):
        mo, X = O.magnetisation_series(O.compose_all_redo(p, tab, b), p.M)
        assert np.abs(me[b] - mo).max() < OBS_TOL
        assert nfrob(R().walsh_right(We[b:b + 1].clone()).cpu().numpy()[0], X) < FROB_TOL


def test_split_exponential_headline_shape_sampled():
    """4096 realisations x d = 1024, three-product GEMMs, Walsh frame with the observable:
    sampled realisations against the oracle's REDO chain."""
    p = W.ising_freezing(n=10, B=4096, N=2)
    t = R().RedoTable.from_problem(p)
    cols, vals = W.observable_ell(p.M)
    D = R().walsh_observable(cols, vals)
    u = torch.tensor(p.u).cuda()
    We, me = t.expm_split_chain(u, precision=1, walsh=D)
    torch.cuda.synchronize()
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    for b in (0, 4095):
        mo, X = O.magnetisation_series(O.compose_all_redo(p, tab, b), p.M)
        assert np.abs(me[b].cpu().numpy() - mo).max() < OBS_TOL
        assert nfrob(R().walsh_right(We[b:b + 1].clone()).cpu().numpy()[0], X) < FROB_TOL


def test_split_exponential_refusals():
    redo = R()
    q = W.nmr_chain(7, 1, 4, 2e-6, 32, 2, 501)
    tq = redo.RedoTable.from_problem(q)
    with pytest.raises(redo.RedoError, match="signed channel"):
        tq.expm_split_chain(torch.tensor(q.u).cuda())
    p = W.ising_freezing(n=7, B=1, N=2)
    t = redo.RedoTable.from_problem(p)
    u = torch.tensor(p.u).cuda()
    U = torch.empty((1, 128, 128), dtype=torch.complex64, device="cuda")
    obs = torch.empty((1, 2), dtype=torch.float64, device="cuda")
    ws = t.workspace(redo.OP_EXPM_CHAIN, 1, 2)
    P = redo._ptr
    # an observable series asked for in the computational basis
    assert redo.lib().redo_expm_split_chain(t._h, 0, P(u), None, 1, 2, 0, 0, None, P(U), 0, None, P(obs), P(ws),
                                            ws.numel(), None) == 1
    torch.cuda.synchronize()
