"""The batched L-BFGS kernels through the C ABI against the FP64 oracle's two-loop
recursion (the direction H g of the limited-memory inverse-curvature estimate), the
history rules, and the REDO-GRAPE driver's ascent."""
import numpy as np
import pytest
import torch

import oracle as O

pytestmark = pytest.mark.gpu


def R():
    from paper_1707_02162_amd import redo
    return redo


def _state(B, P, m, dev="cuda"):
    return (torch.zeros((m, B, P), dtype=torch.float32, device=dev), torch.zeros((m, B, P), dtype=torch.float32, device=dev),
            torch.zeros((m, B), dtype=torch.float64, device=dev), torch.zeros(B, dtype=torch.int32, device=dev),
            torch.zeros(B, dtype=torch.int32, device=dev))


def test_lbfgs_direction_and_history_vs_two_loop():
    """Histories of 6, 2 and 0 pairs (the first wraps the ring of m = 4) built through
    redo_lbfgs_push from iterates of a quadratic with SPD curvature: the direction equals
    the two-loop recursion over the newest m pairs, and gd = g . d."""
    redo = R()
    lib, P_ = redo.lib(), redo._ptr
    rng = np.random.default_rng(7)
    B, P, m = 3, 300, 4
    A = rng.normal(size=(P, P)) / np.sqrt(P)
    A = A @ A.T + 0.5 * np.eye(P)
    S, Y, rho, count, head = _state(B, P, m)
    hist = [[] for _ in range(B)]
    xs = rng.normal(size=(B, P))
    npairs = [6, 2, 0]
    last = max(npairs)
    for it in range(last):
        x = torch.tensor(xs, dtype=torch.float32, device="cuda")
        xn_np = xs + 0.1 * rng.normal(size=(B, P))
        xn = torch.tensor(xn_np, dtype=torch.float32, device="cuda")
        # ascent gradient of F = -x.A.x/2: g = -A x, so y = g - gn = A (xn - x)
        g = torch.tensor(-(xs @ A), dtype=torch.float32, device="cuda")
        gn = torch.tensor(-(xn_np @ A), dtype=torch.float32, device="cuda")
        # instance b accepts its last npairs[b] steps (a rejected step before them clears it)
        take = [it >= last - npairs[b] for b in range(B)]
        acc = torch.tensor([1 if tk else 0 for tk in take], dtype=torch.int32, device="cuda")
        redo._check(lib.redo_lbfgs_push(B, P, m, P_(x), P_(xn), P_(g), P_(gn), P_(acc), P_(S), P_(Y), P_(rho),
                                        P_(count), P_(head), None))
        for b in range(B):
            if take[b]:
                s = (xn.cpu().numpy()[b] - x.cpu().numpy()[b]).astype(np.float64)
                y = (g.cpu().numpy()[b] - gn.cpu().numpy()[b]).astype(np.float64)
                hist[b].append((s, y))
        xs = xn_np
    assert count.cpu().tolist() == [4, 2, 0]
    gq = rng.normal(size=(B, P)).astype(np.float32)
    gt = torch.tensor(gq, device="cuda")
    d = torch.empty_like(gt)
    gd = torch.empty(B, dtype=torch.float64, device="cuda")
    redo._check(lib.redo_lbfgs_direction(B, P, m, P_(gt), P_(S), P_(Y), P_(rho), P_(count), P_(head), 2.5, P_(d),
                                         P_(gd), None))
    d = d.cpu().numpy()
    for b in range(B):
        ref = O.lbfgs_direction(gq[b], hist[b][-m:], 2.5)
        assert np.linalg.norm(d[b] - ref) <= 1e-5 * np.linalg.norm(ref), b
        assert abs(gd[b].item() - float(gq[b].astype(np.float64) @ d[b])) <= 1e-6 * abs(gd[b].item())
    # a rejected step clears the history; a pair without positive curvature is not kept
    x0 = torch.zeros((B, P), dtype=torch.float32, device="cuda")
    x1 = torch.ones((B, P), dtype=torch.float32, device="cuda")
    acc = torch.tensor([0, 1, 1], dtype=torch.int32, device="cuda")
    redo._check(lib.redo_lbfgs_push(B, P, m, P_(x0), P_(x1), P_(x0), P_(x1), P_(acc), P_(S), P_(Y), P_(rho),
                                    P_(count), P_(head), None))
    assert count.cpu().tolist() == [0, 2, 0]


def test_lbfgs_trial_point():
    redo = R()
    lib, P_ = redo.lib(), redo._ptr
    x = torch.randn((2, 5, 3), device="cuda")
    d = torch.randn((2, 5, 3), device="cuda")
    alpha = torch.tensor([0.5, -2.0], dtype=torch.float64, device="cuda")
    xt = torch.empty_like(x)
    redo._check(lib.redo_lbfgs_trial(2, 15, P_(x), P_(d), P_(alpha), P_(xt), None))
    ref = x.double() + alpha.view(2, 1, 1) * d.double()
    assert torch.allclose(xt.double(), ref, rtol=1e-6, atol=1e-6)


def test_grape_lbfgs_ascends_reachable_targets_d16():
    """Reachable 4-qubit targets (d = 16, two phased channels, b = 32, P = 2) from seeded
    random pulses: an instance's F never falls (a step is taken only when it raises F
    strictly), and after 25 iterations L-BFGS is ahead of 25 plain Adam ascent steps on
    the same starts."""
    from paper_1707_02162_amd import lbfgs, warmstart, workloads as W
    redo = R()
    p = W.c5_four_qubit(B=1, N=100)
    t = redo.RedoTable.from_problem(p)
    Uf, _ = warmstart.reachable_targets(t, p, 901, 8)
    u0 = warmstart.random_starts(p, 902, 8)
    u, F, hist = lbfgs.grape_lbfgs(t, u0, Uf, iters=25)
    H = torch.stack(hist).cpu().numpy()
    assert np.all(np.diff(H, axis=0) >= 0)
    _, Fa, _, _ = warmstart.grape(t, u0, Uf, u_max=float(p.u_scale) * 4, iters=25, lr=1000.0)
    print("L-BFGS mean infidelity", float((1 - F).mean()), "Adam", float((1 - Fa).mean()), "start", float((1 - H[0]).mean()))
    assert float((1 - F).mean()) < float((1 - Fa).mean())
    assert float((1 - F).mean()) < 0.5 * float((1 - H[0]).mean())
