"""Learned warm start for REDO-GRAPE (an extension of the method; not in the paper).

A three-layer perceptron (tanh, BF16 weights, FP32 accumulation) maps the
2 d^2 real entries of a global-phase-free target unitary to the initial
control amplitudes of a REDO-GRAPE run.  It is trained on (target, pulse)
pairs whose pulses REDO-GRAPE brought to infidelity <= 1e-4: by default the
smooth pulse that produced each reachable target, refined by REDO-GRAPE where
needed, so that the target -> pulse map it learns is single valued (labels
from REDO-GRAPE runs started at independent random pulses land on different
solutions for the same target, and a least-squares fit averages them into
nothing useful; `--labels grape` keeps that variant).  Plain REDO-GRAPE stays
both the fallback (a random start is used whenever it starts better than the
network's proposal, and after a network start that misses the goal within the
budget) and the arbiter: every reported fidelity is the library's REDO
fidelity.

Every arithmetic step runs in libredo.so: the network's forward and backward
passes, its Adam updates, the target features, the REDO chains and the GRAPE
gradients and amplitude updates.  This module only sequences the calls.

    python -m paper_1707_02162_amd.warmstart --train 20000 --test 256
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import sys
import time
from typing import Optional

import numpy as np
import torch

from . import redo as R
from . import workloads as W


def _p(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def adam_(param: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor, step: int, lr: float,
          sign: float = 1.0, lo: float = -3.0e38, hi: float = 3.0e38, bf16: Optional[torch.Tensor] = None,
          beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> None:
    R._check(R.lib().redo_adam_update(param.numel(), _p(param), _p(bf16), _p(grad), _p(m), _p(v), lr, beta1, beta2,
                                      eps, step, sign, lo, hi, R._stream()))


def target_features(U: torch.Tensor) -> torch.Tensor:
    B, d = U.shape[0], U.shape[-1]
    Uc = U.to(torch.complex64).contiguous()
    out = torch.empty((B, 2 * d * d), dtype=torch.float32, device=U.device)
    R._check(R.lib().redo_mlp_target_features(d, B, _p(Uc), _p(out), R._stream()))
    return out


class WarmStartMLP:
    """FP32 master weights with BF16 copies for the products; Adam state."""

    def __init__(self, sizes, device="cuda", seed: int = 0):
        self.sizes = list(sizes)
        gen = np.random.default_rng(seed)
        self.W, self.b, self.Wh = [], [], []
        for i, o in zip(self.sizes[:-1], self.sizes[1:]):
            lim = math.sqrt(6.0 / (i + o))
            Wl = torch.tensor(gen.uniform(-lim, lim, (o, i)), dtype=torch.float32, device=device)
            self.W.append(Wl)
            self.b.append(torch.zeros(o, dtype=torch.float32, device=device))
            self.Wh.append(Wl.to(torch.bfloat16).contiguous())
        self.gW = [torch.zeros_like(w) for w in self.W]
        self.gb = [torch.zeros_like(b) for b in self.b]
        self.mW = [torch.zeros_like(w) for w in self.W]
        self.vW = [torch.zeros_like(w) for w in self.W]
        self.mb = [torch.zeros_like(b) for b in self.b]
        self.vb = [torch.zeros_like(b) for b in self.b]
        self.step = 0
        self.device = device
        self._loss = torch.zeros(1, dtype=torch.float64, device=device)

    def _net(self):
        n = R._Mlp()
        for l in range(4):
            n.sizes[l] = self.sizes[l]
        for l in range(3):
            n.W[l] = self.Wh[l].data_ptr()
            n.b[l] = self.b[l].data_ptr()
        return n

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        B = x.shape[0]
        acts = torch.empty(B * sum(self.sizes[1:]), dtype=torch.float32, device=self.device)
        net = self._net()
        R._check(R.lib().redo_mlp_forward(ctypes.byref(net), B, _p(x.contiguous()), _p(acts), R._stream()))
        return acts[B * (self.sizes[1] + self.sizes[2]):].view(B, self.sizes[3])

    def loss_and_grads(self, x: torch.Tensor, target: torch.Tensor) -> float:
        B = x.shape[0]
        acts = torch.empty(B * sum(self.sizes[1:]), dtype=torch.float32, device=self.device)
        scratch = torch.empty(2 * B * max(self.sizes[1:]), dtype=torch.float32, device=self.device)
        g = R._MlpGrads()
        for l in range(3):
            g.W[l] = self.gW[l].data_ptr()
            g.b[l] = self.gb[l].data_ptr()
        net = self._net()
        R._check(R.lib().redo_mlp_loss_grad(ctypes.byref(net), B, _p(x.contiguous()), _p(target.contiguous()),
                                            _p(acts), _p(scratch), ctypes.byref(g), _p(self._loss), R._stream()))
        return self._loss

    def train_step(self, x, target, lr: float):
        loss = self.loss_and_grads(x, target)
        self.step += 1
        for l in range(3):
            adam_(self.W[l], self.gW[l], self.mW[l], self.vW[l], self.step, lr, bf16=self.Wh[l])
            adam_(self.b[l], self.gb[l], self.mb[l], self.vb[l], self.step, lr)
        return loss

    def train_step_upstream(self, x, y, dl_dy, lr: float):
        """One Adam step for an arbitrary loss whose gradient with respect to the
        output y (computed by forward(x)) is dl_dy: the least-squares backward
        with the pseudo-target y - (n/2) dl_dy has exactly that upstream
        gradient (n = number of output entries of the batch)."""
        n = y.numel()
        return self.train_step(x, (y - 0.5 * n * dl_dy).contiguous(), lr)


def grape(table: R.RedoTable, u0: torch.Tensor, Uf: torch.Tensor, u_max: float, iters: int, lr: float,
          goal: float = 1e-4, history: bool = False, log=None, tag: str = "grape", lr_final: Optional[float] = None):
    """Batched REDO-GRAPE: Adam ascent on F, amplitudes clamped to [-u_max, u_max],
    step size decaying geometrically from lr to lr_final (default: constant).
    An instance that reaches infidelity <= goal keeps the amplitudes of that
    iteration.  Returns (u, F, iterations to reach the goal (or -1), history);
    progress goes to `log` every 50 iterations."""
    decay = 1.0 if lr_final is None or iters < 1 else (lr_final / lr) ** (1.0 / iters)
    u = u0.clone().contiguous()
    m = torch.zeros_like(u)
    v = torch.zeros_like(u)
    B = u.shape[0]
    reached = torch.full((B,), -1, dtype=torch.int64, device=u.device)
    F = None
    hist = []
    u_best = u.clone()
    F_best = None
    for it in range(iters + 1):
        F, _, g = table.grape(u, Uf)
        if F_best is None:
            F_best = F.clone()
        # instances that already reached the goal keep that point
        frozen = reached >= 0
        F = torch.where(frozen, F_best, F)
        ok = (1.0 - F) <= goal
        reached = torch.where((reached < 0) & ok, torch.full_like(reached, it), reached)
        newly = ok & ~frozen
        u_best = torch.where(newly.view(-1, *([1] * (u.dim() - 1))), u, u_best)
        F_best = torch.where(newly | ~frozen, F, F_best)
        if history:
            hist.append(F.clone())
        if it == iters or bool(ok.all()):
            break
        if log is not None and it % 50 == 0:
            log(f"[warmstart] {tag} iteration {it}: {int(ok.sum())}/{B} at infidelity <= {goal:g}, "
                f"median infidelity {float((1 - F).median()):.2e}")
        adam_(u, g, m, v, it + 1, lr * decay ** it, sign=-1.0, lo=-u_max, hi=u_max)
    done = (reached >= 0).view(-1, *([1] * (u.dim() - 1)))
    return torch.where(done, u_best, u), F, reached, hist


def reachable_targets(table: R.RedoTable, p: W.Problem, config_id: int, B: int, amp: float = 1.0):
    """Targets reached by smooth seeded pulses (so that a solution exists), the
    pulses scaled by `amp`.  Returns (U_f, the pulses that produce them)."""
    gen = W.nmr_chain(4, B, p.N, p.dt, p.base, p.digits, config_id, species=[[0, 1], [2, 3]],
                      targets=False)
    ug = torch.tensor(gen.u * np.float32(amp), device="cuda")
    U, _, _ = table.chain(ug)
    return U, ug


def random_starts(p: W.Problem, config_id: int, B: int, amp: float = 1.0) -> torch.Tensor:
    """Seeded smooth pulses from the targets' own distribution (scaled by `amp`)."""
    st = W.nmr_chain(4, B, p.N, p.dt, p.base, p.digits, config_id, species=[[0, 1], [2, 3]], targets=False)
    return torch.tensor(st.u * np.float32(amp), device="cuda")


def experiment(n_train: int, n_test: int, N: int = 500, grape_iters: int = 2000, lr_grape: float = 1000.0,
               epochs: int = 40, batch: int = 256, lr_net: float = 1e-3, width: int = 512, goal: float = 1e-4,
               labels: str = "source", loss: str = "both", fid_epochs: int = 40, amp: float = 1.0, log=print):
    """C5-shaped run: d = 16, two species with collective X/Y, N steps of 2 us.

    labels "source": each training target is labelled with the smooth pulse
      that produced it, refined by REDO-GRAPE from that pulse to infidelity
      <= goal where needed (a single-valued target -> pulse map);
    labels "grape": REDO-GRAPE from an independent random smooth start (the
      solution reached depends on the start, so the same target can carry
      very different labels).

    loss "mse": least squares to the labels; "fidelity": 1 - F of the
      proposed pulse for its target, its gradient dF/du from the library's
      REDO-GRAPE adjoint back-propagated through the network (any pulse that
      reaches the target is a right answer); "both": least squares, then
      fid_epochs of the fidelity loss.

    amp scales every pulse (sources and random starts alike): at small areas the
    propagator is close to linear in the pulse (first-order Magnus term) and the
    target -> pulse map becomes learnable."""
    p = W.c5_four_qubit(B=1, N=N)
    table = R.RedoTable.from_problem(p)
    table.cache_levels()
    u_max = float(p.u_scale)
    t0 = time.time()
    # training set: reachable targets and REDO-GRAPE-optimised pulses for them
    Uf, ug = reachable_targets(table, p, 501, n_train, amp)
    u0 = ug if labels == "source" else random_starts(p, 502, n_train, amp)
    u_opt, F_opt, it_opt, _ = grape(table, u0, Uf, u_max, grape_iters, lr_grape, goal=goal, log=log, tag="dataset")
    keep = (1.0 - F_opt) <= goal
    log(f"[warmstart] dataset: {int(keep.sum())}/{n_train} optimised to {goal:g} in {time.time() - t0:.1f}s")
    X = target_features(Uf)[keep]
    Y = (u_opt[keep] / u_max).reshape(int(keep.sum()), -1)
    sizes = [X.shape[1], width, width, Y.shape[1]]
    net = WarmStartMLP(sizes, seed=503)
    nb = max(1, X.shape[0] // batch)
    losses = []
    for ep in range(epochs):
        perm = torch.randperm(X.shape[0], device="cuda", generator=torch.Generator(device="cuda").manual_seed(ep))
        tot = 0.0
        for i in range(nb):
            idx = perm[i * batch:(i + 1) * batch]
            tot += float(net.train_step(X[idx], Y[idx], lr_net).item())
        losses.append(tot / nb)
        if ep % 10 == 0:
            log(f"[warmstart] epoch {ep}: loss {losses[-1]:.4f}")
    log(f"[warmstart] trained {epochs} epochs, loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    fid_losses = []
    if loss in ("fidelity", "both"):
        Ufk = Uf[keep].contiguous()
        shape = (batch,) + tuple(u0.shape[1:])
        for ep in range(fid_epochs):
            perm = torch.randperm(X.shape[0], device="cuda", generator=torch.Generator(device="cuda").manual_seed(1000 + ep))
            tot = 0.0
            for i in range(nb):
                idx = perm[i * batch:(i + 1) * batch]
                y = net.forward(X[idx])
                u_b = (y * u_max).reshape((len(idx),) + shape[1:]).contiguous()
                Fb, _, gb = table.grape(u_b, Ufk[idx])
                # loss = mean over the batch of (1 - F); dF/dy = dF/du * u_max
                dl_dy = -(gb.reshape(len(idx), -1) * u_max) / len(idx)
                net.train_step_upstream(X[idx], y, dl_dy, lr_net)
                tot += float((1.0 - Fb).mean())
            fid_losses.append(tot / nb)
            if ep % 10 == 0:
                log(f"[warmstart] fidelity epoch {ep}: mean infidelity of the proposals {fid_losses[-1]:.4f}")
        log(f"[warmstart] fidelity training: mean infidelity {fid_losses[0]:.4f} -> {fid_losses[-1]:.4f}")
    # held-out targets: network start (with fallback) vs random start
    Ut, _ = reachable_targets(table, p, 601, n_test, amp)
    ur = random_starts(p, 602, n_test, amp)
    un = (net.forward(target_features(Ut)) * u_max).reshape(ur.shape).contiguous()
    Fr0, _, _ = table.grape(ur, Ut)
    Fn0, _, _ = table.grape(un, Ut)
    use_net = Fn0 >= Fr0                       # fallback to the random start when it starts better
    us = torch.where(use_net.view(-1, 1, 1, 1), un, ur)
    _, Fr, itr, _ = grape(table, ur, Ut, u_max, grape_iters, lr_grape, goal=goal, log=log, tag="random start")
    _, Fs, its, _ = grape(table, us, Ut, u_max, grape_iters, lr_grape, goal=goal, log=log, tag="network start")
    # second fallback: a network start that does not reach the goal within the budget is
    # followed by the run from the random start (its iterations count after the wasted budget)
    miss = use_net & (its < 0)
    its_fb = torch.where(miss, torch.where(itr >= 0, itr + grape_iters, torch.full_like(itr, -1)), its)
    Fs_fb = torch.where(miss, Fr, Fs)
    conv_r = itr >= 0
    conv_s = its >= 0
    conv_fb = its_fb >= 0
    both = conv_r & conv_fb
    res = dict(
        labels=labels, amp=amp, dataset_grape_iters_median=float(it_opt[keep].double().median()) if keep.any() else None,
        n_train=n_train, n_train_converged=int(keep.sum()), n_test=n_test, N=N, epochs=epochs, goal=goal,
        loss_first=losses[0], loss_last=losses[-1], loss_kind=loss,
        fidelity_loss_first=fid_losses[0] if fid_losses else None,
        fidelity_loss_last=fid_losses[-1] if fid_losses else None,
        start_infidelity_random_median=float((1 - Fr0).median()), start_infidelity_net_median=float((1 - Fn0).median()),
        net_start_used=int(use_net.sum()),
        converged_random=int(conv_r.sum()), converged_warm=int(conv_s.sum()),
        iters_random_median=float(itr[conv_r].double().median()) if conv_r.any() else None,
        iters_warm_median=float(its[conv_s].double().median()) if conv_s.any() else None,
        final_infidelity_random_median=float((1 - Fr).median()), final_infidelity_warm_median=float((1 - Fs).median()),
        fallback_reruns=int(miss.sum()), converged_warm_with_fallback=int(conv_fb.sum()),
        iters_warm_with_fallback_median=float(its_fb[conv_fb].double().median()) if conv_fb.any() else None,
        final_infidelity_warm_with_fallback_median=float((1 - Fs_fb).median()),
        iters_saved_mean=float((itr[both] - its_fb[both]).double().mean()) if both.any() else None,
        grape_iters_budget=grape_iters,
        seconds=time.time() - t0,
    )
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=20000)
    ap.add_argument("--test", type=int, default=256)
    ap.add_argument("--N", type=int, default=500)
    ap.add_argument("--grape-iters", type=int, default=2000)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--goal", type=float, default=1e-4)
    ap.add_argument("--lr-grape", type=float, default=1000.0)
    ap.add_argument("--width", type=int, default=512)
    ap.add_argument("--labels", choices=["source", "grape"], default="source")
    ap.add_argument("--loss", choices=["mse", "fidelity", "both"], default="both")
    ap.add_argument("--fid-epochs", type=int, default=40)
    ap.add_argument("--amp", type=float, default=1.0, help="scale of every pulse (lower-area regime below 1)")
    a = ap.parse_args()
    res = experiment(a.train, a.test, N=a.N, grape_iters=a.grape_iters, lr_grape=a.lr_grape, epochs=a.epochs,
                     goal=a.goal, width=a.width, labels=a.labels, loss=a.loss, fid_epochs=a.fid_epochs, amp=a.amp,
                     log=lambda s: print(s, file=sys.stderr, flush=True))
    print(json.dumps(res))


if __name__ == "__main__":
    main()
