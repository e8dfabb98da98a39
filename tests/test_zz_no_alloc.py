"""The allocation-free GRAPE entry point (d <= 64: scratch in a file-scope device
array) against redo_grape_fidelity_grad with the smallest caller workspace
(redo_grape_workspace_min_bytes: each scan step built from its factors, as the
allocation-free entry does), through the C ABI: two calls in a row, the second
with a smaller input, bit for bit (same kernel, same checkpoint schedule, same
summation order); sizes beyond the array are refused on the host."""
import numpy as np
import pytest
import torch

from paper_1707_02162_amd import workloads as W

pytestmark = pytest.mark.gpu


def R():
    from paper_1707_02162_amd import redo
    return redo


def noalloc_fn():
    lib = R().lib()
    return lib.redo_grape_fidelity_grad_noalloc, int(lib.redo_grape_noalloc_max_bytes())


def call_noalloc(t, u, Uf, ns, checkpoint_every=0):
    redo = R()
    fn, _ = noalloc_fn()
    B = u.shape[0]
    F = torch.empty(B, dtype=torch.float64, device="cuda")
    ov = torch.empty(B, dtype=torch.complex128, device="cuda")
    g = torch.empty_like(u)
    st = fn(t._h, 0, redo._ptr(u), redo._ptr(ns), B, u.shape[1], redo._ptr(Uf), checkpoint_every, redo._ptr(F),
            redo._ptr(ov), redo._ptr(g), redo._stream())
    return st, F, ov, g


def test_noalloc_grape_equals_workspace_entry_two_calls():
    redo = R()
    p = W.nmr_chain(4, 8, 120, 2e-6, 32, 2, 401, per_spin=True, n_drift=3,
                    lengths=np.array([120, 77, 120, 5, 99, 120, 64, 1], np.int32))
    t = redo.RedoTable.from_problem(p)
    u = torch.tensor(p.u).cuda()
    Uf = torch.tensor(p.U_target).cuda().to(torch.complex64)
    ns = torch.tensor(p.n_steps).cuda()
    cases = [(u, Uf, ns, 0), (u[3:6, :50].contiguous(), Uf[3:6].contiguous(), ns[3:6].clamp(max=50).contiguous(), 7)]
    for uu, ff, nn, ck in cases:
        torch.cuda.synchronize()
        print(f"[no-alloc] B={uu.shape[0]} N={uu.shape[1]} checkpoint_every={ck}", flush=True)
        st, F, ov, g = call_noalloc(t, uu, ff, nn, ck)
        assert st == 0, redo.lib().redo_last_error().decode()
        F0, ov0, g0 = t.grape(uu, ff, n_steps=nn, checkpoint_every=ck, precompose=False)
        torch.cuda.synchronize()
        assert torch.equal(F, F0)
        assert torch.equal(ov, ov0)
        assert torch.equal(g, g0)


def test_noalloc_grape_refuses_oversized_and_large_d():
    redo = R()
    _, cap = noalloc_fn()
    p = W.nmr_chain(6, 2, 16, 2e-6, 32, 2, 402)
    t = redo.RedoTable.from_problem(p)
    # checkpoints + one segment of 64 x 64 complex64 states: B * (ceil(N/C) + C) * 32 KiB > cap
    B = cap // (32 * 1024 * 8) + 1
    u = torch.zeros((B, 16, 1, 2), dtype=torch.float32, device="cuda")
    Uf = torch.zeros((B, 64, 64), dtype=torch.complex64, device="cuda")
    st, *_ = call_noalloc(t, u, Uf, None, 4)
    assert st == 6 and "scratch" in redo.lib().redo_last_error().decode()
    q = W.nmr_chain(7, 1, 4, 2e-6, 32, 2, 403)
    t2 = redo.RedoTable.from_problem(q)
    u2 = torch.tensor(q.u).cuda()
    st, *_ = call_noalloc(t2, u2, torch.tensor(q.U_target).cuda().to(torch.complex64), None)
    assert st == 6 and "d <= 64" in redo.lib().redo_last_error().decode()
    torch.cuda.synchronize()
