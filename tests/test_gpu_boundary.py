"""Boundary conditions of the C ABI that need the device: the unitarity
watchdog of the re-projection steps (REDO_WARN_UNITARITY, forced with a
non-unitary start state on the small-d fused chain and on the large-d path),
and the small library kernels the drivers call instead of torch arithmetic
(the projected ascent step of GRAPE, the time average of the order parameter),
against plain float32 / float64 torch references."""
import numpy as np
import pytest
import torch

from paper_1707_02162_amd import workloads as W

pytestmark = pytest.mark.gpu


def R():
    from paper_1707_02162_amd import redo
    return redo


@pytest.mark.parametrize("n", [3, 7])
def test_unitarity_watchdog_fires_on_a_drifted_state(n):
    """A start state 1.01 I is off the unitary group by ||X^dag X - I||_F / sqrt(d) =
    1.01^2 - 1 = 0.0201; the first re-projection step sees it (the steps are unitary),
    the Newton-Schulz step brings it to ~3e-4, below the 1e-3 threshold."""
    redo = R()
    p = W.ising_freezing(n=n, B=3, N=4)
    t = redo.RedoTable.from_problem(p)
    u = torch.tensor(p.u).cuda()
    X0 = (1.01 * torch.eye(p.d, dtype=torch.complex64, device="cuda")).expand(3, p.d, p.d).contiguous()
    torch.cuda.synchronize()
    print(f"[watchdog] d={p.d}", flush=True)
    t.chain(u, X0=X0, reproject_every=1)
    st, _ = t.device_status()
    assert st == 101
    drift, count = t.unitarity_report()
    assert abs(drift - 0.0201) < 1e-5 and count == 3
    # a unitary start: no warning, drift at FP32 rounding
    t.chain(u, reproject_every=1)
    st, _ = t.device_status()
    assert st in (0, 100)
    drift, count = t.unitarity_report()
    assert count == 0 and drift < 1e-5


def test_unitarity_watchdog_ragged_ignores_finished_instances():
    """Instances past their length do not take part in a re-projection step."""
    redo = R()
    p = W.ising_freezing(n=7, B=2, N=4)
    t = redo.RedoTable.from_problem(p)
    u = torch.tensor(p.u).cuda()
    X0 = torch.eye(p.d, dtype=torch.complex64, device="cuda").repeat(2, 1, 1)
    X0[1] *= 1.01
    lens = torch.tensor([4, 2], dtype=torch.int32)
    t.chain(u, X0=X0, n_steps=lens, reproject_every=3, step_offset=0)
    st, _ = t.device_status()
    # the re-projection is after global step 3: instance 1 (length 2) has finished by then
    assert st in (0, 100)
    assert t.unitarity_report()[1] == 0


def test_ascent_step_matches_torch():
    redo = R()
    g = torch.Generator(device="cpu").manual_seed(7)
    u = (torch.rand(1000, generator=g) * 4 - 2).cuda()
    gr = (torch.randn(1000, generator=g)).cuda()
    want = torch.clamp(u + 0.3 * gr, -1.5, 1.5)
    redo.ascent_step(u, gr, 0.3, -1.5, 1.5)
    assert torch.allclose(u, want, rtol=0, atol=1e-6)
    with pytest.raises(redo.RedoError):
        redo.ascent_step(u, gr, 0.3, 1.0, -1.0)


def test_time_average_matches_mean():
    redo = R()
    x = torch.tensor(np.random.default_rng(3).normal(size=(5, 10001)), device="cuda")
    q = redo.time_average(x)
    assert torch.allclose(q, x.mean(dim=1), rtol=1e-13, atol=1e-15)
