"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types an oracle formula: each compares the oracle with a
closed form, a worked example printed in the paper, a brute-force product of
hand-written 2x2 matrices, an invariant, or central finite differences.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_1707_02162_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

SX = np.array([[0, 1], [1, 0]], dtype=complex)
SY = np.array([[0, -1j], [1j, 0]], dtype=complex)
SZ = np.array([[1, 0], [0, -1]], dtype=complex)
I2 = np.eye(2, dtype=complex)


def _rot(theta, n):
    """Textbook spin-1/2 rotation exp(-i theta n.sigma/2)."""
    ns = n[0] * SX + n[1] * SY + n[2] * SZ
    return math.cos(theta / 2) * I2 - 1j * math.sin(theta / 2) * ns


# ------------------------------------------------------------------ T1
def test_t1_single_spin_closed_form():
    rng = np.random.default_rng(1)
    for _ in range(20):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        theta = rng.uniform(-7, 7)
        H = (n[0] * SX + n[1] * SY + n[2] * SZ) / 2
        assert np.allclose(O.expm_herm(H, theta), _rot(theta, n), atol=1e-14, rtol=0)


def test_t1_generator_spin_operators():
    assert np.array_equal(W.spin_op(1, 0, "x"), SX / 2)
    assert np.array_equal(W.spin_op(1, 0, "y"), SY / 2)
    assert np.array_equal(W.spin_op(2, 0, "z"), np.kron(SZ, I2) / 2)   # qubit 1 most significant
    assert np.array_equal(W.spin_z_diag(2, 1), np.diag(np.kron(I2, SZ)).real / 2)
    for n in (2, 3):
        for i in range(n):
            x, y, z = (W.spin_op(n, i, a) for a in "xyz")
            assert np.allclose(x @ y - y @ x, 1j * z, atol=1e-15)
    # collective S_x of n spins has eigenvalues -n/2 .. n/2 with binomial multiplicities
    n = 4
    lam = np.round(np.linalg.eigvalsh(W.collective(n, range(n), "x")) * 2).astype(int)
    vals, counts = np.unique(lam, return_counts=True)
    assert list(vals) == list(range(-n, n + 1, 2))
    assert list(counts) == [math.comb(n, k) for k in range(n + 1)]


# ------------------------------------------------------------------ T3 / T4
def test_t3_worked_example_digits():
    ex = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    b, P = ex["base"], ex["digits"]
    assert O.digits_needed(ex["omega_max"] / ex["eps"], b)[0] == P
    for case in ex["cases"]:
        qz = O.quantise(np.array([case["omega"]], np.float32), ex["eps"], b, P, phased=False)
        assert int(qz["q"][0]) == case["q"]
        assert list(qz["c"][0]) == case["c"]
    S = W.spin_op(1, 0, "x")[None]
    tab = O.DiscreteTable(S, 1e-6, ex["eps"], b, P)
    assert tab.stored_entries == ex["stored_operators"]
    # at most P non-identity factors, i.e. P - 1 products
    assert P - 1 == ex["max_multiplications"]


def test_t4_cost_model():
    cm = json.load(open(os.path.join(GOLDEN, "cost_model.json")))
    for b, P, p, s in cm["rows"]:
        assert O.digits_needed(cm["ratio"], b) == (P, p, s)
        # the paper's estimate p ~ log_b(Omega_max / (b eps)) rounds up to the same p
        assert math.ceil(math.log(cm["ratio"] / b, b)) == p


def test_quantiser_rounding_and_clamp():
    eps = 0.5
    u = np.array([0.0, 0.24, 0.25, 0.26, -0.25, -0.26, 1e9], np.float32)
    qz = O.quantise(u, eps, 4, 2, phased=False)
    assert list(qz["q"]) == [0, 0, 1, 1, 1, 1, 15]
    assert list(qz["sign"]) == [1, 1, 1, 1, -1, -1, 1]
    assert list(qz["clamped"]) == [False] * 6 + [True]
    # phased: magnitude from the Cartesian pair, phase from atan2
    qp = O.quantise(np.array([[3.0, 4.0]], np.float32), 1.0, 10, 1, phased=True)
    assert int(qp["q"][0]) == 5 and abs(qp["phi"][0] - math.atan2(4, 3)) < 1e-15


# ------------------------------------------------------------------ T2
def test_t2_table_product_equals_exponential():
    rng = np.random.default_rng(2)
    A = rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4))
    S = (A + A.conj().T)[None] / 4
    dt, eps, b, P = 5e-6, 37.0, 16, 3
    tab = O.DiscreteTable(S, dt, eps, b, P)
    for q in [0, 1, 15, 16, 255, 256, 1234, 4095]:
        c = [(q // b ** j) % b for j in range(P)]
        R = tab.factor(0, c)
        assert np.abs(R - O.expm_herm(S[0], q * eps * dt)).max() < 1e-13
        Rm = tab.factor(0, c, sign=-1)
        assert np.abs(Rm - O.expm_herm(S[0], -q * eps * dt)).max() < 1e-13


def test_t2_table_entries_are_powers_of_the_base_operator():
    S = W.collective(2, [0, 1], "x")[None]
    b, P, dt, eps = 3, 3, 1e-5, 1000.0
    tab = O.DiscreteTable(S, dt, eps, b, P)
    E = tab.entry(0, 0, 1)
    for j in range(P):
        for c in range(1, b):
            want = np.linalg.matrix_power(E, c * b ** j)
            assert np.abs(tab.entry(0, j, c) - want).max() < 1e-13


# ------------------------------------------------------------------ T5
@pytest.mark.parametrize("n", [1, 3])
def test_t5_quantisation_fidelity(n):
    """Sec. II: F = |Tr[e^{i Omega dt S} e^{-i Omega_hat dt S}]/d|^2; for S with
    eigenvalues lambda_i it equals |(1/d) sum_i e^{i delta dt lambda_i}|^2, and
    for the involutory S = 2 I_x of one spin 1 - F = sin^2(delta dt)."""
    S = W.collective(n, range(n), "x")
    d = 2 ** n
    eps, dt, b, P = 1.0, 5e-6, 64, 3
    tab = O.DiscreteTable(S[None], dt, eps, b, P)
    rng = np.random.default_rng(5)
    for om in rng.uniform(0, 2.6e5, 10).astype(np.float32):
        qz = O.quantise(np.array([om]), eps, b, P, phased=False)
        Rq = tab.factor(0, qz["c"][0])
        Fm = abs(np.trace(O.expm_herm(S, -float(om) * dt) @ Rq) / d) ** 2
        delta = float(om) - int(qz["q"][0]) * eps
        # eigenvalues of collective S_x: -n/2 .. n/2 with binomial multiplicities
        lam = np.concatenate([np.full(math.comb(n, k), n / 2 - k) for k in range(n + 1)])
        Fc = abs(np.exp(1j * delta * dt * lam).sum() / d) ** 2
        assert abs(Fm - Fc) < 1e-14
        if n == 1:
            S2 = 2 * S
            tab2 = O.DiscreteTable(S2[None], dt, eps, b, P)
            F2 = abs(np.trace(O.expm_herm(S2, -float(om) * dt) @ tab2.factor(0, qz["c"][0])) / 2) ** 2
            assert abs((1 - F2) - math.sin(delta * dt) ** 2) < 1e-14


# ------------------------------------------------------------------ T6
def test_t6_dirac_frame_step_equals_lab_split():
    """Sec. III: V(dt) Z (prod_k Xt_k) Z^dag with Dirac-frame Xt equals the
    lab-frame split Z (prod_k X_k) Z^dag V(dt) when [Z, H0] = 0."""
    rng = np.random.default_rng(6)
    n = 3
    d = 2 ** n
    species = [[0, 1], [2]]
    S = np.stack([W.collective(n, sp, "x") for sp in species])
    g = np.stack([W.collective_z_diag(n, sp) for sp in species])
    # drift: offsets + ZZ + isotropic coupling inside species 1 (commutes with its S_z)
    H0 = np.diag(rng.normal(size=d) * 1e4).astype(complex)
    H0 += 2 * np.pi * 150 * sum(W.spin_op(n, 0, a) @ W.spin_op(n, 1, a) for a in "xyz")
    for k in range(2):
        assert np.abs(np.diag(g[k]) @ H0 - H0 @ np.diag(g[k])).max() < 1e-9
    dt = 3e-6
    V = O.expm_herm(H0, dt)
    for _ in range(5):
        amp = rng.normal(size=(2, 2)) * 5e4
        A = O.dirac_step(H0, S, g, amp, dt)
        B = O.step_split(S, g, amp, dt, V)
        assert np.abs(A - B).max() < 1e-13


# ------------------------------------------------------------------ T7
def test_t7_commuting_chain_closed_form():
    """One signed channel and no drift: the REDO chain over thousands of steps
    is exp(-i eps dt (sum_n sign_n q_n) S)."""
    p = W.ising_freezing(n=3, B=1, N=3000, J=0.0)
    p.H0[:] = 0.0
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    U = O.chain(O.compose_all_redo(p, tab, 0))
    qz = O.quantise(p.u[0], p.eps, p.base, p.digits, phased=False)
    total = float((qz["sign"][:, 0] * qz["q"][:, 0]).sum())
    want = O.expm_herm(p.S[0], total * p.eps * p.dt)
    assert np.abs(U - want).max() < 1e-11


# ------------------------------------------------------------------ T8
def test_t8_ising_without_coupling_keeps_magnetisation():
    p = W.ising_freezing(n=4, B=1, N=300, J=0.0)
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    m, _ = O.magnetisation_series(O.compose_all_redo(p, tab, 0), p.M)
    assert np.abs(m - 1.0).max() < 1e-12


def test_t8_ising_without_drive_closed_form():
    """h0 = 0: m(t) = [2 cos(J t) + (n - 2) cos^2(J t)] / n for the open chain."""
    n = 4
    p = W.ising_freezing(n=n, B=1, N=400)
    p.u[:] = 0.0
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    m, _ = O.magnetisation_series(O.compose_all_redo(p, tab, 0), p.M)
    J = p.meta["J"]
    t = (np.arange(1, 401)) * p.dt
    want = (2 * np.cos(J * t) + (n - 2) * np.cos(J * t) ** 2) / n
    assert np.abs(m - want).max() < 1e-12


# ------------------------------------------------------------------ T9
def _one_spin_problem(N=40, seed=9):
    rng = np.random.default_rng(seed)
    nu = 2 * np.pi * 3e3
    dt = 5e-6
    scale = 2 * np.pi * 10e3
    u = (rng.uniform(-1, 1, (1, N, 1, 2)) * scale).astype(np.float32)
    Uf = W.haar_unitary(2, W.rng(99, 2, 0))[None]
    p = W.Problem("one_spin", 2, 1, True, np.array([[nu / 2, -nu / 2]]), True,
                  (SX / 2)[None], np.array([[0.5, -0.5]]), dt, math.sqrt(2) * scale / 255,
                  16, 2, u, None, Uf, None, u_scale=scale)
    return p, nu


def _hand_step(ux, uy, nu, dt):
    om = math.hypot(ux, uy)
    phi = math.atan2(uy, ux)
    C = math.cos(om * dt / 2) * I2 - 1j * math.sin(om * dt / 2) * (math.cos(phi) * SX + math.sin(phi) * SY)
    V = np.diag([np.exp(-0.5j * nu * dt), np.exp(0.5j * nu * dt)])
    return C @ V


def _hand_chain(amp, nu, dt):
    X = I2.copy()
    for n in range(amp.shape[0]):
        X = _hand_step(amp[n, 0, 0], amp[n, 0, 1], nu, dt) @ X
    return X


def test_t9_d2_brute_force_steps_chain_fidelity():
    p, nu = _one_spin_problem()
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    steps = O.compose_all_redo(p, tab, 0)
    qz = O.quantise(p.u[0], p.eps, p.base, p.digits, phased=True)
    om = qz["q"][:, 0] * p.eps
    amp_q = np.stack([om * np.cos(qz["phi"][:, 0]), om * np.sin(qz["phi"][:, 0])], -1)[:, None, :]
    for n in range(p.N):
        assert np.abs(steps[n] - _hand_step(amp_q[n, 0, 0], amp_q[n, 0, 1], nu, p.dt)).max() < 1e-14
        V = O.drift_propagator(p.H0[0], p.dt, True)
        sp = O.step_split(p.S, p.g, p.u[0, n].astype(float), p.dt, V)
        assert np.abs(sp - _hand_step(float(p.u[0, n, 0, 0]), float(p.u[0, n, 0, 1]), nu, p.dt)).max() < 1e-14
    X = O.chain(steps)
    Xh = _hand_chain(amp_q, nu, p.dt)
    assert np.abs(X - Xh).max() < 1e-13
    g, F = O.unitary_fidelity(p.U_target[0], X)
    gh = np.trace(p.U_target[0].conj().T @ Xh) / 2
    assert abs(g - gh) < 1e-13 and abs(F - abs(gh) ** 2) < 1e-13


def test_t9_d2_gradient_vs_finite_differences_of_hand_chain():
    p, nu = _one_spin_problem(N=12)
    Uf = p.U_target[0]

    def F_hand(amp):
        X = _hand_chain(amp, nu, p.dt)
        return abs(np.trace(Uf.conj().T @ X) / 2) ** 2

    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    for model in ("split", "redo"):
        F, _, grad = O.fidelity_and_gradient(p, 0, model=model, table=tab)
        if model == "split":
            amp0 = p.u[0].astype(float)
        else:
            qz = O.quantise(p.u[0], p.eps, p.base, p.digits, phased=True)
            om = qz["q"][:, 0] * p.eps
            amp0 = np.stack([om * np.cos(qz["phi"][:, 0]), om * np.sin(qz["phi"][:, 0])], -1)[:, None, :]
        assert abs(F - F_hand(amp0)) < 1e-13
        h = 1e-6 * p.u_scale
        fd = np.zeros_like(amp0)
        for idx in np.ndindex(*amp0.shape):
            a1 = amp0.copy(); a1[idx] += h
            a2 = amp0.copy(); a2[idx] -= h
            fd[idx] = (F_hand(a1) - F_hand(a2)) / (2 * h)
        assert np.linalg.norm(grad - fd) <= 1e-7 * np.linalg.norm(fd)


# ------------------------------------------------------------------ T10
def test_t10_invariants():
    p = W.c1_two_spin(B=1, N=30)
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    X = O.chain(O.compose_all_redo(p, tab, 0))
    assert np.linalg.norm(X.conj().T @ X - np.eye(4)) / 2 < 1e-13
    _, F1 = O.unitary_fidelity(X, X)
    assert abs(F1 - 1) < 1e-14
    _, Fa = O.unitary_fidelity(p.U_target[0], X)
    _, Fb = O.unitary_fidelity(np.exp(0.7j) * p.U_target[0], X)
    assert abs(Fa - Fb) < 1e-14
    # signed amplitude: R(-u) = R(u)^dag exactly
    S = W.collective(2, [0, 1], "x")[None]
    t2 = O.DiscreteTable(S, 1e-6, 3.0, 8, 3)
    for x in (5.0, 700.0, 1500.0):
        qp = O.quantise(np.array([x], np.float32), 3.0, 8, 3, phased=False)
        qm = O.quantise(np.array([-x], np.float32), 3.0, 8, 3, phased=False)
        assert list(qp["c"][0]) == list(qm["c"][0])
        Rp = t2.factor(0, qp["c"][0], qp["sign"][0])
        Rm = t2.factor(0, qm["c"][0], qm["sign"][0])
        assert np.array_equal(Rm, Rp.conj().T)


# ------------------------------------------------------------------ T12
def _fd_grad(p, b, amp0, model, h):
    fd = np.zeros_like(amp0)
    for idx in np.ndindex(*amp0.shape):
        a1 = amp0.copy(); a1[idx] += h
        a2 = amp0.copy(); a2[idx] -= h
        F1 = O.fidelity_and_gradient(p, b, model=model, amps=a1)[0]
        F2 = O.fidelity_and_gradient(p, b, model=model, amps=a2)[0]
        fd[idx] = (F1 - F2) / (2 * h)
    return fd


@pytest.mark.parametrize("model", ["split", "exact"])
def test_t12_gradient_vs_central_differences_phased(model):
    p = W.c1_two_spin(B=1, N=6)
    amp0 = p.u[0].astype(float)
    _, _, grad = O.fidelity_and_gradient(p, 0, model=model)
    # central differences in normalised amplitude units, h = 1e-6
    fd = _fd_grad(p, 0, amp0, model, 1e-6 * p.u_scale)
    assert np.linalg.norm(grad - fd) <= 1e-7 * np.linalg.norm(fd)


@pytest.mark.parametrize("origin", [(0.0, 0.0), (-0.0, 0.0), (-0.0, -0.0), (0.0, -0.0)])
def test_t12_gradient_at_the_origin_vs_central_differences(origin):
    """A phased channel at the origin: the Cartesian derivatives are those of
    exp(-i dt (u_x S + u_y S^y)), which do not depend on the phase of the zero pair
    (atan2 gives +-pi for a negative zero): every signed zero gives the central
    differences taken across the origin."""
    p = W.c1_two_spin(B=1, N=6)
    amp0 = p.u[0].astype(float)
    amp0[2, 0, :] = origin
    fd = np.zeros(2)
    h = 1e-6 * p.u_scale
    for a in range(2):
        a1 = amp0.copy(); a1[2, 0, a] = h
        a2 = amp0.copy(); a2[2, 0, a] = -h
        F1 = O.fidelity_and_gradient(p, 0, model="split", amps=a1)[0]
        F2 = O.fidelity_and_gradient(p, 0, model="split", amps=a2)[0]
        fd[a] = (F1 - F2) / (2 * h)
    _, _, grad = O.fidelity_and_gradient(p, 0, model="split", amps=amp0)
    assert np.linalg.norm(grad[2, 0] - fd) <= 1e-6 * np.linalg.norm(fd), (grad[2, 0], fd)


def test_t12_gradient_vs_central_differences_signed():
    p = W.ising_freezing(n=3, B=1, N=8)
    p.U_target = W.haar_unitary(8, W.rng(3, 2, 0))[None]
    amp0 = p.u[0].astype(float)
    for model in ("split", "exact"):
        _, _, grad = O.fidelity_and_gradient(p, 0, model=model)
        fd = _fd_grad(p, 0, amp0, model, 1e-6 * p.u_scale)
        assert np.linalg.norm(grad - fd) <= 1e-7 * np.linalg.norm(fd)


def test_t12_redo_gradient_is_split_gradient_at_quantised_point():
    p = W.nmr_chain(3, 1, 10, 2e-6, 32, 2, 44, per_spin=True)
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    Fr, _, gr = O.fidelity_and_gradient(p, 0, model="redo", table=tab)
    qz = O.quantise(p.u[0], p.eps, p.base, p.digits, phased=True)
    om = qz["q"] * p.eps
    amp_q = np.stack([om * np.cos(qz["phi"]), om * np.sin(qz["phi"])], -1)
    fd = _fd_grad(p, 0, amp_q, "split", 1e-6 * p.u_scale)
    assert np.linalg.norm(gr - fd) <= 1e-7 * np.linalg.norm(fd)
    Fs = O.fidelity_and_gradient(p, 0, model="split", amps=amp_q)[0]
    assert abs(Fr - Fs) < 1e-12


def test_method_error_shrinks_with_eps():
    """Sec. II: coarse graining costs O(eps^2 dt^2) per factor; the REDO chain
    approaches the continuous split chain as the quantum shrinks."""
    p = W.c1_two_spin(B=1, N=50)
    V = O.drift_propagator(p.H0[0], p.dt, True)
    Xs = O.chain([O.step_split(p.S, p.g, p.u[0, n].astype(float), p.dt, V) for n in range(p.N)])
    errs = []
    for base in (4, 16, 64):
        p.base, p.digits = base, 2
        p.eps = math.sqrt(2) * p.u_scale / (base ** 2 - 1)
        tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
        Xr = O.chain(O.compose_all_redo(p, tab, 0))
        errs.append(np.linalg.norm(Xr - Xs) / 2)
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-3


def test_t1_exact_step_is_rotation_about_total_field():
    """One spin, drift nu I_z, Cartesian control (u_x, u_y): the unsplit step is
    a rotation by |B| dt about B = (u_x, u_y, nu)  (textbook closed form)."""
    p, nu = _one_spin_problem(N=10)
    H0m = np.diag(p.H0[0]).astype(complex)
    assert np.allclose(O.y_generator(SX / 2, np.array([0.5, -0.5])), SY / 2, atol=1e-15)
    for n in range(p.N):
        ux, uy = (float(v) for v in p.u[0, n, 0])
        B = np.array([ux, uy, nu])
        want = _rot(np.linalg.norm(B) * p.dt, B / np.linalg.norm(B))
        got = O.step_exact(H0m, p.S, p.g, p.u[0, n].astype(float), p.dt)
        assert np.abs(got - want).max() < 1e-14


def test_first_order_gradient_converges_to_exact_as_dt_shrinks():
    """The first-order GRAPE derivative -i dt H_k U_n differs from the exact
    derivative by O(dt^2) per step; at fixed total time its error relative to
    the exact gradient falls linearly with dt."""
    errs = []
    for N in (10, 20, 40):
        p = W.c1_two_spin(B=1, N=N)
        p.dt = 5e-6 * 10 / N
        _, _, ge = O.fidelity_and_gradient(p, 0, model="exact")
        _, _, g1 = O.fidelity_and_gradient(p, 0, model="exact_first_order")
        errs.append(np.linalg.norm(g1 - ge) / np.linalg.norm(ge))
    assert errs[0] > errs[1] > errs[2]
    assert 1.6 < errs[0] / errs[1] < 2.5 and 1.6 < errs[1] / errs[2] < 2.5


def test_mlp_oracle_gradients_vs_central_differences():
    from oracle import mlp_oracle as M
    rng = np.random.default_rng(13)
    sizes = [6, 5, 4, 3]
    params = [(rng.normal(size=(o, i)) * 0.7, rng.normal(size=o) * 0.1) for i, o in zip(sizes[:-1], sizes[1:])]
    x = rng.normal(size=(7, sizes[0]))
    t = rng.uniform(-0.9, 0.9, size=(7, sizes[-1]))
    loss, grads, _ = M.mlp_loss_and_grads(params, x, t)
    h = 1e-6
    for l, (W, b) in enumerate(params):
        for arr, g in ((W, grads[l][0]), (b, grads[l][1])):
            fd = np.zeros_like(arr)
            for idx in np.ndindex(*arr.shape):
                old = arr[idx]
                arr[idx] = old + h
                lp = M.mlp_loss_and_grads(params, x, t)[0]
                arr[idx] = old - h
                lm = M.mlp_loss_and_grads(params, x, t)[0]
                arr[idx] = old
                fd[idx] = (lp - lm) / (2 * h)
            assert np.linalg.norm(g - fd) <= 1e-7 * max(np.linalg.norm(fd), 1e-12)


def test_canonical_features_remove_global_phase():
    from oracle import mlp_oracle as M
    U = W.haar_unitary(4, W.rng(5, 2, 0))
    a = M.canonical_target_features(U)
    b = M.canonical_target_features(np.exp(1.3j) * U)
    assert a.shape == (32,) and np.abs(a - b).max() < 1e-12


# ------------------------------------------------------------------ Strang splitting (NEXT row f1)
def _local_errors(p, dts, splitting):
    """|U_split(dt) - U_exact(dt)| of one step for the given step lengths."""
    out = []
    amp = p.u[0, 0].astype(float)
    H0m = np.diag(p.H0[0]).astype(np.complex128)
    for dt in dts:
        V = O.drift_propagator(p.H0[0], dt, True)
        Vh = O.drift_propagator(p.H0[0], dt / 2, True) if splitting == "strang" else None
        Us = O.step_split(p.S, p.g, amp, dt, V, Vh)
        Ue = O.step_exact(H0m, p.S, p.g, amp, dt)
        out.append(np.linalg.norm(Us - Ue))
    return np.array(out)


def test_strang_step_is_third_order_lie_second_order():
    """Local error of one step: Lie (the paper's split) O(dt^2), Strang O(dt^3):
    halving dt divides it by ~4 and ~8."""
    p = W.c1_two_spin(B=1, N=1)
    dts = 2e-5 / 2.0 ** np.arange(4)
    el = _local_errors(p, dts, "lie")
    es = _local_errors(p, dts, "strang")
    rl, rs = el[:-1] / el[1:], es[:-1] / es[1:]
    assert np.all(np.abs(rl - 4) < 0.25), rl
    assert np.all(np.abs(rs - 8) < 0.5), rs


def test_strang_step_matches_bch_to_fifth_order():
    """exp(A/2) exp(B) exp(A/2) = exp(A + B - [A,[A,B]]/24 - [B,[A,B]]/12 + O(5))
    (symmetric BCH, A = -i dt H0, B = -i dt H_c): the residual after the two
    third-order terms falls ~32x per halving of dt."""
    p = W.c1_two_spin(B=1, N=1)
    amp = p.u[0, 0].astype(float)
    H0m = np.diag(p.H0[0]).astype(np.complex128)
    # the control Hamiltonian of the step: sum_k u_x S_k + u_y S_k^y
    Hc_gen = sum(amp[k, 0] * p.S[k] + amp[k, 1] * O.y_generator(p.S[k], p.g[k]) for k in range(p.K))
    res = []
    for dt in 1e-5 / 2.0 ** np.arange(3):
        A, Bm = -1j * dt * H0m, -1j * dt * Hc_gen
        comm = lambda X, Y: X @ Y - Y @ X
        G = A + Bm - comm(A, comm(A, Bm)) / 24 - comm(Bm, comm(A, Bm)) / 12
        w2, Q2 = np.linalg.eig(G)
        E = Q2 @ np.diag(np.exp(w2)) @ np.linalg.inv(Q2)
        Vh = O.drift_propagator(p.H0[0], dt / 2, True)
        Ustr = Vh @ O.expm_herm(Hc_gen, dt) @ Vh
        res.append(np.linalg.norm(Ustr - E))
    res = np.array(res)
    r = res[:-1] / res[1:]
    assert np.all(r > 24), (res, r)


def test_strang_chain_is_lie_chain_conjugated_by_half_drift():
    """prod_n Vh C_n Vh = Vh (prod_n C_n V) Vh^dag: the Strang chain is the Lie
    chain conjugated by the half-step drift."""
    p = W.c1_two_spin(B=1, N=30)
    ps = W.Problem(**{**p.__dict__, "splitting": "strang"})
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    Xl = O.chain(O.compose_all_redo(p, tab, 0))
    Xs = O.chain(O.compose_all_redo(ps, tab, 0))
    Vh = O.drift_propagator(p.H0[0], p.dt / 2, True)
    assert np.linalg.norm(Xs - Vh @ Xl @ Vh.conj().T) < 1e-12
    assert np.linalg.norm(Xs - Xl) > 1e-6


@pytest.mark.parametrize("maker", ["phased", "signed"])
def test_strang_gradient_vs_central_differences(maker):
    if maker == "phased":
        p = W.c1_two_spin(B=1, N=6)
    else:
        p = W.ising_freezing(n=3, B=1, N=8)
        p.U_target = W.haar_unitary(8, W.rng(3, 2, 0))[None]
    p = W.Problem(**{**p.__dict__, "splitting": "strang"})
    amp0 = p.u[0].astype(float)
    _, _, grad = O.fidelity_and_gradient(p, 0, model="split")
    fd = _fd_grad(p, 0, amp0, "split", 1e-6 * p.u_scale)
    assert np.linalg.norm(grad - fd) <= 1e-7 * np.linalg.norm(fd)


# ------------------------------------------------------------------ state-transfer fidelity (NEXT row f2)
def _fd_state(p, b, amp0, psi0, psif, model, h):
    fd = np.zeros_like(amp0)
    for idx in np.ndindex(*amp0.shape):
        a1 = amp0.copy(); a1[idx] += h
        a2 = amp0.copy(); a2[idx] -= h
        F1 = O.state_fidelity_and_gradient(p, b, psi0, psif, model=model, amps=a1)[0]
        F2 = O.state_fidelity_and_gradient(p, b, psi0, psif, model=model, amps=a2)[0]
        fd[idx] = (F1 - F2) / (2 * h)
    return fd


def test_state_fidelity_single_spin_closed_form():
    """One spin, no drift, x drive of area theta: |<up| exp(-i theta I_x) |up>|^2 = cos^2(theta/2)."""
    S = W.collective(1, [0], "x")[None]
    dt, N = 1e-5, 7
    u = np.full((1, N, 1), 2 * np.pi * 3e3, np.float32)
    p = W.Problem("spin", 2, 1, False, np.zeros((1, 2)), True, S, None, dt, 1.0, 2, 1, u)
    up = np.array([1.0, 0.0])
    F, g, _ = O.state_fidelity_and_gradient(p, 0, up, up, model="split")
    theta = float(u[0, 0, 0]) * dt * N
    assert abs(F - np.cos(theta / 2) ** 2) < 1e-12
    dn = np.array([0.0, 1.0])
    F2, _, _ = O.state_fidelity_and_gradient(p, 0, up, dn, model="split")
    assert abs(F2 - np.sin(theta / 2) ** 2) < 1e-12


def test_state_fidelity_is_a_propagator_entry_and_gradient_matches_fd():
    p = W.c1_two_spin(B=1, N=6)
    tab = O.DiscreteTable(p.S, p.dt, p.eps, p.base, p.digits)
    X = O.chain(O.compose_all_redo(p, tab, 0))
    e = np.eye(4)
    F, g, _ = O.state_fidelity_and_gradient(p, 0, e[1], e[2], model="redo", table=tab)
    assert abs(g - X[2, 1]) < 1e-12 and abs(F - abs(X[2, 1]) ** 2) < 1e-12
    rng = np.random.default_rng(5)
    psi0 = rng.normal(size=4) + 1j * rng.normal(size=4)
    psif = rng.normal(size=4) + 1j * rng.normal(size=4)
    psi0 /= np.linalg.norm(psi0)
    psif /= np.linalg.norm(psif)
    for model in ("split", "exact"):
        _, _, grad = O.state_fidelity_and_gradient(p, 0, psi0, psif, model=model)
        fd = _fd_state(p, 0, p.u[0].astype(float), psi0, psif, model, 1e-6 * p.u_scale)
        assert np.linalg.norm(grad - fd) <= 1e-7 * np.linalg.norm(fd)


def test_lbfgs_oracle_two_loop_equals_explicit_bfgs_inverse():
    """The oracle's two-loop direction equals the explicit BFGS inverse-update matrix
    applied to g (a different computation of the same estimate), and the estimate
    satisfies the secant condition H y = s of its newest pair."""
    import numpy as np
    import oracle as O
    rng = np.random.default_rng(17)
    n = 40
    A = rng.normal(size=(n, n))
    A = A @ A.T / n + 0.3 * np.eye(n)
    pairs = []
    for _ in range(6):
        s = rng.normal(size=n)
        pairs.append((s, A @ s))
    g = rng.normal(size=n)
    s_new, y_new = pairs[-1]
    gamma = (s_new @ y_new) / (y_new @ y_new)
    H = O.bfgs_inverse_matrix(pairs, gamma)
    d = O.lbfgs_direction(g, pairs, 1.0)
    assert np.abs(d - H @ g).max() <= 1e-10 * np.abs(H @ g).max()
    assert np.abs(O.lbfgs_direction(y_new, pairs, 1.0) - s_new).max() <= 1e-10 * np.abs(s_new).max()
    # no history: the gradient scaled to gamma0 in its largest entry
    d0 = O.lbfgs_direction(g, [], 2.5)
    assert abs(np.abs(d0).max() - 2.5) < 1e-12 and np.allclose(d0 / g, d0[0] / g[0])
