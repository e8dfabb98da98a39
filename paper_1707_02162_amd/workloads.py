"""Seeded synthetic inputs for the REDO propagator path.

This module only *draws* problem inputs: spin operators, drift Hamiltonians,
control generators, amplitude sequences, Haar-random targets and noise.  It
holds none of the method's arithmetic (no quantisation, no exponentials, no
products of propagators), so both the FP64 oracle and the GPU library can be
fed from it without sharing any of the computation they are compared on.

Physics follows the paper's NMR setting (Sec. III: internal Hamiltonian with
offsets and couplings, RF controls on collective spin operators of a species)
and the Ising chain of Sec. IV (exotic freezing under a transverse drive).

Every random draw comes from ``numpy.random.Generator(PCG64(SeedSequence(
[170702162, config_id, stream, instance])))`` so that any single instance can
be regenerated on its own.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

ROOT_SEED = 170702162

# stream ids inside one configuration
STREAM_DRIFT = 0
STREAM_PULSE = 1
STREAM_TARGET = 2
STREAM_NOISE = 3
STREAM_LENGTH = 4

TWO_PI = 2.0 * math.pi


def rng(config_id: int, stream: int, instance: int = 0) -> np.random.Generator:
    return np.random.Generator(
        np.random.PCG64(np.random.SeedSequence([ROOT_SEED, config_id, stream, instance])))


# ---------------------------------------------------------------------------
# spin-1/2 operators, qubit 1 is the most significant bit of the basis index
# ---------------------------------------------------------------------------
_PAULI = {
    "x": np.array([[0, 1], [1, 0]], dtype=np.complex128),
    "y": np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    "z": np.array([[1, 0], [0, -1]], dtype=np.complex128),
}


def spin_op(n: int, i: int, axis: str) -> np.ndarray:
    """I_{i,axis} = sigma_axis / 2 acting on spin i (0-based) of n spins."""
    out = np.ones((1, 1), dtype=np.complex128)
    for j in range(n):
        f = _PAULI[axis] / 2 if j == i else np.eye(2, dtype=np.complex128)
        out = np.kron(out, f)
    return out


def spin_z_diag(n: int, i: int) -> np.ndarray:
    """Diagonal of I_{i,z} as a real vector of length 2**n."""
    idx = np.arange(2 ** n)
    bit = (idx >> (n - 1 - i)) & 1
    return np.where(bit == 0, 0.5, -0.5).astype(np.float64)


def collective(n: int, spins, axis: str) -> np.ndarray:
    d = 2 ** n
    out = np.zeros((d, d), dtype=np.complex128)
    for i in spins:
        out += spin_op(n, i, axis)
    return out


def collective_z_diag(n: int, spins) -> np.ndarray:
    out = np.zeros(2 ** n)
    for i in spins:
        out += spin_z_diag(n, i)
    return out


def haar_unitary(d: int, gen: np.random.Generator) -> np.ndarray:
    """Haar-random unitary: QR of a complex Ginibre matrix with the phases of
    R's diagonal moved into Q (Mezzadri's construction)."""
    z = (gen.standard_normal((d, d)) + 1j * gen.standard_normal((d, d))) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    ph = np.diagonal(r) / np.abs(np.diagonal(r))
    return q * ph[None, :]


def smooth_pulse(n_steps: int, dt: float, gen: np.random.Generator, n_terms: int = 8) -> np.ndarray:
    """One Cartesian control component: a sum of ``n_terms`` seeded sinusoids
    sampled at segment midpoints and clipped to [-1, 1]."""
    T = n_steps * dt
    a = gen.uniform(-0.5, 0.5, n_terms)
    f = gen.uniform(0.0, 20.0 / T, n_terms)
    th = gen.uniform(0.0, TWO_PI, n_terms)
    t = (np.arange(n_steps) + 0.5) * dt
    s = (a[None, :] * np.sin(TWO_PI * f[None, :] * t[:, None] + th[None, :])).sum(axis=1)
    return np.clip(s, -1.0, 1.0)


# ---------------------------------------------------------------------------
# problem container
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Problem:
    """Inputs of one REDO workload.

    d, K          Hilbert dimension, number of control channels
    phased        True: channel k is driven by a Cartesian pair (u_x, u_y) and
                  rotated by the diagonal phase generator g[k];
                  False: channel k takes a signed amplitude u.
    H0            drift, real diagonal [n_drift, d] (drift_is_diag) or
                  complex dense [n_drift, d, d]; instance b uses b % n_drift
    S             control generators, complex Hermitian [K, d, d]
    g             phase generators, real [K, d] (phased) or None
    dt, eps       segment length (s), amplitude quantum (rad/s)
    base, digits  REDO base b and number of digits P (codes 0 .. b^P - 1)
    u             float32 amplitudes [B, N, K] or [B, N, K, 2] (rad/s)
    n_steps       int32 [B] per-instance lengths (None: all N)
    U_target      complex [B, d, d] targets (or None)
    M             observable, complex Hermitian [d, d] (or None)
    splitting     "lie": U_n = C_n V (drift first, the paper's split);
                  "strang": U_n = V(dt/2) C_n V(dt/2)
    """
    name: str
    d: int
    K: int
    phased: bool
    H0: np.ndarray
    drift_is_diag: bool
    S: np.ndarray
    g: Optional[np.ndarray]
    dt: float
    eps: float
    base: int
    digits: int
    u: np.ndarray
    n_steps: Optional[np.ndarray] = None
    U_target: Optional[np.ndarray] = None
    M: Optional[np.ndarray] = None
    u_scale: float = 1.0
    meta: dict = dataclasses.field(default_factory=dict)
    splitting: str = "lie"

    @property
    def B(self) -> int:
        return self.u.shape[0]

    @property
    def N(self) -> int:
        return self.u.shape[1]

    @property
    def n_drift(self) -> int:
        return self.H0.shape[0]

    def lengths(self) -> np.ndarray:
        if self.n_steps is None:
            return np.full(self.B, self.N, dtype=np.int32)
        return self.n_steps

    def subset(self, idx) -> "Problem":
        """The instances ``idx`` as a problem of their own (drift and target follow)."""
        idx = np.asarray(idx)
        drift_idx = idx % self.n_drift
        return dataclasses.replace(
            self,
            u=self.u[idx].copy(),
            H0=self.H0[drift_idx].copy(),
            n_steps=None if self.n_steps is None else self.n_steps[idx].copy(),
            U_target=None if self.U_target is None else self.U_target[idx].copy(),
        )


def _nmr_chain_drift(n: int, gen: np.random.Generator, nu_khz: float = 10.0) -> np.ndarray:
    """Diagonal NMR drift 2*pi*(sum nu_i I_iz + sum J_i I_iz I_{i+1,z}),
    nu ~ U(-nu_khz, nu_khz) kHz, nearest-neighbour J ~ U(50, 250) Hz."""
    nu = gen.uniform(-nu_khz * 1e3, nu_khz * 1e3, n)
    J = gen.uniform(50.0, 250.0, max(n - 1, 0))
    h = np.zeros(2 ** n)
    for i in range(n):
        h += TWO_PI * nu[i] * spin_z_diag(n, i)
    for i in range(n - 1):
        h += TWO_PI * J[i] * spin_z_diag(n, i) * spin_z_diag(n, i + 1)
    return h


def _levels_eps(omega_max: float, levels: int) -> float:
    """Quantum such that [0, omega_max] is covered by codes 0 .. levels-1."""
    return omega_max / (levels - 1)


def c1_two_spin(B: int = 1, N: int = 200, config_id: int = 1) -> Problem:
    """Two spins (d=4): H0 = 2pi(nu1 Z1/2 + nu2 Z2/2) + 2pi J Z1Z2/4, nu ~ U(-5,5) kHz,
    J = 200 Hz; X/Y control on each spin as two phased channels; amplitudes
    U(-1,1) * 2pi*10 kHz per Cartesian component; N = 200 segments of 5 us;
    8-bit amplitude levels (b = 16, P = 2); Haar-random targets."""
    n, d = 2, 4
    dt = 5e-6
    scale = TWO_PI * 10e3
    g0 = rng(config_id, STREAM_DRIFT)
    nu = g0.uniform(-5e3, 5e3, 2)
    H0 = (TWO_PI * (nu[0] * spin_z_diag(n, 0) + nu[1] * spin_z_diag(n, 1))
          + TWO_PI * 200.0 * spin_z_diag(n, 0) * spin_z_diag(n, 1))[None, :]
    S = np.stack([spin_op(n, 0, "x"), spin_op(n, 1, "x")])
    g = np.stack([spin_z_diag(n, 0), spin_z_diag(n, 1)])
    u = np.empty((B, N, 2, 2), dtype=np.float32)
    Uf = np.empty((B, d, d), dtype=np.complex128)
    for b in range(B):
        u[b] = (rng(config_id, STREAM_PULSE, b).uniform(-1.0, 1.0, (N, 2, 2)) * scale).astype(np.float32)
        Uf[b] = haar_unitary(d, rng(config_id, STREAM_TARGET, b))
    eps = _levels_eps(math.sqrt(2.0) * scale, 256)
    return Problem("c1_two_spin", d, 2, True, H0, True, S, g, dt, eps, 16, 2, u,
                   None, Uf, None, u_scale=scale)


def nmr_chain(n: int, B: int, N: int, dt: float, base: int, digits: int, config_id: int,
              per_spin: bool = False, species=None, n_drift: int = 1, targets: bool = True,
              lengths=None, name: str = "nmr_chain") -> Problem:
    """n-spin NMR chain with offsets U(-10,10) kHz and nearest-neighbour ZZ
    couplings U(50,250) Hz.  Controls: one collective X/Y phased channel
    (default), one phased channel per spin (per_spin), or one per species
    (species = list of spin lists).  Smooth seeded pulses scaled by 2pi*10 kHz."""
    d = 2 ** n
    scale = TWO_PI * 10e3
    H0 = np.stack([_nmr_chain_drift(n, rng(config_id, STREAM_DRIFT, i)) for i in range(n_drift)])
    if species is None:
        species = [[i] for i in range(n)] if per_spin else [list(range(n))]
    K = len(species)
    S = np.stack([collective(n, sp, "x") for sp in species])
    g = np.stack([collective_z_diag(n, sp) for sp in species])
    u = np.zeros((B, N, K, 2), dtype=np.float32)
    n_steps = None if lengths is None else np.asarray(lengths, dtype=np.int32)
    for b in range(B):
        gen = rng(config_id, STREAM_PULSE, b)
        nb = N if n_steps is None else int(n_steps[b])
        for k in range(K):
            for a in range(2):
                u[b, :nb, k, a] = (smooth_pulse(nb, dt, gen) * scale).astype(np.float32)
    Uf = None
    if targets:
        Uf = np.stack([haar_unitary(d, rng(config_id, STREAM_TARGET, b)) for b in range(B)])
    levels = base ** digits
    eps = _levels_eps(math.sqrt(2.0) * scale, levels)
    return Problem(name, d, K, True, H0, True, S, g, dt, eps, base, digits, u,
                   n_steps, Uf, None, u_scale=scale)


def c2_six_qubit(B: int = 1, N: int = 2000, config_id: int = 2) -> Problem:
    """6-qubit chain (d=64), collective X/Y, N=2000 x 2 us, 10-bit levels (b=32, P=2)."""
    return nmr_chain(6, B, N, 2e-6, 32, 2, config_id, name="c2_six_qubit")


def c4_batched_grape(B: int = 64, n_min: int = 500, n_max: int = 3000, config_id: int = 4) -> Problem:
    """64 independent 5-qubit systems (d=32) with their own drift and Haar target,
    uneven lengths N_b ~ U{n_min..n_max}, X/Y on every spin (5 phased channels),
    2 us segments, b=32, P=2."""
    lens = rng(config_id, STREAM_LENGTH).integers(n_min, n_max + 1, B).astype(np.int32)
    return nmr_chain(5, B, int(lens.max()), 2e-6, 32, 2, config_id, per_spin=True,
                     n_drift=B, lengths=lens, name="c4_batched_grape")


def c5_four_qubit(B: int = 1, N: int = 500, config_id: int = 5, targets: bool = True) -> Problem:
    """4 qubits (d=16), two species {1,2}, {3,4} with collective X/Y each
    (2 phased channels = 4 Cartesian controls), N=500 x 2 us, b=32, P=2."""
    return nmr_chain(4, B, N, 2e-6, 32, 2, config_id, species=[[0, 1], [2, 3]],
                     targets=targets, name="c5_four_qubit")


def c6_grape_1024(B: int = 1, N: int = 500, config_id: int = 6) -> Problem:
    """10-qubit NMR chain (d=1024), one collective X/Y channel, N=500 x 2 us,
    b=32, P=2, Haar target."""
    return nmr_chain(10, B, N, 2e-6, 32, 2, config_id, name="c6_grape_1024")


def ising_freezing(n: int = 10, B: int = 4096, N: int = 5000, sigma: float = 0.05,
                   h0: float = TWO_PI * 20e3, J_ratio: float = 1.0 / 20.0, h0dt: float = 0.1,
                   omega: Optional[float] = None, base: int = 100, digits: int = 2,
                   u_max_ratio: float = 1.3, config_id: int = 3, J: Optional[float] = None,
                   name: str = "c3_ising_freezing") -> Problem:
    """Open Ising chain of n spins under a noisy transverse drive (Sec. IV):
    H_n = -J sum_i 2 I_iz I_{i+1,z} + u_n sum_i I_ix with u_n = -h0 a_n,
    a_n = cos(omega t_n) + sigma xi_n, xi ~ N(0,1), t_n = (n - 1/2) dt.
    Defaults: h0 = 2pi*20 kHz, J = h0/20, h0 dt = 0.1, omega at the first zero
    of J0(2 h0 / omega), signed single-axis channel, b=100, P=2 over
    |u| <= 1.3 h0.  Observable and initial state M = sum_i I_ix."""
    d = 2 ** n
    dt = h0dt / h0
    if J is None:
        J = J_ratio * h0
    if omega is None:
        omega = 2.0 * h0 / 2.404825557695773
    h = np.zeros(d)
    for i in range(n - 1):
        h += -J * 2.0 * spin_z_diag(n, i) * spin_z_diag(n, i + 1)
    H0 = h[None, :]
    S = collective(n, range(n), "x")[None]
    t = (np.arange(N) + 0.5) * dt
    u = np.empty((B, N, 1), dtype=np.float32)
    for b in range(B):
        xi = rng(config_id, STREAM_NOISE, b).standard_normal(N)
        u[b, :, 0] = (-h0 * (np.cos(omega * t) + sigma * xi)).astype(np.float32)
    levels = base ** digits
    eps = _levels_eps(u_max_ratio * h0, levels)
    M = collective(n, range(n), "x")
    return Problem(name, d, 1, False, H0, True, S, None, dt, eps, base, digits, u,
                   None, None, M, u_scale=h0,
                   meta=dict(h0=h0, J=J, omega=omega, sigma=sigma, n_spins=n))


def freezing_sweep(omegas, lambdas, n: int = 3, N: int = 10000, T: float = 20.0 * math.pi,
                   h0: float = 5.0 * math.pi, J_ratio: float = 1.0 / 20.0, base: int = 100, digits: int = 2,
                   coef_eps: float = 1e-4, config_id: int = 7, first: int = 0, count: Optional[int] = None,
                   name: str = "freezing_sweep") -> Problem:
    """The paper's noisy-drive freezing sweep (Sec. IV): an open chain of n
    spins, H(t) = -J sum_i 2 I_iz I_{i+1,z} - h0 c(t) sum_i I_ix with drive
    coefficient c(t) = (1 - lambda) cos(omega t) + lambda eta(t), eta ~ U(-1, 1)
    drawn per time point, J = h0/20, h0 = 5 pi; N time points over [0, T]
    (midpoints of N segments); c is coarse grained with quantum coef_eps
    (b = 100, l = -2, m = -1: eps = 1e-4, P = 2).  Instances are the pairs
    (omega_i, lambda_j), instance index j * len(omegas) + i; this returns
    instances first .. first + count - 1 (seeded per instance index).
    Observable and initial state M = sum_i I_ix; the order parameter is the
    time average of Tr(X M X^dag M) / Tr(M^2)."""
    omegas = np.asarray(omegas, dtype=np.float64)
    lambdas = np.asarray(lambdas, dtype=np.float64)
    total = len(omegas) * len(lambdas)
    if count is None:
        count = total - first
    d = 2 ** n
    dt = T / N
    J = J_ratio * h0
    h = np.zeros(d)
    for i in range(n - 1):
        h += -J * 2.0 * spin_z_diag(n, i) * spin_z_diag(n, i + 1)
    S = collective(n, range(n), "x")[None]
    t = (np.arange(N) + 0.5) * dt
    u = np.empty((count, N, 1), dtype=np.float32)
    om = np.empty(count)
    la = np.empty(count)
    for r in range(count):
        idx = first + r
        om[r] = omegas[idx % len(omegas)]
        la[r] = lambdas[idx // len(omegas)]
        eta = rng(config_id, STREAM_NOISE, idx).uniform(-1.0, 1.0, N)
        u[r, :, 0] = (-h0 * ((1.0 - la[r]) * np.cos(om[r] * t) + la[r] * eta)).astype(np.float32)
    return Problem(name, d, 1, False, h[None, :], True, S, None, dt, coef_eps * h0, base, digits, u,
                   None, None, S[0].copy(), u_scale=h0,
                   meta=dict(h0=h0, J=J, omega=om, lam=la, first=first, n_spins=n))


def observable_ell(M: np.ndarray):
    """A Hermitian observable as fixed-width row lists (ELL): for each row a the
    column indices and values of its nonzeros, padded with (a, 0).  Returns
    (cols int32 [d, w], vals complex128 [d, w])."""
    d = M.shape[0]
    nz = [np.nonzero(M[a])[0] for a in range(d)]
    w = max(1, max(len(x) for x in nz))
    cols = np.empty((d, w), dtype=np.int32)
    vals = np.zeros((d, w), dtype=np.complex128)
    for a in range(d):
        cols[a, :] = a
        cols[a, :len(nz[a])] = nz[a]
        vals[a, :len(nz[a])] = M[a, nz[a]]
    return cols, vals
