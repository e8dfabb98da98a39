"""FP64 oracle: REDO (Bhole & Mahesh, arXiv 1707.02162) written from its definitions.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy in float64 /
complex128, written for a reader to check against the paper by eye: no
blocking, fusion or reordering beyond what each definition states.

Three propagator models are kept apart:

* EXACT  U_n = exp[-i dt (H0 + H_n)]                     (Sec. III, Eq. propUn)
* SPLIT  U_n = Z_n (prod_k X_kn) Z_n^dag V(dt)           (Sec. III, Eqs. vn, vnd:
         the Dirac-frame step rewritten in the lab frame; see ``dirac_step``)
* REDO   SPLIT with every X_kn replaced by a product of table entries
         (Sec. II, processes 1 and 2, Eqs. cgrain, redoform, exp2prod)

Readings of the paper used here (each is listed with its reason in the design doc):
the table entry for digit j and coefficient c is exp(-i c b^j eps dt S)
(the printed exponent of Eq. redoform lacks dt and flips the sign of j,
against Eq. cgrain and the worked example); rounding is to nearest with ties
up on the magnitude, codes clamp at b^P - 1; a signed single-axis amplitude
uses the adjoint factor for negative values; the fidelity normaliser is
Tr(U_f^dag U_f).

Parity pins (tests/test_oracle_pins.py): closed-form spin rotations, the
paper's worked example of the digit split, the cost model, the quantisation
fidelity closed form, the Dirac-frame identity, commuting-chain closed forms,
the Ising special cases, d=2 brute force, invariants and central finite
differences of the gradients.  The MLP oracle lives in ``mlp_oracle``.
"""
from __future__ import annotations

import math
from typing import Dict, Optional, Tuple

import numpy as np

__all__ = [
    "expm_herm", "frechet_expm", "y_generator", "digits_needed", "quantise",
    "DiscreteTable", "drift_propagator", "phase_diag", "step_redo", "step_split",
    "step_exact", "dirac_step", "chain", "unitary_fidelity", "fidelity_and_gradient",
    "magnetisation", "magnetisation_series", "compose_all_redo", "with_drift",
    "state_fidelity_and_gradient",
]


# ---------------------------------------------------------------------------
# exponentials (Sec. II, Eq. untilde: exp(-i Omega dt S) for Hermitian S)
# ---------------------------------------------------------------------------
def _check_hermitian(H: np.ndarray) -> None:
    nrm = np.linalg.norm(H)
    if np.linalg.norm(H - H.conj().T) > 1e-12 * max(nrm, 1e-300):
        raise ValueError("operator is not Hermitian")


def expm_herm(H: np.ndarray, t: float) -> np.ndarray:
    """exp(-i t H) for Hermitian H, from H = W diag(lam) W^dag (numpy eigh)."""
    H = np.asarray(H, dtype=np.complex128)
    _check_hermitian(H)
    lam, W = np.linalg.eigh(H)
    return (W * np.exp(-1j * t * lam)[None, :]) @ W.conj().T


def frechet_expm(H: np.ndarray, t: float, E: np.ndarray) -> np.ndarray:
    """Directional derivative of exp(A), A = -i t H (H Hermitian), in direction
    E: the Daleckii-Krein formula L(A, E) = W [(W^dag E W) o D] W^dag with
    D_pq = (e^{a_p} - e^{a_q}) / (a_p - a_q)  (e^{a_p} when a_p = a_q)."""
    H = np.asarray(H, dtype=np.complex128)
    _check_hermitian(H)
    lam, W = np.linalg.eigh(H)
    a = -1j * t * lam
    ea = np.exp(a)
    delta = a[:, None] - a[None, :]
    small = np.abs(delta) < 1e-300
    safe = np.where(small, 1.0, delta)
    # e^{a_q} (e^{delta} - 1) / delta, stable for small delta
    D = np.where(small, ea[None, :] * np.ones_like(delta), ea[None, :] * np.expm1(delta) / safe)
    Et = W.conj().T @ E @ W
    return W @ (Et * D) @ W.conj().T


def y_generator(S: np.ndarray, g: np.ndarray) -> np.ndarray:
    """y-partner of a phased x-generator: exp(-i pi/2 G) S exp(+i pi/2 G), G = diag(g)."""
    ph = np.exp(-0.5j * math.pi * g)
    return ph[:, None] * S * ph.conj()[None, :]


# ---------------------------------------------------------------------------
# coarse graining (Sec. II, Eq. cgrain and the worked example that follows it)
# ---------------------------------------------------------------------------
def digits_needed(ratio: float, base: int) -> Tuple[int, int, int]:
    """Smallest P with b^P - 1 >= ceil(Omega_max/eps); returns (P, p = P-1
    multiplications, s = (b-1) P stored operators)  (Sec. II, cost model)."""
    need = math.ceil(ratio)
    P = 1
    while base ** P - 1 < need:
        P += 1
    return P, P - 1, (base - 1) * P


def quantise(u: np.ndarray, eps: float, base: int, digits: int, phased: bool) -> Dict[str, np.ndarray]:
    """Coarse-grain amplitudes into base-b digits (Sec. II, Eq. cgrain).

    u: float32 [..., K] (signed single-axis) or [..., K, 2] (Cartesian pair).
    Magnitude Omega = |u| or sqrt(u_x^2 + u_y^2) (float64 from the float32
    inputs), code q = min(floor(Omega/eps + 1/2), b^P - 1), digits
    c_j = floor(q / b^j) mod b by integer arithmetic, j = 0 .. P-1.
    Returns q, c [..., P], sign (+1/-1, +1 at zero), phi (phased: atan2(u_y, u_x)),
    omega (unquantised magnitude) and clamped (bool)."""
    u = np.asarray(u, dtype=np.float32)
    if phased:
        ux = u[..., 0].astype(np.float64)
        uy = u[..., 1].astype(np.float64)
        omega = np.sqrt(ux * ux + uy * uy)
        phi = np.arctan2(uy, ux)
        sign = np.ones_like(omega)
    else:
        x = u.astype(np.float64)
        omega = np.abs(x)
        phi = None
        sign = np.where(x < 0, -1.0, 1.0)
    if not np.all(np.isfinite(omega)):
        raise ValueError("non-finite amplitude")
    qf = np.floor(omega / eps + 0.5)
    qmax = base ** digits - 1
    clamped = qf > qmax
    q = np.minimum(qf, qmax).astype(np.int64)
    c = np.empty(q.shape + (digits,), dtype=np.int64)
    rest = q.copy()
    for j in range(digits):
        c[..., j] = rest % base
        rest = rest // base
    return dict(q=q, c=c, sign=sign, phi=phi, omega=omega, clamped=clamped)


# ---------------------------------------------------------------------------
# process 1: the discrete-operator table (Sec. II, Eq. redoform, reading R1)
# ---------------------------------------------------------------------------
class DiscreteTable:
    """T_k[j][c] = exp(-i c b^j eps dt S_k), c = 0 .. b-1 (c = 0 is the identity),
    j = 0 .. P-1.  Entries come from one eigendecomposition of each S_k and are
    computed on first use and kept."""

    def __init__(self, S: np.ndarray, dt: float, eps: float, base: int, digits: int):
        self.S = np.asarray(S, dtype=np.complex128)
        self.dt, self.eps, self.base, self.digits = float(dt), float(eps), int(base), int(digits)
        self.K, self.d = self.S.shape[0], self.S.shape[1]
        self._eig = []
        for k in range(self.K):
            _check_hermitian(self.S[k])
            self._eig.append(np.linalg.eigh(self.S[k]))
        self._cache: Dict[Tuple[int, int, int], np.ndarray] = {}

    @property
    def stored_entries(self) -> int:
        """Number of non-identity operators kept per channel: s = (b-1) P."""
        return (self.base - 1) * self.digits

    def entry(self, k: int, j: int, c: int) -> np.ndarray:
        key = (k, j, int(c))
        if key not in self._cache:
            if c == 0:
                self._cache[key] = np.eye(self.d, dtype=np.complex128)
            else:
                lam, W = self._eig[k]
                theta = c * (self.base ** j) * self.eps * self.dt
                self._cache[key] = (W * np.exp(-1j * theta * lam)[None, :]) @ W.conj().T
        return self._cache[key]

    def factor(self, k: int, cdig, sign: float = 1.0) -> np.ndarray:
        """Process 2 (Eq. exp2prod): R = T[0][c_0] T[1][c_1] ... T[P-1][c_{P-1}],
        identity digits skipped; the adjoint for a negative signed amplitude."""
        R = np.eye(self.d, dtype=np.complex128)
        for j in range(self.digits):
            if cdig[j] != 0:
                R = R @ self.entry(k, j, cdig[j])
        if sign < 0:
            R = R.conj().T
        return R


# ---------------------------------------------------------------------------
# steps (Sec. III, Eqs. propUn, vn, vnd)
# ---------------------------------------------------------------------------
def drift_propagator(H0: np.ndarray, dt: float, is_diag: bool) -> np.ndarray:
    """V(dt) = exp(-i dt H0); H0 real diagonal vector or dense Hermitian matrix."""
    if is_diag:
        return np.diag(np.exp(-1j * dt * np.asarray(H0, dtype=np.float64)))
    return expm_herm(H0, dt)


def phase_diag(phi: np.ndarray, g: np.ndarray) -> np.ndarray:
    """Z = exp(-i sum_k phi_k G_k), G_k = diag(g_k): a diagonal matrix."""
    theta = (np.asarray(phi)[:, None] * np.asarray(g)).sum(axis=0)
    return np.diag(np.exp(-1j * theta))


def _control_block(factors, Z: Optional[np.ndarray]) -> np.ndarray:
    """prod_k factors[k] with k = 0 rightmost, conjugated by Z when phased."""
    d = factors[0].shape[0]
    P = np.eye(d, dtype=np.complex128)
    for F in factors:
        P = F @ P
    if Z is not None:
        P = Z @ P @ Z.conj().T
    return P


def with_drift(C: np.ndarray, V: np.ndarray, Vh: Optional[np.ndarray] = None) -> np.ndarray:
    """The split step around the control block C: C V (the paper's split, drift
    first), or the symmetric Strang form V(dt/2) C V(dt/2) when the half-step
    drift Vh is given."""
    if Vh is not None:
        return Vh @ C @ Vh
    return C @ V


def step_redo(table: DiscreteTable, qz: Dict[str, np.ndarray], V: np.ndarray,
              g: Optional[np.ndarray], Vh: Optional[np.ndarray] = None) -> np.ndarray:
    """U_n = Z_n (prod_k R_k) Z_n^dag V with R_k the REDO product of the codes of
    one step (qz entries indexed [K] / [K, P]); g is None for signed channels.
    With Vh (Strang): U_n = Vh Z_n (prod_k R_k) Z_n^dag Vh."""
    K = table.K
    if g is not None:
        factors = [table.factor(k, qz["c"][k]) for k in range(K)]
        Z = phase_diag(qz["phi"], g)
    else:
        factors = [table.factor(k, qz["c"][k], qz["sign"][k]) for k in range(K)]
        Z = None
    return with_drift(_control_block(factors, Z), V, Vh)


def step_split(S: np.ndarray, g: Optional[np.ndarray], amp: np.ndarray, dt: float,
               V: np.ndarray, Vh: Optional[np.ndarray] = None) -> np.ndarray:
    """Continuous split step with exact factors X_k = exp(-i Omega_k dt S_k).
    amp: [K, 2] Cartesian pairs (phased) or [K] signed amplitudes.  With the
    half-step drift Vh the step is the Strang form Vh C Vh."""
    amp = np.asarray(amp, dtype=np.float64)
    K = S.shape[0]
    if g is not None:
        om = np.sqrt(amp[:, 0] ** 2 + amp[:, 1] ** 2)
        phi = np.arctan2(amp[:, 1], amp[:, 0])
        factors = [expm_herm(S[k], om[k] * dt) for k in range(K)]
        Z = phase_diag(phi, g)
    else:
        factors = [expm_herm(S[k], amp[k] * dt) for k in range(K)]
        Z = None
    return with_drift(_control_block(factors, Z), V, Vh)


def step_exact(H0m: np.ndarray, S: np.ndarray, g: Optional[np.ndarray], amp: np.ndarray,
               dt: float) -> np.ndarray:
    """U_n = exp[-i dt (H0 + H_n)], H_n = sum_k Omega (cos phi S_k + sin phi S_k^y)
    = sum_k (u_x S_k + u_y S_k^y) for phased channels, sum_k u_k S_k otherwise."""
    amp = np.asarray(amp, dtype=np.float64)
    H = np.array(H0m, dtype=np.complex128)
    for k in range(S.shape[0]):
        if g is not None:
            H = H + amp[k, 0] * S[k] + amp[k, 1] * y_generator(S[k], g[k])
        else:
            H = H + amp[k] * S[k]
    return expm_herm(H, dt)


def dirac_step(H0m: np.ndarray, S: np.ndarray, g: np.ndarray, amp: np.ndarray, dt: float) -> np.ndarray:
    """The paper's Dirac-frame step, literally: U_n = V(dt) Z_n (prod_k Xt_kn) Z_n^dag
    with Xt_kn = exp(-i Omega_kn dt St_k), St_k = V^dag(dt) S_k V(dt)  (Sec. III)."""
    V = expm_herm(H0m, dt)
    amp = np.asarray(amp, dtype=np.float64)
    om = np.sqrt(amp[:, 0] ** 2 + amp[:, 1] ** 2)
    phi = np.arctan2(amp[:, 1], amp[:, 0])
    Z = phase_diag(phi, g)
    P = np.eye(H0m.shape[0], dtype=np.complex128)
    for k in range(S.shape[0]):
        St = V.conj().T @ S[k] @ V
        P = expm_herm(St, om[k] * dt) @ P
    return V @ Z @ P @ Z.conj().T


# ---------------------------------------------------------------------------
# chain, fidelity, observable (Sec. III, Sec. IV)
# ---------------------------------------------------------------------------
def chain(steps, X0: Optional[np.ndarray] = None, keep: bool = False):
    """X_0 = I (or X0), X_n = U_n X_{n-1}; the propagator is U = U_N ... U_1.
    Returns X_N, or the list [X_0, X_1, ..., X_N] when keep is set."""
    steps = list(steps)
    d = steps[0].shape[0] if steps else (X0.shape[0] if X0 is not None else 1)
    X = np.eye(d, dtype=np.complex128) if X0 is None else np.array(X0, dtype=np.complex128)
    out = [X] if keep else None
    for U in steps:
        X = U @ X
        if keep:
            out.append(X)
    return out if keep else X


def unitary_fidelity(Uf: np.ndarray, U: np.ndarray) -> Tuple[complex, float]:
    """g = Tr(U_f^dag U) / Tr(U_f^dag U_f) and F_U = |g|^2 (Sec. III)."""
    g = np.trace(Uf.conj().T @ U) / np.trace(Uf.conj().T @ Uf).real
    return complex(g), float(abs(g) ** 2)


def magnetisation(X: np.ndarray, M: np.ndarray) -> float:
    """<M>(t) / Tr(M^2) for rho(0) = M: Tr(X M X^dag M) / Tr(M M)  (Sec. IV)."""
    rho = X @ M @ X.conj().T
    return float(np.trace(rho @ M).real / np.trace(M @ M).real)


def magnetisation_series(steps, M: np.ndarray):
    """m_n for n = 1 .. N along the chain of ``steps``."""
    d = M.shape[0]
    X = np.eye(d, dtype=np.complex128)
    out = []
    for U in steps:
        X = U @ X
        out.append(magnetisation(X, M))
    return np.array(out), X


# ---------------------------------------------------------------------------
# whole-problem helpers (one instance at a time)
# ---------------------------------------------------------------------------
def _drift_of(prob, b: int):
    H0 = prob.H0[b % prob.n_drift]
    V = drift_propagator(H0, prob.dt, prob.drift_is_diag)
    H0m = np.diag(H0).astype(np.complex128) if prob.drift_is_diag else H0
    return V, H0m


def _half_drift(prob, b: int) -> Optional[np.ndarray]:
    """V(dt/2) of instance b for the Strang splitting, else None."""
    if getattr(prob, "splitting", "lie") != "strang":
        return None
    return drift_propagator(prob.H0[b % prob.n_drift], 0.5 * prob.dt, prob.drift_is_diag)


def _step_codes(qz, n: int):
    return {"c": qz["c"][n], "sign": qz["sign"][n], "phi": None if qz["phi"] is None else qz["phi"][n]}


def compose_all_redo(prob, table: DiscreteTable, b: int, n_steps: Optional[int] = None):
    """REDO steps U_1 .. U_{N_b} of instance b."""
    V, _ = _drift_of(prob, b)
    Vh = _half_drift(prob, b)
    nb = int(prob.lengths()[b]) if n_steps is None else n_steps
    qz = quantise(prob.u[b, :nb], prob.eps, prob.base, prob.digits, prob.phased)
    g = prob.g if prob.phased else None
    return [step_redo(table, _step_codes(qz, n), V, g, Vh) for n in range(nb)]


def _quantised_amplitudes(prob, b: int, nb: int) -> np.ndarray:
    """The straight-through point: Omega_hat (cos phi, sin phi) or sign * Omega_hat."""
    qz = quantise(prob.u[b, :nb], prob.eps, prob.base, prob.digits, prob.phased)
    om = qz["q"] * prob.eps
    if prob.phased:
        return np.stack([om * np.cos(qz["phi"]), om * np.sin(qz["phi"])], axis=-1), qz
    return qz["sign"] * om, qz


def fidelity_and_gradient(prob, b: int, model: str = "redo", table: Optional[DiscreteTable] = None,
                          amps: Optional[np.ndarray] = None):
    """F_U and dF_U/du for instance b.

    model "split": the continuous split model at the amplitudes ``amps``
      (default: the instance's own float amplitudes);
    model "redo": the same derivative at the quantised point (straight
      through), with every step built from REDO table products;
    model "exact": the unsplit step exp[-i dt (H0 + H_n)];
    model "exact_first_order": the unsplit step with the usual first-order
      GRAPE derivative dU_n/du ~ -i dt H_k U_n (the approximation of the
      GRAPE paper the method cites in Sec. III).

    The derivative of each step comes from Daleckii-Krein Frechet derivatives
    of its exponential factors; it is contracted with the chain as
    dg/dtheta = Tr(U_f^dag U_N..U_{n+1} dU_n U_{n-1}..U_1) / Tr(U_f^dag U_f),
    and dF = 2 Re(conj(g) dg).  Returns (F, g, grad) with grad shaped like
    u[b, :N_b]."""
    nb = int(prob.lengths()[b])
    V, H0m = _drift_of(prob, b)
    Vh = _half_drift(prob, b) if model in ("redo", "split") else None
    S, g = prob.S, (prob.g if prob.phased else None)
    K, d = prob.K, prob.d
    Uf = prob.U_target[b]
    if model == "redo":
        amp, qz = _quantised_amplitudes(prob, b, nb)
        steps = [step_redo(table, _step_codes(qz, n), V, g, Vh) for n in range(nb)]
    else:
        amp = (prob.u[b, :nb].astype(np.float64) if amps is None else np.asarray(amps, np.float64))
        if model == "split":
            steps = [step_split(S, g, amp[n], prob.dt, V, Vh) for n in range(nb)]
        elif model in ("exact", "exact_first_order"):
            steps = [step_exact(H0m, S, g, amp[n], prob.dt) for n in range(nb)]
        else:
            raise ValueError(model)
    prefix = chain(steps, keep=True)
    norm = np.trace(Uf.conj().T @ Uf).real
    gval = np.trace(Uf.conj().T @ prefix[-1]) / norm
    grad = np.zeros(amp.shape, dtype=np.float64)
    Lam = Uf.conj().T.copy()                      # U_f^dag U_N ... U_{n+1}
    for n in range(nb - 1, -1, -1):
        for key, dU in _step_derivatives(model, S, g, amp[n], prob.dt, V, H0m, K, d, Vh):
            dg = np.trace(Lam @ dU @ prefix[n]) / norm
            grad[(n,) + key] = 2.0 * (np.conj(gval) * dg).real
        Lam = Lam @ steps[n]
    return float(abs(gval) ** 2), complex(gval), grad


def state_fidelity_and_gradient(prob, b: int, psi0: np.ndarray, psif: np.ndarray, model: str = "redo",
                                table: Optional[DiscreteTable] = None, amps: Optional[np.ndarray] = None):
    """State fidelity of Sec. III, F_S = |<psi_f| U |psi_0>|^2 (unit vectors), and
    dF_S/du for instance b, with the same step models and step derivatives as
    fidelity_and_gradient:
        dg/dtheta_n = <psi_f| U_N .. U_{n+1} dU_n U_{n-1} .. U_1 |psi_0>,
        dF_S = 2 Re(conj(g) dg).
    Returns (F_S, g, grad) with grad shaped like u[b, :N_b]."""
    nb = int(prob.lengths()[b])
    V, H0m = _drift_of(prob, b)
    Vh = _half_drift(prob, b) if model in ("redo", "split") else None
    S, g = prob.S, (prob.g if prob.phased else None)
    K, d = prob.K, prob.d
    psi0 = np.asarray(psi0, dtype=np.complex128)
    psif = np.asarray(psif, dtype=np.complex128)
    if model == "redo":
        amp, qz = _quantised_amplitudes(prob, b, nb)
        steps = [step_redo(table, _step_codes(qz, n), V, g, Vh) for n in range(nb)]
    else:
        amp = (prob.u[b, :nb].astype(np.float64) if amps is None else np.asarray(amps, np.float64))
        if model == "split":
            steps = [step_split(S, g, amp[n], prob.dt, V, Vh) for n in range(nb)]
        elif model == "exact":
            steps = [step_exact(H0m, S, g, amp[n], prob.dt) for n in range(nb)]
        else:
            raise ValueError(model)
    psi = [psi0]                                  # psi_n = U_n .. U_1 psi_0
    for U in steps:
        psi.append(U @ psi[-1])
    gval = np.vdot(psif, psi[-1])
    grad = np.zeros(amp.shape, dtype=np.float64)
    chi = psif.copy()                             # chi_n = U_{n+1}^dag .. U_N^dag psi_f
    for n in range(nb - 1, -1, -1):
        for key, dU in _step_derivatives(model, S, g, amp[n], prob.dt, V, H0m, K, d, Vh):
            dg = np.vdot(chi, dU @ psi[n])
            grad[(n,) + key] = 2.0 * (np.conj(gval) * dg).real
        chi = steps[n].conj().T @ chi
    return float(abs(gval) ** 2), complex(gval), grad


def _step_derivatives(model, S, g, amp_n, dt, V, H0m, K, d, Vh=None):
    """Yield (index, dU_n/dtheta) for every control parameter of one step
    (split models: the derivative of the control block, with the drift
    around it as in the step)."""
    if model == "exact_first_order":
        U = step_exact(H0m, S, g, amp_n, dt)
        for k in range(K):
            if g is not None:
                yield (k, 0), -1j * dt * S[k] @ U
                yield (k, 1), -1j * dt * y_generator(S[k], g[k]) @ U
            else:
                yield (k,), -1j * dt * S[k] @ U
        return
    if model == "exact":
        H = np.array(H0m, dtype=np.complex128)
        gens = []
        for k in range(K):
            if g is not None:
                Sy = y_generator(S[k], g[k])
                H = H + amp_n[k, 0] * S[k] + amp_n[k, 1] * Sy
                gens += [((k, 0), S[k]), ((k, 1), Sy)]
            else:
                H = H + amp_n[k] * S[k]
                gens += [((k,), S[k])]
        for key, G in gens:
            yield key, frechet_expm(H, dt, -1j * dt * G)
        return
    if g is None:
        # U = R_K ... R_1 V, R_k = exp(-i dt u_k S_k)
        R = [expm_herm(S[k], amp_n[k] * dt) for k in range(K)]
        for k in range(K):
            dR = frechet_expm(S[k], amp_n[k] * dt, -1j * dt * S[k])
            P = np.eye(d, dtype=np.complex128)
            for kk in range(K):
                P = (dR if kk == k else R[kk]) @ P
            yield (k,), with_drift(P, V, Vh)
        return
    # phased: U = Z (prod_k X_k) Z^dag V, X_k = exp(-i Omega_k dt S_k), Z = exp(-i sum phi_k G_k)
    om = np.sqrt(amp_n[:, 0] ** 2 + amp_n[:, 1] ** 2)
    phi = np.arctan2(amp_n[:, 1], amp_n[:, 0])
    Z = phase_diag(phi, g)
    X = [expm_herm(S[k], om[k] * dt) for k in range(K)]
    prodX = np.eye(d, dtype=np.complex128)
    for k in range(K):
        prodX = X[k] @ prodX
    for k in range(K):
        dX = frechet_expm(S[k], om[k] * dt, -1j * dt * S[k])          # d/dOmega_k
        P = np.eye(d, dtype=np.complex128)
        for kk in range(K):
            P = (dX if kk == k else X[kk]) @ P
        dU_dom = with_drift(Z @ P @ Z.conj().T, V, Vh)
        G = np.diag(g[k]).astype(np.complex128)
        dZ = -1j * G @ Z                                               # d/dphi_k of Z
        dU_dphi = with_drift(dZ @ prodX @ Z.conj().T + Z @ prodX @ dZ.conj().T, V, Vh)
        if om[k] > 0.0:
            c, s = amp_n[k, 0] / om[k], amp_n[k, 1] / om[k]
            yield (k, 0), c * dU_dom - (s / om[k]) * dU_dphi
            yield (k, 1), s * dU_dom + (c / om[k]) * dU_dphi
        else:
            # at the origin the Cartesian derivatives are the generators themselves: the
            # block exp(-i dt (u_x S + u_y S^y)) has them as its derivatives whatever the
            # phase of the zero pair, so the channel's own phase (atan2 gives +-pi for a
            # negative zero) is left out of the rotation around them
            phi0 = phi.copy()
            phi0[k] = 0.0
            Z0 = phase_diag(phi0, g)
            Sy = y_generator(S[k], g[k])
            P0 = np.eye(d, dtype=np.complex128)
            for kk in range(K):
                if kk != k:
                    P0 = X[kk] @ P0
            for a, Gen in ((0, S[k]), (1, Sy)):
                yield (k, a), with_drift(Z0 @ (-1j * dt * Gen) @ P0 @ Z0.conj().T, V, Vh)
