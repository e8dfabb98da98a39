"""Python binding of libredo.so (argument marshalling only).

Every step of the REDO path runs in the HIP library; this module only moves
torch device tensors across the C ABI of include/redo.h, on torch's current
HIP stream.  If the library is missing the import fails: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libredo.so")

PREC_F32, PREC_F32_3M, PREC_BF16X3 = 0, 1, 2
OP_COMPOSE, OP_CHAIN, OP_GRAPE, OP_EXPM_CHAIN, OP_EXPM_GRAPE, OP_STATE_GRAPE, OP_KRON_CHAIN = 0, 1, 2, 3, 4, 5, 6
STATUS = {0: "REDO_OK", 1: "REDO_ERR_ARG", 2: "REDO_ERR_ALLOC", 3: "REDO_ERR_HIP", 4: "REDO_ERR_NOT_HERMITIAN",
          5: "REDO_ERR_NONFINITE", 6: "REDO_ERR_UNSUPPORTED", 7: "REDO_ERR_WORKSPACE", 100: "REDO_WARN_CLAMPED",
          101: "REDO_WARN_UNITARITY"}

# name -> (restype, argtypes); mirrors include/redo.h
_P = ctypes.c_void_p
_I = ctypes.c_int32
_SIG = {
    "redo_build_table": (_I, [_P, _P, _P, _P, _P, ctypes.POINTER(_P)]),
    "redo_table_destroy": (_I, [_P]),
    "redo_table_query": (_I, [_P, _P, ctypes.POINTER(ctypes.c_size_t)]),
    "redo_cache_levels": (_I, [_P, _I, _I, _P]),
    "redo_level_f64": (_I, [_P, _I, _I, _P, _P]),
    "redo_cache_split_bf16": (_I, [_P, _I, _P]),
    "redo_workspace_bytes": (ctypes.c_size_t, [_P, _I, _I, _I]),
    "redo_grape_workspace_bytes": (ctypes.c_size_t, [_P, _I, _I, _I]),
    "redo_grape_workspace_min_bytes": (ctypes.c_size_t, [_P, _I, _I, _I]),
    "redo_quantise": (_I, [_P, _P, _I, _I, _P, _P, _P]),
    "redo_compose_steps": (_I, [_P, _I, _P, _I, _I, _P, _P, ctypes.c_size_t, _P]),
    "redo_chain_propagator": (_I, [_P, _I, _P, _P, _I, _I, _I, _I, _P, _P, _P, _P, _P, _I, _P, _P,
                                   ctypes.c_size_t, _P]),
    "redo_unitary_fidelity": (_I, [_I, _I, _P, _P, _P, _P, _P]),
    "redo_table_spins": (_I, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "redo_kron_chain": (_I, [_P, _I, _P, _P, _I, _I, _I, _I, _P, _P, _P, _P, _I, _P, _P, ctypes.c_size_t, _P]),
    "redo_grape_fidelity_grad": (_I, [_P, _I, _P, _P, _I, _I, _P, _I, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "redo_expm_chain": (_I, [_P, _I, _P, _P, _I, _I, _I, _I, _P, _P, _P, _P, _I, _P, _P, ctypes.c_size_t, _P]),
    "redo_expm_grape_fidelity_grad": (_I, [_P, _I, _P, _P, _I, _I, _P, _I, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "redo_expm_split_chain": (_I, [_P, _I, _P, _P, _I, _I, _I, _I, _P, _P, _I, _P, _P, _P, ctypes.c_size_t, _P]),
    "redo_grape_state_fidelity_grad": (_I, [_P, _I, _P, _P, _I, _I, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "redo_grape_noalloc_max_bytes": (ctypes.c_size_t, []),
    "redo_grape_fidelity_grad_noalloc": (_I, [_P, _I, _P, _P, _I, _I, _P, _I, _P, _P, _P, _P]),
    "redo_get_device_status": (_I, [_P, _P, ctypes.POINTER(ctypes.c_int64)]),
    "redo_unitarity_report": (_I, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
    "redo_profile_enable": (_I, [_I]),
    "redo_profile_read": (_I, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64), _I]),
    "redo_profile_read_kind": (_I, [_I, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64), _I]),
    "redo_mlp_target_features": (_I, [_I, _I, _P, _P, _P]),
    "redo_mlp_forward": (_I, [_P, _I, _P, _P, _P]),
    "redo_mlp_loss_grad": (_I, [_P, _I, _P, _P, _P, _P, _P, _P, _P]),
    "redo_adam_update": (_I, [ctypes.c_int64, _P, _P, _P, _P, _P, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                              ctypes.c_float, _I, ctypes.c_float, ctypes.c_float, ctypes.c_float, _P]),
    "redo_to_bf16": (_I, [ctypes.c_int64, _P, _P, _P]),
    "redo_ascent_step": (_I, [ctypes.c_int64, _P, _P, ctypes.c_float, ctypes.c_float, ctypes.c_float, _P]),
    "redo_time_average": (_I, [_I, _I, _P, _P, _P]),
    "redo_lbfgs_direction": (_I, [_I, ctypes.c_int64, _I, _P, _P, _P, _P, _P, _P, ctypes.c_double, _P, _P, _P]),
    "redo_lbfgs_trial": (_I, [_I, ctypes.c_int64, _P, _P, _P, _P, _P]),
    "redo_lbfgs_push": (_I, [_I, ctypes.c_int64, _I, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "redo_observable_walsh": (_I, [_I, _P, _P, _I, _P]),
    "redo_walsh_right": (_I, [_I, _I, _P, ctypes.c_int64, _P]),
    "redo_walsh_observable_create": (_I, [_I, _P, _P, _I, ctypes.POINTER(_P)]),
    "redo_walsh_observable_spectrum": (_I, [_P, _P]),
    "redo_walsh_observable_destroy": (_I, [_P]),
    "redo_chain_propagator_walsh": (_I, [_P, _I, _P, _P, _I, _I, _I, _I, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "redo_kron_chain_walsh": (_I, [_P, _I, _P, _P, _I, _I, _I, _I, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "redo_expm_chain_walsh": (_I, [_P, _I, _P, _P, _I, _I, _I, _I, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "redo_status_string": (ctypes.c_char_p, [_I]),
    "redo_last_error": (ctypes.c_char_p, []),
}


def exported_symbols():
    return list(_SIG)


class _Mlp(ctypes.Structure):
    _fields_ = [("sizes", _I * 4), ("W", _P * 3), ("b", _P * 3)]


class _MlpGrads(ctypes.Structure):
    _fields_ = [("W", _P * 3), ("b", _P * 3)]


class _Desc(ctypes.Structure):
    _fields_ = [("d", _I), ("K", _I), ("base", _I), ("digits", _I), ("dt", ctypes.c_double),
                ("eps", ctypes.c_double), ("phased", _I), ("drift_is_diag", _I), ("n_drift", _I),
                ("splitting", _I)]


def load_library(path: str = _LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1707_02162_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIG.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        _lib = load_library()
    return _lib


class RedoError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _check(status: int, allow_warn: bool = False) -> int:
    if status == 0 or (allow_warn and status == 100):
        return status
    raise RedoError(status, lib().redo_last_error().decode())


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(x, dtype, device) -> torch.Tensor:
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x)).to(device=device, dtype=dtype).contiguous()


class RedoTable:
    """A built table of discrete operators (process 1) plus drift propagators."""

    def __init__(self, d: int, K: int, base: int, digits: int, dt: float, eps: float, phased: bool,
                 H0, S, g=None, drift_is_diag: bool = True, device: str = "cuda", splitting: str = "lie"):
        self.device = torch.device(device)
        self.d, self.K, self.base, self.digits = d, K, base, digits
        self.dt, self.eps, self.phased = float(dt), float(eps), bool(phased)
        H0t = _dev(H0, torch.float64 if drift_is_diag else torch.complex128, self.device)
        if H0t.dim() == (1 if drift_is_diag else 2):
            H0t = H0t.unsqueeze(0)
        St = _dev(S, torch.complex128, self.device)
        gt = _dev(g, torch.float64, self.device) if phased else None
        self.n_drift = H0t.shape[0]
        if splitting not in ("lie", "strang"):
            raise ValueError("splitting is 'lie' or 'strang'")
        self.splitting = splitting
        desc = _Desc(d, K, base, digits, self.dt, self.eps, int(phased), int(drift_is_diag), self.n_drift,
                     1 if splitting == "strang" else 0)
        h = ctypes.c_void_p()
        _check(lib().redo_build_table(ctypes.byref(desc), _ptr(H0t), _ptr(St), _ptr(gt), _stream(),
                                      ctypes.byref(h)))
        self._h = h
        self.kk = 2 if phased else 1

    @classmethod
    def from_problem(cls, p, device: str = "cuda") -> "RedoTable":
        return cls(p.d, p.K, p.base, p.digits, p.dt, p.eps, p.phased, p.H0, p.S,
                   p.g if p.phased else None, p.drift_is_diag, device, getattr(p, "splitting", "lie"))

    def close(self):
        if getattr(self, "_h", None):
            lib().redo_table_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def cache_levels(self, q_lo: int = 0, q_hi: Optional[int] = None) -> None:
        """Compose and keep R_k(q) for q_lo <= q <= q_hi (default: every level)."""
        if q_hi is None:
            q_hi = self.base ** self.digits - 1
        _check(lib().redo_cache_levels(self._h, q_lo, q_hi, _stream()))

    def level_f64(self, k: int, q: int) -> torch.Tensor:
        """R_k(q) composed in FP64 on the device as the table build composes it before
        rounding (complex128 [d, d]); a check of process 1, not the hot path."""
        out = torch.empty((self.d, self.d), dtype=torch.complex128, device=self.device)
        _check(lib().redo_level_f64(self._h, k, q, _ptr(out), _stream()))
        return out

    def clear_cache(self) -> None:
        _check(lib().redo_cache_levels(self._h, 0, -1, _stream()))

    def cache_split_bf16(self, keep: bool = True) -> None:
        """Keep the cached levels a second time as pre-split BF16 panels, which the
        split-BF16 products (precision=2, d >= 128) then read without splitting;
        keep=False frees them."""
        _check(lib().redo_cache_split_bf16(self._h, 1 if keep else 0, _stream()))

    @property
    def device_bytes(self) -> int:
        n = ctypes.c_size_t()
        _check(lib().redo_table_query(self._h, None, ctypes.byref(n)))
        return n.value

    def workspace(self, op: int, B: int, N: int) -> torch.Tensor:
        nbytes = lib().redo_workspace_bytes(self._h, op, B, N)
        return torch.empty(max(int(nbytes), 16), dtype=torch.uint8, device=self.device)

    def _u(self, u) -> torch.Tensor:
        t = _dev(u, torch.float32, self.device)
        want = 4 if self.phased else 3
        if t.dim() != want or t.shape[2] != self.K or (self.phased and t.shape[3] != 2):
            raise ValueError(f"u must be [B, N, {self.K}" + (", 2]" if self.phased else "]"))
        return t

    def quantise(self, u):
        ut = self._u(u)
        B, N = ut.shape[:2]
        codes = torch.empty((B, N, self.K), dtype=torch.int32, device=self.device)
        phi = torch.empty((B, N, self.K), dtype=torch.float64, device=self.device) if self.phased else None
        _check(lib().redo_quantise(self._h, _ptr(ut), B, N, _ptr(codes), _ptr(phi), _stream()))
        return codes, phi

    def compose(self, u, precision: int = PREC_F32) -> torch.Tensor:
        ut = self._u(u)
        B, N = ut.shape[:2]
        out = torch.empty((B, N, self.d, self.d), dtype=torch.complex64, device=self.device)
        ws = self.workspace(OP_COMPOSE, B, N)
        _check(lib().redo_compose_steps(self._h, precision, _ptr(ut), B, N, _ptr(out), _ptr(ws), ws.numel(),
                                        _stream()))
        return out

    def chain(self, u, n_steps=None, precision: int = PREC_F32, X0=None, reproject_every: int = 0,
              step_offset: int = 0, prefix: bool = False, observable=None, out: Optional[torch.Tensor] = None,
              walsh=None):
        """Chain of REDO steps.  observable: (cols int32 [d, w], vals complex [d, w]) row lists.
        walsh: a WalshObservable (the observable of the call, with its spectrum; `observable`
        is then not given), or True for the frame without an observable: the states (X0 and
        the result) are then W = X H / sqrt(d), the right Walsh frame.
        Returns (U_total, X_prefix or None, obs or None)."""
        ut = self._u(u)
        B, N = ut.shape[:2]
        ns = None if n_steps is None else _dev(n_steps, torch.int32, self.device)
        X0t = None if X0 is None else _dev(X0, torch.complex64, self.device)
        U = out if out is not None else torch.empty((B, self.d, self.d), dtype=torch.complex64, device=self.device)
        Xp = torch.empty((B, N, self.d, self.d), dtype=torch.complex64, device=self.device) if prefix else None
        cols = vals = obs = None
        w = 0
        if observable is not None:
            cols = _dev(observable[0], torch.int32, self.device)
            vals = _dev(observable[1], torch.complex64, self.device)
            w = cols.shape[1]
            obs = torch.empty((B, N), dtype=torch.float64, device=self.device)
        ws = self.workspace(OP_CHAIN, B, N)
        if walsh is not None:
            if prefix:
                raise ValueError("prefix states are not provided in the Walsh frame")
            h, obs = self._walsh_args(walsh, observable, B, N)
            _check(lib().redo_chain_propagator_walsh(self._h, precision, _ptr(ut), _ptr(ns), B, N, step_offset,
                                                     reproject_every, _ptr(X0t), _ptr(U), h, _ptr(obs), _ptr(ws),
                                                     ws.numel(), _stream()))
            return U, None, obs
        _check(lib().redo_chain_propagator(self._h, precision, _ptr(ut), _ptr(ns), B, N, step_offset,
                                           reproject_every, _ptr(X0t), _ptr(U), _ptr(Xp), _ptr(cols), _ptr(vals),
                                           w, _ptr(obs), _ptr(ws), ws.numel(), _stream()))
        return U, Xp, obs

    def _walsh_args(self, walsh, observable, B, N):
        """(handle or None, obs_out or None) of a Walsh-frame call."""
        if walsh is True:
            if observable is not None:
                raise ValueError("an observable in the Walsh frame comes as a WalshObservable (walsh=...)")
            return None, None
        if not isinstance(walsh, WalshObservable):
            raise TypeError("walsh must be a WalshObservable or True")
        if observable is not None:
            raise ValueError("pass the observable once, as the WalshObservable")
        if walsh.d != self.d:
            raise ValueError("the WalshObservable is of another dimension than the table")
        return walsh._h, torch.empty((B, N), dtype=torch.float64, device=self.device)

    @property
    def spins(self) -> int:
        """n when d = 2^n and every generator is a sum of single-spin terms, else 0."""
        n = ctypes.c_int32(0)
        _check(lib().redo_table_spins(self._h, ctypes.byref(n)))
        return int(n.value)

    def kron_chain(self, u, n_steps=None, quantised: bool = True, X0=None, reproject_every: int = 0,
                   step_offset: int = 0, observable=None, out: Optional[torch.Tensor] = None, walsh=None):
        """Structure-aware chain (spin-factorised control blocks; needs self.spins > 0).
        quantised: REDO codes (True) or the amplitudes as given.  walsh as for chain.
        Returns (U_total, obs or None)."""
        ut = self._u(u)
        B, N = ut.shape[:2]
        ns = None if n_steps is None else _dev(n_steps, torch.int32, self.device)
        X0t = None if X0 is None else _dev(X0, torch.complex64, self.device)
        U = out if out is not None else torch.empty((B, self.d, self.d), dtype=torch.complex64, device=self.device)
        cols = vals = obs = None
        w = 0
        if observable is not None:
            cols = _dev(observable[0], torch.int32, self.device)
            vals = _dev(observable[1], torch.complex64, self.device)
            w = cols.shape[1]
            obs = torch.empty((B, N), dtype=torch.float64, device=self.device)
        ws = self.workspace(OP_KRON_CHAIN, B, N)
        if walsh is not None:
            h, obs = self._walsh_args(walsh, observable, B, N)
            _check(lib().redo_kron_chain_walsh(self._h, 1 if quantised else 0, _ptr(ut), _ptr(ns), B, N,
                                               step_offset, reproject_every, _ptr(X0t), _ptr(U), h, _ptr(obs),
                                               _ptr(ws), ws.numel(), _stream()))
            return U, obs
        _check(lib().redo_kron_chain(self._h, 1 if quantised else 0, _ptr(ut), _ptr(ns), B, N, step_offset,
                                     reproject_every, _ptr(X0t), _ptr(U), _ptr(cols), _ptr(vals), w, _ptr(obs),
                                     _ptr(ws), ws.numel(), _stream()))
        return U, obs

    def grape(self, u, U_target, n_steps=None, checkpoint_every: int = 0, precision: int = PREC_F32,
              precompose: bool = True):
        """Returns (fidelity float64 [B], overlap complex128 [B], grad float32 like u).
        precompose=False passes the smallest workspace (d <= 64: every scan step built
        from its factors instead of from the precomposed step propagators)."""
        ut = self._u(u)
        B, N = ut.shape[:2]
        ns = None if n_steps is None else _dev(n_steps, torch.int32, self.device)
        Uf = _dev(U_target, torch.complex64, self.device)
        F = torch.empty(B, dtype=torch.float64, device=self.device)
        ov = torch.empty(B, dtype=torch.complex128, device=self.device)
        grad = torch.empty_like(ut)
        size = lib().redo_grape_workspace_bytes if precompose else lib().redo_grape_workspace_min_bytes
        nbytes = size(self._h, B, N, checkpoint_every)
        ws = torch.empty(max(int(nbytes), 16), dtype=torch.uint8, device=self.device)
        _check(lib().redo_grape_fidelity_grad(self._h, precision, _ptr(ut), _ptr(ns), B, N, _ptr(Uf),
                                              checkpoint_every, _ptr(F), _ptr(ov), _ptr(grad), _ptr(ws),
                                              ws.numel(), _stream()))
        return F, ov, grad

    def expm_chain(self, u, n_steps=None, precision: int = PREC_F32, X0=None, reproject_every: int = 0,
                   step_offset: int = 0, observable=None, out: Optional[torch.Tensor] = None, walsh=None):
        """The plain per-step exponential chain (comparison point); walsh as for chain.
        Returns (U_total, obs or None)."""
        ut = self._u(u)
        B, N = ut.shape[:2]
        ns = None if n_steps is None else _dev(n_steps, torch.int32, self.device)
        X0t = None if X0 is None else _dev(X0, torch.complex64, self.device)
        U = out if out is not None else torch.empty((B, self.d, self.d), dtype=torch.complex64, device=self.device)
        cols = vals = obs = None
        w = 0
        if observable is not None:
            cols = _dev(observable[0], torch.int32, self.device)
            vals = _dev(observable[1], torch.complex64, self.device)
            w = cols.shape[1]
            obs = torch.empty((B, N), dtype=torch.float64, device=self.device)
        ws = self.workspace(OP_EXPM_CHAIN, B, N)
        if walsh is not None:
            h, obs = self._walsh_args(walsh, observable, B, N)
            _check(lib().redo_expm_chain_walsh(self._h, precision, _ptr(ut), _ptr(ns), B, N, step_offset,
                                               reproject_every, _ptr(X0t), _ptr(U), h, _ptr(obs), _ptr(ws),
                                               ws.numel(), _stream()))
            return U, obs
        _check(lib().redo_expm_chain(self._h, precision, _ptr(ut), _ptr(ns), B, N, step_offset, reproject_every,
                                     _ptr(X0t), _ptr(U), _ptr(cols), _ptr(vals), w, _ptr(obs), _ptr(ws), ws.numel(),
                                     _stream()))
        return U, obs

    def expm_split_chain(self, u, n_steps=None, precision: int = PREC_F32, X0=None, reproject_every: int = 0,
                         step_offset: int = 0, out: Optional[torch.Tensor] = None, walsh=None):
        """The equal-result comparison point: the REDO chain's split model with each control
        factor an exponential at the coarse-grained amplitude (one signed channel, diagonal
        drift).  walsh: None (computational basis, no observable), True (the right Walsh
        frame) or a WalshObservable (the frame and its observable).  Returns (U_total, obs or None)."""
        ut = self._u(u)
        B, N = ut.shape[:2]
        ns = None if n_steps is None else _dev(n_steps, torch.int32, self.device)
        X0t = None if X0 is None else _dev(X0, torch.complex64, self.device)
        U = out if out is not None else torch.empty((B, self.d, self.d), dtype=torch.complex64, device=self.device)
        h, obs = (None, None) if walsh is None else self._walsh_args(walsh, None, B, N)
        ws = self.workspace(OP_EXPM_CHAIN, B, N)
        _check(lib().redo_expm_split_chain(self._h, precision, _ptr(ut), _ptr(ns), B, N, step_offset, reproject_every,
                                           _ptr(X0t), _ptr(U), 0 if walsh is None else 1, h, _ptr(obs), _ptr(ws),
                                           ws.numel(), _stream()))
        return U, obs

    def state_grape(self, u, psi0, psi_f, n_steps=None):
        """State-transfer GRAPE: F_S = |<psi_f|U|psi_0>|^2 and dF_S/du.
        psi0, psi_f complex [B, d].  Returns (F double [B], overlap complex128 [B], grad like u)."""
        ut = self._u(u)
        B, N = ut.shape[:2]
        ns = None if n_steps is None else _dev(n_steps, torch.int32, self.device)
        p0 = _dev(psi0, torch.complex64, self.device)
        pf = _dev(psi_f, torch.complex64, self.device)
        F = torch.empty(B, dtype=torch.float64, device=self.device)
        ov = torch.empty(B, dtype=torch.complex128, device=self.device)
        grad = torch.empty_like(ut)
        ws = self.workspace(OP_STATE_GRAPE, B, N)
        _check(lib().redo_grape_state_fidelity_grad(self._h, PREC_F32, _ptr(ut), _ptr(ns), B, N, _ptr(p0), _ptr(pf),
                                                    _ptr(F), _ptr(ov), _ptr(grad), _ptr(ws), ws.numel(), _stream()))
        return F, ov, grad

    def expm_grape(self, u, U_target, n_steps=None, precision: int = PREC_F32):
        """GRAPE objective and first-order gradient with the plain per-step exponential."""
        ut = self._u(u)
        B, N = ut.shape[:2]
        ns = None if n_steps is None else _dev(n_steps, torch.int32, self.device)
        Uf = _dev(U_target, torch.complex64, self.device)
        F = torch.empty(B, dtype=torch.float64, device=self.device)
        ov = torch.empty(B, dtype=torch.complex128, device=self.device)
        grad = torch.empty_like(ut)
        ws = self.workspace(OP_EXPM_GRAPE, B, N)
        _check(lib().redo_expm_grape_fidelity_grad(self._h, precision, _ptr(ut), _ptr(ns), B, N, _ptr(Uf), 0,
                                                   _ptr(F), _ptr(ov), _ptr(grad), _ptr(ws), ws.numel(), _stream()))
        return F, ov, grad

    def device_status(self):
        """(status, clamped amplitudes) latched since the last call; clears them."""
        n = ctypes.c_int64()
        st = lib().redo_get_device_status(self._h, _stream(), ctypes.byref(n))
        return st, n.value

    def unitarity_report(self):
        """(largest ||X^dag X - I||_F / sqrt(d) at a re-projection step, count above 1e-3)
        as read by the last device_status call."""
        x = ctypes.c_double()
        n = ctypes.c_int64()
        _check(lib().redo_unitarity_report(self._h, ctypes.byref(x), ctypes.byref(n)))
        return x.value, n.value


def profile_enable(on: bool = True) -> None:
    _check(lib().redo_profile_enable(1 if on else 0))


def profile_read(reset: bool = True, kind: int = 0):
    """(summed launch milliseconds, launch count) since the last reset, for the
    batched GEMM (kind 0) or the structure-aware step kernel (kind 1)."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib().redo_profile_read_kind(kind, ctypes.byref(ms), ctypes.byref(n), 1 if reset else 0))
    return ms.value, n.value


def unitary_fidelity(U_target: torch.Tensor, U: torch.Tensor):
    """(overlap complex128 [B], fidelity float64 [B]) of batched d x d unitaries."""
    B, d = U.shape[0], U.shape[-1]
    Uf = _dev(U_target, torch.complex64, U.device)
    Ut = _dev(U, torch.complex64, U.device)
    ov = torch.empty(B, dtype=torch.complex128, device=U.device)
    F = torch.empty(B, dtype=torch.float64, device=U.device)
    _check(lib().redo_unitary_fidelity(d, B, _ptr(Uf), _ptr(Ut), _ptr(ov), _ptr(F), _stream()))
    return ov, F


def ascent_step(u: torch.Tensor, grad: torch.Tensor, alpha: float, lo: float, hi: float) -> torch.Tensor:
    """In place u <- clamp(u + alpha grad, lo, hi) (float32 device tensors of one shape)."""
    if u.dtype != torch.float32 or grad.dtype != torch.float32 or u.shape != grad.shape:
        raise ValueError("u and grad must be float32 tensors of one shape")
    _check(lib().redo_ascent_step(u.numel(), _ptr(u), _ptr(grad), alpha, lo, hi, _stream()))
    return u


def time_average(series: torch.Tensor) -> torch.Tensor:
    """Row means of a float64 [rows, cols] device tensor (the order parameter of a
    magnetisation series)."""
    if series.dtype != torch.float64 or series.dim() != 2:
        raise ValueError("series must be float64 [rows, cols]")
    out = torch.empty(series.shape[0], dtype=torch.float64, device=series.device)
    _check(lib().redo_time_average(series.shape[0], series.shape[1], _ptr(series), _ptr(out), _stream()))
    return out


def walsh_spectrum(cols, vals) -> Optional[np.ndarray]:
    """Walsh spectrum of an observable given as row lists (host arrays, cols int32 [d, w],
    vals complex [d, w]): D = H f (float64 [d]) when M_ij = f(i XOR j) with f real, that is
    M = Hn diag(D) Hn with Hn = H / sqrt(d) the normalised Sylvester-Hadamard matrix; None
    otherwise.  Host-side analysis in the library, no GPU work."""
    c = np.ascontiguousarray(np.asarray(cols, dtype=np.int32))
    v = np.ascontiguousarray(np.asarray(vals, dtype=np.complex64))
    if c.ndim != 2 or v.shape != c.shape:
        raise ValueError("cols and vals must both be [d, w]")
    d, w = c.shape
    D = np.empty(d, dtype=np.float64)
    st = lib().redo_observable_walsh(d, c.ctypes.data_as(_P), v.ctypes.data_as(_P), w, D.ctypes.data_as(_P))
    if st == 6:
        return None
    _check(st)
    return D


class WalshObservable:
    """An observable M_ij = f(i XOR j) (row lists on the host) bound to its Walsh spectrum
    D = H f: the library checks the form and keeps device copies of both, so the
    Walsh-frame chains cannot receive a spectrum of another observable."""

    def __init__(self, cols, vals):
        c = np.ascontiguousarray(np.asarray(cols, dtype=np.int32))
        v = np.ascontiguousarray(np.asarray(vals, dtype=np.complex64))
        if c.ndim != 2 or v.shape != c.shape:
            raise ValueError("cols and vals must both be [d, w]")
        self.d, self.w = c.shape
        h = ctypes.c_void_p()
        _check(lib().redo_walsh_observable_create(self.d, c.ctypes.data_as(_P), v.ctypes.data_as(_P), self.w,
                                                  ctypes.byref(h)))
        self._h = h

    @property
    def spectrum(self) -> np.ndarray:
        D = np.empty(self.d, dtype=np.float64)
        _check(lib().redo_walsh_observable_spectrum(self._h, D.ctypes.data_as(_P)))
        return D

    def close(self):
        if getattr(self, "_h", None):
            lib().redo_walsh_observable_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def walsh_observable(cols, vals) -> Optional[WalshObservable]:
    """WalshObservable of the row lists, or None when M is not a real function of i XOR j."""
    try:
        return WalshObservable(cols, vals)
    except RedoError as e:
        if e.status == 6:
            return None
        raise


def walsh_right(X: torch.Tensor) -> torch.Tensor:
    """In place X <- X Hn for complex64 [B, d, d] on the GPU (its own inverse)."""
    if X.dtype != torch.complex64 or X.dim() != 3 or X.shape[1] != X.shape[2]:
        raise ValueError("X must be complex64 [B, d, d]")
    _check(lib().redo_walsh_right(X.shape[1], X.shape[0], _ptr(X), X.shape[1] * X.shape[2], _stream()))
    return X


class GrapeFidelity(torch.autograd.Function):
    """F = |Tr(U_f^dag U(u)) / Tr(U_f^dag U_f)|^2 of the REDO chain, with the
    gradient from the library's adjoint kernel (straight-through at the
    quantised amplitudes)."""

    @staticmethod
    def forward(ctx, u, table: RedoTable, U_target, n_steps=None, checkpoint_every: int = 0,
                precision: int = PREC_F32):
        F, _, grad = table.grape(u.detach(), U_target, n_steps, checkpoint_every, precision)
        ctx.save_for_backward(grad)
        return F

    @staticmethod
    def backward(ctx, gF):
        (grad,) = ctx.saved_tensors
        shape = (-1,) + (1,) * (grad.dim() - 1)
        return (gF.to(grad.dtype).reshape(shape) * grad, None, None, None, None, None)
