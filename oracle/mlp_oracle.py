"""FP64 oracle of the warm-start network (TEST INFRASTRUCTURE ONLY).

The learned warm start is not part of the paper: a three-layer perceptron maps
the 2 d^2 real entries of a target unitary to the initial control amplitudes
of a REDO-GRAPE run.  Architecture (both sides):

    h1 = tanh(W1 x + b1),  h2 = tanh(W2 h1 + b2),  y = tanh(W3 h2 + b3)

loss = mean over the batch and outputs of (y - t)^2.  Plain numpy float64;
the backward pass is the chain rule written out layer by layer.  Pinned by
central finite differences in tests/test_oracle_pins.py.
"""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

__all__ = ["mlp_forward", "mlp_loss_and_grads", "canonical_target_features"]


def mlp_forward(params: List[Tuple[np.ndarray, np.ndarray]], x: np.ndarray):
    """Returns the activations [x, h1, h2, y] (rows = samples); W_l is [out, in]."""
    acts = [np.asarray(x, dtype=np.float64)]
    for W, b in params:
        z = acts[-1] @ np.asarray(W, np.float64).T + np.asarray(b, np.float64)
        acts.append(np.tanh(z))
    return acts


def mlp_loss_and_grads(params, x, target) -> Tuple[float, List[Tuple[np.ndarray, np.ndarray]], np.ndarray]:
    """Mean squared error and its gradients (dW_l, db_l) and d loss / d y."""
    acts = mlp_forward(params, x)
    y = acts[-1]
    n = y.size
    loss = float(((y - target) ** 2).sum() / n)
    dy = 2.0 * (y - target) / n
    grads = [None] * len(params)
    delta = dy * (1.0 - y * y)                      # through the last tanh
    for l in range(len(params) - 1, -1, -1):
        W, _ = params[l]
        a_in = acts[l]
        grads[l] = (delta.T @ a_in, delta.sum(axis=0))
        if l > 0:
            delta = (delta @ np.asarray(W, np.float64)) * (1.0 - a_in * a_in)
    return loss, grads, dy


def canonical_target_features(U: np.ndarray) -> np.ndarray:
    """2 d^2 reals of a target with its global phase removed: U is rotated so
    that its trace is real and non-negative (any unit-modulus factor of U is
    the same gate)."""
    U = np.asarray(U, dtype=np.complex128)
    tr = np.trace(U, axis1=-2, axis2=-1)
    ph = np.where(np.abs(tr) > 1e-12, tr / np.maximum(np.abs(tr), 1e-300), 1.0)
    V = U * np.conj(ph)[..., None, None]
    d = U.shape[-1]
    return np.concatenate([V.real.reshape(*U.shape[:-2], d * d), V.imag.reshape(*U.shape[:-2], d * d)], axis=-1)
