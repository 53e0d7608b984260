"""Temporal matrices of Lemma 4.2 on a uniform time grid (oracle; test infrastructure).

``Phi_t`` is the Lagrange (hat) basis of continuous piecewise linears on
``N = 2**J`` intervals of length ``tau = 1/N`` (Section 4).  The matrices are
exact integrals of hat functions:

  * ``A_t = <d/dt Phi_t, d/dt Phi_t>``  (stiffness),
  * ``M_t = <Phi_t, Phi_t>``            (mass),
  * ``L   = <d/dt Phi_t, Phi_t>``,       entry (i, j) = integral of phi_i * phi_j'
    (rows come from the second argument of the pairing, the convention under
    which T, N map X_t into the dual of Y_t in Lemma 4.1 and T^T O^{-1} N = L^T
    in the proof of Lemma 4.2),
  * ``Gamma_0 = Phi_t(0) Phi_t(0)^T``    (only entry (0, 0) = 1).

All functions act along axis 0 of a time-major array ``X`` of shape
``(N + 1, ...)`` and return a new array.
"""
from __future__ import annotations

import numpy as np


def stiffness(X: np.ndarray, tau: float) -> np.ndarray:
    """``A_t X``: ``(-X[i-1] + 2 X[i] - X[i+1]) / tau``; one-sided at both ends."""
    Y = np.empty_like(X)
    N = X.shape[0] - 1
    if N == 0:
        raise ValueError("need at least one time interval")
    Y[0] = (X[0] - X[1]) / tau
    Y[N] = (X[N] - X[N - 1]) / tau
    if N > 1:
        Y[1:N] = (2.0 * X[1:N] - X[0:N - 1] - X[2:N + 1]) / tau
    return Y


def mass(X: np.ndarray, tau: float) -> np.ndarray:
    """``M_t X``: ``tau (X[i-1] + 4 X[i] + X[i+1]) / 6``; ``tau (2 X[0] + X[1]) / 6`` at 0."""
    Y = np.empty_like(X)
    N = X.shape[0] - 1
    Y[0] = tau * (2.0 * X[0] + X[1]) / 6.0
    Y[N] = tau * (X[N - 1] + 2.0 * X[N]) / 6.0
    if N > 1:
        Y[1:N] = tau * (X[0:N - 1] + 4.0 * X[1:N] + X[2:N + 1]) / 6.0
    return Y


def L(X: np.ndarray) -> np.ndarray:
    """``L X`` with ``L[i, j] = int phi_i phi_j'``: ``(X[i+1] - X[i-1]) / 2`` inside,
    ``(X[1] - X[0]) / 2`` at 0 and ``(X[N] - X[N-1]) / 2`` at N."""
    Y = np.empty_like(X)
    N = X.shape[0] - 1
    Y[0] = (X[1] - X[0]) / 2.0
    Y[N] = (X[N] - X[N - 1]) / 2.0
    if N > 1:
        Y[1:N] = (X[2:N + 1] - X[0:N - 1]) / 2.0
    return Y


def LT(X: np.ndarray) -> np.ndarray:
    """``L^T X``: ``(X[i-1] - X[i+1]) / 2`` inside, ``-(X[0] + X[1]) / 2`` at 0 and
    ``(X[N-1] + X[N]) / 2`` at N."""
    Y = np.empty_like(X)
    N = X.shape[0] - 1
    Y[0] = -(X[0] + X[1]) / 2.0
    Y[N] = (X[N - 1] + X[N]) / 2.0
    if N > 1:
        Y[1:N] = (X[0:N - 1] - X[2:N + 1]) / 2.0
    return Y


def gamma0(X: np.ndarray) -> np.ndarray:
    """``Gamma_0 X``: row 0 kept, all other rows zero."""
    Y = np.zeros_like(X)
    Y[0] = X[0]
    return Y


def dense(N: int):
    """Dense ``(A_t, M_t, L, Gamma_0)`` for ``N`` intervals (for small checks)."""
    I = np.eye(N + 1)
    tau = 1.0 / N
    return stiffness(I, tau), mass(I, tau), L(I), gamma0(I)
