"""Preconditioned conjugate gradients on ``S-hat w = f-hat`` (oracle; test infrastructure).

Section 3.4: PCG with preconditioner ``K_X`` on the wavelet-in-time system,
recovering ``u = W w``.  The quantity ``r_k^T K_X r_k`` is available inside
PCG and is equivalent to the squared X-norm of the algebraic error (eq.
(stopping)).  The paper stops at an absolute bound on it; here the test is
relative to the first residual, ``sqrt(r_k^T K_X r_k) <= tol sqrt(r_0^T K_X r_0)``
with ``w_0 = 0``, and ``tol = 0`` means "run exactly ``maxit`` iterations".
"""
from __future__ import annotations

import numpy as np

from .schur import Problem


def dot(a, b):
    return float(np.sum(a * b))


def pcg(P: Problem, fhat, tol=1e-8, maxit=100, callback=None, w0=None):
    """Standard Hestenes-Stiefel PCG from ``w = 0``, or from the initial guess
    ``w0``.  Returns ``(w, iterations, history)`` where ``iterations`` counts
    applications of S-hat and ``history`` holds ``sqrt(r_k^T K_X r_k)`` for
    k = 0..iterations.  The stopping test is relative to the data,
    ``sqrt(r_k^T K_X r_k) <= tol sqrt(f-hat^T K_X f-hat)``, which for
    ``w0 = 0`` is the first residual's quantity."""
    if w0 is None:
        w = np.zeros_like(fhat)
        r = fhat.copy()
    else:
        w = np.array(w0, dtype=np.float64, copy=True)
        r = fhat - P.Shat(w)
    z = P.KX(r)
    rho = dot(r, z)
    hist = [np.sqrt(max(rho, 0.0))]
    if rho == 0.0:
        return w, 0, hist
    rho0 = rho if w0 is None else dot(fhat, P.KX(fhat))
    p = z.copy()
    k = 0
    while k < maxit and not (tol > 0 and np.sqrt(rho) <= tol * np.sqrt(rho0)):
        q = P.Shat(p)
        pq = dot(p, q)
        if not pq > 0:
            raise FloatingPointError("PCG breakdown: p^T q <= 0")
        gamma = rho / pq
        w += gamma * p
        r -= gamma * q
        z = P.KX(r)
        rho_new = dot(r, z)
        beta = rho_new / rho
        p = z + beta * p
        rho = rho_new
        k += 1
        hist.append(np.sqrt(max(rho, 0.0)))
        if callback is not None:
            callback(k, w, r)
    return w, k, hist


def solve(J, K, g=None, u0=None, tol=1e-8, maxit=100, **kw):
    """Solve the heat equation's space-time system for nodal data ``g``
    (``(2**J+1, n, n)`` or None) and ``u0`` (``(n, n)``).  Returns
    ``(u, iterations, history)`` with ``u`` the nodal solution, time-major."""
    P = Problem(J, K, **kw)
    if u0 is None:
        u0 = np.zeros(P.shape[1:])
    f = P.rhs(g, u0)
    fhat = P.WT(f)
    w, its, hist = pcg(P, fhat, tol, maxit)
    return P.W(w), its, hist
