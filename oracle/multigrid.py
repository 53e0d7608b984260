"""Symmetric multigrid for ``a A_x + sigma M_x`` (oracle; test infrastructure).

The paper realises ``K_x ~ A_x^{-1}`` (Section 3.1) and
``K_j ~ (alpha A_x + 2^j M_x)^{-1}`` (Theorem 3.1 with the alpha-scaling of
Section 5.1) by multigrid, using 2 V-cycles with 3 Gauss-Seidel smoothing
steps per grid (Section 5.1, Section 5.2).  Because ``K_x`` enters S and f
(Lemma 4.1), the multigrid operator is part of the definition of the discrete
solution, so every detail is fixed here:

  * grids: level ``l`` has mesh width ``2**-l`` and ``(2**l - 1)**2`` interior
    nodes, ``l = K, K-1, ..., 1``; the coarse matrices are ``a A + sigma M_l``
    with ``M_l`` built on that level's mesh (for nested P1 spaces this is
    exactly the Galerkin product ``P^T C P``);
  * smoother: Gauss-Seidel in three colours, node (i, j) has colour
    ``(i + j) mod 3`` (1-based node indices; no two nodes of one colour are
    coupled by the 7-point stencil); a forward step relaxes colours 0, 1, 2
    in turn, a backward step 2, 1, 0; all nodes of one colour are updated
    together from the current values of the others;
  * V-cycle: 3 forward steps, residual, restriction ``P^T``, recursive
    V-cycle from zero, prolongation ``P`` (P1 interpolation), 3 backward
    steps; the one-node grid (level 1) is solved exactly.  Forward pre- and
    backward post-smoothing make the cycle symmetric;
  * the operator applied is two V-cycles from a zero initial guess.
"""
from __future__ import annotations

import numpy as np

from . import spatial


def coefficients(a, sigma, h, D=None, c=0.0):
    """Stencil of ``C = a (A_D + c M) + sigma M`` on mesh width ``h`` (A_D the
    stiffness of the diffusion tensor D, c the reaction coefficient of
    Section 4): (centre, x-neighbours, y-neighbours, "/"-diagonal neighbours)."""
    m = h * h / 12.0
    if D is None and c == 0.0:
        return 4.0 * a + 6.0 * m * sigma, -a + m * sigma, -a + m * sigma, m * sigma
    dxx, dyy, dxy = (1.0, 1.0, 0.0) if D is None else D
    s = sigma + a * c
    return (2.0 * a * (dxx + dyy - dxy) + 6.0 * m * s, a * (dxy - dxx) + m * s,
            a * (dxy - dyy) + m * s, -a * dxy + m * s)


def apply_C(x, a, sigma, h, D=None, c=0.0):
    """``(a (A_D + c M_x) + sigma M_x) x`` on a level with mesh width ``h``."""
    if D is None and c == 0.0:
        return a * spatial.stiffness(x) + sigma * spatial.mass(x, h)
    return a * spatial.stiffness(x, D) + (sigma + a * c) * spatial.mass(x, h)


def colour_masks(n: int):
    """Boolean masks of the three colours on an ``n x n`` grid."""
    i = np.arange(1, n + 1)[None, :]
    j = np.arange(1, n + 1)[:, None]
    c = (i + j) % 3
    return [c == 0, c == 1, c == 2]


def relax_colour(x, b, a, sigma, h, mask, D=None, c=0.0):
    """One colour of Gauss-Seidel: every node in ``mask`` is set to
    ``(b - sum_nb C_nb x_nb) / C_centre`` using the current neighbour values."""
    c0, cx, cy, c2 = coefficients(a, sigma, h, D, c)
    e, w, nth, s, ne, sw = spatial.neighbours(x)
    if D is None and c == 0.0:
        off = cx * (e + w + nth + s) + c2 * (ne + sw)
    else:
        off = cx * (e + w) + cy * (nth + s) + c2 * (ne + sw)
    new = (b - off) / c0
    return np.where(mask, new, x)


def restrict(r):
    """``P^T r``: fine grid ``(2m+1) x (2m+1)`` -> coarse ``m x m``.  Coarse node
    (I, J) sits at fine node (2I, 2J) and collects that node's value plus half
    of each of its six fine neighbours."""
    rp = spatial._padded(r)  # fine node (i, j), 1-based, at rp[..., j, i]
    nf = r.shape[-1]
    m = (nf - 1) // 2
    J2 = 2 * np.arange(1, m + 1)
    c = rp[..., J2[:, None], J2[None, :]]
    half = (rp[..., J2[:, None], J2[None, :] + 1] + rp[..., J2[:, None], J2[None, :] - 1]
            + rp[..., J2[:, None] + 1, J2[None, :]] + rp[..., J2[:, None] - 1, J2[None, :]]
            + rp[..., J2[:, None] + 1, J2[None, :] + 1] + rp[..., J2[:, None] - 1, J2[None, :] - 1])
    return c + 0.5 * half


def prolong(e):
    """``P e``: coarse ``m x m`` -> fine ``(2m+1) x (2m+1)`` by P1 interpolation
    on the "/"-diagonal mesh (boundary values zero)."""
    m = e.shape[-1]
    nf = 2 * m + 1
    ep = spatial._padded(e)  # coarse node (I, J), 0..m+1, at ep[..., J, I]
    out = np.zeros(e.shape[:-2] + (nf + 2, nf + 2), dtype=e.dtype)
    # fine node (2I, 2J) <- e(I, J)
    out[..., 0::2, 0::2] = ep
    # fine node (2I+1, 2J) <- mean of coarse (I, J), (I+1, J)
    out[..., 0::2, 1::2] = 0.5 * (ep[..., :, :-1] + ep[..., :, 1:])
    # fine node (2I, 2J+1) <- mean of coarse (I, J), (I, J+1)
    out[..., 1::2, 0::2] = 0.5 * (ep[..., :-1, :] + ep[..., 1:, :])
    # fine node (2I+1, 2J+1) <- mean of coarse (I, J), (I+1, J+1) (the "/" edge)
    out[..., 1::2, 1::2] = 0.5 * (ep[..., :-1, :-1] + ep[..., 1:, 1:])
    return out[..., 1:-1, 1:-1]


def vcycle(level, b, x, a, sigma, sweeps=3, D=None, c=0.0):
    """One V-cycle for ``C_level x = b`` from the initial guess ``x``."""
    h = 2.0 ** -level
    if level == 1:
        c0 = coefficients(a, sigma, h, D, c)[0]
        return b / c0
    masks = colour_masks(b.shape[-1])
    for _ in range(sweeps):
        for col in (0, 1, 2):
            x = relax_colour(x, b, a, sigma, h, masks[col], D, c)
    r = b - apply_C(x, a, sigma, h, D, c)
    bc = restrict(r)
    ec = vcycle(level - 1, bc, np.zeros_like(bc), a, sigma, sweeps, D, c)
    x = x + prolong(ec)
    for _ in range(sweeps):
        for col in (2, 1, 0):
            x = relax_colour(x, b, a, sigma, h, masks[col], D, c)
    return x


def apply(b, K, a=1.0, sigma=0.0, cycles=2, sweeps=3, D=None, c=0.0):
    """Multigrid approximation of ``(a (A_D + c M_x) + sigma M_x)^{-1} b`` on
    level ``K``: ``cycles`` V-cycles from zero.  ``b`` has shape ``(..., n,
    n)``; ``a`` and ``sigma`` are scalars or arrays broadcasting against
    ``b[..., 0, 0]``; D (None: identity) and c are the diffusion tensor and
    reaction coefficient of Section 4."""
    a = np.asarray(a, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    if a.ndim:
        a = a[..., None, None]
    if sigma.ndim:
        sigma = sigma[..., None, None]
    x = np.zeros_like(b)
    for _ in range(cycles):
        x = vcycle(K, b, x, a, sigma, sweeps, D, c)
    return x
