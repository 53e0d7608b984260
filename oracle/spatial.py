"""Spatial P1 matrices on the uniform right-triangle mesh (oracle; test infrastructure).

The unit square is divided into ``2**K x 2**K`` squares, each cut along its
"/" diagonal (from node (i, j) to node (i+1, j+1)); ``X_x`` is the space of
continuous piecewise linears vanishing on the boundary (Section 4, Section
5.1).  An interior nodal array has shape ``(..., n, n)``, indexed
``[..., j, i]`` with ``n = 2**K - 1``; boundary values are zero and not stored.

Element integrals on this mesh (standard P1 on right triangles of area h^2/2):

  * stiffness ``A_x = <grad Phi_x, grad Phi_x>``: 4 at the node, -1 at the four
    axis neighbours, 0 across the diagonal (independent of h in 2D); with a
    diffusion tensor D (Section 4) see :func:`stiffness`;
  * mass ``M_x = <Phi_x, Phi_x>``: h^2/2 at the node, h^2/12 at each of the six
    neighbours (i+-1, j), (i, j+-1), (i+1, j+1), (i-1, j-1).
"""
from __future__ import annotations

import numpy as np


def _padded(x: np.ndarray) -> np.ndarray:
    shape = x.shape[:-2] + (x.shape[-2] + 2, x.shape[-1] + 2)
    xp = np.zeros(shape, dtype=x.dtype)
    xp[..., 1:-1, 1:-1] = x
    return xp


def neighbours(x: np.ndarray):
    """The six neighbour arrays of every node (zero outside the grid):
    east (i+1), west (i-1), north (j+1), south (j-1), north-east (i+1, j+1),
    south-west (i-1, j-1)."""
    xp = _padded(x)
    e = xp[..., 1:-1, 2:]
    w = xp[..., 1:-1, :-2]
    nth = xp[..., 2:, 1:-1]
    s = xp[..., :-2, 1:-1]
    ne = xp[..., 2:, 2:]
    sw = xp[..., :-2, :-2]
    return e, w, nth, s, ne, sw


def stiffness(x: np.ndarray, D=None) -> np.ndarray:
    """``A_x x`` for the diffusion of Section 4, ``int D grad u . grad v``, with
    the constant symmetric positive definite ``D = [[dxx, dxy], [dxy, dyy]]``
    given as ``(dxx, dyy, dxy)`` (None: the identity, the heat equation).

    On the "/" mesh the P1 element integrals give, independently of h in 2D:
    centre ``2 (dxx + dyy - dxy)``, the two x-neighbours ``dxy - dxx``, the two
    y-neighbours ``dxy - dyy``, the two neighbours across the "/" diagonal
    ``-dxy``; for D = Id the 5-point stencil (4, -1)."""
    e, w, nth, s, ne, sw = neighbours(x)
    if D is None:
        return 4.0 * x - e - w - nth - s
    dxx, dyy, dxy = D
    return (2.0 * (dxx + dyy - dxy) * x + (dxy - dxx) * (e + w) + (dxy - dyy) * (nth + s)
            - dxy * (ne + sw))


def mass(x: np.ndarray, h: float) -> np.ndarray:
    """``M_x x`` for mesh width ``h``."""
    e, w, nth, s, ne, sw = neighbours(x)
    return (h * h / 12.0) * (6.0 * x + e + w + nth + s + ne + sw)


def grid_size(K: int) -> int:
    return 2 ** K - 1


def to_grid(v: np.ndarray, K: int) -> np.ndarray:
    """Flat spatial vectors ``(..., n*n)`` -> grids ``(..., n, n)``."""
    n = grid_size(K)
    return v.reshape(v.shape[:-1] + (n, n))


def to_flat(x: np.ndarray) -> np.ndarray:
    return x.reshape(x.shape[:-2] + (x.shape[-2] * x.shape[-1],))
