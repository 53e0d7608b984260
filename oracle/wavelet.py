"""Three-point wavelet transform in time (oracle; test infrastructure).

Section 3.3 defines ``W_t`` as the change of basis from the wavelet basis
Sigma to the single-scale hat basis Phi_t, built level by level
(eq. (10)); Section 5 uses the three-point wavelets for
continuous piecewise linears.  The coefficients are not printed in the paper;
the basis used here is:

  * level 0: the two hats ``1 - t`` and ``t`` of the one-interval mesh;
  * level ``l = 1..J``, ``k = 0..2**(l-1) - 1``:
    ``psi_{l,k} = 2**(l/2) (phi^l_{2k+1} - b_{2k} phi^l_{2k} - b_{2k+2} phi^l_{2k+2})``
    with ``phi^l`` the hats on the mesh of width ``2**-l``; the weight ``b_e``
    is 1/2 at an interior node and 1 at ``t = 0`` or ``t = 1``, so every
    wavelet has zero integral; the factor ``2**(l/2)`` makes the L2 norms of
    all levels comparable, and ``|lambda| = l``.

Coordinates are stored in place on the ``N + 1 = 2**J + 1`` time rows:
the two level-0 coefficients at rows 0 and N, and the coefficient of
``psi_{l,k}`` at row ``(2k + 1) 2**(J - l)``.  Row ``i`` therefore carries level
``J - ctz(i)`` (level 0 at rows 0 and N).
"""
from __future__ import annotations

import numpy as np


def row_levels(J: int) -> np.ndarray:
    """Level ``|lambda|`` of the coefficient stored at each time row."""
    N = 2 ** J
    lev = np.zeros(N + 1, dtype=np.int64)
    for i in range(1, N):
        tz = 0
        while (i >> tz) & 1 == 0:
            tz += 1
        lev[i] = J - tz
    return lev


def _weight(e: np.ndarray, N: int) -> np.ndarray:
    return np.where((e == 0) | (e == N), 1.0, 0.5)


def synthesis(w: np.ndarray, J: int) -> np.ndarray:
    """``W_t`` along axis 0: wavelet coordinates -> hat-basis coefficients.

    Levels are added coarse to fine: at level ``l`` (stride ``s = 2**(J-l)``)
    the current single-scale function on the coarser mesh is re-expressed on
    the finer mesh (a new node takes the mean of its two neighbours) and the
    level-``l`` wavelets are added."""
    x = np.array(w, dtype=np.float64, copy=True)
    N = 2 ** J
    for l in range(1, J + 1):
        s = 2 ** (J - l)
        c = 2.0 ** (l / 2.0)
        odd = np.arange(s, N, 2 * s)
        d = x[odd].copy()
        left = x[odd - s].copy()
        right = x[odd + s].copy()
        shape = (-1,) + (1,) * (x.ndim - 1)
        bl = _weight(odd - s, N).reshape(shape)
        br = _weight(odd + s, N).reshape(shape)
        x[odd] = 0.5 * (left + right) + c * d
        x[odd - s] -= c * bl * d
        x[odd + s] -= c * br * d
    return x


def analysis(y: np.ndarray, J: int) -> np.ndarray:
    """``W_t^T`` along axis 0 (the transpose of :func:`synthesis`): levels
    fine to coarse, each the transpose of the corresponding synthesis step."""
    x = np.array(y, dtype=np.float64, copy=True)
    N = 2 ** J
    for l in range(J, 0, -1):
        s = 2 ** (J - l)
        c = 2.0 ** (l / 2.0)
        odd = np.arange(s, N, 2 * s)
        yo = x[odd].copy()
        yl = x[odd - s].copy()
        yr = x[odd + s].copy()
        shape = (-1,) + (1,) * (x.ndim - 1)
        bl = _weight(odd - s, N).reshape(shape)
        br = _weight(odd + s, N).reshape(shape)
        x[odd] = c * (yo - bl * yl - br * yr)
        x[odd - s] += 0.5 * yo
        x[odd + s] += 0.5 * yo
    return x
