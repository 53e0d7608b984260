"""Nested iteration over a hierarchy of space-time meshes (oracle; test infrastructure).

Section 4.2 ("Solving to higher accuracy") proposes to solve to an algebraic
error proportional to the discretisation error and to start each solve from
the solution on the next coarser mesh (a nested iteration), which makes the
cost linear in the number of unknowns.  The paper gives no further detail;
the reading taken here:

  * the meshes are (J - d, K - d) for d = D, ..., 1, 0: time and space halved
    together, d = 0 being the target mesh;
  * on each mesh the data are the nodal values of the same g and u0 at that
    mesh's nodes (every coarse node is a fine node), with f and f-hat of
    Lemma 4.1 and eq. (11) assembled there;
  * the coarsest mesh is solved from w = 0; every finer one by PCG from the
    coarser solution carried over to it (see :func:`prolong`);
  * the tolerance on mesh d is ``tol * 2**d``: the X-norm discretisation
    error of lowest-order elements decays with the first power of h and tau
    (Theorem 2.2 with the quasi-optimality of Section 3), so a tolerance that
    tracks the error halves with every refinement;
  * the stopping test is the one of Section 3.4, eq. (13), relative to
    ``sqrt(f-hat^T K_X f-hat)`` of that mesh.

Carrying a solution to the finer mesh.  The three-point wavelets of level
``l <= J - 1`` are the same functions on the meshes of ``J - 1`` and ``J``
intervals, and the coefficient of ``psi_{l,k}`` sits at time row
``(2k + 1) 2**(J-1-l)`` on the coarse mesh and twice that on the fine one
(rows 0 and N for level 0).  A coarse function therefore has, on the fine
mesh, its coarse coefficients at the even rows and zero at the odd rows (the
new finest wavelets).  In space, a coarse P1 function is re-expressed on the
fine mesh by P1 interpolation (``multigrid.prolong``).
"""
from __future__ import annotations

import numpy as np

from . import multigrid
from .pcg import pcg
from .schur import Problem


def prolong(w: np.ndarray) -> np.ndarray:
    """Wavelet-in-time, nodal-in-space coefficients of a solution on mesh
    (J - 1, K - 1), shape ``(2**(J-1) + 1, m, m)``, expressed on mesh (J, K),
    shape ``(2**J + 1, 2m + 1, 2m + 1)``."""
    rows = w.shape[0]
    fine = multigrid.prolong(w)
    out = np.zeros((2 * (rows - 1) + 1,) + fine.shape[1:])
    out[0::2] = fine
    return out


def inject_g(g, J, K, d):
    """Nodal values at the nodes of mesh (J - d, K - d) of data given at the
    nodes of mesh (J, K): every 2**d-th time row and spatial node."""
    s = 2 ** d
    return g[::s, s - 1::s, s - 1::s]


def inject_u0(u0, d):
    s = 2 ** d
    return u0[s - 1::s, s - 1::s]


def levels(J: int, K: int, depth: int) -> int:
    """Number of coarser meshes actually used: at most ``depth``, and the
    coarsest mesh keeps at least one time interval and one interior node."""
    return max(0, min(depth, J, K - 1))


def solve(J, K, g, u0, tol, depth, maxit=200, **kw):
    """Nested iteration on meshes (J - d, K - d), d = D..0 (D = levels(J, K,
    depth)).  Returns ``(u, iterations, history)``: the nodal solution on the
    target mesh, the PCG iterations per mesh (coarsest first), and the target
    mesh's residual history."""
    D = levels(J, K, depth)
    w = None
    its = []
    hist = []
    for d in range(D, -1, -1):
        P = Problem(J - d, K - d, **kw)
        gd = None if g is None else inject_g(g, J, K, d)
        fhat = P.WT(P.rhs(gd, inject_u0(u0, d)))
        w0 = None if w is None else prolong(w)
        w, k, hist = pcg(P, fhat, tol * 2.0 ** d, maxit, w0=w0)
        its.append(k)
    return Problem(J, K, **kw).W(w), its, hist
