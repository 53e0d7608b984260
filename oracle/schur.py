"""Schur-complement operator, right-hand side and preconditioner (oracle; test infrastructure).

Space-time arrays are time-major, shape ``(N + 1, n, n)``: row ``i`` holds the
spatial coefficients at time node ``t_i``.  A Kronecker product
``B_t (x) B_x`` acts by applying ``B_t`` along the time axis and ``B_x`` on
every row, the matrix-free identity of Section 5.2 (eq. (15)).
"""
from __future__ import annotations

import numpy as np

from . import multigrid, space3d, spatial, temporal, wavelet

ALPHA = 0.3  # alpha-scaling of the K_X blocks (Section 5.1)


class Problem:
    """A uniform space-time discretisation: ``N = 2**J`` time intervals and a
    ``2**K x 2**K`` square mesh, with the multigrid parameters of Section 5.1
    (2 V-cycles, 3 smoothing steps, alpha = 0.3)."""

    def __init__(self, J: int, K: int, alpha: float = ALPHA, cycles: int = 2, sweeps: int = 3,
                 D=None, c: float = 0.0, dim: int = 2):
        if J < 0 or K < 1:
            raise ValueError("need J >= 0 and K >= 1")
        if dim not in (2, 3):
            raise ValueError("dim must be 2 or 3")
        if dim == 3 and (D is not None or c != 0.0):
            raise ValueError("the 3D problem is the heat equation (Section 5.2)")
        # dim 3: Omega = [0, 1]^3 on the Kuhn tetrahedral mesh (space3d)
        self.dim = dim
        if D is not None and not (D[0] > 0 and D[1] > 0 and D[0] * D[1] > D[2] ** 2):
            raise ValueError("D must be symmetric positive definite")
        if c < 0:
            raise ValueError("need c >= 0")
        # reaction-diffusion operator of Section 4: A_x = A_D + c M_x
        self.D, self.c = (None if D is None else tuple(float(v) for v in D)), float(c)
        self.J, self.K = J, K
        self.N = 2 ** J
        self.n = 2 ** K - 1
        self.tau = 1.0 / self.N if self.N else 1.0
        self.h = 2.0 ** -K
        self.alpha = alpha
        self.cycles, self.sweeps = cycles, sweeps

    @property
    def shape(self):
        return (self.N + 1,) + (self.n,) * self.dim

    # spatial operators on every row
    def A(self, x):
        """``A_x x``: diffusion (``D``, None = identity) plus reaction ``c M_x``."""
        if self.dim == 3:
            return space3d.stiffness(x, self.h)
        if self.D is None and self.c == 0.0:
            return spatial.stiffness(x)
        return spatial.stiffness(x, self.D) + self.c * spatial.mass(x, self.h)

    def M(self, x):
        if self.dim == 3:
            return space3d.mass(x, self.h)
        return spatial.mass(x, self.h)

    def Kx(self, y):
        """``K_x ~ A_x^{-1}`` by multigrid on every row (Section 3.1)."""
        if self.dim == 3:
            return space3d.mg_apply(y, self.K, 1.0, 0.0, self.cycles, self.sweeps)
        return multigrid.apply(y, self.K, 1.0, 0.0, self.cycles, self.sweeps, self.D, self.c)

    # Lemma 4.2
    def S(self, X):
        """``S X = (A_t (x) M K M + M_t (x) A K A + L^T (x) M K A + L (x) A K M
        + Gamma_0 (x) M) X``, grouped as ``M K y1 + A K y2 + Gamma_0 (x) M``
        with ``y1 = M (A_t X) + A (L^T X)`` and ``y2 = A (M_t X) + M (L X)``."""
        tau = self.tau
        y1 = self.M(temporal.stiffness(X, tau)) + self.A(temporal.LT(X))
        y2 = self.A(temporal.mass(X, tau)) + self.M(temporal.L(X))
        z1 = self.Kx(y1)
        z2 = self.Kx(y2)
        out = self.M(z1) + self.A(z2)
        out[0] += self.M(X[0])
        return out

    # Lemma 4.1 with nodal data (interpolated g and u0)
    def rhs(self, g, u0):
        """``f = B^T K_Y g + u_0`` for nodal interpolants ``g`` (shape
        ``(N+1, n, n)`` or None for g = 0) and ``u0`` (shape ``(n, n)``).

        With ``g`` continuous piecewise linear in time it lies in ``Y_t``, so
        ``O^{-1} N`` reproduces it exactly and the T- and N-parts of B^T pair
        it with ``phi_i'`` and ``phi_i``: ``f_i = M K_x G1_i + A K_x G0_i`` with
        ``G0 = (M_t (x) M) g`` and ``G1 = (L^T (x) M) g``, plus ``M u0`` in row 0."""
        f = np.zeros(self.shape)
        if g is not None:
            G0 = self.M(temporal.mass(g, self.tau))
            G1 = self.M(temporal.LT(g))
            f = self.M(self.Kx(G1)) + self.A(self.Kx(G0))
        f[0] += self.M(u0)
        return f

    # Theorem 3.1 with the alpha-scaling of Section 5.1
    def KX(self, R):
        """Block-diagonal preconditioner: row ``i`` (wavelet level ``l``) gets
        ``K_l A_x K_l r_i`` with ``K_l`` the multigrid for ``alpha A_x + 2^l M_x``."""
        lev = wavelet.row_levels(self.J)
        sigma = 2.0 ** lev.astype(np.float64)
        a = self.alpha
        if self.dim == 3:
            Z = space3d.mg_apply(R, self.K, a, sigma, self.cycles, self.sweeps)
            return space3d.mg_apply(self.A(Z), self.K, a, sigma, self.cycles, self.sweeps)
        Z = multigrid.apply(R, self.K, a, sigma, self.cycles, self.sweeps, self.D, self.c)
        Z = self.A(Z)
        return multigrid.apply(Z, self.K, a, sigma, self.cycles, self.sweeps, self.D, self.c)

    # Section 3.4, eq. (11)
    def W(self, w):
        return wavelet.synthesis(w, self.J)

    def WT(self, y):
        return wavelet.analysis(y, self.J)

    def Shat(self, w):
        return self.WT(self.S(self.W(w)))
