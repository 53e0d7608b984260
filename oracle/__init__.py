"""CPU oracle for the space-time heat-equation solver (FP64, NumPy).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
the benchmark's CPU-baseline leg may import this package.  The GPU library
never calls it, shares no code with it, and fails loudly when its own HIP
build is missing instead of falling back to anything here.

It is a plain, slow, obviously-correct restatement of the method of
van Venetie & Westerdiep, "A parallel algorithm for solving linear parabolic
evolution equations" (arXiv 2009.08875), for the 2D heat equation on the unit
square with lowest-order elements in space and time:

  * ``temporal``   -- the time matrices A_t, M_t, L, L^T, Gamma_0 (Section 4,
                      Lemma 4.2);
  * ``spatial``    -- the P1 stiffness and mass matrices A_x, M_x on the
                      uniform right-triangle mesh (Section 4, Section 5.1);
  * ``multigrid``  -- the symmetric multigrid operators K_x ~ A_x^{-1}
                      (Section 3.1) and K_j ~ (alpha A_x + 2^j M_x)^{-1}
                      (Theorem 3.1, Section 5.1);
  * ``wavelet``    -- the three-point wavelet transform W_t and its transpose
                      (Section 3.3, eq. (10));
  * ``schur``      -- S (Lemma 4.2), the right-hand side f (Lemma 4.1),
                      S-hat = W^T S W and f-hat = W^T f (Section 3.4), K_X
                      (Theorem 3.1);
  * ``pcg``        -- PCG on S-hat w = f-hat with K_X and the stopping test
                      of Section 3.4, from zero or from an initial guess;
  * ``space3d``    -- the 3D spatial operators and multigrid on the Kuhn
                      tetrahedral mesh of the unit cube (Section 5.2's 3D
                      problem);
  * ``nested``     -- nested iteration over meshes (J - d, K - d) with a
                      tolerance that tracks the discretisation error
                      (Section 4.2).

Readings where the paper is silent (listed with reasons in the design notes):
the three-colour Gauss-Seidel ordering, pre-smoothing forward and
post-smoothing backward, recursion to one node solved exactly; the "/"
diagonal of the triangulation; the wavelet normalisation and boundary
weights; nodal interpolation of g and u0; the relative stopping test.

Parity status: every function here is pinned by the CPU tests (brute-force
finite-element assembly, basis evaluation, Lemma 4.1 with an explicit
Legendre basis, closed forms, the one-node worked example, dense solves, the
exact decaying solution, Table 1; the nested iteration's mesh transfer by
direct evaluation of the basis functions, its fixed point by PCG from zero,
and its error against the exact solution).  The solution values at the benchmark
sizes are not printed in the paper: the pins above are what fixes them.
"""
from . import temporal, spatial, space3d, multigrid, wavelet, schur, pcg, nested  # noqa: F401
from .pcg import solve  # noqa: F401
