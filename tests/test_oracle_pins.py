"""Pins of the CPU oracle against facts fixed outside it (no GPU).

Each test checks one oracle function against something other than its own
formula: brute-force finite-element assembly, pointwise basis evaluation,
quadrature, Lemma 4.1 with an explicit Legendre test basis, closed forms,
the one-node worked example, dense solves, or values printed in the paper.
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import multigrid, spatial, temporal, wavelet
from oracle.schur import Problem
from tests import bruteforce as bf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def op_matrix(fn, shape):
    """Dense matrix of a linear map on arrays of ``shape`` (columns = images of unit vectors)."""
    D = int(np.prod(shape))
    E = np.eye(D).reshape((D,) + tuple(shape))
    return np.stack([np.asarray(fn(E[k])).ravel() for k in range(D)], 1)


# --------------------------------------------------------------- temporal (O1)

@pytest.mark.parametrize("N", [1, 2, 5, 8])
def test_temporal_matrices_match_quadrature(N):
    At, Mt, L = bf.temporal_by_quadrature(N)
    At_o, Mt_o, L_o, G_o = temporal.dense(N)
    assert np.allclose(At_o, At, rtol=0, atol=1e-12 * N)
    assert np.allclose(Mt_o, Mt, rtol=0, atol=1e-15)
    assert np.allclose(L_o, L, rtol=0, atol=1e-14)
    LT_o = op_matrix(temporal.LT, (N + 1,))
    assert np.allclose(LT_o, L.T, atol=1e-14)
    G = np.zeros((N + 1, N + 1))
    G[0, 0] = 1.0
    assert np.array_equal(G_o, G)


@pytest.mark.parametrize("N", [1, 4, 16])
def test_temporal_invariants(N):
    At, Mt, L, _ = temporal.dense(N)
    # integration by parts: L + L^T = diag(-1, 0, ..., 0, 1)
    D = np.zeros((N + 1, N + 1))
    D[0, 0], D[N, N] = -1.0, 1.0
    assert np.allclose(L + L.T, D, atol=1e-15)
    one = np.ones(N + 1)
    assert np.allclose(At @ one, 0.0, atol=1e-12)       # constants have no derivative
    assert abs(one @ Mt @ one - 1.0) < 1e-14             # |I| = T = 1
    assert np.allclose(L @ one, 0.0, atol=1e-15)          # L applied to a constant


# ---------------------------------------------------------------- spatial (O2)

@pytest.mark.parametrize("K", [1, 2, 3])
def test_spatial_matrices_match_fe_assembly(K):
    A, M = bf.p1_assembly(K)
    n = 2 ** K - 1
    h = 2.0 ** -K
    assert np.allclose(op_matrix(spatial.stiffness, (n, n)), A, atol=1e-13)
    assert np.allclose(op_matrix(lambda x: spatial.mass(x, h), (n, n)), M, atol=1e-16)


def test_stiffness_spectrum_closed_form():
    K = 3
    n = 2 ** K - 1
    h = 2.0 ** -K
    A = op_matrix(spatial.stiffness, (n, n))
    p = np.arange(1, n + 1)
    lam = (4.0 - 2.0 * np.cos(p[:, None] * np.pi * h) - 2.0 * np.cos(p[None, :] * np.pi * h)).ravel()
    assert np.allclose(np.sort(np.linalg.eigvalsh(A)), np.sort(lam), atol=1e-12)


def test_mass_interior_row_sum():
    K = 4
    h = 2.0 ** -K
    n = 2 ** K - 1
    Mx = spatial.mass(np.ones((n, n)), h)
    assert np.allclose(Mx[1:-1, 1:-1], h * h, atol=1e-18)   # integral of a hat = h^2


# -------------------------------------------------------------- multigrid (O3)

@pytest.mark.parametrize("K,a,sigma", [(2, 1.0, 0.0), (3, 1.0, 0.0), (3, 0.3, 8.0), (4, 0.3, 64.0)])
def test_multigrid_matches_dense_recursive_vcycle(K, a, sigma):
    rng = np.random.default_rng(K)
    n = 2 ** K - 1
    b = rng.standard_normal((n, n))
    ref = bf.dense_mg(b.ravel(), K, a, sigma)
    got = multigrid.apply(b, K, a, sigma)
    assert np.allclose(got.ravel(), ref, rtol=0, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("K,a,sigma", [(3, 1.0, 0.0), (4, 0.3, 2.0 ** 6)])
def test_multigrid_symmetric_positive_definite(K, a, sigma):
    n = 2 ** K - 1
    B = op_matrix(lambda x: multigrid.apply(x, K, a, sigma), (n, n))
    assert np.abs(B - B.T).max() <= 1e-12 * np.abs(B).max()
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0


def test_multigrid_one_node_is_exact_and_contraction_is_mesh_independent():
    # one interior node: the coarse solve is exact
    b = np.array([[3.0]])
    assert multigrid.apply(b, 1, 1.0, 0.0)[0, 0] == pytest.approx(3.0 / 4.0, rel=1e-15)
    assert multigrid.apply(b, 1, 0.3, 8.0)[0, 0] == pytest.approx(3.0 / (1.2 + 1.0), rel=1e-15)
    # two V-cycles contract the C-norm error strongly, uniformly in h
    rates = []
    for K in (3, 4, 5):
        n = 2 ** K - 1
        C = op_matrix(spatial.stiffness, (n, n))
        B = op_matrix(lambda x: multigrid.apply(x, K, 1.0, 0.0), (n, n))
        E = np.eye(n * n) - B @ C
        L = np.linalg.cholesky(C)
        rates.append(np.linalg.norm(L.T @ E @ np.linalg.inv(L.T), 2))
    assert max(rates) < 0.1
    assert max(rates) - min(rates) < 0.05


def test_more_vcycles_converge_to_inverse():
    K = 4
    n = 2 ** K - 1
    b = np.random.default_rng(0).standard_normal((n, n))
    A, M = bf.p1_assembly(K)
    C = 0.3 * A + 16.0 * M
    exact = np.linalg.solve(C, b.ravel())
    err = [np.abs(multigrid.apply(b, K, 0.3, 16.0, cycles=c).ravel() - exact).max() for c in (1, 2, 4, 8)]
    assert err[1] < err[0] and err[2] < err[1] and err[3] < 1e-8 * np.abs(exact).max()


# ---------------------------------------------------------------- wavelet (O5)

@pytest.mark.parametrize("J", [1, 2, 3, 5])
def test_wavelet_synthesis_equals_basis_evaluation(J):
    W_eval = bf.wavelet_basis_matrix(J)
    W_o = op_matrix(lambda w: wavelet.synthesis(w, J), (2 ** J + 1,))
    assert np.allclose(W_o, W_eval, atol=1e-13)


def test_wavelet_J1_explicit():
    r2 = np.sqrt(2.0)
    ref = np.array([[1.0, -r2, 0.0], [0.5, r2, 0.5], [0.0, -r2, 1.0]])
    assert np.allclose(op_matrix(lambda w: wavelet.synthesis(w, 1), (3,)), ref, atol=1e-15)


@pytest.mark.parametrize("J", [1, 3, 6])
def test_wavelet_analysis_is_transpose_and_transform_invertible(J):
    N = 2 ** J
    rng = np.random.default_rng(J)
    x = rng.standard_normal((N + 1, 3))
    y = rng.standard_normal((N + 1, 3))
    lhs = np.sum(wavelet.synthesis(x, J) * y)
    rhs = np.sum(x * wavelet.analysis(y, J))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)
    W = op_matrix(lambda w: wavelet.synthesis(w, J), (N + 1,))
    assert np.linalg.cond(W) < 1e3


def test_wavelets_have_vanishing_integral_and_levels():
    J = 5
    N = 2 ** J
    W = bf.wavelet_basis_matrix(J)
    _, Mt, _, _ = temporal.dense(N)
    ints = np.ones(N + 1) @ Mt @ W
    lev = wavelet.row_levels(J)
    assert np.allclose(ints[lev > 0], 0.0, atol=1e-14)
    assert lev[0] == 0 and lev[N] == 0 and lev[N // 2] == 1 and lev[1] == J and lev[N - 1] == J


# ---------------------------------------------------------- Schur operator (O4)

def _S_lemma41(J, K, Kx_dense, D=None, c=0.0):
    """S = B^T K_Y B + Gamma_0 (x) M with an explicit Legendre Xi and O diagonal;
    A = A_D + c M assembled element by element (Section 4)."""
    N = 2 ** J
    O, T, Nm = bf.legendre_test_space(N)
    A, M = bf.p1_assembly(K, D)
    A = A + c * M
    B = np.kron(T, M) + np.kron(Nm, A)
    KY = np.kron(np.diag(1.0 / O), Kx_dense)
    G = np.zeros((N + 1, N + 1))
    G[0, 0] = 1.0
    return B, KY, B.T @ KY @ B + np.kron(G, M), A, M


@pytest.mark.parametrize("J,K", [(0, 1), (1, 2), (2, 2), (3, 2)])
def test_S_lemma41_equals_lemma42(J, K):
    P = Problem(J, K)
    Kx = op_matrix(P.Kx, (P.n, P.n))
    _, _, S41, _, _ = _S_lemma41(J, K, Kx)
    S42 = op_matrix(P.S, P.shape)
    assert np.abs(S42 - S41).max() <= 1e-12 * np.abs(S41).max()
    assert np.abs(S42 - S42.T).max() <= 1e-13 * np.abs(S42).max()
    assert np.linalg.eigvalsh(0.5 * (S42 + S42.T)).min() > 0


def test_S_closed_form_with_exact_inverse():
    """With K_x = A^{-1}: S = A_t (x) M A^{-1} M + M_t (x) A + e_N e_N^T (x) M."""
    J, K = 2, 2
    P = Problem(J, K)
    A, M = bf.p1_assembly(K)
    Ainv = np.linalg.inv(A)
    P.Kx = lambda y: (Ainv @ y.reshape(y.shape[0], -1).T).T.reshape(y.shape)
    At, Mt, _ = bf.temporal_by_quadrature(2 ** J)
    eN = np.zeros((2 ** J + 1, 2 ** J + 1))
    eN[-1, -1] = 1.0
    ref = np.kron(At, M @ Ainv @ M) + np.kron(Mt, A) + np.kron(eN, M)
    got = op_matrix(P.S, P.shape)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("J,K", [(1, 2), (2, 3)])
def test_rhs_lemma41(J, K):
    """f = B^T K_Y g_vec + u_0 with g_vec = <g_I, Xi (x) Phi_x> of the nodal interpolant."""
    P = Problem(J, K)
    rng = np.random.default_rng(7)
    g = rng.standard_normal(P.shape)
    u0 = rng.standard_normal((P.n, P.n))
    Kx = op_matrix(P.Kx, (P.n, P.n))
    B, KY, _, A, M = _S_lemma41(J, K, Kx)
    _, _, Nm = bf.legendre_test_space(2 ** J)
    gvec = np.kron(Nm, M) @ g.ravel()
    ref = B.T @ KY @ gvec
    ref[: P.n * P.n] += M @ u0.ravel()
    got = P.rhs(g, u0).ravel()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


# ------------------------------------------------------------ worked example

def test_one_node_worked_example_golden():
    with open(os.path.join(GOLDEN, "one_node_J0_K1.json")) as f:
        gold = json.load(f)
    P = Problem(0, 1)
    S = op_matrix(P.S, P.shape)
    assert np.allclose(S * 768.0, np.array(gold["S_times_768"]), rtol=0, atol=1e-12)
    f = P.rhs(None, np.ones((1, 1))).ravel()
    assert np.allclose(f, gold["f"], atol=1e-16)
    u, its, _ = oracle.solve(0, 1, None, np.ones((1, 1)), tol=1e-15, maxit=10)
    exact = np.array(gold["u_num"]) / gold["u_den"]
    assert np.allclose(u.ravel(), exact, rtol=1e-14, atol=0)


# --------------------------------------------------- PCG vs dense solve (O8)

@pytest.mark.parametrize("J,K", [(2, 2), (3, 3), (4, 2)])
def test_pcg_matches_dense_solve(J, K):
    P = Problem(J, K)
    rng = np.random.default_rng(J * 10 + K)
    g = rng.standard_normal(P.shape)
    u0 = rng.standard_normal((P.n, P.n))
    S = op_matrix(P.S, P.shape)
    f = P.rhs(g, u0).ravel()
    exact = np.linalg.solve(S, f)
    u, its, hist = oracle.solve(J, K, g, u0, tol=1e-13, maxit=200)
    rel = np.linalg.norm(u.ravel() - exact) / np.linalg.norm(exact)
    assert rel < 1e-11
    assert its < 40


def test_zero_data_gives_zero_solution():
    u, its, _ = oracle.solve(2, 2, None, np.zeros((3, 3)))
    assert its == 0 and not np.any(u)


# ------------------------------------------------------ Table 1 calibration

def _kappa_direct(J, K, alpha=0.3):
    N = 2 ** J
    At, Mt, L, G = temporal.dense(N)
    A, M = bf.p1_assembly(K)
    Ainv = np.linalg.inv(A)
    S = np.kron(At, M @ Ainv @ M) + np.kron(Mt, A) + np.kron(L.T, M) + np.kron(L, M) + np.kron(G, M)
    Wt = op_matrix(lambda w: wavelet.synthesis(w, J), (N + 1,))
    W = np.kron(Wt, np.eye(A.shape[0]))
    Sh = W.T @ S @ W
    lev = wavelet.row_levels(J)
    nx = A.shape[0]
    Kinv = np.zeros_like(Sh)
    for i in range(N + 1):
        C = alpha * A + 2.0 ** lev[i] * M
        Kinv[i * nx:(i + 1) * nx, i * nx:(i + 1) * nx] = C @ Ainv @ C
    import scipy.linalg as sl
    ev = sl.eigh(Sh, Kinv, eigvals_only=True)
    return ev.max() / ev.min()


def _kappa_matrix_free(J, K, alpha=0.3):
    """kappa_2(K_X S-hat) with direct inverses for sizes where dense matrices
    of the whole space-time system are too large: the extreme eigenvalues of
    the symmetric form L^T S-hat L, K_X = L L^T (blockwise Cholesky), by
    ARPACK.  S (Lemma 4.2 with K_x = A_x^{-1}) acts through the Kronecker
    identity (T (x) B) vec(X) = vec(T X B) for symmetric B, on dense P1
    matrices from element-by-element assembly."""
    from scipy.sparse.linalg import LinearOperator, eigsh

    N = 2 ** J
    At, Mt, L, G = temporal.dense(N)
    A, M = bf.p1_assembly(K)
    Ai = np.linalg.inv(A)
    MAM = M @ Ai @ M
    Wt = bf.wavelet_basis_matrix(J)
    lev = wavelet.row_levels(J)
    chol = {}
    for l in set(int(v) for v in lev):
        Ci = np.linalg.inv(alpha * A + 2.0 ** l * M)
        chol[l] = np.linalg.cholesky(Ci @ A @ Ci)
    Lrow = [chol[int(l)] for l in lev]
    nx = A.shape[0]

    def S(X):
        return At @ X @ MAM + Mt @ X @ A + L.T @ X @ M + L @ X @ M + G @ X @ M

    def B(v):
        V = v.reshape(N + 1, nx)
        Y = np.stack([Lrow[i] @ V[i] for i in range(N + 1)])
        Z = Wt.T @ S(Wt @ Y)
        return np.stack([Lrow[i].T @ Z[i] for i in range(N + 1)]).ravel()

    op = LinearOperator(((N + 1) * nx,) * 2, matvec=B, dtype=np.float64)
    hi = eigsh(op, k=1, which="LA", tol=1e-12, return_eigenvectors=False)[0]
    lo = eigsh(op, k=1, which="SA", tol=1e-12, return_eigenvectors=False)[0]
    return hi / lo


def test_matrix_free_kappa_equals_dense_eigensolve():
    """The matrix-free estimate reproduces the dense generalised eigensolve."""
    k = _kappa_direct(4, 3)
    assert abs(_kappa_matrix_free(4, 3) - k) <= 1e-8 * k


@pytest.mark.slow
def test_table1_condition_number():
    """kappa_2(K_X S-hat) with direct inverses, alpha = 0.3, N_t = 65 dofs,
    N_x = 49 by a dense generalised eigensolve (Table 1 prints 6.34)."""
    with open(os.path.join(GOLDEN, "table1_kappa.json")) as f:
        gold = json.load(f)
    cell = gold["cells"]["Nt65_Nx49"]
    k = _kappa_direct(6, 3)
    assert abs(k - cell["kappa"]) <= gold["tolerance_abs"]


@pytest.mark.slow
@pytest.mark.parametrize("cell", ["Nt65_Nx49", "Nt129_Nx49", "Nt257_Nx49", "Nt65_Nx225"])
def test_table1_all_cells(cell):
    """Every stored cell of Table 1 (growth with N_t at N_x = 49, and the
    N_x = 225 column), by the matrix-free eigenvalue computation."""
    with open(os.path.join(GOLDEN, "table1_kappa.json")) as f:
        gold = json.load(f)
    c = gold["cells"][cell]
    k = _kappa_matrix_free(c["J"], c["K"])
    assert abs(k - c["kappa"]) <= gold["tolerance_abs"], (cell, k)


def test_KX_equals_dense_multigrid_blocks():
    """K_X of Theorem 3.1 with the multigrid K_l: row i of K_X R equals
    K_l A K_l r_i with K_l the dense matrix of the sequential-Gauss-Seidel
    multigrid (tests/bruteforce.py) for alpha A + 2^l M, l = level of row i."""
    J, K = 3, 3
    P = Problem(J, K)
    R = np.random.default_rng(8).standard_normal(P.shape)
    got = P.KX(R)
    A, _ = bf.p1_assembly(K)
    lev = wavelet.row_levels(J)
    mats = {}
    for i in range(P.N + 1):
        l = int(lev[i])
        if l not in mats:
            mats[l] = bf.dense_mg_matrix(K, 0.3, 2.0 ** l)
        Kl = mats[l]
        ref = Kl @ A @ Kl @ R[i].ravel()
        assert np.allclose(got[i].ravel(), ref, rtol=0, atol=1e-13 * np.abs(ref).max()), i


# ---------------------------------------- exact solution and convergence order

def _xnorm_error(J, K, solver=None):
    """Computable X-norm surrogate of u - u_h for u = exp(-2 pi^2 t) sin(pi x) sin(pi y):
    ||grad e||^2 + ||d_t e||^2 / lambda_1 + ||e(1)||^2 (L2 over space-time;
    lambda_1 = 2 pi^2 bounds the dual-norm part by Poincare).  u_h is the
    oracle's solution to 1e-12, or solver(J, K, u0) when given."""
    lam = 2.0 * np.pi ** 2
    n = 2 ** K - 1
    h = 2.0 ** -K
    x = np.arange(1, n + 1) * h
    u0 = np.outer(np.sin(np.pi * x), np.sin(np.pi * x))
    if solver is None:
        uh, its, _ = oracle.solve(J, K, None, u0, tol=1e-12, maxit=200)
    else:
        uh = solver(J, K, u0)
    N = 2 ** J
    tau = 1.0 / N
    At, Mt, _ = bf.temporal_by_quadrature(N)
    A = spatial.stiffness
    M = lambda v: spatial.mass(v, h)
    # int s phi_k over the hat support, s = sin(pi x) sin(pi y), by triangle quadrature
    r, s, w = bf.triangle_rule(10)
    sphi = np.zeros((n, n))
    for jj in range(n):
        for ii in range(n):
            X0, Y0 = (ii + 1) * h, (jj + 1) * h
            tot = 0.0
            for (dx1, dy1), (dx2, dy2) in (((1, 0), (1, 1)), ((1, 1), (0, 1)), ((0, 1), (-1, 0)),
                                         ((-1, 0), (-1, -1)), ((-1, -1), (0, -1)), ((0, -1), (1, 0))):
                px = X0 + h * (dx1 * r + dx2 * s)
                py = Y0 + h * (dy1 * r + dy2 * s)
                # the Jacobian of each of the six triangles is h^2
                tot += h * h * np.sum(w * np.sin(np.pi * px) * np.sin(np.pi * py) * (1.0 - r - s))
            sphi[jj, ii] = tot
    t = np.arange(N + 1) * tau
    a_i = np.array([sum(bf.gauss_interval(lambda tt: np.exp(-lam * tt) * bf.hat(tt, i, tau), e * tau, (e + 1) * tau)
                        for e in (i - 1, i) if 0 <= e < N) for i in range(N + 1)])
    d_i = np.array([sum(bf.gauss_interval(lambda tt: -lam * np.exp(-lam * tt) * bf.hat_dt(tt, i, tau), e * tau, (e + 1) * tau)
                        for e in (i - 1, i) if 0 <= e < N) for i in range(N + 1)])
    E = (1.0 - np.exp(-2.0 * lam)) / (2.0 * lam)
    Qu = E * (np.pi ** 2 / 2.0) + (lam ** 2 * E * 0.25) / lam + np.exp(-2.0 * lam) * 0.25
    # cross terms: int grad u . grad u_h = sum u_h[i,k] a_i * (2 pi^2) int s phi_k
    cross = np.sum(uh * a_i[:, None, None] * lam * sphi[None]) \
        + np.sum(uh * d_i[:, None, None] * sphi[None]) / lam \
        + np.exp(-lam) * np.sum(uh[N] * sphi)
    Quh = np.sum(np.tensordot(Mt, uh, axes=(1, 0)) * A(uh)) \
        + np.sum(np.tensordot(At, uh, axes=(1, 0)) * M(uh)) / lam \
        + np.sum(uh[N] * M(uh[N]))
    return np.sqrt(max(Qu - 2.0 * cross + Quh, 0.0))


@pytest.mark.slow
def test_first_order_convergence_to_exact_solution():
    errs = [_xnorm_error(L, L) for L in (2, 3, 4, 5, 6)]
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:]))
    assert 0.85 <= orders[-1] <= 1.3, (errs, orders)


# ---------------------------------------------------- iteration boundedness

@pytest.mark.slow
def test_iterations_bounded_under_refinement():
    n_of = lambda K: 2 ** K - 1
    its_t = []
    for J in (2, 4, 6, 8):
        K = 3
        x = np.arange(1, n_of(K) + 1) / 2 ** K
        u0 = np.outer(np.sin(np.pi * x), np.sin(np.pi * x))
        its_t.append(oracle.solve(J, K, None, u0, tol=1e-8)[1])
    its_x = []
    for K in (2, 3, 4, 5):
        x = np.arange(1, n_of(K) + 1) / 2 ** K
        u0 = np.outer(np.sin(np.pi * x), np.sin(np.pi * x))
        its_x.append(oracle.solve(3, K, None, u0, tol=1e-8)[1])
    assert max(its_t) <= 30 and max(its_x) <= 30
    steps = [b - a for a, b in zip(its_t, its_t[1:])]
    assert all(d <= 4 for d in steps)            # at most 2 more iterations per doubling of N
    assert steps[-1] <= steps[0]                 # and the growth slows down
    assert max(its_x) - min(its_x) <= 4                         # near-flat in space


# ------------------------------------------------ nested iteration (Section 4.2)

def test_pcg_from_an_initial_guess():
    """PCG started from the discrete solution stops at once; started from any
    other guess it reaches the same solution as from zero (Section 3.4)."""
    from oracle.pcg import pcg

    J, K = 3, 3
    P = Problem(J, K)
    fhat = P.WT(P.rhs(synth.fourier_g(J, K, 4), synth.smooth_u0(K, 4)))
    w_ref, _, _ = pcg(P, fhat, 1e-13, 200)
    _, k, _ = pcg(P, fhat, 1e-6, 200, w0=w_ref)
    assert k == 0
    w, k, _ = pcg(P, fhat, 1e-12, 200, w0=np.random.default_rng(1).standard_normal(P.shape))
    assert k > 0 and np.linalg.norm(w - w_ref) <= 1e-9 * np.linalg.norm(w_ref)


@pytest.mark.parametrize("J,K", [(2, 2), (3, 3), (4, 2)])
def test_nested_prolongation_embeds_the_coarse_function(J, K):
    """The coarse solution carried to the finer mesh represents the same
    function: evaluated through the fine wavelet basis it equals the coarse
    function's nodal values interpolated linearly in time and by P1 in space
    (basis functions and hats evaluated directly, tests/bruteforce.py)."""
    from oracle import nested

    m = 2 ** (K - 1) - 1
    w = np.random.default_rng(J + K).standard_normal((2 ** (J - 1) + 1, m, m))
    fine = nested.prolong(w)
    Wf = bf.wavelet_basis_matrix(J)
    Wc = bf.wavelet_basis_matrix(J - 1)
    Ps = bf.prolongation_by_evaluation(K)
    uc = np.einsum("ti,ijk->tjk", Wc, w).reshape(2 ** (J - 1) + 1, -1)   # coarse nodal values
    tc = np.arange(2 ** (J - 1) + 1) / 2 ** (J - 1)
    tf = np.arange(2 ** J + 1) / 2 ** J
    ut = np.stack([np.interp(tf, tc, uc[:, k]) for k in range(uc.shape[1])], 1)
    ref = ut @ Ps.T
    got = np.einsum("ti,ijk->tjk", Wf, fine).reshape(2 ** J + 1, -1)
    assert np.allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_nested_iteration_reaches_the_discrete_solution():
    """With a tight tolerance the nested iteration returns the solution of
    S u = f on the target mesh (the same as PCG from zero)."""
    from oracle import nested

    J, K = 4, 4
    g, u0 = synth.fourier_g(J, K, 5), synth.smooth_u0(K, 5)
    u_ref, _, _ = oracle.solve(J, K, g, u0, tol=1e-13)
    u, its, _ = nested.solve(J, K, g, u0, 1e-12, depth=3)
    assert len(its) == 4
    assert np.linalg.norm(u - u_ref) <= 1e-9 * np.linalg.norm(u_ref)


@pytest.mark.slow
def test_nested_iteration_error_tracks_the_discretisation_error():
    """Section 4.2: with the algebraic tolerance proportional to the
    discretisation error (0.1 h here), the nested iteration's error against
    the exact solution exp(-2 pi^2 t) sin(pi x) sin(pi y) stays within 1 %
    of the discrete solution's own error, with a few iterations per mesh."""
    from oracle import nested

    for L in (4, 5):
        e_disc = _xnorm_error(L, L)
        e_nest = _xnorm_error(L, L, lambda J, K, u0: nested.solve(J, K, None, u0, 0.1 * 2.0 ** -K, 3)[0])
        assert e_nest <= 1.01 * e_disc, (L, e_nest, e_disc)
        its = nested.solve(L, L, None, np.outer(*[np.sin(np.pi * np.arange(1, 2 ** L) / 2 ** L)] * 2),
                           0.1 * 2.0 ** -L, 3)[1]
        assert max(its) <= 8, its


# ------------------------------------- reaction-diffusion operator (Section 4)

RD = [((2.0, 0.5, 0.3), 0.0), ((1.0, 3.0, -0.4), 5.0), (None, 7.0)]


@pytest.mark.parametrize("D", [(2.0, 0.5, 0.3), (1.0, 3.0, -0.4), (0.7, 0.7, 0.6)])
@pytest.mark.parametrize("K", [2, 3])
def test_stiffness_with_diffusion_tensor_matches_assembly(D, K):
    """int D grad u . grad v on the "/" mesh, element by element."""
    A, _ = bf.p1_assembly(K, D)
    n = 2 ** K - 1
    got = op_matrix(lambda x: spatial.stiffness(x, D), (n, n))
    assert np.allclose(got, A, rtol=0, atol=1e-13)


def test_diagonal_diffusion_spectrum_closed_form():
    """D = diag(dxx, dyy): eigenvalues 2 dxx (1 - cos p pi h) + 2 dyy (1 - cos q pi h)."""
    K, D = 3, (2.0, 0.5, 0.0)
    n, h = 2 ** K - 1, 2.0 ** -K
    Am = op_matrix(lambda x: spatial.stiffness(x, D), (n, n))
    p = np.arange(1, n + 1)
    lam = np.sort((2 * D[0] * (1 - np.cos(p[:, None] * np.pi * h))
                   + 2 * D[1] * (1 - np.cos(p[None, :] * np.pi * h))).ravel())
    assert np.allclose(np.linalg.eigvalsh(Am), lam, atol=1e-12)


@pytest.mark.parametrize("D,c", RD)
@pytest.mark.parametrize("a,sigma", [(1.0, 0.0), (0.3, 16.0)])
def test_multigrid_reaction_diffusion_matches_dense_vcycle(D, c, a, sigma):
    """The multigrid for a (A_D + c M) + sigma M against the dense sequential
    Gauss-Seidel V-cycle on element-assembled matrices."""
    K = 3
    b = np.random.default_rng(11).standard_normal((2 ** K - 1, 2 ** K - 1))
    got = multigrid.apply(b, K, a, sigma, D=D, c=c)
    ref = bf.dense_mg(b.ravel(), K, a, sigma, D=D, c=c)
    assert np.allclose(got.ravel(), ref, rtol=0, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("D,c", RD)
def test_S_lemma41_equals_lemma42_reaction_diffusion(D, c):
    J, K = 2, 2
    P = Problem(J, K, D=D, c=c)
    Kx = op_matrix(P.Kx, (P.n, P.n))
    _, _, S41, _, _ = _S_lemma41(J, K, Kx, D, c)
    S42 = op_matrix(P.S, P.shape)
    assert np.abs(S42 - S41).max() <= 1e-12 * np.abs(S41).max()
    assert np.linalg.eigvalsh(0.5 * (S42 + S42.T)).min() > 0


@pytest.mark.parametrize("D,c", RD)
def test_S_closed_form_with_exact_inverse_reaction_diffusion(D, c):
    """With K_x = A_x^{-1}, A_x = A_D + c M: the closed form of Lemma 4.2."""
    J, K = 2, 2
    P = Problem(J, K, D=D, c=c)
    A, M = bf.p1_assembly(K, D)
    A = A + c * M
    Ainv = np.linalg.inv(A)
    P.Kx = lambda y: (Ainv @ y.reshape(y.shape[0], -1).T).T.reshape(y.shape)
    At, Mt, _ = bf.temporal_by_quadrature(2 ** J)
    eN = np.zeros((2 ** J + 1, 2 ** J + 1))
    eN[-1, -1] = 1.0
    ref = np.kron(At, M @ Ainv @ M) + np.kron(Mt, A) + np.kron(eN, M)
    got = op_matrix(P.S, P.shape)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("D,c", RD)
def test_rhs_lemma41_reaction_diffusion(D, c):
    J, K = 2, 2
    P = Problem(J, K, D=D, c=c)
    rng = np.random.default_rng(17)
    g = rng.standard_normal(P.shape)
    u0 = rng.standard_normal((P.n, P.n))
    Kx = op_matrix(P.Kx, (P.n, P.n))
    B, KY, _, A, M = _S_lemma41(J, K, Kx, D, c)
    _, _, Nm = bf.legendre_test_space(2 ** J)
    ref = B.T @ KY @ (np.kron(Nm, M) @ g.ravel())
    ref[: P.n * P.n] += M @ u0.ravel()
    got = P.rhs(g, u0).ravel()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("D,c", RD)
def test_pcg_matches_dense_solve_reaction_diffusion(D, c):
    J, K = 3, 3
    P = Problem(J, K, D=D, c=c)
    g, u0 = synth.fourier_g(J, K, 8), synth.smooth_u0(K, 8)
    S = op_matrix(P.S, P.shape)
    exact = np.linalg.solve(S, P.rhs(g, u0).ravel())
    u, its, _ = oracle.solve(J, K, g, u0, tol=1e-13, maxit=200, D=D, c=c)
    assert np.linalg.norm(u.ravel() - exact) <= 1e-11 * np.linalg.norm(exact)
    assert its < 40


@pytest.mark.slow
def test_reaction_diffusion_converges_to_exact_solution():
    """u = exp(-((dxx + dyy) pi^2 + c) t) sin(pi x) sin(pi y) solves
    u_t - div(D grad u) + c u = 0 for diagonal D; the nodal error of the
    discrete solution falls by at least 1.8 per joint refinement of h and tau."""
    D, c = (2.0, 0.5, 0.0), 3.0
    rate = (D[0] + D[1]) * np.pi ** 2 + c
    errs = []
    for L in (3, 4, 5):
        n = 2 ** L - 1
        x = np.arange(1, n + 1) / 2 ** L
        s = np.outer(np.sin(np.pi * x), np.sin(np.pi * x))
        u, _, _ = oracle.solve(L, L, None, s, tol=1e-12, maxit=200, D=D, c=c)
        t = np.arange(2 ** L + 1) / 2 ** L
        exact = np.exp(-rate * t)[:, None, None] * s[None]
        errs.append(np.abs(u - exact).max())
    assert errs[0] / errs[1] >= 1.8 and errs[1] / errs[2] >= 1.8, errs


# -------------------------------------------- 3D problem (Section 5.2, Kuhn mesh)

def _cube_sin(K):
    n = 2 ** K - 1
    x = np.arange(1, n + 1) / 2 ** K
    s = np.sin(np.pi * x)
    return np.einsum("i,j,k->kji", s, s, s)


@pytest.mark.parametrize("K", [1, 2])
def test_3d_matrices_match_assembly(K):
    from oracle import space3d

    A, M = bf.p1_assembly_3d(K)
    n, h = 2 ** K - 1, 2.0 ** -K
    assert np.allclose(op_matrix(lambda x: space3d.stiffness(x, h), (n, n, n)), A, atol=1e-14)
    assert np.allclose(op_matrix(lambda x: space3d.mass(x, h), (n, n, n)), M, atol=1e-16)


def test_3d_stiffness_spectrum_and_mass_rows():
    """A_x on the Kuhn mesh is h times the 7-point Laplacian: eigenvalues
    h sum_d (2 - 2 cos(p_d pi h)); interior rows of M sum to h^3."""
    from oracle import space3d

    K = 3
    n, h = 2 ** K - 1, 2.0 ** -K
    Am = op_matrix(lambda x: space3d.stiffness(x, h), (n, n, n))
    c = 2 - 2 * np.cos(np.arange(1, n + 1) * np.pi * h)
    lam = np.sort((h * (c[:, None, None] + c[None, :, None] + c[None, None, :])).ravel())
    assert np.allclose(np.linalg.eigvalsh(Am), lam, atol=1e-12)
    rows = space3d.mass(np.ones((n, n, n)), h)
    assert abs(rows[n // 2, n // 2, n // 2] - h ** 3) <= 1e-16


def test_3d_prolongation_is_interpolation():
    """P carries a coarse P1 function to the fine mesh by its values at the
    fine nodes (located tetrahedron, barycentric coordinates); the
    restriction is its transpose."""
    from oracle import space3d

    K = 3
    e = np.random.default_rng(3).standard_normal((3, 3, 3))
    nf = 2 ** K - 1
    pts = [((i + 1) / 2 ** K, (j + 1) / 2 ** K, (k + 1) / 2 ** K)
           for k in range(nf) for j in range(nf) for i in range(nf)]
    ref = bf.kuhn_eval(e, K - 1, pts)
    assert np.allclose(space3d.prolong(e).ravel(), ref, atol=1e-14)
    P = op_matrix(space3d.prolong, (3, 3, 3))
    R = op_matrix(space3d.restrict, (7, 7, 7))
    assert np.array_equal(P.T, R)


@pytest.mark.parametrize("K,a,sigma", [(2, 1.0, 0.0), (3, 1.0, 0.0), (3, 0.3, 16.0)])
def test_3d_multigrid_matches_dense_vcycle(K, a, sigma):
    from oracle import space3d

    n = 2 ** K - 1
    b = np.random.default_rng(K).standard_normal((n, n, n))
    got = space3d.mg_apply(b, K, a, sigma)
    ref = bf.dense_mg_3d(b.ravel(), K, a, sigma)
    assert np.allclose(got.ravel(), ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def test_3d_multigrid_symmetric_positive_definite():
    from oracle import space3d

    K = 2
    Kd = op_matrix(lambda b: space3d.mg_apply(b, K, 0.3, 4.0), (3, 3, 3))
    assert np.abs(Kd - Kd.T).max() <= 1e-13 * np.abs(Kd).max()
    assert np.linalg.eigvalsh(0.5 * (Kd + Kd.T)).min() > 0


def test_3d_S_lemma41_equals_lemma42():
    J, K = 1, 2
    P = Problem(J, K, dim=3)
    N = 2 ** J
    O, T, Nm = bf.legendre_test_space(N)
    A, M = bf.p1_assembly_3d(K)
    Kx = op_matrix(P.Kx, (P.n,) * 3)
    B = np.kron(T, M) + np.kron(Nm, A)
    G = np.zeros((N + 1, N + 1))
    G[0, 0] = 1.0
    S41 = B.T @ np.kron(np.diag(1.0 / O), Kx) @ B + np.kron(G, M)
    S42 = op_matrix(P.S, P.shape)
    assert np.abs(S42 - S41).max() <= 1e-12 * np.abs(S41).max()


def test_3d_pcg_matches_dense_solve():
    J, K = 2, 2
    P = Problem(J, K, dim=3)
    rng = np.random.default_rng(23)
    g = rng.standard_normal(P.shape)
    u0 = rng.standard_normal(P.shape[1:])
    S = op_matrix(P.S, P.shape)
    exact = np.linalg.solve(S, P.rhs(g, u0).ravel())
    u, its, _ = oracle.solve(J, K, g, u0, tol=1e-13, maxit=200, dim=3)
    assert np.linalg.norm(u.ravel() - exact) <= 1e-11 * np.linalg.norm(exact)


@pytest.mark.slow
def test_3d_converges_to_exact_solution():
    """Section 5.2's 3D solution exp(-3 pi^2 t) sin(pi x) sin(pi y) sin(pi z):
    the nodal error falls by more than 1.8 per joint refinement of h and tau."""
    errs = []
    for L in (2, 3, 4):
        s = _cube_sin(L)
        u, _, _ = oracle.solve(L, L, None, s, tol=1e-12, maxit=200, dim=3)
        t = np.arange(2 ** L + 1) / 2 ** L
        errs.append(np.abs(u - np.exp(-3 * np.pi ** 2 * t)[:, None, None, None] * s[None]).max())
    assert errs[0] / errs[1] >= 1.8 and errs[1] / errs[2] >= 1.8, errs
