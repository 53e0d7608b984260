"""Independent dense brute-force constructions used to pin the oracle.

Nothing here imports the oracle.  Every matrix is built from first
principles: finite-element assembly triangle by triangle, basis functions
evaluated pointwise, Gauss quadrature, and a dense recursive multigrid
written from explicit matrices.
"""
from __future__ import annotations

import numpy as np

# ---------------------------------------------------------------- quadrature

_GX, _GW = np.polynomial.legendre.leggauss(8)


def gauss_interval(f, a, b):
    """8-point Gauss-Legendre rule on [a, b] (exact for degree <= 15)."""
    x = 0.5 * (b - a) * _GX + 0.5 * (a + b)
    return 0.5 * (b - a) * np.sum(_GW * f(x))


def triangle_rule(order=12):
    """Collapsed Gauss rule on the reference triangle {(r, s): r, s >= 0, r + s <= 1}."""
    x, w = np.polynomial.legendre.leggauss(order)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    r = x[:, None] * np.ones_like(x)[None, :]
    s = (1.0 - x[:, None]) * x[None, :]
    ww = w[:, None] * w[None, :] * (1.0 - x[:, None])
    return r.ravel(), s.ravel(), ww.ravel()


# ------------------------------------------------------------ time, 1D hats

def hat(t, k, width):
    """Hat function of node ``k * width`` on a uniform mesh of width ``width``."""
    return np.maximum(0.0, 1.0 - np.abs(t / width - k))


def hat_dt(t, k, width):
    u = t / width - k
    return np.where((u > -1) & (u < 0), 1.0 / width, np.where((u > 0) & (u < 1), -1.0 / width, 0.0))


def temporal_by_quadrature(N):
    """``A_t, M_t, L`` (with ``L[i, j] = int phi_i phi_j'``) by quadrature on each interval."""
    tau = 1.0 / N
    At = np.zeros((N + 1, N + 1))
    Mt = np.zeros((N + 1, N + 1))
    L = np.zeros((N + 1, N + 1))
    for e in range(N):
        a, b = e * tau, (e + 1) * tau
        for i in (e, e + 1):
            for j in (e, e + 1):
                # derivatives are constant on the open interval: evaluate inside
                At[i, j] += gauss_interval(lambda t: hat_dt(t, i, tau) * hat_dt(t, j, tau), a, b)
                Mt[i, j] += gauss_interval(lambda t: hat(t, i, tau) * hat(t, j, tau), a, b)
                L[i, j] += gauss_interval(lambda t: hat(t, i, tau) * hat_dt(t, j, tau), a, b)
    return At, Mt, L


def legendre_test_space(N):
    """Two shifted Legendre polynomials per interval (an orthogonal basis of the
    discontinuous piecewise linears ``Y_t``): returns ``(O, T, Nm)`` with
    ``O = <Xi, Xi>`` (diagonal), ``T[(e,p), j] = int phi_j' xi_{e,p}`` and
    ``Nm[(e,p), j] = int phi_j xi_{e,p}``."""
    tau = 1.0 / N
    O = np.zeros(2 * N)
    T = np.zeros((2 * N, N + 1))
    Nm = np.zeros((2 * N, N + 1))
    for e in range(N):
        a, b = e * tau, (e + 1) * tau
        xis = [lambda t: np.ones_like(t), lambda t, a=a: 2.0 * (t - a) / tau - 1.0]
        for p, xi in enumerate(xis):
            O[2 * e + p] = gauss_interval(lambda t: xi(t) ** 2, a, b)
            for j in (e, e + 1):
                T[2 * e + p, j] = gauss_interval(lambda t: hat_dt(t, j, tau) * xi(t), a, b)
                Nm[2 * e + p, j] = gauss_interval(lambda t: hat(t, j, tau) * xi(t), a, b)
    return O, T, Nm


# ------------------------------------------------------------ space, P1 FEM

def p1_assembly(K, D=None):
    """Stiffness (``int D grad u . grad v``, D = (dxx, dyy, dxy), None =
    identity) and mass of P1 on the ``2**K x 2**K`` square mesh cut by "/"
    diagonals, assembled element by element; rows/columns are the interior
    nodes in order ``(j - 1) n + (i - 1)``."""
    Dm = np.eye(2) if D is None else np.array([[D[0], D[2]], [D[2], D[1]]])
    m = 2 ** K
    h = 1.0 / m
    nn = m + 1
    Afull = np.zeros((nn * nn, nn * nn))
    Mfull = np.zeros((nn * nn, nn * nn))

    def gid(i, j):
        return j * nn + i

    Mloc_ref = np.array([[2.0, 1.0, 1.0], [1.0, 2.0, 1.0], [1.0, 1.0, 2.0]]) / 12.0
    for j in range(m):
        for i in range(m):
            for tri in (((i, j), (i + 1, j), (i + 1, j + 1)), ((i, j), (i + 1, j + 1), (i, j + 1))):
                P = np.array([[1.0, a * h, b * h] for a, b in tri])
                area = 0.5 * abs(np.linalg.det(P))
                G = np.linalg.inv(P)[1:, :]  # gradients of barycentric coordinates
                Kloc = area * G.T @ Dm @ G
                Mloc = area * Mloc_ref
                ids = [gid(a, b) for a, b in tri]
                for r in range(3):
                    for c in range(3):
                        Afull[ids[r], ids[c]] += Kloc[r, c]
                        Mfull[ids[r], ids[c]] += Mloc[r, c]
    interior = [gid(i, j) for j in range(1, m) for i in range(1, m)]
    ix = np.ix_(interior, interior)
    return Afull[ix], Mfull[ix]


def slash_hat(x, y, X0, Y0, H):
    """Hat function of node (X0, Y0) on the "/"-diagonal mesh of width H."""
    u = (x - X0) / H
    v = (y - Y0) / H
    return np.maximum(0.0, 1.0 - np.maximum(np.maximum(np.abs(u), np.abs(v)), np.abs(u - v)))


def prolongation_by_evaluation(Kf):
    """``P``: coarse hats (level Kf - 1) evaluated at the fine interior nodes."""
    nf = 2 ** Kf - 1
    nc = 2 ** (Kf - 1) - 1
    hf = 2.0 ** -Kf
    hc = 2.0 ** -(Kf - 1)
    P = np.zeros((nf * nf, nc * nc))
    fx = np.array([(i + 1) * hf for j in range(nf) for i in range(nf)])
    fy = np.array([(j + 1) * hf for j in range(nf) for i in range(nf)])
    for J in range(nc):
        for I in range(nc):
            P[:, J * nc + I] = slash_hat(fx, fy, (I + 1) * hc, (J + 1) * hc, hc)
    return P


def colour_of_nodes(K):
    n = 2 ** K - 1
    return np.array([((i + 1) + (j + 1)) % 3 for j in range(n) for i in range(n)])


def dense_vcycle_matrix_apply(b, x, K, a, sigma, ops, sweeps=3, react=0.0):
    """One V-cycle written with dense matrices for ``a (A + c M) + sigma M``:
    Gauss-Seidel as a sequential node-by-node loop visiting the colours in
    turn, explicit residual, ``P^T`` and ``P``."""
    A, M = ops[K]
    C = a * (A + react * M) + sigma * M
    if K == 1:
        return b / C[0, 0]
    col = colour_of_nodes(K)
    x = x.copy()
    order_f = [0, 1, 2]
    for _ in range(sweeps):
        for c in order_f:
            idx = np.nonzero(col == c)[0]
            for p in idx:  # plain sequential Gauss-Seidel, node by node
                x[p] = (b[p] - (C[p] @ x - C[p, p] * x[p])) / C[p, p]
    P = ops[("P", K)]
    bc = P.T @ (b - C @ x)
    ec = dense_vcycle_matrix_apply(bc, np.zeros_like(bc), K - 1, a, sigma, ops, sweeps, react)
    x = x + P @ ec
    for _ in range(sweeps):
        for c in order_f[::-1]:
            idx = np.nonzero(col == c)[0]
            for p in idx:
                x[p] = (b[p] - (C[p] @ x - C[p, p] * x[p])) / C[p, p]
    return x


def mg_ops(K, D=None):
    ops = {}
    for k in range(1, K + 1):
        ops[k] = p1_assembly(k, D)
        if k > 1:
            ops[("P", k)] = prolongation_by_evaluation(k)
    return ops


def dense_mg(b, K, a, sigma, cycles=2, sweeps=3, ops=None, D=None, c=0.0):
    ops = ops or mg_ops(K, D)
    x = np.zeros_like(b)
    for _ in range(cycles):
        x = dense_vcycle_matrix_apply(b, x, K, a, sigma, ops, sweeps, c)
    return x


def dense_mg_matrix(K, a, sigma, cycles=2, sweeps=3, D=None, c=0.0):
    ops = mg_ops(K, D)
    n2 = (2 ** K - 1) ** 2
    return np.stack([dense_mg(e, K, a, sigma, cycles, sweeps, ops, D, c) for e in np.eye(n2)], 1)


# ------------------------------------------------------- wavelet by evaluation

def wavelet_basis_matrix(J):
    """Columns: nodal values at ``t_i = i / 2**J`` of the basis functions, in the
    in-place order (level-0 hats at rows 0 and N, psi_{l,k} at row
    ``(2k+1) 2**(J-l)``), each evaluated directly from its definition."""
    N = 2 ** J
    t = np.arange(N + 1) / N
    W = np.zeros((N + 1, N + 1))
    W[:, 0] = 1.0 - t
    W[:, N] = t
    for l in range(1, J + 1):
        hl = 2.0 ** -l
        for k in range(2 ** (l - 1)):
            left, right = 2 * k, 2 * k + 2
            bl = 1.0 if left == 0 else 0.5
            br = 1.0 if right == 2 ** l else 0.5
            psi = hat(t, 2 * k + 1, hl) - bl * hat(t, left, hl) - br * hat(t, right, hl)
            W[:, (2 * k + 1) * 2 ** (J - l)] = 2.0 ** (l / 2.0) * psi
    return W


# ------------------------------------------------------------ space, 3D (Kuhn mesh)

def kuhn_tets_of_cube():
    """The 6 tetrahedra of the unit cube around its (1, 1, 1) diagonal: for each
    ordering of the axes, the path 0 -> e_a -> e_a + e_b -> (1, 1, 1)."""
    import itertools

    tets = []
    for p in itertools.permutations(range(3)):
        v = [(0, 0, 0)]
        for ax in p:
            w = list(v[-1])
            w[ax] += 1
            v.append(tuple(w))
        tets.append(v)
    return tets


def p1_assembly_3d(K):
    """Stiffness and mass of P1 on the Kuhn mesh of the unit cube with 2**K
    cubes per side, assembled element by element over all tetrahedra; rows
    are the interior nodes in order ((k - 1) n + (j - 1)) n + (i - 1)."""
    m = 2 ** K
    h = 1.0 / m
    nn = m + 1

    def gid(i, j, k):
        return (k * nn + j) * nn + i

    A = np.zeros((nn ** 3, nn ** 3))
    M = np.zeros((nn ** 3, nn ** 3))
    tets = kuhn_tets_of_cube()
    for k in range(m):
        for j in range(m):
            for i in range(m):
                for tet in tets:
                    pts = [(i + a, j + b, k + c) for a, b, c in tet]
                    P = np.array([[1.0, a * h, b * h, c * h] for a, b, c in pts])
                    vol = abs(np.linalg.det(P)) / 6.0
                    G = np.linalg.inv(P)[1:, :]
                    Kl = vol * G.T @ G
                    Ml = vol / 20.0 * (np.ones((4, 4)) + np.eye(4))
                    ids = [gid(*q) for q in pts]
                    for r in range(4):
                        for s in range(4):
                            A[ids[r], ids[s]] += Kl[r, s]
                            M[ids[r], ids[s]] += Ml[r, s]
    interior = [gid(i, j, k) for k in range(1, m) for j in range(1, m) for i in range(1, m)]
    ix = np.ix_(interior, interior)
    return A[ix], M[ix]


def kuhn_eval(values, K, pts):
    """The P1 function with interior nodal values ``values`` ((n, n, n),
    zero on the boundary) of the Kuhn mesh with 2**K cubes per side,
    evaluated at points pts (rows x, y, z in [0, 1]) by locating the cube and
    its tetrahedron (sort the local coordinates) and using barycentric
    coordinates."""
    m = 2 ** K
    full = np.zeros((m + 1,) * 3)
    full[1:-1, 1:-1, 1:-1] = values      # [k, j, i]
    out = np.zeros(len(pts))
    for t, p in enumerate(pts):
        q = np.asarray(p) * m
        c = np.minimum(np.floor(q).astype(int), m - 1)
        u = q - c
        order = np.argsort(-u, kind="stable")
        lam = [1.0 - u[order[0]], u[order[0]] - u[order[1]], u[order[1]] - u[order[2]], u[order[2]]]
        v = np.zeros(3, dtype=int)
        val = lam[0] * full[c[2], c[1], c[0]]
        for r in range(3):
            v[order[r]] += 1
            val += lam[r + 1] * full[c[2] + v[2], c[1] + v[1], c[0] + v[0]]
        out[t] = val
    return out


def dense_mg_3d(b, K, a, sigma, cycles=2, sweeps=3):
    """Two V-cycles written with dense matrices: Gauss-Seidel node by node in the
    colours (i + j + k) mod 4 (forward 0..3 before, backward 3..0 after the
    coarse grid), P by evaluating coarse functions at the fine nodes."""
    ops = {k: p1_assembly_3d(k) for k in range(1, K + 1)}

    def colours(k):
        n = 2 ** k - 1
        return np.array([(i + 1 + j + 1 + l + 1) % 4 for l in range(n) for j in range(n)
                         for i in range(n)])

    def prol(k):
        nf, nc = 2 ** k - 1, 2 ** (k - 1) - 1
        pts = [((i + 1) / 2 ** k, (j + 1) / 2 ** k, (l + 1) / 2 ** k)
               for l in range(nf) for j in range(nf) for i in range(nf)]
        P = np.zeros((nf ** 3, nc ** 3))
        for col in range(nc ** 3):
            e = np.zeros(nc ** 3)
            e[col] = 1.0
            P[:, col] = kuhn_eval(e.reshape(nc, nc, nc), k - 1, pts)
        return P

    Ps = {k: prol(k) for k in range(2, K + 1)}

    def cycle(b, x, k):
        A, M = ops[k]
        C = a * A + sigma * M
        if k == 1:
            return b / C[0, 0]
        col = colours(k)
        x = x.copy()
        for _ in range(sweeps):
            for c in range(4):
                for p in np.nonzero(col == c)[0]:
                    x[p] = (b[p] - (C[p] @ x - C[p, p] * x[p])) / C[p, p]
        P = Ps[k]
        ec = cycle(P.T @ (b - C @ x), np.zeros(P.shape[1]), k - 1)
        x = x + P @ ec
        for _ in range(sweeps):
            for c in (3, 2, 1, 0):
                for p in np.nonzero(col == c)[0]:
                    x[p] = (b[p] - (C[p] @ x - C[p, p] * x[p])) / C[p, p]
        return x

    x = np.zeros_like(b)
    for _ in range(cycles):
        x = cycle(b, x, K)
    return x
