"""The three-dimensional spatial discretisation (oracle; test infrastructure).

Section 5.2's 3D problem takes Omega = [0, 1]^3 with a uniform tetrahedral
mesh.  The paper does not say how the cubes are cut; the reading taken here
is the Kuhn (Freudenthal) subdivision: each of the ``2**K`` per side cubes is
split into the 6 tetrahedra ``{0, e_p1, e_p1 + e_p2, e_1 + e_2 + e_3}`` (in
units of h, from the cube's lower corner) for the 6 permutations p of the
axes.  Every edge of this mesh runs along one of the 7 directions e_1, e_2,
e_3, e_1 + e_2, e_1 + e_3, e_2 + e_3, e_1 + e_2 + e_3, so a node couples to at
most 14 neighbours.

The stencils are written out from their definition: the P1 element matrices
of the 6 tetrahedra of one cube (gradients of the barycentric coordinates;
the mass matrix ``vol / 20 (1 + delta_ij)``) are summed over the 8 cubes that
share a node.  Interior nodal arrays have shape ``(..., n, n, n)`` indexed
``[..., k, j, i]`` (z slowest, x fastest), ``n = 2**K - 1``; the flat index of
node (i, j, k) is ``((k - 1) n + (j - 1)) n + (i - 1)``.

Multigrid (``K_x`` and the ``K_l`` of Theorem 3.1, as in 2D with Section
5.1's 2 V-cycles and 3 Gauss-Seidel steps per grid): Gauss-Seidel in four
colours ``(i + j + k) mod 4`` (the 7 edge directions change ``i + j + k`` by 1,
2 or 3, so nodes of one colour are never coupled), forward 0, 1, 2, 3 before
the coarse grid and backward 3, 2, 1, 0 after it; P1 interpolation and its
transpose between levels; the one-node grid solved exactly.
"""
from __future__ import annotations

import itertools

import numpy as np

DIRS = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, 0, 1), (0, 1, 1), (1, 1, 1)]


def _cube_tets():
    """The 6 Kuhn tetrahedra of the unit cube, as lists of 4 corner offsets."""
    tets = []
    for p in itertools.permutations(range(3)):
        v = [np.zeros(3, dtype=int)]
        for ax in p:
            w = v[-1].copy()
            w[ax] += 1
            v.append(w)
        tets.append([tuple(int(c) for c in x) for x in v])
    return tets


def _element_stencils():
    """Stiffness (per unit h) and mass (per unit h^3) couplings of a node with
    the offsets d in {-1, 0, 1}^3, summed over the 6 tetrahedra of each of the
    8 cubes around the node: dicts offset -> value."""
    A, M = {}, {}
    for tet in _cube_tets():
        P = np.array([[1.0, *v] for v in tet])
        vol = abs(np.linalg.det(P)) / 6.0
        G = np.linalg.inv(P)[1:, :]             # gradients of the barycentric coordinates
        Kloc = vol * G.T @ G                    # times h^(3-2) on a cube of side h
        Mloc = vol / 20.0 * (np.ones((4, 4)) + np.eye(4))
        # the node sits at corner a of a cube; its neighbour at corner b
        for a in range(4):
            for b in range(4):
                d = tuple(tet[b][t] - tet[a][t] for t in range(3))
                A[d] = A.get(d, 0.0) + Kloc[a, b]
                M[d] = M.get(d, 0.0) + Mloc[a, b]
    return A, M


_A, _M = _element_stencils()


def stencils():
    """(stiffness, mass) couplings by offset: A in units of h, M in units of h^3."""
    return dict(_A), dict(_M)


def _padded(x):
    shape = x.shape[:-3] + tuple(s + 2 for s in x.shape[-3:])
    xp = np.zeros(shape, dtype=x.dtype)
    xp[..., 1:-1, 1:-1, 1:-1] = x
    return xp


def _shift(xp, d):
    """Values at node + d (d = (di, dj, dk)) of the padded array's interior."""
    di, dj, dk = d
    n = xp.shape[-1] - 2
    return xp[..., 1 + dk:1 + dk + n, 1 + dj:1 + dj + n, 1 + di:1 + di + n]


def apply_stencil(x, st, scale):
    xp = _padded(x)
    out = np.zeros_like(x)
    for d in sorted(st):
        if st[d] != 0.0:
            out += st[d] * _shift(xp, d)
    return scale * out


def stiffness(x, h):
    """``A_x x``: P1 stiffness on the Kuhn mesh of width h (proportional to h)."""
    return apply_stencil(x, _A, h)


def mass(x, h):
    """``M_x x``: P1 mass on the Kuhn mesh of width h (proportional to h^3)."""
    return apply_stencil(x, _M, h ** 3)


def colour_masks(n):
    k, j, i = np.meshgrid(np.arange(1, n + 1), np.arange(1, n + 1), np.arange(1, n + 1),
                          indexing="ij")
    c = (i + j + k) % 4
    return [c == q for q in range(4)]


def apply_C(x, a, sigma, h):
    return a * stiffness(x, h) + sigma * mass(x, h)


def relax_colour(x, b, a, sigma, h, mask):
    """Every node of one colour set to (b - sum_nb C_nb x_nb) / C_centre."""
    xp = _padded(x)
    off = np.zeros_like(x)
    for d in sorted(_M):
        if d == (0, 0, 0):
            continue
        cd = a * h * _A.get(d, 0.0) + sigma * h ** 3 * _M[d]
        off = off + cd * _shift(xp, d)
    c0 = a * h * _A[(0, 0, 0)] + sigma * h ** 3 * _M[(0, 0, 0)]
    return np.where(mask, (b - off) / c0, x)


def prolong(e):
    """P1 interpolation from the coarse grid (m^3 interior nodes) to the fine
    one ((2m + 1)^3): fine node (2I + a, 2J + b, 2K + c) with (a, b, c) in
    {0, 1}^3 is the mean of coarse nodes (I, J, K) and (I + a, J + b, K + c),
    the ends of the coarse edge it bisects (the node itself when (a, b, c) = 0)."""
    m = e.shape[-1]
    nf = 2 * m + 1
    ep = _padded(e)   # coarse node (I, J, K), 0..m+1
    out = np.zeros(e.shape[:-3] + (nf + 2,) * 3)
    for a in (0, 1):
        for b in (0, 1):
            for c in (0, 1):
                lo = ep[..., 0:m + 2 - c, 0:m + 2 - b, 0:m + 2 - a]
                hi = ep[..., c:m + 2, b:m + 2, a:m + 2]
                out[..., c::2, b::2, a::2] = lo if (a, b, c) == (0, 0, 0) else 0.5 * (lo + hi)
    return out[..., 1:-1, 1:-1, 1:-1]


def restrict(r):
    """P^T r: the transpose of :func:`prolong`."""
    nf = r.shape[-1]
    m = (nf - 1) // 2
    rp = _padded(r)   # fine node (i, j, k), 0..nf+1
    I = 2 * np.arange(1, m + 1)
    out = rp[..., I[:, None, None], I[None, :, None], I[None, None, :]].copy()
    for d in DIRS:
        for s in (1, -1):
            di, dj, dk = (s * d[0], s * d[1], s * d[2])
            out += 0.5 * rp[..., (I + dk)[:, None, None], (I + dj)[None, :, None],
                            (I + di)[None, None, :]]
    return out


def vcycle(level, b, x, a, sigma, sweeps=3):
    h = 2.0 ** -level
    if level == 1:
        c0 = a * h * _A[(0, 0, 0)] + sigma * h ** 3 * _M[(0, 0, 0)]
        return b / c0
    masks = colour_masks(b.shape[-1])
    for _ in range(sweeps):
        for q in (0, 1, 2, 3):
            x = relax_colour(x, b, a, sigma, h, masks[q])
    r = b - apply_C(x, a, sigma, h)
    ec = vcycle(level - 1, restrict(r), np.zeros(b.shape[:-3] + ((b.shape[-1] - 1) // 2,) * 3),
                a, sigma, sweeps)
    x = x + prolong(ec)
    for _ in range(sweeps):
        for q in (3, 2, 1, 0):
            x = relax_colour(x, b, a, sigma, h, masks[q])
    return x


def mg_apply(b, K, a=1.0, sigma=0.0, cycles=2, sweeps=3):
    """``cycles`` V-cycles from zero for (a A_x + sigma M_x) x = b on level K;
    a and sigma broadcast against b[..., 0, 0, 0]."""
    a = np.asarray(a, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    if a.ndim:
        a = a[..., None, None, None]
    if sigma.ndim:
        sigma = sigma[..., None, None, None]
    x = np.zeros_like(b)
    for _ in range(cycles):
        x = vcycle(K, b, x, a, sigma, sweeps)
    return x
