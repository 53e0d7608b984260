"""Seeded synthetic inputs for the space-time heat-equation solver.

This module only draws random numbers and samples smooth functions at mesh
nodes.  It holds none of the solver's arithmetic, and it is the one module
that both the CPU oracle and the GPU path's tests and benchmark read their
inputs from.

Geometry (Section 5 of the paper, uniform meshes):
  * time: ``N = 2**J`` uniform intervals on ``I = (0, 1)``, nodes
    ``t_i = i / N`` for ``i = 0..N``;
  * space: the unit square with ``2**K`` cells per side, interior nodes
    ``(x_i, y_j) = (i h, j h)`` for ``1 <= i, j <= n``, ``n = 2**K - 1``,
    ``h = 2**-K``.

Arrays are time-major: a space-time array has shape ``(N + 1, n, n)`` and is
indexed ``[t, j, i]`` (``j`` along ``y``, slow; ``i`` along ``x``, fast), so
the flat spatial index of node ``(x_i, y_j)`` is ``(j - 1) n + (i - 1)``.
"""
from __future__ import annotations

import numpy as np

KMAX = 8  # highest Fourier mode index in each direction


def nodes_1d(K: int) -> np.ndarray:
    """Interior node coordinates ``h, 2h, ..., n h`` of one side."""
    n = 2 ** K - 1
    return np.arange(1, n + 1, dtype=np.float64) / 2.0 ** K


def time_nodes(J: int) -> np.ndarray:
    return np.arange(0, 2 ** J + 1, dtype=np.float64) / 2.0 ** J


def sine_product(K: int, k: int = 1, l: int = 1) -> np.ndarray:
    """Nodal values of ``sin(k pi x) sin(l pi y)`` on the interior nodes, shape (n, n)."""
    x = nodes_1d(K)
    return np.outer(np.sin(l * np.pi * x), np.sin(k * np.pi * x))


def sine_product_3d(K: int) -> np.ndarray:
    """Nodal values of ``sin(pi x) sin(pi y) sin(pi z)`` on the interior nodes of
    the unit cube, shape (n, n, n) indexed [k, j, i] (z slowest)."""
    s = np.sin(np.pi * nodes_1d(K))
    return np.einsum("i,j,k->kji", s, s, s)


def fourier_coefficients(seed: int, kmax: int = KMAX) -> np.ndarray:
    """Coefficients ``c[k-1, l-1, m]`` of the forcing
    ``g = sum c_klm sin(k pi x) sin(l pi y) cos(m pi t)``,
    ``k, l = 1..kmax``, ``m = 0..kmax``, each ``N(0,1) / (k^2 + l^2 + m^2)``,
    drawn from ``numpy.random.default_rng(seed)`` in lexicographic
    ``(k, l, m)`` order."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(kmax * kmax * (kmax + 1)).reshape(kmax, kmax, kmax + 1)
    k = np.arange(1, kmax + 1, dtype=np.float64)[:, None, None]
    l = np.arange(1, kmax + 1, dtype=np.float64)[None, :, None]
    m = np.arange(0, kmax + 1, dtype=np.float64)[None, None, :]
    return z / (k * k + l * l + m * m)


def fourier_g(J: int, K: int, seed: int, kmax: int = KMAX, rows=None) -> np.ndarray:
    """Nodal forcing ``g`` of shape ``(len(rows), n, n)`` (all ``N + 1`` time
    nodes when ``rows`` is None)."""
    c = fourier_coefficients(seed, kmax)
    x = nodes_1d(K)
    t = time_nodes(J)
    if rows is not None:
        t = t[np.asarray(rows)]
    kk = np.arange(1, kmax + 1)
    mm = np.arange(0, kmax + 1)
    sx = np.sin(np.pi * np.outer(kk, x))          # (k, i)
    sy = np.sin(np.pi * np.outer(kk, x))          # (l, j)
    ct = np.cos(np.pi * np.outer(t, mm))          # (t, m)
    tmp = np.einsum("klm,tm->tkl", c, ct)         # (t, k, l)
    tmp = np.einsum("tkl,lj->tkj", tmp, sy)       # (t, k, j)
    return np.einsum("tkj,ki->tji", tmp, sx)      # (t, j, i)


def fourier_g_torch(J: int, K: int, seed: int, device, kmax: int = KMAX,
                    dtype=None, out=None):
    """Same samples as :func:`fourier_g`, evaluated with torch on ``device``
    (used to fill large device-resident inputs without a host copy)."""
    import torch

    dtype = dtype or torch.float64
    c = torch.as_tensor(fourier_coefficients(seed, kmax), dtype=torch.float64, device=device)
    x = torch.as_tensor(nodes_1d(K), device=device)
    t = torch.as_tensor(time_nodes(J), device=device)
    kk = torch.arange(1, kmax + 1, device=device, dtype=torch.float64)
    mm = torch.arange(0, kmax + 1, device=device, dtype=torch.float64)
    sx = torch.sin(torch.pi * torch.outer(kk, x))
    ct = torch.cos(torch.pi * torch.outer(t, mm))
    n = x.numel()
    # (k, l, m) x (m, t) -> (k, l, t); then per t: sy^T (l,j) . (k,l)^T . sx (k,i)
    ckl_t = torch.einsum("klm,tm->tkl", c, ct)               # (t, k, l)
    left = torch.matmul(ckl_t.transpose(1, 2).contiguous(), sx)  # (t, l, i)
    if out is None:
        out = torch.empty((t.numel(), n, n), dtype=dtype, device=device)
    syt = sx.t().contiguous()                                 # (j, l)
    chunk = 64
    for s in range(0, t.numel(), chunk):
        e = min(s + chunk, t.numel())
        out[s:e] = torch.matmul(syt, left[s:e]).to(dtype)     # (j, l) x (l, i)
    return out


def smooth_u0(K: int, seed: int, nmodes: int = 4, kmax: int = 4) -> np.ndarray:
    """Random smooth initial value: ``sum_q a_q sin(k_q pi x) sin(l_q pi y)``
    with ``(k_q, l_q)`` drawn without replacement from ``{1..kmax}^2`` and
    ``a_q ~ N(0,1) / (k_q^2 + l_q^2)``."""
    rng = np.random.default_rng(seed)
    pick = rng.choice(kmax * kmax, size=nmodes, replace=False)
    amp = rng.standard_normal(nmodes)
    u0 = np.zeros((2 ** K - 1, 2 ** K - 1))
    for q in range(nmodes):
        k = int(pick[q]) // kmax + 1
        l = int(pick[q]) % kmax + 1
        u0 += amp[q] / (k * k + l * l) * sine_product(K, k, l)
    return u0


def random_field(shape, seed: int) -> np.ndarray:
    """Standard-normal array, for operator-level parity cases."""
    return np.random.default_rng(seed).standard_normal(shape)


# Named workloads: (J, K, nrhs) and how their data is drawn.
WORKLOADS = {
    "heat2d_J4_K4": dict(J=4, K=4, nrhs=1, g_seed=None, u0="sin"),
    "heat2d_J10_K9": dict(J=10, K=9, nrhs=1, g_seed=2, u0="sin"),
    "heat2d_J12_K9": dict(J=12, K=9, nrhs=1, g_seed=2, u0="sin"),
    "heat2d_J8_K7_B64": dict(J=8, K=7, nrhs=64, g_seed=1000, u0="random4"),
}


def serving_stream(n: int, seed: int = 12345, J_range=(6, 11), K_range=(5, 9),
                   log10_tol_range=(-10.0, -6.0)):
    """A stream of ``n`` solve requests of uneven sizes: ``J`` and ``K``
    uniform over their ranges (so ``N_t`` and ``h`` are log-uniform),
    ``tol = 10**U(log10_tol_range)``, and for each request a data seed
    ``50000 + index`` (forcing from :func:`fourier_g`, initial value from
    :func:`smooth_u0`).  Also returns unit-rate exponential inter-arrival gaps;
    divide them by the arrival rate to get a Poisson process."""
    rng = np.random.default_rng(seed)
    J = rng.integers(J_range[0], J_range[1] + 1, size=n)
    K = rng.integers(K_range[0], K_range[1] + 1, size=n)
    tol = 10.0 ** rng.uniform(log10_tol_range[0], log10_tol_range[1], size=n)
    gaps = rng.exponential(1.0, size=n)
    return [dict(J=int(J[i]), K=int(K[i]), tol=float(tol[i]), seed=50000 + i, gap=float(gaps[i]))
            for i in range(n)]
