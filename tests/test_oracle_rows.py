"""The sampled-output helpers of tests/oracle_rows.py equal the full oracle
operators (CPU, small sizes)."""
import numpy as np
import pytest

import synth
from oracle.schur import Problem
from tests import oracle_rows as orow


@pytest.mark.parametrize("J,K", [(1, 2), (3, 4), (4, 3)])
def test_row_helpers_match_full_operators(J, K):
    P = Problem(J, K)
    X = synth.random_field(P.shape, 5)
    N = P.N
    rows = sorted({0, 1, N // 2, N - 1, N})
    assert np.allclose(orow.S_rows(P, X, rows), P.S(X)[rows], rtol=0, atol=1e-13 * np.abs(P.S(X)).max())
    assert np.allclose(orow.Kx_rows(P, X, rows), P.Kx(X)[rows], rtol=0, atol=1e-14 * np.abs(X).max())
    KX = P.KX(X)
    assert np.allclose(orow.KX_rows(P, X, rows), KX[rows], rtol=0, atol=1e-13 * np.abs(KX).max())
    nodes = [0, 3, P.n * P.n - 1]
    W = P.W(X).reshape(N + 1, -1)[:, nodes]
    WT = P.WT(X).reshape(N + 1, -1)[:, nodes]
    assert np.allclose(orow.W_columns(P, X, nodes), W, rtol=0, atol=1e-13 * np.abs(W).max())
    assert np.allclose(orow.WT_columns(P, X, nodes), WT, rtol=0, atol=1e-13 * np.abs(WT).max())
    g = synth.fourier_g(J, K, 3)
    u0 = synth.smooth_u0(K, 3)
    f = P.rhs(g, u0)
    fr = orow.rhs_rows(P, lambda lo, hi: g[lo:hi + 1], u0, rows)
    assert np.allclose(fr, f[rows], rtol=0, atol=1e-13 * np.abs(f).max())
    f0 = P.rhs(None, u0)
    fr0 = orow.rhs_rows(P, lambda lo, hi: None, u0, rows)
    assert np.allclose(fr0, f0[rows], rtol=0, atol=1e-15 * max(np.abs(f0).max(), 1e-300))
