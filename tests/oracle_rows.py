"""Sampled outputs of the oracle's operators, for checks at sizes where the
oracle cannot apply an operator to the whole space-time array in test time.

Each function returns selected time rows (or spatial columns) of an operator
output, computed from the oracle's own functions applied to just the data
that output depends on:

  * S (Lemma 4.2): row i depends on rows i - 1, i, i + 1 of X (three-point time
    matrices) and needs K_x on two rows;
  * f (Lemma 4.1): row i depends on rows i - 1, i, i + 1 of g;
  * K_x, K_X, A_x, M_x: row i depends on row i only;
  * W, W^T: act on every spatial node's time column separately.

The time matrices are three-point, so applying the oracle's time operators to
the rows ``max(0, i-1) .. min(N, i+1)`` gives row i exactly: the first and
last rows of such a slice are the true ends of the time interval exactly when
i = 0 or i = N.  ``tests/test_oracle_rows.py`` checks every function here
against the full oracle operator on small sizes.
"""
import numpy as np

from oracle import multigrid, temporal, wavelet
from oracle.schur import Problem


def _window(i, N):
    lo, hi = max(0, i - 1), min(N, i + 1)
    return lo, hi, i - lo


def _time_parts(P, X, i):
    """(A_t X)_i, (M_t X)_i, (L X)_i, (L^T X)_i."""
    lo, hi, k = _window(i, P.N)
    Xs = np.asarray(X[lo:hi + 1], dtype=np.float64)
    return (temporal.stiffness(Xs, P.tau)[k], temporal.mass(Xs, P.tau)[k],
            temporal.L(Xs)[k], temporal.LT(Xs)[k])


def S_rows(P: Problem, X, rows):
    out = []
    for i in rows:
        At, Mt, Lx, LTx = _time_parts(P, X, i)
        y = np.stack([P.M(At) + P.A(LTx), P.A(Mt) + P.M(Lx)])
        z = P.Kx(y)
        r = P.M(z[0]) + P.A(z[1])
        if i == 0:
            r = r + P.M(np.asarray(X[0], dtype=np.float64))
        out.append(r)
    return np.stack(out)


def rhs_rows(P: Problem, g_rows_of, u0, rows):
    """Rows of f; ``g_rows_of(lo, hi)`` returns g at time rows lo..hi (or None for g = 0)."""
    out = []
    for i in rows:
        lo, hi, k = _window(i, P.N)
        gs = g_rows_of(lo, hi)
        if gs is None:
            r = np.zeros_like(u0, dtype=np.float64)
        else:
            G0 = P.M(temporal.mass(gs, P.tau)[k])
            G1 = P.M(temporal.LT(gs)[k])
            z = P.Kx(np.stack([G1, G0]))
            r = P.M(z[0]) + P.A(z[1])
        if i == 0:
            r = r + P.M(u0)
        out.append(r)
    return np.stack(out)


def Kx_rows(P: Problem, X, rows):
    return P.Kx(np.asarray(X[list(rows)], dtype=np.float64))


def KX_rows(P: Problem, R, rows):
    rows = list(rows)
    sigma = 2.0 ** wavelet.row_levels(P.J)[rows].astype(np.float64)
    Z = multigrid.apply(np.asarray(R[rows], dtype=np.float64), P.K, P.alpha, sigma, P.cycles,
                        P.sweeps, P.D, P.c)
    return multigrid.apply(P.A(Z), P.K, P.alpha, sigma, P.cycles, P.sweeps, P.D, P.c)


def KX_first_factor(P: Problem, R, rows):
    """y = K_l r on the sampled rows (the first factor of K_X = K_l A K_l)."""
    rows = list(rows)
    sigma = 2.0 ** wavelet.row_levels(P.J)[rows].astype(np.float64)
    return multigrid.apply(np.asarray(R[rows], dtype=np.float64), P.K, P.alpha, sigma, P.cycles,
                           P.sweeps, P.D, P.c)


def W_columns(P: Problem, X, nodes):
    """Columns (time vectors) of W X at flat spatial nodes ``nodes``."""
    cols = np.asarray(X).reshape(P.N + 1, -1)[:, nodes]
    return wavelet.synthesis(cols, P.J)


def WT_columns(P: Problem, X, nodes):
    cols = np.asarray(X).reshape(P.N + 1, -1)[:, nodes]
    return wavelet.analysis(cols, P.J)
