"""Edge sizes through the C-ABI: the longest time axis (J = 14, the largest J
the library accepts: 16385 time rows, 14 wavelet levels) on a small mesh, the
finest mesh (K = 10: 1023 x 1023 nodes, 10 multigrid levels) on a short time
axis, and a context larger than the device.

Operators are compared with the oracle on sampled time rows or spatial
columns (tests/oracle_rows.py) with the tolerances of the small-size parity
tests (K_X: the mesh-dependent bound explained in test_gpu_fullsize.py);
solves are checked through the residual f - S u on sampled rows (bound 1e-6
of f, as in test_gpu_fullsize.py).
"""
import sys

import numpy as np
import pytest

import synth
from oracle.schur import Problem
from tests import oracle_rows as orow

pytestmark = pytest.mark.gpu

CASES = [(14, 4), (2, 10)]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def stp():
    import paper_2009_08875_amd as lib

    return lib


def _rows(N):
    return sorted({0, 1, N // 4, N // 2, N // 2 + 1, N - 1, N})


def _nodes(n):
    return sorted({0, 1, n - 1, n * (n // 2) + n // 2, n * n - 1})


@pytest.mark.parametrize("J,K", CASES)
@pytest.mark.parametrize("opname", ["S", "KX", "W", "WT"])
def test_operator_extreme_sizes(stp, J, K, opname):
    say(f"extreme size J={J} K={K}: {opname}")
    P = Problem(J, K)
    X = synth.random_field(P.shape, 91)
    out = np.zeros(X.size)
    ctx = stp.stp_create(J, K, 1, stp.STP_FP64)
    try:
        stp.stp_apply(ctx, getattr(stp, "STP_OP_" + opname), stp.STP_FP64, 0, X.reshape(-1), out)
    finally:
        stp.stp_destroy(ctx)
    out = out.reshape(P.shape)
    rows, nodes = _rows(P.N), _nodes(P.n)
    tol = 1e-12
    if opname == "S":
        ref, got = orow.S_rows(P, X, rows), out[rows]
    elif opname == "KX":
        ref, got = orow.KX_rows(P, X, rows), out[rows]
        y = orow.KX_first_factor(P, X, rows)
        tol = max(tol, 500 * np.finfo(np.float64).eps / 2 * 8 * np.abs(y).max() / np.abs(P.A(y)).max())
    else:
        fn = orow.W_columns if opname == "W" else orow.WT_columns
        ref, got = fn(P, X, nodes), out.reshape(P.N + 1, -1)[:, nodes]
    err = float(np.abs(got - ref).max() / np.abs(ref).max())
    say(f"  max rel error {err:.2e} (bound {tol:.1e})")
    assert err <= tol


@pytest.mark.parametrize("J,K", CASES)
@pytest.mark.parametrize("opname", ["W", "WT"])
def test_fp32_wavelets_extreme_sizes(stp, J, K, opname):
    """The FP32 transforms (two columns per thread) on the same sizes, against
    the oracle's FP64 columns: FP32 operator bound."""
    say(f"extreme size J={J} K={K}: FP32 {opname}")
    P = Problem(J, K)
    X = synth.random_field(P.shape, 92)
    out = np.zeros(X.size)
    ctx = stp.stp_create(J, K, 1, stp.STP_MIXED)
    try:
        stp.stp_apply(ctx, getattr(stp, "STP_OP_" + opname), stp.STP_MIXED, 0, X.reshape(-1), out)
    finally:
        stp.stp_destroy(ctx)
    nodes = _nodes(P.n)
    fn = orow.W_columns if opname == "W" else orow.WT_columns
    ref, got = fn(P, X, nodes), out.reshape(P.N + 1, -1)[:, nodes]
    err = float(np.abs(got - ref).max() / np.abs(ref).max())
    say(f"  max rel error {err:.2e} (bound 2.0e-4)")
    assert err <= 2e-4


@pytest.mark.parametrize("J,K", CASES)
@pytest.mark.parametrize("prec", ["FP64", "MIXED"])
def test_solve_extreme_sizes(stp, J, K, prec):
    say(f"extreme size J={J} K={K}: solve {prec}")
    P = Problem(J, K)
    g = synth.fourier_g(J, K, 7)
    u0 = synth.smooth_u0(K, 7)
    ctx = stp.stp_create(J, K, 1, getattr(stp, "STP_" + prec))
    try:
        stp.stp_set_g(ctx, 0, g.reshape(-1))
        stp.stp_set_u0(ctx, 0, u0.reshape(-1))
        status, st = stp.stp_solve(ctx, 1e-8)
        u = np.zeros(g.size)
        stp.stp_get_solution(ctx, 0, u)
    finally:
        stp.stp_destroy(ctx)
    say(f"  status {status}, iterations {st[0]['iterations']}")
    assert status == stp.STP_OK
    rows = _rows(P.N)
    f = orow.rhs_rows(P, lambda lo, hi: g[lo:hi + 1], u0, rows)
    r = f - orow.S_rows(P, u.reshape(P.shape), rows)
    res = np.linalg.norm(r.reshape(len(rows), -1), axis=1).max()
    scale = np.linalg.norm(f.reshape(len(rows), -1), axis=1).max()
    say(f"  sampled residual / f = {res / scale:.2e}")
    assert res <= 1e-6 * scale


def test_context_larger_than_the_device_is_rejected(stp):
    """J = 14, K = 10 needs far more than 288 GB: creation fails cleanly with
    STP_E_OUT_OF_MEMORY and the library stays usable."""
    need = stp.stp_footprint(14, 10, 1, stp.STP_FP64)
    say(f"context J=14 K=10 needs {need / 1e12:.2f} TB")
    assert need > 400e9
    with pytest.raises(stp.StpError) as e:
        stp.stp_create(14, 10, 1, stp.STP_FP64)
    assert e.value.status == stp.STP_E_OUT_OF_MEMORY
    ctx = stp.stp_create(2, 3)
    stp.stp_destroy(ctx)
