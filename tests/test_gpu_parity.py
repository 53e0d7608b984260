"""GPU path vs the CPU oracle, operator by operator and for whole solves.

Every case calls the HIP library through the C-ABI (Python ctypes binding) and
compares element by element with the oracle on the same seeded inputs.

Tolerances (FP64 path): the kernels evaluate the same formulas as the oracle
with a different association of a few sums and a reciprocal instead of a
division, so each operator agrees to a small multiple of the unit roundoff
times the number of operations feeding an output; 1e-12 relative (max-norm,
scaled by the output's max) covers the deepest operator (S-hat: two
wavelet transforms and four V-cycles per entry).  FP32 kernels (STP_MIXED)
agree to 2e-4 relative: unit roundoff 6e-8 times the operation depth, amplified
by the multigrid smoothing of the shifted operators (measured up to 4.4e-5 for K_X).
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle.schur import Problem
from tests.gpu_helpers import flat, grid, max_rel, rel_err, sin_u0

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stp():
    import paper_2009_08875_amd as lib  # fails loudly when the HIP build is missing

    return lib


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


# (J, K): several MG tiles with a ragged tail (K = 6: 63 = 32 + 31 nodes per
# side; K = 7: 127), single-interval time (J = 0), the one-node mesh (K = 1) and
# the longest time axes whose columns fit in LDS (J = 9, 10)
OP_CASES = [(0, 1), (1, 2), (2, 3), (3, 6), (2, 7), (5, 4), (9, 3), (10, 2)]


def _op_input(J, K, seed):
    n = 2 ** K - 1
    return synth.random_field((2 ** J + 1, n, n), seed)


def _oracle_op(P, op, X, stp):
    if op == stp.STP_OP_W:
        return P.W(X)
    if op == stp.STP_OP_WT:
        return P.WT(X)
    if op == stp.STP_OP_S:
        return P.S(X)
    if op == stp.STP_OP_SHAT:
        return P.Shat(X)
    if op == stp.STP_OP_KX:
        return P.KX(X)
    if op == stp.STP_OP_KSPACE:
        return P.Kx(X)
    if op == stp.STP_OP_A:
        return P.A(X)
    if op == stp.STP_OP_M:
        return P.M(X)
    raise ValueError(op)


OPS = ["W", "WT", "A", "M", "KSPACE", "KX", "S", "SHAT"]


@pytest.mark.parametrize("J,K", OP_CASES)
@pytest.mark.parametrize("opname", OPS)
def test_operator_fp64(stp, J, K, opname):
    op = getattr(stp, "STP_OP_" + opname)
    say(f"op {opname} FP64 J={J} K={K}")
    P = Problem(J, K)
    X = _op_input(J, K, 100 + J * 16 + K)
    ref = _oracle_op(P, op, X, stp)
    ctx = stp.stp_create(J, K, 1, stp.STP_FP64)
    try:
        out = np.zeros(X.size)
        stp.stp_apply(ctx, op, stp.STP_FP64, 0, flat(X), out)
    finally:
        stp.stp_destroy(ctx)
    assert max_rel(grid(out, J, K), ref) <= 1e-12


@pytest.mark.parametrize("J,K", [(2, 3), (3, 6)])
@pytest.mark.parametrize("opname", OPS)
def test_operator_fp32(stp, J, K, opname):
    op = getattr(stp, "STP_OP_" + opname)
    say(f"op {opname} FP32 J={J} K={K}")
    P = Problem(J, K)
    X = _op_input(J, K, 200 + J * 16 + K)
    ref = _oracle_op(P, op, X, stp)
    ctx = stp.stp_create(J, K, 1, stp.STP_MIXED)
    try:
        out = np.zeros(X.size)
        stp.stp_apply(ctx, op, stp.STP_MIXED, 0, flat(X), out)
    finally:
        stp.stp_destroy(ctx)
    assert max_rel(grid(out, J, K), ref) <= 2e-4


@pytest.mark.parametrize("J,K,seed", [(2, 3, 5), (3, 6, 6), (0, 1, 7)])
def test_rhs_fp64(stp, J, K, seed):
    say(f"rhs J={J} K={K}")
    P = Problem(J, K)
    g = synth.fourier_g(J, K, seed)
    u0 = synth.smooth_u0(K, seed)
    ref = P.rhs(g, u0)
    ctx = stp.stp_create(J, K, 1, stp.STP_FP64)
    try:
        stp.stp_set_g(ctx, 0, flat(g))
        stp.stp_set_u0(ctx, 0, flat(u0))
        out = np.zeros(g.size)
        stp.stp_apply(ctx, stp.STP_OP_RHS, stp.STP_FP64, 0, None, out)
    finally:
        stp.stp_destroy(ctx)
    assert max_rel(grid(out, J, K), ref) <= 1e-12


# ------------------------------------------------------------------ solves

_ORACLE_CACHE = {}


def _oracle_solve(J, K, g, u0, tol, maxit=200):
    """The oracle's solve, computed once per data set within the session."""
    key = (J, K, tol, maxit, None if g is None else g.tobytes(), u0.tobytes())
    if key not in _ORACLE_CACHE:
        _ORACLE_CACHE[key] = oracle.solve(J, K, g, u0, tol=tol, maxit=maxit)
    return _ORACLE_CACHE[key]


def _gpu_solve(stp, J, K, g, u0, tol, prec, maxit=0):
    opts = {"maxit": maxit} if maxit else None
    ctx = stp.stp_create(J, K, 1, prec, opts)
    try:
        if g is not None:
            stp.stp_set_g(ctx, 0, flat(g))
        stp.stp_set_u0(ctx, 0, flat(u0))
        status, stats = stp.stp_solve(ctx, tol)
        u = np.zeros((2 ** J + 1) * (2 ** K - 1) ** 2)
        stp.stp_get_solution(ctx, 0, u)
        its = stp.stp_get_iterations(ctx, 0)
    finally:
        stp.stp_destroy(ctx)
    return grid(u, J, K), its, status, stats[0]


SOLVE_CASES = [
    ("heat2d_J4_K4_sin", 4, 4, None),     # the ~3.8k-unknown configuration, u0 = sin sin, g = 0
    ("fourier_J3_K5", 3, 5, 11),          # seeded Fourier forcing, smooth random u0
    ("fourier_J5_K3", 5, 3, 12),
    ("one_node_J0_K1", 0, 1, None),
    # K >= 6: the streaming multigrid kernels (levels above 5) in whole solves
    ("fourier_J6_K6", 6, 6, 13),
    ("fourier_J4_K7", 4, 7, 14),
]


def _case_data(J, K, seed):
    if seed is None:
        u0 = sin_u0(K) if K > 1 else np.ones((1, 1))
        return None, u0
    return synth.fourier_g(J, K, seed), synth.smooth_u0(K, seed)


@pytest.mark.parametrize("name,J,K,seed", SOLVE_CASES)
def test_solve_fp64_fixed_iterations(stp, name, J, K, seed):
    """Fixed-iteration protocol: the oracle converges to 1e-8 in k iterations;
    the GPU runs exactly k iterations (tol = 0); the iterates agree to 1e-10."""
    say(f"solve FP64 fixed-its {name}")
    g, u0 = _case_data(J, K, seed)
    u_or, k_or, _ = _oracle_solve(J, K, g, u0, 1e-8)
    u_gpu, k_gpu, status, st = _gpu_solve(stp, J, K, g, u0, 0.0, stp.STP_FP64, maxit=max(k_or, 1))
    assert status == stp.STP_OK
    assert k_gpu == k_or or k_or == 0
    assert rel_err(u_gpu, u_or) <= 1e-10


@pytest.mark.parametrize("name,J,K,seed", SOLVE_CASES)
def test_solve_fp64_converges_like_oracle(stp, name, J, K, seed):
    say(f"solve FP64 tol {name}")
    g, u0 = _case_data(J, K, seed)
    u_or, k_or, hist = _oracle_solve(J, K, g, u0, 1e-8)
    u_gpu, k_gpu, status, st = _gpu_solve(stp, J, K, g, u0, 1e-8, stp.STP_FP64)
    assert status == stp.STP_OK
    assert abs(k_gpu - k_or) <= 1
    assert st["rel_residual"] <= 1e-8
    assert rel_err(u_gpu, u_or) <= 1e-7


@pytest.mark.parametrize("name,J,K,seed", SOLVE_CASES[:3] + SOLVE_CASES[4:])
def test_solve_mixed_matches_fp64_oracle(stp, name, J, K, seed):
    say(f"solve mixed {name}")
    g, u0 = _case_data(J, K, seed)
    u_or, k_or, _ = _oracle_solve(J, K, g, u0, 1e-10)
    u_gpu, k_gpu, status, st = _gpu_solve(stp, J, K, g, u0, 1e-8, stp.STP_MIXED)
    assert status == stp.STP_OK
    assert st["outer_iterations"] >= 1
    err = rel_err(u_gpu, u_or)
    say(f"  mixed error vs FP64 oracle: {err:.3e}, inner its {st['iterations']}, outer {st['outer_iterations']}")
    assert err <= 1e-6


def test_solve_mixed_on_device_buffers(stp):
    """Device-pointer path of set_u0 / set_g / get_solution (torch CUDA tensors)."""
    import torch

    J, K, seed = 3, 4, 21
    say("solve mixed, device buffers")
    g, u0 = synth.fourier_g(J, K, seed), synth.smooth_u0(K, seed)
    u_or, _, _ = _oracle_solve(J, K, g, u0, 1e-10)
    dev = torch.device("cuda:0")
    ctx = stp.stp_create(J, K, 1, stp.STP_MIXED, stream=torch.cuda.current_stream())
    try:
        gt = torch.as_tensor(flat(g), device=dev)
        ut = torch.as_tensor(flat(u0), device=dev)
        stp.stp_set_g(ctx, 0, gt)
        stp.stp_set_u0(ctx, 0, ut)
        stp.stp_solve(ctx, 1e-8)
        out = torch.zeros(g.size, dtype=torch.float64, device=dev)
        stp.stp_get_solution(ctx, 0, out)
        torch.cuda.synchronize()
        u = grid(out.cpu().numpy(), J, K)
    finally:
        stp.stp_destroy(ctx)
    assert rel_err(u, u_or) <= 1e-6


@pytest.mark.parametrize("prec", ["FP64", "MIXED"])
def test_batched_equals_solo(stp, prec):
    """nrhs right-hand sides in one context give each one's solo result bitwise."""
    p = getattr(stp, "STP_" + prec)
    J, K, B = 3, 5, 3
    say(f"batched vs solo {prec}")
    data = [(synth.fourier_g(J, K, 1000 + b), synth.smooth_u0(K, 1000 + b)) for b in range(B)]
    ctx = stp.stp_create(J, K, B, p)
    try:
        for b, (g, u0) in enumerate(data):
            stp.stp_set_g(ctx, b, flat(g))
            stp.stp_set_u0(ctx, b, flat(u0))
        status, stats = stp.stp_solve(ctx, 1e-8, nrhs=B)
        ub = []
        for b in range(B):
            u = np.zeros(data[0][0].size)
            stp.stp_get_solution(ctx, b, u)
            ub.append(u)
    finally:
        stp.stp_destroy(ctx)
    assert status == stp.STP_OK
    for b, (g, u0) in enumerate(data):
        us, ks, _, st = _gpu_solve(stp, J, K, g, u0, 1e-8, p)
        assert stats[b]["iterations"] == ks
        assert np.array_equal(ub[b], us.ravel())
        u_or, _, _ = _oracle_solve(J, K, g, u0, 1e-10)
        assert rel_err(us, u_or) <= (1e-7 if prec == "FP64" else 1e-6)


def test_zero_data_gives_zero(stp):
    say("zero data")
    J, K = 2, 3
    u, its, status, st = _gpu_solve(stp, J, K, None, np.zeros((7, 7)), 1e-8, stp.STP_FP64)
    assert status == stp.STP_OK and its == 0 and not np.any(u)


def test_maxit_reports_not_converged(stp):
    say("maxit = 1")
    J, K = 3, 4
    u, its, status, st = _gpu_solve(stp, J, K, None, sin_u0(K), 1e-12, stp.STP_FP64, maxit=1)
    assert status == stp.STP_NOT_CONVERGED and its == 1
    assert np.all(np.isfinite(u)) and np.any(u)


def test_nan_forcing_reports_breakdown(stp):
    say("NaN forcing")
    J, K = 2, 3
    g = np.zeros((5, 7, 7))
    g[2, 3, 3] = np.nan
    ctx = stp.stp_create(J, K, 1, stp.STP_FP64)
    try:
        stp.stp_set_g(ctx, 0, flat(g))
        stp.stp_set_u0(ctx, 0, flat(sin_u0(K)))
        with pytest.raises(stp.StpError) as e:
            stp.stp_solve(ctx, 1e-8)
        assert e.value.status == stp.STP_E_BREAKDOWN
    finally:
        stp.stp_destroy(ctx)


def test_invalid_arguments(stp):
    say("invalid arguments")
    with pytest.raises(stp.StpError) as e:
        stp.stp_create(15, 4)
    assert e.value.status == stp.STP_E_INVALID_ARG
    ctx = stp.stp_create(2, 3)
    try:
        with pytest.raises(stp.StpError):
            stp.stp_set_u0(ctx, 1, np.zeros(49))
        with pytest.raises(stp.StpError):
            stp.stp_get_solution(ctx, 0, np.zeros(5 * 49))  # nothing solved yet
    finally:
        stp.stp_destroy(ctx)


@pytest.mark.parametrize("prec", ["FP64", "MIXED"])
def test_graph_replay_equals_eager(stp, prec):
    """Each PCG iteration replayed from a captured HIP graph gives bitwise the
    eager result, over several solves in a row with other eager work (operator
    applications, new inputs) between the replays."""
    p = getattr(stp, "STP_" + prec)
    J, K = 3, 5
    say(f"graph replay vs eager {prec}")
    cases = [(synth.fourier_g(J, K, 40 + k), synth.smooth_u0(K, 40 + k)) for k in range(3)]
    eager = stp.stp_create(J, K, 1, p, {"graph": -1})
    graph = stp.stp_create(J, K, 1, p, {"graph": 1})
    try:
        probe = flat(_op_input(J, K, 3))
        for k, (g, u0) in enumerate(cases):
            res = []
            for ctx in (eager, graph):
                stp.stp_set_g(ctx, 0, flat(g))
                stp.stp_set_u0(ctx, 0, flat(u0))
                status, st = stp.stp_solve(ctx, 1e-8)
                u = np.zeros(g.size)
                stp.stp_get_solution(ctx, 0, u)
                res.append((status, st[0]["iterations"], u))
                out = np.zeros(g.size)
                stp.stp_apply(ctx, stp.STP_OP_SHAT, p, 0, probe, out)
            assert res[0][0] == res[1][0] == stp.STP_OK
            assert res[0][1] == res[1][1]
            assert np.array_equal(res[0][2], res[1][2]), f"solve {k}"
    finally:
        stp.stp_destroy(eager)
        stp.stp_destroy(graph)


def test_mixed_edge_cases(stp):
    """The device-side control of the mixed form: zero data stops at once
    with u = 0; a single outer step with one inner iteration reports
    NOT_CONVERGED with a finite iterate; non-finite data reports breakdown."""
    say("mixed form: zero data, limits, NaN")
    J, K = 3, 4
    n = 2 ** K - 1
    u, its, status, st = _gpu_solve(stp, J, K, None, np.zeros((n, n)), 1e-8, stp.STP_MIXED)
    assert status == stp.STP_OK and its == 0 and not np.any(u)

    ctx = stp.stp_create(J, K, 1, stp.STP_MIXED, {"maxit": 1, "max_outer": 1})
    try:
        stp.stp_set_u0(ctx, 0, flat(sin_u0(K)))
        status, st = stp.stp_solve(ctx, 1e-10)
        u = np.zeros((2 ** J + 1) * n * n)
        stp.stp_get_solution(ctx, 0, u)
    finally:
        stp.stp_destroy(ctx)
    assert status == stp.STP_NOT_CONVERGED and st[0]["iterations"] == 1
    # two FP64 residuals: f-hat, and that of the refined (returned) iterate
    assert st[0]["outer_iterations"] == 2
    assert 1e-10 < st[0]["rel_residual"] < 1.0
    assert np.all(np.isfinite(u)) and np.any(u)

    g = np.zeros((2 ** J + 1, n, n))
    g[3, 5, 5] = np.inf
    ctx = stp.stp_create(J, K, 1, stp.STP_MIXED)
    try:
        stp.stp_set_g(ctx, 0, flat(g))
        stp.stp_set_u0(ctx, 0, flat(sin_u0(K)))
        with pytest.raises(stp.StpError) as e:
            stp.stp_solve(ctx, 1e-8)
        assert e.value.status == stp.STP_E_BREAKDOWN
    finally:
        stp.stp_destroy(ctx)


def test_context_is_reusable_after_a_failed_solve(stp):
    """A breakdown leaves the context usable: new data solve normally and
    give the same result as a fresh context."""
    say("context reuse after breakdown")
    J, K = 2, 3
    g_bad = np.zeros((5, 7, 7))
    g_bad[1, 2, 2] = np.nan
    g, u0 = synth.fourier_g(J, K, 31), synth.smooth_u0(K, 31)
    ctx = stp.stp_create(J, K, 1, stp.STP_FP64)
    try:
        stp.stp_set_g(ctx, 0, flat(g_bad))
        stp.stp_set_u0(ctx, 0, flat(u0))
        with pytest.raises(stp.StpError):
            stp.stp_solve(ctx, 1e-8)
        stp.stp_set_g(ctx, 0, flat(g))
        status, st = stp.stp_solve(ctx, 1e-8)
        u = np.zeros(g.size)
        stp.stp_get_solution(ctx, 0, u)
    finally:
        stp.stp_destroy(ctx)
    u_fresh, its, s2, _ = _gpu_solve(stp, J, K, g, u0, 1e-8, stp.STP_FP64)
    assert status == stp.STP_OK and st[0]["iterations"] == its
    assert np.array_equal(u, u_fresh.ravel())
