"""Batched PCG iterations between the host's flag reads (stp_options.lookahead).

The stopping test of Section 3.4 is taken on the device, and a right-hand
side that has stopped gets gamma = 0, so iterations enqueued after its stop
leave its w, r, iteration count and residual as they were.  Solves with the
flags read after every iteration (lookahead = -1) and in batches (default)
must therefore agree bit for bit: FP64 and mixed, a batch of right-hand sides
that stop at different iterations, the fixed-iteration protocol (tol 0) and
the iteration limit.  The per-solve times of a small problem are printed."""
import sys
import time

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def stp():
    import paper_2009_08875_amd as lib

    return lib


def _run(stp, J, K, nrhs, prec, tol, lookahead, maxit=0, reps=1):
    n = (2 ** K - 1) ** 2
    ctx = stp.stp_create(J, K, nrhs, prec, {"lookahead": lookahead, "maxit": maxit})
    try:
        for b in range(nrhs):
            # right-hand sides of different difficulty: their own seeds and
            # forcing scales, one with zero forcing
            g = synth.fourier_g(J, K, 300 + b) * (0.0 if b == 1 else 10.0 ** (b % 3))
            stp.stp_set_g(ctx, b, g.reshape(-1))
            stp.stp_set_u0(ctx, b, synth.smooth_u0(K, 300 + b).reshape(-1).copy())
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            status, st = stp.stp_solve(ctx, tol, nrhs=nrhs)
            times.append(time.perf_counter() - t0)
        us = []
        for b in range(nrhs):
            u = np.zeros(((1 << J) + 1) * n)
            stp.stp_get_solution(ctx, b, u)
            us.append(u)
    finally:
        stp.stp_destroy(ctx)
    return status, st, us, times


@pytest.mark.parametrize("prec", ["FP64", "MIXED"])
@pytest.mark.parametrize("tol,maxit", [(1e-8, 0), (1e-10, 0), (0.0, 9), (1e-12, 6)])
def test_batched_iterations_equal_per_iteration_reads(stp, prec, tol, maxit):
    p = getattr(stp, "STP_" + prec)
    J, K, nrhs = 4, 5, 4
    s1, st1, u1, _ = _run(stp, J, K, nrhs, p, tol, -1, maxit)
    s0, st0, u0, _ = _run(stp, J, K, nrhs, p, tol, 0, maxit)
    say(f"{prec} tol={tol} maxit={maxit}: iterations "
        f"{[s['iterations'] for s in st1]} / {[s['iterations'] for s in st0]}")
    assert s0 == s1
    for b in range(nrhs):
        for key in ("iterations", "outer_iterations", "rel_residual", "status"):
            assert st0[b][key] == st1[b][key], (b, key)
        assert np.array_equal(u0[b], u1[b]), b
    if maxit and tol == 0.0 and prec == "FP64":
        assert all(s["iterations"] == maxit for b, s in enumerate(st0) if b != 1)


def test_small_solve_times(stp):
    """Time per solve of a small problem (J = 6, K = 5: about 0.06 ms of
    kernel work per iteration) with the flags read after every iteration and
    in batches; reported, and the batched form must not be slower by more
    than noise."""
    res = {}
    for la in (-1, 0):
        _, st, u, times = _run(stp, 6, 5, 1, stp.STP_FP64, 1e-8, la, reps=12)
        res[la] = (float(np.median(times[2:])), st[0]["iterations"], u[0])
    say(f"J=6 K=5 FP64 solve: {res[-1][0] * 1e3:.2f} ms reading flags every iteration, "
        f"{res[0][0] * 1e3:.2f} ms in batches ({res[0][1]} iterations)")
    assert res[-1][1] == res[0][1] and np.array_equal(res[-1][2], res[0][2])
    assert res[0][0] <= 1.5 * res[-1][0]
