"""Nested iteration (Section 4.2) on the GPU against the oracle's nested
iteration (oracle/nested.py): meshes (J - d, K - d), each solved from the
coarser solution carried over, to a tolerance proportional to the
discretisation error (0.1 h on the target mesh, doubling per coarser mesh).

At that tolerance the two results may stop one iteration apart on some mesh,
so they are compared at the scale of the tolerance itself: relative L2
difference at most 10 x tol = h, the order of the discretisation error.  With
a tight tolerance the GPU's nested result is the discrete solution (the
oracle's PCG from zero) to 1e-8."""
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import nested
from tests.gpu_helpers import flat, grid, rel_err

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def stp():
    import paper_2009_08875_amd as lib

    return lib


def _gpu_nested(stp, J, K, depth, g, u0, tol):
    ctx = stp.stp_create(J, K, 1, stp.STP_FP64, {"nested": depth})
    try:
        stp.stp_set_g(ctx, 0, flat(g))
        stp.stp_set_u0(ctx, 0, flat(u0))
        status, st = stp.stp_solve(ctx, tol)
        u = np.zeros(g.size)
        stp.stp_get_solution(ctx, 0, u)
    finally:
        stp.stp_destroy(ctx)
    return status, st[0], grid(u, J, K)


# (J, K, depth): the coarsest meshes (J = 1 and K = 2 reached), a case whose
# target mesh uses the streaming multigrid (K = 7), and a depth beyond J
CASES = [(4, 4, 3), (5, 5, 3), (3, 7, 2), (2, 5, 4)]


@pytest.mark.parametrize("J,K,depth", CASES)
def test_nested_matches_oracle_at_the_discretisation_tolerance(stp, J, K, depth):
    tol = 0.1 * 2.0 ** -K
    g, u0 = synth.fourier_g(J, K, 70 + J), synth.smooth_u0(K, 70 + J)
    say(f"nested J={J} K={K} depth={depth} tol={tol:.2e}")
    u_or, its_or, _ = nested.solve(J, K, g, u0, tol, depth)
    status, st, u = _gpu_nested(stp, J, K, depth, g, u0, tol)
    err = rel_err(u, u_or)
    say(f"  oracle its per mesh {its_or}; GPU target {st['iterations']}, coarser "
        f"{st['coarse_iterations']}; rel L2 {err:.2e}")
    assert status == stp.STP_OK
    assert abs(st["iterations"] - its_or[-1]) <= 1
    assert abs(st["coarse_iterations"] - sum(its_or[:-1])) <= len(its_or) - 1
    assert err <= 10 * tol


def test_nested_reaches_the_discrete_solution(stp):
    J, K = 4, 6
    g, u0 = synth.fourier_g(J, K, 81), synth.smooth_u0(K, 81)
    say("nested with tol 1e-10 vs the oracle's discrete solution")
    u_ref, _, _ = oracle.solve(J, K, g, u0, tol=1e-12)
    status, st, u = _gpu_nested(stp, J, K, 3, g, u0, 1e-10)
    err = rel_err(u, u_ref)
    say(f"  target its {st['iterations']}, coarser {st['coarse_iterations']}, rel L2 {err:.2e}")
    assert status == stp.STP_OK and err <= 1e-8


def test_nested_saves_target_mesh_iterations(stp):
    """At a tolerance tied to the discretisation error the target mesh needs
    fewer iterations from the carried-over solution than from zero."""
    J, K = 8, 8
    tol = 0.1 * 2.0 ** -K
    g, u0 = synth.fourier_g(J, K, 90), synth.smooth_u0(K, 90)
    status0, st0, u0_sol = _gpu_nested(stp, J, K, 0, g, u0, tol)
    status1, st1, u1_sol = _gpu_nested(stp, J, K, 4, g, u0, tol)
    say(f"  J=8 K=8 tol {tol:.1e}: from zero {st0['iterations']} its; nested "
        f"{st1['iterations']} on the target mesh + {st1['coarse_iterations']} coarser; "
        f"difference {rel_err(u1_sol, u0_sol):.2e}")
    assert status0 == status1 == stp.STP_OK
    assert st1["iterations"] < st0["iterations"]
    assert rel_err(u1_sol, u0_sol) <= 10 * tol


def test_nested_needs_fp64(stp):
    with pytest.raises(stp.StpError) as e:
        stp.stp_create(3, 4, 1, stp.STP_MIXED, {"nested": 2})
    assert e.value.status == stp.STP_E_UNSUPPORTED
