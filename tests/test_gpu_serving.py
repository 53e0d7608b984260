"""Serving form on the GPU: continuous batching through the C-ABI.

Requests of uneven sizes and precisions are submitted while others run; each
result must equal the same request solved alone (stp_solve on a context of
its own) within 1e-12 relative in FP64 and 1e-9 in the mixed form (the path
is deterministic, so equality is expected to be bitwise), and match the CPU
oracle on a small case.
"""
import sys
import time

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_helpers import flat, grid, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stp():
    import paper_2009_08875_amd as lib

    return lib


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _data(J, K, seed):
    return synth.fourier_g(J, K, seed), synth.smooth_u0(K, seed)


def _solo(stp, J, K, prec, tol, g, u0):
    ctx = stp.stp_create(J, K, 1, prec)
    try:
        stp.stp_set_g(ctx, 0, flat(g))
        stp.stp_set_u0(ctx, 0, flat(u0))
        status, st = stp.stp_solve(ctx, tol)
        u = np.zeros(g.size)
        stp.stp_get_solution(ctx, 0, u)
    finally:
        stp.stp_destroy(ctx)
    return status, st[0], u


def _wait(stp, server, ids, timeout=120.0):
    done = {}
    t0 = time.time()
    while len(done) < len(ids):
        for rid in ids:
            if rid in done:
                continue
            r = stp.stp_server_poll(server, rid)
            if r is not None:
                done[rid] = r
        assert time.time() - t0 < timeout, "server did not finish in time"
        time.sleep(0.002)
    return done


# (J, K, precision, tol, seed): three of one shape (batched together), other
# shapes, both precisions, tolerances 1e-6 .. 1e-10; the K = 6 and K = 7
# requests (two of them grouped) run the streaming multigrid kernels, whose
# launch shapes the tuner picks per number of rows, so a group of two gets
# other shapes than a solo solve
MIX = [
    (3, 5, "FP64", 1e-8, 201), (3, 5, "FP64", 1e-6, 202), (3, 5, "FP64", 1e-10, 203),
    (4, 4, "MIXED", 1e-8, 204), (2, 6, "FP64", 1e-9, 205), (5, 3, "MIXED", 1e-7, 206),
    (3, 5, "MIXED", 1e-8, 207), (0, 1, "FP64", 1e-8, 208),
    (4, 7, "FP64", 1e-8, 209), (4, 7, "FP64", 1e-9, 210), (4, 7, "MIXED", 1e-8, 211),
    (5, 6, "MIXED", 1e-8, 212),
]


def test_each_result_is_the_same_alone_and_in_the_mix(stp):
    say("serving: mixed stream vs solo solves")
    server = stp.stp_server_create(8 << 30, max_slots=4, max_batch=4)
    try:
        ids, outs = [], []
        for k, (J, K, prec, tol, seed) in enumerate(MIX):
            g, u0 = _data(J, K, seed)
            u = np.zeros(g.size)
            outs.append(u)
            ids.append(stp.stp_server_submit(server, J, K, getattr(stp, "STP_" + prec), tol,
                                             flat(u0), flat(g), u))
            if k == 3:
                time.sleep(0.05)  # later requests arrive while the first ones run
        res = _wait(stp, server, ids)
        info = stp.stp_server_info(server)
    finally:
        stp.stp_server_destroy(server)
    say(f"  server info {info}")
    assert info["requests_started"] == len(MIX)
    for (J, K, prec, tol, seed), rid, u in zip(MIX, ids, outs):
        status, st, lat = res[rid]
        g, u0 = _data(J, K, seed)
        s_status, s_st, u_solo = _solo(stp, J, K, getattr(stp, "STP_" + prec), tol, g, u0)
        say(f"  J={J} K={K} {prec} tol={tol:g}: its {st['iterations']} (solo {s_st['iterations']}), "
            f"latency {lat * 1e3:.1f} ms, bitwise {np.array_equal(u, u_solo)}")
        assert status == s_status == stp.STP_OK
        assert st["iterations"] == s_st["iterations"]
        assert rel_err(u, u_solo) <= (1e-12 if prec == "FP64" else 1e-9)


def test_many_new_contexts_concurrently(stp):
    """Sixteen requests of distinct shapes submitted at once: every admission
    creates a context while others run on the server's other streams.  Each
    result equals its solo solve (iteration count and values)."""
    say("serving: concurrent context creation")
    shapes = [(J, K) for J in (1, 2, 3, 4) for K in (2, 3, 4, 5)]
    server = stp.stp_server_create(8 << 30, max_slots=4, max_batch=1)
    try:
        ids, outs, data = [], [], []
        for k, (J, K) in enumerate(shapes):
            g, u0 = _data(J, K, 600 + k)
            u = np.zeros(g.size)
            data.append((g, u0))
            outs.append(u)
            ids.append(stp.stp_server_submit(server, J, K, stp.STP_MIXED, 1e-8, flat(u0), flat(g), u))
        res = _wait(stp, server, ids)
    finally:
        stp.stp_server_destroy(server)
    for (J, K), rid, u, (g, u0) in zip(shapes, ids, outs, data):
        status, st, _ = res[rid]
        s_status, s_st, u_solo = _solo(stp, J, K, stp.STP_MIXED, 1e-8, g, u0)
        assert status == s_status == stp.STP_OK, (J, K)
        assert st["iterations"] == s_st["iterations"], (J, K)
        assert rel_err(u, u_solo) <= 1e-9, (J, K)


def test_served_result_matches_oracle(stp):
    J, K, seed = 3, 4, 301
    say("serving: result vs oracle")
    g, u0 = _data(J, K, seed)
    u_or, _, _ = oracle.solve(J, K, g, u0, tol=1e-10)
    server = stp.stp_server_create(1 << 30, max_slots=2, max_batch=2)
    try:
        u = np.zeros(g.size)
        rid = stp.stp_server_submit(server, J, K, stp.STP_FP64, 1e-10, flat(u0), flat(g), u)
        status, st, lat = _wait(stp, server, [rid])[rid]
    finally:
        stp.stp_server_destroy(server)
    assert status == stp.STP_OK
    assert rel_err(grid(u, J, K), u_or) <= 1e-8


def test_device_buffers_and_context_reuse(stp):
    """Device-pointer requests, run in two waves so the second reuses the
    first wave's cached contexts; results equal the host-buffer solo solves."""
    import torch

    J, K = 3, 5
    say("serving: device buffers, context reuse")
    dev = torch.device("cuda:0")
    server = stp.stp_server_create(4 << 30, max_slots=2, max_batch=2)
    try:
        for wave in range(2):
            seeds = [400 + 10 * wave + k for k in range(3)]
            bufs, ids = [], []
            for sd in seeds:
                g, u0 = _data(J, K, sd)
                gt = torch.as_tensor(flat(g), device=dev)
                ut = torch.as_tensor(flat(u0), device=dev)
                out = torch.zeros(g.size, dtype=torch.float64, device=dev)
                torch.cuda.synchronize()
                bufs.append((gt, ut, out))
                ids.append(stp.stp_server_submit(server, J, K, stp.STP_MIXED, 1e-8, ut, gt, out))
            res = _wait(stp, server, ids)
            for sd, rid, (gt, ut, out) in zip(seeds, ids, bufs):
                assert res[rid][0] == stp.STP_OK
                g, u0 = _data(J, K, sd)
                _, _, u_solo = _solo(stp, J, K, stp.STP_MIXED, 1e-8, g, u0)
                assert rel_err(out.cpu().numpy(), u_solo) <= 1e-9
    finally:
        stp.stp_server_destroy(server)


def test_request_larger_than_budget_is_rejected(stp):
    server = stp.stp_server_create(1 << 20, max_slots=1)
    try:
        with pytest.raises(stp.StpError) as e:
            stp.stp_server_submit(server, 6, 7, stp.STP_FP64, 1e-8)
        assert e.value.status == stp.STP_E_OUT_OF_MEMORY
    finally:
        stp.stp_server_destroy(server)


def test_breakdown_is_reported_per_request(stp):
    """A request with non-finite data fails alone; its batch mates finish."""
    J, K = 2, 3
    say("serving: breakdown in a batch")
    g_bad = np.zeros((5, 7, 7))
    g_bad[2, 3, 3] = np.nan
    g_ok, u0 = _data(J, K, 501)
    server = stp.stp_server_create(1 << 30, max_slots=1, max_batch=2)
    try:
        u_ok = np.zeros(g_ok.size)
        r_bad = stp.stp_server_submit(server, J, K, stp.STP_FP64, 1e-8, flat(u0), flat(g_bad), None)
        r_ok = stp.stp_server_submit(server, J, K, stp.STP_FP64, 1e-8, flat(u0), flat(g_ok), u_ok)
        stp.stp_server_drain(server)
        with pytest.raises(stp.StpError) as e:
            stp.stp_server_poll(server, r_bad)
        assert e.value.status == stp.STP_E_BREAKDOWN
        status, st, _ = stp.stp_server_poll(server, r_ok)
    finally:
        stp.stp_server_destroy(server)
    assert status == stp.STP_OK
    _, _, u_solo = _solo(stp, J, K, stp.STP_FP64, 1e-8, g_ok, u0)
    assert np.array_equal(u_ok, u_solo)
