"""The allocation-free K_x entry point (stp_kspace_apply_static) against the
context-based stp_apply(STP_OP_KSPACE): same kernels, so the same values bit
for bit, on consecutive calls of different sizes that share the library's
fixed device array (the second call smaller than the first), including a
call that needs several chunks of rows."""
import sys

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


def _reference(stp, torch, J, K, x):
    ctx = stp.stp_create(J, K, 1, stp.STP_FP64, stream=torch.cuda.current_stream())
    try:
        out = torch.empty_like(x)
        stp.stp_apply(ctx, stp.STP_OP_KSPACE, stp.STP_FP64, 0, x, out)
        torch.cuda.synchronize()
    finally:
        stp.stp_destroy(ctx)
    return out


def test_static_kspace_equals_context_path(stp):
    import torch

    dev = torch.device("cuda:0")
    # (J, K): a chunked call (33 rows of 261121 nodes > the array), then
    # smaller ones reusing the array's stale contents
    cases = [(5, 9), (3, 6), (2, 4)]
    for J, K in cases:
        rows, n = 2 ** J + 1, 2 ** K - 1
        say(f"static K_x: {rows} rows, K={K}")
        x = torch.as_tensor(synth.random_field((rows, n * n), 300 + K), device=dev).reshape(-1)
        got = torch.full_like(x, float("nan"))
        stp.stp_kspace_apply_static(K, rows, x, got, torch.cuda.current_stream())
        torch.cuda.synchronize()
        ref = _reference(stp, torch, J, K, x)
        err = ((got - ref).abs().max() / ref.abs().max()).item()
        say(f"  bitwise equal: {torch.equal(got, ref)}, max rel diff {err:.2e}")
        assert torch.isfinite(got).all()
        assert err <= 1e-12


def test_static_kspace_rejects_bad_arguments(stp):
    import torch

    x = torch.zeros(49, dtype=torch.float64, device="cuda:0")
    p = x.data_ptr()
    for K, rows, a, b in [(0, 1, p, p), (11, 1, p, p), (3, -1, p, p), (3, 1, None, p)]:
        status = stp._lib.stp_kspace_apply_static(K, rows, a, b, None)
        assert status == stp.STP_E_INVALID_ARG, (K, rows)
        assert "stp_kspace_apply_static" in stp.stp_last_error()
    assert stp._lib.stp_kspace_apply_static(3, 0, None, None, None) == stp.STP_OK
