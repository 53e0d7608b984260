"""CPU checks of the C-ABI library: it loads, exports every declared symbol,
and its host-side logic (footprints, argument checks, status strings) works
without a GPU.  No compute call is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(stp_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def stp():
    import paper_2009_08875_amd as lib

    return lib


def test_library_exports_every_declared_symbol(stp):
    lib = ctypes.CDLL(stp.LIBRARY_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert declared_functions(), "no declarations parsed"
    assert not missing, missing


def test_footprint_and_sizes(stp):
    small = stp.stp_footprint(4, 4, 1, stp.STP_FP64)
    assert 0 < small < 8 << 20
    # the configurations that have to fit in 288 GB of HBM
    assert stp.stp_footprint(10, 9, 1, stp.STP_FP64) < 64 << 30
    assert stp.stp_footprint(12, 9, 1, stp.STP_MIXED) < 200 << 30
    assert stp.stp_footprint(8, 7, 64, stp.STP_MIXED) < 64 << 30
    # more right-hand sides cost more
    assert stp.stp_footprint(4, 4, 2, stp.STP_FP64) > small


@pytest.mark.parametrize("J,K,nrhs,prec", [(-1, 4, 1, 0), (15, 4, 1, 0), (4, 0, 1, 0), (4, 11, 1, 0),
                                           (4, 4, 0, 0), (4, 4, 1, 7)])
def test_footprint_rejects_bad_sizes(stp, J, K, nrhs, prec):
    with pytest.raises(stp.StpError) as e:
        stp.stp_footprint(J, K, nrhs, prec)
    assert e.value.status == stp.STP_E_INVALID_ARG


def test_status_strings(stp):
    for s in (0, 1, -1, -2, -3, -4, -5, -6):
        assert stp.stp_status_string(s)
    assert stp.stp_status_string(42) == "unknown status"


def test_null_context_is_rejected(stp):
    assert stp._lib.stp_solve(None, 1e-8, None) == stp.STP_E_INVALID_ARG
    assert "NULL" in stp.stp_last_error()


def test_server_argument_checks(stp):
    """Argument validation of the serving entry points happens before any
    device call."""
    out = ctypes.c_void_p()
    assert stp._lib.stp_server_create(0, 4, 1, None, ctypes.byref(out)) == stp.STP_E_INVALID_ARG
    assert stp._lib.stp_server_create(1 << 30, 0, 1, None, ctypes.byref(out)) == stp.STP_E_INVALID_ARG
    assert stp._lib.stp_server_create(1 << 30, 4, 65, None, ctypes.byref(out)) == stp.STP_E_INVALID_ARG
    assert stp._lib.stp_server_create(1 << 30, 4, 1, None, None) == stp.STP_E_INVALID_ARG
    rid = ctypes.c_uint64()
    req = stp.stp_request(4, 4, stp.STP_FP64, 1e-8, None, None, None, 0)
    assert stp._lib.stp_server_submit(None, ctypes.byref(req), ctypes.byref(rid)) == stp.STP_E_INVALID_ARG
    assert stp._lib.stp_server_poll(None, 1, None, None) == stp.STP_E_INVALID_ARG
    assert stp._lib.stp_server_drain(None) == stp.STP_E_INVALID_ARG
    assert stp._lib.stp_server_info(None, None) == stp.STP_E_INVALID_ARG
    assert stp._lib.stp_server_destroy(None) == stp.STP_OK
