"""C-ABI contract checks that need no GPU."""
import ctypes
import os
import subprocess

import pytest

import paper_2301_12584_amd as krps


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(krps.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return krps.lib()


def test_every_declared_symbol_is_exported(L):
    names = krps.declared_symbols()
    assert len(names) >= 14
    out = subprocess.run(["nm", "-D", "--defined-only", krps.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [n for n in names if n not in exported]
    assert not missing, missing


def test_version_and_error_strings(L):
    assert b"krps" in L.krps_version()
    assert isinstance(L.krps_last_error(), bytes)


def _ws(dims, R, F=0, p=1):
    n = len(dims)
    arr = (ctypes.c_int64 * n)(*dims)
    out = ctypes.c_size_t()
    code = krps.lib().krps_sampler_workspace_bytes(n, arr, R, F, p, ctypes.byref(out))
    return code, out.value


def test_workspace_query_validates_on_the_host(L):
    code, nbytes = _ws([1000, 2000], 32)
    assert code == 0 and nbytes > 0
    assert _ws([1000], 0)[0] == -1                 # R < 1
    assert _ws([1000], 129)[0] == -1               # R > 128
    assert _ws([0, 5], 8)[0] == -1                 # empty factor
    assert _ws([5] * 10, 8)[0] == 0                # N = 10 is the largest
    assert _ws([5] * 11, 8)[0] == -1               # N > 10
    assert _ws([5, 5], 8, F=-1)[0] == -1
    assert _ws([5, 5], 8, p=7)[0] == -1            # unknown precision
    assert b"R must be" in L.krps_last_error() or b"precision" in L.krps_last_error()


def test_workspace_grows_with_the_factor_and_precision(L):
    _, a = _ws([1 << 12], 32, p=1)
    _, b = _ws([1 << 14], 32, p=1)
    _, c = _ws([1 << 14], 32, p=0)
    assert b > a and c > b
    # stored nodes: root + left children of T_{I,F}, packed upper triangles
    _, d = _ws([1 << 20], 32, p=1)
    tri = 32 * 33 // 2
    assert d >= (1 << 20) // 32 * tri * 4


def test_null_handles_are_rejected(L):
    assert L.krps_sampler_refresh(None, 0) == -1
    assert L.krps_ctx_sync(None) == -1
    out = ctypes.c_size_t()
    assert L.krps_sample_workspace_bytes(None, ctypes.byref(out)) == -1
    assert L.krps_sample(None, -1, 1, None, None, None, None, None, 0, 0) == -1
