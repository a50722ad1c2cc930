"""The C ABI: the library loads, exports every declared symbol, and its host
logic (parameter checks, sizes) behaves -- no GPU needed, no compute calls."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(elsar_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def elsar():
    import paper_2305_05671_amd as e
    return e


def test_every_declared_symbol_is_exported(elsar):
    names = _declared()
    assert "elsar_sort" in names and "elsar_partition" in names and "elsar_sample_fit" in names
    assert "elsar_sort_buckets" in names
    lib = ctypes.CDLL(elsar.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_defaults_and_status_strings(elsar):
    p = elsar.fit_params()
    assert (p.record_bytes, p.key_bytes, p.num_buckets) == (100, 10, 0)
    for s in range(6):
        assert elsar.status_string(s)


def test_argument_checks_return_before_any_work(elsar):
    lib = elsar.lib()
    sz = ctypes.c_size_t()
    p = elsar.fit_params()
    assert lib.elsar_sort_workspace_size(ctypes.byref(p), 1000, ctypes.byref(sz)) == elsar.OK and sz.value > 0
    bad = elsar.fit_params(record_bytes=102)
    assert lib.elsar_sort_workspace_size(ctypes.byref(bad), 10, ctypes.byref(sz)) == elsar.E_UNSUPPORTED
    bad = elsar.fit_params(key_bytes=29)
    assert lib.elsar_sort_workspace_size(ctypes.byref(bad), 10, ctypes.byref(sz)) == elsar.E_UNSUPPORTED
    bad = elsar.fit_params(key_bytes=7)
    assert lib.elsar_sort_workspace_size(ctypes.byref(bad), 10, ctypes.byref(sz)) == elsar.E_UNSUPPORTED
    # keys of 13..28 bytes take the run fix-up, whose scratch the workspace includes
    long_k = elsar.fit_params(key_bytes=28, region_pct=1)
    assert lib.elsar_sort_workspace_size(ctypes.byref(long_k), 1000, ctypes.byref(sz)) == elsar.OK
    assert sz.value >= 1000 * (100 + 40)
    # the batch's small-job kernel sorts at most 12 key bytes
    job = elsar.Job()
    job.n = 10
    long16 = elsar.fit_params(key_bytes=16)
    assert lib.elsar_sort_batch_workspace_size(ctypes.byref(job), 1, ctypes.byref(long16),
                                               ctypes.byref(sz)) == elsar.E_UNSUPPORTED
    bad = elsar.fit_params(record_bytes=36, key_bytes=10)
    assert lib.elsar_sort_workspace_size(ctypes.byref(bad), 10, ctypes.byref(sz)) == elsar.E_UNSUPPORTED
    bad = elsar.fit_params(num_buckets=(1 << 21) + 1)
    assert lib.elsar_sort_workspace_size(ctypes.byref(bad), 10, ctypes.byref(sz)) == elsar.E_INVALID_ARG
    assert lib.elsar_sort_workspace_size(ctypes.byref(p), 2 * 10 ** 9, ctypes.byref(sz)) == elsar.E_UNSUPPORTED
    # the in-HBM ceiling: input, output and workspace of the largest sort fit
    # one MI355X's 288 GB; one record more is refused before any work
    top = 400_000_000
    assert elsar.MAX_DEVICE_RECORDS == top
    assert lib.elsar_sort_workspace_size(ctypes.byref(p), top, ctypes.byref(sz)) == elsar.OK
    assert sz.value + 2 * 100 * top <= 288 * 10 ** 9
    assert lib.elsar_sort_workspace_size(ctypes.byref(p), top + 1, ctypes.byref(sz)) == elsar.E_UNSUPPORTED
    assert lib.elsar_sort(16, top + 1, 32, ctypes.byref(p), 64, 10 ** 12, None) == elsar.E_UNSUPPORTED
    assert lib.elsar_sort_workspace_size(None, 10, ctypes.byref(sz)) == elsar.E_INVALID_ARG
    # n == 0 is a no-op; null buffers with n > 0 are rejected before anything is enqueued
    assert lib.elsar_sort(None, 0, None, ctypes.byref(p), None, 0, None) == elsar.OK
    assert lib.elsar_sort(None, 5, None, ctypes.byref(p), None, 0, None) == elsar.E_INVALID_ARG
    assert lib.elsar_sort(16, 5, 32, ctypes.byref(p), 64, 10, None) == elsar.E_NO_MEMORY
    assert lib.elsar_sort(17, 5, 32, ctypes.byref(p), 64, 10 ** 12, None) == elsar.E_INVALID_ARG
    assert lib.elsar_partition(None, None, 0, None, 0, None, None) == elsar.E_INVALID_ARG
    # a misaligned partition buffer or offsets array is refused before the
    # model or any device memory is touched (the pointers are never dereferenced)
    assert lib.elsar_partition(64, None, 0, 32 + 8, 1 << 20, 64, None) == elsar.E_INVALID_ARG
    assert lib.elsar_partition(64, None, 0, 32, 1 << 20, 64 + 4, None) == elsar.E_INVALID_ARG
    assert lib.elsar_sort_buckets(64, 32 + 8, 1 << 20, 0, 64, None, None) == elsar.E_INVALID_ARG
    assert lib.elsar_sort_buckets(64, 32, 1 << 20, 0, 64 + 4, None, None) == elsar.E_INVALID_ARG


def test_noalloc_argument_checks(elsar):
    # the no-allocation entry refuses null buffers and sizes whose workspace
    # exceeds its fixed scratch before it touches the device
    lib = elsar.lib()
    p = elsar.fit_params()
    assert lib.elsar_sort_noalloc(None, 0, None, ctypes.byref(p), None) == elsar.OK
    assert lib.elsar_sort_noalloc(None, 5, None, ctypes.byref(p), None) == elsar.E_INVALID_ARG
    assert lib.elsar_sort_noalloc(16, 10 ** 7, 32, ctypes.byref(p), None) == elsar.E_NO_MEMORY
    assert lib.elsar_sort_noalloc(16, 5, 32, None, None) == elsar.E_INVALID_ARG
    assert elsar.sort_workspace_size(500_000, p) <= elsar.NOALLOC_SCRATCH_BYTES


def test_workspace_grows_linearly(elsar):
    lib = elsar.lib()
    p = elsar.fit_params()
    out = []
    for n in [10 ** 5, 10 ** 6, 10 ** 7]:
        sz = ctypes.c_size_t()
        assert lib.elsar_sort_workspace_size(ctypes.byref(p), n, ctypes.byref(sz)) == elsar.OK
        out.append(sz.value / n)
    # regions (<= 2.5n slots) + spill (n slots) of 128 bytes, plus small arrays
    assert all(420 < b < 520 for b in out), out


def test_record_size_limits(elsar):
    lib = elsar.lib()
    sz = ctypes.c_size_t()
    for R, ok in [(40, True), (100, True), (128, True), (132, False), (36, False), (102, False)]:
        p = elsar.fit_params(record_bytes=R, key_bytes=10)
        rc = lib.elsar_sort_workspace_size(ctypes.byref(p), 1000, ctypes.byref(sz))
        assert (rc == elsar.OK) == ok, (R, rc)
