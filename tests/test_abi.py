"""The C-ABI library loads on any host and exports every function declared in
include/bc.h; argument and CSR validation happen before any device call."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", "bc.h"), os.path.join(ROOT, "include", "bc_server.h")]


@pytest.fixture(scope="module")
def bc():
    from paper_2403_07858_amd import build as b
    if not os.path.exists(b.LIB):
        b.build()
    from paper_2403_07858_amd import bc as m
    return m


def declared_functions():
    text = "\n".join(open(h).read() for h in HEADERS)
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bc_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("bc_build", "bc_count", "bc_count_roots", "bc_count_batch", "bc_free", "bc_status_string",
                 "bc_last_error"):
        assert must in names


def test_every_declared_symbol_is_exported(bc):
    lib = ctypes.CDLL(bc.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(bc.EXPORTED) <= set(declared_functions())


def test_status_strings(bc):
    assert bc.bc_status_string(0) == "BC_OK"
    assert bc.bc_status_string(bc.BC_E_OVERFLOW) == "BC_E_OVERFLOW"
    assert bc.bc_status_string(-1234) == "BC_E_UNKNOWN"


def _u(x):
    return np.array(x, dtype=np.uint64)


def _i(x):
    return np.array(x, dtype=np.uint32)


def test_duplicate_edge_rejected(bc):
    with pytest.raises(bc.BCError) as e:
        bc.bc_build(2, 2, _u([0, 2, 3]), _i([0, 0, 1]), _u([0, 2, 3]), _i([0, 0, 1]))
    assert e.value.status == bc.BC_E_BAD_CSR


def test_out_of_range_id_rejected(bc):
    with pytest.raises(bc.BCError) as e:
        bc.bc_build(1, 2, _u([0, 1]), _i([7]), _u([0, 0, 1]), _i([0]))
    assert e.value.status == bc.BC_E_BAD_CSR


def test_bad_indptr_rejected(bc):
    with pytest.raises(bc.BCError) as e:
        bc.bc_build(2, 2, _u([0, 2, 1]), _i([0, 1]), _u([0, 1, 2]), _i([0, 0]))
    assert e.value.status == bc.BC_E_BAD_CSR


def test_non_transpose_rejected(bc):
    # U says 0-0, 1-1; V says 0-1, 1-0
    with pytest.raises(bc.BCError) as e:
        bc.bc_build(2, 2, _u([0, 1, 2]), _i([0, 1]), _u([0, 1, 2]), _i([1, 0]))
    assert e.value.status == bc.BC_E_INCONSISTENT
    # same degrees on both sides, different edges: U has 0-0, 1-1; V has 0-1, 1-0
    with pytest.raises(bc.BCError) as e:
        bc.bc_build(2, 3, _u([0, 1, 2]), _i([0, 1]), _u([0, 1, 2, 2]), _i([1, 0]))
    assert e.value.status == bc.BC_E_INCONSISTENT


def test_null_and_range_arguments(bc):
    lib = bc._lib
    out = bc.bc_u128()
    assert lib.bc_count(None, 2, 2, None, ctypes.byref(out), None) == bc.BC_E_INVALID_ARG
    assert lib.bc_build(None, None, None, None) == bc.BC_E_INVALID_ARG
    assert lib.bc_count_roots(None, 2, 2, 0, 0, 1, None, ctypes.byref(out), None) == bc.BC_E_INVALID_ARG
    assert lib.bc_graph_info(None, None, None, None) == bc.BC_E_INVALID_ARG
    lib.bc_free(None)  # NULL is ignored
    assert out.lo == 0 and out.hi == 0
    counts = (bc.bc_u128 * 4)()
    assert lib.bc_count_per_vertex(None, 2, 2, 0, None, counts) == bc.BC_E_INVALID_ARG
    assert lib.bc_count_noalloc(None, 2, 2, None, ctypes.byref(out)) == bc.BC_E_INVALID_ARG
    assert all(c.lo == 0 and c.hi == 0 for c in counts)


def test_tune_batch_argument_errors(bc):
    lib = ctypes.CDLL(bc.LIB_PATH)
    lib.bc_tune_batch.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_size_t] + [ctypes.c_void_p] * 2
    lib.bc_tune_batch.restype = ctypes.c_int32
    # no output, or items without arrays: refused before any device work
    assert lib.bc_tune_batch(None, None, None, 0, None, None) == bc.BC_E_INVALID_ARG
    tuned = bc.bc_opts()
    assert lib.bc_tune_batch(None, None, None, 3, None, ctypes.byref(tuned)) == bc.BC_E_INVALID_ARG
    # an empty batch keeps the base options
    base = bc.make_opts(waves_per_cu=8, lds_words=256)
    assert lib.bc_tune_batch(None, None, None, 0, ctypes.byref(base), ctypes.byref(tuned)) == bc.BC_OK
    assert tuned.waves_per_cu == 8 and tuned.lds_words == 256


def test_option_values_checked_before_device_work(bc):
    # a valid 1x1 graph with out-of-range option values: refused by bc_build
    # before any device call (so this runs without a GPU)
    args = (1, 1, _u([0, 1]), _i([0]), _u([0, 1]), _i([0]))
    for bad in ({"order_key": 5}, {"switch_depth": 1}, {"switch_depth": 4}, {"roots_per_wave": 65},
                {"root_build": 2}, {"anchor": 3}):
        with pytest.raises(bc.BCError) as e:
            bc.bc_build(*args, **bad)
        assert e.value.status == bc.BC_E_INVALID_ARG, bad
    half = bc.Allocator(lambda n, st: 0, lambda p, st: None)
    half.struct.free = ctypes.cast(None, type(half.struct.free))
    with pytest.raises(bc.BCError) as e:
        bc.bc_build(*args, allocator=half)
    assert e.value.status == bc.BC_E_INVALID_ARG


def test_older_shorter_opts_are_accepted(bc):
    # struct_size covering only the first fields: later fields are not read
    # (a garbage value past struct_size must not be seen as a bad option)
    o = bc.make_opts(switch_depth=9)
    o.struct_size = bc.bc_opts.timeout_ms.offset + 4
    lib = bc._lib
    args = (1, 1, _u([0, 1]), _i([0]), _u([0, 1]), _i([0]))
    keep = []
    cu = bc._csr(args[0], args[1], args[2], args[3], keep)
    cv = bc._csr(args[1], args[0], args[4], args[5], keep)
    # validation passes the option check and goes on; without a GPU the call
    # may then fail on the device, but never with BC_E_INVALID_ARG
    h = ctypes.c_void_p()
    s = lib.bc_build(ctypes.byref(cu), ctypes.byref(cv), ctypes.byref(o), ctypes.byref(h))
    assert s != bc.BC_E_INVALID_ARG
    if s == bc.BC_OK:
        lib.bc_free(h)
