"""The C-ABI library: it loads, exports every declared symbol, and its
host-side argument rules and quick returns behave as the header states.
These run without a GPU (no compute call is made)."""
import ctypes
import os
import re

import pytest

from paper_2203_09353_amd import bgemm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols(header, prefix):
    with open(os.path.join(ROOT, "include", header)) as f:
        text = f.read()
    return set(re.findall(r"\b(%s_[a-z0-9_]+)\s*\(" % prefix, text))


def test_library_exports_every_declared_symbol():
    L = bgemm.lib()
    declared = _declared_symbols("bgemm.h", "bg")
    assert declared == set(bgemm.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name


def test_library_exports_the_request_loop():
    from paper_2203_09353_amd import serve
    L = serve._lib()
    declared = _declared_symbols("bgserve.h", "bs")
    assert declared == {"bs_create", "bs_destroy", "bs_bytes_needed", "bs_reset",
                        "bs_run_schedule", "bs_state", "bs_fill_factor", "bs_simulate",
                        "bs_set_max_active", "bs_run_sweeps", "bs_set_policy",
                        "bs_memory_stats", "bs_set_tick_launch"}
    for name in declared:
        assert hasattr(L, name), name
    # host-side argument checks need no device
    assert L.bs_destroy(None) == 5
    assert L.bs_reset(None) == 5
    assert L.bs_fill_factor(1, 0, 0, 0, None, None) == 1
    assert L.bs_set_policy(None, 1) == 5
    assert L.bs_memory_stats(None, None, None, None) == 5
    assert L.bs_set_tick_launch(None, 1) == 5


def test_version_and_status_strings():
    L = bgemm.lib()
    assert L.bg_version() >= 100
    assert L.bg_status_string(0) == b"BG_STATUS_SUCCESS"
    assert L.bg_status_string(6) == b"BG_STATUS_WORKSPACE_TOO_SMALL"


def test_null_handle_is_rejected_without_device():
    L = bgemm.lib()
    assert L.bg_dgemm_batched(None, b"N", b"N", 1, 1, 1, 1.0, None, 1, None, 1, 0.0, None, 1, 1) == 5
    assert L.bg_destroy(None) == 5
    assert L.bg_last_invalid_arg(None) == 0


P = 0x1000  # a non-NULL placeholder; the host check never dereferences it


@pytest.mark.parametrize("args,expect", [
    (("N", "N", 4, 3, 2, P, 4, P, 2, P, 4, 5), 0),
    (("X", "N", 4, 3, 2, P, 4, P, 2, P, 4, 5), 1),
    (("N", "q", 4, 3, 2, P, 4, P, 2, P, 4, 5), 2),
    (("N", "N", -1, 3, 2, P, 4, P, 2, P, 4, 5), 3),
    (("N", "N", 4, -3, 2, P, 4, P, 2, P, 4, 5), 4),
    (("N", "N", 4, 3, -2, P, 4, P, 2, P, 4, 5), 5),
    (("N", "N", 4, 3, 2, P, 3, P, 2, P, 4, 5), 8),       # lda < m
    (("T", "N", 4, 3, 2, P, 1, P, 2, P, 4, 5), 8),       # lda < k for 'T'
    (("T", "N", 4, 3, 2, P, 2, P, 2, P, 4, 5), 0),
    (("N", "N", 4, 3, 2, P, 4, P, 1, P, 4, 5), 10),      # ldb < k
    (("N", "T", 4, 3, 2, P, 4, P, 2, P, 4, 5), 10),      # ldb < n for 'T'
    (("N", "c", 4, 3, 2, P, 4, P, 3, P, 4, 5), 0),
    (("N", "N", 4, 3, 2, P, 4, P, 2, P, 3, 5), 13),      # ldc < m
    (("N", "N", 4, 3, 2, P, 4, P, 2, P, 4, -1), 14),     # batch < 0
    (("N", "N", 0, 0, 0, P, 0, P, 1, P, 1, 5), 8),       # ld >= 1 even for empty
    (("N", "N", 4, 3, 2, 0, 4, P, 2, P, 4, 5), 7),       # NULL A array
    (("N", "N", 4, 3, 2, P, 4, 0, 2, P, 4, 5), 9),       # NULL B array
    (("N", "N", 4, 3, 2, P, 4, P, 2, 0, 4, 5), 12),      # NULL C array
    (("N", "N", 4, 3, 0, 0, 4, 0, 1, P, 4, 5), 0),       # k == 0: A, B not read
    (("N", "N", 0, 3, 2, 0, 1, 0, 2, 0, 1, 5), 0),       # m == 0: nothing read
    (("N", "N", 4, 3, 2, 0, 4, 0, 2, 0, 4, 0), 0),       # batch == 0
    (("X", "?", -1, -1, -1, 0, 0, 0, 0, 0, 0, -1), 1),   # first failing rule wins
])
def test_host_argument_rules(args, expect):
    ta, tb, m, n, k, A, lda, B, ldb, C, ldc, batch = args
    assert bgemm.check_batched_args(ta, tb, m, n, k, A, lda, B, ldb, C, ldc, batch) == expect


def test_argument_rules_match_oracle():
    import oracle
    import itertools
    for ta, tb, m, n, k in itertools.product("NTx", "NT", [-1, 0, 3], [0, 2], [-1, 0, 4]):
        for lda, ldb, ldc in itertools.product([0, 1, 3, 4], [1, 2, 4], [0, 3]):
            o = oracle.check_args(ta, tb, m, n, k, lda, ldb, ldc)
            g = bgemm.check_batched_args(ta, tb, m, n, k, P, lda, P, ldb, P, ldc, 1)
            assert -o == g, (ta, tb, m, n, k, lda, ldb, ldc)


def test_missing_library_fails_loudly():
    # no fallback: without the built HIP library every entry point raises
    from paper_2203_09353_amd import bgemm
    saved = bgemm._lib
    bgemm._lib = None
    try:
        with pytest.raises(RuntimeError, match="not built"):
            bgemm.lib("/nonexistent/libbgemm.so")
    finally:
        bgemm._lib = saved
