"""C-ABI checks that need no GPU: the library loads, exports every symbol that
include/gbs.h declares, its host helpers agree with the oracle's layout, and
bad arguments are rejected on the host before anything is launched."""
import ctypes
import math
import os
import re

import pytest

import oracle as O
import paper_2511_14923_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "gbs.h")).read()
    return sorted(set(re.findall(r"GBS_API\s+[\w\s\*]+?\b(gbs_\w+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    decl = _declared_symbols()
    assert set(decl) == set(P.EXPORTS)
    for name in ("gbs_correlators", "gbs_cumulants", "gbs_cumulant_grad"):
        assert name in decl


def test_library_exports_every_declared_symbol():
    lib = P.lib()
    for name in _declared_symbols():
        assert hasattr(lib, name), name
        assert ctypes.cast(getattr(lib, name), ctypes.c_void_p).value


def test_counts_and_offsets():
    for M, K in [(1, 1), (16, 3), (100, 4), (144, 5), (2048, 2)]:
        assert P.gbs_total_outputs(M, K) == O.total_outputs(M, K)
        for d in range(1, K + 1):
            assert P.gbs_num_subsets(M, d) == math.comb(M, d)
            assert P.gbs_order_offset(M, d) == O.order_offset(M, d)
    assert P.gbs_total_outputs(0, 1) == -1
    assert P.gbs_total_outputs(4, 5) == -1
    assert P.gbs_total_outputs(10, 6) == -1
    assert P.gbs_num_subsets(2049, 1) == -1


def test_colex_rank_unrank_match_layout():
    for d in range(1, 6):
        for S in list(O.subsets_colex(11, d))[::7]:
            r = P.gbs_colex_rank(S)
            assert r == O.colex_rank(S)
            assert P.gbs_colex_unrank(d, r) == tuple(S)
    big = (100, 1900, 2047, 5, 733)
    assert P.gbs_colex_unrank(5, P.gbs_colex_rank(big)) == tuple(sorted(big))
    assert P.gbs_colex_rank((3, 3)) == -1
    assert P.gbs_colex_rank((2048,)) == -1
    with pytest.raises(P.GBSError):
        P.gbs_colex_unrank(6, 0)
    with pytest.raises(P.GBSError):
        P.gbs_colex_unrank(2, math.comb(2048, 2))


def test_invalid_arguments_rejected_on_host():
    lib = P.lib()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: the checks fail first
    assert lib.gbs_cumulants(0, fake, 1, 0, None, fake, None) == P.GBS_E_INVALID_ARG
    assert lib.gbs_cumulants(4, fake, 5, 0, None, fake, None) == P.GBS_E_INVALID_ARG
    assert lib.gbs_cumulants(10, fake, 6, 0, None, fake, None) == P.GBS_E_INVALID_ARG
    assert lib.gbs_cumulants(10, fake, 3, 32, None, fake, None) == P.GBS_E_INVALID_ARG
    assert lib.gbs_cumulants(10, None, 3, 0, None, fake, None) == P.GBS_E_INVALID_ARG
    assert lib.gbs_cumulants(10, fake, 3, 0, fake, None, None) == P.GBS_E_INVALID_ARG
    assert lib.gbs_correlators(2049, fake, 1, 0, fake, None) == P.GBS_E_INVALID_ARG
    assert lib.gbs_correlators(10, fake, 2, 0, None, None) == P.GBS_E_INVALID_ARG
    assert lib.gbs_cumulant_grad(10, fake, 3, P.GBS_MIXED, None, fake, fake, None) in (
        P.GBS_E_INVALID_ARG, P.GBS_E_UNSUPPORTED)
    assert lib.gbs_cumulant_grad(10, fake, 3, 0, None, fake, None, None) == P.GBS_E_INVALID_ARG
    assert lib.gbs_cumulants_batched(0, None, 3, 0, None) == P.GBS_E_INVALID_ARG
    # displaced states: mu required, FP64 only
    assert lib.gbs_cumulants_displaced(10, fake, None, 3, 0, None, fake, None) == \
        P.GBS_E_INVALID_ARG
    assert lib.gbs_cumulants_displaced(10, fake, fake, 6, 0, None, fake, None) == \
        P.GBS_E_INVALID_ARG
    assert lib.gbs_cumulants_displaced(10, fake, fake, 3, 0, None, None, None) == \
        P.GBS_E_INVALID_ARG
    assert lib.gbs_cumulants_displaced(10, fake, fake, 3, P.GBS_MIXED, None, fake, None) == \
        P.GBS_E_UNSUPPORTED
    # sampler: orders 3 and 5 only, mode limits, required buffers, flags
    S = lib.gbs_sample
    assert S(10, fake, 4, 8, fake, fake, None, None, 0, 0, None) == P.GBS_E_UNSUPPORTED
    assert S(10, fake, 3, -1, fake, fake, None, None, 0, 0, None) == P.GBS_E_INVALID_ARG
    assert S(4, fake, 5, 8, fake, fake, None, None, 0, 0, None) == P.GBS_E_INVALID_ARG
    assert S(257, fake, 3, 8, fake, fake, None, None, 0, 0, None) == P.GBS_E_INVALID_ARG
    assert S(201, fake, 5, 8, fake, fake, None, None, 0, 0, None) == P.GBS_E_INVALID_ARG
    assert S(10, None, 3, 8, fake, fake, None, None, 0, 0, None) == P.GBS_E_INVALID_ARG
    assert S(10, fake, 3, 8, None, fake, None, None, 0, 0, None) == P.GBS_E_INVALID_ARG
    assert S(10, fake, 3, 8, fake, None, None, None, 0, 0, None) == P.GBS_E_INVALID_ARG
    assert S(10, fake, 3, 8, fake, fake, None, None, -1, 0, None) == P.GBS_E_INVALID_ARG
    assert S(10, fake, 3, 8, fake, fake, None, None, 0, P.GBS_PARITY, None) == P.GBS_E_INVALID_ARG
    assert S(10, fake, 3, 0, None, None, None, None, 0, 0, None) == P.GBS_OK  # nothing to do
    # sample statistics
    C = lib.gbs_sample_cumulants
    assert C(0, 10, fake, 1, fake, 0, None) == P.GBS_E_INVALID_ARG
    assert C(257, 10, fake, 1, fake, 0, None) == P.GBS_E_INVALID_ARG
    assert C(10, 3, fake, 4, fake, 0, None) == P.GBS_E_INVALID_ARG  # fewer samples than the order
    assert C(10, 10, fake, 6, fake, 0, None) == P.GBS_E_INVALID_ARG
    assert C(10, 10, None, 2, fake, 0, None) == P.GBS_E_INVALID_ARG
    assert C(10, 10, fake, 2, None, 0, None) == P.GBS_E_INVALID_ARG
    assert C(10, 1 << 32, fake, 2, fake, 0, None) == P.GBS_E_INVALID_ARG
    assert lib.gbs_pearson(1, fake, fake, fake, 0, None) == P.GBS_E_INVALID_ARG
    assert lib.gbs_pearson(5, fake, None, fake, 0, None) == P.GBS_E_INVALID_ARG
    # shards: ranges inside the order, FP64 only
    Sh = lib.gbs_cumulants_shard
    assert Sh(10, fake, 3, 0, 121, 0, None, fake, None) == P.GBS_E_INVALID_ARG  # 121 > C(10, 3)
    assert Sh(10, fake, 3, 100, 21, 0, None, fake, None) == P.GBS_E_INVALID_ARG
    assert Sh(10, fake, 3, -1, 5, 0, None, fake, None) == P.GBS_E_INVALID_ARG
    assert Sh(10, fake, 3, 0, 5, 0, None, None, None) == P.GBS_E_INVALID_ARG
    assert Sh(10, fake, 6, 0, 5, 0, None, fake, None) == P.GBS_E_INVALID_ARG
    assert Sh(10, fake, 3, 0, 5, P.GBS_MIXED, None, fake, None) == P.GBS_E_UNSUPPORTED


def test_status_strings():
    for s in range(6):
        assert P.gbs_status_string(s)
    assert "unknown" in P.gbs_status_string(99)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    import paper_2511_14923_amd._binding as B
    monkeypatch.setattr(B, "_lib", None)
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        B.lib()
