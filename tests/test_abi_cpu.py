"""The C-ABI library loads, exports every function include/lor.h declares,
and rejects bad arguments on the host. No GPU needed: every call here returns
before any device work is enqueued."""
import ctypes

import numpy as np
import pytest

from paper_1404_3448_amd import lor


@pytest.fixture(scope="module")
def L():
    return lor.lib()


def test_exports_every_declared_function(L):
    names = lor.header_functions()
    assert len(names) >= 20
    for name in names:
        assert hasattr(L, name), name


def test_version_and_status_strings(L):
    assert L.lor_version() == 1
    for s in range(7):
        assert L.lor_status_string(s)
    assert L.lor_status_string(99) == b"unknown status"


FAKE = ctypes.c_void_p(1 << 20)        # never dereferenced: validation fails first


def offsets(*xs):
    o = np.array(xs, dtype=np.int64)
    return o, o.ctypes.data_as(ctypes.c_void_p)


def test_build_sa_argument_errors(L):
    o, op = offsets(0, 5, 9)
    ws = lor.lor_build_sa_workspace(9, 2)
    assert ws > 0
    assert L.lor_build_sa(FAKE, op, 0, None, FAKE, FAKE, ws, None) == lor.LOR_EINVAL        # num_seqs 0
    assert L.lor_build_sa(FAKE, op, 252, None, FAKE, FAKE, ws, None) == lor.LOR_EINVAL      # > 251
    bad, bp = offsets(0, 5, 3)
    assert L.lor_build_sa(FAKE, bp, 2, None, FAKE, FAKE, ws, None) == lor.LOR_EINVAL
    assert b"decrease" in L.lor_last_error()
    bad0, b0 = offsets(1, 5, 9)
    assert L.lor_build_sa(FAKE, b0, 2, None, FAKE, FAKE, ws, None) == lor.LOR_EINVAL
    assert L.lor_build_sa(FAKE, op, 2, None, None, FAKE, ws, None) == lor.LOR_EINVAL         # sa_out NULL
    assert L.lor_build_sa(FAKE, op, 2, None, FAKE, FAKE, ws - 1, None) == lor.LOR_EWORKSPACE
    assert L.lor_build_sa(FAKE, op, 2, None, FAKE, ctypes.c_void_p((1 << 20) + 8), ws, None) == lor.LOR_EINVAL
    assert L.lor_build_sa(FAKE, op, 2, ctypes.c_void_p((1 << 20) + 1), FAKE, FAKE, ws, None) == lor.LOR_EINVAL
    big, gp = offsets(0, 1 << 30, (1 << 31) - 2)
    assert L.lor_build_sa(FAKE, gp, 2, None, FAKE, FAKE, ws, None) == lor.LOR_ETOOLARGE


def test_other_argument_errors(L):
    assert L.lor_suffix_array_i32(FAKE, 10, 0, FAKE, FAKE, 1 << 30, None) == lor.LOR_EINVAL
    assert L.lor_suffix_array_i32(FAKE, 1 << 31, 4, FAKE, FAKE, 1 << 30, None) == lor.LOR_ETOOLARGE
    assert L.lor_suffix_array_i32(FAKE, 10, 4, FAKE, FAKE, 16, None) == lor.LOR_EWORKSPACE
    assert L.lor_build_lcp(None, 10, FAKE, FAKE, None, FAKE, 1 << 30, None) == lor.LOR_EINVAL
    assert L.lor_build_lcp(FAKE, 10, FAKE, FAKE, None, FAKE, 8, None) == lor.LOR_EWORKSPACE
    h = lor.lor_rmq()
    assert L.lor_rmq_build(FAKE, 100, FAKE, 8, ctypes.byref(h), None) == lor.LOR_EWORKSPACE
    assert L.lor_rmq_query(ctypes.byref(h), FAKE, FAKE, 2, FAKE, FAKE, 5, FAKE, None, None) == lor.LOR_EINVAL
    h.n = 100
    h.levels = 3                                    # floor(log2 100) = 6
    h.table = 1 << 20
    assert L.lor_rmq_query(ctypes.byref(h), FAKE, FAKE, 1, FAKE, FAKE, 5, FAKE, None, None) == lor.LOR_ESTALE
    assert L.lor_rmq_query(ctypes.byref(h), FAKE, None, 1, FAKE, FAKE, 5, FAKE, None, None) == lor.LOR_EINVAL
    o, op = offsets(0, 4, 8)
    out = lor.lor_overlap()
    assert L.lor_longest_overlap(FAKE, FAKE, 9, op, 2, ctypes.byref(out), FAKE, 1 << 20, None) == lor.LOR_EINVAL
    assert L.lor_longest_overlap(FAKE, FAKE, 10, op, 2, ctypes.byref(out), FAKE, 8, None) == lor.LOR_EWORKSPACE
    assert L.lor_sort_pairs_u32(FAKE, FAKE, 10, 5, 5, FAKE, 1 << 20, None) == lor.LOR_EINVAL
    assert L.lor_sort_pairs_u32(FAKE, FAKE, 10, 0, 33, FAKE, 1 << 20, None) == lor.LOR_EINVAL
    assert L.lor_sort_pairs_u64(FAKE, FAKE, 10, 0, 64, FAKE, 16, None) == lor.LOR_EWORKSPACE


def test_size_queries():
    n = (1 << 30) + 16
    hdr = 64                                              # header words (the largest LCP value, width)
    assert lor.lor_rmq_bytes(1) == 0
    assert lor.lor_rmq_bytes(2) == 4 * (hdr + 1)          # one level, one window
    assert lor.lor_rmq_bytes(5) == 4 * (hdr + (5 - 1) + (5 - 3))
    levels = n.bit_length() - 1
    assert lor.lor_rmq_bytes(n) == 4 * (hdr + sum(n - (1 << k) + 1 for k in range(1, levels + 1)))
    # the DC3 workspace grows linearly (a bound of the level footprints)
    a = lor.lor_build_sa_workspace(1 << 20, 2)
    b = lor.lor_build_sa_workspace(1 << 24, 2)
    assert 10 < b / a < 20
    assert lor.lor_build_sa_workspace(1 << 30, 16) < 40 * (1 << 30)
    assert lor.lor_build_sa_workspace((1 << 31), 2) == 0
    assert lor.lor_build_lcp_workspace(1000) >= 4000
    assert lor.lor_sort_pairs_workspace(1000, 3) == 0


def test_plan_validation():
    assert lor.lor_plan_get().as_dict() == lor.lor_plan_default().as_dict()
    lor.lor_plan_set({"digit_bits": 6, "merge_items": 4})
    assert lor.lor_plan_get().digit_bits == 6
    for bad in ({"digit_bits": 9}, {"digit_bits": 0}, {"radix_items_u32": 10}, {"radix_items_u64": 24}, {"radix_items_u64": 4}, {"merge_items": 16},
                {"plcp_steps": 4}):
        with pytest.raises(lor.LorError):
            lor.lor_plan_set(bad)
    lor.lor_plan_set(None)
    assert lor.lor_plan_get().as_dict() == lor.lor_plan_default().as_dict()
    # workspace sizes do not depend on the plan
    a = lor.lor_build_sa_workspace(1 << 20, 2)
    lor.lor_plan_set({"merge_items": 4, "digit_bits": 4})
    assert lor.lor_build_sa_workspace(1 << 20, 2) == a
    lor.lor_plan_set(None)


def test_graph_argument_errors(L):
    o, op = offsets(0, 5, 9)
    h = ctypes.c_void_p()
    ws = lor.lor_longest_overlap_batched_workspace(9, 1)
    # the null stream cannot be captured
    assert L.lor_longest_overlap_batched_graph_create(FAKE, op, 1, None, FAKE, FAKE, ws, None,
                                                      ctypes.byref(h)) == lor.LOR_EINVAL
    assert b"null stream" in L.lor_last_error()
    assert L.lor_longest_overlap_batched_graph_create(FAKE, op, 1, None, FAKE, FAKE, ws, FAKE, None) == lor.LOR_EINVAL
    assert L.lor_longest_overlap_batched_graph_create(FAKE, op, 0, None, FAKE, FAKE, ws, FAKE,
                                                      ctypes.byref(h)) == lor.LOR_EINVAL
    assert L.lor_longest_overlap_batched_graph_create(FAKE, op, 1, None, FAKE, FAKE, ws - 1, FAKE,
                                                      ctypes.byref(h)) == lor.LOR_EWORKSPACE
    assert not h.value
    assert L.lor_longest_overlap_batched_graph_launch(None, None) == lor.LOR_EINVAL
    assert L.lor_longest_overlap_batched_graph_status(None, None) == lor.LOR_EINVAL
    assert L.lor_longest_overlap_batched_graph_levels(None) == -1
    L.lor_longest_overlap_batched_graph_destroy(None)


def test_rmq_compact_sizes_and_handles(L):
    def expect(n):
        nb = -(-n // 64)
        levels = nb.bit_length() - 1 if nb >= 2 else 0
        return 4 * (nb + sum(nb - (1 << k) + 1 for k in range(1, levels + 1)))
    for n in (1, 2, 63, 64, 65, 129, 4097, 100003, (1 << 30) + 16, (1 << 31) - 1):
        assert lor.lor_rmq_compact_bytes(n) == expect(n), n
    assert lor.lor_rmq_compact_bytes(0) == 0
    n = (1 << 30) + 16
    assert lor.lor_rmq_compact_bytes(n) * 60 < lor.lor_rmq_bytes(n)       # the point of the variant
    h = lor.lor_rmq()
    assert L.lor_rmq_compact_build(FAKE, 100, FAKE, 8, ctypes.byref(h), None) == lor.LOR_EWORKSPACE
    h.n, h.table, h.kind = 100000, 1 << 20, 1
    h.levels = 3                                    # ceil(100000/64) = 1563 blocks: 10 levels
    assert L.lor_rmq_query(ctypes.byref(h), FAKE, FAKE, 0, FAKE, FAKE, 5, FAKE, None, None) == lor.LOR_ESTALE
    h.kind = 2
    h.levels = 10
    assert L.lor_rmq_query(ctypes.byref(h), FAKE, FAKE, 0, FAKE, FAKE, 5, FAKE, None, None) == lor.LOR_ESTALE


def test_ref_queries_argument_errors(L):
    o, op = offsets(0, 10, 14, 20)        # reference + 2 queries
    ws = lor.lor_longest_overlap_ref_workspace(20, 2)
    assert ws > 0
    assert L.lor_longest_overlap_ref(FAKE, op, 0, FAKE, FAKE, ws, None) == lor.LOR_EINVAL
    bad, bp = offsets(0, 10, 9, 20)
    assert L.lor_longest_overlap_ref(FAKE, bp, 2, FAKE, FAKE, ws, None) == lor.LOR_EINVAL
    assert L.lor_longest_overlap_ref(FAKE, op, 2, None, FAKE, ws, None) == lor.LOR_EINVAL
    assert L.lor_longest_overlap_ref(FAKE, op, 2, FAKE, FAKE, ws - 1, None) == lor.LOR_EWORKSPACE
    big, gp = offsets(0, 1 << 30, (1 << 31) - 2, (1 << 31) - 2)
    assert L.lor_longest_overlap_ref(FAKE, gp, 2, FAKE, FAKE, ws, None) == lor.LOR_ETOOLARGE
    assert lor.lor_longest_overlap_ref_workspace(-1, 2) == 0
    assert lor.lor_longest_overlap_ref_workspace(20, 0) == 0


def test_matrix_argument_errors(L):
    o, op = offsets(0, 5, 9)
    ws = lor.lor_overlap_matrix_workspace(11, 2)
    assert ws > 0
    assert L.lor_overlap_matrix(FAKE, FAKE, 12, op, 2, FAKE, FAKE, ws, None) == lor.LOR_EINVAL     # n != 9 + 2
    assert L.lor_overlap_matrix(FAKE, FAKE, 11, op, 0, FAKE, FAKE, ws, None) == lor.LOR_EINVAL
    assert L.lor_overlap_matrix(FAKE, FAKE, 11, op, 2, None, FAKE, ws, None) == lor.LOR_EINVAL
    assert L.lor_overlap_matrix(FAKE, FAKE, 11, op, 2, FAKE, FAKE, ws - 1, None) == lor.LOR_EWORKSPACE
    assert lor.lor_overlap_matrix_workspace(11, 252) == 0


def test_build_sa_static_size_and_argument_errors(L):
    import re
    with open(lor.HEADER_PATH) as f:
        m = re.search(r"#define LOR_STATIC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", f.read())
    assert m and int(m.group(1)) << int(m.group(2)) == lor.STATIC_SCRATCH_BYTES
    o, op = offsets(0, 5, 9)
    assert L.lor_build_sa_static(FAKE, op, 0, None, FAKE, None) == lor.LOR_EINVAL
    bad, bp = offsets(0, 5, 3)
    assert L.lor_build_sa_static(FAKE, bp, 2, None, FAKE, None) == lor.LOR_EINVAL
    # the largest joined length whose workspace fits, with the joined text given
    lo, hi = 1, 1 << 24
    while lo < hi:
        mid = (lo + hi + 1) // 2
        lo, hi = (mid, hi) if lor.lor_suffix_array_workspace(mid) <= lor.STATIC_SCRATCH_BYTES else (lo, mid - 1)
    assert 1_500_000 < lo < 2_100_000
    big, gp = offsets(0, lo - 1, lo - 1)   # joined length lo + 1: one symbol too many
    assert L.lor_build_sa_static(FAKE, gp, 2, FAKE, FAKE, None) == lor.LOR_ETOOLARGE
    assert b"static workspace" in L.lor_last_error()
    fits, fp = offsets(0, lo - 2, lo - 2)
    assert lor.lor_suffix_array_workspace(lo) <= lor.STATIC_SCRATCH_BYTES
    # without joined_out the joined text also needs room in the array
    assert L.lor_build_sa_static(FAKE, fp, 2, None, FAKE, None) == lor.LOR_ETOOLARGE


def test_batched_state_argument_errors(L):
    o, op = offsets(0, 5, 9)
    ws = lor.lor_longest_overlap_batched_workspace(9, 1)
    assert L.lor_longest_overlap_batched_state(FAKE, op, 1, None, FAKE, None, FAKE, FAKE, ws, None) == lor.LOR_EINVAL
    assert L.lor_longest_overlap_batched_state(FAKE, op, 1, None, FAKE, FAKE, None, FAKE, ws, None) == lor.LOR_EINVAL
    assert b"lcp_out" in L.lor_last_error()
    assert L.lor_longest_overlap_batched_state(FAKE, op, 1, None, FAKE, FAKE, FAKE, FAKE, ws - 1, None) == \
        lor.LOR_EWORKSPACE
    assert L.lor_longest_overlap_batched_state(FAKE, op, 0, None, FAKE, FAKE, FAKE, FAKE, ws, None) == lor.LOR_EINVAL
    assert list(lor.pair_starts([0, 5, 9, 9, 12])) == [0, 11, 16]


def test_lor_check_argument_errors(L):
    assert L.lor_check(None, None) == lor.LOR_EINVAL
    assert L.lor_check(ctypes.c_void_p((1 << 20) + 8), None) == lor.LOR_EINVAL
    assert L.lor_status_string(lor.LOR_ESTALE).startswith(b"stale")
