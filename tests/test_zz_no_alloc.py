"""lor_build_sa_static (the allocation-free form of lor_build_sa, whose
workspace is the library's fixed per-GPU array) against lor_build_sa with a
caller workspace: two calls in a row on the same array, the second with a
smaller input, then one with the joined text left to the array. Every SA and
joined text must be identical to the workspace call's; the smallest is also
checked against the oracle."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
from paper_1404_3448_amd import lor, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True, file=sys.stderr)


def _reference(d, offsets):
    sa, joined = lor.lor_build_sa(d, offsets)
    torch.cuda.synchronize()
    return sa.cpu().numpy(), joined.cpu().numpy()


def _static(d, offsets):
    n = int(offsets[-1]) + len(offsets) - 1
    joined = torch.full((n,), 255, dtype=torch.uint8, device="cuda")
    sa = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    lor.lor_build_sa_static(d, offsets, joined, sa)
    return sa, joined


def test_static_workspace_matches_caller_workspace_on_two_calls():
    big = synth.noncoding_pair(seed=21, n=790_000, segments=4)
    small = synth.tiny_pair(seed=22, n=60_000, planted_len=300)
    assert lor.lor_suffix_array_workspace(big.joined_length) <= lor.STATIC_SCRATCH_BYTES
    db = torch.from_numpy(big.concat).cuda()
    ds = torch.from_numpy(small.concat).cuda()

    say("static call 1:", big.joined_length, "symbols")
    sa1, j1 = _static(db, big.offsets)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    say("static call 2:", small.joined_length, "symbols")
    sa2, j2 = _static(ds, small.offsets)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free1, "the static call allocated device memory"
    sa1, j1, sa2, j2 = sa1.cpu().numpy(), j1.cpu().numpy(), sa2.cpu().numpy(), j2.cpu().numpy()

    say("workspace calls")
    rsa1, rj1 = _reference(db, big.offsets)
    rsa2, rj2 = _reference(ds, small.offsets)
    assert np.array_equal(j1, rj1) and np.array_equal(sa1, rsa1)
    assert np.array_equal(j2, rj2) and np.array_equal(sa2, rsa2)
    joined = oracle.join(small.concat, small.offsets)
    assert np.array_equal(sa2, oracle.suffix_array(joined))


def test_static_workspace_keeps_joined_text_itself():
    w = synth.tiny_pair(seed=23, n=120_000, planted_len=500)
    d = torch.from_numpy(w.concat).cuda()
    n = w.joined_length
    sa = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    o = np.ascontiguousarray(w.offsets, dtype=np.int64)
    say("static call, joined text in the array:", n, "symbols")
    st = lor.lib().lor_build_sa_static(ctypes.c_void_p(d.data_ptr()), o.ctypes.data_as(ctypes.c_void_p),
                                       len(o) - 1, None, ctypes.c_void_p(sa.data_ptr()),
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == lor.LOR_OK, lor.lib().lor_last_error()
    torch.cuda.synchronize()
    rsa, _ = _reference(d, w.offsets)
    assert np.array_equal(sa.cpu().numpy(), rsa)
