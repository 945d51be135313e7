"""Results are identical under every tuning plan (a plan changes speed only)."""
import numpy as np
import pytest

import oracle
from paper_1404_3448_amd import lor, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PLANS = [
    dict(digit_bits=8, radix_items_u32=16, radix_items_u64=8, merge_items=8, plcp_steps=128),
    dict(digit_bits=6, radix_items_u32=8, radix_items_u64=8, merge_items=4, plcp_steps=16),
    dict(digit_bits=7, radix_items_u32=24, radix_items_u64=16, merge_items=12, plcp_steps=512),
    dict(digit_bits=5, radix_items_u32=12, radix_items_u64=12, merge_items=8, plcp_steps=64),
    dict(digit_bits=8, radix_items_u32=16, radix_items_u64=16, merge_items=4, plcp_steps=32),   # tuned, gfx950
    dict(digit_bits=3, radix_items_u32=24, radix_items_u64=12, merge_items=12, plcp_steps=1024),
]


@pytest.fixture
def restore_plan():
    yield
    lor.lor_plan_set(None)


@pytest.mark.parametrize("plan", range(len(PLANS)))
def test_plans_give_identical_results(plan, restore_plan):
    lor.lor_plan_set(PLANS[plan])
    w = synth.noncoding_pair(seed=31, n=200_000, segments=5)
    d = torch.from_numpy(w.concat).cuda()
    r = lor.longest_overlap_region(d, w.offsets, want_isa=True)
    joined = oracle.join(w.concat, w.offsets)
    sa = oracle.suffix_array(joined)
    lcp = oracle.lcp(joined, sa)
    assert np.array_equal(r["sa"].cpu().numpy(), sa)
    assert np.array_equal(r["lcp"].cpu().numpy(), lcp)
    assert r["overlap"] == oracle.overlap(sa, lcp, w.offsets)
    rng = np.random.default_rng(plan)
    for alphabet in (3, 70000, (1 << 29) + 3):
        t = rng.integers(1, alphabet + 1, size=5003).astype(np.int32)
        got = lor.lor_suffix_array_i32(torch.from_numpy(t).cuda(), alphabet).cpu().numpy()
        assert np.array_equal(got, oracle.suffix_array(t))
    keys = rng.integers(0, 1 << 62, size=30001, dtype=np.uint64)
    k = torch.from_numpy(keys.view(np.int64)).cuda()
    v = torch.arange(keys.size, dtype=torch.int32).cuda()
    lor.lor_sort_pairs_u64(k, v, 3, 50)
    order = np.argsort((keys >> np.uint64(3)) & np.uint64((1 << 47) - 1), kind="stable")
    assert np.array_equal(v.cpu().numpy(), order.astype(np.int32))


def test_batched_per_call_plan():
    ws = synth.batched_pairs(seed=12, num_pairs=40, lo=1e3, hi=5e4)
    seqs = [s for w in ws for s in w.seqs]
    offs = np.concatenate([[0], np.cumsum([s.size for s in seqs])]).astype(np.int64)
    d = torch.from_numpy(np.concatenate(seqs)).cuda()
    base = lor.records_to_tuples(lor.lor_longest_overlap_batched(d, offs))
    for p in PLANS[1:]:
        assert lor.records_to_tuples(lor.lor_longest_overlap_batched(d, offs, plan=p)) == base
    assert lor.lor_plan_get().as_dict() == lor.lor_plan_default().as_dict()


@pytest.mark.parametrize("digit_bits", [1, 2, 3, 5])
def test_narrow_digits_sort_identically(digit_bits):
    """Digits down to the one bit per pass of Section IV give the same stable order."""
    rng = np.random.default_rng(digit_bits)
    n = 100003
    keys = rng.integers(0, 1 << 20, size=n, dtype=np.uint64).astype(np.uint32)
    keys[rng.random(n) < 0.2] = keys[0]
    order = np.argsort(keys, kind="stable")
    saved = lor.lor_plan_get().as_dict()
    try:
        lor.lor_plan_set(dict(saved, digit_bits=digit_bits))
        k = torch.from_numpy(keys.view(np.int32)).cuda()
        v = torch.arange(n, dtype=torch.int32, device="cuda")
        lor.lor_sort_pairs_u32(k, v, 0, 20)
        assert np.array_equal(k.cpu().numpy().view(np.uint32), keys[order])
        assert np.array_equal(v.cpu().numpy(), order.astype(np.int32))
    finally:
        lor.lor_plan_set(saved)
