"""Ablation of the paper's radix-sort design choices on MI355X.

Section IV sorts DC3's sample triples with its own kernel design (Alg. 1):
every thread block sorts one chunk with a split of one bit per pass, and the
sorted chunks are then merged. Table V times that sort for inputs whose size
is or is not a multiple of the warp size (32 on the paper's GPU). This
measures, on the level-0 sample keys of a noncoding-like text (15-bit packed
triples of 5-bit symbols):

* the paper's design (lor_sort_pairs_split_u32: 2048-key chunks, 15 one-bit
  splits in LDS, then pairwise merges of sorted runs) against this library's
  digit sort (lor_sort_pairs_u32), both checked against numpy's stable sort;
* digit width: the library's sort with 1-, 2-, 4- and 8-bit digits;
* size alignment: both sorts at sizes that are and are not multiples of the
  wavefront (64 lanes), of the chunk and of the sort tile.

    python -m paper_1404_3448_amd.ablation      # prints one JSON object
"""
from __future__ import annotations

import json
import time

import numpy as np

from . import lor, synth


def sample_keys(n_text: int, seed: int = 3) -> np.ndarray:
    """Packed triples (t_i, t_{i+1}, t_{i+2}) of 5-bit symbols (base + 1,
    end of text 0) for the positions i mod 3 != 0 of one noncoding-like
    sequence followed by its separator (symbol 5)."""
    rng = synth.rng_for(seed)
    t = np.concatenate([synth.noncoding_like(rng, n_text - 1) + 1, [5]]).astype(np.uint32)
    t = np.concatenate([t, [0, 0]])
    pos = np.arange(n_text)
    pos = pos[pos % 3 != 0]
    return ((t[pos] << 10) | (t[pos + 1] << 5) | t[pos + 2]).astype(np.uint32)


def _time_sort(keys_d, vals_d, kk, vv, ws, bits: int, reps: int = 5, fn=None) -> float:
    import torch
    fn = fn or lor.lor_sort_pairs_u32
    ts = []
    for _ in range(reps + 1):
        kk.copy_(keys_d)
        vv.copy_(vals_d)
        torch.cuda.synchronize()
        t = time.perf_counter()
        fn(kk, vv, 0, bits, ws=ws)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
    return float(np.median(ts[1:]))


def run(n_text: int = 3 * (1 << 23)) -> dict:
    import torch
    dev = torch.device("cuda:0")
    saved = lor.lor_plan_get().as_dict()
    keys = sample_keys(n_text)
    n = keys.size
    kd = torch.from_numpy(keys.view(np.int32)).to(dev)
    vd = torch.arange(n, dtype=torch.int32, device=dev)
    kk, vv = torch.empty_like(kd), torch.empty_like(vd)
    ws = torch.empty(lor.lor_sort_pairs_workspace(n, 4), dtype=torch.uint8, device=dev)
    out = {"workload": f"level-0 sample keys of a {n_text}-base noncoding-like text: {n} 15-bit keys",
           "paper_split_radix": {}, "digit_width": {}, "size_alignment": {}}
    want = np.argsort(keys, kind="stable").astype(np.int32)
    ref = None
    try:
        t = _time_sort(kd, vd, kk, vv, ws, 15, fn=lor.lor_sort_pairs_split_u32)
        same = bool(np.array_equal(vv.cpu().numpy(), want))
        merges = max(0, int(np.ceil(np.log2(max(1, -(-n // 2048))))))
        out["paper_split_radix"] = {"design": "2048-key chunks, one-bit splits in LDS, pairwise merges of runs",
                                    "splits": 15, "merge_passes": merges, "ms": round(1e3 * t, 3),
                                    "Mkeys_per_s": round(n / t / 1e6, 1),
                                    "same_result_as_stable_argsort": same}
        for d in (1, 2, 4, 8):
            lor.lor_plan_set(dict(saved, digit_bits=d))
            t = _time_sort(kd, vd, kk, vv, ws, 15)
            got = (kk.cpu().numpy(), vv.cpu().numpy())
            same = (np.array_equal(got[1], want) and
                    (ref is None or (np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]))))
            ref = ref or got
            out["digit_width"][f"{d}-bit"] = {"passes": -(-15 // d), "ms": round(1e3 * t, 3),
                                              "Mkeys_per_s": round(n / t / 1e6, 1), "same_result": bool(same)}
        lor.lor_plan_set(saved)
        tile = 256 * int(saved["radix_items_u32"])
        base = (n // tile) * tile
        for label, m in (("tile multiple", base), ("+1", base + 1), ("wave multiple, not tile", base - tile + 64),
                         ("-1", base - 1)):
            t = _time_sort(kd[:m], vd[:m], kk[:m], vv[:m], ws, 15)
            ts = _time_sort(kd[:m], vd[:m], kk[:m], vv[:m], ws, 15, fn=lor.lor_sort_pairs_split_u32)
            out["size_alignment"][label] = {"n": m, "wave_multiple": m % 64 == 0, "ms": round(1e3 * t, 3),
                                            "Mkeys_per_s": round(m / t / 1e6, 1),
                                            "paper_split_ms": round(1e3 * ts, 3),
                                            "paper_split_Mkeys_per_s": round(m / ts / 1e6, 1)}
    finally:
        lor.lor_plan_set(saved)
    return out


if __name__ == "__main__":
    print(json.dumps(run()))
