"""Parity at the measured sizes, in the launch configuration the benchmark times.

Medium workload: the whole step's generation (2.51e9 candidates) and its dedup-merge
into S.  Large workload: one 32,768-source mini-batch (1.18e10 candidates) streamed
in the pool chunks the benchmark streams (five equal chunks of 2,367,488,000) into S.  The
oracle computes sampled sources one by one.
Every key of each union is checked: the key space is cut into ranges at union keys,
and in each range the union must equal a library sort + unique of every candidate
(and selected key) that falls in it (the large mini-batch's candidates are
regenerated chunk by chunk for that); the range counts must add up to the union's
size, and the union is strictly ascending at full size.
"""
import numpy as np
import pytest
import torch

import oracle
from tests.gpu_common import H_TOL, ham, pick_sources, require_gpu, say, system

pytestmark = pytest.mark.gpu

SIGN = -(1 << 63)  # xor with this maps unsigned 64-bit order onto signed order
SLICE = 1 << 30    # boolean selection works on at most 2^31 - 1 elements at a time
# Two-word keys are handled as two 1-D columns (top word, low word ^ SIGN): boolean
# row selections of 2-D tensors on this torch build return wrong rows once the result
# exceeds 2^27 rows (measured: every regenerated key valid, 2^27 of a 2.4e8-row
# selection not), while 1-D selections and gathers of this size are exact.
ROWS = 1 << 28     # keys per slice of the regenerated candidates


def _free():
    import gc
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _rows_order(w1, w0):
    """(w1, w0 ^ SIGN) compared as signed pairs: the key order of two-word keys whose
    top word is below 2^63."""
    return w1, w0 ^ SIGN


def _first_top_word_at_least(union, n, v):
    """Index of the first of union[:n] whose top word is >= v (the union is sorted, so
    its top words are non-decreasing); a host binary search over single elements,
    which stays exact at any size."""
    lo, hi = 0, n
    while lo < hi:
        mid = (lo + hi) // 2
        if int(union[mid, 1].item()) < v:
            lo = mid + 1
        else:
            hi = mid
    return lo


def _sort_unique_cols(h, l):
    """Pairs (h[i], l[i]) of signed int64 columns, sorted lexicographically and made
    unique; returns the two columns."""
    if h.shape[0] == 0:
        return h, l
    idx = torch.sort(l, stable=True).indices
    h, l = h[idx], l[idx]
    idx = torch.sort(h, stable=True).indices
    h, l = h[idx], l[idx]
    del idx
    keep = torch.ones(h.shape[0], dtype=torch.bool, device=h.device)
    keep[1:] = (h[1:] != h[:-1]) | (l[1:] != l[:-1])
    return h[keep], l[keep]


def _merge_cols(acc, h, l):
    """acc (two columns, sorted unique) merged with the pairs (h, l)."""
    return _sort_unique_cols(torch.cat([acc[0], h]), torch.cat([acc[1], l]))


def test_medium_full_generation_and_dedup():
    sci = require_gpu()
    s = system("medium")
    h = ham("medium")
    _free()
    sel = sci.keys_to_device(s.dets)
    n_src, N = s.dets.shape[0], h.n_coupled
    total = n_src * N
    say(f"medium full: {n_src} sources x {N} = {total} candidates")
    keys, hij, _, n_out, flags = sci.gen_coupled(h, sel)
    torch.cuda.synchronize()
    assert sci.check_flags(flags, "gen") == 0
    assert int(n_out.item()) == total
    # sampled sources, element by element against the oracle (dense order is source-major)
    rows = pick_sources(n_src, 16, 41)
    ok, oh, _ = oracle.gen_coupled(s.n_orb, s.n_alpha, s.n_beta, s.h1, s.eri, s.dets[rows])
    idx = (torch.from_numpy(rows).cuda()[:, None] * N + torch.arange(N, device="cuda")[None, :]).reshape(-1)
    assert np.array_equal(sci.keys_to_host(keys[idx]), ok)
    err = float(np.max(np.abs(hij[idx].cpu().numpy() - oh)))
    say(f"  16 sampled sources: keys exact, max |dH| = {err:.3e}")
    assert err <= H_TOL
    del hij, idx
    _free()

    union, n_union, _, _, flags = sci.dedup_merge(keys, sel, 1)
    torch.cuda.synchronize()
    assert sci.check_flags(flags, "dedup") == 0
    n = int(n_union.item())
    say(f"  union of {n} keys")
    u = union[:n, 0]  # one-word keys of 52 bits: signed order is the key order
    for a in range(0, n - 1, SLICE):
        b = min(a + SLICE + 1, n)
        assert bool((u[a + 1:b] > u[a:b - 1]).all()), "union not strictly ascending"
    # every selected determinant is in the union
    pos = torch.searchsorted(u, sel[:, 0])
    assert bool((pos < n).all()) and bool((u[pos.clamp(max=n - 1)] == sel[:, 0]).all())
    # every union key, checked exactly: the key space is cut into R ranges at union keys
    # (the first range open below, the last open above), and the union's keys in each
    # range are the sorted unique candidates and selected keys that fall in it
    R = 6
    cuts = [(r * n) // R for r in range(R + 1)]
    bounds = [None] + [int(u[cuts[r]].item()) for r in range(1, R)] + [None]
    checked = 0
    for r in range(R):
        lo, hi = bounds[r], bounds[r + 1]

        def inside(k):
            m = torch.ones_like(k, dtype=torch.bool)
            if lo is not None:
                m &= k >= lo
            if hi is not None:
                m &= k < hi
            return m

        parts = []
        for a in range(0, total, SLICE):
            k = keys[a:a + SLICE, 0]
            parts.append(k[inside(k)])
        sk = sel[:, 0]
        parts.append(sk[inside(sk)])
        expect = torch.unique(torch.cat(parts), sorted=True)
        i, j = cuts[r], cuts[r + 1]
        assert torch.equal(expect, u[i:j]), f"union differs in range {r}"
        checked += expect.shape[0]
        del parts, expect
    assert checked == n, f"ranges hold {checked} unique keys, the union {n}"
    say(f"  all {n} union keys checked exactly in {R} ranges")
    del keys, union, u
    _free()


def test_large_streamed_minibatch_exact_ranges():
    sci = require_gpu()
    s = system("large")
    h = ham("large")
    assert h.W == 2
    _free()
    n_src = 32768
    sel = sci.keys_to_device(s.dets)
    dets = sel[:n_src]
    total = n_src * h.n_coupled
    # the pool chunk the benchmark streams: the fewest equal chunks of at most 2.4e9
    chunk = -(-total // -(-total // 2_400_000_000))
    cap = 3_300_000_000
    say(f"large mini-batch: {total} candidates, chunks of {chunk}, set capacity {cap}")
    union, n_union, flags = sci.stream_dedup(h, dets, chunk, sel, cap, dedup_stream=torch.cuda.Stream())
    torch.cuda.synchronize()
    assert sci.check_flags(flags, "stream") == 0
    n = int(n_union.item())
    say(f"  union of {n} keys")
    assert s.dets.shape[0] <= n <= cap
    _free()
    # strictly ascending at full size (top words hold 56 bits)
    for a in range(0, n - 1, SLICE):
        b = min(a + SLICE + 1, n)
        h1, l1 = _rows_order(union[a:b, 1], union[a:b, 0])
        up = (h1[1:] > h1[:-1]) | ((h1[1:] == h1[:-1]) & (l1[1:] > l1[:-1]))
        assert bool(up.all()), "union not strictly ascending"
        del h1, l1, up
    # every union key, checked exactly.  The key space is cut into ranges at top-word
    # values of union keys (the key order is the top word first), so a candidate's
    # range follows from its top word alone; the union's keys of one range are a
    # contiguous slice.  Per group of ranges, every candidate of the mini-batch is
    # regenerated chunk by chunk and those of the group's ranges are kept; each range
    # is then sorted and made unique by the library sort and compared with its slice.
    R = 16
    cuts = sorted(set(int(union[(r * n) // R, 1].item()) for r in range(1, R)))
    hb = torch.tensor(cuts, dtype=torch.int64, device="cuda")
    n_ranges = len(cuts) + 1
    starts = [_first_top_word_at_least(union, n, v) for v in cuts]
    slices = list(zip([0] + starts, starts + [n]))
    sel_ids = torch.searchsorted(hb, sel[:, 1].contiguous(), right=True)
    G = 4
    checked = 0
    for g0 in range(0, n_ranges, G):
        group = list(range(g0, min(g0 + G, n_ranges)))
        # each range's distinct keys so far (its selected keys to start with), merged
        # with every chunk's candidates in the range as the chunks are regenerated:
        # memory stays near the range's share of the union
        acc = {}
        s1, s0 = _rows_order(sel[:, 1].contiguous(), sel[:, 0].contiguous())
        for r in group:
            m = sel_ids == r
            acc[r] = _sort_unique_cols(s1[m], s0[m])
        seen = {r: 0 for r in group}
        for a in range(0, total, chunk):
            b = min(a + chunk, total)
            k, _, _, n_k, fl = sci.gen_coupled(h, dets, exc_begin=a, exc_end=b)
            torch.cuda.synchronize()
            assert sci.check_flags(fl, "gen") == 0 and int(n_k.item()) == b - a
            for c in range(0, b - a, ROWS):
                k1, k0 = _rows_order(k[c:c + ROWS, 1].contiguous(), k[c:c + ROWS, 0].contiguous())
                ids = torch.searchsorted(hb, k1, right=True)
                for r in group:
                    m = ids == r
                    p1, p0 = k1[m], k0[m]
                    seen[r] += p1.shape[0]
                    acc[r] = _merge_cols(acc[r], p1, p0)
                    del m, p1, p0
                del ids, k1, k0
            del k
            _free()
        for r in group:
            e1, e0 = acc.pop(r)
            i, j = slices[r]
            u1, u0 = _rows_order(union[i:j, 1], union[i:j, 0])
            assert torch.equal(e1, u1) and torch.equal(e0, u0), f"union differs in range {r} [{i}, {j})"
            checked += e1.shape[0]
            say(f"  range {r} [{i}, {j}): {j - i} keys exact from {seen[r]} candidates")
            del e1, e0, u1, u0
            _free()
    assert checked == n, f"ranges hold {checked} unique keys, the union {n}"
    say(f"  all {n} union keys checked exactly in {n_ranges} ranges")
    _free()
    # reverse index at this size: a hash table would take sci_index_bytes (2^33 slots of
    # 32 bytes, 275 GB), so the index is of the sorted kind (every 256th key sampled)
    n_dev = torch.tensor([n], dtype=torch.int64, device="cuda")
    table_bytes = sci.sci_index_bytes(2, n)
    index, fl = sci.build_index(union, n_dev, n, 2)
    assert sci.index_kind(index) == "sorted" and table_bytes > 2 * 10**11
    say(f"  reverse index: sorted kind, {index.numel()} bytes (a table would take {table_bytes})")
    # every candidate of the first chunk is found, at a position holding its key
    k, _, _, _, _ = sci.gen_coupled(h, dets, exc_begin=0, exc_end=chunk)
    idx = sci.inverse_map(index, k, 2)
    torch.cuda.synchronize()
    assert sci.check_flags(fl, "index") == 0
    assert bool((idx >= 0).all()), "a generated candidate is missing from the index"
    # gathers read from union slices of 2^28 keys (a gather from the whole set buffer,
    # 6.6e9 elements, is refused by this torch build's index kernel)
    for c in range(0, chunk, 1 << 26):
        ic = idx[c:c + (1 << 26)]
        k1, k0 = k[c:c + (1 << 26), 1].contiguous(), k[c:c + (1 << 26), 0].contiguous()
        for u0 in range(0, n, 1 << 28):
            u1 = min(u0 + (1 << 28), n)
            m = (ic >= u0) & (ic < u1)
            part = union[u0:u1]
            j = ic[m] - u0
            assert torch.equal(part[:, 1][j], k1[m]) and torch.equal(part[:, 0][j], k0[m])
            del m, part, j
        del ic, k1, k0
    del k, idx
    _free()
    # against the oracle on one range's slice of the union: members at random positions
    # and the same keys with their lowest bit flipped (same top word, so same range)
    i, j = slices[n_ranges // 2]
    rng = np.random.Generator(np.random.PCG64(2604157690))
    pos = torch.from_numpy(rng.integers(0, j - i, size=500_000)).cuda()
    members = union[i:j][pos]
    flipped = members.clone()
    flipped[:, 0] ^= 1
    cand = torch.cat([members, flipped])
    got = sci.inverse_map(index, cand, 2).cpu().numpy()
    u_slice = sci.keys_to_host(union[i:j])
    want = oracle.inverse_map(2, u_slice, sci.keys_to_host(cand))
    want = np.where(want >= 0, want + i, -1)
    assert np.array_equal(got, want), "sorted reverse index differs from the oracle"
    say(f"  1e6 lookups in [{i}, {j}) equal the oracle ({int((want >= 0).sum())} found)")
    del union, index, u_slice
    _free()


def _strictly_ascending_rows(union, n):
    for a in range(0, n - 1, SLICE):
        b = min(a + SLICE + 1, n)
        h1, l1 = _rows_order(union[a:b, 1], union[a:b, 0])
        up = (h1[1:] > h1[:-1]) | ((h1[1:] == h1[:-1]) & (l1[1:] > l1[:-1]))
        if not bool(up.all()):
            return False
        del h1, l1, up
    return True


def test_large_whole_selected_space_streamed():
    """All 200,000 sources of the large workload (7.2e10 candidates) streamed in pool
    chunks of 2^29 into one set on one GPU.  Checked at full size: no overflow, strictly
    ascending; and exactly on two sampled key ranges (cut at top-word
    values of union keys) against a library sort + unique of every candidate of the
    whole stream that falls in them, regenerated chunk by chunk."""
    sci = require_gpu()
    s = system("large")
    h = ham("large")
    _free()
    sel = sci.keys_to_device(s.dets)
    n_src, chunk = sel.shape[0], 1 << 29
    total = n_src * h.n_coupled
    cap = 5_600_000_000
    say(f"large, whole S: {total} candidates, chunks of {chunk}, set capacity {cap}")
    union, n_union, flags = sci.stream_dedup(h, sel, chunk, sel, cap, dedup_stream=torch.cuda.Stream())
    torch.cuda.synchronize()
    assert sci.check_flags(flags, "stream") == 0
    n = int(n_union.item())
    say(f"  union of {n} keys")
    assert s.dets.shape[0] <= n <= cap
    _free()
    assert _strictly_ascending_rows(union, n), "union not strictly ascending"
    # two sampled ranges of about 4e7 union keys, cut at top-word values
    ranges = []
    for f in (0.3, 0.7):
        i0 = int(f * n)
        lo_v = int(union[i0, 1].item())
        hi_v = int(union[min(i0 + 40_000_000, n - 1), 1].item())
        if hi_v == lo_v:
            hi_v = lo_v + 1
        ranges.append((lo_v, hi_v, _first_top_word_at_least(union, n, lo_v), _first_top_word_at_least(union, n, hi_v)))
    # each range's distinct keys, merged with every chunk's candidates in it as the
    # chunks are regenerated
    empty = sel.new_empty(0)
    acc = [(empty, empty) for _ in ranges]
    seen = [0 for _ in ranges]

    def take(k_all):
        for c in range(0, k_all.shape[0], ROWS):
            k1, k0 = _rows_order(k_all[c:c + ROWS, 1].contiguous(), k_all[c:c + ROWS, 0].contiguous())
            for q, (lo, hi_, _, _) in enumerate(ranges):
                m = (k1 >= lo) & (k1 < hi_)
                p1, p0 = k1[m], k0[m]
                seen[q] += p1.shape[0]
                acc[q] = _merge_cols(acc[q], p1, p0)
                del m, p1, p0
            del k1, k0

    for a in range(0, total, chunk):
        b = min(a + chunk, total)
        k, _, _, n_k, fl = sci.gen_coupled(h, sel, exc_begin=a, exc_end=b)
        assert int(n_k.item()) == b - a
        take(k)
        del k
    torch.cuda.synchronize()
    assert sci.check_flags(fl, "gen") == 0
    take(sel)
    for q, (lo, hi_, i, j) in enumerate(ranges):
        e1, e0 = acc[q]
        u1, u0 = _rows_order(union[i:j, 1], union[i:j, 0])
        assert torch.equal(e1, u1) and torch.equal(e0, u0), f"union differs in [{i}, {j})"
        say(f"  range [{i}, {j}): {j - i} keys exact from {seen[q]} candidates")
        del e1, e0, u1, u0
        _free()
    del acc, union
    _free()
