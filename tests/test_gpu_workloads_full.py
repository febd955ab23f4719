"""Parity at the measured sizes, in the launch configuration the benchmark times.

Medium workload: the whole step's generation (2.51e9 candidates) and its dedup-merge
into S.  Large workload: one 32,768-source mini-batch (1.18e10 candidates) streamed
in pool chunks of 2^30 into S.  The oracle computes sampled sources one by one; the
sets are checked exactly on whole key ranges against a library sort of every
candidate that falls in the range (the candidates of the large mini-batch are
regenerated chunk by chunk for that), and as sorted sets at full size.
"""
import numpy as np
import pytest
import torch

import oracle
from tests.gpu_common import H_TOL, ham, pick_sources, require_gpu, say, system

pytestmark = pytest.mark.gpu

SIGN = -(1 << 63)  # xor with this maps unsigned 64-bit order onto signed order
SLICE = 1 << 30    # boolean selection works on at most 2^31 - 1 elements at a time


def _free():
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _rows_order(w1, w0):
    """(w1, w0 ^ SIGN) compared as signed pairs: the key order of two-word keys whose
    top word is below 2^63."""
    return w1, w0 ^ SIGN


def _sort_unique_rows(a):
    """Rows (hi, lo) of signed int64, sorted lexicographically and made unique."""
    if a.shape[0] == 0:
        return a
    a = a[torch.sort(a[:, 1], stable=True).indices]
    a = a[torch.sort(a[:, 0], stable=True).indices]
    keep = torch.ones(a.shape[0], dtype=torch.bool, device=a.device)
    keep[1:] = (a[1:] != a[:-1]).any(dim=1)
    return a[keep]


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
    # exact on whole ranges: the union's keys in [u[i], u[j]) are the sorted unique
    # candidates and selected keys in that range
    R = 6
    cuts = [(r * n) // R for r in range(R + 1)]
    checked = 0
    for r in (0, 2, R - 1):
        i, j = cuts[r], cuts[r + 1]
        lo = int(u[i].item())
        hi = int(u[j].item()) if j < n else None
        parts = []
        for a in range(0, total, SLICE):
            k = keys[a:a + SLICE, 0]
            m = k >= lo if hi is None else (k >= lo) & (k < hi)
            parts.append(k[m])
        sk = sel[:, 0]
        parts.append(sk[(sk >= lo) if hi is None else (sk >= lo) & (sk < hi)])
        expect = torch.unique(torch.cat(parts), sorted=True)
        assert torch.equal(expect, u[i:j]), f"union differs in range {r}"
        checked += j - i
        del parts, expect
    say(f"  {checked} union keys checked exactly in 3 of {R} ranges")
    del keys, union, u
    _free()


def test_large_streamed_minibatch_exact_ranges():
    sci = require_gpu()
    s = system("large")
    h = ham("large")
    assert h.W == 2
    _free()
    n_src, chunk = 32768, 1 << 30
    sel = sci.keys_to_device(s.dets)
    dets = sel[:n_src]
    total = n_src * h.n_coupled
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
    # exact on three ranges of the union: regenerate every candidate of the mini-batch,
    # chunk by chunk, and keep those inside [u[i], u[j])
    ranges = []
    for f in (0.2, 0.5, 0.8):
        i = int(f * n)
        j = min(i + 3_000_000, n)
        lo = _rows_order(union[i, 1], union[i, 0])
        hi = _rows_order(union[j, 1], union[j, 0]) if j < n else None
        ranges.append((i, j, lo, hi))
    parts = [[] for _ in ranges]

    def take(k, out):
        w1, w0 = _rows_order(k[:, 1], k[:, 0])
        for (i, j, lo, hi), p in zip(ranges, out):
            m = (w1 > lo[0]) | ((w1 == lo[0]) & (w0 >= lo[1]))
            if hi is not None:
                m &= (w1 < hi[0]) | ((w1 == hi[0]) & (w0 < hi[1]))
            p.append(torch.stack([w1[m], w0[m]], dim=1))

    for a in range(0, total, chunk):
        b = min(a + chunk, total)
        k, _, _, n_k, fl = sci.gen_coupled(h, dets, exc_begin=a, exc_end=b)
        torch.cuda.synchronize()
        assert sci.check_flags(fl, "gen") == 0 and int(n_k.item()) == b - a
        for c in range(0, b - a, SLICE):
            take(k[c:c + SLICE], parts)
        del k
    take(sel, parts)
    for (i, j, _, _), p in zip(ranges, parts):
        expect = _sort_unique_rows(torch.cat(p))
        w1, w0 = _rows_order(union[i:j, 1], union[i:j, 0])
        got = torch.stack([w1, w0], dim=1)
        assert torch.equal(expect, got), f"union differs in range [{i}, {j})"
        say(f"  range [{i}, {j}): {j - i} keys exact from {sum(x.shape[0] for x in p)} candidates")
    del parts, union
    _free()
