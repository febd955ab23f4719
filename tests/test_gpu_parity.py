"""GPU parity: HIP path (through the C ABI binding) vs the CPU oracle.

Bar: keys, sources and sets bit-exact; H_ij within 1e-12 Ha; E within 1e-10 Ha;
gradient within 1e-10 per component.
"""
import numpy as np
import pytest
import torch  # imported at collection: the first import on a fresh box is slow

import oracle
import sci_inputs as si
from tests.gpu_common import E_TOL, G_TOL, H_TOL, ham, pick_sources, require_gpu, say, system

pytestmark = pytest.mark.gpu


def _gen(sci, h, dets_np, **kw):
    import torch
    d = sci.keys_to_device(dets_np)
    keys, hij, src, n_out, flags = sci.gen_coupled(h, d, **kw)
    torch.cuda.synchronize()
    return keys, hij, src, n_out, flags


# ---------------------------------------------------------------------------
# generation
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name,n_src", [("tiny", None), ("medium", 48), ("large", 12)])
def test_gen_dense_matches_oracle(name, n_src):
    sci = require_gpu()
    s = system(name)
    h = ham(name)
    dets = s.dets if n_src is None else s.dets[pick_sources(s.dets.shape[0], n_src, 7)]
    say(f"gen dense {name}: {dets.shape[0]} sources x {h.n_coupled}")
    keys, hij, src, n_out, flags = _gen(sci, h, dets, with_src=True)
    assert sci.check_flags(flags, "gen") == 0
    assert int(n_out.item()) == dets.shape[0] * h.n_coupled
    ok, oh, osrc = oracle.gen_coupled(s.n_orb, s.n_alpha, s.n_beta, s.h1, s.eri, dets)
    gk = sci.keys_to_host(keys)
    assert np.array_equal(gk, ok), "coupled determinants differ"
    assert np.array_equal(src.cpu().numpy(), osrc)
    gh = hij.cpu().numpy()
    err = np.max(np.abs(gh - oh))
    say(f"  max |dH| = {err:.3e}, exact fraction = {np.mean(gh == oh):.4f}")
    assert err <= H_TOL
    # signs are exact: any sign flip shows as |dH| = 2|H|
    assert np.all(np.sign(gh[np.abs(oh) > 1e-9]) == np.sign(oh[np.abs(oh) > 1e-9]))


def test_gen_chunked_ranges_equal_full():
    """Arbitrary [exc_begin, exc_end) windows, across source boundaries, equal the full output."""
    sci = require_gpu()
    s = system("medium")
    h = ham("medium")
    dets = s.dets[:7]
    full_k, full_h, _, _, _ = _gen(sci, h, dets)
    total = 7 * h.n_coupled
    rng = np.random.Generator(np.random.PCG64(3))
    cuts = sorted(set([0, total, 1, total - 1, h.n_coupled, 2 * h.n_coupled + 5] +
                      rng.integers(0, total, 6).tolist()))
    for a, b in zip(cuts[:-1], cuts[1:]):
        k, hh, _, n_out, flags = _gen(sci, h, dets, exc_begin=a, exc_end=b)
        assert int(n_out.item()) == b - a
        assert np.array_equal(sci.keys_to_host(k), sci.keys_to_host(full_k[a:b]))
        assert np.array_equal(hh.cpu().numpy(), full_h[a:b].cpu().numpy())


def _srckey(src, keys):
    """(source, key words) rows as a structured int64 array: sorting it orders the rows
    lexicographically, so two multisets compare equal exactly when their sorts do."""
    m = np.ascontiguousarray(np.concatenate([np.asarray(src, dtype=np.int64)[:, None], keys.view(np.int64)], axis=1))
    return m.view([(f"f{i}", np.int64) for i in range(m.shape[1])]).ravel()


def _screened_check(sci, h, n_orb, na, nb, h1, eri, dets, quantile=0.87):
    """Screened generation (|H| > eps kept, compacted in any order) against the oracle's
    dense output filtered by the same rule, compared as (source, key) multisets with
    the values matched entry by entry; entries within 1e-12 of eps are left out on
    both sides (rounding may decide them either way).  Then the overflow case:
    capacity below the kept count."""
    ok, oh, _ = oracle.gen_coupled(n_orb, na, nb, h1, eri, dets)
    eps = float(np.quantile(np.abs(oh), quantile))
    keys, hij, src, n_out, flags = _gen(sci, h, dets, eps=eps)
    assert sci.check_flags(flags, "gen") == 0
    n = int(n_out.item())
    osrc = np.repeat(np.arange(dets.shape[0]), h.n_coupled)
    border = np.abs(np.abs(oh) - eps) < 1e-12
    keep = (np.abs(oh) > eps) & ~border
    g = _srckey(src[:n].cpu().numpy(), sci.keys_to_host(keys[:n]))
    gh = hij[:n].cpu().numpy()
    order = np.argsort(g, kind="stable")
    g, gh = g[order], gh[order]
    b = np.sort(_srckey(osrc[border], ok[border]))
    if b.shape[0]:
        i = np.minimum(np.searchsorted(b, g), b.shape[0] - 1)
        g_keep = ~(b[i] == g)
        g, gh = g[g_keep], gh[g_keep]
    want = _srckey(osrc[keep], ok[keep])
    worder = np.argsort(want, kind="stable")
    want, want_h = want[worder], oh[keep][worder]
    say(f"  eps={eps:.4e}: kept {n} of {ok.shape[0]} ({n / ok.shape[0]:.3f}), {b.shape[0]} borderline")
    assert np.array_equal(g, want), "screened (source, key) multiset differs"
    err = float(np.max(np.abs(gh - want_h), initial=0.0))
    assert err <= H_TOL, f"kept values differ by {err:.3e}"
    # overflow: capacity below the kept count sets the flag and still reports the count
    keys2, _, _, n2, flags2 = _gen(sci, h, dets, eps=eps, capacity=max(1, n // 2))
    assert int(n2.item()) == n
    assert sci.check_flags(flags2, "gen", allow=sci.FLAG_OVERFLOW) & sci.FLAG_OVERFLOW
    return n


@pytest.mark.parametrize("name,n_src", [("tiny", None), ("medium", 16), ("large", 6)])
def test_gen_screened_matches_oracle(name, n_src):
    """Screened mode for one-word (tiny, medium) and two-word (large) keys."""
    sci = require_gpu()
    s = system(name)
    h = ham(name)
    dets = s.dets if n_src is None else s.dets[pick_sources(s.dets.shape[0], n_src, 9)]
    say(f"gen screened {name} (W={h.W}): {dets.shape[0]} sources x {h.n_coupled}")
    _screened_check(sci, h, s.n_orb, s.n_alpha, s.n_beta, s.h1, s.eri, dets)


def test_gen_bad_determinant_flag():
    sci = require_gpu()
    s = system("tiny")
    h = ham("tiny")
    bad = s.dets[:3].copy()
    bad[1, 0] ^= np.uint64(1) << np.uint64(2 * s.n_orb + 1)  # a bit beyond 2*n_orb
    keys, hij, _, _, flags = _gen(sci, h, bad)
    assert sci.check_flags(flags, "gen", allow=sci.FLAG_BAD_DET) & sci.FLAG_BAD_DET
    nc = h.n_coupled
    ok, oh, _ = oracle.gen_coupled(s.n_orb, s.n_alpha, s.n_beta, s.h1, s.eri, s.dets[:1])
    assert np.array_equal(sci.keys_to_host(keys[:nc]), ok)
    assert np.all(hij[nc:2 * nc].cpu().numpy() == 0.0)


def test_gen_empty_range():
    sci = require_gpu()
    s = system("tiny")
    h = ham("tiny")
    keys, hij, _, n_out, flags = _gen(sci, h, s.dets[:2], exc_begin=5, exc_end=5)
    assert int(n_out.item()) == 0 and keys.shape[0] == 0


def _edge_system(n, na, nb, n_dets=6):
    rng = np.random.Generator(np.random.PCG64(n + 100 * na + nb))
    h1 = si.make_h1(rng, n)
    eri = si.make_eri(rng, n, 6)
    W = si.n_words(n)
    picks = set()
    while len(picks) < n_dets:
        picks.add(si.pack_int(rng.choice(n, na, replace=False), rng.choice(n, nb, replace=False), n))
    return h1, eri, si.sort_keys(si.ints_to_words(sorted(picks), W))


# (50, 25, 25) and (64, 32, 32): n_alpha * v_alpha above 512, so the single excitations
# are evaluated per lane instead of from the source's LDS table; (50, 10, 25) has only
# the beta block above 512, which also sends both spins to the per-lane branch
@pytest.mark.parametrize("n,na,nb", [(5, 1, 1), (6, 3, 0), (33, 2, 3), (40, 20, 19), (64, 3, 4),
                                     (50, 25, 25), (50, 10, 25), (64, 32, 32)])
def test_gen_edge_shapes(n, na, nb):
    """Edge shapes: one electron per spin, an empty spin, W=2 boundary, half filling,
    n_orb=64, and the per-lane single-excitation branch."""
    sci = require_gpu()
    h1, eri, dets = _edge_system(n, na, nb)
    say(f"gen edge n={n} na={na} nb={nb}: {dets.shape[0]} sources x {sci.sci_n_coupled(n, na, nb)}")
    h = sci.Ham(n, na, nb, h1, eri)
    keys, hij, _, _, flags = _gen(sci, h, dets)
    assert sci.check_flags(flags, "gen") == 0
    ok, oh, _ = oracle.gen_coupled(n, na, nb, h1, eri, dets)
    assert np.array_equal(sci.keys_to_host(keys), ok)
    assert np.max(np.abs(hij.cpu().numpy() - oh), initial=0.0) <= H_TOL


@pytest.mark.parametrize("n,na,nb", [(50, 25, 25), (64, 32, 32)])
def test_gen_screened_per_lane_singles(n, na, nb):
    """Screened mode (two-word keys) through the per-lane single-excitation branch."""
    sci = require_gpu()
    h1, eri, dets = _edge_system(n, na, nb, n_dets=3)
    say(f"gen screened edge n={n} na={na} nb={nb}")
    h = sci.Ham(n, na, nb, h1, eri)
    _screened_check(sci, h, n, na, nb, h1, eri, dets)


# ---------------------------------------------------------------------------
# de-duplication
# ---------------------------------------------------------------------------

def _dedup_check(sci, cand_np, set_np, W, want_novel=True):
    import torch
    cand = sci.keys_to_device(cand_np) if cand_np.shape[0] else torch.empty((0, W), dtype=torch.int64, device="cuda")
    setin = sci.keys_to_device(set_np) if set_np.shape[0] else torch.empty((0, W), dtype=torch.int64, device="cuda")
    out, n_out, nov, n_nov, flags = sci.dedup_merge(cand, setin, W, want_novel=want_novel)
    torch.cuda.synchronize()
    assert sci.check_flags(flags, "dedup") == 0
    ou, onov = oracle.dedup_merge(W, cand_np, set_np)
    n = int(n_out.item())
    assert n == ou.shape[0], f"|union| {n} != {ou.shape[0]}"
    assert np.array_equal(sci.keys_to_host(out[:n]), ou)
    if want_novel:
        m = int(n_nov.item())
        assert m == onov.shape[0]
        assert np.array_equal(sci.keys_to_host(nov[:m]), onov)


def _random_keys(rng, n, W, pool=None, top=True):
    if pool is None:
        pool = max(1, n // 3)
    base = rng.integers(0, 2**63, size=(pool, W), dtype=np.int64).astype(np.uint64)
    if top:
        base[: pool // 2, -1] |= np.uint64(1) << np.uint64(63)
    return base[rng.integers(0, pool, n)]


@pytest.mark.parametrize("W", [1, 2])
@pytest.mark.parametrize("n", [0, 1, 100, 2047, 2048, 2049, 4096, 4097, 50_000, 1_200_000])
def test_dedup_random_matches_oracle(W, n):
    sci = require_gpu()
    rng = np.random.Generator(np.random.PCG64(n * 7 + W))
    say(f"dedup random W={W} n={n}")
    cand = _random_keys(rng, n, W)
    setin = si.sort_keys(np.unique(_random_keys(rng, 300, W, pool=600), axis=0)) if n % 2 == 0 else \
        np.zeros((0, W), np.uint64)
    if setin.shape[0] and n:
        setin = si.sort_keys(np.concatenate([setin, cand[:5]]))
        setin = setin[np.concatenate([[True], np.any(setin[1:] != setin[:-1], axis=1)])]
    _dedup_check(sci, cand, setin, W)


@pytest.mark.parametrize("W", [1, 2])
def test_dedup_heavy_hitters(W):
    """A few keys repeated far beyond one LDS bucket (oversized-bucket path)."""
    sci = require_gpu()
    rng = np.random.Generator(np.random.PCG64(40 + W))
    few = _random_keys(rng, 5, W, pool=5)
    many = _random_keys(rng, 20_000, W, pool=20_000)
    cand = np.concatenate([np.repeat(few, 60_000, axis=0), many])
    cand = cand[rng.permutation(cand.shape[0])]
    say(f"dedup heavy W={W} n={cand.shape[0]}")
    _dedup_check(sci, cand, np.zeros((0, W), np.uint64), W)
    # everything equal
    _dedup_check(sci, np.repeat(few[:1], 300_000, axis=0), few[1:2][np.argsort([0])], W)


@pytest.mark.parametrize("W,n_distinct,n_cand", [(1, 8_000_000, 110_000_000), (2, 2_000_000, 16_000_000)])
def test_dedup_sample_runs_path(W, n_distinct, n_cand):
    """Level-1 splitters from more samples than one LDS sort holds (sorted runs, then
    each sample ranked in their merged order): every key of a known distinct set D
    occurs at least once among n_cand candidates in random order, so the union is D
    plus the set keys, and the novel keys are D minus the set."""
    sci = require_gpu()
    rng = np.random.Generator(np.random.PCG64(90 + W))
    d = rng.integers(0, 2**63, size=(n_distinct, W), dtype=np.int64).astype(np.uint64)
    d[: n_distinct // 2, -1] |= np.uint64(1) << np.uint64(63)
    d = si.sort_keys(d)
    d = d[np.concatenate([[True], np.any(d[1:] != d[:-1], axis=1)])]
    extra = si.sort_keys(_random_keys(rng, 1000, W, pool=1000))
    setin = si.sort_keys(np.concatenate([d[::7], extra]))
    setin = setin[np.concatenate([[True], np.any(setin[1:] != setin[:-1], axis=1)])]
    say(f"dedup sample-runs W={W} distinct={d.shape[0]} n={n_cand}")
    dev = torch.device("cuda")
    dd = sci.keys_to_device(d)
    gen = torch.Generator(device=dev)
    gen.manual_seed(91 + W)
    idx = torch.cat([torch.arange(d.shape[0], device=dev),
                     torch.randint(0, d.shape[0], (n_cand - d.shape[0],), device=dev, generator=gen)])
    idx = idx[torch.randperm(n_cand, device=dev, generator=gen)]
    cand = dd[idx].contiguous()
    del idx
    out, n_out, nov, n_nov, flags = sci.dedup_merge(cand, sci.keys_to_device(setin), W, want_novel=True)
    torch.cuda.synchronize()
    assert sci.check_flags(flags, "dedup") == 0
    union = si.sort_keys(np.concatenate([d, setin]))
    union = union[np.concatenate([[True], np.any(union[1:] != union[:-1], axis=1)])]
    n = int(n_out.item())
    assert n == union.shape[0]
    assert torch.equal(out[:n], sci.keys_to_device(union))
    # novel: the keys of D that are not set keys
    row = np.dtype((np.void, 8 * W))
    novel = d[~np.isin(np.ascontiguousarray(d).view(row).ravel(), np.ascontiguousarray(setin).view(row).ravel())]
    m = int(n_nov.item())
    assert m == novel.shape[0]
    assert torch.equal(nov[:m], sci.keys_to_device(novel))


@pytest.mark.parametrize("W", [1, 2])
def test_dedup_heavy_hitter_among_dense_neighbours(W):
    """One key repeated millions of times amid runs of distinct neighbours: the samples
    are nearly all that key, so its final bucket also holds more distinct neighbours than
    one LDS unit (the streamed unit gives way to the global-memory sort)."""
    sci = require_gpu()
    rng = np.random.Generator(np.random.PCG64(70 + W))
    heavy = rng.integers(1 << 40, 1 << 62, size=W, dtype=np.int64).astype(np.uint64)
    d = 40_000
    offs = np.concatenate([-1 - np.arange(d), 1 + np.arange(d)]).astype(np.int64)
    near = np.repeat(heavy[None, :], 2 * d, axis=0)
    near[:, 0] = (near[:, 0].astype(np.int64) + offs).astype(np.uint64)
    cand = np.concatenate([np.repeat(heavy[None, :], 4_000_000, axis=0), near])
    cand = cand[rng.permutation(cand.shape[0])]
    setin = si.sort_keys(np.concatenate([heavy[None, :], near[::97], _random_keys(rng, 500, W, pool=500)]))
    setin = setin[np.concatenate([[True], np.any(setin[1:] != setin[:-1], axis=1)])]
    say(f"dedup heavy among neighbours W={W} n={cand.shape[0]} set={setin.shape[0]}")
    _dedup_check(sci, cand, setin, W)


@pytest.mark.parametrize("n_straggle", [2, 1000])
def test_dedup_shared_top_word_with_stragglers(n_straggle):
    """Two-word keys nearly all sharing one top word X, with a few keys at X-1 and X+1.
    Two per side are almost never among a level-2 bucket's ~4,000 samples: the
    segment's splitters then all have the top word X, its histogram searches low words
    only and must send the stragglers to its first or last bucket.  A thousand per
    side are sampled and split off as usual.  Units holding a straggler sort both
    words.  Union and novel keys against the oracle, with a set that also holds keys
    of all three top words."""
    sci = require_gpu()
    rng = np.random.Generator(np.random.PCG64(123 + n_straggle))
    X = np.uint64(0x0123456789ABCDEF)
    main = np.empty((2_000_000, 2), np.uint64)
    main[:, 0] = rng.integers(0, 2**63, size=main.shape[0], dtype=np.int64).astype(np.uint64) << np.uint64(1)
    main[:, 1] = X
    low = main[:n_straggle].copy()
    low[:, 1] = X - np.uint64(1)
    high = main[n_straggle:2 * n_straggle].copy()
    high[:, 1] = X + np.uint64(1)
    cand = np.concatenate([main, main[::3], low, high])  # repeats as well
    cand = cand[rng.permutation(cand.shape[0])]
    setin = si.sort_keys(np.concatenate([main[::11], low[::2], high[1::2]]))
    setin = setin[np.concatenate([[True], np.any(setin[1:] != setin[:-1], axis=1)])]
    say(f"dedup shared top word: n={cand.shape[0]} set={setin.shape[0]}")
    _dedup_check(sci, cand, setin, 2)


@pytest.mark.parametrize("W,shared_top", [(1, False), (2, False), (2, True)])
@pytest.mark.parametrize("n_novel", [2, 3, 63, 64, 65, 127, 128, 129, 300, 511, 512, 513, 700])
def test_dedup_single_unit_novel_counts(W, shared_top, n_novel):
    """A dedup small enough to be one unit (the candidates fit the LDS capacity), so its
    novel-key count is set exactly: counts on the edges of the register sort of small
    units (64-key runs per wave, merge rounds, at most 512 keys) and just above it,
    where the radix passes take over.  Each distinct key appears once or twice; 200
    more distinct candidates are already in the set, which also holds 50 keys no
    candidate has.  With shared_top every key has one top word (the low words are
    sorted alone).  Union and novel keys against the oracle."""
    sci = require_gpu()
    rng = np.random.Generator(np.random.PCG64(1000 * W + 10 * n_novel + shared_top))
    n_dist = n_novel + 250
    keys = np.empty((0, W), np.uint64)
    while keys.shape[0] < n_dist:  # distinct rows
        more = rng.integers(0, 2**63, size=(2 * n_dist, W), dtype=np.int64).astype(np.uint64)
        if shared_top:
            more[:, 1] = np.uint64(0x00F0F0F0F0F0F0F0)
        keys = np.unique(np.concatenate([keys, more]), axis=0)
    keys = keys[rng.permutation(keys.shape[0])[:n_dist]]
    cand_keys = keys[:n_novel + 200]  # the last 50 are set-only
    cand = np.concatenate([cand_keys, cand_keys[::2]])
    cand = cand[rng.permutation(cand.shape[0])]
    setin = si.sort_keys(keys[n_novel:])
    say(f"dedup one unit W={W} shared_top={shared_top} novel={n_novel} n={cand.shape[0]} set={setin.shape[0]}")
    _dedup_check(sci, cand, setin, W)


@pytest.mark.parametrize("name", ["tiny", "medium"])
def test_dedup_of_generated_candidates(name):
    """Skewed real keys: coupled sets of a selected-set slice merged into the selected set."""
    import torch
    sci = require_gpu()
    s = system(name)
    h = ham(name)
    dets = s.dets if name == "tiny" else s.dets[:2000]
    keys, _, _, _, _ = _gen(sci, h, dets)
    cand_np = sci.keys_to_host(keys)
    say(f"dedup generated {name}: {cand_np.shape[0]} candidates")
    _dedup_check(sci, cand_np, s.dets, s.W)


def test_dedup_flags():
    import torch
    sci = require_gpu()
    rng = np.random.Generator(np.random.PCG64(5))
    cand = _random_keys(rng, 10_000, 1)
    c = sci.keys_to_device(cand)
    empty = torch.empty((0, 1), dtype=torch.int64, device="cuda")
    out, n_out, _, _, flags = sci.dedup_merge(c, empty, 1, set_capacity=10)
    torch.cuda.synchronize()
    ou, _ = oracle.dedup_merge(1, cand)
    assert int(n_out.item()) == ou.shape[0]
    assert sci.check_flags(flags, "dedup", allow=sci.FLAG_OVERFLOW) & sci.FLAG_OVERFLOW
    unsorted = sci.keys_to_device(np.array([[5], [3], [9]], dtype=np.uint64))
    _, _, _, _, flags2 = sci.dedup_merge(c, unsorted, 1)
    torch.cuda.synchronize()
    assert sci.check_flags(flags2, "dedup", allow=sci.FLAG_UNSORTED) & sci.FLAG_UNSORTED


@pytest.mark.parametrize("W", [1, 2])
def test_dedup_unsorted_set_against_large_runs(W):
    """A set passed out of order is flagged, and the merge stays inside its buffers even
    where a unit's run exceeds LDS (windowed merge, whose split points are not monotone
    for such a set); the same inputs with the set in order then give the oracle's union."""
    import torch
    sci = require_gpu()
    rng = np.random.Generator(np.random.PCG64(110 + W))
    heavy = rng.integers(1 << 40, 1 << 62, size=W, dtype=np.int64).astype(np.uint64)
    d = 40_000
    offs = np.concatenate([-1 - np.arange(d), 1 + np.arange(d)]).astype(np.int64)
    near = np.repeat(heavy[None, :], 2 * d, axis=0)
    near[:, 0] = (near[:, 0].astype(np.int64) + offs).astype(np.uint64)
    spread = _random_keys(rng, 300_000, W, pool=200_000)
    cand = np.concatenate([np.repeat(heavy[None, :], 400_000, axis=0), near, spread])
    cand = cand[rng.permutation(cand.shape[0])]
    setin = si.sort_keys(np.concatenate([near[::5], spread[::3], _random_keys(rng, 5000, W, pool=5000)]))
    setin = setin[np.concatenate([[True], np.any(setin[1:] != setin[:-1], axis=1)])]
    say(f"dedup unsorted set W={W} n={cand.shape[0]} set={setin.shape[0]}")
    c = sci.keys_to_device(cand)
    for order in (setin[::-1], setin[rng.permutation(setin.shape[0])]):
        out, n_out, nov, n_nov, flags = sci.dedup_merge(c, sci.keys_to_device(np.ascontiguousarray(order)), W,
                                                        want_novel=True)
        torch.cuda.synchronize()
        assert sci.check_flags(flags, "dedup", allow=sci.FLAG_UNSORTED | sci.FLAG_OVERFLOW) & sci.FLAG_UNSORTED
    _dedup_check(sci, cand, setin, W)


# ---------------------------------------------------------------------------
# energy
# ---------------------------------------------------------------------------

METHODS = ["pairs", "enum"]


def _method(sci, name):
    return {"pairs": sci.ENERGY_PAIRS, "enum": sci.ENERGY_ENUM}[name]


@pytest.mark.parametrize("method", METHODS)
def test_energy_tiny_matches_oracle(method):
    import torch
    sci = require_gpu()
    s = system("tiny")
    h = ham("tiny")
    sel = sci.keys_to_device(s.dets)
    psi = torch.from_numpy(s.psi).cuda()
    m = _method(sci, method)
    e, hp, g, flags = sci.energy(h, sel, psi, method=m)
    torch.cuda.synchronize()
    assert sci.check_flags(flags, "energy") == 0
    oe, ohp, og = oracle.energy(s.n_orb, s.n_alpha, s.n_beta, s.h1, s.eri, s.dets, s.psi)
    say(f"energy tiny: gpu {e.item():.15f} oracle {oe:.15f}")
    assert abs(e.item() - oe) <= E_TOL
    assert np.max(np.abs(hp.cpu().numpy() - ohp)) <= H_TOL * 10
    assert np.max(np.abs(g.cpu().numpy() - og)) <= G_TOL
    # bit-reproducible
    e2, hp2, g2, _ = sci.energy(h, sel, psi, method=m)
    torch.cuda.synchronize()
    assert e2.item() == e.item() and torch.equal(hp2, hp) and torch.equal(g2, g)


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("n,na,nb,n_sel", [
    (5, 1, 0, None),     # one electron: the screening bias 2 - N is positive
    (6, 1, 1, None),     # two electrons: every pair of the space is connected
    (7, 2, 1, None),     # three electrons
    (16, 2, 2, None),    # 2n = 32 spin orbitals: one 32-bit chunk
    (17, 3, 2, 3000),    # 2n = 34: a second, mostly empty chunk
    (33, 2, 2, 4000),    # two words, 2n = 66: three chunks
    (64, 2, 3, 3000),    # two words, 2n = 128: four full chunks
])
def test_energy_shapes_match_oracle(n, na, nb, n_sel, method):
    """E, H psi and the gradient against the oracle on spaces that exercise the edges of
    the pair screening: electron counts of 1-3, spin-orbital counts that fill one, part
    of two, three or four 32-bit chunks, and row or column blocks left partly empty."""
    import torch
    sci = require_gpu()
    sm = si.make_system(si.small_workload(n, na, nb, n_sel=n_sel, seed=300 + n + na))
    say(f"energy shape n={n} {na}a+{nb}b n_sel={sm.dets.shape[0]} {method}")
    h = sci.Ham(sm.n_orb, sm.n_alpha, sm.n_beta, sm.h1, sm.eri)
    e, hp, g, flags = sci.energy(h, sci.keys_to_device(sm.dets), torch.from_numpy(sm.psi).cuda(),
                                 method=_method(sci, method))
    torch.cuda.synchronize()
    assert sci.check_flags(flags, "energy") == 0
    oe, ohp, og = oracle.energy(sm.n_orb, sm.n_alpha, sm.n_beta, sm.h1, sm.eri, sm.dets, sm.psi)
    assert abs(e.item() - oe) <= E_TOL
    assert np.max(np.abs(hp.cpu().numpy() - ohp)) <= H_TOL * 10
    assert np.max(np.abs(g.cpu().numpy() - og)) <= G_TOL


@pytest.mark.parametrize("method", METHODS)
def test_energy_full_space_eigenvector(method):
    import torch
    sci = require_gpu()
    n, na, nb = 6, 3, 2
    rng = np.random.Generator(np.random.PCG64(12))
    h1 = si.make_h1(rng, n)
    eri = si.make_eri(rng, n, 8)
    basis = si.all_determinants(n, na, nb)
    hd = oracle.dense_h_sc(n, na, nb, h1, eri, basis)
    w, v = np.linalg.eigh(hd)
    h = sci.Ham(n, na, nb, h1, eri)
    e, hp, g, flags = sci.energy(h, sci.keys_to_device(basis), torch.from_numpy(v[:, 0].copy()).cuda(),
                                 method=_method(sci, method))
    torch.cuda.synchronize()
    assert abs(e.item() - w[0]) <= E_TOL
    assert np.max(np.abs(g.cpu().numpy())) <= 1e-9


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("name,n_rows", [("medium", 24), ("large", 8)])
def test_energy_sampled_rows(name, n_rows, method):
    import torch
    sci = require_gpu()
    s = system(name)
    h = ham(name)
    sel = sci.keys_to_device(s.dets)
    psi = torch.from_numpy(s.psi).cuda()
    say(f"energy {name} ({method}): n_sel={s.dets.shape[0]}")
    e, hp, g, flags = sci.energy(h, sel, psi, method=_method(sci, method))
    torch.cuda.synchronize()
    assert sci.check_flags(flags, "energy") == 0
    rows = pick_sources(s.dets.shape[0], n_rows, 21)
    ohp = oracle.hpsi_rows(s.n_orb, s.n_alpha, s.n_beta, s.h1, s.eri, s.dets, s.psi, rows)
    ghp = hp.cpu().numpy()
    err = np.max(np.abs(ghp[rows] - ohp))
    say(f"  sampled rows max |d(H psi)| = {err:.3e}")
    assert err <= 1e-11
    # properties at full size: E = psi.Hpsi/psi.psi, g = 2(Hpsi - E psi)/psi.psi, psi.g = 0
    num = float(np.dot(s.psi, ghp))
    den = float(np.dot(s.psi, s.psi))
    assert abs(e.item() - num / den) <= E_TOL
    gg = g.cpu().numpy()
    assert np.max(np.abs(gg - 2 * (ghp - e.item() * s.psi) / den)) <= G_TOL
    assert abs(float(np.dot(s.psi, gg))) <= 1e-9


@pytest.mark.parametrize("method", METHODS)
def test_energy_flags(method):
    import torch
    sci = require_gpu()
    s = system("tiny")
    h = ham("tiny")
    sel = sci.keys_to_device(s.dets[::-1].copy())
    _, _, _, flags = sci.energy(h, sel, torch.from_numpy(s.psi).cuda(), method=_method(sci, method))
    torch.cuda.synchronize()
    assert sci.check_flags(flags, "energy", allow=sci.FLAG_UNSORTED) & sci.FLAG_UNSORTED
    bad = s.dets.copy()
    bad[3, 0] ^= np.uint64(1) << np.uint64(2 * s.n_orb + 1)  # a bit beyond 2 n_orb
    _, _, _, flags = sci.energy(h, sci.keys_to_device(bad), torch.from_numpy(s.psi).cuda(),
                                method=_method(sci, method))
    torch.cuda.synchronize()
    assert sci.check_flags(flags, "energy", allow=sci.FLAG_BAD_DET | sci.FLAG_UNSORTED) & sci.FLAG_BAD_DET


def test_energy_methods_agree_and_auto_choice():
    """Both membership methods give the same H psi (to rounding) on the medium system and
    on a small-orbital system (N_c = 804) of the kind the batched workload holds, and the
    automatic choice gives one of them."""
    import torch
    sci = require_gpu()
    s = system("medium")
    h = ham("medium")
    sel = sci.keys_to_device(s.dets)
    psi = torch.from_numpy(s.psi).cuda()
    e1, hp1, g1, f1 = sci.energy(h, sel, psi, method=sci.ENERGY_PAIRS)
    e2, hp2, g2, f2 = sci.energy(h, sel, psi, method=sci.ENERGY_ENUM)
    torch.cuda.synchronize()
    assert sci.check_flags(f1, "pairs") == 0 and sci.check_flags(f2, "enum") == 0
    assert abs(e1.item() - e2.item()) <= E_TOL
    assert float((hp1 - hp2).abs().max().item()) <= 1e-11
    assert float((g1 - g2).abs().max().item()) <= G_TOL
    assert sci.sci_energy_method(h, s.dets.shape[0]) == sci.ENERGY_PAIRS  # N_c = 25,137 >> |S| / 64
    # a small-orbital system of the batched workload: N_c = 804 for n_orb = 10, 4a+4b
    wl = si.small_workload(10, 4, 4, n_sel=17_000, selection="levels")
    sm = si.make_system(wl)
    hs = sci.Ham(sm.n_orb, sm.n_alpha, sm.n_beta, sm.h1, sm.eri)
    sels = sci.keys_to_device(sm.dets)
    psis = torch.from_numpy(sm.psi).cuda()
    auto = sci.sci_energy_method(hs, sm.dets.shape[0])
    say(f"  small system: n_sel={sm.dets.shape[0]}, N_c={hs.n_coupled}, auto method {auto}")
    assert auto == sci.ENERGY_ENUM  # N_c * 8 < |S|: enumeration (measured 5.6x faster here)
    ea, hpa, _, fa = sci.energy(hs, sels, psis, method=sci.ENERGY_ENUM)
    ep, hpp, _, fp = sci.energy(hs, sels, psis, method=sci.ENERGY_PAIRS)
    e0, hp0, _, f0 = sci.energy(hs, sels, psis)
    torch.cuda.synchronize()
    assert sci.check_flags(fa, "enum") == 0 and sci.check_flags(fp, "pairs") == 0 and sci.check_flags(f0, "auto") == 0
    assert abs(ea.item() - ep.item()) <= E_TOL
    assert float((hpa - hpp).abs().max().item()) <= 1e-11
    assert torch.equal(hp0, hpa if auto == sci.ENERGY_ENUM else hpp)
    rows = pick_sources(sm.dets.shape[0], 16, 8)
    ohp = oracle.hpsi_rows(sm.n_orb, sm.n_alpha, sm.n_beta, sm.h1, sm.eri, sm.dets, sm.psi, rows)
    assert np.max(np.abs(hpa.cpu().numpy()[rows] - ohp)) <= 1e-11


@pytest.mark.parametrize("W", [1, 2])
@pytest.mark.parametrize("n_cand", [1000, 3000, 300_000])
def test_dedup_large_set_few_candidates(W, n_cand):
    """Running set much larger than the candidate batch: many set keys per bucket range,
    keys below/above every candidate, half of the candidates already in the set."""
    sci = require_gpu()
    rng = np.random.Generator(np.random.PCG64(900 + W + n_cand))
    setk = si.sort_keys(np.unique(_random_keys(rng, 200_000, W, pool=400_000), axis=0))
    fresh = _random_keys(rng, n_cand // 2, W, pool=n_cand)
    old = setk[rng.integers(0, setk.shape[0], n_cand - n_cand // 2)]
    cand = np.concatenate([fresh, old])
    cand = cand[rng.permutation(cand.shape[0])]
    say(f"dedup large set W={W} n_cand={n_cand} n_set={setk.shape[0]}")
    _dedup_check(sci, cand, setk, W)


@pytest.mark.parametrize("W", [1, 2])
def test_dedup_streamed_chunks(W):
    """Two candidate batches merged one after the other equal one merge of both."""
    sci = require_gpu()
    rng = np.random.Generator(np.random.PCG64(77 + W))
    c0 = _random_keys(rng, 150_000, W, pool=90_000)
    c1 = np.concatenate([c0[:40_000], _random_keys(rng, 110_000, W, pool=70_000)])
    empty = np.zeros((0, W), np.uint64)
    u0, _ = oracle.dedup_merge(W, c0, empty)
    _dedup_check(sci, c0, empty, W)
    _dedup_check(sci, c1, u0, W)


@pytest.mark.parametrize("name,n_src,chunk", [("tiny", None, 1000), ("medium", 300, 1_000_003), ("large", 24, 3_000_000)])
def test_stream_dedup_matches_oracle(name, n_src, chunk):
    """Pool streaming (generation of chunk k+1 overlapping dedup of chunk k on a second
    stream) equals the oracle's union of every coupled set with the selected set."""
    sci = require_gpu()
    s = system(name)
    h = ham(name)
    dets = s.dets if n_src is None else s.dets[pick_sources(s.dets.shape[0], n_src, 31)]
    d = sci.keys_to_device(dets)
    sel = sci.keys_to_device(s.dets)
    total = dets.shape[0] * h.n_coupled
    say(f"stream dedup {name}: {total} candidates in chunks of {chunk}")
    side = torch.cuda.Stream()
    out, n_out, flags = sci.stream_dedup(h, d, chunk, sel, total + s.dets.shape[0], dedup_stream=side)
    torch.cuda.synchronize()
    assert sci.check_flags(flags, "stream") == 0
    ok, _, _ = oracle.gen_coupled(s.n_orb, s.n_alpha, s.n_beta, s.h1, s.eri, dets)
    ou, _ = oracle.dedup_merge(s.W, ok, s.dets)
    n = int(n_out.item())
    assert n == ou.shape[0]
    assert np.array_equal(sci.keys_to_host(out[:n]), ou)
    # a sub-range of the excitation space, including partial first and last sources
    a0, a1 = h.n_coupled // 3, total - h.n_coupled // 5
    out2, n2, _ = sci.stream_dedup(h, d, chunk, sel, total + s.dets.shape[0], exc_begin=a0, exc_end=a1)
    torch.cuda.synchronize()
    ou2, _ = oracle.dedup_merge(s.W, ok[a0:a1], s.dets)
    assert int(n2.item()) == ou2.shape[0]
    assert np.array_equal(sci.keys_to_host(out2[:int(n2.item())]), ou2)


def test_stream_dedup_rejects_chunks_above_one_dedup_call():
    """A chunk of 2^32 candidates or more is refused before anything is enqueued."""
    import ctypes
    import torch
    sci = require_gpu()
    h = ham("tiny")
    s = system("tiny")
    sel = sci.keys_to_device(s.dets)
    d = torch.zeros(1, dtype=torch.int64, device="cuda")
    P = ctypes.c_void_p
    fin = ctypes.c_int32(0)
    rc = sci._lib.sci_stream_dedup(h._h, P(sel.data_ptr()), sel.shape[0], 0, 10, 1 << 32, P(sel.data_ptr()),
                                   P(d.data_ptr()), P(d.data_ptr()), P(d.data_ptr() + 8), 1, P(d.data_ptr()),
                                   ctypes.byref(fin), P(d.data_ptr()), 8, P(d.data_ptr()), None, None)
    assert rc == sci.SCI_EUNSUPPORTED
    assert "exceeds one dedup call" in sci._lib.sci_last_error().decode()


def test_stream_dedup_overflow_truncates_running_set():
    """When the running set overflows its capacity mid-stream, later chunks merge into the
    kept (first set_capacity) keys only.  Expected values follow that rule with the oracle:
    R_0 = set_in, R_k = first cap keys of sorted(R_(k-1) | chunk_k), count = |R_(K-1) | chunk_K|."""
    sci = require_gpu()
    s = system("medium")
    h = ham("medium")
    dets = s.dets[pick_sources(s.dets.shape[0], 24, 7)]
    ok, _, _ = oracle.gen_coupled(s.n_orb, s.n_alpha, s.n_beta, s.h1, s.eri, dets)
    chunk = 150_000
    bounds = [(e, min(e + chunk, ok.shape[0])) for e in range(0, ok.shape[0], chunk)]
    assert len(bounds) == 5

    def emulate(cap):
        run, need = dets, dets.shape[0]
        for e0, e1 in bounds:
            u, _ = oracle.dedup_merge(s.W, ok[e0:e1], run)
            need = u.shape[0]
            run = u[:cap]
        return run, need

    sizes = []
    run = dets
    for e0, e1 in bounds[:2]:
        run, _ = oracle.dedup_merge(s.W, ok[e0:e1], run)
        sizes.append(run.shape[0])
    cap = (sizes[0] + sizes[1]) // 2  # the second chunk overflows, three more follow
    want, want_n = emulate(cap)
    say(f"stream overflow: {ok.shape[0]} candidates, chunks of {chunk}, capacity {cap}")
    d = sci.keys_to_device(dets)
    out, n_out, flags = sci.stream_dedup(h, d, chunk, d, cap, dedup_stream=torch.cuda.Stream())
    torch.cuda.synchronize()
    assert sci.check_flags(flags, "stream", allow=sci.FLAG_OVERFLOW) & sci.FLAG_OVERFLOW
    n = int(n_out.item())
    assert n == want_n and n >= cap
    assert np.array_equal(sci.keys_to_host(out[:min(n, cap)]), want)


# ---------------------------------------------------------------------------
# differentiation: autograd wrapper, finite differences, dense-H gradient
# ---------------------------------------------------------------------------

def test_autograd_matches_adjoint_and_fd():
    sci = require_gpu()
    s = system("tiny")
    h = ham("tiny")
    sel = sci.keys_to_device(s.dets)
    psi = torch.from_numpy(s.psi).cuda().requires_grad_(True)
    e = sci.SciEnergy.apply(psi, h, sel)
    e.backward()
    _, _, g, _ = sci.energy(h, sel, psi.detach())
    torch.cuda.synchronize()
    assert torch.equal(psi.grad, g), "autograd gradient differs from the adjoint kernel"
    oe, _, og = oracle.energy(s.n_orb, s.n_alpha, s.n_beta, s.h1, s.eri, s.dets, s.psi)
    assert abs(e.item() - oe) <= E_TOL
    # central differences of the GPU energy along a seeded unit direction: O(h^2) to a round-off floor
    rng = np.random.Generator(np.random.PCG64(11))
    v = rng.standard_normal(s.psi.shape[0])
    v /= np.linalg.norm(v)
    vt = torch.from_numpy(v).cuda()
    gv = float(torch.dot(g, vt).item())
    errs = []
    for step in (1e-3, 1e-4, 1e-5):
        ep = sci.energy(h, sel, psi.detach() + step * vt, want_hpsi=False, want_grad=False)[0].item()
        em = sci.energy(h, sel, psi.detach() - step * vt, want_hpsi=False, want_grad=False)[0].item()
        errs.append(abs((ep - em) / (2 * step) - gv))
    say(f"  FD errors {errs}")
    assert errs[1] < errs[0] and errs[1] < 1e-7


def test_gradient_dense_h_subset_large():
    """The large workload's Hamiltonian on a 2,000-determinant subset of S: the GPU
    gradient equals the gradient of the dense Rayleigh quotient built from oracle rows."""
    sci = require_gpu()
    s = system("large")
    h = ham("large")
    rng = np.random.Generator(np.random.PCG64(2604157684))
    idx = np.sort(np.concatenate([[0], rng.choice(np.arange(1, s.dets.shape[0]), 1999, replace=False)]))
    sub = s.dets[idx]
    psi = s.psi[idx] / np.linalg.norm(s.psi[idx])
    e, hp, g, flags = sci.energy(h, sci.keys_to_device(sub), torch.from_numpy(psi).cuda())
    torch.cuda.synchronize()
    assert sci.check_flags(flags, "energy") == 0
    hd = oracle.dense_h_sc(s.n_orb, s.n_alpha, s.n_beta, s.h1, s.eri, sub)
    assert np.max(np.abs(hd - hd.T)) < 1e-13
    e_ref = psi @ hd @ psi / (psi @ psi)
    g_ref = 2 * (hd @ psi - e_ref * psi) / (psi @ psi)
    say(f"  large subset: E gpu {e.item():.12f} dense {e_ref:.12f}")
    assert abs(e.item() - e_ref) <= E_TOL
    assert np.max(np.abs(g.cpu().numpy() - g_ref)) <= G_TOL


def test_gradient_finite_differences_large():
    """Central differences of the GPU energy over the whole large selected space (2e5
    two-word determinants) along one seeded unit direction and 8 seeded coordinates,
    h in {1e-4, 1e-5, 1e-6}, against the adjoint's g.v.  The difference quotient's
    error is h^2/6 E''' (truncation) plus about 2 dE/(2h) (round-off of E): it must
    shrink from h = 1e-4 to 1e-5 unless it is already at the round-off floor, and the
    best step must reach 1e-7."""
    sci = require_gpu()
    s = system("large")
    h = ham("large")
    sel = sci.keys_to_device(s.dets)
    psi = torch.from_numpy(s.psi).cuda()
    e0, _, g, flags = sci.energy(h, sel, psi, want_hpsi=False)
    torch.cuda.synchronize()
    assert sci.check_flags(flags, "energy") == 0
    rng = np.random.Generator(np.random.PCG64(2604157684 + 7))
    v = rng.standard_normal(s.psi.shape[0])
    v /= np.linalg.norm(v)
    coords = rng.choice(s.psi.shape[0], 8, replace=False)
    dirs = [("unit", torch.from_numpy(v).cuda())]
    for c in coords:
        ec = torch.zeros_like(psi)
        ec[int(c)] = 1.0
        dirs.append((f"e_{int(c)}", ec))
    steps = (1e-4, 1e-5, 1e-6)
    # round-off of one energy evaluation, estimated from scale invariance E(c psi) = E(psi)
    dE = max(abs(sci.energy(h, sel, c * psi, want_hpsi=False, want_grad=False)[0].item() - e0.item())
             for c in (1.0 + 1e-3, 1.0 - 1e-3, 3.0))
    floor = 4.0 * dE / steps[1]  # round-off part of the quotient's error at h = 1e-5, with margin
    say(f"  energy round-off {dE:.2e} -> floor at h=1e-5: {floor:.2e}")
    worst_best = 0.0
    for name, d in dirs:
        gv = float(torch.dot(g, d).item())
        errs = []
        for hstep in steps:
            ep = sci.energy(h, sel, psi + hstep * d, want_hpsi=False, want_grad=False)[0].item()
            em = sci.energy(h, sel, psi - hstep * d, want_hpsi=False, want_grad=False)[0].item()
            errs.append(abs((ep - em) / (2 * hstep) - gv))
        say(f"  {name}: g.v = {gv:+.6e}, |FD - g.v| at h = 1e-4, 1e-5, 1e-6: "
            + ", ".join(f"{x:.2e}" for x in errs))
        best = min(errs)
        worst_best = max(worst_best, best)
        assert best <= 1e-7, f"{name}: finite differences do not reach the adjoint gradient"
        # O(h^2): a tenfold smaller step cuts the error unless round-off already dominates
        assert errs[1] <= max(0.1 * errs[0], floor, 1e-12), f"{name}: error does not fall with h"
    say(f"  worst best-step error {worst_best:.2e}, E = {e0.item():.12f}")
