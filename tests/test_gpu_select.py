"""GPU parity of the reverse index and the top-K selection against the oracle
(bit-exact: positions, masks and keys are integers)."""
import numpy as np
import pytest
import torch  # imported at collection: the first import on a fresh box is slow

import oracle
from tests.gpu_common import ham, pick_sources, require_gpu, say, system

pytestmark = pytest.mark.gpu


def _sorted_unique(rng, n, W, hi):
    k = np.unique(rng.integers(0, hi, size=(n, W), dtype=np.uint64), axis=0)
    order = np.lexsort(tuple(k[:, j] for j in range(W)))  # last key of lexsort = most significant = word W-1
    return k[order]


# the sorted kind (the paper's search of the sorted set) on sets below one sample block,
# not a multiple of the 256-key block, and above 2048 x 256 keys (a top level of every
# R-th sample, R > 1)
@pytest.mark.parametrize("kind", ["hash", "sorted"])
@pytest.mark.parametrize("W,n_set,n_cand", [(1, 0, 10), (1, 1, 1000), (1, 5000, 100_000), (2, 3000, 50_000),
                                            (1, 200_000, 1_000_000), (1, 3_000_001, 2_000_000),
                                            (2, 700_000, 500_000)])
def test_inverse_map_matches_oracle(W, n_set, n_cand, kind):
    sci = require_gpu()
    rng = np.random.Generator(np.random.PCG64(100 + n_set))
    hi = max(4 * n_set, 8)
    u = _sorted_unique(rng, n_set, W, hi) if n_set else np.zeros((0, W), dtype=np.uint64)
    cand = rng.integers(0, hi, size=(n_cand, W), dtype=np.uint64)
    if n_set:  # half the candidates are members of the set, in random order and repeated
        cand[: n_cand // 2] = u[rng.integers(0, u.shape[0], size=n_cand // 2)]
        rng.shuffle(cand)
    if n_set > 1:  # keys below the first and above the last set key
        cand[0] = np.zeros(W, dtype=np.uint64)
        cand[1] = np.full(W, np.iinfo(np.uint64).max, dtype=np.uint64)
    say(f"inverse map ({kind}) W={W} |U|={u.shape[0]} n={n_cand}")
    ud = sci.keys_to_device(u) if u.shape[0] else torch.zeros((1, W), dtype=torch.int64, device="cuda")
    nd = torch.tensor([u.shape[0]], dtype=torch.int64, device="cuda")
    index, flags = sci.build_index(ud, nd, u.shape[0], W, kind=kind)
    assert sci.index_kind(index) == kind
    idx = sci.inverse_map(index, sci.keys_to_device(cand), W)
    torch.cuda.synchronize()
    assert sci.check_flags(flags, "index") == 0
    want = oracle.inverse_map(W, u, cand)
    got = idx.cpu().numpy()
    assert np.array_equal(got, want)
    if n_set:  # the two boundary keys may have replaced members
        assert (got >= 0).sum() >= n_cand // 2 - 2 and (got < 0).any()


def test_inverse_map_of_generated_candidates():
    """Every coupled candidate of a generated chunk is found in the union the dedup built."""
    sci = require_gpu()
    s = system("medium")
    dets = s.dets[pick_sources(s.dets.shape[0], 40, 3)]
    keys, _, _, _, f1 = sci.gen_coupled(ham("medium"), sci.keys_to_device(dets))
    union, n_union, _, _, f2 = sci.dedup_merge(keys, sci.keys_to_device(s.dets), s.W)
    torch.cuda.synchronize()
    nu = int(n_union.item())
    index, f3 = sci.build_index(union, n_union, nu, s.W)
    idx = sci.inverse_map(index, keys, s.W)
    torch.cuda.synchronize()
    for f, w in ((f1, "gen"), (f2, "dedup"), (f3, "index")):
        assert sci.check_flags(f, w) == 0
    got = idx.cpu().numpy()
    u = sci.keys_to_host(union[:nu])
    k = sci.keys_to_host(keys)
    assert (got >= 0).all()
    assert np.array_equal(u[got], k)
    assert np.array_equal(got, oracle.inverse_map(s.W, u, k))


@pytest.mark.parametrize("kind", ["hash", "sorted"])
def test_index_overflow_flag(kind):
    sci = require_gpu()
    u = np.arange(1, 101, dtype=np.uint64).reshape(-1, 1)
    nd = torch.tensor([100], dtype=torch.int64, device="cuda")
    index, flags = sci.build_index(sci.keys_to_device(u), nd, 50, 1, kind=kind)
    idx = sci.inverse_map(index, sci.keys_to_device(u), 1)
    torch.cuda.synchronize()
    assert sci.check_flags(flags, "index", allow=sci.FLAG_OVERFLOW) & sci.FLAG_OVERFLOW
    got = idx.cpu().numpy()
    assert np.array_equal(got[:50], np.arange(50)) and (got[50:] == -1).all()


def _psi(rng, n, kind):
    if kind == "ties":
        return rng.integers(-30, 31, size=n).astype(np.float64) * 0.25
    if kind == "lognormal":
        return rng.choice([-1.0, 1.0], size=n) * np.exp(rng.normal(-8.0, 3.0, size=n))
    return np.full(n, 0.5)  # every magnitude equal: the smallest keys win


@pytest.mark.parametrize("W,n,k,kind", [(1, 1, 1, "ties"), (1, 1000, 0, "ties"), (1, 1000, 1, "lognormal"),
                                        (1, 5000, 777, "ties"), (1, 5000, 5000, "lognormal"),
                                        (1, 5000, 9000, "ties"), (2, 4000, 123, "same"), (2, 20000, 1500, "ties"),
                                        (1, 300_000, 10_000, "lognormal"), (1, 300_000, 20_000, "ties")])
def test_topk_matches_oracle(W, n, k, kind):
    sci = require_gpu()
    rng = np.random.Generator(np.random.PCG64(7 * n + k))
    keys = _sorted_unique(rng, int(n * 1.2) + 10, W, 1 << 50)[:n]
    rng.shuffle(keys)
    n = keys.shape[0]
    psi = _psi(rng, n, kind)
    say(f"topk W={W} n={n} k={k} {kind}")
    ok, op, n_out, flags = sci.topk(sci.keys_to_device(keys), torch.from_numpy(psi).cuda(), k, W)
    torch.cuda.synchronize()
    assert sci.check_flags(flags, "topk") == 0
    mask = oracle.topk(W, keys, psi, k)
    m = int(n_out.item())
    assert m == mask.sum() == min(k, n)
    assert np.array_equal(sci.keys_to_host(ok[:m]), keys[mask])  # input order
    assert np.array_equal(op[:m].cpu().numpy(), psi[mask])


def test_topk_selection_merges_into_set():
    """Selected novel candidates merged into S: the S-expansion step."""
    sci = require_gpu()
    s = system("tiny")
    keys, _, _, _, _ = sci.gen_coupled(ham("tiny"), sci.keys_to_device(s.dets))
    _, _, novel, n_novel, _ = sci.dedup_merge(keys, sci.keys_to_device(s.dets), s.W, want_novel=True)
    torch.cuda.synchronize()
    nn = int(n_novel.item())
    nov = sci.keys_to_host(novel[:nn])
    rng = np.random.Generator(np.random.PCG64(9))
    psi = rng.normal(size=nn)
    sel, _, n_sel, _ = sci.topk(novel[:nn].contiguous(), torch.from_numpy(psi).cuda(), 50, s.W)
    grown, n_grown, _, _, fl = sci.dedup_merge(sel[:50], sci.keys_to_device(s.dets), s.W)
    torch.cuda.synchronize()
    want, _ = oracle.dedup_merge(s.W, nov[oracle.topk(s.W, nov, psi, 50)], s.dets)
    assert int(n_grown.item()) == s.dets.shape[0] + 50
    assert np.array_equal(sci.keys_to_host(grown[:int(n_grown.item())]), want)
