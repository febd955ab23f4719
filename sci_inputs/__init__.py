"""Seeded synthetic workloads for the NNQS-SCI hot path.

This module only *draws inputs*: one-electron integrals h_pq, two-electron
integrals (pq|rs) in chemists' notation, a selected determinant set S and real
amplitudes psi.  It computes no matrix element, no fermionic sign, no coupled
set and no de-duplication, so both the CPU oracle and the HIP path can consume
its output without sharing any of the method's arithmetic.

Determinant encoding (shared by every consumer): spin orbital k = p + sigma*n_orb
(sigma = 0 for alpha, 1 for beta), bit k of a little-endian array of
W = ceil(2*n_orb/64) uint64 words; keys compare as unsigned W*64-bit integers
with word W-1 most significant.  The reference determinant occupies alpha
orbitals 0..n_alpha-1 and beta orbitals 0..n_beta-1.

Recipe (paper section 2.1: configurations are bitstrings of length m with n ones;
section 2.2: selected configurations are drawn from those coupled to the
reference):

* h: A ~ N(0,1)/n elementwise, h = (A + A^T)/2, then h_pp += -2 + 2p/(n-1).
* (pq|rs) = sum_x L^x_pq L^x_rs with L^x = (B^x + B^x^T)/2, B^x ~ N(0, 0.1);
  the tensor is then made bitwise 8-fold symmetric by copying the value at a
  canonical index to every member of its symmetry orbit.
* S: per workload (random excitation walk, uniform draws over excitation
  levels 1..4, or reference + all singles + sampled doubles), stored sorted.
* psi ~ N(0,1), normalised.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 2604157680


def n_words(n_orb: int) -> int:
    return (2 * n_orb + 63) // 64


@dataclass(frozen=True)
class Workload:
    name: str
    n_orb: int
    n_alpha: int
    n_beta: int
    rank: int
    n_sel: int
    selection: str  # "walk" | "levels" | "hf_sd" | "all"
    seed: int
    extra: dict = field(default_factory=dict)

    @property
    def W(self) -> int:
        return n_words(self.n_orb)


# The three single-system workloads: tiny (oracle-sized), medium (fits in HBM
# whole), large (two words per determinant, streamed through a device pool).
WORKLOADS = {
    "tiny": Workload("tiny", 7, 5, 5, 20, 200, "walk", SEED_BASE + 0),
    "medium": Workload("medium", 26, 7, 7, 100, 100_000, "levels", SEED_BASE + 1),
    "large": Workload("large", 60, 10, 10, 240, 200_000, "hf_sd", SEED_BASE + 2),
}


# ---------------------------------------------------------------------------
# integrals
# ---------------------------------------------------------------------------

def make_h1(rng: np.random.Generator, n: int) -> np.ndarray:
    a = rng.standard_normal((n, n)) / n
    h = (a + a.T) / 2.0
    if n > 1:
        h[np.arange(n), np.arange(n)] += -2.0 + 2.0 * np.arange(n) / (n - 1)
    else:
        h[0, 0] += -2.0
    return np.ascontiguousarray(h)


def symmetrize8(m4: np.ndarray) -> np.ndarray:
    """Copy m4 at the canonical member of each 8-fold orbit to every member.

    Orbit of (p,q,r,s): pairs (pq),(rs) unordered, and the two pairs swapped.
    Canonical member: P>=Q, R>=S, and compound index P*n+Q >= R*n+S.
    """
    n = m4.shape[0]
    flat = m4.reshape(n * n, n * n)
    idx = np.arange(n, dtype=np.int64)
    big = np.maximum.outer(idx, idx)
    small = np.minimum.outer(idx, idx)
    pair = (big * n + small).reshape(-1)  # canonical compound index of (p,q)
    hi = np.maximum.outer(pair, pair)
    lo = np.minimum.outer(pair, pair)
    # flat[row=hi_pair, col=lo_pair] where both pairs are in canonical (big, small) form
    out = flat[hi, lo]
    return np.ascontiguousarray(out.reshape(n, n, n, n))


def make_eri(rng: np.random.Generator, n: int, rank: int) -> np.ndarray:
    b = rng.normal(0.0, 0.1, size=(rank, n, n))
    l = (b + b.transpose(0, 2, 1)) / 2.0
    lf = l.reshape(rank, n * n)
    m = lf.T @ lf
    return symmetrize8(m.reshape(n, n, n, n))


# ---------------------------------------------------------------------------
# determinant packing
# ---------------------------------------------------------------------------

def reference_occupations(n_orb: int, n_alpha: int, n_beta: int):
    return list(range(n_alpha)), list(range(n_beta))


def pack_int(alpha_occ, beta_occ, n_orb: int) -> int:
    v = 0
    for p in alpha_occ:
        v |= 1 << int(p)
    for p in beta_occ:
        v |= 1 << (int(p) + n_orb)
    return v


def ints_to_words(vals, W: int) -> np.ndarray:
    out = np.zeros((len(vals), W), dtype=np.uint64)
    mask = (1 << 64) - 1
    for i, v in enumerate(vals):
        for w in range(W):
            out[i, w] = (v >> (64 * w)) & mask
    return out


def words_to_ints(arr: np.ndarray):
    arr = np.asarray(arr, dtype=np.uint64)
    if arr.ndim == 1:
        arr = arr[:, None]
    res = []
    for row in arr:
        v = 0
        for w in range(arr.shape[1] - 1, -1, -1):
            v = (v << 64) | int(row[w])
        res.append(v)
    return res


def sort_keys(dets: np.ndarray) -> np.ndarray:
    """Sort (n, W) uint64 rows as unsigned W*64-bit integers (word W-1 major)."""
    if dets.shape[0] == 0:
        return dets
    order = np.lexsort(tuple(dets[:, w] for w in range(dets.shape[1])))
    return np.ascontiguousarray(dets[order])


def _pack_bits(bits: np.ndarray, W: int) -> np.ndarray:
    """bits: (m, 2*n_orb) bool -> (m, W) uint64."""
    m, nb = bits.shape
    out = np.zeros((m, W), dtype=np.uint64)
    for k in range(nb):
        col = bits[:, k].astype(np.uint64) << np.uint64(k & 63)
        out[:, k >> 6] |= col
    return out


def _unique_rows_first(dets: np.ndarray):
    """Indices of first occurrences of each distinct row, in original order."""
    view = np.ascontiguousarray(dets).view(np.dtype((np.void, dets.dtype.itemsize * dets.shape[1])))
    _, first = np.unique(view.reshape(-1), return_index=True)
    return np.sort(first)


# ---------------------------------------------------------------------------
# selected sets
# ---------------------------------------------------------------------------

def _random_excitation_bits(rng, bits: np.ndarray, n_orb: int, n_alpha: int, n_beta: int):
    """One uniform pick among all spin-conserving singles and doubles of `bits`.

    Class sizes (alpha single, beta single, alpha-alpha, beta-beta, alpha-beta)
    weight the class draw, then holes and particles are uniform within it, so
    every single/double excitation is equally likely.
    """
    occ_a = np.flatnonzero(bits[:n_orb]); vir_a = np.flatnonzero(~bits[:n_orb])
    occ_b = np.flatnonzero(bits[n_orb:]); vir_b = np.flatnonzero(~bits[n_orb:])
    va, vb = n_orb - n_alpha, n_orb - n_beta
    sizes = np.array([
        n_alpha * va, n_beta * vb,
        math.comb(n_alpha, 2) * math.comb(va, 2), math.comb(n_beta, 2) * math.comb(vb, 2),
        n_alpha * va * n_beta * vb,
    ], dtype=np.float64)
    cls = rng.choice(5, p=sizes / sizes.sum())
    out = bits.copy()
    if cls == 0 or cls == 4:
        out[rng.choice(occ_a)] = False
        out[rng.choice(vir_a)] = True
    if cls == 1 or cls == 4:
        out[n_orb + rng.choice(occ_b)] = False
        out[n_orb + rng.choice(vir_b)] = True
    if cls == 2:
        out[rng.choice(occ_a, 2, replace=False)] = False
        out[rng.choice(vir_a, 2, replace=False)] = True
    if cls == 3:
        out[n_orb + rng.choice(occ_b, 2, replace=False)] = False
        out[n_orb + rng.choice(vir_b, 2, replace=False)] = True
    return out


def select_walk(rng, n_orb, n_alpha, n_beta, n_sel) -> np.ndarray:
    """S = {ref}; repeat: pick a uniform member, apply a uniform single/double, insert if new."""
    ref = np.zeros(2 * n_orb, dtype=bool)
    ref[:n_alpha] = True
    ref[n_orb:n_orb + n_beta] = True
    members = [ref]
    seen = {ref.tobytes()}
    guard = 0
    while len(members) < n_sel:
        src = members[rng.integers(len(members))]
        new = _random_excitation_bits(rng, src, n_orb, n_alpha, n_beta)
        key = new.tobytes()
        if key not in seen:
            seen.add(key)
            members.append(new)
        guard += 1
        if guard > 1000 * n_sel:
            raise RuntimeError("walk cannot reach the requested size")
    return sort_keys(_pack_bits(np.array(members), n_words(n_orb)))


def _level_populations(n_orb, n_alpha, n_beta, max_level):
    va, vb = n_orb - n_alpha, n_orb - n_beta
    splits = []
    for la in range(0, max_level + 1):
        for lb in range(0, max_level + 1 - la):
            if la + lb == 0:
                continue
            pop = math.comb(n_alpha, la) * math.comb(va, la) * math.comb(n_beta, lb) * math.comb(vb, lb)
            if pop > 0:
                splits.append((la, lb, pop))
    return splits


def _subset_rows(rng, m, n, k):
    """m uniform k-subsets of range(n), as an (m, k) index array."""
    if k == 0:
        return np.zeros((m, 0), dtype=np.int64)
    return np.argsort(rng.random((m, n)), axis=1)[:, :k]


def select_levels(rng, n_orb, n_alpha, n_beta, n_sel, max_level=4) -> np.ndarray:
    """ref + uniform draws (without replacement) over all dets of excitation level 1..max_level.

    The (level_alpha, level_beta) split is drawn in proportion to its population,
    then holes and particles are uniform subsets of the reference's occupied and
    virtual orbitals of each spin; repeated draws are rejected.
    """
    W = n_words(n_orb)
    splits = _level_populations(n_orb, n_alpha, n_beta, max_level)
    pops = np.array([s[2] for s in splits], dtype=np.float64)
    total = pops.sum()
    if n_sel - 1 > total:
        raise ValueError("not enough determinants up to the requested level")
    if n_sel - 1 > 0.25 * total and math.comb(n_orb, n_alpha) * math.comb(n_orb, n_beta) <= 4_000_000:
        # a large share of a small space: enumerate it and take a uniform subset
        return _select_levels_enumerated(rng, n_orb, n_alpha, n_beta, n_sel, max_level)
    ref_bits = np.zeros(2 * n_orb, dtype=bool)
    ref_bits[:n_alpha] = True
    ref_bits[n_orb:n_orb + n_beta] = True
    chosen = _pack_bits(ref_bits[None, :], W)
    va, vb = n_orb - n_alpha, n_orb - n_beta
    while chosen.shape[0] < n_sel:
        need = n_sel - chosen.shape[0]
        m = int(need * 1.05) + 16
        which = rng.choice(len(splits), size=m, p=pops / total)
        batch = np.zeros((m, 2 * n_orb), dtype=bool)
        batch[:] = ref_bits
        for si, (la, lb, _) in enumerate(splits):
            rows = np.flatnonzero(which == si)
            if rows.size == 0:
                continue
            r = rows.size
            ha = _subset_rows(rng, r, n_alpha, la)
            pa = _subset_rows(rng, r, va, la) + n_alpha
            hb = _subset_rows(rng, r, n_beta, lb) + n_orb
            pb = _subset_rows(rng, r, vb, lb) + n_beta + n_orb
            for cols, val in ((ha, False), (pa, True), (hb, False), (pb, True)):
                if cols.shape[1]:
                    sub = batch[rows]
                    np.put_along_axis(sub, cols, val, axis=1)
                    batch[rows] = sub
        allk = np.concatenate([chosen, _pack_bits(batch, W)])
        keep = _unique_rows_first(allk)
        chosen = allk[keep][: n_sel]
    return sort_keys(chosen)


def _select_levels_enumerated(rng, n_orb, n_alpha, n_beta, n_sel, max_level):
    full = all_determinants(n_orb, n_alpha, n_beta)
    W = n_words(n_orb)
    ref = np.zeros(2 * n_orb, dtype=bool)
    ref[:n_alpha] = True
    ref[n_orb:n_orb + n_beta] = True
    ref_w = _pack_bits(ref[None, :], W)[0]
    x = full ^ ref_w
    moved = np.zeros(full.shape[0], dtype=np.int64)
    for j in range(W):
        moved += np.unpackbits(x[:, j:j + 1].view(np.uint8), axis=1).sum(axis=1).astype(np.int64)
    level = moved // 2
    pool = np.flatnonzero((level >= 1) & (level <= max_level))
    pick = rng.choice(pool.shape[0], size=n_sel - 1, replace=False)
    chosen = np.concatenate([ref_w[None, :], full[pool[np.sort(pick)]]])
    return sort_keys(chosen)


def select_hf_sd(rng, n_orb, n_alpha, n_beta, n_sel) -> np.ndarray:
    """ref + every single of the reference + uniform doubles without replacement."""
    W = n_words(n_orb)
    occ_a = np.arange(n_alpha); vir_a = np.arange(n_alpha, n_orb)
    occ_b = np.arange(n_beta) + n_orb; vir_b = np.arange(n_beta, n_orb) + n_orb
    ref_bits = np.zeros(2 * n_orb, dtype=bool)
    ref_bits[:n_alpha] = True
    ref_bits[n_orb:n_orb + n_beta] = True

    def flip_rows(flips):
        rows = np.repeat(ref_bits[None, :], flips.shape[0], axis=0)
        rows[np.arange(flips.shape[0])[:, None], flips] ^= True
        return rows

    singles = np.concatenate([
        np.array([[p, a] for p in occ_a for a in vir_a], dtype=np.int64).reshape(-1, 2),
        np.array([[p, a] for p in occ_b for a in vir_b], dtype=np.int64).reshape(-1, 2),
    ])
    pa = np.array([(p, q) for i, p in enumerate(occ_a) for q in occ_a[i + 1:]], dtype=np.int64).reshape(-1, 2)
    va = np.array([(a, b) for i, a in enumerate(vir_a) for b in vir_a[i + 1:]], dtype=np.int64).reshape(-1, 2)
    pb = np.array([(p, q) for i, p in enumerate(occ_b) for q in occ_b[i + 1:]], dtype=np.int64).reshape(-1, 2)
    vb = np.array([(a, b) for i, a in enumerate(vir_b) for b in vir_b[i + 1:]], dtype=np.int64).reshape(-1, 2)
    sa = np.array([(p, a) for p in occ_a for a in vir_a], dtype=np.int64).reshape(-1, 2)
    sb = np.array([(p, a) for p in occ_b for a in vir_b], dtype=np.int64).reshape(-1, 2)
    n_aa = len(pa) * len(va)
    n_bb = len(pb) * len(vb)
    n_ab = len(sa) * len(sb)
    n_doubles = n_aa + n_bb + n_ab
    n_dbl_pick = n_sel - 1 - len(singles)
    if n_dbl_pick < 0 or n_dbl_pick > n_doubles:
        raise ValueError("selected-set size does not fit reference + singles + doubles")
    pick = np.sort(rng.choice(n_doubles, size=n_dbl_pick, replace=False))
    flips = np.zeros((n_dbl_pick, 4), dtype=np.int64)
    m = pick < n_aa
    i = pick[m]
    flips[m] = np.concatenate([pa[i // len(va)], va[i % len(va)]], axis=1)
    m2 = (pick >= n_aa) & (pick < n_aa + n_bb)
    i = pick[m2] - n_aa
    flips[m2] = np.concatenate([pb[i // len(vb)], vb[i % len(vb)]], axis=1)
    m3 = pick >= n_aa + n_bb
    i = pick[m3] - n_aa - n_bb
    flips[m3] = np.concatenate([sa[i // len(sb)], sb[i % len(sb)]], axis=1)
    rows = np.concatenate([ref_bits[None, :], flip_rows(singles), flip_rows(flips)])
    return sort_keys(_pack_bits(rows, W))


def all_determinants(n_orb, n_alpha, n_beta) -> np.ndarray:
    """Every determinant of the space (full-CI basis), sorted."""
    from itertools import combinations
    W = n_words(n_orb)
    vals = []
    for ca in combinations(range(n_orb), n_alpha):
        for cb in combinations(range(n_orb), n_beta):
            vals.append(pack_int(ca, cb, n_orb))
    return sort_keys(ints_to_words(vals, W))


# ---------------------------------------------------------------------------
# whole systems
# ---------------------------------------------------------------------------

@dataclass
class System:
    workload: Workload
    h1: np.ndarray
    eri: np.ndarray
    dets: np.ndarray  # (n_sel, W) uint64, strictly ascending
    psi: np.ndarray   # (n_sel,) float64, unit norm

    @property
    def n_orb(self):
        return self.workload.n_orb

    @property
    def n_alpha(self):
        return self.workload.n_alpha

    @property
    def n_beta(self):
        return self.workload.n_beta

    @property
    def W(self):
        return self.workload.W


def make_system(wl: Workload) -> System:
    rng = np.random.Generator(np.random.PCG64(wl.seed))
    h1 = make_h1(rng, wl.n_orb)
    eri = make_eri(rng, wl.n_orb, wl.rank)
    if wl.selection == "walk":
        dets = select_walk(rng, wl.n_orb, wl.n_alpha, wl.n_beta, wl.n_sel)
    elif wl.selection == "levels":
        dets = select_levels(rng, wl.n_orb, wl.n_alpha, wl.n_beta, wl.n_sel)
    elif wl.selection == "hf_sd":
        dets = select_hf_sd(rng, wl.n_orb, wl.n_alpha, wl.n_beta, wl.n_sel)
    elif wl.selection == "all":
        dets = all_determinants(wl.n_orb, wl.n_alpha, wl.n_beta)
    else:
        raise ValueError(wl.selection)
    prng = np.random.Generator(np.random.PCG64(wl.seed + 4))
    psi = prng.standard_normal(dets.shape[0])
    psi /= np.linalg.norm(psi)
    return System(wl, h1, eri, dets, psi)


BATCH_SEED = SEED_BASE + 3


def batch_workloads(n_sys: int = 64, seed: int = BATCH_SEED):
    """The batched workload: n_sys systems of uneven size.  Shapes come from one
    stream seeded with `seed`: n_orb ~ U{10..40}, f ~ U[0.4, 0.6],
    n_alpha = n_beta = round(f * n_orb), Cholesky rank 4 n_orb, and
    n_sel = round(exp(U[ln 1e3, ln 5e4])) capped at the reference plus every
    determinant of excitation level 1-4; system k's integrals and selected set
    (reference + uniform levels 1-4, as the medium workload) use seed + 1000 (k + 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(n_sys):
        n = int(rng.integers(10, 41))
        f = float(rng.uniform(0.4, 0.6))
        ne = int(math.floor(f * n + 0.5))
        n_sel = int(math.floor(math.exp(rng.uniform(math.log(1e3), math.log(5e4))) + 0.5))
        avail = 1 + sum(p for _, _, p in _level_populations(n, ne, ne, 4))
        out.append(Workload(f"batch{k}", n, ne, ne, 4 * n, min(n_sel, avail), "levels", seed + 1000 * (k + 1)))
    return out


def small_workload(n_orb, n_alpha, n_beta, n_sel=None, seed=SEED_BASE + 77, rank=None, selection=None):
    """A seeded tiny system for tests (full space when n_sel is None)."""
    if rank is None:
        rank = 2 * n_orb + 2
    if selection is None:
        selection = "all" if n_sel is None else "walk"
    if n_sel is None:
        n_sel = math.comb(n_orb, n_alpha) * math.comb(n_orb, n_beta)
    return Workload(f"small_{n_orb}_{n_alpha}_{n_beta}", n_orb, n_alpha, n_beta, rank, n_sel, selection, seed)


def random_orthogonal(rng, n):
    q, r = np.linalg.qr(rng.standard_normal((n, n)))
    return q * np.sign(np.diag(r))


def rotate_integrals(h1, eri, u):
    """Integrals in the rotated orbital basis phi'_i = sum_p phi_p U_pi."""
    h2 = u.T @ h1 @ u
    e = np.einsum("pqrs,pi->iqrs", eri, u)
    e = np.einsum("iqrs,qj->ijrs", e, u)
    e = np.einsum("ijrs,rk->ijks", e, u)
    e = np.einsum("ijks,sl->ijkl", e, u)
    return np.ascontiguousarray((h2 + h2.T) / 2), symmetrize8(e)
