"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Nothing here re-types the oracle's formulas: each check is a closed form, an
invariant, an independent library routine, or brute force on a tiny space.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle
import sci_inputs as si

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _tiny_system(n_orb, na, nb, seed=11, rank=None):
    rng = np.random.Generator(np.random.PCG64(seed))
    h1 = si.make_h1(rng, n_orb)
    eri = si.make_eri(rng, n_orb, rank or 2 * n_orb + 2)
    return h1, eri


def _ints(keys):
    return si.words_to_ints(keys)


# ---------------------------------------------------------------------------
# excitation counts and structure (Eq. 4, section 2.1: at most two moved ones)
# ---------------------------------------------------------------------------

def _closed_form_count(n, na, nb):
    va, vb = n - na, n - nb
    return (na * va + nb * vb + math.comb(na, 2) * math.comb(va, 2)
            + math.comb(nb, 2) * math.comb(vb, 2) + na * va * nb * vb)


def test_tiny_regression_fixture():
    """The stored tiny-workload results (written once by tests/golden/make_golden.py
    from the oracle) still come out of the oracle: a regression pin of the oracle and
    of the seeded input generator together.  Counts that the mathematics fixes are
    checked against the closed form besides: 200 sources x 140 coupled candidates,
    and the union with S is the whole 441-determinant space (C(7,5)^2)."""
    import hashlib
    with open(os.path.join(GOLDEN, "tiny_oracle.json")) as f:
        ref = json.load(f)
    wl = si.WORKLOADS["tiny"]
    s = si.make_system(wl)
    keys, hij, _ = oracle.gen_coupled(wl.n_orb, wl.n_alpha, wl.n_beta, s.h1, s.eri, s.dets)
    assert keys.shape[0] == ref["n_candidates"] == 200 * _closed_form_count(7, 5, 5)
    assert hashlib.sha256(np.ascontiguousarray(keys).tobytes()).hexdigest() == ref["keys_sha256"]
    assert np.allclose(hij[:8], ref["hij_first"], rtol=0, atol=1e-13)
    assert abs(float(np.abs(hij).sum()) - ref["hij_abs_sum"]) <= 1e-9
    u, nov = oracle.dedup_merge(wl.W, keys, s.dets)
    assert u.shape[0] == ref["n_unique_with_sel"] == math.comb(7, 5) ** 2
    assert nov.shape[0] == ref["n_novel"] == 441 - s.dets.shape[0]
    e, hp, g = oracle.energy(wl.n_orb, wl.n_alpha, wl.n_beta, s.h1, s.eri, s.dets, s.psi)
    assert abs(e - ref["energy"]) <= 1e-12
    assert np.allclose(hp[:4], ref["hpsi_first"], rtol=0, atol=1e-12)
    assert np.allclose(g[:4], ref["grad_first"], rtol=0, atol=1e-12)


def test_golden_counts_fixture():
    with open(os.path.join(GOLDEN, "coupled_counts.json")) as f:
        data = json.load(f)
    for row in data["cases"]:
        assert oracle.n_coupled(row["n_orb"], row["n_alpha"], row["n_beta"]) == row["per_source"]
        assert _closed_form_count(row["n_orb"], row["n_alpha"], row["n_beta"]) == row["per_source"]


@pytest.mark.parametrize("n,na,nb", [(7, 5, 5), (6, 3, 2), (5, 1, 1), (8, 2, 0), (9, 4, 3), (34, 3, 2)])
def test_coupled_set_structure(n, na, nb):
    h1, eri = _tiny_system(n, na, nb)
    W = si.n_words(n)
    rng = np.random.Generator(np.random.PCG64(5))
    srcs = []
    for _ in range(6):
        a = rng.choice(n, na, replace=False)
        b = rng.choice(n, nb, replace=False)
        srcs.append(si.pack_int(a, b, n))
    dets = si.sort_keys(si.ints_to_words(sorted(set(srcs)), W))
    keys, hij, src = oracle.gen_coupled(n, na, nb, h1, eri, dets)
    nc = _closed_form_count(n, na, nb)
    assert keys.shape[0] == nc * dets.shape[0]
    amask = (1 << n) - 1
    for i, d in enumerate(_ints(dets)):
        ci = _ints(keys[i * nc:(i + 1) * nc])
        assert len(set(ci)) == nc, "duplicates inside C_i"
        assert d not in ci
        for c in ci:
            x = c ^ d
            assert bin(x).count("1") in (2, 4)
            assert bin(c & amask).count("1") == na
            assert bin(c >> n).count("1") == nb
        # brute force: every det at <=2 moved electrons of each kind
        brute = set()
        occ = [k for k in range(2 * n) if d >> k & 1]
        vir = [k for k in range(2 * n) if not d >> k & 1]
        for r in (1, 2):
            for holes in itertools.combinations(occ, r):
                for parts in itertools.combinations(vir, r):
                    e = d
                    for k in holes + parts:
                        e ^= 1 << k
                    if bin(e & amask).count("1") == na and bin(e >> n).count("1") == nb:
                        brute.add(e)
        assert brute == set(ci)


def test_canonical_order_classes():
    """Dense order: alpha singles, beta singles, aa, bb, ab (class boundaries by closed form)."""
    n, na, nb = 6, 3, 2
    h1, eri = _tiny_system(n, na, nb)
    d = si.ints_to_words([si.pack_int([0, 2, 4], [1, 3], n)], 1)
    keys, _, _ = oracle.gen_coupled(n, na, nb, h1, eri, d)
    src = _ints(d)[0]
    va, vb = n - na, n - nb
    bounds = np.cumsum([0, na * va, nb * vb, math.comb(na, 2) * math.comb(va, 2),
                        math.comb(nb, 2) * math.comb(vb, 2), na * va * nb * vb])
    amask = (1 << n) - 1
    for cls in range(5):
        for c in _ints(keys[bounds[cls]:bounds[cls + 1]]):
            x = c ^ src
            ka, kb = bin(x & amask).count("1"), bin(x >> n).count("1")
            assert (ka, kb) == [(2, 0), (0, 2), (4, 0), (0, 4), (2, 2)][cls]
    # within each class the keys follow the hole/particle lexicographic order;
    # for the mixed class check (p,q,a,b) monotone
    ab = _ints(keys[bounds[4]:bounds[5]])
    tup = []
    for c in ab:
        x = c ^ src
        p = [k for k in range(n) if (x >> k & 1) and (src >> k & 1)][0]
        a = [k for k in range(n) if (x >> k & 1) and not (src >> k & 1)][0]
        q = [k for k in range(n) if (x >> (k + n) & 1) and (src >> (k + n) & 1)][0]
        b = [k for k in range(n) if (x >> (k + n) & 1) and not (src >> (k + n) & 1)][0]
        tup.append((p, q, a, b))
    assert tup == sorted(tup)


# ---------------------------------------------------------------------------
# literal tier == Slater-Condon tier (sets exactly, values to 1e-13)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,na,nb", [(7, 5, 5), (5, 2, 3), (6, 1, 2), (4, 2, 2), (33, 2, 1)])
def test_literal_equals_slater_condon(n, na, nb):
    h1, eri = _tiny_system(n, na, nb, seed=n * 31 + na)
    W = si.n_words(n)
    rng = np.random.Generator(np.random.PCG64(n))
    picks = set()
    while len(picks) < 5:
        picks.add(si.pack_int(rng.choice(n, na, replace=False), rng.choice(n, nb, replace=False), n))
    dets = si.sort_keys(si.ints_to_words(sorted(picks), W))
    nc = _closed_form_count(n, na, nb)
    keys, hij, _ = oracle.gen_coupled(n, na, nb, h1, eri, dets)
    for i in range(dets.shape[0]):
        lk, lv = oracle.literal_row(n, na, nb, h1, eri, dets[i])
        lit = dict(zip(_ints(lk), lv))
        d = _ints(dets[i:i + 1])[0]
        dval = lit.pop(d)
        assert abs(dval - oracle.diag(n, na, nb, h1, eri, dets[i])) < 1e-12
        sc = dict(zip(_ints(keys[i * nc:(i + 1) * nc]), hij[i * nc:(i + 1) * nc]))
        assert set(lit) == set(sc)
        for k in sc:
            assert abs(lit[k] - sc[k]) < 1e-13


# ---------------------------------------------------------------------------
# textbook two-electron closed forms (signs and two-body indices)
# ---------------------------------------------------------------------------

def test_two_electron_opposite_spin_closed_form():
    n = 5
    h1, eri = _tiny_system(n, 1, 1, seed=3)
    basis = si.all_determinants(n, 1, 1)
    for H in (oracle.dense_h_literal(n, 1, 1, h1, eri, basis), oracle.dense_h_sc(n, 1, 1, h1, eri, basis)):
        for i, di in enumerate(_ints(basis)):
            p = (di & ((1 << n) - 1)).bit_length() - 1
            q = (di >> n).bit_length() - 1
            for j, dj in enumerate(_ints(basis)):
                r = (dj & ((1 << n) - 1)).bit_length() - 1
                s = (dj >> n).bit_length() - 1
                ref = h1[p, r] * (q == s) + (p == r) * h1[q, s] + eri[p, r, q, s]
                assert abs(H[i, j] - ref) < 1e-13


def test_two_electron_same_spin_closed_form():
    n = 6
    h1, eri = _tiny_system(n, 2, 0, seed=4)
    basis = si.all_determinants(n, 2, 0)
    for H in (oracle.dense_h_literal(n, 2, 0, h1, eri, basis), oracle.dense_h_sc(n, 2, 0, h1, eri, basis)):
        for i, di in enumerate(_ints(basis)):
            p, q = [k for k in range(n) if di >> k & 1]
            for j, dj in enumerate(_ints(basis)):
                r, s = [k for k in range(n) if dj >> k & 1]
                ref = (h1[p, r] * (q == s) + h1[q, s] * (p == r) - h1[p, s] * (q == r) - h1[q, r] * (p == s)
                       + eri[p, r, q, s] - eri[p, s, q, r])
                assert abs(H[i, j] - ref) < 1e-13


# ---------------------------------------------------------------------------
# full-CI invariants on tiny spaces
# ---------------------------------------------------------------------------

def test_fci_hermitian_and_sc_matches_literal():
    wl = si.WORKLOADS["tiny"]
    sysm = si.make_system(wl)
    basis = si.all_determinants(wl.n_orb, wl.n_alpha, wl.n_beta)
    assert basis.shape[0] == math.comb(7, 5) ** 2 == 441
    hl = oracle.dense_h_literal(wl.n_orb, wl.n_alpha, wl.n_beta, sysm.h1, sysm.eri, basis)
    hs = oracle.dense_h_sc(wl.n_orb, wl.n_alpha, wl.n_beta, sysm.h1, sysm.eri, basis)
    assert np.max(np.abs(hl - hs)) < 1e-12
    assert np.max(np.abs(hs - hs.T)) < 1e-14
    # j in C_i <=> i in C_j (structural)
    assert np.array_equal(hs != 0, (hs != 0).T)
    # variational bound: every Rayleigh quotient lies above the lowest eigenvalue
    lam = np.linalg.eigvalsh(hs)[0]
    rng = np.random.Generator(np.random.PCG64(1))
    for _ in range(5):
        v = rng.standard_normal(basis.shape[0])
        assert v @ hs @ v / (v @ v) >= lam - 1e-12


def test_noninteracting_ground_state():
    """ERI = 0: E0 = sum of the lowest n_alpha + lowest n_beta eigenvalues of h."""
    for n, na, nb in [(6, 3, 2), (5, 2, 2), (7, 3, 4)]:
        h1, _ = _tiny_system(n, na, nb, seed=9 + n)
        eri = np.zeros((n,) * 4)
        basis = si.all_determinants(n, na, nb)
        hs = oracle.dense_h_sc(n, na, nb, h1, eri, basis)
        eps = np.linalg.eigvalsh(h1)
        assert abs(np.linalg.eigvalsh(hs)[0] - (eps[:na].sum() + eps[:nb].sum())) < 1e-12
        # the whole spectrum is the set of sums of occupied orbital energies
        spec = sorted(sum(eps[list(a)]) + sum(eps[list(b)])
                      for a in itertools.combinations(range(n), na)
                      for b in itertools.combinations(range(n), nb))
        assert np.max(np.abs(np.linalg.eigvalsh(hs) - np.array(spec))) < 1e-11


@pytest.mark.parametrize("n,na,nb", [(5, 2, 2), (6, 3, 1)])
def test_orbital_rotation_invariance(n, na, nb):
    h1, eri = _tiny_system(n, na, nb, seed=21)
    rng = np.random.Generator(np.random.PCG64(22))
    u = si.random_orthogonal(rng, n)
    h2, eri2 = si.rotate_integrals(h1, eri, u)
    basis = si.all_determinants(n, na, nb)
    e1 = np.linalg.eigvalsh(oracle.dense_h_sc(n, na, nb, h1, eri, basis))
    e2 = np.linalg.eigvalsh(oracle.dense_h_sc(n, na, nb, h2, eri2, basis))
    assert np.max(np.abs(e1 - e2)) < 1e-10
    # a sign mistake breaks the invariance: flip the sign convention of the
    # two-body part and the spectra disagree (sanity of the test itself)
    e3 = np.linalg.eigvalsh(oracle.dense_h_sc(n, na, nb, h2, -eri2, basis))
    assert np.max(np.abs(e1 - e3)) > 1e-3


def test_screening_keeps_strictly_greater():
    n, na, nb = 6, 3, 2
    h1, eri = _tiny_system(n, na, nb)
    d = si.ints_to_words([si.pack_int([0, 2, 4], [1, 3], n)], 1)
    k0, h0, _ = oracle.gen_coupled(n, na, nb, h1, eri, d)
    eps = float(np.median(np.abs(h0)))
    k1, h1v, s1 = oracle.gen_coupled(n, na, nb, h1, eri, d, eps=eps)
    want = [(int(k[0]), v) for k, v in zip(k0, h0) if abs(v) > eps]
    assert [(int(k[0]), v) for k, v in zip(k1, h1v)] == want
    assert np.all(s1 == 0)


# ---------------------------------------------------------------------------
# de-duplication set algebra (section 4.1)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("W", [1, 2])
def test_dedup_set_algebra(W):
    rng = np.random.Generator(np.random.PCG64(7 + W))
    pool = rng.integers(0, 2**63, size=(300, W), dtype=np.int64).astype(np.uint64)
    pool[:, -1] |= np.uint64(1) << np.uint64(63)  # exercise the unsigned top bit
    pool[:50, -1] = 0  # and small keys
    a = pool[rng.integers(0, 300, 2000)]
    b = pool[rng.integers(0, 300, 700)]
    ua, _ = oracle.dedup_merge(W, a)
    assert _ints(ua) == sorted(set(_ints(a)))
    assert all(x < y for x, y in zip(_ints(ua), _ints(ua)[1:]))
    again, nov = oracle.dedup_merge(W, ua, ua)
    assert _ints(again) == _ints(ua) and nov.shape[0] == 0
    ub, _ = oracle.dedup_merge(W, b)
    m, novel = oracle.dedup_merge(W, a, ub)
    both, _ = oracle.dedup_merge(W, np.concatenate([a, b]))
    assert _ints(m) == _ints(both)
    assert set(_ints(novel)) == set(_ints(a)) - set(_ints(b))
    assert not set(_ints(novel)) & set(_ints(ub))
    with pytest.raises(ValueError):
        oracle.dedup_merge(W, a, a[:10][::-1])
    e, en = oracle.dedup_merge(W, np.zeros((0, W), np.uint64), ub)
    assert _ints(e) == _ints(ub) and en.shape[0] == 0


# ---------------------------------------------------------------------------
# energy and gradient (Eq. 1)
# ---------------------------------------------------------------------------

def test_energy_matches_dense_rayleigh_quotient():
    wl = si.WORKLOADS["tiny"]
    s = si.make_system(wl)
    e, hp, g = oracle.energy(wl.n_orb, wl.n_alpha, wl.n_beta, s.h1, s.eri, s.dets, s.psi)
    hd = oracle.dense_h_literal(wl.n_orb, wl.n_alpha, wl.n_beta, s.h1, s.eri, s.dets)
    assert np.max(np.abs(hd @ s.psi - hp)) < 1e-12
    assert abs(e - s.psi @ hd @ s.psi / (s.psi @ s.psi)) < 1e-12
    # scale invariance and orthogonality of the gradient
    e2, _, g2 = oracle.energy(wl.n_orb, wl.n_alpha, wl.n_beta, s.h1, s.eri, s.dets, 3.5 * s.psi)
    assert abs(e2 - e) < 1e-13
    assert abs(s.psi @ g) < 1e-13
    assert np.max(np.abs(g2 * 3.5 - g)) < 1e-12


def test_gradient_complex_step_and_finite_difference():
    wl = si.WORKLOADS["tiny"]
    s = si.make_system(wl)
    _, _, g = oracle.energy(wl.n_orb, wl.n_alpha, wl.n_beta, s.h1, s.eri, s.dets, s.psi)
    hd = oracle.dense_h_literal(wl.n_orb, wl.n_alpha, wl.n_beta, s.h1, s.eri, s.dets)
    rng = np.random.Generator(np.random.PCG64(3))
    v = rng.standard_normal(s.psi.shape[0])
    v /= np.linalg.norm(v)
    # complex step on the analytic continuation E(z) = z^T H z / z^T z
    h = 1e-30
    z = s.psi + 1j * h * v
    cs = ((z @ hd @ z) / (z @ z)).imag / h
    assert abs(cs - g @ v) < 1e-13
    # central differences through the oracle itself, O(h^2)
    errs = []
    for step in (1e-3, 1e-4):
        ep, _, _ = oracle.energy(wl.n_orb, wl.n_alpha, wl.n_beta, s.h1, s.eri, s.dets, s.psi + step * v)
        em, _, _ = oracle.energy(wl.n_orb, wl.n_alpha, wl.n_beta, s.h1, s.eri, s.dets, s.psi - step * v)
        errs.append(abs((ep - em) / (2 * step) - g @ v))
    assert errs[1] < 1e-7 and errs[1] < errs[0]


def test_eigenvector_has_zero_gradient():
    n, na, nb = 5, 2, 2
    h1, eri = _tiny_system(n, na, nb, seed=8)
    basis = si.all_determinants(n, na, nb)
    hd = oracle.dense_h_literal(n, na, nb, h1, eri, basis)
    w, v = np.linalg.eigh(hd)
    e, _, g = oracle.energy(n, na, nb, h1, eri, basis, v[:, 0])
    assert abs(e - w[0]) < 1e-12
    assert np.max(np.abs(g)) < 1e-11


def test_hpsi_rows_match_full():
    wl = si.WORKLOADS["tiny"]
    s = si.make_system(wl)
    _, hp, _ = oracle.energy(wl.n_orb, wl.n_alpha, wl.n_beta, s.h1, s.eri, s.dets, s.psi)
    rows = np.array([0, 5, 199, 17])
    got = oracle.hpsi_rows(wl.n_orb, wl.n_alpha, wl.n_beta, s.h1, s.eri, s.dets, s.psi, rows)
    assert np.max(np.abs(got - hp[rows])) < 1e-15


def test_invalid_inputs_rejected():
    n, na, nb = 6, 3, 2
    h1, eri = _tiny_system(n, na, nb)
    bad = si.ints_to_words([si.pack_int([0, 1], [1, 3], n)], 1)
    with pytest.raises(ValueError):
        oracle.gen_coupled(n, na, nb, h1, eri, bad)
    d = si.all_determinants(n, na, nb)[:4]
    with pytest.raises(ValueError):
        oracle.energy(n, na, nb, h1, eri, d[::-1], np.ones(4))
