"""CPU oracle for the NNQS-SCI hot path — TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package; the product path (the HIP library and its binding) never imports it.
It shares no code with the HIP path.

The arithmetic lives in ``sci_oracle.c`` (plain C, OpenMP over sources):

* ``literal_row``   — H|D> by applying every term of the second-quantised
  Hamiltonian with explicit creation/annihilation operators (the definition;
  paper Eqs. 1-4).
* ``gen_coupled``   — the coupled set C_i of Eq. 4 (spin-conserving singles and
  doubles) with Slater–Condon elements, operators still applied explicitly.
* ``dedup_merge``   — sorted set union / difference (section 4.1).
* ``energy``        — Rayleigh quotient of Eq. 1 over the selected space and its
  gradient 2(H psi - E psi)/(psi.psi); ``hpsi_rows`` for sampled rows.

Python helpers here only assemble dense matrices from those rows for the
numpy eigen-solver checks.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sci_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libsci_oracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP) into oracle/libsci_oracle.so."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i32, i64, f64 = ctypes.c_int, ctypes.c_int64, ctypes.c_double
        lib.ora_literal_row.argtypes = [i32, i32, i32, i32, P, P, P, P, P, i64]
        lib.ora_literal_row.restype = i64
        lib.ora_n_coupled.argtypes = [i32, i32, i32]
        lib.ora_n_coupled.restype = i64
        lib.ora_diag.argtypes = [i32, i32, i32, i32, P, P, P]
        lib.ora_diag.restype = f64
        lib.ora_gen_coupled.argtypes = [i32, i32, i32, i32, P, P, P, i64, f64, P, P, P, i64]
        lib.ora_gen_coupled.restype = i64
        lib.ora_dedup_merge.argtypes = [i32, P, i64, P, i64, P, i64, P, i64, P]
        lib.ora_dedup_merge.restype = i64
        lib.ora_energy.argtypes = [i32, i32, i32, i32, P, P, P, i64, P, P, P, P]
        lib.ora_energy.restype = i32
        lib.ora_hpsi_rows.argtypes = [i32, i32, i32, i32, P, P, P, i64, P, P, i64, P]
        lib.ora_hpsi_rows.restype = i32
        lib.ora_dense_h.argtypes = [i32, i32, i32, i32, P, P, P, i64, P]
        lib.ora_dense_h.restype = i32
        lib.ora_inverse_map.argtypes = [i32, P, i64, P, i64, P]
        lib.ora_inverse_map.restype = i32
        lib.ora_topk.argtypes = [i32, P, P, i64, i64, P]
        lib.ora_topk.restype = i64
        lib.ora_num_threads.argtypes = []
        lib.ora_num_threads.restype = i32
        _lib = lib
        return lib


class use_library:
    """Context manager: route every oracle call to another build of the oracle
    source (the tests use it to check that planted mistakes fail the pins)."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib
        _load()
        self._saved = _lib
        lib = ctypes.CDLL(self.path)
        for fn in ("ora_literal_row", "ora_n_coupled", "ora_diag", "ora_gen_coupled", "ora_dedup_merge",
                   "ora_energy", "ora_hpsi_rows", "ora_dense_h", "ora_num_threads"):
            src = getattr(self._saved, fn)
            dst = getattr(lib, fn)
            dst.argtypes = src.argtypes
            dst.restype = src.restype
        _lib = lib
        return lib

    def __exit__(self, *exc):
        global _lib
        _lib = self._saved
        return False


def compile_variant(source_text: str, out_path: str) -> str:
    """Compile C source text (a modified copy of the oracle) to a shared library."""
    c_path = out_path + ".c"
    with open(c_path, "w") as f:
        f.write(source_text)
    subprocess.run(["gcc", "-O1", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", out_path, c_path, "-lm"],
                   check=True)
    return out_path


def source_text() -> str:
    with open(_SRC) as f:
        return f.read()


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _ham(h1, eri):
    return (np.ascontiguousarray(h1, dtype=np.float64), np.ascontiguousarray(eri, dtype=np.float64))


def _dets(d, W):
    d = np.ascontiguousarray(d, dtype=np.uint64)
    return d.reshape(-1, W)


def words(n_orb: int) -> int:
    return (2 * n_orb + 63) // 64


def num_threads() -> int:
    return int(_load().ora_num_threads())


def n_coupled(n_orb: int, n_alpha: int, n_beta: int) -> int:
    return int(_load().ora_n_coupled(n_orb, n_alpha, n_beta))


def literal_row(n_orb, n_alpha, n_beta, h1, eri, det):
    """(keys (m,W), values (m,)) of H|det>, every determinant any term reaches."""
    W = words(n_orb)
    h1, eri = _ham(h1, eri)
    det = _dets(det, W)[0].copy()
    cap = 4096
    while True:
        keys = np.zeros((cap, W), dtype=np.uint64)
        vals = np.zeros(cap, dtype=np.float64)
        n = _load().ora_literal_row(n_orb, n_alpha, n_beta, W, _p(h1), _p(eri), _p(det), _p(keys), _p(vals), cap)
        if n == -1:
            cap *= 4
            continue
        if n < 0:
            raise ValueError("invalid determinant")
        return keys[:n], vals[:n]


def diag(n_orb, n_alpha, n_beta, h1, eri, det) -> float:
    W = words(n_orb)
    h1, eri = _ham(h1, eri)
    det = _dets(det, W)[0].copy()
    v = _load().ora_diag(n_orb, n_alpha, n_beta, W, _p(h1), _p(eri), _p(det))
    if np.isnan(v):
        raise ValueError("invalid determinant")
    return float(v)


def gen_coupled(n_orb, n_alpha, n_beta, h1, eri, dets, eps=-1.0):
    """Coupled singles+doubles of every source.

    eps < 0: dense canonical order, (keys (n*Nc, W), hij, src).
    eps >= 0: |H| > eps only, source-major/rank order.
    """
    W = words(n_orb)
    h1, eri = _ham(h1, eri)
    dets = _dets(dets, W)
    n = dets.shape[0]
    nc = n_coupled(n_orb, n_alpha, n_beta)
    cap = n * nc
    keys = np.zeros((cap, W), dtype=np.uint64)
    hij = np.zeros(cap, dtype=np.float64)
    src = np.zeros(cap, dtype=np.int32)
    got = _load().ora_gen_coupled(n_orb, n_alpha, n_beta, W, _p(h1), _p(eri), _p(dets), n, float(eps),
                                  _p(keys), _p(hij), _p(src), cap)
    if got < 0:
        raise ValueError("oracle gen_coupled failed (%d)" % got)
    return keys[:got], hij[:got], src[:got]


def dedup_merge(W, cand, set_in=None):
    """(sorted(set(cand) | set(set_in)), sorted(set(cand) - set(set_in)))."""
    cand = _dets(cand, W) if np.asarray(cand).size else np.zeros((0, W), dtype=np.uint64)
    if set_in is None or np.asarray(set_in).size == 0:
        set_in = np.zeros((0, W), dtype=np.uint64)
    set_in = _dets(set_in, W)
    cap = cand.shape[0] + set_in.shape[0]
    out = np.zeros((max(cap, 1), W), dtype=np.uint64)
    novel = np.zeros((max(cand.shape[0], 1), W), dtype=np.uint64)
    nn = ctypes.c_int64(0)
    got = _load().ora_dedup_merge(W, _p(cand), cand.shape[0], _p(set_in), set_in.shape[0],
                                  _p(out), out.shape[0], _p(novel), novel.shape[0], ctypes.byref(nn))
    if got == -1:
        raise ValueError("set_in is not strictly ascending")
    if got < 0:
        raise RuntimeError("oracle dedup capacity")
    return out[:got], novel[: nn.value]


def inverse_map(W, u, cand):
    """Position of each candidate in the strictly ascending set u (-1 if absent)."""
    u = _dets(u, W) if np.asarray(u).size else np.zeros((0, W), dtype=np.uint64)
    cand = _dets(cand, W) if np.asarray(cand).size else np.zeros((0, W), dtype=np.uint64)
    idx = np.zeros(max(cand.shape[0], 1), dtype=np.int64)
    rc = _load().ora_inverse_map(W, _p(u), u.shape[0], _p(cand), cand.shape[0], _p(idx))
    if rc != 0:
        raise ValueError("u is not strictly ascending")
    return idx[: cand.shape[0]]


def topk(W, keys, psi, K):
    """Mask of the K entries of largest |psi| (equal magnitudes: smaller key first)."""
    keys = _dets(keys, W) if np.asarray(keys).size else np.zeros((0, W), dtype=np.uint64)
    psi = np.ascontiguousarray(psi, dtype=np.float64)
    assert psi.shape[0] == keys.shape[0]
    mask = np.zeros(max(keys.shape[0], 1), dtype=np.uint8)
    got = _load().ora_topk(W, _p(keys), _p(psi), keys.shape[0], int(K), _p(mask))
    if got < 0:
        raise ValueError("keys are not distinct")
    return mask[: keys.shape[0]].astype(bool)


def energy(n_orb, n_alpha, n_beta, h1, eri, sel, psi):
    """(E, H psi, grad) over the selected space."""
    W = words(n_orb)
    h1, eri = _ham(h1, eri)
    sel = _dets(sel, W)
    psi = np.ascontiguousarray(psi, dtype=np.float64)
    n = sel.shape[0]
    e = np.zeros(1)
    hp = np.zeros(n)
    g = np.zeros(n)
    rc = _load().ora_energy(n_orb, n_alpha, n_beta, W, _p(h1), _p(eri), _p(sel), n, _p(psi), _p(e), _p(hp), _p(g))
    if rc != 0:
        raise ValueError("oracle energy failed (%d)" % rc)
    return float(e[0]), hp, g


def hpsi_rows(n_orb, n_alpha, n_beta, h1, eri, sel, psi, rows):
    W = words(n_orb)
    h1, eri = _ham(h1, eri)
    sel = _dets(sel, W)
    psi = np.ascontiguousarray(psi, dtype=np.float64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.zeros(rows.shape[0])
    rc = _load().ora_hpsi_rows(n_orb, n_alpha, n_beta, W, _p(h1), _p(eri), _p(sel), sel.shape[0], _p(psi),
                               _p(rows), rows.shape[0], _p(out))
    if rc != 0:
        raise ValueError("oracle hpsi_rows failed (%d)" % rc)
    return out


# ---------------------------------------------------------------------------
# dense helpers (numpy) built from oracle rows
# ---------------------------------------------------------------------------

def _index_of(sorted_dets):
    return {tuple(int(x) for x in row): i for i, row in enumerate(sorted_dets)}


def dense_h_literal(n_orb, n_alpha, n_beta, h1, eri, basis):
    """Dense <i|H|j> on `basis` (sorted dets) from literal-tier rows."""
    idx = _index_of(basis)
    n = basis.shape[0]
    hm = np.zeros((n, n))
    for j in range(n):
        keys, vals = literal_row(n_orb, n_alpha, n_beta, h1, eri, basis[j])
        for k, v in zip(keys, vals):
            i = idx.get(tuple(int(x) for x in k))
            if i is not None:
                hm[i, j] += v
    return hm


def dense_h_sc(n_orb, n_alpha, n_beta, h1, eri, basis):
    """Dense <i|H|j> on `basis` (strictly ascending) from the Slater–Condon tier."""
    W = words(n_orb)
    h1, eri = _ham(h1, eri)
    basis = _dets(basis, W)
    n = basis.shape[0]
    out = np.zeros((n, n))
    rc = _load().ora_dense_h(n_orb, n_alpha, n_beta, W, _p(h1), _p(eri), _p(basis), n, _p(out))
    if rc != 0:
        raise ValueError("oracle dense_h failed (%d)" % rc)
    return np.ascontiguousarray(out.T)  # out[j, i] = <i|H|j>
