"""Python binding of libsci (MI355X / gfx950 HIP kernels for the NNQS-SCI hot path).

Argument marshalling only: every step of generation, de-duplication and
energy runs in the HIP kernels of ``libsci.so``.  PyTorch supplies device
memory (tensors; determinant keys are stored as int64 bit patterns) and the
current HIP stream.  The functions mirror the C ABI of ``include/sci.h``:

    sci_ham_create / sci_ham_destroy      -> Ham
    sci_gen_coupled, sci_dedup_merge, sci_energy, sci_*_workspace_bytes,
    sci_n_coupled, sci_words

plus allocating conveniences (``gen_coupled``, ``dedup_merge``, ``energy``)
that size outputs and check the device flags.  There is no fallback: if the
library is not built, importing the binding fails.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsci.so")

SCI_OK, SCI_EINVAL, SCI_ECAPACITY, SCI_ENOMEM, SCI_EHIP, SCI_EUNSUPPORTED = range(6)
ENERGY_AUTO, ENERGY_PAIRS, ENERGY_ENUM = 0, 1, 2
FLAG_OVERFLOW, FLAG_BAD_DET, FLAG_UNSORTED = 0x1, 0x2, 0x4
MAX_WORDS = 2
MAX_ORB = 64

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libsci.so is not built ({LIB_PATH}); run __graft_entry__.build()")

_lib = ctypes.CDLL(LIB_PATH)
_P = ctypes.c_void_p
_i32, _i64, _f64, _sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t

_lib.sci_status_string.argtypes = [_i32]
_lib.sci_status_string.restype = ctypes.c_char_p
_lib.sci_last_error.argtypes = []
_lib.sci_last_error.restype = ctypes.c_char_p
_lib.sci_words.argtypes = [_i32]
_lib.sci_words.restype = _i32
_lib.sci_n_coupled.argtypes = [_i32, _i32, _i32]
_lib.sci_n_coupled.restype = _i64
_lib.sci_ham_create.argtypes = [_i32, _i32, _i32, _P, _P, ctypes.POINTER(_P)]
_lib.sci_ham_create.restype = _i32
_lib.sci_ham_destroy.argtypes = [_P]
_lib.sci_ham_destroy.restype = _i32
_lib.sci_gen_coupled.argtypes = [_P, _P, _i64, _i64, _i64, _f64, _P, _P, _P, _i64, _P, _P, _P]
_lib.sci_gen_coupled.restype = _i32
_lib.sci_dedup_workspace_bytes.argtypes = [_i32, _i64]
_lib.sci_dedup_workspace_bytes.restype = _sz
_lib.sci_dedup_merge.argtypes = [_i32, _P, _i64, _P, _P, _P, _P, _i64, _P, _P, _i64, _P, _sz, _P, _P]
_lib.sci_dedup_merge.restype = _i32
_lib.sci_energy_workspace_bytes.argtypes = [_i64]
_lib.sci_energy_workspace_bytes.restype = _sz
_lib.sci_energy.argtypes = [_P, _P, _i64, _P, _P, _P, _P, _P, _sz, _P, _P]
_lib.sci_energy.restype = _i32
_lib.sci_energy_ex.argtypes = [_P, _P, _i64, _P, _P, _P, _P, _i32, _P, _sz, _P, _P]
_lib.sci_energy_ex.restype = _i32
_lib.sci_energy_method.argtypes = [_P, _i64]
_lib.sci_energy_method.restype = _i32
_lib.sci_energy_noalloc_max_sel.argtypes = []
_lib.sci_energy_noalloc_max_sel.restype = _i64
_lib.sci_energy_noalloc.argtypes = [_P, _P, _i64, _P, _P, _P, _P, _P, _P]
_lib.sci_energy_noalloc.restype = _i32
_lib.sci_stream_workspace_bytes.argtypes = [_P, _i64]
_lib.sci_stream_workspace_bytes.restype = _sz
_lib.sci_stream_dedup.argtypes = [_P, _P, _i64, _i64, _i64, _i64, _P, _P, _P, _P, _i64, _P,
                                  ctypes.POINTER(_i32), _P, _sz, _P, _P, _P]
_lib.sci_stream_dedup.restype = _i32
_lib.sci_index_bytes.argtypes = [_i32, _i64]
_lib.sci_index_bytes.restype = _sz
_lib.sci_index_bytes_sorted.argtypes = [_i32, _i64]
_lib.sci_index_bytes_sorted.restype = _sz
_lib.sci_index_build.argtypes = [_i32, _P, _P, _i64, _P, _sz, _P, _P]
_lib.sci_index_build.restype = _i32
_lib.sci_index_lookup.argtypes = [_i32, _P, _sz, _P, _i64, _P, _P]
_lib.sci_index_lookup.restype = _i32
_lib.sci_topk_workspace_bytes.argtypes = [_i64]
_lib.sci_topk_workspace_bytes.restype = _sz
_lib.sci_topk.argtypes = [_i32, _P, _P, _i64, _i64, _P, _P, _P, _i64, _P, _sz, _P, _P]
_lib.sci_topk.restype = _i32
class SciGenItem(ctypes.Structure):
    _fields_ = [("ham", _P), ("dets", _P), ("n_dets", _i64), ("exc_begin", _i64), ("exc_end", _i64),
                ("out_keys", _P), ("out_hij", _P)]


_lib.sci_gen_batch_create.argtypes = [ctypes.POINTER(SciGenItem), _i32, _i64, _P, ctypes.POINTER(_P)]
_lib.sci_gen_batch_create.restype = _i32
_lib.sci_gen_batch_destroy.argtypes = [_P]
_lib.sci_gen_batch_destroy.restype = _i32
_lib.sci_gen_coupled_batched.argtypes = [_P, _P]
_lib.sci_gen_coupled_batched.restype = _i32
_lib.sci_gen_batch_autotune.argtypes = [_P, _P, ctypes.POINTER(_i64)]
_lib.sci_gen_batch_autotune.restype = _i32
class SciEnergyItem(ctypes.Structure):
    _fields_ = [("ham", _P), ("sel", _P), ("n_sel", _i64), ("psi", _P), ("energy", _P), ("h_psi", _P),
                ("grad", _P)]


_lib.sci_energy_batch_create.argtypes = [ctypes.POINTER(SciEnergyItem), _i32, _P, ctypes.POINTER(_P)]
_lib.sci_energy_batch_create.restype = _i32
_lib.sci_energy_batch_destroy.argtypes = [_P]
_lib.sci_energy_batch_destroy.restype = _i32
_lib.sci_energy_batched.argtypes = [_P, _P]
_lib.sci_energy_batched.restype = _i32
_lib.sci_profile_enable.argtypes = [_i32]
_lib.sci_profile_enable.restype = _i32
_lib.sci_profile_read.argtypes = [ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_float), _i32]
_lib.sci_profile_read.restype = _i32


class SciError(RuntimeError):
    def __init__(self, status, where):
        msg = _lib.sci_last_error().decode()
        super().__init__(f"{where}: {_lib.sci_status_string(status).decode()} ({msg})")
        self.status = status


def _check(status, where):
    if status != SCI_OK:
        raise SciError(status, where)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


# Host-side shape / dtype checks before raw pointers reach the kernels: a wrong
# dtype, a strided view or a short buffer would otherwise be read past its end.

def _need(cond, msg):
    if not cond:
        raise ValueError(msg)


def _check_keys(t, W, rows, name, device=None):
    """t: contiguous int64 device tensor holding at least `rows` keys of W words."""
    if t is None:
        _need(rows == 0, f"{name}: missing")
        return
    _need(t.is_cuda, f"{name}: expected a device tensor")
    _need(t.dtype == torch.int64, f"{name}: expected int64 key words, got {t.dtype}")
    _need(t.is_contiguous(), f"{name}: expected a contiguous tensor")
    if t.dim() == 2:
        _need(t.shape[1] == W, f"{name}: keys have {t.shape[1]} words, the call needs W={W}")
    _need(t.numel() >= rows * W, f"{name}: holds {t.numel() // max(W, 1)} keys, the call needs {rows}")
    if device is not None:
        _need(t.device == device, f"{name}: on {t.device}, expected {device}")


def _check_vec(t, dtype, n, name, device=None):
    """t: contiguous device tensor of `dtype` with at least n elements (None allowed when n == 0)."""
    if t is None:
        return
    _need(t.is_cuda, f"{name}: expected a device tensor")
    _need(t.dtype == dtype, f"{name}: expected {dtype}, got {t.dtype}")
    _need(t.is_contiguous(), f"{name}: expected a contiguous tensor")
    _need(t.numel() >= n, f"{name}: has {t.numel()} elements, the call needs {n}")
    if device is not None:
        _need(t.device == device, f"{name}: on {t.device}, expected {device}")


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def sci_words(n_orb: int) -> int:
    return int(_lib.sci_words(n_orb))


def sci_n_coupled(n_orb: int, n_alpha: int, n_beta: int) -> int:
    return int(_lib.sci_n_coupled(n_orb, n_alpha, n_beta))


def sci_dedup_workspace_bytes(n_words: int, n_cand: int) -> int:
    return int(_lib.sci_dedup_workspace_bytes(n_words, n_cand))


def sci_energy_workspace_bytes(n_sel: int) -> int:
    return int(_lib.sci_energy_workspace_bytes(n_sel))


def sci_profile_enable(on: bool) -> None:
    _lib.sci_profile_enable(1 if on else 0)


def sci_profile_read(cap: int = 4096):
    """[(kernel name, ms), ...] of the launches recorded since the last read."""
    names = (ctypes.c_char_p * cap)()
    ms = (ctypes.c_float * cap)()
    n = _lib.sci_profile_read(names, ms, cap)
    if n < 0:
        raise SciError(SCI_EHIP, "sci_profile_read")
    return [(names[i].decode(), float(ms[i])) for i in range(min(n, cap))]


class Ham:
    """Device Hamiltonian handle (sci_ham_create / sci_ham_destroy)."""

    def __init__(self, n_orb, n_alpha, n_beta, h1, eri):
        h1 = np.ascontiguousarray(h1, dtype=np.float64)
        eri = np.ascontiguousarray(eri, dtype=np.float64)
        if h1.shape != (n_orb, n_orb) or eri.shape != (n_orb,) * 4:
            raise ValueError("integral shapes do not match n_orb")
        h = _P()
        _check(_lib.sci_ham_create(n_orb, n_alpha, n_beta, h1.ctypes.data_as(_P), eri.ctypes.data_as(_P),
                                   ctypes.byref(h)), "sci_ham_create")
        self._h = h
        self.n_orb, self.n_alpha, self.n_beta = n_orb, n_alpha, n_beta
        self.W = sci_words(n_orb)
        self.n_coupled = sci_n_coupled(n_orb, n_alpha, n_beta)

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h is not None and self._h.value:
            torch.cuda.synchronize()
            _lib.sci_ham_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sci_ham_create(n_orb, n_alpha, n_beta, h1, eri) -> Ham:
    return Ham(n_orb, n_alpha, n_beta, h1, eri)


def sci_ham_destroy(ham: Ham) -> None:
    ham.close()


def sci_gen_coupled(ham: Ham, dets, n_dets, exc_begin, exc_end, eps, out_keys, out_hij, out_src,
                    capacity, n_out, dev_flags, stream=None):
    dev = dets.device if dets is not None else None
    _check_keys(dets, ham.W, n_dets, "dets")
    count = max(0, exc_end - exc_begin)
    # dense mode writes exactly `count` slots; screened mode up to min(capacity, count)
    slots = count if eps < 0 else min(capacity, count)
    _check_keys(out_keys, ham.W, slots, "out_keys", dev)
    _check_vec(out_hij, torch.float64, slots, "out_hij", dev)
    _check_vec(out_src, torch.int32, slots, "out_src", dev)
    _check_vec(n_out, torch.int64, 1, "n_out", dev)
    _check_vec(dev_flags, torch.int32, 1, "dev_flags", dev)
    _check(_lib.sci_gen_coupled(ham.handle, _ptr(dets), n_dets, exc_begin, exc_end, float(eps),
                                _ptr(out_keys), _ptr(out_hij), _ptr(out_src), capacity, _ptr(n_out),
                                _ptr(dev_flags), _stream(stream)), "sci_gen_coupled")


def sci_dedup_merge(n_words, cand, n_cand, set_in, n_set_in, set_out, n_set_out, set_capacity,
                    novel, n_novel, novel_capacity, workspace, workspace_bytes, dev_flags, stream=None):
    dev = set_out.device if set_out is not None else None
    _check_keys(cand, n_words, n_cand, "cand", dev)
    if set_in is not None:
        _check_keys(set_in, n_words, 0, "set_in", dev)
        _check_vec(n_set_in, torch.int64, 1, "n_set_in", dev)
    _check_keys(set_out, n_words, set_capacity, "set_out", dev)
    _check_vec(n_set_out, torch.int64, 1, "n_set_out", dev)
    if novel is not None:
        _check_keys(novel, n_words, novel_capacity, "novel", dev)
        _check_vec(n_novel, torch.int64, 1, "n_novel", dev)
    _check_vec(workspace, torch.uint8, workspace_bytes, "workspace", dev)
    _check_vec(dev_flags, torch.int32, 1, "dev_flags", dev)
    _check(_lib.sci_dedup_merge(n_words, _ptr(cand), n_cand, _ptr(set_in), _ptr(n_set_in), _ptr(set_out),
                                _ptr(n_set_out), set_capacity, _ptr(novel), _ptr(n_novel), novel_capacity,
                                _ptr(workspace), workspace_bytes, _ptr(dev_flags), _stream(stream)),
           "sci_dedup_merge")


def sci_energy_method(ham: Ham, n_sel: int) -> int:
    """The membership method sci_energy picks for n_sel determinants (ENERGY_PAIRS / ENERGY_ENUM)."""
    return int(_lib.sci_energy_method(ham.handle, n_sel))


def sci_energy(ham: Ham, sel, n_sel, psi, energy, h_psi, grad, workspace, workspace_bytes, dev_flags,
               stream=None, method=ENERGY_AUTO):
    dev = sel.device
    _check_keys(sel, ham.W, n_sel, "sel")
    _check_vec(psi, torch.float64, n_sel, "psi", dev)
    _check_vec(energy, torch.float64, 1, "energy", dev)
    _check_vec(h_psi, torch.float64, n_sel, "h_psi", dev)
    _check_vec(grad, torch.float64, n_sel, "grad", dev)
    _check_vec(workspace, torch.uint8, workspace_bytes, "workspace", dev)
    _check_vec(dev_flags, torch.int32, 1, "dev_flags", dev)
    _check(_lib.sci_energy_ex(ham.handle, _ptr(sel), n_sel, _ptr(psi), _ptr(energy), _ptr(h_psi), _ptr(grad),
                              int(method), _ptr(workspace), workspace_bytes, _ptr(dev_flags), _stream(stream)),
           "sci_energy")


def sci_energy_noalloc_max_sel() -> int:
    return int(_lib.sci_energy_noalloc_max_sel())


def sci_energy_noalloc(ham: Ham, sel, n_sel, psi, energy, h_psi, grad, dev_flags, stream=None):
    """sci_energy without a workspace: the library's own per-device scratch (n_sel limited)."""
    dev = sel.device
    _check_keys(sel, ham.W, n_sel, "sel")
    _check_vec(psi, torch.float64, n_sel, "psi", dev)
    _check_vec(energy, torch.float64, 1, "energy", dev)
    _check_vec(h_psi, torch.float64, n_sel, "h_psi", dev)
    _check_vec(grad, torch.float64, n_sel, "grad", dev)
    _check_vec(dev_flags, torch.int32, 1, "dev_flags", dev)
    _check(_lib.sci_energy_noalloc(ham.handle, _ptr(sel), n_sel, _ptr(psi), _ptr(energy), _ptr(h_psi), _ptr(grad),
                                   _ptr(dev_flags), _stream(stream)), "sci_energy_noalloc")


def sci_stream_workspace_bytes(ham: Ham, chunk: int) -> int:
    return int(_lib.sci_stream_workspace_bytes(ham.handle, chunk))


def sci_stream_dedup(ham: Ham, dets, n_dets, exc_begin, exc_end, chunk, set_in, n_set_in, set_a, set_b,
                     set_capacity, n_set_out, workspace, workspace_bytes, dev_flags, gen_stream=None,
                     dedup_stream=None) -> bool:
    """Returns True when the final set is set_b."""
    dev = set_a.device
    _check_keys(dets, ham.W, n_dets, "dets", dev)
    if set_in is not None:
        _check_keys(set_in, ham.W, 0, "set_in", dev)
        _check_vec(n_set_in, torch.int64, 1, "n_set_in", dev)
    _check_keys(set_a, ham.W, set_capacity, "set_a", dev)
    _check_keys(set_b, ham.W, set_capacity, "set_b", dev)
    _check_vec(n_set_out, torch.int64, 1, "n_set_out", dev)
    _check_vec(workspace, torch.uint8, workspace_bytes, "workspace", dev)
    _check_vec(dev_flags, torch.int32, 1, "dev_flags", dev)
    fb = _i32(0)
    _check(_lib.sci_stream_dedup(ham.handle, _ptr(dets), n_dets, exc_begin, exc_end, chunk, _ptr(set_in),
                                 _ptr(n_set_in), _ptr(set_a), _ptr(set_b), set_capacity, _ptr(n_set_out),
                                 ctypes.byref(fb), _ptr(workspace), workspace_bytes, _ptr(dev_flags),
                                 _stream(gen_stream), _stream(dedup_stream)), "sci_stream_dedup")
    return bool(fb.value)


# ---------------------------------------------------------------------------
# allocating conveniences
# ---------------------------------------------------------------------------

def keys_to_device(keys: np.ndarray, device="cuda") -> torch.Tensor:
    """(n, W) uint64 numpy -> (n, W) int64 device tensor holding the same bits."""
    a = np.ascontiguousarray(keys, dtype=np.uint64)
    return torch.from_numpy(a.view(np.int64)).to(device)


def keys_to_host(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint64)


def new_flags(device="cuda") -> torch.Tensor:
    return torch.zeros(1, dtype=torch.int32, device=device)


def check_flags(flags: torch.Tensor, where: str, allow=0):
    v = int(flags.item()) & 0xFFFFFFFF
    if v & ~allow:
        names = [n for b, n in ((FLAG_OVERFLOW, "OVERFLOW"), (FLAG_BAD_DET, "BAD_DET"),
                                (FLAG_UNSORTED, "UNSORTED")) if v & b]
        raise RuntimeError(f"{where}: device flags {names}")
    return v


def gen_coupled(ham: Ham, dets: torch.Tensor, exc_begin=0, exc_end=None, eps=-1.0, with_src=False,
                capacity=None, flags=None):
    """Dense (eps<0) or screened coupled generation; returns (keys, hij, src, n_out tensor)."""
    _need(dets.dim() == 2, "dets: expected an (n, W) tensor")
    n = dets.shape[0]
    if exc_end is None:
        exc_end = n * ham.n_coupled
    count = exc_end - exc_begin
    if capacity is None:
        capacity = count
    dev = dets.device
    keys = torch.empty((capacity, ham.W), dtype=torch.int64, device=dev)
    hij = torch.empty(capacity, dtype=torch.float64, device=dev)
    src = torch.empty(capacity, dtype=torch.int32, device=dev) if (with_src or eps >= 0) else None
    n_out = torch.zeros(1, dtype=torch.int64, device=dev)
    own_flags = flags is None
    if own_flags:
        flags = new_flags(dev)
    sci_gen_coupled(ham, dets, n, exc_begin, exc_end, eps, keys, hij, src, capacity, n_out, flags)
    return keys, hij, src, n_out, flags


def dedup_merge(cand: torch.Tensor, set_in: torch.Tensor, n_words: int, want_novel=False, set_capacity=None,
                flags=None, workspace=None):
    """sorted(set(cand) | set(set_in)) and optionally sorted(set(cand) - set(set_in)), on the device."""
    _need(cand.dim() == 2 and set_in.dim() == 2, "cand, set_in: expected (n, W) tensors")
    dev = cand.device
    n_cand = cand.shape[0]
    n_set = set_in.shape[0]
    if set_capacity is None:
        set_capacity = n_cand + n_set
    n_set_in = torch.tensor([n_set], dtype=torch.int64, device=dev)
    set_out = torch.empty((max(set_capacity, 1), n_words), dtype=torch.int64, device=dev)
    n_set_out = torch.zeros(1, dtype=torch.int64, device=dev)
    novel = torch.empty((max(n_cand, 1), n_words), dtype=torch.int64, device=dev) if want_novel else None
    n_novel = torch.zeros(1, dtype=torch.int64, device=dev) if want_novel else None
    ws_bytes = sci_dedup_workspace_bytes(n_words, n_cand)
    if workspace is None:
        workspace = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=dev)
    if flags is None:
        flags = new_flags(dev)
    sci_dedup_merge(n_words, cand, n_cand, set_in, n_set_in, set_out, n_set_out, set_capacity,
                    novel, n_novel, n_cand if want_novel else 0, workspace, workspace.numel(), flags)
    return set_out, n_set_out, novel, n_novel, flags


def energy(ham: Ham, sel: torch.Tensor, psi: torch.Tensor, want_hpsi=True, want_grad=True, flags=None,
           workspace=None, method=ENERGY_AUTO):
    _need(sel.dim() == 2 and psi.dim() == 1 and psi.shape[0] == sel.shape[0],
          "energy: expected sel (n, W) and psi (n,)")
    dev = sel.device
    n = sel.shape[0]
    e = torch.zeros(1, dtype=torch.float64, device=dev)
    hp = torch.empty(n, dtype=torch.float64, device=dev) if want_hpsi else None
    g = torch.empty(n, dtype=torch.float64, device=dev) if want_grad else None
    ws_bytes = sci_energy_workspace_bytes(n)
    if workspace is None:
        workspace = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=dev)
    if flags is None:
        flags = new_flags(dev)
    sci_energy(ham, sel, n, psi, e, hp, g, workspace, workspace.numel(), flags, method=method)
    return e, hp, g, flags


def stream_dedup(ham: Ham, dets: torch.Tensor, chunk: int, set_in: torch.Tensor, set_capacity: int,
                 exc_begin=0, exc_end=None, gen_stream=None, dedup_stream=None, flags=None):
    """Streamed generation + dedup-merge of all coupled determinants of `dets` into `set_in`.

    The work runs on gen_stream / dedup_stream (default: the current stream); on return
    the current stream waits for both, and every tensor the enqueued work touches is
    recorded on the streams that use it, so the caching allocator reuses none of them
    before that work is done.  The results may be read on the current stream."""
    dev = dets.device
    n = dets.shape[0]
    if exc_end is None:
        exc_end = n * ham.n_coupled
    W = ham.W
    set_a = torch.empty((max(set_capacity, 1), W), dtype=torch.int64, device=dev)
    set_b = torch.empty_like(set_a)
    n_in = torch.tensor([set_in.shape[0]], dtype=torch.int64, device=dev)
    n_out = torch.zeros(1, dtype=torch.int64, device=dev)
    ws = torch.empty(max(sci_stream_workspace_bytes(ham, chunk), 1), dtype=torch.uint8, device=dev)
    if flags is None:
        flags = new_flags(dev)
    cur = torch.cuda.current_stream(dev)
    gs = gen_stream if gen_stream is not None else cur
    ds = dedup_stream if dedup_stream is not None else cur
    # inputs written on the current stream (n_in, the flags) are ready before either stream starts
    for s_ in (gs, ds):
        if s_ != cur:
            s_.wait_stream(cur)
    is_b = sci_stream_dedup(ham, dets, n, exc_begin, exc_end, chunk, set_in, n_in, set_a, set_b, set_capacity, n_out,
                            ws, ws.numel(), flags, gs, ds)
    for s_ in (gs, ds):
        if s_ != cur:
            cur.wait_stream(s_)
            for t in (dets, set_in, n_in, set_a, set_b, n_out, ws, flags):
                if t is not None:
                    t.record_stream(s_)
    return (set_b if is_b else set_a), n_out, flags


def sci_index_bytes(n_words: int, set_bound: int) -> int:
    return int(_lib.sci_index_bytes(n_words, set_bound))


def sci_index_build(n_words, set_keys, n_set, set_bound, index, index_bytes, dev_flags, stream=None):
    _check(_lib.sci_index_build(n_words, _ptr(set_keys), _ptr(n_set), set_bound, _ptr(index), index_bytes,
                                _ptr(dev_flags), _stream(stream)), "sci_index_build")


def sci_index_lookup(n_words, index, index_bytes, cand, n_cand, idx, stream=None):
    _check(_lib.sci_index_lookup(n_words, _ptr(index), index_bytes, _ptr(cand), n_cand, _ptr(idx), _stream(stream)),
           "sci_index_lookup")


def sci_topk_workspace_bytes(n: int) -> int:
    return int(_lib.sci_topk_workspace_bytes(n))


def sci_topk(n_words, keys, psi, n, k, out_keys, out_psi, n_out, capacity, workspace, workspace_bytes, dev_flags,
             stream=None):
    _check(_lib.sci_topk(n_words, _ptr(keys), _ptr(psi), n, k, _ptr(out_keys), _ptr(out_psi), _ptr(n_out), capacity,
                         _ptr(workspace), workspace_bytes, _ptr(dev_flags), _stream(stream)), "sci_topk")


def sci_index_bytes_sorted(n_words: int, set_bound: int) -> int:
    return int(_lib.sci_index_bytes_sorted(n_words, set_bound))


def build_index(set_keys: torch.Tensor, n_set: torch.Tensor, set_bound: int, W: int, flags=None, kind="auto",
                reserve_bytes=8 << 30):
    """Reverse index over the strictly ascending set (count n_set on the device).

    kind "hash": an open-addressing table (32-64 bytes per key); "sorted": samples of
    the sorted set (1/256 of its bytes) searched together with the set itself, which
    must then stay unchanged while the index is used; "auto": the table when it fits in
    free device memory with `reserve_bytes` to spare, else the sorted kind."""
    dev = set_keys.device
    if kind == "auto":
        free_bytes = torch.cuda.mem_get_info(dev)[0]
        kind = "hash" if sci_index_bytes(W, set_bound) + reserve_bytes <= free_bytes else "sorted"
    if kind not in ("hash", "sorted"):
        raise ValueError(f"unknown index kind {kind!r}")
    nbytes = sci_index_bytes(W, set_bound) if kind == "hash" else sci_index_bytes_sorted(W, set_bound)
    if kind == "sorted":
        # the library picks the kind from the buffer size: stay below a table's size
        nbytes = min(nbytes, sci_index_bytes(W, set_bound) - 1)
    index = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    if flags is None:
        flags = new_flags(dev)
    sci_index_build(W, set_keys, n_set, set_bound, index, nbytes, flags)
    return index, flags


def index_kind(index: torch.Tensor) -> str:
    """"hash" or "sorted": the kind of a built index (reads its device header)."""
    tag = int(index[16:24].view(torch.int64).item())
    return "sorted" if tag == 0x534F525445444958 else "hash"


def inverse_map(index: torch.Tensor, cand: torch.Tensor, W: int):
    """Position of each candidate in the indexed set, -1 when absent."""
    n = cand.shape[0]
    idx = torch.empty(max(n, 1), dtype=torch.int64, device=cand.device)
    sci_index_lookup(W, index, index.numel(), cand, n, idx)
    return idx[:n]


def topk(keys: torch.Tensor, psi: torch.Tensor, k: int, W: int, flags=None):
    """The min(k, n) entries of largest |psi| (ties: smaller key), in input order."""
    dev = keys.device
    n = keys.shape[0]
    kk = min(k, n)
    out_keys = torch.empty((max(kk, 1), W), dtype=torch.int64, device=dev)
    out_psi = torch.empty(max(kk, 1), dtype=torch.float64, device=dev)
    n_out = torch.zeros(1, dtype=torch.int64, device=dev)
    ws = torch.empty(max(sci_topk_workspace_bytes(n), 1), dtype=torch.uint8, device=dev)
    if flags is None:
        flags = new_flags(dev)
    sci_topk(W, keys, psi, n, k, out_keys, out_psi, n_out, kk, ws, ws.numel(), flags)
    return out_keys, out_psi, n_out, flags


class GenBatch:
    """A batch of dense-mode generation calls over several systems, run as one
    persistent launch per key width (sci_gen_batch_create / sci_gen_coupled_batched).

    items: (ham, dets, exc_begin, exc_end, out_keys, out_hij) tuples; the tensors
    are kept alive by the batch."""

    def __init__(self, items, tile_candidates=1 << 18, flags=None):
        arr = (SciGenItem * max(len(items), 1))()
        keep = []
        dev = None
        for i, (ham, dets, e0, e1, keys, hij) in enumerate(items):
            arr[i] = SciGenItem(ham.handle.value, dets.data_ptr(), dets.shape[0], e0, e1, keys.data_ptr(),
                                hij.data_ptr())
            keep += [ham, dets, keys, hij]
            dev = dets.device
        self.flags = flags if flags is not None else new_flags(dev if dev is not None else "cuda")
        h = _P()
        _check(_lib.sci_gen_batch_create(arr, len(items), int(tile_candidates), _ptr(self.flags), ctypes.byref(h)),
               "sci_gen_batch_create")
        self._h = h
        self._keep = keep

    def launch(self, stream=None):
        _check(_lib.sci_gen_coupled_batched(self._h, _stream(stream)), "sci_gen_coupled_batched")

    def autotune(self, stream=None) -> int:
        tc = _i64(0)
        _check(_lib.sci_gen_batch_autotune(self._h, _stream(stream), ctypes.byref(tc)), "sci_gen_batch_autotune")
        return int(tc.value)

    def close(self):
        if self._h is not None and self._h.value:
            torch.cuda.synchronize()
            _lib.sci_gen_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class EnergyBatch:
    """Energies (and optionally H psi and gradients) of several systems in a few
    launches (sci_energy_batch_create / sci_energy_batched).

    items: (ham, sel, psi) tuples.  Outputs are allocated here: `energy` [n_items],
    `h_psi` and `grad` lists of per-system tensors."""

    def __init__(self, items, want_grad=True, flags=None):
        arr = (SciEnergyItem * len(items))()
        dev = items[0][1].device
        self.energy = torch.zeros(len(items), dtype=torch.float64, device=dev)
        self.h_psi, self.grad, keep = [], [], []
        for i, (ham, sel, psi) in enumerate(items):
            hp = torch.empty(sel.shape[0], dtype=torch.float64, device=dev)
            g = torch.empty(sel.shape[0], dtype=torch.float64, device=dev) if want_grad else None
            self.h_psi.append(hp)
            self.grad.append(g)
            arr[i] = SciEnergyItem(ham.handle.value, sel.data_ptr(), sel.shape[0], psi.data_ptr(),
                                   self.energy[i:].data_ptr(), hp.data_ptr(), g.data_ptr() if g is not None else None)
            keep += [ham, sel, psi]
        self.flags = flags if flags is not None else new_flags(dev)
        h = _P()
        _check(_lib.sci_energy_batch_create(arr, len(items), _ptr(self.flags), ctypes.byref(h)),
               "sci_energy_batch_create")
        self._h = h
        self._keep = keep

    def launch(self, stream=None):
        _check(_lib.sci_energy_batched(self._h, _stream(stream)), "sci_energy_batched")

    def close(self):
        if self._h is not None and self._h.value:
            torch.cuda.synchronize()
            _lib.sci_energy_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SciEnergy(torch.autograd.Function):
    """E(psi) = psi.H psi / psi.psi with the hand-written adjoint dE/dpsi = 2(H psi - E psi)/psi.psi.

    Forward stores nothing but psi; backward recomputes H psi (H_ij never stored).
    """

    @staticmethod
    def forward(ctx, psi, ham, sel):
        e, _, _, flags = energy(ham, sel, psi.detach(), want_hpsi=False, want_grad=False)
        # a selected set that is unsorted or holds malformed determinants has no energy:
        # raise instead of returning a number (this reads the flags, one host sync)
        check_flags(flags, "SciEnergy.forward")
        ctx.ham = ham
        ctx.save_for_backward(psi, sel)
        return e[0]

    @staticmethod
    def backward(ctx, grad_out):
        psi, sel = ctx.saved_tensors
        _, _, g, _ = energy(ctx.ham, sel, psi.detach(), want_hpsi=False, want_grad=True)
        return grad_out * g, None, None
