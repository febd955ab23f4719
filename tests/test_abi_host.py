"""Host-side checks of the C ABI: the library loads, exports what include/sci.h
declares, sizes follow the closed forms, and argument errors are reported
before anything touches a device.  No compute call is made here."""
import ctypes
import os
import re

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sci.h")


def _lib():
    sci = pytest.importorskip("paper_2604_15768_amd")
    return sci, sci._lib


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sci_[a-z0-9_]+)\s*\(", text)))


def test_header_symbols_exported():
    _, lib = _lib()
    names = _declared()
    assert "sci_gen_coupled" in names and "sci_dedup_merge" in names and "sci_energy" in names
    for name in names:
        assert hasattr(lib, name), f"{name} declared in sci.h but not exported"


def test_sizes_match_closed_forms():
    sci, _ = _lib()
    for n, na, nb in [(7, 5, 5), (26, 7, 7), (60, 10, 10), (5, 0, 3), (64, 32, 32), (1, 1, 0)]:
        assert sci.sci_n_coupled(n, na, nb) == oracle.n_coupled(n, na, nb)
        assert sci.sci_words(n) == (2 * n + 63) // 64
    assert sci.sci_n_coupled(4, 5, 1) == -1
    assert sci.sci_n_coupled(26, 7, 7) * 100_000 == 2_513_700_000


def test_status_strings():
    sci, lib = _lib()
    for code, name in enumerate(["SCI_OK", "SCI_EINVAL", "SCI_ECAPACITY", "SCI_ENOMEM", "SCI_EHIP",
                                 "SCI_EUNSUPPORTED"]):
        assert lib.sci_status_string(code).decode() == name


def test_workspace_sizes_monotone():
    sci, _ = _lib()
    for W in (1, 2):
        prev = 0
        for n in (0, 1, 4096, 10**6, 10**8):
            b = sci.sci_dedup_workspace_bytes(W, n)
            assert b >= prev and b >= 2 * n * 8 * W
            prev = b
    assert sci.sci_dedup_workspace_bytes(3, 10) == 0
    assert sci.sci_energy_workspace_bytes(1000) >= 8000


def test_argument_errors_before_device():
    sci, lib = _lib()
    P = ctypes.c_void_p
    fake = P(0x1000)  # never dereferenced: every call below fails validation first
    # NULL handle
    assert lib.sci_gen_coupled(None, fake, 1, 0, 1, -1.0, fake, fake, None, 1, None, fake, None) == sci.SCI_EINVAL
    assert lib.sci_energy(None, fake, 1, fake, fake, None, None, fake, 100, fake, None) == sci.SCI_EINVAL
    assert "NULL handle" in lib.sci_last_error().decode()
    # dedup: bad word counts, negative sizes, workspace too small, aliasing
    args = dict(cand=fake, n_cand=10, set_in=None, n_set_in=None, set_out=P(0x2000), n_set_out=fake,
                cap=10, novel=None, n_novel=None, ncap=0, ws=fake, wsb=1, flags=fake)

    def dd(**kw):
        a = dict(args)
        a.update(kw)
        W = kw.pop("W", 1)
        return lib.sci_dedup_merge(a.get("W", W), a["cand"], a["n_cand"], a["set_in"], a["n_set_in"], a["set_out"],
                                   a["n_set_out"], a["cap"], a["novel"], a["n_novel"], a["ncap"], a["ws"], a["wsb"],
                                   a["flags"], None)

    assert dd(W=0) == sci.SCI_EINVAL
    assert dd(W=3) == sci.SCI_EUNSUPPORTED
    assert dd(n_cand=-1) == sci.SCI_EINVAL
    assert dd() == sci.SCI_ECAPACITY
    assert dd(set_out=fake) == sci.SCI_EINVAL  # aliases cand
    assert dd(set_in=fake) == sci.SCI_EINVAL  # set_in without its count
    # ham_create: bad sizes are rejected before any allocation
    h = P()
    d = (ctypes.c_double * 4)()
    assert lib.sci_ham_create(2, 3, 1, d, d, ctypes.byref(h)) == sci.SCI_EINVAL
    assert lib.sci_ham_create(65, 3, 1, d, d, ctypes.byref(h)) == sci.SCI_EUNSUPPORTED
    assert lib.sci_ham_create(2, 1, 1, None, d, ctypes.byref(h)) == sci.SCI_EINVAL
    assert lib.sci_ham_destroy(None) == sci.SCI_OK


def _overcommit_mode():
    try:
        return int(open("/proc/sys/vm/overcommit_memory").read().strip())
    except (OSError, ValueError):
        return None


def test_host_allocation_failure_maps_to_enomem():
    """A host allocation inside the library that cannot be satisfied comes back as
    SCI_ENOMEM with a message, never as a C++ exception through the C ABI (which
    would abort the Python process here).  A batch of 2^31 - 1 items asks for about
    480 GB of host item records before any item is read; with heuristic overcommit
    that allocation is refused."""
    sci, lib = _lib()
    if _overcommit_mode() == 1:
        pytest.skip("the kernel grants every allocation (vm.overcommit_memory = 1)")
    item = sci.SciGenItem()  # ham NULL: only read if the allocation were granted
    h = ctypes.c_void_p()
    rc = lib.sci_gen_batch_create(ctypes.byref(item), 2**31 - 1, 1 << 18, ctypes.c_void_p(0x1000), ctypes.byref(h))
    assert rc == sci.SCI_ENOMEM, lib.sci_last_error().decode()
    assert "sci_gen_batch_create" in lib.sci_last_error().decode()
    assert not h.value
    # the library keeps working afterwards
    assert lib.sci_gen_batch_create(ctypes.byref(item), 1, 1 << 18, ctypes.c_void_p(0x1000),
                                    ctypes.byref(h)) == sci.SCI_EINVAL
    assert "no handle" in lib.sci_last_error().decode()


def test_product_path_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_2604_15768_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text
                assert "sci_oracle" not in text and "ora_" not in text
