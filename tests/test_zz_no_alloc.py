"""sci_energy_noalloc (the entry point that allocates nothing) against sci_energy.

Two calls in a row through the C ABI, the second on a smaller input: the
per-device scratch keeps the first call's contents, and the results must still
equal sci_energy's bit for bit (same kernels, same fixed reduction order).
"""
import numpy as np
import pytest
import torch

import sci_inputs as si
from tests.gpu_common import require_gpu, say, system

pytestmark = pytest.mark.gpu


def _plain_and_noalloc(sci, ham, sel, psi):
    n = sel.shape[0]
    dev = sel.device
    outs = []
    for kind in ("plain", "noalloc"):
        e = torch.full((1,), np.nan, dtype=torch.float64, device=dev)
        hp = torch.full((n,), np.nan, dtype=torch.float64, device=dev)
        g = torch.full((n,), np.nan, dtype=torch.float64, device=dev)
        flags = sci.new_flags(dev)
        if kind == "plain":
            ws = torch.empty(sci.sci_energy_workspace_bytes(n), dtype=torch.uint8, device=dev)
            sci.sci_energy(ham, sel, n, psi, e, hp, g, ws, ws.numel(), flags)
        else:
            sci.sci_energy_noalloc(ham, sel, n, psi, e, hp, g, flags)
        torch.cuda.synchronize()
        assert sci.check_flags(flags, kind) == 0
        outs.append((e.cpu().numpy(), hp.cpu().numpy(), g.cpu().numpy()))
    return outs


def test_noalloc_energy_matches_plain_twice():
    sci = require_gpu()
    assert sci.sci_energy_noalloc_max_sel() == 1 << 18
    # first call: 150,000 determinants of the large workload (two-word keys, pair screening)
    s = system("large")
    big = sci.Ham(s.n_orb, s.n_alpha, s.n_beta, s.h1, s.eri)
    n1 = 150_000
    sel1 = sci.keys_to_device(s.dets[:n1])
    psi1 = torch.from_numpy(s.psi[:n1].copy()).cuda()
    # second call, smaller: 17,000 determinants of a 10-orbital system (one-word keys,
    # enumeration + search)
    wl = si.small_workload(10, 4, 4, n_sel=17_000, selection="levels")
    sm = si.make_system(wl)
    small = sci.Ham(sm.n_orb, sm.n_alpha, sm.n_beta, sm.h1, sm.eri)
    sel2 = sci.keys_to_device(sm.dets)
    psi2 = torch.from_numpy(sm.psi).cuda()
    assert sci.sci_energy_method(big, n1) == sci.ENERGY_PAIRS
    assert sci.sci_energy_method(small, sel2.shape[0]) == sci.ENERGY_ENUM
    for name, ham, sel, psi in (("large[:150000]", big, sel1, psi1), ("10-orbital 17,000", small, sel2, psi2)):
        say(f"noalloc vs plain: {name}")
        (e0, h0, g0), (e1, h1, g1) = _plain_and_noalloc(sci, ham, sel, psi)
        assert np.isfinite(e0).all() and np.isfinite(h0).all() and np.isfinite(g0).all()
        assert np.array_equal(e0, e1), f"{name}: energy {e0[0]!r} vs {e1[0]!r}"
        assert np.array_equal(h0, h1), f"{name}: H psi differs (max {np.max(np.abs(h0 - h1)):.3e})"
        assert np.array_equal(g0, g1), f"{name}: gradient differs (max {np.max(np.abs(g0 - g1)):.3e})"
    big.close()
    small.close()


def test_noalloc_energy_rejects_above_limit():
    sci = require_gpu()
    s = system("tiny")
    ham = sci.Ham(s.n_orb, s.n_alpha, s.n_beta, s.h1, s.eri)
    n = sci.sci_energy_noalloc_max_sel() + 1
    dev = torch.device("cuda")
    sel = torch.zeros((n, ham.W), dtype=torch.int64, device=dev)
    psi = torch.zeros(n, dtype=torch.float64, device=dev)
    e = torch.zeros(1, dtype=torch.float64, device=dev)
    flags = sci.new_flags(dev)
    with pytest.raises(sci.SciError) as err:
        sci.sci_energy_noalloc(ham, sel, n, psi, e, None, None, flags)
    assert err.value.status == sci.SCI_ECAPACITY
    torch.cuda.synchronize()
    assert int(flags.item()) == 0 and float(e.item()) == 0.0  # nothing was enqueued
    ham.close()
