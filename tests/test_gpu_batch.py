"""GPU parity of batched generation (several systems of both key widths, one
persistent launch per width) against the oracle and the plain per-system call,
after autotuning, and replayed from a captured graph."""
import numpy as np
import pytest
import torch  # imported at collection: the first import on a fresh box is slow

import oracle
import sci_inputs as si
from tests.gpu_common import H_TOL, pick_sources, require_gpu, say, system

pytestmark = pytest.mark.gpu


def _batch_systems():
    """tiny (W=1), the smallest W=1 and W=2 systems of the batched workload, and
    a W=2 test system; a few sources of each."""
    wls = si.batch_workloads()
    w1 = min((w for w in wls if w.W == 1), key=lambda w: w.n_orb)
    w2 = min((w for w in wls if w.W == 2), key=lambda w: w.n_orb)
    out = [system("tiny"), si.make_system(w1), si.make_system(w2),
           si.make_system(si.small_workload(34, 3, 2, n_sel=40, seed=si.SEED_BASE + 91))]
    return out


def _items(sci, systems, n_src=5):
    """(Ham, dets, range, outputs) per system: full ranges, a partial range and an empty one."""
    rows = []
    for k, s in enumerate(systems):
        h = sci.Ham(s.n_orb, s.n_alpha, s.n_beta, s.h1, s.eri)
        idx = pick_sources(s.dets.shape[0], n_src, 40 + k)
        dets = s.dets[idx]
        total = dets.shape[0] * h.n_coupled
        if k == 1:
            e0, e1 = h.n_coupled // 3, total - h.n_coupled // 5  # partial first and last sources
        else:
            e0, e1 = 0, total
        n = e1 - e0
        keys = torch.full((max(n, 1), s.W), -1, dtype=torch.int64, device="cuda")
        hij = torch.full((max(n, 1),), np.nan, dtype=torch.float64, device="cuda")
        rows.append((s, h, dets, sci.keys_to_device(dets), e0, e1, keys, hij))
    s0 = systems[0]
    h0 = rows[0][1]
    rows.append((s0, h0, s0.dets[:3], sci.keys_to_device(s0.dets[:3]), 7, 7,
                 torch.zeros((1, s0.W), dtype=torch.int64, device="cuda"),
                 torch.zeros(1, dtype=torch.float64, device="cuda")))
    return rows


def _expected(rows):
    out = []
    for s, h, dets, _, e0, e1, _, _ in rows:
        ok, oh, _ = oracle.gen_coupled(s.n_orb, s.n_alpha, s.n_beta, s.h1, s.eri, dets)
        out.append((ok[e0:e1], oh[e0:e1]))
    return out


def _check(sci, rows, want, where):
    for (s, h, dets, _, e0, e1, keys, hij), (ok, oh) in zip(rows, want):
        n = e1 - e0
        if n == 0:
            continue
        got_k = sci.keys_to_host(keys[:n])
        assert np.array_equal(got_k, ok), f"{where}: keys differ (n_orb={s.n_orb})"
        assert np.max(np.abs(hij[:n].cpu().numpy() - oh)) <= H_TOL, f"{where}: H_ij differ (n_orb={s.n_orb})"


def test_batched_generation_matches_oracle_and_plain():
    sci = require_gpu()
    systems = _batch_systems()
    rows = _items(sci, systems)
    say("batched generation: " + ", ".join(f"n={r[0].n_orb} W={r[0].W} [{r[4]},{r[5]})" for r in rows))
    batch = sci.GenBatch([(h, dd, e0, e1, k, x) for _, h, _, dd, e0, e1, k, x in rows], tile_candidates=20_000)
    batch.launch()
    torch.cuda.synchronize()
    assert sci.check_flags(batch.flags, "batched gen") == 0
    want = _expected(rows)
    _check(sci, rows, want, "batched")
    # the plain call on each item gives the same bits
    for s, h, _, dd, e0, e1, keys, hij in rows:
        if e1 == e0:
            continue
        k2, x2, _, _, f = sci.gen_coupled(h, dd, exc_begin=e0, exc_end=e1)
        torch.cuda.synchronize()
        assert torch.equal(k2[: e1 - e0], keys[: e1 - e0]) and torch.equal(x2[: e1 - e0], hij[: e1 - e0])
    batch.close()


def test_batched_generation_autotune_and_graph_replays():
    sci = require_gpu()
    systems = _batch_systems()
    rows = _items(sci, systems, n_src=3)
    batch = sci.GenBatch([(h, dd, e0, e1, k, x) for _, h, _, dd, e0, e1, k, x in rows])
    chosen = batch.autotune()
    torch.cuda.synchronize()
    assert chosen in (1 << 14, 1 << 16, 1 << 18, 1 << 20, 1 << 22)
    want = _expected(rows)
    _check(sci, rows, want, f"autotuned ({chosen})")
    # capture one batched launch, then replay it with eager work in between
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            batch.launch()
    torch.cuda.synchronize()
    for rep in range(3):
        for r in rows:
            r[6].fill_(-1)
            r[7].fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _check(sci, rows, want, f"graph replay {rep}")
    assert sci.check_flags(batch.flags, "batched gen") == 0
    batch.close()


def test_batch_rejects_bad_items():
    sci = require_gpu()
    s = system("tiny")
    h = sci.Ham(s.n_orb, s.n_alpha, s.n_beta, s.h1, s.eri)
    d = sci.keys_to_device(s.dets[:2])
    k = torch.zeros((1, 1), dtype=torch.int64, device="cuda")
    x = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(sci.SciError):
        sci.GenBatch([(h, d, 0, 2 * h.n_coupled + 1, k, x)])  # range past the last source
    with pytest.raises(sci.SciError):
        sci.GenBatch([(h, d, 5, 3, k, x)])


def test_batched_energy_matches_plain_and_oracle():
    """Every system's E, H psi and gradient from the batch equal its own sci_energy
    call bit for bit, and the oracle within the energy tolerances."""
    from tests.gpu_common import E_TOL, G_TOL
    sci = require_gpu()
    wls = si.batch_workloads()
    picks = sorted(wls, key=lambda w: w.n_sel)[:5] + [w for w in wls if w.W == 2][:2]
    systems = [si.make_system(w) for w in picks] + [system("tiny")]
    rows = []
    for s in systems:
        h = sci.Ham(s.n_orb, s.n_alpha, s.n_beta, s.h1, s.eri)
        rows.append((s, h, sci.keys_to_device(s.dets), torch.from_numpy(s.psi).cuda()))
    say("batched energy: " + ", ".join(f"n={s.n_orb} W={s.W} |S|={s.dets.shape[0]}" for s, *_ in rows))
    batch = sci.EnergyBatch([(h, d, p) for _, h, d, p in rows])
    batch.launch()
    torch.cuda.synchronize()
    assert sci.check_flags(batch.flags, "batched energy") == 0
    for k, (s, h, d, p) in enumerate(rows):
        e, hp, g, f = sci.energy(h, d, p)
        torch.cuda.synchronize()
        assert batch.energy[k].item() == e.item(), f"system {k}: energy differs from the plain call"
        assert torch.equal(batch.h_psi[k], hp) and torch.equal(batch.grad[k], g)
    # the oracle on the smaller systems (its cost is |S| times the coupled-set size)
    checked = 0
    for k, (s, h, d, p) in enumerate(rows):
        if s.dets.shape[0] * h.n_coupled > 3e7:
            continue
        checked += 1
        oe, _, og = oracle.energy(s.n_orb, s.n_alpha, s.n_beta, s.h1, s.eri, s.dets, s.psi)
        assert abs(batch.energy[k].item() - oe) <= E_TOL
        assert np.max(np.abs(batch.grad[k].cpu().numpy() - og)) <= G_TOL
    assert checked >= 3
    batch.close()


def test_streaming_chunk_loop_graph_replays():
    """The pool-streaming loop (generation of chunk k+1 on one stream, dedup of chunk k
    on a second) captured once and replayed: every replay equals the eager result."""
    from tests.gpu_common import ham
    sci = require_gpu()
    s = system("medium")
    h = ham("medium")
    dets = s.dets[pick_sources(s.dets.shape[0], 12, 5)]
    d = sci.keys_to_device(dets)
    sel = sci.keys_to_device(s.dets)
    n = dets.shape[0]
    total = n * h.n_coupled
    chunk = 70_000
    cap = total + s.dets.shape[0]
    dev = torch.device("cuda")
    set_a = torch.empty((cap, 1), dtype=torch.int64, device=dev)
    set_b = torch.empty_like(set_a)
    n_in = torch.tensor([s.dets.shape[0]], dtype=torch.int64, device=dev)
    n_out = torch.zeros(1, dtype=torch.int64, device=dev)
    ws = torch.empty(sci.sci_stream_workspace_bytes(h, chunk), dtype=torch.uint8, device=dev)
    flags = sci.new_flags(dev)
    dd = torch.cuda.Stream()

    def run():
        cur = torch.cuda.current_stream()
        is_b = sci.sci_stream_dedup(h, d, n, 0, total, chunk, sel, n_in, set_a, set_b, cap, n_out, ws, ws.numel(),
                                    flags, cur, dd)
        cur.wait_stream(dd)
        return is_b

    say(f"captured streaming loop: {total} candidates in chunks of {chunk}")
    is_b = run()
    torch.cuda.synchronize()
    m = int(n_out.item())
    ref = (set_b if is_b else set_a)[:m].clone()
    ok, _, _ = oracle.gen_coupled(s.n_orb, s.n_alpha, s.n_beta, s.h1, s.eri, dets)
    ou, _ = oracle.dedup_merge(1, ok, s.dets)
    assert m == ou.shape[0] and np.array_equal(sci.keys_to_host(ref), ou)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            is_b2 = run()
    torch.cuda.synchronize()
    assert is_b2 == is_b
    for rep in range(3):
        set_a.fill_(0)
        set_b.fill_(0)
        n_out.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int(n_out.item()) == m, f"replay {rep}: count"
        assert torch.equal((set_b if is_b else set_a)[:m], ref), f"replay {rep}: keys"
    assert sci.check_flags(flags, "captured stream") == 0
