#!/usr/bin/env python3
"""Throughput of the NNQS-SCI hot path on one MI355X.

One step = one pass of the whole path over the medium workload
(n_orb = 26 spatial orbitals, 7 alpha + 7 beta electrons, Cholesky rank 100,
100,000 selected determinants as one uint64 each), inputs resident in HBM:

  1. sci_gen_coupled   all 2,513,700,000 coupled determinants + H_ij (FP64, dense)
  2. sci_dedup_merge   global de-duplication of those keys, merged into S
  3. sci_energy        E(psi) over S and dE/dpsi

Printed: one JSON line.  `value` = coupled candidates carried through the whole
step per second.  Per-stage times come from HIP events on the stream the
library launches on; per-kernel times come from the library's own event pairs
around each launch (sci_profile_enable).  `roofline` describes the kernel with
the largest share of the step, against its algorithmic bytes per launch;
`cpu_baseline` times the CPU oracle on a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="medium", choices=["tiny", "medium"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sources", type=int, default=8000)
    ap.add_argument("--cpu-single-sources", type=int, default=500,
                    help="sources of the single-thread oracle sample (0: skip)")
    ap.add_argument("--cpu-only", action="store_true",
                    help="time only the oracle on --cpu-sources sources and print it (no GPU)")
    ap.add_argument("--calib-copy-gib", type=float, default=0.0,
                    help="run one plain device copy of this size first (counter calibration)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the large-workload streaming and energy/autograd timings")
    ap.add_argument("--extras", default="select,screened,large,batch",
                    help="comma list of the extra measurements to run (select, screened, large, batch)")
    ap.add_argument("--large-sources", type=int, default=32768)
    ap.add_argument("--large-chunk", type=int, default=0, help="pool chunk (candidates); 0: pick the fastest of 2^28..2^30")
    ap.add_argument("--batch-chunks", type=int, default=32,
                    help="chunks of the batched workload (each one batch over all systems)")
    return ap.parse_args()


def _median_ms(fn, reps, torch):
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts))


def screened_extras(torch, sci, ham, sel, n_sel, n_cand, keys, hij, dense_ms):
    """Screened generation over the medium workload: keep |H_ij| > eps, with eps the 87th
    percentile of |H_ij| over the candidates of one sampled source (so about an eighth of
    the structural candidates survive, the paper's post-screening ratio)."""
    dev = keys.device
    W = ham.W
    nc = ham.n_coupled
    mid = n_sel // 2
    k1 = torch.empty((nc, W), dtype=torch.int64, device=dev)
    h1 = torch.empty(nc, dtype=torch.float64, device=dev)
    n1 = torch.zeros(1, dtype=torch.int64, device=dev)
    flags = sci.new_flags(dev)
    sci.sci_gen_coupled(ham, sel[mid:mid + 1], 1, 0, nc, -1.0, k1, h1, None, nc, n1, flags)
    eps = float(torch.quantile(h1.abs(), 0.87).item())
    src = torch.empty(n_cand, dtype=torch.int32, device=dev)
    n_out = torch.zeros(1, dtype=torch.int64, device=dev)
    run = lambda: sci.sci_gen_coupled(ham, sel, n_sel, 0, n_cand, eps, keys, hij, src, n_cand, n_out, flags)
    run()
    torch.cuda.synchronize()
    sci.check_flags(flags, "screened generation")
    t_ms = _median_ms(run, 5, torch)
    kept = int(n_out.item())
    del src, k1, h1
    return {"workload": f"medium, all {n_sel} sources, |H_ij| > eps kept (staged per wave in LDS, one "
                        f"output reservation per 512 kept entries and per workgroup at the end of a source)",
            "eps": eps, "eps_rule": f"87th percentile of |H_ij| over the {nc} candidates of source {mid}",
            "n_candidates": n_cand, "n_kept": kept, "kept_fraction": kept / n_cand, "ms": t_ms,
            "candidates_per_s": n_cand / (t_ms / 1000.0), "kept_per_s": kept / (t_ms / 1000.0),
            "dense_ms": dense_ms}


def select_extras(torch, sci, keys, n_cand, union, n_union_dev, n_union, sel, n_sel, W, ws_d):
    """Reverse index of every generated candidate into the union, and top-K of
    synthetic amplitudes over the novel candidates (union minus S)."""
    dev = keys.device
    out = {}
    index = torch.empty(sci.sci_index_bytes(W, n_union), dtype=torch.uint8, device=dev)
    idx = torch.empty(n_cand, dtype=torch.int64, device=dev)
    flags = sci.new_flags(dev)
    build = lambda: sci.sci_index_build(W, union, n_union_dev, n_union, index, index.numel(), flags)
    look = lambda: sci.sci_index_lookup(W, index, index.numel(), keys, n_cand, idx)
    build()
    look()
    torch.cuda.synchronize()
    sci.check_flags(flags, "reverse index")
    assert int((idx[:: max(1, n_cand // 100000)] < 0).sum().item()) == 0, "reverse index: candidate not found"
    b_ms = _median_ms(build, 3, torch)
    l_ms = _median_ms(look, 3, torch)
    out["index"] = {"n_set": n_union, "table_bytes": index.numel(), "build_ms": b_ms, "n_lookups": n_cand,
                    "lookup_ms": l_ms, "lookups_per_s": n_cand / (l_ms / 1000.0),
                    "lookup_stream_GBps": n_cand * (8 * W + 8) / (l_ms / 1000.0) / 1e9}
    del index, idx
    torch.cuda.empty_cache()
    # the novel set, and amplitudes for it drawn on the device (synthetic stand-in for inference)
    n_set_in = torch.tensor([n_sel], dtype=torch.int64, device=dev)
    novel = torch.empty((n_union, W), dtype=torch.int64, device=dev)
    n_novel = torch.zeros(1, dtype=torch.int64, device=dev)
    tmp = torch.empty((n_union + n_sel, W), dtype=torch.int64, device=dev)
    n_tmp = torch.zeros(1, dtype=torch.int64, device=dev)
    sci.sci_dedup_merge(W, keys, n_cand, sel, n_set_in, tmp, n_tmp, tmp.shape[0], novel, n_novel, n_union,
                        ws_d, ws_d.numel(), flags)
    torch.cuda.synchronize()
    del tmp
    nn = int(n_novel.item())
    g = torch.Generator(device=dev)
    g.manual_seed(2604157680)
    psi = torch.randn(nn, dtype=torch.float64, device=dev, generator=g)
    K = 100_000
    ok = torch.empty((K, W), dtype=torch.int64, device=dev)
    n_out = torch.zeros(1, dtype=torch.int64, device=dev)
    ws = torch.empty(sci.sci_topk_workspace_bytes(nn), dtype=torch.uint8, device=dev)
    run = lambda: sci.sci_topk(W, novel, psi, nn, K, ok, None, n_out, K, ws, ws.numel(), flags)
    run()
    torch.cuda.synchronize()
    sci.check_flags(flags, "topk")
    t_ms = _median_ms(run, 3, torch)
    out["topk"] = {"n": nn, "k": K, "ms": t_ms, "entries_per_s": nn / (t_ms / 1000.0), "n_selected": int(n_out.item())}
    return out


def batch_extras(args, torch, sci, si):
    """The batched workload (64 systems of uneven size, both key widths): full
    generation of every system, cut into chunks that each cover a slice of every
    system, as batched launches, as one captured graph replayed, and as 64
    sequential plain calls per chunk; energies of all 64 systems batched vs plain."""
    wls = si.batch_workloads()
    systems = [si.make_system(w) for w in wls]
    dev = torch.device("cuda", 0)
    hams = [sci.Ham(s.n_orb, s.n_alpha, s.n_beta, s.h1, s.eri) for s in systems]
    sels = [sci.keys_to_device(s.dets) for s in systems]
    E = [s.dets.shape[0] * h.n_coupled for s, h in zip(systems, hams)]
    total = sum(E)
    K = args.batch_chunks
    rng = [[(j * e // K, (j + 1) * e // K) for e in E] for j in range(K)]
    words = max(sum((r1 - r0) * h.W for (r0, r1), h in zip(rng[j], hams)) for j in range(K))
    cmax = max(sum(r1 - r0 for r0, r1 in rng[j]) for j in range(K))
    pool_k = torch.empty(words + 1, dtype=torch.int64, device=dev)
    pool_h = torch.empty(cmax + 1, dtype=torch.float64, device=dev)
    flags = sci.new_flags(dev)

    def views(j):
        out, ok, oh = [], 0, 0
        for (r0, r1), h in zip(rng[j], hams):
            n = r1 - r0
            out.append((pool_k[ok: ok + n * h.W].view(n, h.W), pool_h[oh: oh + n]))
            ok += n * h.W
            oh += n
        return out

    def items(j):
        return [(h, d, r0, r1, kv, hv) for h, d, (r0, r1), (kv, hv) in zip(hams, sels, rng[j], views(j))]

    first = sci.GenBatch(items(0), flags=flags)
    tile = first.autotune()
    batches = [first] + [sci.GenBatch(items(j), tile_candidates=tile, flags=flags) for j in range(1, K)]
    torch.cuda.synchronize()

    def run_batched():
        for b in batches:
            b.launch()

    all_views = [views(j) for j in range(K)]

    def run_plain():
        for k, (h, d) in enumerate(zip(hams, sels)):
            for j in range(K):
                r0, r1 = rng[j][k]
                kv, hv = all_views[j][k]
                sci.sci_gen_coupled(h, d, d.shape[0], r0, r1, -1.0, kv, hv, None, r1 - r0, None, flags)

    run_batched()
    run_plain()
    torch.cuda.synchronize()
    b_ms = _median_ms(run_batched, 3, torch)
    p_ms = _median_ms(run_plain, 3, torch)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            run_batched()
    torch.cuda.synchronize()
    g_ms = _median_ms(graph.replay, 3, torch)
    sci.check_flags(flags, "batched generation")
    del graph
    gen = {"workload": f"{len(wls)} systems (n_orb {min(w.n_orb for w in wls)}-{max(w.n_orb for w in wls)}, "
                       f"{sum(w.W == 2 for w in wls)} with W=2, {sum(w.n_sel for w in wls)} selected dets), "
                       f"full generation in {K} chunks",
           "n_candidates": total, "tile_candidates": tile,
           "batched_ms": b_ms, "graph_ms": g_ms, "sequential_plain_ms": p_ms,
           "batched_candidates_per_s": total / (b_ms / 1000.0), "graph_candidates_per_s": total / (g_ms / 1000.0),
           "sequential_candidates_per_s": total / (p_ms / 1000.0), "speedup_vs_sequential": p_ms / b_ms}
    for b in batches:
        b.close()
    del pool_k, pool_h
    # energies (with gradients) of all systems
    psis = [torch.from_numpy(s.psi).to(dev) for s in systems]
    eb = sci.EnergyBatch([(h, d, p) for h, d, p in zip(hams, sels, psis)], flags=flags)
    outs = [(torch.zeros(1, dtype=torch.float64, device=dev), torch.empty(d.shape[0], dtype=torch.float64, device=dev),
             torch.empty(d.shape[0], dtype=torch.float64, device=dev),
             torch.empty(sci.sci_energy_workspace_bytes(d.shape[0]), dtype=torch.uint8, device=dev)) for d in sels]

    def plain_energy():
        for h, d, p, (e, hp, g, ws) in zip(hams, sels, psis, outs):
            sci.sci_energy(h, d, d.shape[0], p, e, hp, g, ws, ws.numel(), flags)

    eb.launch()
    plain_energy()
    torch.cuda.synchronize()
    same = all(eb.energy[k].item() == outs[k][0].item() for k in range(len(outs)))
    eb_ms = _median_ms(eb.launch, 5, torch)
    ep_ms = _median_ms(plain_energy, 5, torch)
    sci.check_flags(flags, "batched energy")
    eb.close()
    en = {"workload": f"E and dE/dpsi of all {len(wls)} systems", "batched_ms": eb_ms, "sequential_plain_ms": ep_ms,
          "speedup_vs_sequential": ep_ms / eb_ms, "bit_identical_to_plain": same}
    return gen, en


def large_extras(args, torch, sci, si):
    """Large workload (n_orb=60, 10a+10b, W=2): one mini-batch of `large_sources` sources
    of S (32768 by default, over 1e10 candidates) streamed through the device pool
    (generation of chunk k+1 overlapping dedup-merge of chunk k into S), and E / E+dE/dpsi
    over all of S, plain and through autograd."""
    wl = si.WORKLOADS["large"]
    sysm = si.make_system(wl)
    dev = torch.device("cuda", 0)
    ham = sci.Ham(wl.n_orb, wl.n_alpha, wl.n_beta, sysm.h1, sysm.eri)
    sel = sci.keys_to_device(sysm.dets)
    n_sel = sel.shape[0]
    n_src = min(args.large_sources, n_sel)
    dets = sel[:n_src]
    total = n_src * ham.n_coupled
    chunks = [args.large_chunk] if args.large_chunk > 0 else [1 << 28, 1 << 29, 1 << 30]
    W = ham.W
    ws_bytes = max(sci.sci_stream_workspace_bytes(ham, c) for c in chunks)
    # the two set buffers take what HBM has left (the union is far below the candidate count)
    free_bytes = torch.cuda.mem_get_info(dev)[0]
    cap = int(min(total + n_sel, (free_bytes - ws_bytes - (8 << 30)) // (2 * W * 8)))
    set_a = torch.empty((cap, W), dtype=torch.int64, device=dev)
    set_b = torch.empty_like(set_a)
    n_in = torch.tensor([n_sel], dtype=torch.int64, device=dev)
    n_out = torch.zeros(1, dtype=torch.int64, device=dev)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    flags = sci.new_flags(dev)
    gen_stream = torch.cuda.current_stream()
    dd_stream = torch.cuda.Stream()

    def run_chunk(c):
        sci.sci_stream_dedup(ham, dets, n_src, 0, total, c, sel, n_in, set_a, set_b, cap, n_out,
                             ws, ws.numel(), flags, gen_stream, dd_stream)
        torch.cuda.current_stream().wait_stream(dd_stream)

    # pool chunk: the fastest of the candidates, one timed pass each after a warm-up pass
    torch.cuda.reset_peak_memory_stats(dev)
    sweep = {}
    for c in chunks:
        run_chunk(c)
        torch.cuda.synchronize()
        sci.check_flags(flags, "large stream warmup")
        sweep[c] = _median_ms(lambda: run_chunk(c), 1, torch)
    peak_alloc = torch.cuda.max_memory_allocated(dev)
    chunk = min(sweep, key=sweep.get)
    run = lambda: run_chunk(chunk)
    sci.sci_profile_read()
    sci.sci_profile_enable(True)
    t_ms = _median_ms(run, 3, torch)
    torch.cuda.synchronize()
    kern = {}
    for name, ms in sci.sci_profile_read():
        kern[name] = kern.get(name, 0.0) + ms / 3
    sci.sci_profile_enable(False)
    sci.check_flags(flags, "large stream")
    n_union = int(n_out.item())
    del set_a, set_b, ws
    out = {
        "workload": f"{wl.name}: n_orb={wl.n_orb} {wl.n_alpha}a+{wl.n_beta}b rank={wl.rank} n_sel={n_sel} W={W}; "
                    f"one mini-batch of the first {n_src} sources streamed in pool chunks of {chunk} candidates, merged into S",
        "n_candidates": total, "n_unique_union": n_union, "ms": t_ms,
        "chunk": chunk, "chunk_sweep_ms": {str(c): round(v, 1) for c, v in sweep.items()},
        "device_bytes": {"pool_and_workspace": ws_bytes, "set_buffers": 2 * cap * W * 8,
                         "peak_allocated": peak_alloc},
        "candidates_per_s": total / (t_ms / 1000.0),
        "kernel_ms": {k: round(v, 3) for k, v in sorted(kern.items(), key=lambda x: -x[1]) if v >= 0.05},
    }
    # energy and gradient over the large S: plain entry point and the autograd path
    psi = torch.from_numpy(sysm.psi).to(dev)
    e_ms = _median_ms(lambda: sci.energy(ham, sel, psi, want_hpsi=False, want_grad=False), 5, torch)
    eg_ms = _median_ms(lambda: sci.energy(ham, sel, psi, want_hpsi=False, want_grad=True), 5, torch)

    def auto():
        p = psi.clone().requires_grad_(True)
        e = sci.SciEnergy.apply(p, ham, sel)
        e.backward()

    ag_ms = _median_ms(auto, 5, torch)
    energy = {"workload": f"{wl.name}: E over all {n_sel} selected determinants", "n_sel": n_sel,
              "energy_ms": e_ms, "energy_grad_ms": eg_ms, "autograd_fwd_bwd_ms": ag_ms}
    return out, energy


def _template_args(name, fam):
    """Template arguments of `fam` in a kernel name, as strings ([] when not a template)."""
    i = name.find(fam + "<")
    if i < 0:
        return []
    j, depth = i + len(fam) + 1, 1
    k = j
    while k < len(name) and depth:
        depth += {"<": 1, ">": -1}.get(name[k], 0)
        k += 1
    return [a.strip() for a in name[j:k - 1].split(",")]


def recorded_traffic(kernel_name, W):
    """HBM bytes per launch of `kernel_name` from the committed PMC record, or None when
    there is none or the kernel's source file changed since the counters were taken."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", "kernel_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    fam = kernel_name.strip("()").split("<")[0]
    # the label's template arguments as the compiled kernel spells them
    fan = {"C::F1": "4096", "C::F2": "512" if W == 1 else "256"}
    want = [str(W) if a == "W" else fan.get(a, a) for a in _template_args(kernel_name, fam)]
    for name, e in rec.get("kernels", {}).items():
        if e.get("family") != fam or _template_args(name, fam) != want:
            continue
        src = os.path.join(here, e["source"])
        if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != e["source_sha256"]:
            return None
        return e["read_bytes"] + e["write_bytes"]
    return None


def copy_bandwidth(torch, dev, gib=4.0, reps=3):
    """Read + write GB/s of a plain device-to-device copy of `gib` GiB (median of `reps`)."""
    nel = int(gib * 2**30) // 8
    a = torch.empty(nel, dtype=torch.int64, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    del a, b
    torch.cuda.empty_cache()
    return 2 * nel * 8 / (float(np.median(ts)) / 1000.0) / 1e9


def gen_dedup_traffic(per_kernel, W, stage_ms, copy_gbps):
    """HBM bytes the counters recorded for the generation and dedup kernels of one step
    (PMC FETCH_SIZE + WRITE_SIZE, calibrated, per launch) over the two stages' time.
    Kernels without a current record (small ones, or source changed since the counters
    were taken) are left out; `time_covered` is the share of kernel time that has one."""
    tot_bytes, covered_ms, all_ms = 0.0, 0.0, 0.0
    for name, k in per_kernel.items():
        if "hpsi" in name or "reduce" in name or "grad" in name:
            continue  # energy stage
        ms = k["ms_per_launch"] * k["launches_per_step"]
        all_ms += ms
        b = recorded_traffic(name, W)
        if b is not None:
            tot_bytes += b * k["launches_per_step"]
            covered_ms += ms
    if covered_ms == 0.0:
        return {"bytes_per_step": None, "achieved": None, "copy_GBps": copy_gbps, "time_covered": 0.0}
    gbps = tot_bytes / (stage_ms / 1000.0) / 1e9
    return {"bytes_per_step": tot_bytes, "stage_ms": stage_ms, "achieved": gbps, "unit": "GB/s",
            "frac_of_peak": gbps / HBM_PEAK_GBS, "peak": HBM_PEAK_GBS,
            "copy_GBps": copy_gbps, "frac_of_copy": gbps / copy_gbps, "time_covered": covered_ms / all_ms}


def cpu_baseline(sysm, n_src):
    """The oracle, as it stands, on the first n_src sources: generation,
    dedup of their candidates into S, and H psi for the same rows."""
    import oracle
    wl = sysm.workload
    dets = sysm.dets[:n_src]
    t0 = time.perf_counter()
    keys, _, _ = oracle.gen_coupled(wl.n_orb, wl.n_alpha, wl.n_beta, sysm.h1, sysm.eri, dets)
    oracle.dedup_merge(wl.W, keys, sysm.dets)
    oracle.hpsi_rows(wl.n_orb, wl.n_alpha, wl.n_beta, sysm.h1, sysm.eri, sysm.dets, sysm.psi,
                     np.arange(n_src, dtype=np.int64))
    dt = time.perf_counter() - t0
    n_cand = keys.shape[0]
    return {"value": n_cand / dt, "unit": "candidates/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"first {n_src} of {dets.shape[0] if n_src > dets.shape[0] else sysm.dets.shape[0]} "
                      f"sources: generation ({n_cand} candidates), dedup into S, H psi rows; {dt:.1f} s"}


def single_thread_baseline(n_src):
    """The oracle on one host thread, timed in a child process (OpenMP fixes its thread
    count when the library loads); the child runs only the CPU oracle."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-only", "--cpu-sources", str(n_src)]
    r = subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        return {"error": r.stderr[-300:]}
    return json.loads(r.stdout.strip().splitlines()[-1])


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported in this build", file=sys.stderr)
        sys.exit(2)
    if args.cpu_only:
        import sci_inputs as si
        print(json.dumps(cpu_baseline(si.make_system(si.WORKLOADS[args.workload]), args.cpu_sources)), flush=True)
        return
    import torch

    import paper_2604_15768_amd as sci
    import sci_inputs as si

    wl = si.WORKLOADS[args.workload]
    sysm = si.make_system(wl)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    ham = sci.Ham(wl.n_orb, wl.n_alpha, wl.n_beta, sysm.h1, sysm.eri)
    n_sel = sysm.dets.shape[0]
    n_cand = n_sel * ham.n_coupled
    W = ham.W

    # resident inputs and preallocated outputs / workspaces
    sel = sci.keys_to_device(sysm.dets)
    psi = torch.from_numpy(sysm.psi).to(dev)
    keys = torch.empty((n_cand, W), dtype=torch.int64, device=dev)
    hij = torch.empty(n_cand, dtype=torch.float64, device=dev)
    n_gen = torch.zeros(1, dtype=torch.int64, device=dev)
    set_cap = n_cand + n_sel
    n_set_in = torch.tensor([n_sel], dtype=torch.int64, device=dev)
    set_out = torch.empty((set_cap, W), dtype=torch.int64, device=dev)
    n_set_out = torch.zeros(1, dtype=torch.int64, device=dev)
    ws_d = torch.empty(sci.sci_dedup_workspace_bytes(W, n_cand), dtype=torch.uint8, device=dev)
    ws_e = torch.empty(sci.sci_energy_workspace_bytes(n_sel), dtype=torch.uint8, device=dev)
    energy = torch.zeros(1, dtype=torch.float64, device=dev)
    hpsi = torch.empty(n_sel, dtype=torch.float64, device=dev)
    grad = torch.empty(n_sel, dtype=torch.float64, device=dev)
    flags = sci.new_flags(dev)
    stream = torch.cuda.current_stream()

    if args.calib_copy_gib > 0:
        nel = int(args.calib_copy_gib * 2**30) // 8
        a = torch.empty(nel, dtype=torch.int64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # bandwidth a plain device copy reaches here (read + write), the practical ceiling
    copy_gbps = copy_bandwidth(torch, dev)

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]

    def step(record=False):
        if record:
            ev[0].record(stream)
        sci.sci_gen_coupled(ham, sel, n_sel, 0, n_cand, -1.0, keys, hij, None, n_cand, n_gen, flags, stream)
        if record:
            ev[1].record(stream)
        sci.sci_dedup_merge(W, keys, n_cand, sel, n_set_in, set_out, n_set_out, set_cap, None, None, 0,
                            ws_d, ws_d.numel(), flags, stream)
        if record:
            ev[2].record(stream)
        sci.sci_energy(ham, sel, n_sel, psi, energy, hpsi, grad, ws_e, ws_e.numel(), flags, stream)
        if record:
            ev[3].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    sci.check_flags(flags, "bench warmup")
    n_unique = int(n_set_out.item())

    t_gen, t_dd, t_en = [], [], []
    kern_ms, kern_calls = {}, {}
    torch.cuda.synchronize()
    sci.sci_profile_read()
    sci.sci_profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(record=True)
        ev[3].synchronize()
        t_gen.append(ev[0].elapsed_time(ev[1]))
        t_dd.append(ev[1].elapsed_time(ev[2]))
        t_en.append(ev[2].elapsed_time(ev[3]))
        for name, ms in sci.sci_profile_read():
            kern_ms[name] = kern_ms.get(name, 0.0) + ms
            kern_calls[name] = kern_calls.get(name, 0) + 1
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sci.sci_profile_enable(False)
    sci.check_flags(flags, "bench")
    ms_step = 1000.0 * wall / args.steps

    g_ms = float(np.mean(t_gen))
    d_ms = float(np.mean(t_dd))
    e_ms = float(np.mean(t_en))
    gen_bytes = n_cand * (8 * W + 8) + n_sel * 8 * W       # written keys + H_ij, read sources
    dedup_lb_bytes = 2 * n_cand * 8 * W                    # any sort reads and writes every key once
    # algorithmic bytes per launch of each kernel family (what the work must move at least)
    algo = {
        "gen_kernel": ("hbm", gen_bytes),
        "bucket_kernel": ("hbm", (n_cand + n_unique) * 8 * W),
        "emit_kernel": ("hbm", 2 * n_unique * 8 * W),
        "scatter_kernel": ("hbm", 2 * n_cand * 8 * W),
        "hist_kernel": ("hbm", n_cand * 8 * W),
        "merge_kernel": ("hbm", (n_unique + n_sel + n_unique) * 8 * W),
        "merge_union_kernel": ("hbm", (n_unique + n_sel + n_unique) * 8 * W),
    }
    per_kernel = {}
    for name, tot in kern_ms.items():
        per_kernel[name] = {"ms_per_launch": tot / kern_calls[name], "launches_per_step": kern_calls[name] / args.steps}
    dom = max(kern_ms, key=lambda k: kern_ms[k])
    fam = next((f for f in algo if f in dom), None)
    dom_ms = kern_ms[dom] / kern_calls[dom]
    if fam is not None:
        bound, nbytes = algo[fam]
        roof = {"kernel": dom, "bound": bound, "achieved": nbytes / (dom_ms / 1000.0) / 1e9, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": nbytes / (dom_ms / 1000.0) / 1e9 / HBM_PEAK_GBS,
                "traffic": recorded_traffic(dom, W),
                "algorithmic_bytes_per_launch": nbytes, "ms_per_launch": dom_ms}
    else:
        roof = {"kernel": dom, "bound": "alu", "achieved": None, "peak": None, "unit": None, "frac": None,
                "traffic": None, "ms_per_launch": dom_ms}
    result = {
        "metric": "coupled dets+H_ij/s and dedup keys/s (HBM GB/s); E+dE/dpsi time",
        "value": n_cand / (ms_step / 1000.0),
        "unit": "candidates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{wl.name}: n_orb={wl.n_orb} {wl.n_alpha}a+{wl.n_beta}b rank={wl.rank} "
                        f"n_sel={n_sel} W={W}; full generation + dedup-merge into S + energy",
            "n_candidates": n_cand,
            "n_unique_union": n_unique,
            "stage_ms": {"gen_coupled": g_ms, "dedup_merge": d_ms, "energy_grad": e_ms},
            "gen_candidates_per_s": n_cand / (g_ms / 1000.0),
            "dedup_keys_per_s": n_cand / (d_ms / 1000.0),
            "dedup_lower_bound_GBps": dedup_lb_bytes / (d_ms / 1000.0) / 1e9,
            "energy": float(energy.item()),
        },
        "roofline": roof,
        "kernels": per_kernel,
        "gen_roofline": {"bound": "hbm", "achieved": gen_bytes / (g_ms / 1000.0) / 1e9, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": gen_bytes / (g_ms / 1000.0) / 1e9 / HBM_PEAK_GBS},
        "gen_dedup_hbm": gen_dedup_traffic(per_kernel, W, g_ms + d_ms, copy_gbps),
    }
    if not args.no_extras:
        want = set(args.extras.split(","))
        result["extras"] = {}
        if "select" in want:
            result["extras"]["reverse_index_topk"] = select_extras(torch, sci, keys, n_cand, set_out, n_set_out,
                                                                   n_unique, sel, n_sel, W, ws_d)
        if "screened" in want:
            result["extras"]["screened_generation"] = screened_extras(torch, sci, ham, sel, n_sel, n_cand, keys,
                                                                      hij, g_ms)
        del keys, hij, set_out, ws_d
        torch.cuda.empty_cache()
        if "large" in want:
            ls, eg = large_extras(args, torch, sci, si)
            result["extras"].update({"large_stream": ls, "energy_grad_large": eg})
            torch.cuda.empty_cache()
        if "batch" in want:
            bg, be = batch_extras(args, torch, sci, si)
            result["extras"].update({"batched_generation": bg, "batched_energy": be})
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(sysm, args.cpu_sources)
        if args.cpu_single_sources > 0:
            result["cpu_baseline"]["single_thread"] = single_thread_baseline(args.cpu_single_sources)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
