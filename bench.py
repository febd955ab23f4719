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
    ap.add_argument("--calib-copy-gib", type=float, default=0.0,
                    help="run one plain device copy of this size first (counter calibration)")
    return ap.parse_args()


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
    for name, e in rec.get("kernels", {}).items():
        if e.get("family") != fam or f"{fam}<{W}" not in name:
            continue
        if fam in ("hist_kernel", "scatter_kernel"):  # two instantiations: match the fan-out
            lvl = "4096" if "C::F1" in kernel_name else ("512" if W == 1 else "256")
            if f", {lvl}>" not in name:
                continue
        src = os.path.join(here, e["source"])
        if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != e["source_sha256"]:
            return None
        return e["read_bytes"] + e["write_bytes"]
    return None


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


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported in this build", file=sys.stderr)
        sys.exit(2)
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
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(sysm, args.cpu_sources)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
