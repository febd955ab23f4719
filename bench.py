#!/usr/bin/env python3
"""Throughput of the NNQS-SCI hot path on one MI355X.

Headline step (default, the large workload: n_orb = 60 spatial orbitals,
10 alpha + 10 beta electrons, Cholesky rank 240, 200,000 selected determinants
as two uint64 words each), inputs resident in HBM:

  1. sci_stream_dedup  one mini-batch of 32,768 sources of S: all their
                       11,837,440,000 coupled determinants + H_ij (FP64, dense),
                       generated into a two-buffer device pool in chunks of 2^30
                       candidates and de-duplicated + merged into S chunk by chunk
                       (generation of chunk k+1 overlaps the dedup of chunk k)
  2. sci_energy        E(psi) over all of S and dE/dpsi

Printed: one JSON line.  `value` = coupled candidates carried through the whole
step per second.  Stage times come from HIP events on the launching stream;
per-kernel times come from the library's own event pairs around each launch
(sci_profile_enable), on the stream each kernel is launched on.  `roofline`
describes the kernel with the largest share of the step against its
algorithmic bytes (defined per kernel below, from per-chunk set sizes measured
in an untimed pass before the timed steps); `cpu_baseline` times the CPU oracle
on a bounded sample of the same workload.  Extras (same line) cover the whole
large selected space streamed into one set (7.2e10 candidates), the medium
workload's full step, screened generation, the reverse index and top-K, energy
and autograd timings, and the batched workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload large|medium]
                    [--no-extras] [--extras LIST] [--no-cpu-baseline]
    python bench.py --record-traffic FETCH_DIR WRITE_DIR WORKLOAD   (host only)
"""
import argparse
import glob
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
HERE = os.path.dirname(os.path.abspath(__file__))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="large", choices=["large", "medium", "tiny"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sources", type=int, default=0,
                    help="sources of the oracle sample (0: 480 large, 8000 medium, all tiny)")
    ap.add_argument("--cpu-single-sources", type=int, default=-1,
                    help="sources of the single-thread oracle sample (0: skip; -1: per workload)")
    ap.add_argument("--medium-cpu-sources", type=int, default=25000,
                    help="sources of the oracle leg of the medium extra (0: skip)")
    ap.add_argument("--cpu-only", action="store_true",
                    help="time only the oracle on --cpu-sources sources of --workload and print it (no GPU)")
    ap.add_argument("--calib-copy-gib", type=float, default=0.0,
                    help="run one plain device copy of this size first (counter calibration)")
    ap.add_argument("--counters", action="store_true",
                    help="a run for counter collection: no size pass, no extras, no CPU baseline")
    ap.add_argument("--no-extras", action="store_true", help="skip every extra measurement")
    ap.add_argument("--extras", default="whole,medium,select,screened,energy,batch",
                    help="comma list of extras (whole, medium, select, screened, energy, batch)")
    ap.add_argument("--large-sources", type=int, default=32768)
    ap.add_argument("--large-chunk", type=int, default=-1,
                    help="pool chunk in candidates (-1: the fewest equal chunks of at most LARGE_CHUNK_MAX; "
                         "0: time 2^29, 2^30, 2^31 and the default once each and keep the fastest)")
    ap.add_argument("--energy-after", action="store_true",
                    help="run E and dE/dpsi after the stream of chunks instead of beside it")
    ap.add_argument("--batch-chunks", type=int, default=32,
                    help="chunks of the batched workload (each one batch over all systems)")
    ap.add_argument("--summarize-trace", nargs=2, metavar=("KERNEL_TRACE_CSV", "BENCH_OUTPUT"),
                    help="print a markdown table of the kernels of the timed steps of a profiled run of this "
                         "script (rocprofv3 --kernel-trace CSV + that run's JSON line), then exit")
    ap.add_argument("--record-traffic", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "WORKLOAD"),
                    help="turn two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of this script into "
                         "profiles/kernel_traffic.json entries for WORKLOAD, then exit")
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


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


# ---------------------------------------------------------------------------
# counter records (rocprofv3 --pmc) -> calibrated HBM bytes per kernel launch
# ---------------------------------------------------------------------------

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


def equal_chunks(total, max_chunk):
    """The fewest equal pool chunks of at most max_chunk candidates: (chunk, count)."""
    n = -(-total // max_chunk)
    chunk = -(-total // n)
    return chunk, -(-total // chunk)


# largest pool chunk of the large-workload mini-batch (candidates): with two pool buffers
# of (key + H_ij) and the dedup workspace it leaves about 140 GB of HBM for the set
# buffers, which hold the 3.06e9-key union of the mini-batch twice with room to spare
LARGE_CHUNK_MAX = 2_400_000_000
# the same for all of S streamed into one set, whose 5.5e9-key union needs 179 GB of
# set buffers
WHOLE_CHUNK_MAX = 1_600_000_000

# fan-outs of the two partition levels as the compiled kernels spell them (DCfg<W>)
FANOUT = {1: {"C::F1": "4096", "C::F2": "512"}, 2: {"C::F1": "4096", "C::F2": "1024"}}


def family(name):
    return name.strip("()").split("<")[0].split("(")[0].split("::")[-1].strip()


def recorded_traffic(kernel_name, W, workload=None):
    """HBM bytes per launch of `kernel_name` from the committed PMC record, or None when
    there is none or the kernel's source file changed since the counters were taken."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "kernel_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    fam = family(kernel_name)
    want = [str(W) if a == "W" else FANOUT.get(int(W), {}).get(a, a) for a in _template_args(kernel_name, fam)]
    if "workloads" in rec:
        tables = [rec["workloads"].get(workload, {}).get("kernels", {})] if workload else \
            [w.get("kernels", {}) for w in rec["workloads"].values()]
    else:
        tables = [rec.get("kernels", {})]
    root = os.path.dirname(path)
    for table in tables:
        for name, e in table.items():
            if e.get("family") != fam or _template_args(name, fam) != want:
                continue
            src = os.path.join(os.path.dirname(root), e["source"])
            if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != e["source_sha256"]:
                return None
            return e["read_bytes"] + e["write_bytes"]
    return None


def _read_pmc_csv(d):
    """{kernel name: [value per dispatch]} from the counter CSV files under d."""
    import csv
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    out, calib = {}, []
    for f in files:
        for row in csv.DictReader(open(f)):
            name = row.get("Kernel_Name") or row.get("Kernel-Name") or ""
            val = float(row.get("Counter_Value") or row.get("Counter-Value") or 0.0)
            out.setdefault(name, []).append(val)
    return out


def record_traffic(fetch_dir, write_dir, workload):
    """Calibrated FETCH_SIZE / WRITE_SIZE (KiB per dispatch in the CSV) per launch of every
    library kernel of a run, stored under `workload` in profiles/kernel_traffic.json
    with the SHA-256 of the kernel's source file.  The run includes a plain device copy
    of --calib-copy-gib GiB (__amd_rocclr_copyBuffer): its counters against the bytes it
    moves give the scale factors."""
    fetch, write = _read_pmc_csv(fetch_dir), _read_pmc_csv(write_dir)
    copy = [k for k in fetch if "copyBuffer" in k]
    if not copy:
        raise SystemExit("no calibration copy in the fetch run (use --calib-copy-gib)")
    big_f = max(fetch[copy[0]])
    big_w = max(write[[k for k in write if "copyBuffer" in k][0]])
    gib = max(big_f, big_w) / 2**20  # the copy moves the same bytes each way
    moved = round(gib) * 2**30
    read_scale, write_scale = moved / (big_f * 1024.0), moved / (big_w * 1024.0)
    srcs = {}
    for f in glob.glob(os.path.join(HERE, "paper_2604_15768_amd", "csrc", "*.hip")):
        srcs[f] = open(f).read()
    kernels = {}
    for name, vals in fetch.items():
        if "sci::" not in name or name not in write:
            continue
        fam = family(name.split("(")[0])
        # the file that defines the kernel: "__global__ ... fam(" with no ';' or '{' between
        pat = re.compile(r"__global__[^;{]*?\b" + re.escape(fam) + r"\s*\(", re.S)
        src = next((p for p, t in srcs.items() if pat.search(t)), None)
        if src is None:
            continue
        kernels[name] = {"family": fam, "source": os.path.relpath(src, HERE),
                         "source_sha256": hashlib.sha256(open(src, "rb").read()).hexdigest(),
                         "launches": len(vals),
                         "read_bytes": float(np.mean(vals)) * 1024.0 * read_scale,
                         "write_bytes": float(np.mean(write[name])) * 1024.0 * write_scale}
    path = os.path.join(HERE, "profiles", "kernel_traffic.json")
    rec = json.load(open(path)) if os.path.exists(path) else {}
    if "workloads" not in rec:
        rec = {"workloads": {}}
    rec["workloads"][workload] = {"read_scale": read_scale, "write_scale": write_scale,
                                  "calibration": f"{round(gib)} GiB device copy", "kernels": kernels}
    json.dump(rec, open(path, "w"), indent=1)
    print(f"{len(kernels)} kernels recorded for {workload} (read x{read_scale:.3f}, write x{write_scale:.3f})")


def summarize_trace(trace_csv, bench_out):
    """Per-kernel durations of the timed steps of a profiled run: for every kernel the
    bench saw, its last steps x launches_per_step dispatches in the trace (dispatch
    order), next to the average the bench measured with HIP events in the same run."""
    import csv
    res = None
    for line in open(bench_out):
        line = line.strip()
        if line.startswith("{") and '"metric"' in line:
            res = json.loads(line)
    if res is None:
        raise SystemExit(f"no JSON line in {bench_out}")
    rows = list(csv.DictReader(open(trace_csv)))
    rows.sort(key=lambda r: int(r.get("Dispatch_Id") or 0))
    by = {}
    for r in rows:
        name = r.get("Kernel_Name", "")
        ns = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        by.setdefault(name, []).append(ns)
    steps = res["steps"]
    kernels = res["kernels"] if "kernels" in res else res["medium"]["kernels"]
    m = re.search(r"W=(\d)", res["config"]["workload"])
    W = m.group(1) if m else "1"
    out = []
    for bench_name, k in kernels.items():
        n_last = int(round(k["launches_per_step"] * steps))
        fam = family(bench_name)
        want = [W if a == "W" else FANOUT.get(int(W), {}).get(a, a) for a in _template_args(bench_name, fam)]
        for t, d_all in by.items():
            tn = t.split("(")[0].replace("void ", "") if "<" not in t.split("(")[0] else t
            if family(tn.split("(")[0].split("<")[0] + ("<" if "<" in t else "")) != fam and \
                    t.split("(")[0].replace("void ", "").split("::")[-1].split("<")[0] != fam:
                continue
            if _template_args(t, fam) != want:
                continue
            d = d_all[-n_last:] if n_last else []
            if d:
                out.append((t, len(d), sum(d) / len(d) / 1e6, k["ms_per_launch"], k["launches_per_step"]))
    out.sort(key=lambda x: -x[2] * x[4])
    print("| kernel | dispatches (timed steps) | avg ms (trace) | avg ms (bench events) | ms per step (trace) |")
    print("|---|---:|---:|---:|---:|")
    for t, n, ms, bms, lps in out:
        print(f"| `{t.split('(')[0].replace('void ', '')}` | {n} | {ms:.3f} | {bms:.3f} | {ms * lps:.1f} |")


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


def gen_dedup_traffic(per_kernel, W, stage_ms, copy_gbps, workload=None):
    """HBM bytes the counters recorded for the generation and dedup kernels of one step
    (PMC FETCH_SIZE + WRITE_SIZE, calibrated, per launch) over the stage time.  Kernels
    without a current record (small ones, or source changed since the counters were
    taken) are left out; `time_covered` is the share of kernel time that has one."""
    tot_bytes, covered_ms, all_ms = 0.0, 0.0, 0.0
    for name, k in per_kernel.items():
        if "hpsi" in name or "reduce" in name or "grad" in name:
            continue  # energy stage
        ms = k["ms_per_launch"] * k["launches_per_step"]
        all_ms += ms
        b = recorded_traffic(name, W, workload)
        if b is not None:
            tot_bytes += b * k["launches_per_step"]
            covered_ms += ms
    if covered_ms == 0.0:
        return {"bytes_per_step": None, "achieved": None, "copy_GBps": copy_gbps, "time_covered": 0.0}
    gbps = tot_bytes / (stage_ms / 1000.0) / 1e9
    return {"bytes_per_step": tot_bytes, "stage_ms": stage_ms, "achieved": gbps, "unit": "GB/s",
            "frac_of_peak": gbps / HBM_PEAK_GBS, "peak": HBM_PEAK_GBS,
            "copy_GBps": copy_gbps, "frac_of_copy": gbps / copy_gbps, "time_covered": covered_ms / all_ms}


# ---------------------------------------------------------------------------
# timing helpers
# ---------------------------------------------------------------------------

def timed_steps(torch, sci, step, steps, stage_names):
    """Run `steps` steps; step(ev) records len(stage_names)+1 events on the launching
    stream.  Returns (ms per step from the host clock, mean stage ms, per-kernel table)."""
    n_ev = len(stage_names) + 1
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(n_ev)]
    stage = [[] for _ in stage_names]
    kern_ms, kern_calls = {}, {}
    torch.cuda.synchronize()
    sci.sci_profile_read()
    sci.sci_profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        step(ev)
        ev[-1].synchronize()
        for i in range(len(stage_names)):
            stage[i].append(ev[i].elapsed_time(ev[i + 1]))
        for name, ms in sci.sci_profile_read():
            kern_ms[name] = kern_ms.get(name, 0.0) + ms
            kern_calls[name] = kern_calls.get(name, 0) + 1
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sci.sci_profile_enable(False)
    per_kernel = {name: {"ms_per_launch": kern_ms[name] / kern_calls[name],
                         "launches_per_step": kern_calls[name] / steps} for name in kern_ms}
    return 1000.0 * wall / steps, {n: float(np.mean(v)) for n, v in zip(stage_names, stage)}, per_kernel


def roofline(per_kernel, algo_bytes_per_step, W, workload):
    """The kernel with the largest time per step, against its algorithmic bytes.  Kernels
    launched several times per step (one per chunk) are averaged: bytes per launch =
    bytes per step / launches per step."""
    dom = max(per_kernel, key=lambda k: per_kernel[k]["ms_per_launch"] * per_kernel[k]["launches_per_step"])
    k = per_kernel[dom]
    nb = algo_bytes_per_step(dom)
    if nb is None:
        return {"kernel": dom, "bound": "alu", "achieved": None, "peak": None, "unit": None, "frac": None,
                "traffic": None, "ms_per_launch": k["ms_per_launch"]}
    per_launch = nb / k["launches_per_step"]
    gbps = per_launch / (k["ms_per_launch"] / 1000.0) / 1e9
    return {"kernel": dom, "bound": "hbm", "achieved": gbps, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbps / HBM_PEAK_GBS, "traffic": recorded_traffic(dom, W, workload),
            "algorithmic_bytes_per_launch": per_launch, "ms_per_launch": k["ms_per_launch"],
            "launches_per_step": k["launches_per_step"]}


def kernel_rates(per_kernel, algo_bytes_per_step):
    """Algorithmic GB/s of every kernel that has a definition (fraction of HBM peak)."""
    out = {}
    for name, k in per_kernel.items():
        nb = algo_bytes_per_step(name)
        if nb is None:
            continue
        gbps = nb / (k["ms_per_launch"] * k["launches_per_step"] / 1000.0) / 1e9
        out[name] = {"GBps": round(gbps, 1), "frac": round(gbps / HBM_PEAK_GBS, 4),
                     "ms_per_step": round(k["ms_per_launch"] * k["launches_per_step"], 3)}
    return out


# ---------------------------------------------------------------------------
# headline: one large-workload mini-batch streamed through the pool + energy
# ---------------------------------------------------------------------------

def large_chunk_sizes(torch, sci, ham, dets, sel, total, chunk):
    """Untimed pass: the same chunks merged one by one into S with host-visible counts.
    Per chunk: n (candidates), u (distinct keys of the chunk), m0 / m1 (set size
    before / after).  Also the final union size, which the streamed run must equal."""
    dev = dets.device
    W = ham.W
    n_sel = sel.shape[0]
    keys = torch.empty((chunk, W), dtype=torch.int64, device=dev)
    hij = torch.empty(chunk, dtype=torch.float64, device=dev)
    ws = torch.empty(sci.sci_dedup_workspace_bytes(W, chunk), dtype=torch.uint8, device=dev)
    cap = int(min(total + n_sel, 3_400_000_000))
    set_a = torch.empty((cap, W), dtype=torch.int64, device=dev)
    set_b = torch.empty_like(set_a)
    set_a[:n_sel] = sel
    n_a = torch.tensor([n_sel], dtype=torch.int64, device=dev)
    n_b = torch.zeros(1, dtype=torch.int64, device=dev)
    n_u = torch.zeros(1, dtype=torch.int64, device=dev)
    flags = sci.new_flags(dev)
    sizes = []
    cur, nxt, n_cur, n_nxt = set_a, set_b, n_a, n_b
    for a in range(0, total, chunk):
        b = min(a + chunk, total)
        sci.sci_gen_coupled(ham, dets, dets.shape[0], a, b, -1.0, keys, hij, None, chunk, None, flags)
        # distinct keys of the chunk: a merge into nothing, count only (output in set_b's tail is
        # not possible while it is the target, so the pool's H buffer is not used: use nxt)
        sci.sci_dedup_merge(W, keys, b - a, None, None, nxt, n_u, cap, None, None, 0, ws, ws.numel(), flags)
        u = int(n_u.item())
        m0 = int(n_cur.item())
        sci.sci_dedup_merge(W, keys, b - a, cur, n_cur, nxt, n_nxt, cap, None, None, 0, ws, ws.numel(), flags)
        m1 = int(n_nxt.item())
        sizes.append({"n": b - a, "u": u, "m0": m0, "m1": m1})
        cur, nxt, n_cur, n_nxt = nxt, cur, n_nxt, n_cur
    torch.cuda.synchronize()
    sci.check_flags(flags, "chunk size pass")
    del keys, hij, ws, set_a, set_b, cur, nxt, n_cur, n_nxt
    torch.cuda.empty_cache()
    return sizes


def large_algo(sizes, n_src, W):
    """Algorithmic bytes per step of each kernel of the streamed mini-batch (8W-byte keys):
      gen_kernel      every candidate's key + H_ij written, every source read once
      hist_kernel     every candidate key read (one level)
      scatter_kernel  every candidate key read and written (one level)
      bucket_kernel   chunk keys read, the running set's keys read once (each is compared
                      with the chunk's distinct keys), the distinct keys the set lacks written
      emit_kernel     those keys + the running set read, the new set written
    Others (splitters, scans, oversized units) have no definition here."""
    kb = 8 * W
    n = sum(s["n"] for s in sizes)
    m0 = sum(s["m0"] for s in sizes)
    m1 = sum(s["m1"] for s in sizes)
    table = {"gen_kernel": n * (kb + 8) + n_src * kb, "hist_kernel": n * kb, "scatter_kernel": 2 * n * kb,
             "bucket_kernel": (n + m0 + (m1 - m0)) * kb, "emit_kernel": ((m1 - m0) + m0 + m1) * kb}
    return lambda name: table.get(family(name))


def large_headline(args, torch, sci, si, copy_gbps):
    wl = si.WORKLOADS["large"]
    sysm = si.make_system(wl)
    dev = torch.device("cuda", 0)
    ham = sci.Ham(wl.n_orb, wl.n_alpha, wl.n_beta, sysm.h1, sysm.eri)
    W = ham.W
    sel = sci.keys_to_device(sysm.dets)
    psi = torch.from_numpy(sysm.psi).to(dev)
    n_sel = sel.shape[0]
    n_src = min(args.large_sources, n_sel)
    dets = sel[:n_src]
    total = n_src * ham.n_coupled
    cur = torch.cuda.current_stream()
    dd = torch.cuda.Stream()
    out = {}

    def buffers(chunk):
        ws_bytes = sci.sci_stream_workspace_bytes(ham, chunk)
        free_bytes = torch.cuda.mem_get_info(dev)[0]
        # the two set buffers take what HBM has left (the union is far below the candidate count)
        cap = int(min(total + n_sel, (free_bytes - ws_bytes - (6 << 30)) // (2 * W * 8)))
        return (torch.empty(ws_bytes, dtype=torch.uint8, device=dev),
                torch.empty((cap, W), dtype=torch.int64, device=dev),
                torch.empty((cap, W), dtype=torch.int64, device=dev), cap)

    n_in = torch.tensor([n_sel], dtype=torch.int64, device=dev)
    n_out = torch.zeros(1, dtype=torch.int64, device=dev)
    energy = torch.zeros(1, dtype=torch.float64, device=dev)
    hpsi = torch.empty(n_sel, dtype=torch.float64, device=dev)
    grad = torch.empty(n_sel, dtype=torch.float64, device=dev)
    ws_e = torch.empty(sci.sci_energy_workspace_bytes(n_sel), dtype=torch.uint8, device=dev)
    flags = sci.new_flags(dev)

    # Every chunk merges into the whole running set, so fewer chunks read and rewrite it
    # fewer times; equal chunks of at most LARGE_CHUNK_MAX candidates leave room for the
    # set buffers of the union beside the two pool buffers and the dedup workspace
    equal_chunk, _ = equal_chunks(total, LARGE_CHUNK_MAX)
    chunk = args.large_chunk if args.large_chunk > 0 else equal_chunk
    if args.large_chunk == 0:  # sweep: one timed pass each after a warm-up pass
        sweep = {}
        for c in (1 << 29, 1 << 30, 1 << 31, equal_chunk):
            ws, set_a, set_b, cap = buffers(c)
            run = lambda: (sci.sci_stream_dedup(ham, dets, n_src, 0, total, c, sel, n_in, set_a, set_b, cap, n_out,
                                                ws, ws.numel(), flags, cur, dd), cur.wait_stream(dd))
            run()
            torch.cuda.synchronize()
            sweep[c] = _median_ms(run, 1, torch)
            del ws, set_a, set_b
            torch.cuda.empty_cache()
        chunk = min(sweep, key=sweep.get)
        out["chunk_sweep_ms"] = {str(c): round(v, 1) for c, v in sweep.items()}

    sizes = None if args.counters else large_chunk_sizes(torch, sci, ham, dets, sel, total, chunk)
    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats(dev)
    ws, set_a, set_b, cap = buffers(chunk)
    if sizes is not None and cap < sizes[-1]["m1"]:
        raise SystemExit(f"set buffers of {cap} keys cannot hold the union of {sizes[-1]['m1']}")

    # E and dE/dpsi over S read only S and psi, not the union the stream builds: by
    # default they run on a stream of their own beside the stream of chunks (the step
    # ends when both have); the step's stages are the stream of chunks, then the rest
    # of the energy that did not fit beside it
    es = torch.cuda.Stream()

    def step(ev):
        ev[0].record(cur)
        if not args.energy_after:
            es.wait_stream(cur)
            sci.sci_energy(ham, sel, n_sel, psi, energy, hpsi, grad, ws_e, ws_e.numel(), flags, es)
        sci.sci_stream_dedup(ham, dets, n_src, 0, total, chunk, sel, n_in, set_a, set_b, cap, n_out,
                             ws, ws.numel(), flags, cur, dd)
        cur.wait_stream(dd)
        ev[1].record(cur)
        if args.energy_after:
            sci.sci_energy(ham, sel, n_sel, psi, energy, hpsi, grad, ws_e, ws_e.numel(), flags, cur)
        else:
            cur.wait_stream(es)
        ev[2].record(cur)

    warm = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    for _ in range(args.warmup):
        step(warm)
    torch.cuda.synchronize()
    sci.check_flags(flags, "bench warmup")
    ms_step, stages, per_kernel = timed_steps(torch, sci, step, args.steps, ["stream", "energy"])
    sci.check_flags(flags, "bench")
    n_union = int(n_out.item())
    peak = torch.cuda.max_memory_allocated(dev)
    s_ms = stages["stream"]
    kb = 8 * W
    gen_bytes = total * (kb + 8) + n_src * kb
    dedup_lb = 2 * total * kb
    res = {
        "metric": "coupled dets+H_ij/s and dedup keys/s (HBM GB/s); E+dE/dpsi time",
        "value": total / (ms_step / 1000.0),
        "unit": "candidates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {
            "workload": f"{wl.name}: n_orb={wl.n_orb} {wl.n_alpha}a+{wl.n_beta}b rank={wl.rank} n_sel={n_sel} W={W}; "
                        f"one mini-batch of the first {n_src} sources ({total} candidates) streamed through the "
                        f"device pool in chunks of {chunk} into S (sci_stream_dedup) + E and dE/dpsi over S",
            "n_candidates": total, "n_unique_union": n_union, "chunk": chunk,
            "n_chunks": -(-total // chunk),
            "stage_ms": {"gen_dedup_stream": s_ms,
                         ("energy_grad" if args.energy_after else "energy_grad_after_stream"): stages["energy"]},
            "energy_placement": "after the stream" if args.energy_after else "beside the stream (own stream)",
            "candidates_per_s_stream": total / (s_ms / 1000.0),
            "energy": float(energy.item()),
            "device_bytes": {"pool_and_workspace": ws.numel(), "set_buffers": 2 * cap * kb, "peak_allocated": peak},
        },
        "kernels": per_kernel,
    }
    if sizes is not None:
        assert sizes[-1]["m1"] == n_union, "streamed union differs from the chunk-by-chunk merges"
        algo = large_algo(sizes, n_src, W)
        res["roofline"] = roofline(per_kernel, algo, W, "large")
        res["kernel_rates"] = kernel_rates(per_kernel, algo)
        res["config"]["chunk_sizes"] = sizes
        res["gen_dedup_algorithmic"] = {
            "bytes_per_step": gen_bytes + dedup_lb, "stage_ms": s_ms,
            "achieved": (gen_bytes + dedup_lb) / (s_ms / 1000.0) / 1e9, "unit": "GB/s",
            "frac_of_peak": (gen_bytes + dedup_lb) / (s_ms / 1000.0) / 1e9 / HBM_PEAK_GBS,
            "definition": "generation (keys + H_ij written, sources read) + dedup lower bound "
                          "(every candidate key read once and written once), over the stream stage time"}
        res["gen_dedup_hbm"] = gen_dedup_traffic(per_kernel, W, s_ms, copy_gbps, "large")
    res.update(out)
    del ws, set_a, set_b
    torch.cuda.empty_cache()
    return res, (ham, sel, psi, sysm)


# ---------------------------------------------------------------------------
# extras
# ---------------------------------------------------------------------------

def medium_step(args, torch, sci, si, copy_gbps):
    """The medium workload's whole step (all 100,000 sources): generation of every coupled
    determinant (2.51e9, dense, one launch), dedup-merge into S, energy + gradient."""
    wl = si.WORKLOADS["medium"]
    sysm = si.make_system(wl)
    dev = torch.device("cuda", 0)
    ham = sci.Ham(wl.n_orb, wl.n_alpha, wl.n_beta, sysm.h1, sysm.eri)
    n_sel = sysm.dets.shape[0]
    n_cand = n_sel * ham.n_coupled
    W = ham.W
    sel = sci.keys_to_device(sysm.dets)
    psi = torch.from_numpy(sysm.psi).to(dev)
    keys = torch.empty((n_cand, W), dtype=torch.int64, device=dev)
    hij = torch.empty(n_cand, dtype=torch.float64, device=dev)
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

    def step(ev):
        ev[0].record(stream)
        sci.sci_gen_coupled(ham, sel, n_sel, 0, n_cand, -1.0, keys, hij, None, n_cand, None, flags, stream)
        ev[1].record(stream)
        sci.sci_dedup_merge(W, keys, n_cand, sel, n_set_in, set_out, n_set_out, set_cap, None, None, 0,
                            ws_d, ws_d.numel(), flags, stream)
        ev[2].record(stream)
        sci.sci_energy(ham, sel, n_sel, psi, energy, hpsi, grad, ws_e, ws_e.numel(), flags, stream)
        ev[3].record(stream)

    warm = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    for _ in range(2):
        step(warm)
    torch.cuda.synchronize()
    sci.check_flags(flags, "medium warmup")
    # distinct candidate keys (a merge into nothing, untimed): the bucket kernel's output size
    n_zero = torch.zeros(1, dtype=torch.int64, device=dev)
    sci.sci_dedup_merge(W, keys, n_cand, None, None, set_out, n_zero, set_cap, None, None, 0, ws_d, ws_d.numel(),
                        flags, stream)
    torch.cuda.synchronize()
    n_distinct = int(n_zero.item())
    step(warm)  # the union again (set_out was used above)
    torch.cuda.synchronize()
    n_union = int(n_set_out.item())
    ms_step, st, per_kernel = timed_steps(torch, sci, step, 10, ["gen", "dedup", "energy"])
    sci.check_flags(flags, "medium")
    kb = 8 * W
    gen_bytes = n_cand * (kb + 8) + n_sel * kb
    dedup_lb = 2 * n_cand * kb
    n_novel = n_union - n_sel
    table = {"gen_kernel": gen_bytes, "hist_kernel": n_cand * kb, "scatter_kernel": 2 * n_cand * kb,
             "bucket_kernel": (n_cand + n_sel + n_novel) * kb, "emit_kernel": (n_novel + n_sel + n_union) * kb}
    algo = lambda name: table.get(family(name))
    res = {
        "workload": f"{wl.name}: n_orb={wl.n_orb} {wl.n_alpha}a+{wl.n_beta}b rank={wl.rank} n_sel={n_sel} W={W}; "
                    f"full generation (one launch) + dedup-merge into S + E and dE/dpsi",
        "n_candidates": n_cand, "n_distinct_candidates": n_distinct, "n_unique_union": n_union,
        "ms_per_step": ms_step, "candidates_per_s": n_cand / (ms_step / 1000.0), "stage_ms": st,
        "gen_candidates_per_s": n_cand / (st["gen"] / 1000.0), "dedup_keys_per_s": n_cand / (st["dedup"] / 1000.0),
        "roofline": roofline(per_kernel, algo, W, "medium"),
        "kernel_rates": kernel_rates(per_kernel, algo),
        "gen_dedup_algorithmic": {
            "bytes_per_step": gen_bytes + dedup_lb, "achieved": (gen_bytes + dedup_lb) / ((st["gen"] + st["dedup"]) / 1000.0) / 1e9,
            "frac_of_peak": (gen_bytes + dedup_lb) / ((st["gen"] + st["dedup"]) / 1000.0) / 1e9 / HBM_PEAK_GBS},
        "gen_dedup_hbm": gen_dedup_traffic(per_kernel, W, st["gen"] + st["dedup"], copy_gbps, "medium"),
        "energy": float(energy.item()),
        "kernels": per_kernel,
    }
    ctx = dict(ham=ham, sel=sel, n_sel=n_sel, keys=keys, hij=hij, n_cand=n_cand, set_out=set_out,
               n_set_out=n_set_out, n_union=n_union, ws_d=ws_d, gen_ms=st["gen"], sysm=sysm)
    return res, ctx


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


def whole_extras(args, torch, sci, ham, sel):
    """All selected determinants of the large workload as sources (7.2e10 candidates)
    streamed through the device pool into one set on one GPU (sci_stream_dedup): time
    of one pass, union size, peak device memory."""
    dev = sel.device
    W = ham.W
    n_sel = sel.shape[0]
    total = n_sel * ham.n_coupled
    # the fewest equal chunks of at most 1.6e9 candidates: set buffers for the 5.5e9-key
    # union take 179 GB, the pool and dedup workspace of such a chunk about 105 GB
    chunk, _ = equal_chunks(total, WHOLE_CHUNK_MAX)
    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats(dev)
    ws_bytes = sci.sci_stream_workspace_bytes(ham, chunk)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    free_bytes = torch.cuda.mem_get_info(dev)[0]
    # the union lies in the determinants of excitation level <= 4 of the reference
    # (5.55e9 for this system), so larger set buffers would stay unused
    cap = int(min(total + n_sel, 5_600_000_000, (free_bytes - (8 << 30)) // (2 * W * 8)))
    set_a = torch.empty((cap, W), dtype=torch.int64, device=dev)
    set_b = torch.empty_like(set_a)
    n_in = torch.tensor([n_sel], dtype=torch.int64, device=dev)
    n_out = torch.zeros(1, dtype=torch.int64, device=dev)
    flags = sci.new_flags(dev)
    cur = torch.cuda.current_stream()
    dd = torch.cuda.Stream()
    fb = [False]

    def run():
        fb[0] = sci.sci_stream_dedup(ham, sel, n_sel, 0, total, chunk, sel, n_in, set_a, set_b, cap, n_out,
                                     ws, ws.numel(), flags, cur, dd)
        cur.wait_stream(dd)

    t_ms = _median_ms(run, 1, torch)
    sci.check_flags(flags, "whole selected space")
    n_union = int(n_out.item())
    peak = torch.cuda.max_memory_allocated(dev)
    res = set_b if fb[0] else set_a
    del ws, set_a, set_b
    torch.cuda.empty_cache()
    # strictly ascending at full size, checked on the device in slices
    ok = True
    for a0 in range(0, n_union - 1, 1 << 30):
        b0 = min(a0 + (1 << 30) + 1, n_union)
        hi, lo = res[a0:b0, 1], res[a0:b0, 0] ^ (-(1 << 63))
        up = (hi[1:] > hi[:-1]) | ((hi[1:] == hi[:-1]) & (lo[1:] > lo[:-1]))
        ok = ok and bool(up.all())
        del hi, lo, up
    out = {"workload": f"large: all {n_sel} selected determinants as sources ({total} candidates) streamed in "
                       f"chunks of {chunk} into one set (sci_stream_dedup), one pass",
           "n_candidates": total, "chunk": chunk, "n_chunks": -(-total // chunk), "ms": t_ms,
           "candidates_per_s": total / (t_ms / 1000.0), "n_unique_union": n_union, "union_ascending": ok,
           "redundancy": total / n_union, "set_capacity": cap,
           "device_bytes": {"pool_and_workspace": ws_bytes, "set_buffers": 2 * cap * W * 8,
                            "peak_allocated": peak}}
    del res
    torch.cuda.empty_cache()
    return out


def energy_methods(torch, sci, ham, sel, psi, reps):
    """E + dE/dpsi with each membership method (pair screening, enumeration + search of
    S) and the method the cost model picks for this shape."""
    n_sel = sel.shape[0]
    out = {"n_sel": n_sel, "n_coupled": ham.n_coupled,
           "auto": {sci.ENERGY_PAIRS: "pairs", sci.ENERGY_ENUM: "enum"}[sci.sci_energy_method(ham, n_sel)]}
    for name, m in (("pairs", sci.ENERGY_PAIRS), ("enum", sci.ENERGY_ENUM)):
        fn = lambda: sci.energy(ham, sel, psi, want_hpsi=False, want_grad=True, method=m)
        fn()
        torch.cuda.synchronize()
        out[f"{name}_ms"] = _median_ms(fn, reps, torch)
    out["faster"] = "pairs" if out["pairs_ms"] <= out["enum_ms"] else "enum"
    return out


def energy_extras(torch, sci, si, ham, sel, psi):
    """E and E + dE/dpsi over all of the large S: the plain entry point and the autograd path
    (forward + backward, which recomputes H psi); both membership methods on the large S
    and on a small-orbital system (n_orb=10, 4a+4b, 17,000 determinants)."""
    n_sel = sel.shape[0]
    e_ms = _median_ms(lambda: sci.energy(ham, sel, psi, want_hpsi=False, want_grad=False), 5, torch)
    eg_ms = _median_ms(lambda: sci.energy(ham, sel, psi, want_hpsi=False, want_grad=True), 5, torch)
    methods = {"large": energy_methods(torch, sci, ham, sel, psi, 1)}
    wl = si.small_workload(10, 4, 4, n_sel=17_000, selection="levels")
    sm = si.make_system(wl)
    hs = sci.Ham(sm.n_orb, sm.n_alpha, sm.n_beta, sm.h1, sm.eri)
    methods["small_10_4_4"] = energy_methods(torch, sci, hs, sci.keys_to_device(sm.dets),
                                             torch.from_numpy(sm.psi).to(sel.device), 5)

    def auto():
        p = psi.clone().requires_grad_(True)
        e = sci.SciEnergy.apply(p, ham, sel)
        e.backward()

    ag_ms = _median_ms(auto, 5, torch)
    return {"workload": f"large: E over all {n_sel} selected determinants", "n_sel": n_sel,
            "energy_ms": e_ms, "energy_grad_ms": eg_ms, "autograd_fwd_bwd_ms": ag_ms, "methods": methods}


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


# ---------------------------------------------------------------------------
# CPU baseline: the oracle as it stands on a bounded sample
# ---------------------------------------------------------------------------

DEFAULT_CPU_SOURCES = {"large": 480, "medium": 8000, "tiny": 200}
DEFAULT_SINGLE_SOURCES = {"large": 16, "medium": 500, "tiny": 200}


def cpu_baseline(sysm, n_src):
    """The oracle, as it stands, on the first n_src sources: generation, dedup of their
    candidates into S, and H psi for the same rows (enumeration + search in S)."""
    import oracle
    wl = sysm.workload
    n_src = min(n_src, sysm.dets.shape[0])
    dets = sysm.dets[:n_src]
    t0 = time.perf_counter()
    keys, _, _ = oracle.gen_coupled(wl.n_orb, wl.n_alpha, wl.n_beta, sysm.h1, sysm.eri, dets)
    oracle.dedup_merge(wl.W, keys, sysm.dets)
    oracle.hpsi_rows(wl.n_orb, wl.n_alpha, wl.n_beta, sysm.h1, sysm.eri, sysm.dets, sysm.psi,
                     np.arange(n_src, dtype=np.int64))
    dt = time.perf_counter() - t0
    n_cand = keys.shape[0]
    return {"value": n_cand / dt, "unit": "candidates/s", "cores": oracle.num_threads(), "kind": "oracle",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "sample": f"{wl.name}: first {n_src} of {sysm.dets.shape[0]} sources: generation ({n_cand} candidates), "
                      f"dedup into S, H psi rows; {dt:.1f} s"}


def single_thread_baseline(workload, n_src):
    """The oracle on one host thread, timed in a child process (OpenMP fixes its thread
    count when the library loads); the child runs only the CPU oracle."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-only", "--workload", workload,
           "--cpu-sources", str(n_src)]
    r = subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=900)
    if r.returncode != 0:
        return {"error": r.stderr[-300:]}
    return json.loads(r.stdout.strip().splitlines()[-1])


def main():
    args = parse()
    if args.record_traffic:
        record_traffic(*args.record_traffic)
        return
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    import sci_inputs as si
    if args.cpu_only:
        n = args.cpu_sources or DEFAULT_CPU_SOURCES[args.workload]
        print(json.dumps(cpu_baseline(si.make_system(si.WORKLOADS[args.workload]), n)), flush=True)
        return
    import torch

    import paper_2604_15768_amd as sci

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.calib_copy_gib > 0:
        nel = int(args.calib_copy_gib * 2**30) // 8
        a = torch.empty(nel, dtype=torch.int64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        torch.cuda.empty_cache()
    # bandwidth a plain device copy reaches here (read + write), the practical ceiling
    copy_gbps = copy_bandwidth(torch, dev)

    extras = set() if (args.no_extras or args.counters) else set(args.extras.split(","))
    ctx_large = None
    if args.workload == "large":
        result, ctx_large = large_headline(args, torch, sci, si, copy_gbps)
        head_sysm = ctx_large[3]
    else:
        m, ctx = medium_step(args, torch, sci, si, copy_gbps) if args.workload == "medium" else (None, None)
        if m is None:
            raise SystemExit("--workload tiny is for --cpu-only")
        result = {"metric": "coupled dets+H_ij/s and dedup keys/s (HBM GB/s); E+dE/dpsi time",
                  "value": m["candidates_per_s"], "unit": "candidates/s", "n_gpus": 1, "steps": 10, "warmup": 2,
                  "ms_per_step": m["ms_per_step"], "higher_is_better": True, "scaling": "weak",
                  "vs_baseline": None, "dtype": "f64", "data": "synthetic",
                  "config": {"workload": m["workload"], "n_candidates": m["n_candidates"]},
                  "roofline": m["roofline"], "medium": m}
        head_sysm = ctx["sysm"]
        extras.discard("medium")
    result["copy_GBps"] = copy_gbps
    result["extras"] = {}
    if "energy" in extras and ctx_large is not None:
        ham, sel, psi, _ = ctx_large
        result["extras"]["energy_grad_large"] = energy_extras(torch, sci, si, ham, sel, psi)
    if "whole" in extras and ctx_large is not None:
        ham, sel, _, _ = ctx_large
        result["extras"]["large_whole_stream"] = whole_extras(args, torch, sci, ham, sel)
    ctx_large = None
    torch.cuda.empty_cache()
    if extras & {"medium", "select", "screened"}:
        m, ctx = medium_step(args, torch, sci, si, copy_gbps)
        result["extras"]["medium_step"] = m
        if "select" in extras:
            result["extras"]["reverse_index_topk"] = select_extras(
                torch, sci, ctx["keys"], ctx["n_cand"], ctx["set_out"], ctx["n_set_out"], ctx["n_union"],
                ctx["sel"], ctx["n_sel"], ctx["ham"].W, ctx["ws_d"])
        if "screened" in extras:
            result["extras"]["screened_generation"] = screened_extras(
                torch, sci, ctx["ham"], ctx["sel"], ctx["n_sel"], ctx["n_cand"], ctx["keys"], ctx["hij"],
                ctx["gen_ms"])
        if args.medium_cpu_sources > 0 and not args.no_cpu_baseline:
            m["cpu_baseline"] = cpu_baseline(ctx["sysm"], args.medium_cpu_sources)
        ctx = None
        torch.cuda.empty_cache()
    if "batch" in extras:
        bg, be = batch_extras(args, torch, sci, si)
        result["extras"].update({"batched_generation": bg, "batched_energy": be})
    if not args.no_cpu_baseline and not args.counters:
        n = args.cpu_sources or DEFAULT_CPU_SOURCES[args.workload]
        result["cpu_baseline"] = cpu_baseline(head_sysm, n)
        n1 = args.cpu_single_sources if args.cpu_single_sources >= 0 else DEFAULT_SINGLE_SOURCES[args.workload]
        if n1 > 0:
            result["cpu_baseline"]["single_thread"] = single_thread_baseline(args.workload, n1)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
