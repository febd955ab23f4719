"""Host logic of bench.py that turns counter records into reported figures (no GPU)."""
import importlib.util
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_template_args(bench):
    ta = bench._template_args
    assert ta("void sci::hist_kernel<1, 4096>(sci::LevelArgs)", "hist_kernel") == ["1", "4096"]
    assert ta("(scatter_kernel<W, C::F2>)", "scatter_kernel") == ["W", "C::F2"]
    assert ta("void sci::bucket_kernel<2>(sci::BucketArgs)", "bucket_kernel") == ["2"]
    assert ta("sci::scan_apply_kernel(long*, long const*)", "scan_apply_kernel") == []
    # nested template arguments stay whole
    assert ta("f<Key<2>, 3>(x)", "f") == ["Key<2>", "3"]


@pytest.mark.parametrize("workload,W", [("medium", 1), ("large", 2)])
def test_recorded_traffic_matches_instantiation(bench, workload, W):
    path = os.path.join(ROOT, "profiles", "kernel_traffic.json")
    rec = json.load(open(path))["workloads"][workload]["kernels"]
    fams = {e["family"] for e in rec.values()}
    assert {"gen_kernel", "bucket_kernel", "hist_kernel", "scatter_kernel", "emit_kernel"} <= fams
    # the two levels of the partition are told apart by their fan-out argument
    lvl1 = bench.recorded_traffic("(hist_kernel<W, C::F1>)", W, workload)
    lvl2 = bench.recorded_traffic("(hist_kernel<W, C::F2>)", W, workload)
    if lvl1 is not None and lvl2 is not None:
        names = [n for n, e in rec.items() if e["family"] == "hist_kernel"]
        by_arg = {bench._template_args(n, "hist_kernel")[1]: e for n, e in rec.items() if n in names}
        f2 = "512" if W == 1 else "1024"
        assert lvl1 == pytest.approx(by_arg["4096"]["read_bytes"] + by_arg["4096"]["write_bytes"])
        assert lvl2 == pytest.approx(by_arg[f2]["read_bytes"] + by_arg[f2]["write_bytes"])
    # a kernel without a record, and a width without one, give nothing
    assert bench.recorded_traffic("no_such_kernel<W>", W, workload) is None
    assert bench.recorded_traffic("bucket_kernel<W>", 7, workload) is None


def test_summarize_trace_takes_the_timed_steps(bench, tmp_path, capsys):
    # 2 timed steps of a kernel launched twice per step, after an untimed launch: the
    # summary averages the last 4 dispatches only
    rows = ["Dispatch_Id,Kernel_Name,Start_Timestamp,End_Timestamp"]
    durs = [9_000_000, 1_000_000, 2_000_000, 3_000_000, 4_000_000]
    t = 0
    for i, d in enumerate(durs):
        rows.append(f'{i + 1},"void sci::emit_kernel<2>(sci::EmitArgs)",{t},{t + d}')
        t += d + 10
    csv_path = tmp_path / "trace.csv"
    csv_path.write_text("\n".join(rows) + "\n")
    res = {"metric": "m", "steps": 2, "config": {"workload": "large: W=2"},
           "kernels": {"emit_kernel<W>": {"ms_per_launch": 2.5, "launches_per_step": 2.0}}}
    out_path = tmp_path / "bench.out"
    out_path.write_text("noise\n" + json.dumps(res) + "\n")
    bench.summarize_trace(str(csv_path), str(out_path))
    text = capsys.readouterr().out
    line = [l for l in text.splitlines() if "emit_kernel<2>" in l][0]
    cells = [c.strip() for c in line.strip("|").split("|")]
    assert cells[1] == "4" and float(cells[2]) == pytest.approx(2.5) and float(cells[4]) == pytest.approx(5.0)


def test_recorded_traffic_refuses_changed_source(bench, tmp_path, monkeypatch):
    # a record whose source hash does not match the file is not reported
    fake_root = tmp_path
    (fake_root / "profiles").mkdir()
    (fake_root / "src.hip").write_text("kernel text")
    rec = {"kernels": {"void sci::bucket_kernel<1>(sci::BucketArgs)": {
        "family": "bucket_kernel", "source": "src.hip", "source_sha256": "0" * 64,
        "read_bytes": 1.0, "write_bytes": 2.0}}}
    (fake_root / "profiles" / "kernel_traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "__file__", str(fake_root / "bench.py"))
    assert bench.recorded_traffic("bucket_kernel<W>", 1) is None
    import hashlib
    rec["kernels"]["void sci::bucket_kernel<1>(sci::BucketArgs)"]["source_sha256"] = \
        hashlib.sha256(b"kernel text").hexdigest()
    (fake_root / "profiles" / "kernel_traffic.json").write_text(json.dumps(rec))
    assert bench.recorded_traffic("bucket_kernel<W>", 1) == 3.0


def test_gen_dedup_traffic_sums_per_step(bench, monkeypatch):
    per_kernel = {
        "(gen_kernel<1, true>)": {"ms_per_launch": 10.0, "launches_per_step": 1.0},
        "scan_apply_kernel": {"ms_per_launch": 0.5, "launches_per_step": 4.0},
        "hpsi_kernel<1>": {"ms_per_launch": 3.0, "launches_per_step": 1.0},  # energy stage: left out
        "emit_kernel<W>": {"ms_per_launch": 5.0, "launches_per_step": 1.0},
    }
    table = {"(gen_kernel<1, true>)": 40e9, "scan_apply_kernel": 1e9, "emit_kernel<W>": None}
    monkeypatch.setattr(bench, "recorded_traffic", lambda name, W, *rest: table.get(name))
    r = bench.gen_dedup_traffic(per_kernel, 1, 20.0, 5000.0)
    assert r["bytes_per_step"] == pytest.approx(40e9 + 4e9)
    assert r["achieved"] == pytest.approx(44e9 / 0.020 / 1e9)
    assert r["frac_of_copy"] == pytest.approx(r["achieved"] / 5000.0)
    assert r["time_covered"] == pytest.approx(12.0 / 17.0)
    # nothing recorded: the copy rate is still reported
    monkeypatch.setattr(bench, "recorded_traffic", lambda name, W, *rest: None)
    r0 = bench.gen_dedup_traffic(per_kernel, 1, 20.0, 5000.0)
    assert r0["achieved"] is None and r0["copy_GBps"] == 5000.0 and r0["time_covered"] == 0.0


def test_equal_chunks_of_the_large_streams(bench):
    # the large mini-batch: 32,768 sources x 361,250 candidates in five equal chunks
    total = 32768 * 361250
    chunk, n = bench.equal_chunks(total, bench.LARGE_CHUNK_MAX)
    assert (chunk, n) == (2_367_488_000, 5) and chunk * n == total
    # all 200,000 selected determinants as sources
    whole = 200000 * 361250
    chunk, n = bench.equal_chunks(whole, bench.WHOLE_CHUNK_MAX)
    assert n == 46 and chunk <= bench.WHOLE_CHUNK_MAX and (n - 1) * chunk < whole <= n * chunk
    # exact multiples and a single chunk
    assert bench.equal_chunks(10, 5) == (5, 2)
    assert bench.equal_chunks(3, 5) == (3, 1)
