"""Host logic of the measurement and tuning tools (no GPU): the one-GPU guard
of the bench, its byte accounting, the gating of stored counter readings by
the kernel sources they were taken on, the parsing of counter files, and the
committed launch table."""
import csv
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2505_08482_amd import traffic  # noqa: E402


@pytest.mark.parametrize("args,env", [(["--gpus", "2"], {}), (["--gpus", "8"], {}), ([], {"WORLD_SIZE": "2"})])
def test_bench_runs_on_one_gpu_only(args, env):
    """More than one GPU is refused before anything touches a device: exit 2,
    a message on stderr and no JSON line on stdout."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args, capture_output=True, text=True,
                       timeout=300, cwd=ROOT, env=dict(os.environ, **env))
    assert r.returncode == 2, r.stderr
    assert "one GPU only" in r.stderr
    assert r.stdout.strip() == ""


def test_pass_byte_accounting():
    """Per-pass bytes per grid point add up to the step figure; the dataset
    grouping of the adjoint density pass changes only its g_c term; with one
    dataset nothing is amortised."""
    alg, moved = bench.pass_bytes(8), bench.pass_bytes(8, moved=True)
    assert set(alg) == set(traffic.PASS_OF[i][1] for i in range(len(traffic.PASS_OF)))
    assert sum(alg.values()) == pytest.approx(186.0) and bench.STEP_BYTES == pytest.approx(186.0)
    # g_c slice: read and written once per time step (8 B) for all K, or once per group of 4 datasets
    assert moved["adj_row_rho"] - alg["adj_row_rho"] == pytest.approx(8 / 4 - 8 / 8)
    assert all(moved[k] == alg[k] for k in alg if k != "adj_row_rho")
    one = bench.pass_bytes(1)
    assert one["fwd_row_rho"] == pytest.approx(32 + 4) and one["adj_row_rho"] == pytest.approx(32 + 4 + 8)
    assert bench.pass_bytes(1, moved=True) == one
    # column passes move half spectra only (4 B/pt each): 1 read + 2 written, 2 + 2, 2 + 1, 2 + 2
    assert (alg["fwd_col_grad"], alg["fwd_col_div"], alg["adj_col_summ"], alg["adj_col_grad"]) == (12, 16, 12, 16)


def _copy_sources(dst):
    os.makedirs(os.path.join(dst, "csrc"))
    for name in bench.KERNEL_SOURCES:
        shutil.copy(os.path.join(os.path.dirname(bench.TRAFFIC_FILE), "csrc", name), os.path.join(dst, "csrc", name))


def test_committed_counter_readings_match_the_committed_kernels():
    """The stored readings were taken on the kernel sources as committed, cover
    every pass, and each is within 0-30 % above the pass's algorithmic bytes
    (no pass re-reads its data)."""
    with open(bench.TRAFFIC_FILE) as f:
        t = json.load(f)
    assert t["source_sha256"] == bench.kernel_source_digest()
    assert set(t["passes"]) == set(bench.PASS_BYTES)
    moved = bench.pass_bytes(8, moved=True)
    for kind, e in t["passes"].items():
        got = bench.measured_traffic(kind, t["workload"])
        assert got == pytest.approx(e["fetch_kib"] * 1024 * t["fetch_scale"] + e["write_kib"] * 1024 * t["write_scale"])
        ratio = got / (moved[kind] * 512 * 512 * 8)
        assert 0.97 <= ratio <= 1.3, (kind, ratio)
    assert bench.measured_traffic("adj_row_rho", "another_workload") is None
    assert bench.measured_traffic("no_such_pass", t["workload"]) is None


def test_counter_readings_are_dropped_once_a_kernel_source_changes(tmp_path, monkeypatch):
    with open(bench.TRAFFIC_FILE) as f:
        t = json.load(f)
    _copy_sources(tmp_path)
    rec = tmp_path / "traffic.json"
    rec.write_text(json.dumps(t))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(rec))
    assert bench.kernel_source_digest() == t["source_sha256"]
    assert bench.measured_traffic("fwd_row_u", t["workload"]) is not None
    with open(tmp_path / "csrc" / bench.KERNEL_SOURCES[0], "a") as f:
        f.write("\n// edited\n")
    assert bench.measured_traffic("fwd_row_u", t["workload"]) is None
    rec.write_text("not json")
    assert bench.measured_traffic("fwd_row_u", t["workload"]) is None


def _counter_csv(path, rows):
    path.parent.mkdir(parents=True, exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (k, c, v) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": k, "Grid_Size": 512, "Counter_Name": c, "Counter_Value": v})


def test_counter_file_parsing_and_pass_matching(tmp_path):
    """Means per kernel over dispatches and files; every pass kind found by
    its own kernel name only (the column passes differ by their mode)."""
    names = {
        "fwd_col_grad": "void pat::fast::k_col<512, 0, 4, false>(pat::Tables, float2*)",
        "fwd_row_u": "void pat::fast::k_fwd_u<512>(pat::Tables)",
        "fwd_col_div": "void pat::fast::k_col<512, 2, 4, false>(pat::Tables, float2*)",
        "fwd_row_rho": "void pat::fast::k_fwd_rho<512>(pat::Tables)",
        "adj_col_summ": "void pat::fast::k_col<512, 3, 4, false>(pat::Tables, float2*)",
        "adj_row_rho": "void pat::fast::k_adj_rho<512, 4>(pat::Tables)",
        "adj_col_grad": "void pat::fast::k_col<512, 1, 4, false>(pat::Tables, float2*)",
        "adj_row_u": "void pat::fast::k_adj_u<512>(pat::Tables)",
    }
    fetch_rows, write_rows = [], []
    for j, (kind, k) in enumerate(names.items()):
        for d in range(3):
            fetch_rows.append((k, "FETCH_SIZE", 1000.0 * (j + 1) + d))      # mean 1000 (j+1) + 1
            write_rows.append((k, "WRITE_SIZE", 10.0 * (j + 1)))
        fetch_rows.append((k, "OTHER", 5.0))
    fetch_rows.append(("void pat::fast::k_col<128, 0, 4, false>(pat::Tables)", "FETCH_SIZE", 1.0))
    # readings split over two files, as rocprofv3 writes one per agent or process
    _counter_csv(tmp_path / "f" / "a" / "run_counter_collection.csv", fetch_rows[: len(fetch_rows) // 2])
    _counter_csv(tmp_path / "f" / "b" / "run_counter_collection.csv", fetch_rows[len(fetch_rows) // 2:])
    _counter_csv(tmp_path / "w" / "run_counter_collection.csv", write_rows)
    fetch = traffic.read_counter(str(tmp_path / "f"), "FETCH_SIZE")
    write = traffic.read_counter(str(tmp_path / "w"), "WRITE_SIZE")
    assert fetch[names["adj_row_rho"]] == (3, pytest.approx(6001.0))
    passes = traffic.pass_readings(fetch, write)
    assert set(passes) == set(names)
    for j, (kind, k) in enumerate(names.items()):
        e = passes[kind]
        assert e["kernel"] == k.split("(")[0]
        assert (e["dispatches"], e["fetch_kib"], e["write_kib"]) == (3, 1000.0 * (j + 1) + 1, 10.0 * (j + 1))
    del write[names["adj_col_summ"]]
    with pytest.raises(RuntimeError, match="adj_col_summ"):
        traffic.pass_readings(fetch, write)
    with pytest.raises(RuntimeError):
        traffic.read_counter(str(tmp_path / "empty"), "FETCH_SIZE")


def test_committed_launch_table(tmp_path, monkeypatch):
    """Every committed choice is one of the candidates, and the lookup returns
    it without measuring (no GPU needed) on the architecture it was taken on."""
    from paper_2505_08482_amd import tune
    tab = tune._table()
    assert tab
    monkeypatch.setattr(tune, "_arch", lambda: "gfx950")
    monkeypatch.setenv("PAT_TUNE_CACHE", str(tmp_path / "cache.json"))
    for key, v in tab.items():
        kind, arch, n, K = key.split("/")
        assert kind == "launch" and arch == "gfx950"
        assert (v["tile"], v["seq"]) in tune.CANDIDATES
        assert tune.launch_for(int(n), int(K)) == {"tile": v["tile"], "seq": v["seq"]}
    assert not (tmp_path / "cache.json").exists()


def test_cpu_thread_budget(monkeypatch):
    """The CPU baseline's thread count: the affinity set, capped by the thread
    budget the host exports."""
    n = len(os.sched_getaffinity(0))
    monkeypatch.delenv("OMP_NUM_THREADS", raising=False)
    assert bench.cpu_cores() == n
    monkeypatch.setenv("OMP_NUM_THREADS", "1")
    assert bench.cpu_cores() == 1
    monkeypatch.setenv("OMP_NUM_THREADS", "not a number")
    assert bench.cpu_cores() == n
