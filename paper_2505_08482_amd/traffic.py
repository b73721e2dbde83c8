"""Measured HBM traffic of the fused passes at the throughput workload
(512 x 512, K = 8): writes ``traffic.json`` next to this file, which
``bench.py`` reports as ``roofline.traffic`` while the kernel sources still
hash to the digest stored with the readings.

    python -m paper_2505_08482_amd.traffic [--work DIR] [--out FILE]

Four rocprofv3 counter runs, each in a process of its own (FETCH_SIZE and
WRITE_SIZE, in KiB per dispatch, cannot share a run):

* calibration: a device copy of 2^28 float32 (1 GiB read, 1 GiB written);
  the scale of each counter is the known byte count over its reading;
* the benchmark on a short time axis (the per-dispatch readings of a pass do
  not depend on the number of time samples): the average reading of every
  pass kernel, times the counter's scale, is its measured bytes per launch.

rocprofv3 runs as a child process; this process never touches the GPU.
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import re
import subprocess
import sys
import tempfile
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
OUT = os.path.join(HERE, "traffic.json")
WORKLOAD = "w1_512x512_K8_nt4000"
BENCH = [sys.executable, os.path.join(ROOT, "bench.py"), "--nt", "100", "--steps", "1", "--warmup", "0",
         "--no-cpu", "--no-extras", "--tile", "0"]
COPY = [sys.executable, "-c",
        "import torch; x = torch.ones(1 << 28, device='cuda'); y = torch.empty_like(x); "
        "torch.cuda.synchronize(); [y.copy_(x) for _ in range(4)]; torch.cuda.synchronize()"]
COPY_KIB = (1 << 28) * 4 / 1024.0

# fused pass kinds by kernel name (power-of-two kernels at 512)
PASS_OF = [
    (r"k_col<512, 0\b", "fwd_col_grad"), (r"k_fwd_u<512>", "fwd_row_u"), (r"k_col<512, 2\b", "fwd_col_div"),
    (r"k_fwd_rho<512>", "fwd_row_rho"), (r"k_col<512, 3\b", "adj_col_summ"), (r"k_adj_rho<512,", "adj_row_rho"),
    (r"k_col<512, 1\b", "adj_col_grad"), (r"k_adj_u<512>", "adj_row_u"),
]


def counter_run(counter: str, cmd, work: str, tag: str):
    """Per-kernel (dispatch count, mean reading) of one counter run."""
    d = os.path.join(work, f"{tag}_{counter}")
    full = ["timeout", "-s", "KILL", "180", "rocprofv3", "--pmc", counter, "-d", d, "-o", "run",
            "--output-format", "csv", "--"] + cmd
    print("[traffic] " + " ".join(full), flush=True)
    with open(d + ".log", "w") as log:
        subprocess.run(full, check=True, stdout=log, stderr=subprocess.STDOUT, cwd=ROOT)
    return read_counter(d, counter)


def read_counter(d: str, counter: str):
    """Per-kernel (dispatch count, mean reading) of ``counter`` in the
    rocprofv3 counter-collection CSV files under folder ``d``."""
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise RuntimeError(f"no counter file under {d}")
    acc = defaultdict(list)
    for f in files:
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] == counter:
                    acc[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return {k: (len(v), sum(v) / len(v)) for k, v in acc.items()}


def pass_readings(fetch, write):
    """The fused passes' readings (kernel name, dispatches, mean FETCH_SIZE
    and WRITE_SIZE in KiB) from the per-kernel results of the two runs."""
    passes = {}
    for pattern, kind in PASS_OF:
        for kname, (n, f) in fetch.items():
            if re.search(pattern, kname) and kname in write:
                passes[kind] = {"kernel": kname.split("(")[0], "dispatches": n, "fetch_kib": round(f, 1),
                                "write_kib": round(write[kname][1], 1)}
                break
    missing = [k for _, k in PASS_OF if k not in passes]
    if missing:
        raise RuntimeError(f"pass kernels not found in the counter runs: {missing}")
    return passes


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--work", default=os.path.join(tempfile.gettempdir(), "pat_traffic"),
                    help="folder for the counter runs' raw output")
    ap.add_argument("--out", default=OUT)
    a = ap.parse_args(argv)
    os.makedirs(a.work, exist_ok=True)
    sys.path.insert(0, ROOT)
    import bench  # noqa: E402  (the digest of the kernel sources)

    scale = {}
    for counter, expect in (("FETCH_SIZE", COPY_KIB), ("WRITE_SIZE", COPY_KIB)):
        runs = counter_run(counter, COPY, a.work, "copy")
        # the copy's kernel (the fill that makes the source writes the same 1 GiB)
        copies = {k: v for k, v in runs.items() if "copy" in k.lower()} or runs
        name, (n, val) = max(copies.items(), key=lambda kv: kv[1][1])
        scale[counter] = expect / val
        print(f"[traffic] calibration {counter}: {name} x{n}, {val:.1f} KiB -> scale {scale[counter]:.4f}",
              flush=True)
    readings = {c: counter_run(c, BENCH, a.work, "bench") for c in ("FETCH_SIZE", "WRITE_SIZE")}
    passes = pass_readings(readings["FETCH_SIZE"], readings["WRITE_SIZE"])
    out = {"workload": WORKLOAD, "source_sha256": bench.kernel_source_digest(),
           "fetch_scale": round(scale["FETCH_SIZE"], 4), "write_scale": round(scale["WRITE_SIZE"], 4),
           "calibration": "device copy of 2^28 float32 (1 GiB read, 1 GiB written), largest dispatch",
           "command": "rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) -d <dir> -o run --output-format csv -- "
                      + " ".join(["python3", "bench.py"] + BENCH[2:]),
           "passes": passes}
    with open(a.out, "w") as f:
        json.dump(out, f, indent=1)
    print(f"[traffic] wrote {a.out}", flush=True)
    for kind, e in passes.items():
        mb = (e["fetch_kib"] * scale["FETCH_SIZE"] + e["write_kib"] * scale["WRITE_SIZE"]) * 1024 / 1e6
        print(f"[traffic] {kind:13s} {e['kernel']:40s} fetch {e['fetch_kib']:9.1f} KiB write "
              f"{e['write_kib']:9.1f} KiB -> {mb:.2f} MB/launch", flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
