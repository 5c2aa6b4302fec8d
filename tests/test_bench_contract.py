"""CPU checks of bench.py's contract: one GPU only, the counter summary that
feeds the roofline's traffic figure, and the kernel-source fingerprint that
decides whether that figure still applies."""
import csv
import glob
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def _write_counter_csv(path, counter, rows):
    fields = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=fields)
        w.writeheader()
        for name, value in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_counter_summary_scales_by_the_calibration_copy(tmp_path):
    """Counters read in KiB per dispatch; each is divided by its reading per byte
    for the 1 GiB calibration copy, and averaged over a kernel's dispatches."""
    gib = float(1 << 30)
    # the copy's FETCH_SIZE reads half its bytes, WRITE_SIZE all of them
    fetch = [("__amd_rocclr_copyBuffer", gib / 2 / 1024),
             ("void stig::k<1>(double const*)", 100.0), ("void stig::k<1>(double const*)", 300.0)]
    write = [("__amd_rocclr_copyBuffer", gib / 1024),
             ("void stig::k<1>(double const*)", 50.0), ("void stig::k<1>(double const*)", 50.0)]
    fp, wp = tmp_path / "f.csv", tmp_path / "w.csv"
    _write_counter_csv(fp, "FETCH_SIZE", fetch)
    _write_counter_csv(wp, "WRITE_SIZE", write)
    out = bench.summarize_counters(str(fp), str(wp), copy_bytes=gib)
    assert abs(out["fetch_scale"] - 0.5) < 1e-12 and abs(out["write_scale"] - 1.0) < 1e-12
    k = out["kernels"]["stig::k<1>"]
    assert k["dispatches"] == 2
    assert abs(k["fetch_bytes"] - 200.0 * 1024 / 0.5) < 1e-6
    assert abs(k["write_bytes"] - 50.0 * 1024) < 1e-6
    assert out["fingerprint"] == bench.kernel_fingerprint()


def test_fingerprint_covers_every_kernel_source():
    csrc = os.path.join(ROOT, "paper_1909_07309_amd", "csrc")
    sources = {os.path.relpath(p, ROOT) for p in glob.glob(os.path.join(csrc, "kernels_*.h"))}
    sources.add(os.path.relpath(os.path.join(csrc, "stig.hip"), ROOT))
    assert sources <= set(bench.KERNEL_SOURCES), sources - set(bench.KERNEL_SOURCES)
