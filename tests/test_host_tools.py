"""Host-side tools: the bench's one-GPU contract and the HBM-traffic table built from rocprofv3
counter CSVs (synthetic CSVs here, in the layout rocprofv3 writes)."""
import csv
import json
import os
import subprocess
import sys

from paper_2112_14640_amd import traffic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WILSON = ("void dirac::(anonymous namespace)::wilson_rows_kernel<3, 1, false, dirac::PrecF32, 0>"
          "(dirac::PrecF32::G const*, dirac::PrecF32::S const*)")
WILSON_DAG = WILSON.replace("1, false,", "1, true,")


def _write(dirname, counter, rows):
    os.makedirs(dirname, exist_ok=True)
    with open(os.path.join(dirname, "bench_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, value in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "exactly one GPU" in r.stderr


def test_traffic_scale_comes_from_the_large_copies_only(tmp_path):
    copy = "__amd_rocclr_copyBuffer"
    # five 512 MiB calibration copies (FETCH reads half, WRITE all of the bytes) and two tiny result copies
    _write(tmp_path / "f", "FETCH_SIZE", [(copy, 262144.0)] * 5 + [(copy, 0.1)] * 2 +
           [(WILSON, 250000.0), (WILSON, 260000.0), (WILSON_DAG, 300000.0)])
    _write(tmp_path / "w", "WRITE_SIZE", [(copy, 524288.0)] * 5 + [(copy, 0.2)] * 2 +
           [(WILSON, 147456.0), (WILSON, 147456.0), (WILSON_DAG, 147456.0)])
    fetch = traffic.counter_means(str(tmp_path / "f"), "FETCH_SIZE")
    write = traffic.counter_means(str(tmp_path / "w"), "WRITE_SIZE")
    assert fetch["copy"] == 262144.0 and write["copy"] == 524288.0
    assert fetch["wilson"] == 255000.0 and fetch["wilson_dagger"] == 300000.0
    out_json, out_txt = tmp_path / "t.json", tmp_path / "t.txt"
    subprocess.run([sys.executable, "-m", "paper_2112_14640_amd.traffic", str(tmp_path / "f"), str(tmp_path / "w"),
                    "--out-json", str(out_json), "--out-txt", str(out_txt)], check=True, cwd=ROOT,
                   capture_output=True, timeout=120)
    table = json.loads(out_json.read_text())
    ent = table["wilson_fp32_16x32_nv12"]
    # FETCH x2, WRITE x1: 255000 KiB read -> 510000 KiB, the 144 MiB output written once
    assert ent["fetch_bytes"] == 2 * 255000 * 1024
    assert ent["write_bytes"] == 147456 * 1024
    assert ent["algorithmic_bytes"] == traffic.algorithmic_bytes("wilson")
    assert ent["source_hash"] == traffic.source_hash(ent["sources"])
    assert "FETCH x2.0000, WRITE x1.0000" in out_txt.read_text()


def test_algorithmic_bytes_per_site():
    vol = 16 * 16 * 16 * 32
    assert traffic.algorithmic_bytes("wilson") == vol * 2592
    assert traffic.algorithmic_bytes("staggered") == vol * 864
    assert traffic.algorithmic_bytes("brillouin") == vol * 5184
