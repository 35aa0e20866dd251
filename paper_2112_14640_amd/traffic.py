"""L2-to-fabric traffic of the stencil launches of bench.py from two rocprofv3 counter runs.

    python -m paper_2112_14640_amd.traffic FETCH_DIR WRITE_DIR [--out-json profiles/traffic.json]
                                          [--out-txt profiles/<name>.txt]

FETCH_DIR and WRITE_DIR are the output directories of

    rocprofv3 --pmc FETCH_SIZE --output-format csv -d FETCH_DIR -o bench -- \
        python3 bench.py --steps 3 --warmup 1 --no-cg --no-cpu --no-scale --ceilings --copy-calibration
    rocprofv3 --pmc WRITE_SIZE --output-format csv -d WRITE_DIR -o bench -- (same command)

FETCH_SIZE and WRITE_SIZE (KiB per dispatch) count the bytes that the L2 caches request from and
write to the data fabric: reads served by the MALL (Infinity Cache) are included, so they bound the
HBM traffic from above.  Each counter is scaled by the ratio of known bytes to its reading for two
kernels whose bytes are exact: a 512 MiB device copy (``--copy-calibration``: torch's copy_, run as
__amd_rocclr_copyBuffer; the largest copyBuffer dispatches, since small result copies run under that
name too) and the row-by-row copy of the measurement library (k_row_gather<1>: every row read once
with the stencils' 16-byte row loads and written once) at the 16^3 x 32 Wilson and staggered site
blocks.  The row-copy factor, taken with the stencils' own access pattern, scales the stencil
launches; the plain-copy factor is printed beside it as a check.  The same run's seven-row gather
probe (k_row_gather<7>) gives the traffic of the stencils' pattern without their arithmetic.

The JSON records, per launch, the scaled bytes next to the algorithmic bytes and a hash of the kernel
sources; bench.py reports the traffic only while the sources still hash to it.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_BYTES = 512 * 2 ** 20
SOURCES = {
    "wilson": "paper_2112_14640_amd/csrc/wilson.hip",
    "staggered": "paper_2112_14640_amd/csrc/staggered.hip",
    "brillouin": "paper_2112_14640_amd/csrc/brillouin.hip",
}
COMMON = ["paper_2112_14640_amd/csrc/common.h", "paper_2112_14640_amd/csrc/tile.h",
          "paper_2112_14640_amd/csrc/kernels.h", "paper_2112_14640_amd/csrc/api.hip"]
KERNEL = re.compile(r"(wilson|staggered|brillouin)\w*kernel<\d+, \d+, (true|false)")
GATHER = re.compile(r"k_row_gather<(\d)>")
# probe shapes of bench.py's ceilings: threads per launch -> (name, vector bytes)
VOL16 = 16 * 16 * 16 * 32
PROBE_SHAPES = {
    8192 * 192: ("wilson_16x32", VOL16 * 1152),
    65536 * 384: ("wilson_32x64", 32 * 32 * 32 * 64 * 1152),
    8192 * 64: ("staggered_16x32", VOL16 * 288),
    221184 * 192: ("staggered_48x96", 48 * 48 * 48 * 96 * 288),
}
VECTOR_BYTES = {name: vec for name, vec in PROBE_SHAPES.values()}


def source_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_means(root, counter):
    """{launch key: mean KiB per dispatch} for one counter run: the stencil launches, 'copy' (the calibration
    copies) and gather<n>_<shape> for the measurement library's row probes."""
    agg = collections.defaultdict(list)
    for f in glob.glob(os.path.join(root, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] != counter:
                continue
            name = r["Kernel_Name"]
            if "copyBuffer" in name:
                key = "copy"
            elif GATHER.search(name):
                shape = PROBE_SHAPES.get(int(r.get("Grid_Size", 0) or 0))
                if not shape:
                    continue
                key = f"gather{GATHER.search(name).group(1)}_{shape[0]}"
            elif "links_kernel<3, HIP_vector_type<float" in name:
                key = "links"
            else:
                m = KERNEL.search(name)
                if not m:
                    continue
                key = m.group(1) + ("_dagger" if m.group(2) == "true" else "")
            agg[key].append(float(r["Counter_Value"]))
    out = {k: sum(v) / len(v) for k, v in agg.items() if k != "copy"}
    if agg.get("copy"):
        top = max(agg["copy"])
        big = [c for c in agg["copy"] if c >= 0.9 * top]
        out["copy"] = sum(big) / len(big)
    return out


def algorithmic_bytes(op, dims=(16, 16, 16, 32), nc=3, nv=12, w_s=4, w_g=4):
    """Compulsory bytes of one FP32 apply: input read once, output written once, links read once; for the
    link build, the links V read once and the 40 stored directions written once."""
    vol = dims[0] * dims[1] * dims[2] * dims[3]
    if op == "links":
        return vol * (4 + 40) * 2 * nc * nc * w_g
    spin = 1 if op == "staggered" else 4
    dirs = 40 if op == "brillouin" else 4
    return vol * (2 * (2 * nc * spin * nv) * w_s + dirs * 2 * nc * nc * w_g)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("fetch_dir")
    ap.add_argument("write_dir")
    ap.add_argument("--out-json", default=os.path.join(ROOT, "profiles", "traffic.json"))
    ap.add_argument("--out-txt", default=None)
    a = ap.parse_args()
    fetch = counter_means(a.fetch_dir, "FETCH_SIZE")
    write = counter_means(a.write_dir, "WRITE_SIZE")
    text = []
    copy_f = COPY_BYTES / (fetch["copy"] * 1024) if "copy" in fetch else None
    copy_w = COPY_BYTES / (write["copy"] * 1024) if "copy" in write else None
    row_f, row_w = [], []
    for shape in ("wilson_16x32", "staggered_16x32"):
        vec = VECTOR_BYTES[shape]
        k = f"gather1_{shape}"
        if k in fetch and k in write:
            row_f.append(vec / (fetch[k] * 1024))
            row_w.append(vec / (write[k] * 1024))
            text.append(f"# row copy {shape}: known {vec / 1e6:.1f} MB read and written; FETCH reads "
                        f"{fetch[k] * 1024 / 1e6:.1f} MB (x{row_f[-1]:.4f}), WRITE {write[k] * 1024 / 1e6:.1f} MB "
                        f"(x{row_w[-1]:.4f})")
    if copy_f:
        text.append(f"# 512 MiB device copy: FETCH x{copy_f:.4f}, WRITE x{copy_w:.4f}")
    f_scale = sum(row_f) / len(row_f) if row_f else copy_f
    w_scale = sum(row_w) / len(row_w) if row_w else copy_w
    basis = "row-copy" if row_f else "512 MiB copy"
    text.insert(0, f"# scale used: FETCH x{f_scale:.4f}, WRITE x{w_scale:.4f} ({basis} calibration)")
    table = {"_about": ("L2-to-fabric bytes per launch (MALL hits included: an upper bound on HBM traffic) from "
                        "rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE (KiB per dispatch), scaled by the ratio of known "
                        f"bytes to the counters' reading for the row-by-row copy probe (FETCH x{f_scale:.4f}, WRITE "
                        f"x{w_scale:.4f}); valid while the listed sources hash to source_hash")}
    for key in ("wilson", "wilson_dagger", "brillouin", "brillouin_dagger", "staggered", "staggered_dagger", "links"):
        if key not in fetch or key not in write:
            continue
        op = key.split("_")[0]
        fb = fetch[key] * 1024 * f_scale
        wb = write[key] * 1024 * w_scale
        alg = algorithmic_bytes(op)
        srcs = [SOURCES["brillouin" if op == "links" else op]] + COMMON
        table[f"{key}_fp32_16x32_nv12" if op != "links" else "links_fp32_16x32"] = {
            "bytes_per_launch": int(round(fb + wb)), "fetch_bytes": int(round(fb)), "write_bytes": int(round(wb)),
            "algorithmic_bytes": alg, "sources": srcs, "source_hash": source_hash(srcs)}
        text.append(f"{key:18s} fetch {fb / 1e6:8.1f} MB  write {wb / 1e6:7.1f} MB  total {(fb + wb) / 1e6:8.1f} MB  "
                    f"algorithmic {alg / 1e6:7.1f} MB  ratio {(fb + wb) / alg:.2f}")
    for shape, vec in VECTOR_BYTES.items():
        k = f"gather7_{shape}"
        if k in fetch and k in write:
            fb, wb = fetch[k] * 1024 * f_scale, write[k] * 1024 * w_scale
            text.append(f"gather7 {shape:16s} fetch {fb / 1e6:8.1f} MB  write {wb / 1e6:7.1f} MB  "
                        f"vector {vec / 1e6:7.1f} MB  fetch/vector {fb / vec:.2f}")
    with open(a.out_json, "w") as f:
        json.dump(table, f, indent=1)
    if a.out_txt:
        with open(a.out_txt, "w") as f:
            f.write("\n".join(text) + "\n")
    print("\n".join(text))


if __name__ == "__main__":
    main()
