#!/usr/bin/env python
"""Dirac-apply benchmark on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cg] [--no-cpu]

Workload (one "step"): the Wilson, Brillouin and staggered applies and their adjoints
(six stencil launches) on a 16^3 x 32 lattice, Nc = 3, Nv = 12 right-hand sides, FP32,
near-identity SU(3) links exp(i 0.3 H), m = 0.05, antiperiodic in t, all inputs resident in
HBM.  `value` is the App. E flop count of the six applies divided by the measured step
time.  Four input sets are rotated so that consecutive launches do not find their operands
in the 256 MB Infinity Cache.

Also reported (outside the timed steps): per-kernel durations and rooflines from HIP events
on the launch stream (against the published peaks and against the device's measured copy and
FMA ceilings), the Brillouin link build, the same applies at the large sizes (Wilson 32^3 x 64,
staggered and Brillouin 48^3 x 96, Haar links), the mixed-precision vs FP64 CG time-to-solution
on D_W^dag D_W at 32^3 x 64 (Nv = 12, exp(i 0.5 H) links, m = 0.01, true FP64 relative residual
1e-10), BiCGstab on D_B at 32^3 x 64 (mixed FP64/FP32 and plain FP64, to 1e-8), and the FP64
NumPy oracle timed on the host on a bounded sample (12^3 x 24, same Nc, Nv).
Progress goes to stderr; stdout carries exactly one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# 256 CUs x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz without packed FP32 instructions
FP32_VECTOR_PEAK_TFS = 78.6
FP32_PACKED_PEAK_TFS = 157.3
FP64_VECTOR_PEAK_TFS = 78.6


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def bytes_per_site(op, nc, nv, w_s, w_g):
    """Compulsory HBM bytes per site: input read once, output written once, links read once."""
    spin = 1 if op == "staggered" else 4
    dirs = 40 if op == "brillouin" else 4
    return 2 * (2 * nc * spin * nv) * w_s + dirs * 2 * nc * nc * w_g


def source_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_key, nbytes_alg):
    """HBM traffic per launch from committed PMC counters, if taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        table = json.load(f)
    ent = table.get(kernel_key)
    if not ent or ent.get("source_hash") != source_hash(ent["sources"]):
        return None
    return ent["bytes_per_launch"]


def run_applies(args, torch, dirac, si):
    dev = "cuda:0"
    cfg = si.config("apply_16x32")
    dims, nc, nv, m = cfg["dims"], cfg["nc"], cfg["nv"], cfg["mass"]
    nx, ny, nz, nt = dims
    vol = nx * ny * nz * nt
    gen = torch.Generator(device=dev)
    sets = []
    link_ms = []
    for k in range(args.sets):
        gen.manual_seed(1000 + k)
        U = si.near_identity_su_n_t(gen, (nt, nz, ny, nx, 4), nc, cfg["spread"], dev, torch.complex64)
        s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s0.record()
        W = dirac.brillouin_links(U)
        s1.record()
        torch.cuda.synchronize()
        link_ms.append(s0.elapsed_time(s1))
        psi = si.complex_gaussian_t(gen, (nt, nz, ny, nx, nc, 4, nv), dev, torch.complex64)
        phi = si.complex_gaussian_t(gen, (nt, nz, ny, nx, nc, nv), dev, torch.complex64)
        sets.append(dict(U=U, W=W, psi=psi, phi=phi, vw=torch.empty_like(psi), vs=torch.empty_like(phi)))
    log(f"[bench] inputs ready: {args.sets} sets at {dims}, Nc={nc}, Nv={nv}")

    kernels = [("wilson", False), ("wilson", True), ("brillouin", False), ("brillouin", True), ("staggered", False),
               ("staggered", True)]

    def launch(s, op, dag):
        fn = dirac.apply_dagger if dag else dirac.apply
        if op == "wilson":
            fn(op, s["U"], s["psi"], m, out=s["vw"])
        elif op == "brillouin":
            fn(op, s["W"], s["psi"], m, out=s["vw"])
        else:
            fn(op, s["U"], s["phi"], m, out=s["vs"])

    for i in range(args.warmup):
        for op, dag in kernels:
            launch(sets[i % args.sets], op, dag)
    torch.cuda.synchronize()
    log(f"[bench] warmup {args.warmup} steps done")

    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in kernels]
          for _ in range(args.steps)]
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record()
    for i in range(args.steps):
        s = sets[i % args.sets]
        for k, (op, dag) in enumerate(kernels):
            ev[i][k][0].record()
            launch(s, op, dag)
            ev[i][k][1].record()
    t1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_step = t0.elapsed_time(t1) / args.steps
    log(f"[bench] timed {args.steps} steps: {ms_step:.3f} ms/step (wall {wall:.2f} s)")

    per = {}
    for k, (op, dag) in enumerate(kernels):
        per[(op, dag)] = sum(ev[i][k][0].elapsed_time(ev[i][k][1]) for i in range(args.steps)) / args.steps
    flops_site = {op: dirac.flops_per_site(op, nc) for op in ("wilson", "brillouin", "staggered")}
    step_flops = sum(flops_site[op] * vol * nv for op, _ in kernels)
    value = step_flops / (ms_step * 1e-3) / 1e9

    rooflines = {}
    for (op, dag), ms in per.items():
        name = op + ("_dagger" if dag else "")
        alg_bytes = bytes_per_site(op, nc, nv, 4, 4) * vol
        flops = flops_site[op] * vol * nv
        gflops = flops / (ms * 1e-3) / 1e9
        if op == "brillouin":
            achieved = flops / (ms * 1e-3) / 1e12
            rl = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP32_VECTOR_PEAK_TFS, "unit": "TFLOP/s",
                  "frac": round(achieved / FP32_VECTOR_PEAK_TFS, 4),
                  "frac_of_packed_fp32_peak": round(achieved / FP32_PACKED_PEAK_TFS, 4)}
        else:
            achieved = alg_bytes / (ms * 1e-3) / 1e9
            rl = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": round(achieved / HBM_PEAK_GBS, 4)}
        tr = measured_traffic(f"{name}_fp32_16x32_nv12", alg_bytes)
        rl["traffic"] = tr
        rl["ms"] = round(ms, 4)
        rl["gflops"] = round(gflops, 1)
        rl["alg_bytes"] = alg_bytes
        rooflines[name] = rl
    dominant = max(per, key=per.get)
    dom_name = dominant[0] + ("_dagger" if dominant[1] else "")
    return dict(value=value, ms_step=ms_step, rooflines=rooflines, dominant=dom_name,
                link_build_ms=round(min(link_ms), 3), dims=dims, nc=nc, nv=nv)


def run_ceilings(torch, dirac):
    """The device's sustained copy bandwidth and non-packed FMA rates (the measured roofline denominators)."""
    n = 2 ** 30 // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    copy = dirac.probe_copy(src, dst, reps=10)
    del src, dst
    torch.cuda.empty_cache()
    out = {"copy_GBps": round(copy / 1e9, 1), "fp32_fma_TFLOPs": round(dirac.probe_fma("fp32") / 1e12, 2),
           "fp64_fma_TFLOPs": round(dirac.probe_fma("fp64") / 1e12, 2),
           "how": "dirac_probe_copy: 1 GiB device copy, 16 B per lane, 10 launches; dirac_probe_fma: 16 independent "
                  "non-packed FMA chains per thread, 16 work-groups of 256 threads per CU"}
    log(f"[bench] ceilings: copy {out['copy_GBps']} GB/s, FMA fp32 {out['fp32_fma_TFLOPs']} / fp64 "
        f"{out['fp64_fma_TFLOPs']} TFLOP/s")
    return out


def time_apply(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def run_scale(torch, dirac, si, ceil):
    """The applies at the large sizes (Haar links, m = 0.05, Nc = 3, Nv = 12, FP32), far above the caches."""
    dev = "cuda:0"
    nc, nv, m = 3, 12, 0.05
    out = {}
    gen = torch.Generator(device=dev)

    def report(name, op, dims, ms):
        vol = dims[0] * dims[1] * dims[2] * dims[3]
        alg = bytes_per_site(op, nc, nv, 4, 4) * vol
        flops = dirac.flops_per_site(op, nc) * vol * nv
        r = {"lattice": list(dims), "ms": round(ms, 3), "gflops": round(flops / (ms * 1e-3) / 1e9, 1)}
        if op == "brillouin":
            tf = flops / (ms * 1e-3) / 1e12
            r.update(bound="alu", achieved=round(tf, 2), unit="TFLOP/s", frac=round(tf / FP32_VECTOR_PEAK_TFS, 4))
            if ceil:
                r["frac_of_measured"] = round(tf / ceil["fp32_fma_TFLOPs"], 4)
        else:
            gb = alg / (ms * 1e-3) / 1e9
            r.update(bound="hbm", achieved=round(gb, 1), unit="GB/s", frac=round(gb / HBM_PEAK_GBS, 4))
            if ceil:
                r["frac_of_measured"] = round(gb / ceil["copy_GBps"], 4)
        out[name] = r
        log(f"[bench] scale {name}: {ms:.3f} ms, {r['achieved']} {r['unit']}")

    # Wilson at 32^3 x 64: two rotated sets (5 GB of spinors)
    dims = (32, 32, 32, 64)
    nx, ny, nz, nt = dims
    sets = []
    for k in range(2):
        gen.manual_seed(2000 + k)
        U = si.haar_su_n_t(gen, (nt, nz, ny, nx, 4), nc, dev, torch.complex64)
        u = si.complex_gaussian_t(gen, (nt, nz, ny, nx, nc, 4, nv), dev, torch.complex64)
        sets.append((U, u, torch.empty_like(u)))
    it = [0]

    def w():
        U, u, v = sets[it[0] % 2]
        it[0] += 1
        dirac.apply("wilson", U, u, m, out=v)
    report("wilson_32x64", "wilson", dims, time_apply(torch, w, 20))
    del sets
    torch.cuda.empty_cache()
    # staggered and Brillouin at 48^3 x 96
    dims = (48, 48, 48, 96)
    nx, ny, nz, nt = dims
    gen.manual_seed(2100)
    U = si.haar_su_n_t(gen, (nt, nz, ny, nx, 4), nc, dev, torch.complex64)
    phi = si.complex_gaussian_t(gen, (nt, nz, ny, nx, nc, nv), dev, torch.complex64)
    vs = torch.empty_like(phi)
    report("staggered_48x96", "staggered", dims, time_apply(torch, lambda: dirac.apply("staggered", U, phi, m, out=vs), 10))
    del phi, vs
    W = dirac.brillouin_links(U)
    del U
    torch.cuda.empty_cache()
    psi = si.complex_gaussian_t(gen, (nt, nz, ny, nx, nc, 4, nv), dev, torch.complex64)
    vb = torch.empty_like(psi)
    report("brillouin_48x96", "brillouin", dims, time_apply(torch, lambda: dirac.apply("brillouin", W, psi, m, out=vb), 4))
    del W, psi, vb
    torch.cuda.empty_cache()
    return out


def run_bicgstab(torch, dirac, si):
    """BiCGstab on D_B at 32^3 x 64 (Haar links, m = 0.05, Nv = 12): FP64-outer/FP32-inner and plain FP64 to 1e-8."""
    dev = "cuda:0"
    dims, nc, nv, m = (32, 32, 32, 64), 3, 12, 0.05
    nx, ny, nz, nt = dims
    gen = torch.Generator(device=dev)
    gen.manual_seed(2200)
    U = si.haar_su_n_t(gen, (nt, nz, ny, nx, 4), nc, dev, torch.complex128)
    W64 = dirac.brillouin_links(U)
    del U
    W32 = W64.to(torch.complex64)
    b = si.complex_gaussian_t(gen, (nt, nz, ny, nx, nc, 4, nv), dev, torch.complex128)
    out = {"workload": f"BiCGstab on D_B, {nx}x{ny}x{nz}x{nt}, Nc={nc}, Nv={nv}, Haar links, m={m}, tol=1e-8"}
    for name, inner in (("fp64", None), ("mixed_fp32", "fp32")):
        torch.cuda.synchronize()
        t = time.perf_counter()
        x, info = dirac.bicgstab("brillouin", W64, b, m, tol=1e-8, maxit=3000, inner=inner,
                                 gauge_lo=W32 if inner else None)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        out[name] = {"seconds": round(dt, 3), "iterations": info.iterations, "outer_iterations": info.outer_iterations,
                     "reason": info.reason, "max_true_relres": max(info.true_relres)}
        log(f"[bench] bicgstab {name}: {dt:.2f} s, {info.iterations} it, {info.reason}")
        del x
        torch.cuda.empty_cache()
    if out["mixed_fp32"]["reason"] == "converged":
        out["mixed_fp32"]["speedup_vs_fp64"] = round(out["fp64"]["seconds"] / out["mixed_fp32"]["seconds"], 3)
    del W64, W32, b
    torch.cuda.empty_cache()
    return out


def run_cg(torch, dirac, si):
    """Mixed-precision vs FP64 CG on D_W^dag D_W at 32^3 x 64, Nv = 12, to a true residual 1e-10."""
    dev = "cuda:0"
    cfg = si.config("cg_32x64")
    dims, nc, nv, m = cfg["dims"], cfg["nc"], cfg["nv"], cfg["mass"]
    nx, ny, nz, nt = dims
    gen = torch.Generator(device=dev)
    gen.manual_seed(cfg["seed"])
    U = si.near_identity_su_n_t(gen, (nt, nz, ny, nx, 4), nc, cfg["spread"], dev, torch.complex128)
    U32 = U.to(torch.complex64)
    b = si.complex_gaussian_t(gen, (nt, nz, ny, nx, nc, 4, nv), dev, torch.complex128)
    out = {"workload": f"CG on D_W^dag D_W, {nx}x{ny}x{nz}x{nt}, Nc={nc}, Nv={nv}, m={m}, tol=1e-10"}
    runs = [("fp64", None, {}), ("mixed_fp32", "fp32", {}), ("mixed_bf16", "bf16", {})]
    for name, inner, opts in runs:
        torch.cuda.synchronize()
        t = time.perf_counter()
        x, info = dirac.cg("wilson", U, b, m, tol=1e-10, maxit=6000, inner=inner,
                           gauge_lo=U32 if inner else None, opts=opts)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        out[name] = {"seconds": round(dt, 3), "iterations": info.iterations, "fp64_recomputes": info.outer_iterations,
                     "reason": info.reason, "max_true_relres": max(info.true_relres)}
        log(f"[bench] cg {name}: {dt:.2f} s, {info.iterations} it, {info.reason}, "
            f"max relres {max(info.true_relres):.2e}")
        del x
        torch.cuda.empty_cache()
    base = out["fp64"]["seconds"]
    for name in ("mixed_fp32", "mixed_bf16"):
        if out[name]["reason"] == "converged":
            out[name]["speedup_vs_fp64"] = round(base / out[name]["seconds"], 3)
    return out


def run_cpu_baseline(si):
    """The FP64 NumPy oracle on the host: the same six applies on a 12^3 x 24 sample lattice."""
    import numpy as np

    from oracle.brillouin import brillouin_apply, brillouin_apply_dagger, brillouin_links
    from oracle.staggered import staggered_apply, staggered_apply_dagger
    from oracle.wilson import wilson_apply, wilson_apply_dagger

    dims, nc, nv, m = (12, 12, 12, 24), 3, 12, 0.05
    vol = 12 * 12 * 12 * 24
    rng = np.random.default_rng(0)
    U = si.gauge_field(rng, dims, nc, "near", 0.3)
    psi = si.wilson_vector(rng, dims, nc, nv)
    phi = si.staggered_vector(rng, dims, nc, nv)
    W = brillouin_links(U)
    calls = [(wilson_apply, U, psi, 128 * 9 + 72 * 3), (wilson_apply_dagger, U, psi, 128 * 9 + 72 * 3),
             (brillouin_apply, W, psi, 2560 * 9 + 2376 * 3), (brillouin_apply_dagger, W, psi, 2560 * 9 + 2376 * 3),
             (staggered_apply, U, phi, 64 * 9 + 6), (staggered_apply_dagger, U, phi, 64 * 9 + 6)]
    total_t, total_f = 0.0, 0.0
    for fn, g, v, f in calls:
        t = time.perf_counter()
        fn(g, v, m)
        total_t += time.perf_counter() - t
        total_f += f * vol * nv
    log(f"[bench] cpu oracle: {total_t:.2f} s for the six applies on 12^3x24")
    return {"value": round(total_f / total_t / 1e9, 4), "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
            "sample": "the six applies (W, W^dag, B, B^dag, S, S^dag) once each on a 12^3x24 lattice, Nc=3, Nv=12, "
                      "FP64 NumPy, single thread", "seconds": round(total_t, 2),
            "host_cores_available": len(os.sched_getaffinity(0))}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--sets", type=int, default=4)
    ap.add_argument("--no-cg", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-scale", action="store_true", help="skip the large-lattice applies, BiCGstab and ceilings")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 512 MiB device copy (outside the timed steps) whose HBM counters "
                         "scale the PMC byte counts of the stencil kernels")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported (the multi-GPU "
              "domain decomposition is designed but not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch

    import synthetic_inputs as si
    from paper_2112_14640_amd import dirac

    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(512 * 2 ** 20 // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] calibration copies done: 5 x 512 MiB read + 512 MiB write")
        del src, dst
    ceil = None if args.no_scale else run_ceilings(torch, dirac)
    res = run_applies(args, torch, dirac, si)
    if ceil:
        for name, r in res["rooflines"].items():
            r["frac_of_measured"] = round(r["achieved"] / (ceil["fp32_fma_TFLOPs"] if r["bound"] == "alu"
                                                           else ceil["copy_GBps"]), 4)
    scale = None if args.no_scale else run_scale(torch, dirac, si, ceil)
    cg = None if args.no_cg else run_cg(torch, dirac, si)
    bicg = None if (args.no_cg or args.no_scale) else run_bicgstab(torch, dirac, si)
    cpu = None if args.no_cpu else run_cpu_baseline(si)
    nx, ny, nz, nt = res["dims"]
    rl = dict(res["rooflines"][res["dominant"]])
    line = {
        "metric": "Dirac-apply GFLOP/s + % HBM roofline at Nv=12; mixed vs FP64 CG time",
        "value": round(res["value"], 1),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["ms_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"Wilson, Brillouin and staggered applies and adjoints, {nx}x{ny}x{nz}x{nt}, "
                               f"Nc={res['nc']}, Nv={res['nv']}, FP32, exp(i 0.3 H) links, m=0.05",
                   "lattice": [nx, ny, nz, nt], "nc": res["nc"], "nv": res["nv"], "input_sets_rotated": args.sets},
        "roofline": {k: rl[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic", "frac_of_measured")
                     if k in rl},
        "roofline_kernel": res["dominant"],
        "kernels": res["rooflines"],
        "brillouin_link_build_ms": res["link_build_ms"],
        "ceilings": ceil,
        "scale": scale,
        "cg": cg,
        "bicgstab": bicg,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
