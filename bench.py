#!/usr/bin/env python3
"""Benchmark: CG time-to-solution (mixed vs FP64) and Mhat^dag Mhat bandwidth on one MI355X.

One step is one pass of the hot path over one batch of synthetic input at
32^3 x 64 (kappa 0.1255, c_sw 1.0, links exp(iH) with H of width 0.2): the 8
Gaussian sources solved (M x = b to tol 1e-10) together in one mixed-precision
and one FP64 multi-source solve (sources interleaved site by site, each link
and clover block read once per site for all of them), one single-source solve
of each precision for comparison, one fermion force with the mixed solve
inside, and a timed run of the stencil kernels (k1, k2, Mhat^dag Mhat) for
one and for 8 sources.  After the timed region the CPU-baseline leg times the
oracle (one Mhat^dag Mhat at 32^3 x 64, full solves at 4^4, 8x8x16x16 and
16^4) and applies the oracle's FP64 operator to every GPU solution of the
headline solve (relative residual per source and precision).  `value` is the mixed time to solution per source:
the multi-source solve's time over 8.  All input fields are resident in GPU
memory before the timed region starts.

Prints one JSON line on stdout; progress goes to stderr.

    python bench.py [--steps K] [--warmup W] [--sources S] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "CG time-to-solution + M†M GB/s (% HBM peak), mixed vs FP64, 16^4 & 32^3x64"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
# FP32 vector FMA rate without packed-FP32 instructions (the HIP sources are
# compiled with them disabled): 256 CUs x 64 lanes x 2 flops x 2.4 GHz
FP32_VALU_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12
FLOPS_PER_SITE = 1824.0  # 1320 hopping + 504 clover per site per M application
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_dslash_32x32x32x64.md")
# kernels whose HBM traffic the committed counter summary records: the k2 and
# k1 launches of the multi-source solves (mixed: the timed headline; FP64:
# its reliable updates and the FP64 solve) and of the single-source ones
TRAFFIC_KERNELS = {
    "k2_mixed_multi": ("dslash_kernel<float, 2, false, false, true,", "LinkH18, qcd::CloverHC,"),
    "k1_mixed_multi": ("dslash_kernel<float, 0, true, false, true,", "LinkH18", "CloverH>"),
    "k1_mixed_single": ("dslash_kernel<float, 0, true, false, false,", "LinkH12", "CloverH>"),
    "k2_fp64_multi": ("dslash_kernel<double, 2, false, false, true,", "qcd::CloverF64C, qcd::CloverNone>"),
    "k1_fp64_multi": ("dslash_kernel<double, 0, true, false, true,", "qcd::CloverNone, qcd::CloverF64>"),
    "k2_fp64_single": ("dslash_kernel<double, 2, false, false, false,", "qcd::CloverF64C, qcd::CloverNone>"),
    "k1_fp64_single": ("dslash_kernel<double, 0, true, false, false,", "qcd::CloverNone, qcd::CloverF64>"),
}
KERNEL_SOURCES = [os.path.join(ROOT, "paper_0910_0262_amd", "csrc", f) for f in ("qcd_device.h", "qcd_internal.h", "dslash.hip")]


def log(msg: str) -> None:
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


# algorithmic bytes per even site (each field read once, neighbours counted once)
def k1_bytes_per_site(prec: str, link_recon=12, mixed_clover=16) -> float:
    if prec == "fp64":
        return 192 + 8 * (16 * (6 if link_recon == 12 else 9)) + 576 + 192
    return 52 + 8 * 24 + (288 if mixed_clover == 32 else 152) + 52


# A_ee of k2 in the compact form (26 reals per chiral block instead of 36):
# FP64 416 B instead of 576, binary16 104 B + 8 B of scales instead of 152
def ee_clover_saving(prec: str, link_recon=12, mixed_clover=16) -> float:
    if prec == "fp64":
        return 160.0 if link_recon == 12 else 0.0
    return 40.0 if mixed_clover == 16 else 0.0


def k2_bytes_per_site(prec: str, link_recon=12, mixed_clover=16) -> float:
    return (k1_bytes_per_site(prec, link_recon, mixed_clover) + (192 if prec == "fp64" else 52)
            - ee_clover_saving(prec, link_recon, mixed_clover))


def mdagm_bytes_per_site(prec: str, mixed_clover=16) -> float:
    return 2 * (k1_bytes_per_site(prec, mixed_clover=mixed_clover) + k2_bytes_per_site(prec, mixed_clover=mixed_clover))


# the same with nr interleaved right-hand sides: spinors nr times, links and clover once
def spinor_bytes(prec: str) -> float:
    return 192.0 if prec == "fp64" else 52.0


def k1_bytes_multi(prec: str, nr: int, mixed_clover=16) -> float:
    """The mixed multi-source kernels read all nine binary16 link entries
    (36 B per link) instead of two rows (24 B)."""
    sp = spinor_bytes(prec)
    links = 8 * 12 if prec == "mixed" and nr > 1 else 0
    return k1_bytes_per_site(prec, mixed_clover=mixed_clover) + 2 * sp * (nr - 1) + links


def k2_bytes_multi(prec: str, nr: int, mixed_clover=16) -> float:
    return k1_bytes_multi(prec, nr, mixed_clover) + spinor_bytes(prec) * nr - ee_clover_saving(prec, 12, mixed_clover)


def mdagm_bytes_multi(prec: str, nr: int, mixed_clover=16) -> float:
    return 2 * (k1_bytes_multi(prec, nr, mixed_clover) + k2_bytes_multi(prec, nr, mixed_clover))


def _read_traffic_file():
    with open(TRAFFIC_FILE) as f:
        text = f.read()
    block = text.split("```json", 1)[1].split("```", 1)[0]
    return json.loads(block)


def traffic_for(key: str, vh: int):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summary, if it still describes the current kernel source; else None."""
    try:
        t = _read_traffic_file()
    except (OSError, ValueError, IndexError):
        return None
    if t.get("source_sha256") != kernel_source_hash() or t.get("vh") != vh or key not in t.get("kernels", {}):
        return None
    return t["kernels"][key]["traffic_bytes"]


def traffic_summary(fetch_csv: str, write_csv: str, vh: int, command: str, nr: int = 8) -> None:
    """Write the committed traffic summary from two rocprofv3 --pmc runs
    (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch).  Each counter is scaled by
    what it reads for the 2 GiB copy kernel that bench.py runs (2 GiB read,
    2 GiB written); dispatches that returned at once (halted iterations) are
    left out."""
    import csv

    def rows_of(path):
        return list(csv.DictReader(open(path)))

    def mean_of(rows, tokens):
        k = [float(r["Counter_Value"]) for r in rows if all(t in r["Kernel_Name"] for t in tokens)]
        med = float(np.median(k))
        k = [v for v in k if v > 0.5 * med]
        return float(np.mean(k)), len(k)

    fr, wr = rows_of(fetch_csv), rows_of(write_csv)
    f_c, _ = mean_of(fr, ("stream_copy_k",))
    w_c, _ = mean_of(wr, ("stream_copy_k",))
    copy_bytes = float(2 << 30)
    fs, ws = copy_bytes / (f_c * 1024.0), copy_bytes / (w_c * 1024.0)
    alg = {"k2_mixed_multi": k2_bytes_multi("mixed", nr) * vh, "k1_mixed_multi": k1_bytes_multi("mixed", nr) * vh,
           "k1_mixed_single": k1_bytes_per_site("mixed") * vh,
           "k2_fp64_multi": k2_bytes_multi("fp64", nr) * vh, "k1_fp64_multi": k1_bytes_multi("fp64", nr) * vh,
           "k2_fp64_single": k2_bytes_per_site("fp64") * vh, "k1_fp64_single": k1_bytes_per_site("fp64") * vh}
    kernels = {}
    for key, tokens in TRAFFIC_KERNELS.items():
        f_k, n_f = mean_of(fr, tokens)
        w_k, n_w = mean_of(wr, tokens)
        traffic = f_k * 1024.0 * fs + w_k * 1024.0 * ws
        kernels[key] = {"kernel": " ".join(tokens), "fetch_kib": f_k, "write_kib": w_k, "dispatches": [n_f, n_w],
                        "traffic_bytes": traffic, "algorithmic_bytes": alg[key],
                        "traffic_over_algorithmic": traffic / alg[key]}
    rec = {"vh": vh, "nr_multi": nr, "copy_fetch_kib": f_c, "copy_write_kib": w_c, "copy_bytes": copy_bytes,
           "fetch_scale": fs, "write_scale": ws, "kernels": kernels, "source_sha256": kernel_source_hash()}
    with open(TRAFFIC_FILE, "w") as f:
        f.write("# HBM traffic of the stencils at 32x32x32x64 (rocprofv3 counters)\n\n")
        f.write("Two counter passes (FETCH_SIZE, then WRITE_SIZE) over the same program, run from the repository "
                "root on one MI355X:\n\n")
        f.write("```\n" + command + "\n```\n\n")
        f.write(f"FETCH_SIZE reads {f_c:.0f} KiB and WRITE_SIZE {w_c:.0f} KiB per dispatch of the 2 GiB copy "
                f"kernel, so they are scaled by {fs:.3f} and {ws:.3f}.\n\n")
        f.write("| kernel | dispatches | HBM traffic per launch | algorithmic | ratio |\n|---|---:|---:|---:|---:|\n")
        for key, k in kernels.items():
            f.write(f"| {key} (`{k['kernel']}`) | {k['dispatches'][0]} | {k['traffic_bytes'] / 1e6:.1f} MB | "
                    f"{k['algorithmic_bytes'] / 1e6:.1f} MB | {k['traffic_over_algorithmic']:.3f} |\n")
        f.write("\n`source_sha256` is the hash of the kernel sources the counters were taken on; bench.py "
                "reports traffic as null once they change.\n\n")
        f.write("```json\n" + json.dumps(rec, indent=1) + "\n```\n")
    print(json.dumps(rec))


def host_cpu() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(dims, kappa, csw, u_np, b_np, fp64_iters: int):
    """The oracle as it stands, timed on the host: one Mhat^dag Mhat at the full
    workload (the sample), scaled by the FP64 CG iteration count of the same solve.
    Returns the record and the oracle's setup (reused for the residual check)."""
    import oracle as O

    t0 = time.perf_counter()
    setup = O.CloverSetup(torch.as_tensor(u_np), kappa, csw)
    t_setup = time.perf_counter() - t0
    e, _ = O.to_eo(torch.as_tensor(b_np), dims)
    t0 = time.perf_counter()
    setup.MdagM(e)
    t_app = time.perf_counter() - t0
    return {
        "value": t_app * fp64_iters,
        "unit": "s",
        "cores": torch.get_num_threads(),
        "host_cpu": host_cpu(),
        "kind": "oracle",
        "sample": (f"one oracle Mhat^dag Mhat application at {dims[0]}x{dims[1]}x{dims[2]}x{dims[3]} "
                   f"({t_app:.2f} s, after a {t_setup:.1f} s clover setup) x {fp64_iters} FP64 CG "
                   f"iterations of source 0 = extrapolated oracle CG time-to-solution"),
    }, setup


def oracle_residuals(setup, b_np, xs_host):
    """The oracle's FP64 operator on every GPU solution of the headline workload:
    relative residual |b - M x| / |b| per source and precision."""
    out = {}
    for prec, xs in xs_host.items():
        res = []
        for k, x in enumerate(xs):
            b = torch.as_tensor(b_np[k])
            res.append(float(torch.linalg.norm(b - setup.M(x)) / torch.linalg.norm(b)))
        out[prec] = res
        log(f"oracle residuals of the {prec} solutions: max {max(res):.2e}")
    return out


def oracle_small_solves():
    """Oracle full solves (tol 1e-10) of the two small workloads, timed on the host:
    4^4 (kappa 0.12, width 0.3) and 8x8x16x16 (kappa 0.124, width 0.5), c_sw 1, seed 0."""
    import oracle as O
    from paper_0910_0262_amd import synth

    out = {}
    for name, dims, width, kappa in (("4^4", (4, 4, 4, 4), 0.3, 0.12), ("8x8x16x16", (8, 8, 16, 16), 0.5, 0.124)):
        u = synth.random_su3_field(dims, width, 0)
        b = synth.gaussian_source(dims, 0, 0)
        t0 = time.perf_counter()
        ref = O.solve_full(O.CloverSetup(torch.as_tensor(u), kappa, 1.0), torch.as_tensor(b), 1e-10)
        t = time.perf_counter() - t0
        out[name] = {"dims": list(dims), "oracle_solve_s": t, "iters": ref.iters, "true_rel_res": ref.true_rel_res,
                     "cores": torch.get_num_threads()}
        log(f"oracle solve {name}: {t:.2f} s, {ref.iters} iterations")
    return out


def oracle_check_16(tol_gpu=1e-12):
    """Part of the CPU-baseline leg: the oracle's full solve of the 16^4 workload
    (kappa 0.125, c_sw 1, width 0.3, source 0; tol 1e-13), timed on the host, and
    the relative solution error of the GPU's FP64 and mixed solves against it."""
    import oracle as O
    from paper_0910_0262_amd import Lattice, synth

    dims, kappa, csw = (16, 16, 16, 16), 0.125, 1.0
    u = synth.random_su3_field(dims, 0.3, 0)
    b = synth.gaussian_source(dims, 0, 0)
    t0 = time.perf_counter()
    ref = O.solve_full(O.CloverSetup(torch.as_tensor(u), kappa, csw), torch.as_tensor(b), 1e-13)
    t_oracle = time.perf_counter() - t0
    lat = Lattice(dims, kappa, csw)
    lat.load_gauge(torch.as_tensor(u).cuda())
    out = {"dims": list(dims), "oracle_solve_s": t_oracle, "oracle_iters": ref.iters,
           "cores": torch.get_num_threads(), "gpu_tol": tol_gpu}
    for prec in ("fp64", "mixed"):
        x, st = lat.solve(torch.as_tensor(b).cuda(), prec=prec, tol=tol_gpu)
        out[f"{prec}_rel_solution_error"] = float(torch.linalg.norm(x.cpu() - ref.x) / torch.linalg.norm(ref.x))
    lat.close()
    log(f"oracle 16^4 solve {t_oracle:.1f} s; GPU relative solution error fp64 "
        f"{out['fp64_rel_solution_error']:.1e}, mixed {out['mixed_rel_solution_error']:.1e}")
    return out


def secondary(name, dims, width, kappa, csw, tol, reps, n_apps):
    """Smaller lattices of the paper (abstract: 8x8x16x16 and 16^4): solve times
    and n_apps standalone Mhat^dag Mhat applications; not part of `value`."""
    from paper_0910_0262_amd import Lattice, synth

    lx, ly, lz, lt = dims
    vh = lx * ly * lz * lt // 2
    lat = Lattice(dims, kappa, csw)
    lat.load_gauge(torch.as_tensor(synth.random_su3_field(dims, width, 0)).cuda())
    b = torch.as_tensor(synth.gaussian_source(dims, 0, 0)).cuda()
    out = {"dims": list(dims), "width": width, "kappa": kappa}
    for prec in ("mixed", "fp64"):
        lat.solve(b, prec=prec, tol=tol)
        ts, its = [], []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st = lat.solve(b, prec=prec, tol=tol)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
            its.append(st["iters"])
        k1, k2, app = lat.time_stencil(prec, n_apps)
        gbs = mdagm_bytes_per_site(prec) * vh / (app * 1e-3) / 1e9
        out[prec] = {"tts_s": float(np.median(ts)), "iters": int(np.median(its)), "mdagm_ms": app,
                     "mdagm_GB_s": gbs, "mdagm_GFLOP_s": 2 * FLOPS_PER_SITE * 2 * vh / (app * 1e-3) / 1e9,
                     "us_per_iter": 1e6 * float(np.median(ts)) / max(1, int(np.median(its)))}
    # the same lattice with 8 sources solved together (latency shared by all of them)
    bm = torch.stack([torch.as_tensor(synth.gaussian_source(dims, 0, k)).cuda() for k in range(8)])
    for prec in ("mixed", "fp64"):
        lat.solve_multi(bm, prec=prec, tol=tol)
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, sts = lat.solve_multi(bm, prec=prec, tol=tol)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        out[prec]["multi8_tts_per_source_s"] = float(np.median(ts)) / 8
        out[prec]["multi8_iters"] = sts[0]["iters"]
    del bm
    lat.close()
    log(f"secondary {name}: mixed {out['mixed']['tts_s'] * 1e3:.2f} ms, fp64 {out['fp64']['tts_s'] * 1e3:.2f} ms; "
        f"8 sources together: {out['mixed']['multi8_tts_per_source_s'] * 1e3:.2f} / "
        f"{out['fp64']['multi8_tts_per_source_s'] * 1e3:.2f} ms per source")
    return out


def trajectory_run(lat, dims, u_dev, n_steps, dt, beta, prec, tol, seed=0):
    """One R-algorithm trajectory (n_f = 2, clover determinant, gauge action,
    reunitarisation) from u_dev with fresh momenta; not part of `value`."""
    from paper_0910_0262_amd import synth

    lx, ly, lz, lt = dims
    U = u_dev.clone()
    P = torch.as_tensor(synth.momenta(dims, seed)).cuda()
    xi = torch.as_tensor(np.stack([synth.heatbath_xi(dims, seed + k) for k in range(n_steps)])).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    acts, st = lat.md_trajectory(U, P, xi, dt, n_steps, beta=beta, n_f=2.0, clover_det=True, reunitarize=True,
                                 prec=prec, tol=tol)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    out = {"dims": list(dims), "n_steps": n_steps, "dt": dt, "beta": beta, "n_f": 2.0, "prec": prec, "tol": tol,
           "s": t, "ms_per_md_step": 1e3 * t / n_steps, "solver_iters_per_step": st["iters"] / n_steps,
           "actions_first": acts[0], "actions_last": acts[-1]}
    log(f"trajectory {lx}x{ly}x{lz}x{lt}: {n_steps} steps in {t:.3f} s ({out['ms_per_md_step']:.1f} ms/step, "
        f"{out['solver_iters_per_step']:.0f} CG iterations/step)")
    del U, P, xi
    return out


def trajectory_secondary(dims, width, kappa, csw, n_steps, dt, beta, prec, tol):
    from paper_0910_0262_amd import Lattice, synth

    lat = Lattice(dims, kappa, csw)
    u = torch.as_tensor(synth.random_su3_field(dims, width, 0)).cuda()
    lat.load_gauge(u)
    trajectory_run(lat, dims, u, 1, dt, beta, prec, tol)  # warm-up
    out = trajectory_run(lat, dims, u, n_steps, dt, beta, prec, tol)
    lat.close()
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sources", type=int, default=8)
    ap.add_argument("--dims", type=str, default="32,32,32,64")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--stencil-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-force", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--no-trajectory", action="store_true")
    ap.add_argument("--beta", type=float, default=5.6, help="gauge coupling of the MD trajectories")
    ap.add_argument("--mixed-clover", type=int, default=16, choices=(16, 32))
    ap.add_argument("--traffic-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the committed traffic summary from two rocprofv3 --pmc counter CSVs and exit")
    ap.add_argument("--traffic-command", type=str, default="")
    args = ap.parse_args()
    if args.traffic_summary:
        if not args.traffic_command.strip():
            ap.error("--traffic-summary needs --traffic-command: the rocprofv3 commands the CSVs came from")
        d = tuple(int(v) for v in args.dims.split(","))
        traffic_summary(args.traffic_summary[0], args.traffic_summary[1], d[0] * d[1] * d[2] * d[3] // 2,
                        args.traffic_command)
        return 0

    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path; use --gpus 1",
              file=sys.stderr)
        return 2
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2

    from paper_0910_0262_amd import Lattice, capi, synth

    capi.lib()
    dims = tuple(int(v) for v in args.dims.split(","))
    kappa, csw, width = 0.1255, 1.0, 0.2
    lx, ly, lz, lt = dims
    V = lx * ly * lz * lt
    Vh = V // 2
    log(f"generating inputs {dims}")
    u_np = synth.random_su3_field(dims, width, 0)
    b_np = [synth.gaussian_source(dims, 0, k) for k in range(args.sources)]
    xi_np = synth.heatbath_xi(dims, 0)

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    U = torch.as_tensor(u_np).to(dev)
    B = [torch.as_tensor(b).to(dev) for b in b_np]
    XI = torch.as_tensor(xi_np).to(dev)
    lat = Lattice(dims, kappa, csw)
    lat.set_option(capi.QCD_OPT_MIXED_CLOVER, args.mixed_clover)
    lat.load_gauge(U)
    phi = lat.apply("Mhatdag", XI)
    torch.cuda.synchronize()

    # bandwidth calibration: plain copy of 2 GiB through the library's copy kernel
    nbytes = 2 << 30
    src = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    lat.stream_copy(dst, src)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(5):
        lat.stream_copy(dst, src)
    ev1.record()
    ev1.synchronize()
    copy_gbs = 5 * 2 * nbytes / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
    del src, dst
    log(f"copy kernel: {copy_gbs:.0f} GB/s (read + write)")

    NR = args.sources
    B_all = torch.stack(B) if NR > 1 else None

    def one_step(record):
        # the headline: all sources in one multi-source solve per precision
        xs = {}
        for prec in ("mixed", "fp64"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if NR > 1:
                x, sts = lat.solve_multi(B_all, prec=prec, tol=args.tol)
            else:
                x1, st1 = lat.solve(B[0], prec=prec, tol=args.tol)
                x, sts = x1.unsqueeze(0), [st1]
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            record["multi"].append({"prec": prec, "s": dt, "per_source_s": dt / NR, "iters": sts[0]["iters"],
                                    "reliable_updates": sts[0]["reliable_updates"],
                                    "true_rel_res_max": max(st["true_rel_res"] for st in sts),
                                    "converged_all": all(st["converged"] == 1 for st in sts),
                                    "flops": sum(st["flops"] for st in sts)})
            xs[prec] = x
        for k in range(NR):
            record["mixed_vs_fp64"].append(float(torch.linalg.norm(xs["mixed"][k] - xs["fp64"][k])
                                                 / torch.linalg.norm(xs["fp64"][k])))
        del xs
        # one source on its own, for comparison
        for prec in ("mixed", "fp64"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, st = lat.solve(B[0], prec=prec, tol=args.tol)
            torch.cuda.synchronize()
            record["single"].append({"prec": prec, "s": time.perf_counter() - t0, **st})
            del x
        if not args.no_force:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            S, G, F, X, st = lat.action_force(phi, prec="mixed", tol=args.tol, want_X=False)
            torch.cuda.synchronize()
            record["force"].append({"s": time.perf_counter() - t0, "S": S, "iters": st["iters"]})
            del G, F
        # stencil kernels, timed with HIP events on the library's stream
        lat.apply("MdagM", XI)
        lat.apply("MdagM", XI, prec="mixed")
        for prec in ("mixed", "fp64"):
            record["stencil"][prec].append(lat.time_stencil(prec, args.stencil_reps))
            if NR > 1:
                record["stencil_multi"][prec].append(lat.time_stencil_multi(NR, prec, args.stencil_reps))

    def new_record():
        return {"multi": [], "single": [], "mixed_vs_fp64": [], "force": [],
                "stencil": {"mixed": [], "fp64": []}, "stencil_multi": {"mixed": [], "fp64": []}}

    for w in range(args.warmup):
        log(f"warmup step {w + 1}/{args.warmup}")
        one_step(new_record())
    rec = new_record()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for s in range(args.steps):
        one_step(rec)
        log(f"timed step {s + 1}/{args.steps} done")
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start

    def multi_of(prec, key):
        return [r[key] for r in rec["multi"] if r["prec"] == prec]

    def single_of(prec, key):
        return [r[key] for r in rec["single"] if r["prec"] == prec]

    tts = {p: float(np.mean(multi_of(p, "per_source_s"))) for p in ("mixed", "fp64")}
    tts_single = {p: float(np.mean(single_of(p, "s"))) for p in ("mixed", "fp64")}
    mc = args.mixed_clover

    def stencil_summary(ms3, prec, nr):
        k1_ms, k2_ms, app_ms = (float(v) for v in ms3)
        gbs = mdagm_bytes_multi(prec, nr, mc) * Vh / (app_ms * 1e-3) / 1e9
        return {"n_rhs": nr, "ms": app_ms, "ms_per_rhs": app_ms / nr, "GB_s": gbs,
                "pct_hbm_peak": 100.0 * gbs / HBM_PEAK_GBS, "pct_copy_bw": 100.0 * gbs / copy_gbs,
                "GFLOP_s": 2 * FLOPS_PER_SITE * V * nr / (app_ms * 1e-3) / 1e9,
                "k1_ms": k1_ms, "k2_ms": k2_ms,
                "k1_GB_s": k1_bytes_multi(prec, nr, mc) * Vh / (k1_ms * 1e-3) / 1e9,
                "k2_GB_s": k2_bytes_multi(prec, nr, mc) * Vh / (k2_ms * 1e-3) / 1e9}

    mdagm = {p: stencil_summary(np.mean(np.array(rec["stencil"][p]), axis=0), p, 1) for p in ("mixed", "fp64")}
    mdagm_multi = ({p: stencil_summary(np.mean(np.array(rec["stencil_multi"][p]), axis=0), p, NR)
                    for p in ("mixed", "fp64")} if NR > 1 else None)
    # roofline: the dominant kernel of the timed (multi-source) solve, the
    # mixed k2 (with k2^dag, 326 of the solve's launches against 163 + 163 for
    # k1 and k1^dag).  With 8 sources sharing each link and clover load it is
    # bound by vector instruction issue (counters: over 80 % of the VALU issue
    # capacity), not HBM, so it is placed against the FP32 FMA peak; its HBM
    # rate is reported beside.  The mixed k1 of the same solve follows as
    # roofline_k1_multi.  With one source the kernels are HBM-bound.
    head = mdagm_multi["mixed"] if NR > 1 else mdagm["mixed"]
    clover_name = "FP32" if mc == 32 else "binary16"

    def alu_or_hbm(which: str):
        k = "k2" if which == "k2" else "k1"
        if NR > 1:
            nbytes = (k2_bytes_multi if k == "k2" else k1_bytes_multi)("mixed", NR, mc) * Vh
        else:
            nbytes = (k2_bytes_per_site if k == "k2" else k1_bytes_per_site)("mixed", mixed_clover=mc) * Vh
        flops = FLOPS_PER_SITE * Vh * NR
        secs = head[k + "_ms"] * 1e-3
        tkey = f"{k}_mixed_{'multi' if NR > 1 else 'single'}"
        traffic = traffic_for(tkey, Vh) if (mc == 16 and (NR == 8 or NR == 1)) else None
        what = ("k2: A_ee p_e - kappa^2 H_eo t_o" if k == "k2" else "k1: t_o = A_oo^-1 H_oe p_e")
        kname = (f"dslash_kernel<float, {2 if k == 'k2' else 0}, {'false' if k == 'k2' else 'true'}, false, "
                 f"{'true' if NR > 1 else 'false'}, ...> (mixed {what} for {NR} interleaved sources, binary16 "
                 f"spinors/links, {clover_name} clover)")
        if NR > 1:
            achieved = flops / secs / 1e12
            return {"bound": "alu", "achieved": achieved, "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": achieved / FP32_VALU_PEAK_TFLOPS, "traffic": traffic, "kernel": kname,
                    "flops_per_launch": flops, "bytes_per_launch": nbytes,
                    "hbm_GB_s": nbytes / secs / 1e9, "hbm_frac": nbytes / secs / 1e9 / HBM_PEAK_GBS}
        achieved = nbytes / secs / 1e9
        return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kname, "bytes_per_launch": nbytes}

    roofline = alu_or_hbm("k2")
    roofline_k1 = alu_or_hbm("k1")
    # the single-source k1, HBM-bound, for reference
    s_k1 = mdagm["mixed"]["k1_ms"] * 1e-3
    s_bytes = k1_bytes_per_site("mixed", mixed_clover=mc) * Vh
    roofline_single = {"bound": "hbm", "achieved": s_bytes / s_k1 / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": s_bytes / s_k1 / 1e9 / HBM_PEAK_GBS,
                       "traffic": traffic_for("k1_mixed_single", Vh) if mc == 16 else None,
                       "kernel": "dslash_kernel<float, 0, true, false, false, ...CloverH> (mixed k1, one source)",
                       "bytes_per_launch": s_bytes}

    out = {
        "metric": METRIC,
        "value": tts["mixed"],
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t_total / args.steps,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (binary16 storage) + f64 reliable updates",
        "data": "synthetic",
        "config": {"workload": f"{lx}x{ly}x{lz}x{lt} even-odd Wilson-clover CG to tol {args.tol:g}, "
                               f"kappa {kappa}, c_sw {csw}, SU(3) links exp(iH) width {width}, "
                               f"{args.sources} Gaussian sources solved together (time per source), "
                               f"mixed vs FP64 + force",
                   "dims": list(dims), "sources": args.sources, "tol": args.tol},
        "mixed_tts_s": tts["mixed"],
        "fp64_tts_s": tts["fp64"],
        "speedup_mixed_vs_fp64": tts["fp64"] / tts["mixed"],
        "iters": {p: float(np.mean(multi_of(p, "iters"))) for p in ("mixed", "fp64")},
        "reliable_updates_mixed": float(np.mean(multi_of("mixed", "reliable_updates"))),
        "true_rel_res_max": {p: float(np.max(multi_of(p, "true_rel_res_max"))) for p in ("mixed", "fp64")},
        "converged_all": all(r["converged_all"] for r in rec["multi"]),
        "mixed_vs_fp64_rel_diff_max": float(np.max(rec["mixed_vs_fp64"])),
        "solver_GFLOP_s": {p: float(np.mean([r["flops"] / r["s"] for r in rec["multi"] if r["prec"] == p])) / 1e9
                           for p in ("mixed", "fp64")},
        "single_source": {p: {"tts_s": tts_single[p], "iters": float(np.mean(single_of(p, "iters"))),
                              "true_rel_res": float(np.max(single_of(p, "true_rel_res")))}
                          for p in ("mixed", "fp64")},
        "multi_source_speedup": {p: tts_single[p] / tts[p] for p in ("mixed", "fp64")},
        "mdagm": mdagm,
        "mdagm_multi": mdagm_multi,
        "copy_GB_s": copy_gbs,
        "force_s": float(np.mean([f["s"] for f in rec["force"]])) if rec["force"] else None,
        "roofline": roofline,
        "roofline_k1_multi": roofline_k1,
        "roofline_single_source": roofline_single,
        "context": "Cell/B.E. QS20 (the paper): ~10 GFLOPS and ~20 GB/s per kernel; "
                   "8.7x / 9.6x over one 2.33 GHz Xeon core (whole application)",
    }
    out["mixed_clover_bits"] = args.mixed_clover
    # the headline solutions (the solves are bit-reproducible), kept on the host
    # for the oracle's residual check after the GPU work; before the trajectory,
    # which leaves its evolved links in the context
    xs_host = None
    if not args.no_cpu_baseline:
        xs_host = {}
        for prec in ("mixed", "fp64"):
            if NR > 1:
                x, _ = lat.solve_multi(B_all, prec=prec, tol=args.tol)
            else:
                x1, _ = lat.solve(B[0], prec=prec, tol=args.tol)
                x = x1.unsqueeze(0)
            xs_host[prec] = [x[k].cpu() for k in range(NR)]
            del x
    if not args.no_trajectory:
        out["trajectory"] = {f"{lx}x{ly}x{lz}x{lt}": trajectory_run(lat, dims, U, 2, 0.02, args.beta, "mixed",
                                                                     args.tol)}
    lat.close()
    del B, B_all, U, XI, phi
    torch.cuda.empty_cache()
    if not args.no_secondary:
        out["secondary"] = {
            "16^4": secondary("16^4", (16, 16, 16, 16), 0.3, 0.125, csw, args.tol, 5, 100),
            "8x8x16x16": secondary("8x8x16x16", (8, 8, 16, 16), 0.5, 0.124, csw, args.tol, 5, 100),
        }
        if not args.no_trajectory:
            for prec in ("mixed", "fp64"):
                out["trajectory"][f"16^4-{prec}"] = trajectory_secondary((16, 16, 16, 16), 0.3, 0.125, csw, 10,
                                                                         0.02, args.beta, prec, args.tol)
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle Mhat^dag Mhat at the full workload")
        fp64_iters = int(round(np.mean(single_of("fp64", "iters"))))
        out["cpu_baseline"], setup = cpu_baseline(dims, kappa, csw, u_np, b_np[0], fp64_iters)
        if xs_host is not None:
            res = oracle_residuals(setup, b_np, xs_host)
            out["oracle_residual_32"] = {"per_source": res,
                                         "max": {p: max(v) for p, v in res.items()},
                                         "what": "|b - M x| / |b| with the oracle's FP64 M, every GPU solution "
                                                 "of the headline solve (tol 1e-10 on the normal equations)"}
        del setup
        out["oracle_16x4"] = oracle_check_16()
        out["oracle_small_solves"] = oracle_small_solves()
    else:
        out["cpu_baseline"] = None
        out["oracle_16x4"] = None
    kids = []
    try:
        import psutil

        kids = [f"{c.pid} {' '.join(c.cmdline()[:3])}" for c in psutil.Process().children(recursive=True)]
    except Exception as e:  # pragma: no cover
        kids = [f"unknown ({e})"]
    log(f"child processes at exit: {kids if kids else 'none'}")
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
