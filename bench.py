#!/usr/bin/env python3
"""Benchmark of the INT8 Ozaki-I ZGEMM emulation on one MI355X.

Workload (default): the large ill-conditioned complex product, M = N = K =
16384, complex Gaussian A and B with every row of A and every column of B
scaled by 2^r, r ~ U-int[-30, 30] (seed 1004). One step is one whole
ozaki_zgemm call (exponent scan, slicing, fused slice GEMM + recombination)
on operands already resident in HBM.

Before timing, the oracle leg sweeps the slice count for both slice kinds
(8-bit balanced and trunc-7) and measures the componentwise error err_comp of
each product against the double-double reference on sampled entries (4096
random entries plus 4 whole rows and 4 whole columns); the headline is the
faster of the two slice kinds at its smallest s reaching 1e-12.

Printed on stdout: one JSON line. `value` is effective FP64 TFLOP/s
(8 m n k / wall time per call). Beside it: the per-s error and time table, the
hand-written native FP64-MFMA ZGEMM on the same buffers (time and err_comp),
per-phase times from HIP events recorded on the launch stream, the roofline
of the dominant kernel (the fused INT8 slice GEMM) and the CPU baseline (the
oracle's emulation model, the double-double reference and host-BLAS FP64
GEMM, timed on bounded samples of the same workload on the host cores).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "effective FP64 TFLOP/s, INT8-Ozaki ZGEMM vs native FP64 MFMA at ≤1e-12 rel err"
TARGET = 1e-12
INT8_PEAK_TOPS = 5000.0      # MI355X dense INT8 matrix peak
FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 matrix peak
HBM_PEAK_GBS = 8000.0
GEMM_SOURCES = [os.path.join(ROOT, "paper_2603_29975_amd", "csrc", f)
                for f in ("ozaki_gemm.hip", "ozaki_gemm_tile.hpp")]
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "ozgemm_{workload}_{split}_s{slices}_traffic.txt")
TUNE_CACHE = os.path.join(ROOT, "paper_2603_29975_amd", "tune_gfx950.json")
S_MAX = {"t7": 12, "b8": 8}

# workload name -> (record name, kind, slice sweep per slice kind)
WORKLOADS = {
    "ill16384": ("illcond_zgemm_16384", "z", {"b8": range(4, 9), "t7": range(4, 11)}),
    "ill4096": ("illcond_zgemm_4096", "z", {"b8": range(4, 9), "t7": range(4, 11)}),
    "kkr2048": ("kkr_zgemm_2048", "z", {"b8": range(4, 9), "t7": range(4, 10)}),
    "binade256": ("binade_dgemm_256", "d", {"b8": range(3, 9), "t7": range(3, 9)}),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name: str):
    from workloads import illcond_operands, kkr_operands, uniform_binade
    if name == "kkr2048":
        A, B = kkr_operands(64, seed=1002)
        return dict(key=name, name="kkr_zgemm_2048", kind="z", A=A, B=B, seed=1002,
                    desc="A = I - T G (64 blocks of 32, |T| log-uniform in [1e-3,1], G decaying "
                         "1/(1+d)), B complex Gaussian")
    if name == "binade256":
        A, B = uniform_binade(256, 256, 256, seed=1001)
        return dict(key=name, name="binade_dgemm_256", kind="d", A=A, B=B, seed=1001,
                    desc="u*2^e, u~U(-1,1), e~U-int[-4,4]")
    if name in ("ill4096", "ill16384"):
        N = 4096 if name == "ill4096" else 16384
        A, B = illcond_operands(N, N, N, seed=1004, rmax=30)
        return dict(key=name, name=WORKLOADS[name][0], kind="z", A=A, B=B, seed=1004,
                    desc="complex Gaussian, rows of A / columns of B scaled by 2^r, "
                         "r~U-int[-30,30]")
    raise SystemExit(f"unknown workload {name}")


def source_hash(paths) -> str:
    """sha256 (first 16 hex digits) of the concatenated kernel sources."""
    h = hashlib.sha256()
    for path in paths:
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(workload_key: str, tune_id: int, slices: int, split: str):
    """HBM bytes per launch of the fused GEMM kernel from the committed counter
    summary, or None when it is missing or was taken on another kernel source,
    tuning id, slice count or slice kind."""
    try:
        vals = {}
        with open(TRAFFIC_SUMMARY.format(workload=workload_key, split=split, slices=slices)) as fh:
            for line in fh:
                if "=" in line and not line.startswith("#"):
                    k, v = line.split("=", 1)
                    vals[k.strip()] = v.strip()
        if vals.get("kernel_source_sha256_16") != source_hash(GEMM_SOURCES):
            return None
        if int(vals.get("tune_id", "-1")) != tune_id:
            return None
        if int(vals.get("slices", "0")) != slices or vals.get("split", "t7") != split:
            return None
        return float(vals["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def cpu_info() -> dict:
    """Host cores and CPU model of the machine the CPU legs run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.lower().startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "model": model, "blas_threads": blas_threads(),
            "omp_threads": int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()}


def blas_threads() -> int:
    try:
        from threadpoolctl import threadpool_info
        return max([p.get("num_threads", 1) for p in threadpool_info()
                    if p.get("user_api") == "blas"] or [1])
    except Exception:   # noqa: BLE001
        return os.cpu_count() or 1


def upload_colmajor(X, dev):
    """Column-major device copy of the row-major host matrix X: uploaded as it
    is, then transposed on the device (a (cols, rows) row-major tensor)."""
    import torch
    t = torch.from_numpy(X).to(dev)
    out = t.t().contiguous()
    del t
    return out


# ------------------------------------------------------------------ records
def single_record(wl, m, n, k, cplx, method, split, s, steps, warmup, ms_per_step, phases,
                  roofline, cpu, native_rec, accuracy, tuning, alternatives=None, interposer=None):
    """The JSON record of a single-product workload."""
    flops = (8.0 if cplx else 2.0) * m * n * k
    value = flops / (ms_per_step * 1e-3) / 1e12
    ozaki2 = method == "ozaki2"
    pairs = s if ozaki2 else s * (s + 1) // 2
    return {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(ms_per_step, 4),
        "us_per_call": round(ms_per_step * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8",
        "data": "synthetic",
        "config": {"workload": wl["name"], "m": m, "n": n, "k": k,
                   "operands": "complex128" if cplx else "float64",
                   "method": method,
                   **({} if ozaki2 else {"split": split}),
                   ("moduli" if ozaki2 else "slices"): s,
                   ("int8_products" if ozaki2 else "pairs"): pairs,
                   "seed": wl["seed"], "inputs": wl["desc"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "native_fp64": native_rec,
        "speedup_vs_native": (round(native_rec["ms_per_call"] / ms_per_step, 3)
                              if native_rec else None),
        "phases_ms": {p: round(v, 4) for p, v in phases.items() if ozaki2 or p != "recon"},
        "interposer": interposer,
        "tuning": tuning,
        "accuracy": accuracy,
        "alternatives": alternatives,
    }


def roofline_record(int8_ops, gemm_ms, kernel, traffic):
    achieved = int8_ops / (gemm_ms * 1e-3) / 1e12
    return {"bound": "mfma", "achieved": round(achieved, 2), "peak": INT8_PEAK_TOPS,
            "unit": "TFLOP/s", "frac": round(achieved / INT8_PEAK_TOPS, 4),
            "traffic": traffic, "kernel": kernel,
            "ops_per_launch": int8_ops, "avg_launch_ms": round(gemm_ms, 4),
            "note": "INT8 MFMA work counted as 2 ops per multiply-add against the "
                    "5000 TOP/s dense INT8 peak"}


def batched_record(nb, s, flops, ms_range, steps, warmup, graph_ms, eager_ms, phases, roofline,
                   cpu):
    return {
        "metric": METRIC, "value": round(flops / (graph_ms * 1e-3) / 1e12, 3), "unit": "TFLOP/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": round(graph_ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int8",
        "data": "synthetic",
        "config": {"workload": "batched_zgemm_512", "problems": nb, "slices": s,
                   "sum_8mnk": flops, "m_range": ms_range, "seed": 1003,
                   "inputs": "m,n,k in 32..1024 (P(32j) ~ 1/j); per-matrix exponent spread "
                             "U[0,20] binades"},
        "roofline": roofline, "cpu_baseline": cpu,
        "eager_ms_per_step": round(eager_ms, 4), "graph_ms_per_step": round(graph_ms, 4),
        "phases_ms": {p: round(v, 4) for p, v in phases.items() if p != "recon"},
    }


def selector_record(flops, steps, target, selector_name, margin, kappa, res):
    return {
        "metric": METRIC, "value": round(flops / (res["ms_learned"] * 1e-3) / 1e12, 3),
        "unit": "TFLOP/s", "n_gpus": 1, "steps": steps, "warmup": 1,
        "ms_per_step": round(res["ms_learned"], 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int8", "data": "synthetic",
        "config": {"workload": "batched_zgemm_512_learned_slices", "target_err_comp": target,
                   "selector": selector_name, "margin": margin, "kappa": kappa, "seed": 1003},
        "roofline": None, "cpu_baseline": None, "selector": res,
    }


def lu_record(n, nb, split, s, steps, warmup, ms, ms_nat, dev_err, errs, resid):
    flops = 8.0 * n ** 3      # complex LU (8/3 n^3) + inverse from the factors (16/3 n^3)
    return {
        "metric": "effective FP64 TFLOP/s, blocked LU + inverse of the KKR matrix (8 n^3 flops)",
        "value": round(flops / (ms * 1e-3) / 1e12, 3), "unit": "TFLOP/s", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int8",
        "data": "synthetic",
        "config": {"workload": "kkr_lu_inverse_2048", "n": n, "nb": nb, "split": split,
                   "slices": s, "seed": 1002},
        "native_updates": {"ms_per_step": round(ms_nat, 4),
                           "tflops": round(flops / (ms_nat * 1e-3) / 1e12, 3)},
        "inverse_deviation_from_native": dev_err,
        "inverse_deviation_by_slices": errs,
        "residual_max_abs_XA_minus_I": resid,
        "roofline": None, "cpu_baseline": None,
    }


# ------------------------------------------------------------------ main
def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    # the GPU clock ramps up over the first tens of milliseconds of load
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--slices", type=int, default=None,
                    help="slice count (default: the smallest s meeting 1e-12 in the sweep; "
                         "6 with --split b8 and 7 with --split t7 when the sweep is skipped)")
    ap.add_argument("--split", choices=["auto", "t7", "b8"], default="auto",
                    help="Ozaki-I slice kind: the faster of the two at its smallest s meeting "
                         "1e-12 (default), 8-bit balanced or trunc-7 slices")
    ap.add_argument("--moduli", type=int, default=None,
                    help="run the Ozaki-II (CRT) path with this many moduli instead of Ozaki-I")
    ap.add_argument("--workload", default="ill16384",
                    choices=sorted(WORKLOADS) + ["batched512", "selector512", "kkrinv2048"])
    ap.add_argument("--nb", type=int, default=128, help="kkrinv2048: LU panel width")
    ap.add_argument("--selector", default=os.path.join(ROOT, "paper_2603_29975_amd",
                                                         "selector_weights.npz"),
                    help="trained selector weights (selector512 workload)")
    ap.add_argument("--kappa", type=float, default=None,
                    help="selector512: probe safety factor (default: the one stored with "
                         "the weights)")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle leg (slice sweep against double-double, CPU timing)")
    ap.add_argument("--cpu-seconds", type=float, default=8.0,
                    help="target CPU time of each timed oracle sample")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the slice sweep (accuracy only at the timed s and s - 1)")
    ap.add_argument("--no-native", action="store_true")
    ap.add_argument("--interposer", action="store_true",
                    help="also time the Fortran-BLAS interposer on host copies of the operands "
                         "(PCIe transfers included)")
    ap.add_argument("--tune", choices=["cache", "auto", "off"], default="cache",
                    help="tile selection: the committed tuning table (autotune if it is "
                         "missing), autotune now, or the default id")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one plain device copy of this size (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the emulator runs on a single MI355X and has no "
              "multi-GPU path (--gpus must be 1).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2603_29975_amd as oz

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    oz.library()   # fails loudly if the HIP library is not built
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload in ("batched512", "selector512") and args.slices is None:
        args.slices = 7          # the batched path uses 7-bit slices
    if args.workload == "kkrinv2048":
        return run_lu(args)
    if args.workload == "batched512":
        return run_batched(args)
    if args.workload == "selector512":
        return run_selector(args)
    return run_single(args)


def run_single(args):
    import numpy as np
    import torch
    import paper_2603_29975_amd as oz

    dev = torch.device("cuda:0")
    t_gen = time.perf_counter()
    wl = workload(args.workload)
    A, B = wl["A"], wl["B"]
    kind = wl["kind"]
    m, k = A.shape
    n = B.shape[1]
    cplx = kind == "z"
    ozaki2 = args.moduli is not None
    log(f"workload {wl['name']} m={m} n={n} k={k}: operands drawn in "
        f"{time.perf_counter() - t_gen:.1f} s")
    Ad = upload_colmajor(A, dev)
    Bd = upload_colmajor(B, dev)
    tdt = torch.complex128 if cplx else torch.float64
    Cd = torch.zeros((n, m), dtype=tdt, device=dev)
    Cn = torch.zeros((n, m), dtype=tdt, device=dev)
    native = oz.ozaki_native_zgemm if cplx else oz.ozaki_native_dgemm
    flops = (8.0 if cplx else 2.0) * m * n * k          # effective FP64 flops per call
    oracle = not args.no_cpu_baseline

    def gemm_fn(split):
        if ozaki2:
            return oz.ozaki2_zgemm if cplx else oz.ozaki2_dgemm
        return oz.ozaki_zgemm if cplx else oz.ozaki_dgemm

    def run_ozaki(split, slices, out=Cd):
        if not ozaki2 and oz.ozaki_set_split(split) != 0:
            raise SystemExit(f"unknown split {split}")
        fn = gemm_fn(split)
        rc = fn("N", "N", m, n, k, 1.0, Ad, m, Bd, k, 0.0, out, m, slices)
        if rc != 0:
            raise RuntimeError(f"{fn.__name__}: {oz.ozaki_status_string(rc)}")

    def run_native():
        rc = native("N", "N", m, n, k, 1.0, Ad, m, Bd, k, 0.0, Cn, m)
        if rc != 0:
            raise RuntimeError(f"{native.__name__}: {oz.ozaki_status_string(rc)}")

    def wall(fn, reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps

    if not ozaki2:
        load_tiles(oz, args.tune)

    # ------------------------------------------------ oracle leg: sampled dd reference
    sref = None
    ref_thread = None
    holder = {}
    if oracle:
        from oracle.sampled import SampledReference, sample_entries
        Bt_host = Bd.cpu().numpy()      # op(B)^T row-major, the layout dd wants
        small = m * n <= (1 << 18)      # small products: every entry
        ref_args = dict(nrand=0 if small else 4096, nrows=m if small else 4,
                        ncols=0 if small else 4, seed=2024)
        ri, cj, _, _ = sample_entries(m, n, **ref_args)

        def build_ref():
            t0 = time.perf_counter()
            holder["ref"] = SampledReference(A, Bt=Bt_host, **ref_args)
            holder["seconds"] = time.perf_counter() - t0

        # runs on the host cores while the GPU sweeps (ctypes releases the GIL)
        ref_thread = threading.Thread(target=build_ref)
        ref_thread.start()

    def join_ref():
        ref_thread.join()
        if "ref" not in holder:
            raise RuntimeError("double-double reference failed")
        log(f"double-double reference on {holder['ref'].count} sampled entries: "
            f"{holder['seconds']:.1f} s")
        return holder["ref"]

    # ------------------------------------------------ slice sweep
    sweep = {}
    samples = {}
    if oracle and not args.no_sweep and not ozaki2:
        ri_d = torch.from_numpy(ri).to(dev)
        cj_d = torch.from_numpy(cj).to(dev)
        splits = ["b8", "t7"] if args.split == "auto" else [args.split]
        big = flops > 1e12
        timing = {}
        for split in splits:
            for s in WORKLOADS[args.workload][2][split]:
                run_ozaki(split, s)                       # untimed: warms up, fills C
                samples[(split, s)] = Cd[cj_d, ri_d].cpu().numpy()
                timing[(split, s)] = wall(lambda: run_ozaki(split, s), 2 if big else 20)
                log(f"sweep {split} s={s}: {timing[(split, s)]:.3f} ms")
        sref = join_ref()
        for (split, s), ms_s in timing.items():
            err = sref.err_comp(samples[(split, s)])
            sweep.setdefault(split, {})[s] = {"err_comp": err, "ms": round(ms_s, 4),
                                              "tflops": round(flops / (ms_s * 1e-3) / 1e12, 2)}
            log(f"sweep {split} s={s}: err_comp {err:.3e}  {sweep[split][s]['tflops']} TFLOP/s")

    # ------------------------------------------------ the timed configuration
    def min_s(split):
        ok = [s for s, r in sweep.get(split, {}).items() if r["err_comp"] <= TARGET]
        return min(ok) if ok else None

    candidates = []
    if ozaki2:
        candidates = [(None, args.moduli)]
    elif args.slices is not None:
        candidates = [("b8" if args.split == "auto" else args.split, args.slices)]
    elif sweep:
        for split in sweep:
            s = min_s(split)
            if s is not None:
                candidates.append((split, s))
        if not candidates:
            raise RuntimeError("no slice count in the sweep reaches 1e-12")
    else:
        split = "b8" if args.split == "auto" else args.split
        candidates = [(split, 6 if split == "b8" else 7)]

    results = {}
    for split, s in candidates:
        tuning = None if ozaki2 else tile_id(oz, args.tune, kind, m, n, k, s, split)
        for _ in range(args.warmup):
            run_ozaki(split, s)
        torch.cuda.synchronize()
        oz.ozaki_timing_enable(True)
        oz.ozaki_timing_read()                               # clear
        ms = wall(lambda: run_ozaki(split, s), args.steps)
        rc, phase_ms, calls = oz.ozaki_timing_read()
        oz.ozaki_timing_enable(False)
        if rc != 0 or calls != args.steps:
            raise RuntimeError(f"phase timing failed: rc={rc} calls={calls}")
        phases = {p: v / args.steps for p, v in phase_ms.items()}
        results[(split, s)] = (ms, phases, tuning)
        log(f"ozaki {split or 'crt'} s={s}: {ms:.3f} ms/call  "
            f"{flops / (ms * 1e-3) / 1e12:.2f} eff TFLOP/s  phases {phases}")
    best = min(results, key=lambda key: results[key][0])
    split, s = best
    ms_per_step, phases, tuning = results[best]
    alternatives = {f"{sp or 'crt'}_s{sv}": {"ms_per_step": round(r[0], 4),
                                            "tflops": round(flops / (r[0] * 1e-3) / 1e12, 3)}
                    for (sp, sv), r in results.items()}
    run_ozaki(split, s)                                   # leave the timed product in C
    pairs = s if ozaki2 else s * (s + 1) // 2
    int8_ops = pairs * flops
    if ozaki2:
        kernel = (f"fused INT8 modular products over {s} moduli + CRT rebuild + FP64 epilogue "
                  "(k_oz2gemm); the residue kernels are timed in phases_ms")
        traffic = None
    else:
        kernel = ("fused INT8 slice-pair GEMM + FP64 recombination (k_ozgemm, tuning id "
                  f"{tuning['tune_id']})")
        traffic = read_traffic(args.workload, tuning["tune_id"], s, split)
    roofline = roofline_record(int8_ops, phases["gemm"], kernel, traffic)

    # ------------------------------------------------ native FP64 on the same buffers
    native_rec = None
    if not args.no_native:
        run_native()
        torch.cuda.synchronize()
        t1 = wall(run_native, 1)
        reps = max(2, min(args.steps, int(4000.0 / max(t1, 1e-3))))
        nms = wall(run_native, reps)
        ntf = flops / (nms * 1e-3) / 1e12
        native_rec = {"kernel": "k_native (FP64 MFMA)", "ms_per_call": round(nms, 4),
                      "calls": reps, "tflops": round(ntf, 2),
                      "frac_of_fp64_peak": round(ntf / FP64_PEAK_TFLOPS, 4)}
        log(f"native: {nms:.3f} ms/call  {ntf:.2f} TFLOP/s")
        # context: the vendor library's FP64 GEMM on the same buffers (torch.matmul,
        # i.e. rocBLAS); C^T = op(B)^T op(A)^T in the row-major view of the buffers
        Cl = torch.empty_like(Cn)
        lib = lambda: torch.matmul(Bd, Ad, out=Cl)
        lib()
        torch.cuda.synchronize()
        lms = wall(lib, reps)
        del Cl
        native_rec["vendor_library_fp64"] = {
            "kernel": "torch.matmul (rocBLAS) on the same buffers, for context",
            "ms_per_call": round(lms, 4), "tflops": round(flops / (lms * 1e-3) / 1e12, 2)}
        log(f"vendor library FP64: {lms:.3f} ms/call  {flops / (lms * 1e-3) / 1e12:.2f} TFLOP/s")

    # ------------------------------------------------ host-BLAS interposer
    interposer = None
    if args.interposer:
        interposer = time_interposer(oz, A, B, Cd, m, n, k, cplx, ozaki2, s, args.steps,
                                     flops, None if ozaki2 else split)

    if args.copy_calibration_mib:
        nb = args.copy_calibration_mib << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        log(f"copy calibration: {nb} bytes read, {nb} bytes written (torch.neg)")

    # ------------------------------------------------ oracle leg: accuracy and CPU baseline
    cpu = None
    accuracy = None
    if oracle:
        if sref is None:
            sref = join_ref()
        accuracy = accuracy_record(oz, torch, sref, Cd, Cn if native_rec else None, sweep,
                                   samples, split, s, ozaki2, run_ozaki, A, B, m, n)
        cpu = cpu_baseline(wl, A, B, m, n, k, split, s, ozaki2, args.cpu_seconds)

    out = single_record(wl, m, n, k, cplx, "ozaki2" if ozaki2 else "ozaki1", split, s,
                        args.steps, args.warmup, ms_per_step, phases, roofline, cpu, native_rec,
                        accuracy, tuning, alternatives, interposer)
    print(json.dumps(out), flush=True)


def load_tiles(oz, mode):
    oz.ozaki_tune_clear()
    if mode == "cache" and os.path.exists(TUNE_CACHE):
        rc = oz.ozaki_tune_load(TUNE_CACHE)
        if rc != 0:
            raise RuntimeError(f"ozaki_tune_load: {oz.ozaki_status_string(rc)}")


def tile_id(oz, mode, kind, m, n, k, s, split):
    """Tile selection for the workload shape, outside the timed region."""
    oz.ozaki_set_split(split)
    source = "cache" if mode == "cache" and os.path.exists(TUNE_CACHE) else "default"
    if mode == "auto" or (mode == "cache" and source == "default"):
        rc, _, _ = oz.ozaki_autotune(kind, m, n, k, s, reps=5)
        if rc != 0:
            raise RuntimeError(f"ozaki_autotune: {oz.ozaki_status_string(rc)}")
        source = "autotune"
    tid = oz.ozaki_tune_get(kind, m, n, k, s)
    log(f"tiles: tuning id {tid} ({source})")
    return {"tune_id": tid, "source": source, "ids": oz.ozaki_tune_configs()}


def accuracy_record(oz, torch, sref, Cd, Cn, sweep, samples, split, s, ozaki2, run_ozaki, A, B,
                    m, n):
    """err_comp of the timed product (and of the previous slice count, and of
    the native FP64 product) against the sampled double-double reference, and
    an 8 x 8 block of the timed product bit for bit against the oracle model."""
    import numpy as np
    from oracle import ozaki as ozaki_model
    from oracle import ozaki2 as ozaki2_model
    from oracle import ozaki_b8
    dev = Cd.device
    ri_d = torch.from_numpy(sref.ri).to(dev)
    cj_d = torch.from_numpy(sref.cj).to(dev)
    torch.cuda.synchronize()
    err_s = sref.err_comp(Cd[cj_d, ri_d].cpu().numpy())
    if (split, s - 1) in samples:
        err_prev = sref.err_comp(samples[(split, s - 1)])
    elif s > (2 if ozaki2 else 1):
        Cprev = torch.zeros_like(Cd)
        run_ozaki(split, s - 1, Cprev)
        torch.cuda.synchronize()
        err_prev = sref.err_comp(Cprev[cj_d, ri_d].cpu().numpy())
        del Cprev
        run_ozaki(split, s)
    else:
        err_prev = None
    err_native = sref.err_comp(Cn[cj_d, ri_d].cpu().numpy()) if Cn is not None else None
    model = (ozaki2_model.ozaki2_gemm if ozaki2 else
             ozaki_b8.ozaki_gemm_b8 if split == "b8" else ozaki_model.ozaki_gemm)
    rng = np.random.default_rng(2025)
    rs = np.sort(np.concatenate([rng.choice(m, 7, replace=False), [m - 1]]))
    cs = np.sort(np.concatenate([rng.choice(n, 7, replace=False), [n - 1]]))
    torch.cuda.synchronize()
    got = Cd[torch.from_numpy(cs).to(dev)][:, torch.from_numpy(rs).to(dev)].cpu().numpy().T
    ref = model("N", "N", A[rs], B[:, cs], s)
    exact = bool(np.array_equal(np.ascontiguousarray(got).view(np.uint64),
                                np.ascontiguousarray(ref).view(np.uint64)))
    table = {sp: {str(sv): r for sv, r in rows.items()} for sp, rows in sweep.items()}
    min_s = {sp: min([sv for sv, r in rows.items() if r["err_comp"] <= TARGET], default=None)
             for sp, rows in sweep.items()}
    log(f"accuracy: err_comp({s}) {err_s:.3e}  ({s - 1}) {err_prev}  native {err_native}  "
        f"bit-exact 8x8 {exact}")
    return {"err_comp_sampled": err_s, "err_comp_sampled_s_minus_1": err_prev,
            "err_comp_native_fp64": err_native, "entries": sref.count,
            "sample": f"{sref.count - sref.rows.size * n - sref.cols.size * m} random entries + "
                      f"{sref.rows.size} whole rows + {sref.cols.size} whole columns",
            "reference": "double-double (oracle)", "target": TARGET,
            "meets_target": bool(err_s <= TARGET), "oracle_bit_exact_8x8": exact,
            "min_slices_at_target": min_s, "by_slices": table}


def cpu_baseline(wl, A, B, m, n, k, split, s, ozaki2, target_s):
    """The oracle timed on bounded samples of the same workload on the host
    cores: its emulation model (the reported value), its double-double
    reference and plain host-BLAS FP64 GEMM (numpy.matmul, not this project's
    code). Each sample is a block of rows of op(A) against a block of columns
    of op(B) over the whole contraction, doubled until it takes about
    target_s seconds."""
    import numpy as np
    from oracle import dd
    from oracle import ozaki as ozaki_model
    from oracle import ozaki2 as ozaki2_model
    from oracle import ozaki_b8
    cplx = np.iscomplexobj(A)
    per = 8.0 if cplx else 2.0
    model = (ozaki2_model.ozaki2_gemm if ozaki2 else
             ozaki_b8.ozaki_gemm_b8 if split == "b8" else ozaki_model.ozaki_gemm)

    def grow(fn, r0, rmax_r, cmax_c):
        r, c = r0, r0
        while True:
            t0 = time.perf_counter()
            fn(r, c)
            t = time.perf_counter() - t0
            if t >= target_s / 2.5 or (r >= rmax_r and c >= cmax_c):
                return r, c, t
            if c < cmax_c:
                c = min(2 * c, cmax_c)
            if r < rmax_r and (c >= cmax_c or r < c):
                r = min(2 * r, rmax_r)

    r, c, t = grow(lambda r, c: model("N", "N", A[:r], B[:, :c], s), 4, m, n)
    info = cpu_info()
    what = f"moduli={s}" if ozaki2 else f"{split} s={s}"
    emul = {"value": round(per * r * c * k / t / 1e12, 9), "unit": "TFLOP/s",
            "cores": info["blas_threads"], "kind": "oracle",
            "sample": f"oracle emulation model ({what}; numpy + host BLAS on integer slices) on "
                      f"rows 0..{r - 1} of op(A) x columns 0..{c - 1} of op(B), k={k}: "
                      f"{r}x{c}x{k} in {t:.2f} s"}
    rd, cd, td = grow(lambda r, c: dd.dd_gemm("N", "N", A[:r], B[:, :c]), 2, m, n)
    dd_rec = {"value": round(per * rd * cd * k / td / 1e12, 9), "unit": "TFLOP/s",
              "threads": dd.threads_used(),
              "sample": f"double-double GEMM (oracle, C/OpenMP) on {rd}x{cd}x{k} in {td:.2f} s"}
    rb, cb, tb = grow(lambda r, c: np.matmul(A[:r], B[:, :c]), 64, m, n)
    blas = {"value": round(per * rb * cb * k / tb / 1e12, 6), "unit": "TFLOP/s",
            "threads": info["blas_threads"],
            "sample": f"numpy.matmul FP64 on {rb}x{cb}x{k} in {tb:.2f} s"}
    out = dict(emul)
    out.update({"host": info, "dd_reference": dd_rec, "host_blas_fp64": blas})
    log(f"cpu baseline: {out}")
    return out


def time_interposer(oz, A, B, Cd, m, n, k, cplx, ozaki2, s, steps, flops, split):
    import numpy as np
    from paper_2603_29975_amd import blas
    if split is not None:
        oz.ozaki_set_split(split)
    blas.ozaki_blas_config(0 if ozaki2 else s, s if ozaki2 else 0)
    Ah, Bh = np.asfortranarray(A), np.asfortranarray(B)
    Ch = np.zeros((m, n), dtype=A.dtype, order="F")
    host_gemm = blas.zgemm_ if cplx else blas.dgemm_
    for _ in range(2):
        host_gemm("N", "N", m, n, k, 1.0, Ah, m, Bh, k, 0.0, Ch, m)
    reps = max(3, steps // 4)
    t0 = time.perf_counter()
    for _ in range(reps):
        host_gemm("N", "N", m, n, k, 1.0, Ah, m, Bh, k, 0.0, Ch, m)
    ims = (time.perf_counter() - t0) * 1e3 / reps
    dev_c = np.ascontiguousarray(Cd.cpu().numpy().T)
    same = bool(np.array_equal(np.ascontiguousarray(Ch).view(np.uint64), dev_c.view(np.uint64)))
    rec = {"ms_per_call": round(ims, 4), "tflops": round(flops / (ims * 1e-3) / 1e12, 2),
           "calls": reps, "bit_identical_to_device_call": same,
           "note": "zgemm_/dgemm_ on pageable host arrays: copies of A, B to HBM and "
                   "of C back included"}
    blas.ozaki_blas_release()
    log(f"interposer: {rec}")
    return rec


def run_batched(args):
    """512 independent complex GEMMs (m, n, k in 32..1024, log-uniform; per
    matrix exponent spread U[0, 20] binades; seed 1003) at fixed s in one
    ozaki_zgemm_batched call: batched scan, batched split, grouped persistent
    GEMM, replayed from a captured HIP graph."""
    import numpy as np
    import torch
    import paper_2603_29975_amd as oz
    from workloads import batched_problems

    s = args.slices
    probs, (ms, ns, ks) = batched_problems(512, 1003)
    nb = len(probs)
    log(f"workload batched512: {nb} problems, s={s}")
    Ad = [torch.from_numpy(np.ascontiguousarray(A.T)).cuda() for A, _ in probs]
    Bd = [torch.from_numpy(np.ascontiguousarray(B.T)).cuda() for _, B in probs]
    Cd = [torch.zeros((int(n), int(m)), dtype=torch.complex128, device="cuda") for m, n in zip(ms, ns)]
    flops = float(np.sum(8.0 * ms * ns * ks))
    pairs = s * (s + 1) // 2
    call_args = (["N"] * nb, ["N"] * nb, list(ms), list(ns), list(ks), [1.0] * nb, Ad, list(ms),
                 Bd, list(ks), [0.0] * nb, Cd, list(ms), nb, [s] * nb)

    def run():
        rc = oz.ozaki_zgemm_batched(*call_args)
        if rc != 0:
            raise RuntimeError(f"ozaki_zgemm_batched: {oz.ozaki_status_string(rc)}")

    def timed(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            run()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    # eager launches with per-phase events (same kernels as the graph)
    oz.ozaki_batched_graphs(False)
    for _ in range(args.warmup):
        run()
    oz.ozaki_timing_enable(True)
    oz.ozaki_timing_read()
    eager_ms = timed(args.steps)
    rc, phase_ms, calls = oz.ozaki_timing_read()
    oz.ozaki_timing_enable(False)
    phases = {p: v / max(calls, 1) for p, v in phase_ms.items()}
    # graph replay: the measured configuration
    oz.ozaki_batched_graphs(True)
    for _ in range(args.warmup):
        run()
    graph_ms = timed(args.steps)
    log(f"batched: graph {graph_ms:.3f} ms  eager {eager_ms:.3f} ms  "
        f"{flops / (graph_ms * 1e-3) / 1e12:.2f} eff TFLOP/s  phases {phases}")
    roofline = roofline_record(pairs * flops, phases["gemm"],
                               "k_ozgemm grouped (persistent over all problems' tiles)", None)
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import ozaki
        t0 = time.perf_counter()
        done_flops = 0.0
        cnt = 0
        for b in range(nb):
            A, B = probs[b]
            ozaki.ozaki_gemm("N", "N", A, B, s)
            done_flops += 8.0 * A.shape[0] * B.shape[1] * A.shape[1]
            cnt += 1
            if time.perf_counter() - t0 > args.cpu_seconds:
                break
        t = time.perf_counter() - t0
        info = cpu_info()
        cpu = {"value": round(done_flops / t / 1e12, 6), "unit": "TFLOP/s",
               "cores": info["blas_threads"], "kind": "oracle",
               "sample": f"oracle Ozaki model on the first {cnt} of the {nb} problems, s={s}, "
                         f"{t:.2f} s",
               "host": info}
    out = batched_record(nb, s, flops, [int(ms.min()), int(ms.max())], args.steps, args.warmup,
                         graph_ms, eager_ms, phases, roofline, cpu)
    print(json.dumps(out), flush=True)


def run_selector(args):
    """Learned slice selection (+ residual probe) against the best fixed slice
    count on the 512-problem batch, at a componentwise target of 1e-11."""
    import numpy as np
    from paper_2603_29975_amd import selector
    from workloads import batched_problems
    theta, margin, target, meta = selector.load(args.selector, with_meta=True)
    kappa = args.kappa if args.kappa is not None else float(meta.get("kappa", selector.KAPPA))
    res = selector.evaluate_gain(theta, margin, target, kappa=kappa, steps=args.steps, log=log)
    _, (ms, ns, ks) = batched_problems(512, 1003)
    flops = float(np.sum(8.0 * ms * ns * ks))
    out = selector_record(flops, args.steps, target, os.path.basename(args.selector), margin,
                          kappa, res)
    print(json.dumps(out), flush=True)


def run_lu(args):
    """Blocked LU + inverse of the 2048 x 2048 KKR matrix A = I - T G (seed 1002)
    with emulated trailing updates, beside the same algorithm with the native
    FP64 ZGEMM; reports the inverse's deviation from the native-update inverse."""
    import numpy as np
    import torch
    import paper_2603_29975_amd as oz
    from workloads import kkr_operands
    split = "b8" if args.split == "auto" else args.split
    if args.slices is None:
        args.slices = 6 if split == "b8" else 7
    s = args.slices
    if oz.ozaki_set_split(split) != 0:
        raise SystemExit(f"unknown split {split}")
    load_tiles(oz, args.tune)
    A, _ = kkr_operands(64, seed=1002)
    n = A.shape[0]
    dev = torch.device("cuda:0")
    A0 = torch.from_numpy(np.ascontiguousarray(A.T)).to(dev)
    W = torch.empty_like(A0)
    X = torch.empty_like(A0)
    ipiv = torch.zeros(n, dtype=torch.int64, device=dev)
    log(f"workload kkrinv2048: n={n} nb={args.nb} split={split} s={s}")

    def step(slices):
        W.copy_(A0)
        rc = oz.ozaki_zgetrf(n, W, n, ipiv, args.nb, slices)
        if rc != 0:
            raise RuntimeError(f"ozaki_zgetrf: {oz.ozaki_status_string(rc)}")
        rc = oz.ozaki_zgetri(n, W, n, ipiv, X, n, args.nb, slices)
        if rc != 0:
            raise RuntimeError(f"ozaki_zgetri: {oz.ozaki_status_string(rc)}")

    def timed(slices):
        for _ in range(args.warmup):
            step(slices)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(slices)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / args.steps

    ms_nat = timed(0)
    X_nat = X.clone()
    ms = timed(s)
    scale = X_nat.abs().max().item()
    dev_err = (X - X_nat).abs().max().item() / scale
    eye = torch.eye(n, dtype=A0.dtype, device=dev)
    resid = (X.T @ A0.T - eye).abs().max().item()         # row-major views: (A^-1 A)^T
    errs = {}
    for sv in range(max(3, s - 2), s + 2):
        if sv > S_MAX[split]:
            continue
        step(sv)
        errs[sv] = (X - X_nat).abs().max().item() / scale
    out = lu_record(n, args.nb, split, s, args.steps, args.warmup, ms, ms_nat, dev_err, errs,
                    resid)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
