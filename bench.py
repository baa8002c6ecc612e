#!/usr/bin/env python3
"""Throughput of the Triad-ATRG coarse-graining step (4D Ising) on one MI355X.

Workload: chi = 32, r = 3 (L = 96), q = 2, beta = 0.1496947, seed 0, 40 RG steps (a periodic
lattice of 2^40 sites) -- the configuration the headline metric is quoted on.  A "step" is
one full RG step of the hot path (canonical form, bond swap, isometries, triad tensors,
squeezers, contraction, rotation), all on the device; inputs are resident in HBM when the
timed region starts.  W untimed warm-up steps, then exactly K timed steps, bracketed by
device synchronisation; W + K <= 64 (W + K = 40 gives the full run and its free energy,
compared with the FP64 oracle when tests/golden/C3.json is present).

The headline line is the split-precision path (contraction GEMMs as three bf16 planes per
operand, six products on the BF16 matrix cores with FP32 accumulation; everything else in
FP64); the plain FP64 path is timed beside it on the same device (`fp64_path`).

Prints one JSON line.  `roofline` reports the contraction GEMMs of Eqs. (makeMG)/(makeMH)
(2 L^2 chi^5 flops per launch, four launches per step) timed live with HIP events on the
library's stream; on the split path the executed bf16 work is six times that and is priced
against the BF16 peak.  `cpu_baseline` times the FP64 oracle on the host's cores on a
bounded sample (see its "sample" field).
"""
import argparse
import json
import os
import sys
import time

CPU_THREADS = max(1, min(16, os.cpu_count() or 1))
os.environ.setdefault("OPENBLAS_NUM_THREADS", str(CPU_THREADS))
os.environ.setdefault("OMP_NUM_THREADS", str(CPU_THREADS))

HERE = os.path.dirname(os.path.abspath(__file__))
FP64_PEAK_TFLOPS = 78.6          # MI355X dense FP64 matrix peak
BF16_PEAK_TFLOPS = 2500.0        # MI355X dense BF16 matrix peak
METRIC = "Triad-ATRG RG steps/s at chi=32, MFMA TFLOP/s %peak, |delta f| vs FP64 oracle"


def model_flops_per_step(chi, r, q):
    """Leading-order algorithmic flops of one RG step (swap products on the full cell middle,
    Grams, squeezers, contraction), float64 multiply-adds counted as 2."""
    L = min(r * chi, chi * chi)
    ls = min(r * chi, chi ** 4)
    c5, c6, c7 = chi ** 5, chi ** 6, chi ** 7
    swap = (2 * q + 2) * 4 * c6 * ls          # products with the cell middle M
    iso = 4 * 2 * c7                          # four Grams over chi^3
    sqz = 6 * 2 * 2 * c7 + 4 * 2 * L * c5     # pair Grams and projected tensors
    contraction = 8 * L * L * c5 + 4 * L * c5 + 4 * L * L * chi ** 4
    return swap + iso + sqz + contraction, contraction


def cpu_baseline(chi, r, q, seed):
    """Time the oracle's contraction stage (Eqs. (makeMG)/(makeMH)) of one step at the
    benchmark's shapes, on random inputs of those shapes."""
    import numpy as np
    sys.path.insert(0, HERE)
    from oracle import tatrg as t
    L = min(r * chi, chi * chi)
    rng = np.random.default_rng(seed)
    e = rng.standard_normal((chi, L, chi, chi))
    f = rng.standard_normal((chi, L, chi, chi))
    g = rng.standard_normal((chi, L, chi, chi))
    h = rng.standard_normal((chi, L, chi, chi))
    us = [np.linalg.qr(rng.standard_normal((chi * chi, L)))[0].reshape(chi, chi, L)
          for _ in range(4)]
    sq = {mu: (rng.standard_normal((chi, chi, chi)), rng.standard_normal((chi, chi, chi)), None)
          for mu in (2, 3, 4)}
    t0 = time.perf_counter()
    t.contract(e, f, g, h, us[0], us[1], us[2], us[3], sq)
    dt = time.perf_counter() - t0
    return {"value": 1.0 / dt, "unit": "RG steps/s", "cores": CPU_THREADS, "kind": "oracle",
            "seconds": dt,
            "sample": "oracle contraction stage (Eqs. makeMG/makeMH) of one chi=32 r=3 RG step "
                      "on random inputs of the step's shapes; the other stages of the step "
                      "are excluded, so this is an upper bound on the oracle's RG steps/s"}


TRAFFIC_PROFILE = os.path.join(HERE, "profiles", "contraction_gemm_bf16x3_chi32.md")
KERNEL_SOURCE = os.path.join(HERE, "paper_2412_14104_amd", "csrc", "gemm_bf16x3.hip")


def measured_traffic():
    """HBM bytes per launch of the split contraction GEMM, from the rocprofv3 FETCH_SIZE /
    WRITE_SIZE passes recorded in profiles/ (calibrated against a plain copy).  None unless
    the summary was taken on the kernel source as it stands (its SHA-256 is recorded)."""
    import hashlib
    import re
    try:
        with open(TRAFFIC_PROFILE) as fh:
            text = fh.read()
        with open(KERNEL_SOURCE, "rb") as fh:
            digest = hashlib.sha256(fh.read()).hexdigest()
    except OSError:
        return None
    m = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)\s+source_sha256:\s*([0-9a-f]{64})",
                  text)
    if not m or m.group(2) != digest:
        return None
    return float(m.group(1))


def run_path(pkg, torch, precision, chi, r, q, seed, beta, warmup, steps):
    """W untimed steps, then K steps timed with HIP events on the library's stream (bracketed
    by device synchronisation); returns the timing, the live contraction-GEMM timing and, for
    a full run, the free energy."""
    n_total = warmup + steps
    eng = pkg.Engine(chi, r, q, n_total, seed=seed, precision=precision, record_spectra=False)
    st = eng.stream
    eng.init(beta)
    for _ in range(warmup):
        eng.step()
    torch.cuda.synchronize()
    eng.profile_enable(4 * steps)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(st)
    t0 = time.perf_counter()
    for _ in range(steps):
        eng.step()
    ev1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    k_ms, launches, flops_launch = eng.profile_read()
    out = {"ms_per_step": gpu_ms / steps, "value": steps / (gpu_ms / 1e3), "wall_s": wall,
           "contraction_ms": k_ms, "launches": launches, "flops_per_launch": flops_launch}
    if n_total == 40:
        out["f"], out["lnZV"] = eng.free_energy()
    del eng
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=38)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", choices=["bf16x3", "fp64"], default="bf16x3",
                    help="path of the headline line (the other is timed beside it)")
    ap.add_argument("--no-fp64-comparison", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the Triad-ATRG step runs on a single device "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0 or args.steps + args.warmup > 64:
        print("need steps >= 1, warmup >= 0, steps + warmup <= 64", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("no HIP device visible", file=sys.stderr)
        sys.exit(1)
    sys.path.insert(0, HERE)
    import paper_2412_14104_amd as pkg
    from paper_2412_14104_amd.configs import PRESETS

    cfg = PRESETS["C3"]
    chi, r, q, seed = cfg["chi"], cfg["r"], cfg["q"], cfg["seed"]
    beta = cfg["betas"][0]
    n_total = args.warmup + args.steps
    split = args.precision == "bf16x3"
    prec = pkg.BF16X3 if split else pkg.FP64
    main_run = run_path(pkg, torch, prec, chi, r, q, seed, beta, args.warmup, args.steps)
    other = None
    if not args.no_fp64_comparison:
        other = run_path(pkg, torch, pkg.FP64 if split else pkg.BF16X3, chi, r, q, seed, beta,
                         args.warmup, args.steps)

    total_flops, contr_flops = model_flops_per_step(chi, r, q)
    launches = main_run["launches"]
    avg_launch_s = (main_run["contraction_ms"] / launches) / 1e3 if launches else float("nan")
    alg = main_run["flops_per_launch"] / avg_launch_s / 1e12   # 2 M N K per launch
    if split:
        # six bf16 x bf16 products per GEMM on the BF16 matrix cores
        roofline = {"bound": "mfma", "achieved": 6 * alg, "peak": BF16_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": 6 * alg / BF16_PEAK_TFLOPS, "traffic": None,
                    "fp64_equivalent_tflops": alg,
                    "fp64_equivalent_frac_of_fp64_peak": alg / FP64_PEAK_TFLOPS}
    else:
        roofline = {"bound": "mfma", "achieved": alg, "peak": FP64_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": alg / FP64_PEAK_TFLOPS, "traffic": None}
    if split:
        roofline["traffic"] = measured_traffic()
    roofline.update({"kernel": "contraction GEMMs (P = E.FM4 and Phi = Qt^T.P, both halves)",
                     "launches": launches, "flops_per_launch": main_run["flops_per_launch"],
                     "avg_launch_ms": avg_launch_s * 1e3})
    out = {
        "metric": METRIC,
        "value": main_run["value"],
        "unit": "RG steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3+f64" if split else "f64",
        "data": "synthetic",
        "config": {"workload": "4D Ising Triad-ATRG, chi=32, r=3 (L=96), q=2, "
                               "beta=0.1496947, seed 0, RG steps %d" % n_total,
                   "chi": chi, "r": r, "q": q, "beta": beta, "n_steps": n_total,
                   "precision": args.precision},
        "roofline": roofline,
        "step_model_tflops": total_flops * main_run["value"] / 1e12,
        "step_model_flops": total_flops,
        "wall_s": main_run["wall_s"],
    }
    ref = None
    gpath = os.path.join(HERE, "tests", "golden", "C3.json")
    if os.path.exists(gpath):
        with open(gpath) as fh:
            ref = json.load(fh)["runs"][0]
    if "f" in main_run:
        out["f"], out["lnZV"] = main_run["f"], main_run["lnZV"]
        if ref is not None:
            out["delta_f_rel_vs_oracle"] = abs(main_run["f"] - ref["f"]) / abs(ref["f"])
    if other is not None:
        key = "fp64_path" if split else "bf16x3_path"
        o = {"value": other["value"], "ms_per_step": other["ms_per_step"],
             "contraction_avg_launch_ms": other["contraction_ms"] / max(other["launches"], 1)}
        if "f" in other:
            o["f"] = other["f"]
            if ref is not None:
                o["delta_f_rel_vs_oracle"] = abs(other["f"] - ref["f"]) / abs(ref["f"])
            if "f" in main_run:
                out["delta_f_rel_split_vs_fp64_path"] = abs(main_run["f"] - other["f"]) / abs(
                    other["f"])
        out[key] = o
        out["speedup_vs_" + key.split("_")[0]] = main_run["value"] / other["value"]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(chi, r, q, seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
