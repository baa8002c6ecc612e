#!/usr/bin/env python3
"""Throughput of the Triad-ATRG coarse-graining step (4D Ising) on one MI355X.

Workload: chi = 32, r = 3 (L = 96), q = 2, beta = 0.1496947, seed 0, 40 RG steps (a periodic
lattice of 2^40 sites) -- the configuration the headline metric is quoted on.  A "step" is
one full RG step of the hot path (canonical form, bond swap, isometries, triad tensors,
squeezers, contraction, rotation), all on the device; inputs are resident in HBM when the
timed region starts.  W untimed warm-up steps, then exactly K timed steps, bracketed by
device synchronisation; W + K <= 64.  After the timed region the run continues untimed to
40 steps (when W + K <= 40) and its free energy is compared with the FP64 oracle's stored
result (tests/golden/C3.json), on both paths.

The headline line is the split-precision path (contraction GEMMs as three bf16 planes per
operand, six products on the BF16 matrix cores with FP32 accumulation; everything else in
FP64); the plain FP64 path is timed beside it on the same device (`fp64_path`).

Prints one JSON line.  `roofline` reports the contraction GEMMs of Eqs. (makeMG)/(makeMH)
timed live with HIP events on the library's stream: the method's 2 L^2 chi^5 flops per
launch over the mean launch time, against the dense peak of the precision the kernel issues
(BF16 on the split path; `bf16_issue_*` counts the six bf16 products per multiply-add).
`roofline_fp64_stages` prices the FP64 stages S1-S4 (algorithmic flops from
stage_model_flops over their event-timed share of the step) against the FP64 peak;
`stages` gives every stage's time.  `cpu_baseline` times one full RG step of the FP64 oracle
on the host's cores.
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


def widths(chi, r):
    """Internal-line width L = min(r chi, chi^2) and swap sketch width Ls = min(r chi, chi^4)."""
    return min(r * chi, chi * chi), min(r * chi, chi ** 4)


def stage_model_flops(chi, r, q):
    """Leading-order algorithmic flops of the stages of one RG step (one temperature), at the
    steady-state bond dimension chi, multiply-adds counted as 2:
      S0 canonical form            8 chi^6
      S1 bond swap                 8 chi^7 (compression and back-projection of the cell
                                   middle) + (2q + 2)(4 chi^5 Ls + 2 chi^3 Ls^2) (its RSVD)
                                   -- Table 1 prices bond swapping at O(q r chi^6)
      S2 isometries                8 chi^7 + 44 chi^6 (Grams, RSVD ranges)
      S3 triad tensors             8 chi^5 L
      S4 squeezers                 16 chi^7 + 8 chi^5 L + 114 chi^6
      S5 contraction               8 L^2 chi^5 + 4 L chi^5 + 4 L^2 chi^4 + 4 L chi^4
                                   (Eqs. (makeMG), (makeMH): the O(r^2 chi^7) bottleneck)"""
    L, ls = widths(chi, r)
    c3, c4, c5, c6, c7 = chi ** 3, chi ** 4, chi ** 5, chi ** 6, chi ** 7
    return {
        "S0": 8 * c6,
        "S1": 8 * c7 + (2 * q + 2) * (4 * c5 * ls + 2 * c3 * ls * ls),
        "S2": 8 * c7 + 44 * c6,
        "S3": 8 * c5 * L,
        "S4": 16 * c7 + 8 * c5 * L + 114 * c6,
        "S5": 8 * L * L * c5 + 4 * L * c5 + 4 * L * L * c4 + 4 * L * c4,
    }


def model_flops_per_step(chi, r, q):
    """(whole step, contraction) algorithmic flops of one RG step."""
    st = stage_model_flops(chi, r, q)
    return sum(st.values()), st["S5"]


def cpu_baseline(chi, r, q, seed, beta):
    """Time one full RG step of the FP64 oracle (canonical form, swap, isometries, triad,
    squeezers, contraction, rotation) at the benchmark's shapes, from the initial tensor.
    The oracle works on the zero-padded static shapes, so this step costs what any step of
    the run costs."""
    sys.path.insert(0, HERE)
    from oracle import tatrg as t
    phi, psi = t.initial_state(beta, chi)
    t0 = time.perf_counter()
    t.step(phi, psi, 0, chi, r, q, seed)
    dt = time.perf_counter() - t0
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": 1.0 / dt, "unit": "RG steps/s", "cores": CPU_THREADS, "kind": "oracle",
            "seconds": dt, "cpu_model": model, "nproc": os.cpu_count(),
            "sample": "one full RG step of the FP64 numpy/LAPACK oracle at chi=32, r=3, q=2 "
                      "(step 0 from the initial tensor; static zero-padded shapes, so every "
                      "step costs the same), BLAS and generator threads = cores"}


GEMM_PROFILE = os.path.join(HERE, "profiles", "contraction_gemm_bf16x3_chi32.md")
KERNEL_SOURCE = os.path.join(HERE, "paper_2412_14104_amd", "csrc", "gemm_bf16x3.hip")


def profiled_value(key):
    """A per-launch figure of the split contraction GEMM recorded in its rocprofv3 summary
    (profiles/): `traffic_bytes_per_launch` (FETCH_SIZE and WRITE_SIZE passes, calibrated
    against a plain copy) or `mfma_busy_frac` (SQ_VALU_MFMA_BUSY_CYCLES over GRBM_GUI_ACTIVE
    times the SIMD count).  None unless the summary was taken on the kernel source as it
    stands (its SHA-256 is recorded beside the figure)."""
    import hashlib
    import re
    try:
        with open(GEMM_PROFILE) as fh:
            text = fh.read()
        with open(KERNEL_SOURCE, "rb") as fh:
            digest = hashlib.sha256(fh.read()).hexdigest()
    except OSError:
        return None
    m = re.search(re.escape(key) + r":\s*([0-9.eE+-]+)\s+source_sha256:\s*([0-9a-f]{64})", text)
    if not m or m.group(2) != digest:
        return None
    return float(m.group(1))


def run_path(pkg, torch, precision, chi, r, q, seed, beta, warmup, steps, finish=True):
    """W untimed steps, then K steps timed with HIP events on the library's stream (bracketed
    by device synchronisation), then -- untimed, unless finish is False -- the rest of the
    40-step run and its free energy.  Returns the timing, the live contraction-GEMM and stage
    timings and f."""
    n_total = max(warmup + steps, 40) if finish else warmup + steps
    eng = pkg.Engine(chi, r, q, n_total, seed=seed, precision=precision, record_spectra=False)
    st = eng.stream
    eng.init(beta)
    # measured work-group order of the split GEMMs (results do not depend on it); before the
    # warm-up, outside the timed region
    tuned = eng.autotune()
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
    stage_ms, stage_steps = eng.profile_read_stages()
    eng.profile_enable(0)
    swap_paths = [eng.swap_compressed(k) for k in range(warmup + steps)]
    f = lnzv = None
    if finish:
        for _ in range(n_total - warmup - steps):
            eng.step()
        f, lnzv = eng.free_energy()
    out = {"ms_per_step": gpu_ms / steps, "value": steps / (gpu_ms / 1e3), "wall_s": wall,
           "contraction_ms": k_ms, "launches": launches, "flops_per_launch": flops_launch,
           "stage_ms_per_step": [x / max(stage_steps, 1) for x in stage_ms],
           "n_total": n_total, "f": f, "lnZV": lnzv,
           "swap_compressed_timed_steps": sum(1 for p in swap_paths[warmup:] if p == 1),
           "autotune": tuned}
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
    ap.add_argument("--no-finish", action="store_true",
                    help="skip the untimed rest of the 40-step run and the free energy (for "
                         "short profiler runs)")
    ap.add_argument("--split-products", type=int, choices=[3, 6], default=6,
                    help="products per split GEMM: 6 (the engine) or 3 (accuracy ablation, "
                         "i + j <= 1)")
    ap.add_argument("--calibrate-copy", type=int, metavar="MIB", default=0,
                    help="only copy a MIB-sized float64 device buffer three times (a plain "
                         "copy of known size, to calibrate rocprofv3's HBM byte counters) "
                         "and exit")
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
    if args.calibrate_copy > 0:
        n = args.calibrate_copy * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print("copied %d MiB x 3 (read %d MiB + write %d MiB per copy)"
              % (args.calibrate_copy, args.calibrate_copy, args.calibrate_copy), flush=True)
        return
    sys.path.insert(0, HERE)
    import paper_2412_14104_amd as pkg
    from paper_2412_14104_amd.configs import PRESETS

    if args.split_products != 6:
        pkg.lib.tatrg_test_split_products(args.split_products)
    cfg = PRESETS["C3"]
    chi, r, q, seed = cfg["chi"], cfg["r"], cfg["q"], cfg["seed"]
    beta = cfg["betas"][0]
    split = args.precision == "bf16x3"
    prec = pkg.BF16X3 if split else pkg.FP64
    fin = not args.no_finish
    main_run = run_path(pkg, torch, prec, chi, r, q, seed, beta, args.warmup, args.steps, fin)
    other = None
    if not args.no_fp64_comparison:
        other = run_path(pkg, torch, pkg.FP64 if split else pkg.BF16X3, chi, r, q, seed, beta,
                         args.warmup, args.steps, fin)

    stages = stage_model_flops(chi, r, q)
    total_flops, contr_flops = model_flops_per_step(chi, r, q)
    launches = main_run["launches"]
    avg_launch_s = (main_run["contraction_ms"] / launches) / 1e3 if launches else float("nan")
    alg = main_run["flops_per_launch"] / avg_launch_s / 1e12   # 2 M N K per launch, TFLOP/s
    peak = BF16_PEAK_TFLOPS if split else FP64_PEAK_TFLOPS
    roofline = {"bound": "mfma", "achieved": alg, "peak": peak, "unit": "TFLOP/s",
                "frac": alg / peak,
                "traffic": (profiled_value("traffic_bytes_per_launch")
                            if split and args.split_products == 6 else None),
                "kernel": "gemm_bf16x3_kernel: contraction GEMMs P = E.FM4 and Phi = Qt^T.P "
                          "(both halves)" if split else
                          "gemm_f64_kernel: contraction GEMMs P = E.FM4 and Phi = Qt^T.P",
                "launches": launches, "flops_per_launch": main_run["flops_per_launch"],
                "avg_launch_ms": avg_launch_s * 1e3}
    if split:
        # the split product issues six (three in the ablation) bf16 x bf16 MFMA products per
        # multiply-add of the method
        roofline["bf16_issue_tflops"] = args.split_products * alg
        roofline["bf16_issue_frac"] = args.split_products * alg / BF16_PEAK_TFLOPS
        roofline["mfma_busy_frac"] = (profiled_value("mfma_busy_frac")
                                      if args.split_products == 6 else None)
    sm = main_run["stage_ms_per_step"]
    names = ["S0", "S1", "S2", "S3", "S4", "S5"]
    fam_flops = sum(stages[k] for k in ("S1", "S2", "S3", "S4"))
    fam_ms = sum(sm[1:5])
    roofline_fp64 = {"bound": "mfma", "kernel": "FP64 stages S1-S4 (bond swap, isometries, "
                     "triad tensors, squeezers: FP64 MFMA GEMMs with their small "
                     "factorisations)", "achieved": fam_flops / (fam_ms / 1e3) / 1e12,
                     "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": fam_flops / (fam_ms / 1e3) / 1e12 / FP64_PEAK_TFLOPS,
                     "algorithmic_flops_per_step": fam_flops, "ms_per_step": fam_ms}
    stage_report = {n: {"ms": sm[i], "model_flops": stages[n],
                        "model_tflops": stages[n] / (sm[i] / 1e3) / 1e12 if sm[i] > 0 else None}
                    for i, n in enumerate(names)}
    n_total = main_run["n_total"]
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
                   "precision": args.precision, "split_products": args.split_products},
        "roofline": roofline,
        "roofline_fp64_stages": roofline_fp64,
        "swap_compressed_timed_steps": main_run["swap_compressed_timed_steps"],
        "split_gemm_grouping": main_run["autotune"],
        "stages": stage_report,
        "step_model_flops": total_flops,
        "step_model_tflops": total_flops * main_run["value"] / 1e12,
        "wall_s": main_run["wall_s"],
        "f": main_run["f"], "lnZV": main_run["lnZV"],
    }
    ref = None
    gpath = os.path.join(HERE, "tests", "golden", "C3.json")
    if os.path.exists(gpath) and n_total == 40 and fin:
        with open(gpath) as fh:
            ref = json.load(fh)["runs"][0]
    out["delta_f_rel_vs_oracle"] = (abs(main_run["f"] - ref["f"]) / abs(ref["f"])
                                    if ref is not None else None)
    if other is not None:
        key = "fp64_path" if split else "bf16x3_path"
        o = {"value": other["value"], "ms_per_step": other["ms_per_step"],
             "contraction_avg_launch_ms": other["contraction_ms"] / max(other["launches"], 1),
             "stage_ms_per_step": dict(zip(names, other["stage_ms_per_step"])),
             "f": other["f"],
             "delta_f_rel_vs_oracle": (abs(other["f"] - ref["f"]) / abs(ref["f"])
                                       if ref is not None else None)}
        out[key] = o
        out["delta_f_rel_split_vs_fp64_path"] = (abs(main_run["f"] - other["f"]) / abs(other["f"])
                                                 if fin else None)
        out["speedup_vs_" + key.split("_")[0]] = main_run["value"] / other["value"]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(chi, r, q, seed, beta)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
