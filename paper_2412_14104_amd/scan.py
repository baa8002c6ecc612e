"""Temperature scan of the 4D Ising model with Triad-ATRG on one MI355X.

Runs every temperature of a preset (C4: 64 values of beta in [0.140, 0.160], chi = 24,
r = 2, q = 2, 40 steps) as batches of the library (include/tatrg.h, batch = B), all sharing
the same Gaussian sketches.  The temperatures are dealt to `--engines` handles, each with a
stream and a host thread of its own, so that the device runs them concurrently (a step at
this size is mostly chains of small latency-bound kernels).  Every temperature's
result is that of a batch-1 run.  Prints one JSON line with the free energy per site and the
order parameter X^(m) = (Tr A)^2 / Tr A^2 (Section 3) of every temperature, the throughput,
and the transition estimate: for each isotropic block (m a multiple of 4, the 2^m-site
hypercube) the beta at which X^(m) crosses 3/2, halfway between the disordered (X = 1) and
ordered (X = 2) fixed points, by linear interpolation between neighbouring temperatures.

    python -m paper_2412_14104_amd.scan [--preset C4] [--precision fp64|bf16x3]
"""
import argparse
import json
import os
import sys
import time


def crossing(betas, xs, level=1.5):
    """First beta (ascending) at which xs crosses `level`, linearly interpolated; None if it
    does not."""
    pairs = sorted(zip(betas, xs))
    for (b0, x0), (b1, x1) in zip(pairs, pairs[1:]):
        if (x0 - level) * (x1 - level) <= 0 and x0 != x1:
            return b0 + (level - x0) * (b1 - b0) / (x1 - x0)
    return None


def run_scan(betas, chi, r, q, n, seed=0, precision="fp64", engines=4, progress=False):
    """Every temperature of `betas` through n RG steps, dealt in contiguous chunks to
    `engines` handles (each a batch with its own stream).  Each handle is driven by a host
    thread of its own: a step synchronises its stream once per temperature (the bond swap's
    conditioning verdict), and with one thread per handle that wait never holds back the
    other handles.  Returns the wall time between device synchronisations and, per
    temperature, f, ln Z / V and X^(m) for m = 0..n."""
    import threading

    import torch
    from . import BF16X3, FP64, Engine

    prec = BF16X3 if precision == "bf16x3" else FP64
    ne = max(1, min(engines, len(betas)))
    bounds = [len(betas) * e // ne for e in range(ne + 1)]
    chunks = [betas[bounds[e]:bounds[e + 1]] for e in range(ne)]
    device = torch.cuda.current_device()
    engs = []
    for chunk in chunks:
        st = torch.cuda.Stream()
        eng = Engine(chi, r, q, n, seed=seed, precision=prec, record_spectra=True,
                     batch=len(chunk), stream=st)
        if ne > 1:
            # the handles already fill the device: no second stream each
            eng.set_side_stream(False)
        eng.init(chunk)
        engs.append(eng)
    torch.cuda.synchronize()
    errors = []

    def drive(e):
        try:
            torch.cuda.set_device(device)
            for k in range(n):
                engs[e].step()
                if progress and e == 0 and k % 8 == 7:
                    print("handle 0: step %d of %d" % (k + 1, n), file=sys.stderr, flush=True)
        except Exception as exc:  # reported after the join
            errors.append(exc)

    t0 = time.perf_counter()
    threads = [threading.Thread(target=drive, args=(e,)) for e in range(ne)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize()
    seconds = time.perf_counter() - t0
    if errors:
        raise errors[0]
    f, lnzv, xs = [], [], []
    for eng, chunk in zip(engs, chunks):
        fe, le = eng.free_energy()
        f += fe if isinstance(fe, list) else [fe]
        lnzv += le if isinstance(le, list) else [le]
        xs += [[eng.order_parameter(m, b) for m in range(n + 1)] for b in range(len(chunk))]
    return {"seconds": seconds, "engines": ne, "f": f, "lnZV": lnzv, "X": xs}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--preset", default="C4")
    ap.add_argument("--precision", choices=["fp64", "bf16x3"], default="fp64")
    ap.add_argument("--engines", type=int, default=8,
                    help="handles (streams, host threads) the temperatures are dealt to")
    args = ap.parse_args(argv)
    # one hardware queue per handle's stream (HIP's default is 4 per process); read when the
    # runtime starts, so it is set before torch initialises the device
    os.environ.setdefault("GPU_MAX_HW_QUEUES", str(min(max(args.engines, 4), 16)))

    import torch
    if not torch.cuda.is_available():
        print("no HIP device visible", file=sys.stderr)
        return 1
    from .configs import PRESETS

    cfg = PRESETS[args.preset]
    betas = list(cfg["betas"])
    chi, r, q, n = cfg["chi"], cfg["r"], cfg["q"], cfg["n_steps"]
    res = run_scan(betas, chi, r, q, n, cfg["seed"], args.precision, args.engines,
                   progress=True)
    xs = res["X"]
    est = {}
    for m in range(4, n + 1, 4):
        est[str(m)] = crossing(betas, [x[m] for x in xs])
    gpu_s = res["seconds"]
    out = {
        "workload": "4D Ising Triad-ATRG beta scan, preset %s: %d temperatures in [%g, %g], "
                    "chi=%d, r=%d, q=%d, %d RG steps each" % (args.preset, len(betas),
                                                             min(betas), max(betas), chi, r,
                                                             q, n),
        "precision": args.precision,
        "n_betas": len(betas),
        "engines": res["engines"],
        "seconds": gpu_s,            # wall time between device synchronisations
        "rg_steps_per_s": len(betas) * n / gpu_s,
        "ms_per_rg_step": gpu_s * 1e3 / (len(betas) * n),
        "betas": betas, "f": res["f"], "lnZV": res["lnZV"],
        "X_last": [x[n] for x in xs],
        "X": {str(m): [x[m] for x in xs] for m in range(0, n + 1, 4)},
        "beta_c_from_X_crossing_by_block": est,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
