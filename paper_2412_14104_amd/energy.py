"""Derivatives of ln Z / V in beta: internal energy u = -d(ln Z/V)/d beta and specific heat
c = beta^2 d^2(ln Z/V)/d beta^2 of the 4D Ising model (Section 3, Z = tTr prod T).

The library runs each temperature beta as a triple (beta - d, beta, beta + d) in one batch;
the three runs share the Gaussian sketches, so the truncated ln Z / V is a smooth function of
beta and tatrg_lnz_derivatives takes central differences of it (include/tatrg.h).  `LnZ` is
a torch.autograd.Function over that call: forward returns ln Z / V, backward multiplies by
the derivative the same batch produced.

    python -m paper_2412_14104_amd.energy --preset C5 [--precision fp64|bf16x3] [--delta D]
prints one JSON line with ln Z / V, u and c per temperature of the preset.
"""
import argparse
import json
import sys
import time


def derivatives(betas, chi, r, q, n_steps, seed=0, delta=1e-4, precision=None, stream=None,
                progress=False):
    """(ln Z/V, d(ln Z/V)/d beta, d^2(ln Z/V)/d beta^2) per beta, one batch of 3 len(betas)."""
    from . import FP64, Engine
    eng = Engine(chi, r, q, n_steps, seed=seed, precision=FP64 if precision is None else precision,
                 record_spectra=False, batch=3 * len(betas), stream=stream)
    eng.init([b + s * delta for b in betas for s in (-1.0, 0.0, 1.0)])
    t0 = time.perf_counter()
    for k in range(n_steps):
        eng.step()
        if progress:
            print("  step %d of %d, %.1f s" % (k + 1, n_steps, time.perf_counter() - t0),
                  file=sys.stderr, flush=True)
    return eng.lnz_derivatives()


def _lnz_function():
    import torch

    class LnZ(torch.autograd.Function):
        """ln Z / V of the truncated RG at a scalar beta (a 0-dim float64 CPU tensor), with
        d(ln Z/V)/d beta for the backward pass."""

        @staticmethod
        def forward(ctx, beta, chi, r, q, n_steps, seed=0, delta=1e-4, precision=None):
            l0, d1, _ = derivatives([float(beta)], chi, r, q, n_steps, seed, delta, precision)
            ctx.save_for_backward(torch.tensor(d1[0], dtype=torch.float64))
            return torch.tensor(l0[0], dtype=torch.float64)

        @staticmethod
        def backward(ctx, grad):
            (d1,) = ctx.saved_tensors
            return (grad * d1,) + (None,) * 7

    return LnZ


def __getattr__(name):
    if name == "LnZ":
        return _lnz_function()
    raise AttributeError(name)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--preset", default="C5")
    ap.add_argument("--precision", choices=["fp64", "bf16x3"], default="fp64")
    ap.add_argument("--delta", type=float, default=1e-4)
    args = ap.parse_args(argv)
    import torch
    if not torch.cuda.is_available():
        print("no HIP device visible", file=sys.stderr)
        return 1
    from . import BF16X3, FP64
    from .configs import PRESETS
    cfg = PRESETS[args.preset]
    prec = BF16X3 if args.precision == "bf16x3" else FP64
    out = {"workload": "4D Ising Triad-ATRG, preset %s: chi=%d, r=%d, q=%d, %d RG steps, "
                       "beta in %s, central differences d=%g over common sketches"
                       % (args.preset, cfg["chi"], cfg["r"], cfg["q"], cfg["n_steps"],
                          cfg["betas"], args.delta),
           "precision": args.precision, "betas": list(cfg["betas"]), "runs": []}
    t0 = time.perf_counter()
    for beta in cfg["betas"]:
        t1 = time.perf_counter()
        l0, d1, d2 = derivatives([beta], cfg["chi"], cfg["r"], cfg["q"], cfg["n_steps"],
                                 cfg["seed"], args.delta, prec, progress=True)
        torch.cuda.synchronize()
        run = {"beta": beta, "lnZV": l0[0], "dlnZV_dbeta": d1[0], "d2lnZV_dbeta2": d2[0],
               "u": -d1[0], "c": beta * beta * d2[0], "seconds": time.perf_counter() - t1}
        out["runs"].append(run)
        print("beta %.7f: u %.10f, c %.6f, %.1f s" % (beta, run["u"], run["c"], run["seconds"]),
              file=sys.stderr, flush=True)
    out["seconds"] = time.perf_counter() - t0
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
