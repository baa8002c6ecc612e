"""Stored central-difference derivatives of ln Z/V in beta (test infrastructure).

Calls only the FP64 oracle (oracle/tatrg.py lnz_derivatives: runs at beta - h, beta, beta + h
with the common sketches).  Usage:
    python tests/golden/make_fd_golden.py        # about five minutes on two cores
writes tests/golden/FD.json with ln Z/V, d(ln Z/V)/d beta and d^2(ln Z/V)/d beta^2 for the
presets C1 (chi = 6, 16 steps) and C2 (chi = 16, 40 steps) at h = 1e-4.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import tatrg  # noqa: E402
with open(os.path.join(ROOT, "paper_2412_14104_amd", "presets.json")) as _fh:
    PRESETS = {k: v for k, v in json.load(_fh).items() if not k.startswith("_")}

DELTA = 1e-4


def main():
    out = {"delta": DELTA, "cases": [],
           "source": "oracle/tatrg.py lnz_derivatives(), float64, written by "
                     "tests/golden/make_fd_golden.py"}
    for name in ("C1", "C2"):
        cfg = PRESETS[name]
        beta = cfg["betas"][0]
        t0 = time.time()
        l0, d1, d2 = tatrg.lnz_derivatives(beta, DELTA, cfg["chi"], cfg["r"], cfg["q"],
                                           cfg["seed"], cfg["n_steps"])
        out["cases"].append({"config": name, "beta": beta, "chi": cfg["chi"], "r": cfg["r"],
                             "q": cfg["q"], "seed": cfg["seed"], "n_steps": cfg["n_steps"],
                             "lnZV": l0, "dlnZV_dbeta": d1, "d2lnZV_dbeta2": d2,
                             "oracle_seconds": time.time() - t0})
        print(name, beta, l0, d1, d2, "%.1f s" % (time.time() - t0), flush=True)
    with open(os.path.join(HERE, "FD.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
