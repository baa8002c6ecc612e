"""Write the oracle's results for three temperatures of the beta scan (test infrastructure).

Calls only the FP64 oracle (oracle/).  The scan preset C4 has 64 temperatures in
[0.140, 0.160] at chi = 24, r = 2, 40 steps; the oracle runs the first, a middle and the last
one (about 15 minutes each on two cores).  Usage:
    python tests/golden/make_scan_golden.py
writes tests/golden/C4_subset.json with, per temperature, ln Z / V, f, ln c_k and the order
parameter X^(m) for m = 0..40.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import tatrg  # noqa: E402
# the workload presets are plain data; read them without importing the product package
with open(os.path.join(ROOT, "paper_2412_14104_amd", "presets.json")) as _fh:
    PRESETS = {k: v for k, v in json.load(_fh).items() if not k.startswith("_")}

INDICES = (0, 31, 63)


def main():
    cfg = PRESETS["C4"]
    runs = []
    for i in INDICES:
        beta = cfg["betas"][i]
        t0 = time.time()
        res = tatrg.run(beta, cfg["chi"], cfg["r"], cfg["q"], cfg["seed"], cfg["n_steps"],
                        record=False)
        runs.append({"index": i, "beta": beta, "lnZV": res["lnZV"], "f": res["f"],
                     "lnc": [st["lnc"] for st in res["steps"]],
                     "X": [st["X"] for st in res["steps"]] + [res["X_final"]],
                     "oracle_seconds": time.time() - t0})
        print(i, beta, res["f"], "%.1f s" % (time.time() - t0), flush=True)
    out = {"config": "C4", "chi": cfg["chi"], "r": cfg["r"], "q": cfg["q"], "seed": cfg["seed"],
           "n_steps": cfg["n_steps"], "runs": runs,
           "source": "oracle/tatrg.py run(), float64, written by "
                     "tests/golden/make_scan_golden.py"}
    with open(os.path.join(HERE, "C4_subset.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
