"""Write the oracle's results for three temperatures of the beta scan (test infrastructure).

Calls only the FP64 oracle (oracle/).  The scan preset C4 has 64 temperatures in
[0.140, 0.160] at chi = 24, r = 2, 40 steps; the oracle runs the first, a middle and the last
one (about 15 minutes each on two cores), or eight neighbouring ones around the X = 3/2
crossing.  Usage:
    python tests/golden/make_scan_golden.py [C4_subset | C4_crossing] [workers]
writes tests/golden/<set>.json with, per temperature, ln Z / V, f, ln c_k and the order
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

SETS = {
    # the first, a middle and the last temperature of the scan
    "C4_subset": (0, 31, 63),
    # eight neighbouring temperatures around the X = 3/2 crossing (beta ~ 0.1497)
    "C4_crossing": tuple(range(28, 36)),
}


def run_one(i):
    cfg = PRESETS["C4"]
    beta = cfg["betas"][i]
    t0 = time.time()
    res = tatrg.run(beta, cfg["chi"], cfg["r"], cfg["q"], cfg["seed"], cfg["n_steps"],
                    record=False)
    print(i, beta, res["f"], "%.1f s" % (time.time() - t0), flush=True)
    return {"index": i, "beta": beta, "lnZV": res["lnZV"], "f": res["f"],
            "lnc": [st["lnc"] for st in res["steps"]],
            "X": [st["X"] for st in res["steps"]] + [res["X_final"]],
            "oracle_seconds": time.time() - t0}


def main(name, workers=1):
    cfg = PRESETS["C4"]
    if workers > 1:
        from concurrent.futures import ProcessPoolExecutor
        with ProcessPoolExecutor(max_workers=workers) as ex:
            runs = list(ex.map(run_one, SETS[name]))
    else:
        runs = [run_one(i) for i in SETS[name]]
    out = {"config": "C4", "chi": cfg["chi"], "r": cfg["r"], "q": cfg["q"], "seed": cfg["seed"],
           "n_steps": cfg["n_steps"], "runs": runs,
           "source": "oracle/tatrg.py run(), float64, written by "
                     "tests/golden/make_scan_golden.py"}
    with open(os.path.join(HERE, name + ".json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "C4_subset",
         int(sys.argv[2]) if len(sys.argv) > 2 else 1)
