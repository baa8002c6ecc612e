"""Write the oracle's reference results for the parity tests.

Calls only the FP64 oracle (oracle/).  Usage:
    python tests/golden/make_golden.py C1 C2        # a few minutes
    python tests/golden/make_golden.py C3           # about two hours on 8 cores
Each run writes tests/golden/<name>.json with ln Z / V, f, and per step ln c_k and the
singular spectra (canonical s, swap sigma, squeezer S for mu = 2, 3, 4).
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


def main(names):
    for name in names:
        cfg = PRESETS[name]
        runs = []
        for beta in cfg["betas"][:1]:
            t0 = time.time()
            res = tatrg.run(beta, cfg["chi"], cfg["r"], cfg["q"], cfg["seed"], cfg["n_steps"])
            runs.append({
                "beta": beta, "lnZV": res["lnZV"], "f": res["f"],
                "lnc_final": res["lnc_final"], "ttr": res["ttr"],
                "steps": [{"lnc": st["lnc"], "s": st["s"].tolist(),
                           "sigma": st["sigma"].tolist(),
                           "sqz": {str(mu): st["sqz"][mu].tolist() for mu in (2, 3, 4)}}
                          for st in res["steps"]],
                "oracle_seconds": time.time() - t0,
            })
            print(name, beta, res["lnZV"], res["f"], "%.1f s" % (time.time() - t0), flush=True)
        out = {"config": name, "chi": cfg["chi"], "r": cfg["r"], "q": cfg["q"],
               "seed": cfg["seed"], "n_steps": cfg["n_steps"], "runs": runs,
               "source": "oracle/tatrg.py run(), float64, written by tests/golden/make_golden.py"}
        with open(os.path.join(HERE, name + ".json"), "w") as fh:
            json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main(sys.argv[1:] or ["C1", "C2"])
