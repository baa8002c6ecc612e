"""Write the plain-ATRG oracle's results for the r = chi identity test (test
infrastructure; calls only oracle/).

Plain ATRG (oracle/atrg.py: the O(chi^9) direct contraction of Table 1's ATRG column) at
beta = 0.1496947, q = 2, seed 0, full sketch widths chi^2, for (chi, N) = (6, 16), (5, 12) and (4, 16):
ln Z / V, f and per step ln c_k and the spectra s, sigma, S^(mu).  The triad path with
r = chi must reproduce them (Section 2, the remark on r = chi).  chi = 7 and 8 are left out:
there degenerate multiplets of the swap spectrum straddle the kept chi-th value, so which
part of a multiplet is kept depends on rounding, and two correct implementations differ at
the truncation level (parity-fragile cuts).  Usage:
    python tests/golden/make_atrg_golden.py        # about 15 s
writes tests/golden/ATRG.json.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import atrg  # noqa: E402

BETA = 0.1496947
CASES = ((6, 16), (5, 12), (4, 16))


def main():
    runs = []
    for chi, n in CASES:
        t0 = time.time()
        res = atrg.run(BETA, chi, 2, 0, n)
        runs.append({
            "chi": chi, "n_steps": n, "beta": BETA, "q": 2, "seed": 0,
            "lnZV": res["lnZV"], "f": res["f"],
            "steps": [{"lnc": st["lnc"], "s": st["s"].tolist(), "sigma": st["sigma"].tolist(),
                       "sqz": {str(mu): st["sqz"][mu].tolist() for mu in (2, 3, 4)}}
                      for st in res["steps"]],
            "oracle_seconds": time.time() - t0})
        print(chi, n, res["f"], "%.1f s" % (time.time() - t0), flush=True)
    with open(os.path.join(HERE, "ATRG.json"), "w") as fh:
        json.dump({"runs": runs, "source": "oracle/atrg.py run(), float64, written by "
                                           "tests/golden/make_atrg_golden.py"}, fh, indent=1)


if __name__ == "__main__":
    main()
