"""Self-sensitivity of the oracle's singular spectra, per RG step (test infrastructure).

Runs the FP64 oracle (oracle/ only) for a preset with relative noise of 1e-15 added to
(Phi, Psi) after every step, and records per step the largest deviation of each stored
spectrum from the unperturbed run in tests/golden/<name>.json, relative to that spectrum's
maximum.  The parity tests bound the GPU's spectra by a multiple of this: the RG flow
amplifies rounding, and this measures how much for the oracle itself.  Usage:
    python tests/golden/make_sensitivity.py C3      # about 70 minutes on 8 cores
writes tests/golden/<name>_spectra_sensitivity.json.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import tatrg  # noqa: E402
from paper_2412_14104_amd.configs import PRESETS  # noqa: E402

NOISE = 1e-15
NOISE_SEED = 5


def main(name):
    cfg = PRESETS[name]
    ref = json.load(open(os.path.join(HERE, name + ".json")))["runs"][0]["steps"]
    beta, chi, r, q, seed = cfg["betas"][0], cfg["chi"], cfg["r"], cfg["q"], cfg["seed"]
    rng = np.random.default_rng(NOISE_SEED)
    phi, psi = tatrg.initial_state(beta, chi)
    out = []
    for k in range(cfg["n_steps"]):
        phi, psi, info = tatrg.step(phi, psi, k, chi, r, q, seed)
        dev = {}
        for key in ("s", "sigma"):
            rs = np.array(ref[k][key])
            dev[key] = float(np.abs(info[key] - rs).max() / rs.max())
        for mu in (2, 3, 4):
            rs = np.array(ref[k]["sqz"][str(mu)])
            dev[str(mu)] = float(np.abs(info["sqz"][mu] - rs).max() / rs.max())
        out.append(dev)
        print(k, " ".join("%s=%.1e" % kv for kv in dev.items()), flush=True)
        phi = phi + NOISE * np.abs(phi).max() * rng.standard_normal(phi.shape)
        psi = psi + NOISE * np.abs(psi).max() * rng.standard_normal(psi.shape)
    with open(os.path.join(HERE, name + "_spectra_sensitivity.json"), "w") as fh:
        json.dump({"config": name, "noise": NOISE, "noise_seed": NOISE_SEED, "steps": out,
                   "source": "oracle/tatrg.py step() with 1e-15 relative noise after every "
                             "step, written by tests/golden/make_sensitivity.py"}, fh, indent=1)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "C3")
