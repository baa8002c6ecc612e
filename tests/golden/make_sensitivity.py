"""Self-sensitivity of the oracle's per-step records (test infrastructure).

Runs the FP64 oracle (oracle/ only) with relative noise of 1e-15 added to (Phi, Psi) after
every step and records, per step, how far the perturbed run moves from the unperturbed one
stored in tests/golden/.  The parity tests bound the GPU by a multiple of this: the RG flow
amplifies rounding, and this measures how much for the oracle itself.  Usage:
    python tests/golden/make_sensitivity.py C3          # about 70 minutes on 8 cores
        spectra (relative to each spectrum's maximum) of the run in C3.json
        -> tests/golden/C3_spectra_sensitivity.json
    python tests/golden/make_sensitivity.py C4_subset   # about 50 minutes on 2 cores
        order parameter X^(m) of the three runs in C4_subset.json
        -> tests/golden/C4_subset_X_sensitivity.json
    python tests/golden/make_sensitivity.py C4_crossing 8   # 8 worker processes
        the same for the eight runs in C4_crossing.json
        -> tests/golden/C4_crossing_X_sensitivity.json
    python tests/golden/make_sensitivity.py C3_one_step_k2   # about two minutes
        Phi, Psi of the one step stored in C3_one_step_k2.npz
        -> tests/golden/C3_one_step_k2_sensitivity.json
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import tatrg  # noqa: E402
# the workload presets are plain data; read them without importing the product package
with open(os.path.join(ROOT, "paper_2412_14104_amd", "presets.json")) as _fh:
    PRESETS = {k: v for k, v in json.load(_fh).items() if not k.startswith("_")}

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


def x_deviation(g, run):
    chi, r, q, seed, n = g["chi"], g["r"], g["q"], g["seed"], g["n_steps"]
    rng = np.random.default_rng(NOISE_SEED)
    phi, psi = tatrg.initial_state(run["beta"], chi)
    dev = []
    for k in range(n):
        phi, psi, info = tatrg.step(phi, psi, k, chi, r, q, seed)
        dev.append(abs(info["X"] - run["X"][k]))
        phi = phi + NOISE * np.abs(phi).max() * rng.standard_normal(phi.shape)
        psi = psi + NOISE * np.abs(psi).max() * rng.standard_normal(psi.shape)
    dev.append(abs(tatrg.order_parameter(phi, psi, n) - run["X"][n]))
    print(run["beta"], " ".join("%.1e" % d for d in dev), flush=True)
    return {"beta": run["beta"], "X_dev": dev}


def main_x(name, workers=1):
    g = json.load(open(os.path.join(HERE, name + ".json")))
    if workers > 1:
        from concurrent.futures import ProcessPoolExecutor
        with ProcessPoolExecutor(max_workers=workers) as ex:
            out = list(ex.map(x_deviation, [g] * len(g["runs"]), g["runs"]))
    else:
        out = [x_deviation(g, run) for run in g["runs"]]
    with open(os.path.join(HERE, name + "_X_sensitivity.json"), "w") as fh:
        json.dump({"config": name, "noise": NOISE, "noise_seed": NOISE_SEED, "runs": out,
                   "source": "oracle/tatrg.py step() with 1e-15 relative noise after every "
                             "step, written by tests/golden/make_sensitivity.py"}, fh, indent=1)


def main_one_step(name):
    """Phi and Psi of one step from the state stored in <name>.npz (make_one_step.py), with
    1e-15 relative noise added to that state: the deviation from the stored sample of output
    rows, after the gamma gauge is aligned from Phi (tests/gamma_gauge.py), relative to the
    stored max |Phi|, max |Psi|."""
    sys.path.insert(0, os.path.dirname(HERE))
    from gamma_gauge import align_gamma
    z = np.load(os.path.join(HERE, name + ".npz"))
    chi, r, q, seed, k = (int(z[key]) for key in ("chi", "r", "q", "seed", "k"))
    rng = np.random.default_rng(NOISE_SEED)
    phi = z["phi_in"] + NOISE * np.abs(z["phi_in"]).max() * rng.standard_normal(
        z["phi_in"].shape)
    psi = z["psi_in"] + NOISE * np.abs(z["psi_in"]).max() * rng.standard_normal(
        z["psi_in"].shape)
    phi_o, psi_o, _ = tatrg.step(phi, psi, k, chi, r, q, seed)
    rows = z["rows"]
    pg, sg, n_live = align_gamma(phi_o.reshape(-1, chi)[rows], psi_o.reshape(-1, chi)[rows],
                                 z["phi_rows"], z["sigma"])
    dphi = float(np.abs(pg - z["phi_rows"]).max() / float(z["phi_absmax"]))
    dpsi = float(np.abs(sg[:, :n_live] - z["psi_rows"][:, :n_live]).max()
                 / float(z["psi_absmax"]))
    print(name, "dphi %.2e dpsi %.2e" % (dphi, dpsi), flush=True)
    with open(os.path.join(HERE, name + "_sensitivity.json"), "w") as fh:
        json.dump({"case": name, "noise": NOISE, "noise_seed": NOISE_SEED,
                   "phi_dev": dphi, "psi_dev": dpsi,
                   "source": "oracle/tatrg.py step() from the stored state with 1e-15 "
                             "relative noise, written by tests/golden/make_sensitivity.py"},
                  fh, indent=1)


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "C3"
    if which.startswith("C4_"):
        main_x(which, int(sys.argv[2]) if len(sys.argv) > 2 else 1)
    elif "_one_step_" in which:
        main_one_step(which)
    else:
        main(which)
