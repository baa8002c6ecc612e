"""Write the oracle's input and output of one RG step for the element-by-element test of the
contraction (test infrastructure; calls only oracle/).

The chi = 32, r = 3 workload (beta = 0.1496947, seed 0) is run by the oracle for K steps;
the state entering step K (Phi, Psi, the log-norm accumulator) is stored whole (zero-padded
tensors compress well), and of the state after step K -- Phi and Psi of Eqs. (makeMG),
(makeMH) after the slot rotation, chi^4 rows of chi gamma values each -- a seeded sample of
rows is stored: 4096 rows drawn from the block where the oracle's output is not identically
zero, 512 from outside it.  Also stored: ln c_K, the swap spectrum sigma of step K (it fixes
which gamma columns carry weight) and max |Phi|, max |Psi| over the whole output.  Usage:
    python tests/golden/make_one_step.py [K]      # K = 2: about five minutes on 8 cores
writes tests/golden/C3_one_step_k<K>.npz.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import tatrg  # noqa: E402

with open(os.path.join(ROOT, "paper_2412_14104_amd", "presets.json")) as _fh:
    PRESETS = {k: v for k, v in json.load(_fh).items() if not k.startswith("_")}

N_IN = 4096
N_OUT = 512
SAMPLE_SEED = 2024


def extents(t):
    """Per leg, one past the last index at which t is not identically zero."""
    out = []
    for ax in range(t.ndim):
        other = tuple(j for j in range(t.ndim) if j != ax)
        nz = np.nonzero(np.abs(t).max(axis=other) > 0)[0]
        out.append(int(nz[-1]) + 1 if nz.size else 0)
    return out


def main(k):
    cfg = PRESETS["C3"]
    beta, chi, r, q, seed = cfg["betas"][0], cfg["chi"], cfg["r"], cfg["q"], cfg["seed"]
    t0 = time.time()
    phi, psi, acc = tatrg.run_partial(beta, chi, r, q, seed, k)
    phi_o, psi_o, info = tatrg.step(phi, psi, k, chi, r, q, seed)
    ext = [max(a, b) for a, b in zip(extents(phi_o), extents(psi_o))]
    rng = np.random.default_rng(SAMPLE_SEED)
    inside = np.stack([rng.integers(0, e, N_IN) for e in ext[:4]], axis=1)
    outside = []
    while len(outside) < N_OUT:
        idx = rng.integers(0, chi, 4)
        if any(idx[j] >= ext[j] for j in range(4)):
            outside.append(idx)
    rows4 = np.concatenate([inside, np.array(outside)], axis=0)
    rows = np.ravel_multi_index(tuple(rows4.T), (chi,) * 4)
    po = phi_o.reshape(-1, chi)
    so = psi_o.reshape(-1, chi)
    np.savez_compressed(
        os.path.join(HERE, "C3_one_step_k%d.npz" % k),
        beta=beta, chi=chi, r=r, q=q, seed=seed, k=k,
        phi_in=phi, psi_in=psi, acc_in=acc, lnc=info["lnc"], sigma=info["sigma"],
        rows=rows, phi_rows=po[rows], psi_rows=so[rows],
        phi_absmax=np.abs(po).max(), psi_absmax=np.abs(so).max(), extents=np.array(ext),
        source="oracle/tatrg.py run_partial + step, float64, tests/golden/make_one_step.py")
    print("k=%d extents %s, %.1f s" % (k, ext, time.time() - t0), flush=True)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 2)
