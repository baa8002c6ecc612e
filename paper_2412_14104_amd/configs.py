"""Workload presets of the 4D Ising Triad-ATRG runs (pure data, no arithmetic).

Each preset is the input of one run: inverse temperature(s), bond dimension chi,
internal-line oversampling r, QR iterations q of every randomized SVD, Philox seed and the
number of RG steps N (a periodic lattice of 2^N sites).  The values live in presets.json
beside this file, which the oracle-only writers of stored results read directly.
"""
import json
import os

PRESETS_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "presets.json")

with open(PRESETS_PATH) as _fh:
    PRESETS = {k: v for k, v in json.load(_fh).items() if not k.startswith("_")}

BETA_NEAR_CRITICAL = PRESETS["C2"]["betas"][0]
