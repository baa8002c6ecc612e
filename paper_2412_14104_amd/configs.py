"""Workload presets of the 4D Ising Triad-ATRG runs (pure data, no arithmetic).

Each preset is the input of one run: inverse temperature(s), bond dimension chi,
internal-line oversampling r, QR iterations q of every randomized SVD, Philox seed and the
number of RG steps N (a periodic lattice of 2^N sites).
"""
BETA_NEAR_CRITICAL = 0.1496947

PRESETS = {
    # small case: chi = 6, 16 steps (2^16 sites), plain FP64
    "C1": dict(betas=[0.15], chi=6, r=2, q=2, seed=0, n_steps=16, precision="fp64"),
    # near-critical chi = 16, 40 steps (2^40 sites), FP64
    "C2": dict(betas=[BETA_NEAR_CRITICAL], chi=16, r=2, q=2, seed=0, n_steps=40,
               precision="fp64"),
    # chi = 32, r = 3, 40 steps: the headline throughput workload (FP64 and split bf16)
    "C3": dict(betas=[BETA_NEAR_CRITICAL], chi=32, r=3, q=2, seed=0, n_steps=40,
               precision="bf16x3"),
    # temperature scan: 64 betas in [0.140, 0.160], chi = 24
    "C4": dict(betas=[0.140 + 0.020 * i / 63 for i in range(64)], chi=24, r=2, q=2, seed=0,
               n_steps=40, precision="fp64"),
    # differentiated run: chi = 48, 30 steps, three temperatures
    "C5": dict(betas=[0.145, BETA_NEAR_CRITICAL, 0.155], chi=48, r=2, q=2, seed=0,
               n_steps=30, precision="fp64"),
}
