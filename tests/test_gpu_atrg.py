"""The r = chi limit on the GPU: with r chi = chi^2 internal lines the triad step is plain
ATRG (Section 2, the remark on r = chi; Table 1), so the GPU's triad path at r = chi must
reproduce the plain-ATRG oracle (oracle/atrg.py, its O(chi^9) direct contraction), whose
results tests/golden/make_atrg_golden.py stored."""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))
REL_F = 1e-9
SPEC_TOL = 1e-8


@pytest.fixture(scope="module")
def pkg():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2412_14104_amd as p
    return p


def runs():
    with open(os.path.join(HERE, "golden", "ATRG.json")) as fh:
        return json.load(fh)["runs"]


@pytest.mark.parametrize("idx", [0, 1, 2])
def test_triad_path_at_r_equal_chi_reproduces_plain_atrg(pkg, idx):
    run = runs()[idx]
    chi, n = run["chi"], run["n_steps"]
    print("r = chi identity: chi", chi, "steps", n, flush=True)
    eng = pkg.Engine(chi, chi, run["q"], n, seed=run["seed"])
    f, lnzv = eng.run(run["beta"])
    print("  f_gpu %.15f f_atrg %.15f" % (f, run["f"]), flush=True)
    assert abs(f - run["f"]) <= REL_F * abs(run["f"])
    assert abs(lnzv - run["lnZV"]) <= REL_F * abs(run["lnZV"])
    for k, st in enumerate(run["steps"]):
        for which, key in ((0, "s"), (1, "sigma"), (2, "2"), (3, "3"), (4, "4")):
            ref = np.array(st[key] if which < 2 else st["sqz"][key])
            got = np.array(eng.spectrum(k, which))
            assert np.abs(got - ref).max() <= SPEC_TOL * ref.max(), (k, key)
