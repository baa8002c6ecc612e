"""Host-side logic that needs no device: the transition estimate of the scan and the model
flop count the benchmark prices the step with."""
import importlib
import os
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def scan():
    sys.path.insert(0, ROOT)
    return importlib.import_module("paper_2412_14104_amd.scan")


def test_crossing_interpolates_the_first_crossing(scan):
    betas = [0.10, 0.12, 0.14, 0.16]
    xs = [1.0, 1.2, 1.8, 2.0]
    # between 0.12 (1.2) and 0.14 (1.8): 0.12 + 0.3 / 0.6 * 0.02 = 0.13
    assert abs(scan.crossing(betas, xs) - 0.13) < 1e-15
    # the order of the temperatures does not matter
    assert abs(scan.crossing(betas[::-1], xs[::-1]) - 0.13) < 1e-15


def test_crossing_none_without_a_crossing_and_exact_hits(scan):
    assert scan.crossing([0.1, 0.2, 0.3], [1.0, 1.1, 1.2]) is None
    assert scan.crossing([0.1, 0.2, 0.3], [1.0, 1.5, 2.0]) == 0.2
    # a flat segment exactly at the level is skipped (no division by zero); the next segment
    # starts at the level, so the crossing is its left end
    assert scan.crossing([0.1, 0.2, 0.3], [1.5, 1.5, 2.0]) == 0.2


def test_model_flops_contraction_term():
    """The contraction part of the step model is 8 L^2 chi^5 + 4 L chi^5 + 4 L^2 chi^4
    + 4 L chi^4 (two halves of the P and Phi GEMMs and the small brackets); at chi = 32,
    r = 3 the P and Phi GEMMs alone are 8 L^2 chi^5 = 2.47e12 flops and the whole step
    3.94e12."""
    sys.path.insert(0, ROOT)
    bench = importlib.import_module("bench")
    total, contraction = bench.model_flops_per_step(32, 3, 2)
    L = 96
    assert contraction == (8 * L * L * 32 ** 5 + 4 * L * 32 ** 5 + 4 * L * L * 32 ** 4
                           + 4 * L * 32 ** 4)
    assert total > contraction > 2.4e12
    assert 3.9e12 < total < 4.0e12
    st = bench.stage_model_flops(32, 3, 2)
    # bond swap: compression 8 chi^7 plus six products of the compressed operand with
    # chi^3 x 96 panels and their chi^3 x 96 x 96 Grams
    assert st["S1"] == 8 * 32 ** 7 + 6 * (4 * 32 ** 5 * 96 + 2 * 32 ** 3 * 96 * 96)


def test_golden_writers_run_without_the_product_library():
    """The writers of stored expected values load only oracle/ and the preset data: with any
    import of the product package made to fail, each module still loads and sees the
    presets."""
    import subprocess
    code = (
        "import sys, importlib.util\n"
        "sys.modules['paper_2412_14104_amd'] = None\n"
        "sys.path.insert(0, %r)\n"
        "for name in ('make_golden', 'make_scan_golden', 'make_sensitivity'):\n"
        "    spec = importlib.util.spec_from_file_location(name, %r + '/' + name + '.py')\n"
        "    mod = importlib.util.module_from_spec(spec)\n"
        "    spec.loader.exec_module(mod)\n"
        "    assert mod.PRESETS['C3']['chi'] == 32 and len(mod.PRESETS['C4']['betas']) == 64\n"
        "assert 'paper_2412_14104_amd.configs' not in sys.modules\n"
        "print('ok')\n" % (ROOT, os.path.join(HERE, "golden")))
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                         timeout=300)
    assert res.returncode == 0 and res.stdout.strip() == "ok", res.stderr


def test_presets_data_matches_the_workloads():
    sys.path.insert(0, ROOT)
    from paper_2412_14104_amd.configs import PRESETS
    assert PRESETS["C3"] == {**PRESETS["C3"], "chi": 32, "r": 3, "q": 2, "n_steps": 40,
                             "betas": [0.1496947]}
    betas = PRESETS["C4"]["betas"]
    assert betas == [0.140 + 0.020 * i / 63 for i in range(64)]


def test_qt_contraction_orders_agree():
    """The step forms Qt[kA][kX][k2][k3] = sum I[(i2a i3a)][kA] S2[i2a][i2b][k2]
    S3[i3a][i3b][k3] J[(i2b i3b)][kX] as (I S2)(S3 J) contracted over (i3a, i2b), with the
    leg orders of its GEMMs; this checks those index orders against the defining sum (small
    chi and L, numpy)."""
    import numpy as np
    rng = np.random.default_rng(7)
    c, L = 3, 4
    n2 = c * c
    I = rng.standard_normal((n2, L))
    J = rng.standard_normal((n2, L))
    S2 = rng.standard_normal((c, c, c))
    S3 = rng.standard_normal((c, c, c))
    ref = np.einsum("pqA,pbk,qel,beX->AXkl", I.reshape(c, c, L), S2, S3, J.reshape(c, c, L))
    # q1[(i3a kA),(i2b k2)] = I^T S2 over i2a, as the first GEMM (A viewed [i2a][(i3a kA)])
    q1 = I.reshape(c, c * L).T @ S2.reshape(c, c * c)
    fap = q1.reshape(c, L, c, c).transpose(1, 3, 0, 2).reshape(L * c, c * c)  # [kA k2][i3a i2b]
    s3p = S3.transpose(0, 2, 1).reshape(c * c, c)                             # [i3a k3][i3b]
    jp = J.reshape(c, c, L).transpose(1, 0, 2).reshape(c, c * L)              # [i3b][i2b kX]
    fb = s3p @ jp                                                             # [i3a k3][i2b kX]
    fbp = fb.reshape(c, c, c, L).transpose(0, 2, 1, 3).reshape(c * c, c * L)  # [i3a i2b][k3 kX]
    out = fap @ fbp                                                           # [kA k2][k3 kX]
    qt = out.reshape(L, c, c, L).transpose(0, 3, 1, 2)                        # [kA kX k2 k3]
    assert np.allclose(qt, ref, rtol=1e-13, atol=1e-13)
