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
    (two halves of the P and Phi GEMMs and the small brackets); at chi = 32, r = 3 the P and
    Phi GEMMs alone are 8 L^2 chi^5 = 2.47e12 flops."""
    sys.path.insert(0, ROOT)
    bench = importlib.import_module("bench")
    total, contraction = bench.model_flops_per_step(32, 3, 2)
    L = 96
    assert contraction == 8 * L * L * 32 ** 5 + 4 * L * 32 ** 5 + 4 * L * L * 32 ** 4
    assert total > contraction > 2.4e12
