"""Regression anchors of the oracle (values written by tests/golden/make_golden.py)."""
import json
import os

import numpy as np

from oracle import dense, fastcheck
from paper_2405_19246_amd import inputs

_G = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_values.json")))


def test_dense_l3_n64_values_reproduce():
    g = _G["l3_n64_eps0.1_500_sweeps"][0]
    u, h, eps = inputs.workload("l3_n64_eps0.1", instance=g["instance"])
    r = fastcheck.sinkhorn(u, h, eps, itmax=500, check_every=500)
    assert abs(r["W"] - g["W"]) < 1e-13
    np.testing.assert_allclose(r["log_phi"][0, :4], g["log_phi_0_first"], rtol=1e-12)
    # the dense oracle itself, for fewer sweeps than stored but the same path
    rd = dense.sinkhorn(u, h, eps, itmax=30)
    rf = fastcheck.sinkhorn(u, h, eps, itmax=30)
    np.testing.assert_allclose(rd["log_phi"], rf["log_phi"], rtol=1e-12, atol=1e-12)


def test_fastcheck_l4_n1000_values_reproduce():
    g = _G["l4_n1000_eps0.01_fastcheck_200_sweeps"][0]
    u, h, eps = inputs.workload("l4_n1000_eps0.01", instance=g["instance"])
    r = fastcheck.sinkhorn(u, h, eps, itmax=200, check_every=200)
    assert abs(r["W"] - g["W"]) < 1e-12
    assert abs(r["res"] - g["res"]) < 1e-9 * g["res"]
