"""The performance model against the numbers Sect. 2.2 prints (tests/golden/paper_numbers.json)."""
import json
import math
import os

import pytest

from paper_1112_5588_amd import model

G = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))


@pytest.mark.parametrize("case", G["code_balance_dp"]["cases"])
def test_code_balance(case):
    assert model.code_balance_dp(case["alpha"], case["n_nzr"]) == case["bytes_per_flop"]


@pytest.mark.parametrize("case", G["pcie_thresholds"]["cases"])
def test_pcie_thresholds(case):
    # "alpha = 1/N_nzr" is small next to 3/2; the paper's worst-case figures drop it
    alpha = 0.0 if case["alpha"] == "1/N_nzr" else float(case["alpha"])
    if case["eq"] == 3:
        bound = model.nnzr_bound_half_penalty(case["bw_ratio"], alpha)
        assert math.floor(bound) == case["n_nzr_bound"]
    else:
        bound = model.nnzr_bound_tenth_penalty(case["bw_ratio"], alpha)
        assert math.ceil(bound) == case["n_nzr_bound"]


def test_thresholds_are_where_the_times_cross():
    # eq. (3) and (4) are eq. (2) solved for N_nzr: check by evaluating eq. (2) there
    n, b_pci = 1e6, 8e9
    for ratio, alpha in ((20, 0.05), (10, 1.0)):
        nz = model.nnzr_bound_half_penalty(ratio, alpha)
        assert math.isclose(model.t_mvm(n, nz, alpha, ratio * b_pci), model.t_pci(n, b_pci), rel_tol=1e-12)
        nz = model.nnzr_bound_tenth_penalty(ratio, alpha)
        assert math.isclose(model.t_mvm(n, nz, alpha, ratio * b_pci), 10 * model.t_pci(n, b_pci), rel_tol=1e-12)


def test_byte_counts():
    assert model.alg_bytes_spmv(100, 10) == 12 * 100 + 16 * 10
    assert model.alg_bytes_spmv(100, 10, 4) == 8 * 100 + 8 * 10
    # eq. (2) at alpha = 1/N_nzr counts y read and written: 8 bytes more per row than ours
    n, nz = 1000, 12
    assert model.t_mvm(n, nz, 1 / nz, 1.0) == pytest.approx(model.alg_bytes_spmv(n * nz, n) + 8 * n)
