"""The error measures every parity test passes through (oracle/compare.py),
checked on inputs whose figures are known by construction."""
import numpy as np
import pytest

from oracle.compare import sed_errors, t_errors


def test_t_errors_known_perturbation():
    T_ref = np.array([[10.0, 20.0], [40.0, 80.0]])
    H_ref = np.ones_like(T_ref)
    T = T_ref * np.array([[1.0 + 1e-5, 1.0], [1.0 - 4e-5, 1.0 + 2e-5]])
    e = t_errors(T, T_ref, H_ref)
    assert e["max"] == pytest.approx(4e-5, rel=1e-9)
    assert e["mean"] == pytest.approx((1e-5 + 0 + 4e-5 + 2e-5) / 4, rel=1e-9)
    assert e["zero_pairs_ok"]


def test_t_errors_nan_gives_inf_and_zero_heating_is_checked():
    T_ref = np.array([[10.0, 0.0, 30.0]])
    H_ref = np.array([[1.0, 0.0, 1.0]])
    e = t_errors(np.array([[np.nan, 0.0, 30.0]]), T_ref, H_ref)
    assert e["max"] == float("inf")
    # a pair without heating must have T = 0 exactly; anything else is flagged
    assert t_errors(np.array([[10.0, 0.0, 30.0]]), T_ref, H_ref)["zero_pairs_ok"]
    assert not t_errors(np.array([[10.0, 1e-30, 30.0]]), T_ref, H_ref)["zero_pairs_ok"]
    # pairs are selected by H, not by T: no heating anywhere gives zeros
    e0 = t_errors(np.zeros((1, 2)), np.zeros((1, 2)), np.zeros((1, 2)))
    assert e0["max"] == 0.0 and e0["zero_pairs_ok"]


def test_sed_errors_floor_energy_and_weighted_ratio():
    dlam = np.array([1.0, 2.0, 1.0, 1.0])
    L_ref = np.array([[1.0, 10.0, 1e-9, 5.0],
                      [2.0, 20.0, 4.0, 1e-12]])
    L = L_ref.copy()
    L[0, 1] *= 1.0 + 3e-4
    L[0, 2] *= 2.0      # below 1e-6 of the row's peak: not in the element-wise error
    L[1, 0] *= 1.0 - 1e-4
    e = sed_errors(L, L_ref, dlam)
    assert e["max"] == pytest.approx(3e-4, rel=1e-9)
    # energy-weighted L1 per cell, largest over cells:
    # cell 0: (10 * 3e-4 * 2 + 1e-9) / (1 + 20 + 1e-9 + 5), cell 1: 2e-4 / (2 + 40 + 4 + 1e-12)
    e0 = (10 * 3e-4 * 2 + 1e-9) / (1 + 20 + 1e-9 + 5)
    e1 = (2 * 1e-4) / (2 + 40 + 4 + 1e-12)
    assert e["energy_l1"] == pytest.approx(max(e0, e1), rel=1e-9)
    # per wavelength, sum_c L / sum_c L_ref (the paper's SED-weighted mean ratio)
    w = L_ref.sum(axis=0)
    ratio = L.sum(axis=0) / w
    sel = w >= 1e-6 * w.max()
    assert e["weighted_ratio_dev"] == pytest.approx(np.max(np.abs(ratio[sel] - 1)), rel=1e-9)


def test_sed_errors_nan_gives_inf():
    dlam = np.ones(3)
    L_ref = np.array([[1.0, 2.0, 3.0]])
    e = sed_errors(np.array([[1.0, np.nan, 3.0]]), L_ref, dlam)
    assert e["max"] == float("inf")
    assert not np.isfinite(e["energy_l1"])


def test_sed_errors_all_dark_cell():
    e = sed_errors(np.zeros((2, 3)), np.zeros((2, 3)), np.ones(3))
    assert e["max"] == 0.0 and e["energy_l1"] == 0.0 and e["weighted_ratio_dev"] == 0.0
