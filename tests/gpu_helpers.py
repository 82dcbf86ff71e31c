"""Shared helpers of the GPU parity tests and the benchmark's checker."""
from __future__ import annotations

import numpy as np

import oracle
from oracle.compare import sed_errors, t_errors

# Tolerances.  T and SED are the targets of the method (relative T error
# <= 1e-4, SED error <= 1e-3).  H: FP32 accumulation of NL positive terms is
# bounded by NL * 2^-24 (6e-5 at NL = 1000); the bf16 hi+lo split drops the
# lo*lo product and represents each operand to 2^-16, i.e. about 3e-5 more in
# the worst case.  Observed errors are one to two orders of magnitude smaller.
T_TOL = 1e-4
SED_TOL = 1e-3
H_TOL = 1e-4


def strided_rows(n_cells, n_sample):
    if n_cells <= n_sample:
        return np.arange(n_cells)
    step = n_cells // n_sample
    return np.arange(n_sample) * step


# The production T-table of Sections 2 and 5: 2000 points, 3 K to 1500 K.
TABLE = (2000, 3.0, 1500.0)


def oracle_on_rows(grid, J_rows, m_rows, Q=None, table=None):
    """FP64 oracle on the exact FP32 J (and Q) rows the GPU consumed (upcast)."""
    Q = None if Q is None else np.asarray(Q, dtype=np.float64)
    return oracle.run(grid, np.asarray(J_rows, dtype=np.float64), m_rows, Q=Q, table=table)


def check_against_oracle(grid, J_rows, m_rows, T_rows, L_rows, H_rows=None, t_tol=T_TOL,
                         sed_tol=SED_TOL, h_tol=H_TOL, Q=None, table=None):
    H_ref, T_ref, L_ref = oracle_on_rows(grid, J_rows, m_rows, Q=Q, table=table)
    if Q is not None:  # the GPU's H is the absorbed part only
        H_ref_abs = H_ref - np.asarray(Q, dtype=np.float64)
    else:
        H_ref_abs = H_ref
    res = {"T": t_errors(T_rows, T_ref, H_ref), "SED": sed_errors(L_rows, L_ref, grid.dlam)}
    if H_rows is not None:
        pos = H_ref_abs > 0
        rel = np.abs(np.asarray(H_rows, np.float64)[pos] - H_ref_abs[pos]) / H_ref_abs[pos]
        res["H"] = float(rel.max()) if rel.size else 0.0
        assert res["H"] <= h_tol, res
    assert res["T"]["max"] <= t_tol, res
    assert res["T"]["zero_pairs_ok"], res
    assert res["SED"]["max"] <= sed_tol, res
    assert res["SED"]["energy_l1"] <= sed_tol, res
    assert res["SED"]["weighted_ratio_dev"] <= sed_tol, res
    return res
