"""Error measures of a GPU result against the FP64 oracle (test infrastructure).

Temperature: relative error |T - T_ref| / T_ref over every pair with H_ref > 0
(pairs with H_ref == 0 must have T == 0 exactly).

SED: the FP32 Wien tail underflows long before it matters (the paper's
Section 5.1 and its accuracy figure make the same point), so element-wise
errors are measured where L_ref >= 1e-6 of the cell's peak.  Reported:
  * max and 99.9th-percentile relative error over those elements,
  * the per-cell energy-weighted L1 error sum_l |dL| dlam / sum_l L_ref dlam,
  * the paper's measure: per wavelength, the mean over cells of L/L_ref
    weighted by L_ref, returned as its largest deviation from 1.
"""
from __future__ import annotations

import numpy as np


def t_errors(T, T_ref, H_ref=None):
    T = np.asarray(T, dtype=np.float64)
    T_ref = np.asarray(T_ref, dtype=np.float64)
    pos = T_ref > 0 if H_ref is None else np.asarray(H_ref) > 0
    out = {}
    if np.any(pos):
        rel = np.abs(T[pos] - T_ref[pos]) / T_ref[pos]
        out["max"] = float(np.max(rel)) if np.all(np.isfinite(rel)) else float("inf")
        out["p999"] = float(np.percentile(rel, 99.9))
        out["mean"] = float(np.mean(rel))
    else:
        out["max"] = out["p999"] = out["mean"] = 0.0
    zero = ~pos
    out["zero_pairs_ok"] = bool(np.all(T[zero] == 0.0)) if np.any(zero) else True
    return out


def sed_errors(L, L_ref, dlam, floor=1e-6):
    L = np.asarray(L, dtype=np.float64)
    L_ref = np.asarray(L_ref, dtype=np.float64)
    peak = L_ref.max(axis=1, keepdims=True)
    sel = (L_ref >= floor * peak) & (peak > 0)
    out = {}
    if np.any(sel):
        rel = np.abs(L[sel] - L_ref[sel]) / L_ref[sel]
        out["max"] = float(np.max(rel)) if np.all(np.isfinite(rel)) else float("inf")
        out["p999"] = float(np.percentile(rel, 99.9))
    else:
        out["max"] = out["p999"] = 0.0
    e_ref = (L_ref * dlam[None, :]).sum(axis=1)
    e_err = (np.abs(L - L_ref) * dlam[None, :]).sum(axis=1)
    ok = e_ref > 0
    out["energy_l1"] = float(np.max(e_err[ok] / e_ref[ok])) if np.any(ok) else 0.0
    w = L_ref.sum(axis=0)
    with np.errstate(invalid="ignore", divide="ignore"):
        ratio = np.where(w > 0, (L * (L_ref > 0)).sum(axis=0) / np.where(w > 0, w, 1), 1.0)
    lam_sel = w >= floor * w.max() if w.max() > 0 else np.zeros_like(w, dtype=bool)
    out["weighted_ratio_dev"] = float(np.max(np.abs(ratio[lam_sel] - 1.0))) if np.any(lam_sel) else 0.0
    return out
