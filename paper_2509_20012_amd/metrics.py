"""Plan-evaluation helpers applied to final dose / LETd arrays (host side).

These are evaluation, not part of the optimizer: the same functions are applied to
the HIP path's output and to the oracle's output when the two are compared.
"""
from __future__ import annotations

import math

import numpy as np


def d_percent(dose: np.ndarray, volume_fraction: float) -> float:
    """D_v: the minimum dose received by the hottest `volume_fraction` of the voxels,
    i.e. the ascending sort's element at 1-based rank ceil((1 - v) * n) clamped to
    [1, n] (D95 -> v = 0.95, D98 -> v = 0.98; the PTV criterion of Section 2.4.1 is
    D98 >= 95 % of the prescription)."""
    v = np.sort(np.asarray(dose, dtype=np.float64))
    n = v.size
    if n == 0:
        return 0.0
    k = int(math.ceil((1.0 - volume_fraction) * n - 1e-12))
    k = min(max(k, 1), n)
    return float(v[k - 1])


def mean_letd(dose: np.ndarray, letd: np.ndarray) -> float:
    """Arithmetic mean of LETd over voxels that receive dose (d > 0)."""
    d = np.asarray(dose, dtype=np.float64)
    m = d > 0
    if not m.any():
        return 0.0
    return float(np.mean(np.asarray(letd, dtype=np.float64)[m]))


def dose_weighted_mean_letd(dose: np.ndarray, letd: np.ndarray) -> float:
    d = np.asarray(dose, dtype=np.float64)
    s = d.sum()
    return float(np.sum(d * np.asarray(letd, dtype=np.float64)) / s) if s > 0 else 0.0


def plan_report(dose: np.ndarray, letd: np.ndarray, roi: dict) -> dict:
    """D95 / D98 / Dmax of the PTV and mean LETd of every OAR."""
    out = {}
    if "PTV" in roi and len(roi["PTV"]):
        dp = np.asarray(dose)[roi["PTV"]]
        out["PTV_D95"] = d_percent(dp, 0.95)
        out["PTV_D98"] = d_percent(dp, 0.98)
        out["PTV_Dmax"] = float(np.max(dp))
    for name, rows in roi.items():
        if name.startswith("OAR") and len(rows):
            out[f"{name}_mean_LETd"] = mean_letd(np.asarray(dose)[rows], np.asarray(letd)[rows])
            out[f"{name}_Dmean"] = float(np.mean(np.asarray(dose, dtype=np.float64)[rows]))
    return out
