"""Error metrics for grading GPU results against the oracle (test helper).

For every (species k, cell i) entry, with the oracle's gross scale
S_ik = sum_j |nu_kj| (q_f + q_r) and net scale N_ik = sum_j |nu_kj| |q_f - q_r|:

* M1 = |omega - omega_ref| / S           (all entries)
* M2 = |omega - omega_ref| / N           (entries with N >= S / kappa_max)
* M3 = |omega - omega_ref| / |omega_ref| (reported; |omega_ref| >= 1e-3 S)

Entries with S below ``s_floor`` (outside FP32's normal range) are excluded
and counted.
"""

import numpy as np


def grade(om, ref, S, N, kappa_max=1e4, s_floor=0.0):
    om = np.asarray(om, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.longdouble)
    S = np.asarray(S, dtype=np.longdouble)
    N = np.asarray(N, dtype=np.longdouble)
    keep = S > s_floor
    d = np.abs(om.astype(np.longdouble) - ref)
    with np.errstate(divide="ignore", invalid="ignore"):
        m1 = np.where(keep, d / S, 0).astype(np.float64)
        sel2 = keep & (N >= S / kappa_max) & (N > 0)
        m2 = np.where(sel2, d / N, 0).astype(np.float64)
        sel3 = keep & (np.abs(ref) >= 1e-3 * S) & (S > 0)
        m3 = np.where(sel3, d / np.abs(ref), 0).astype(np.float64)
    out = {
        "m1_max": float(m1.max()) if m1.size else 0.0,
        "m1_median": float(np.median(m1[keep])) if keep.any() else 0.0,
        "m2_max": float(m2.max()) if m2.size else 0.0,
        "m2_n": int(sel2.sum()),
        "m3_median": float(np.median(m3[sel3])) if sel3.any() else 0.0,
        "m3_p99": float(np.quantile(m3[sel3], 0.99)) if sel3.any() else 0.0,
        "m3_max": float(m3.max()) if m3.size else 0.0,
        "excluded": int((~keep).sum()),
        "nonfinite": int((~np.isfinite(om)).sum()),
    }
    return out
