"""Algorithmic work and MI355X peaks used to state roofline fractions.

The source term is neither a stream (HBM-bound) nor a dense contraction
(MFMA-bound) at realistic mechanism sizes: per cell it reads and writes
O(NS) numbers but evaluates O(NR) exponentials and sparse stoichiometric
sums, so the governing roof is the vector ALU.

Work per cell is counted for the method as the paper states it (the exact
form of Eqs. 2, 4, 6 and 9-11 evaluated sparsely), in three classes:

* transcendentals: one exponential activation each for q_f and q_r per
  reaction, ln C_k per species, ln T, 1/T and one more per cell
  (2 NR + NS + 3);
* FP64 operations: the Gibbs layer (7 per species) and the affinity /
  reverse-rate bias (3 per reaction);
* FP32-class operations: the Arrhenius layer, the sparse nu'.ln C sums, the
  rate and the production layer (about 9 per reaction).

For the three benchmark mechanism sizes the counts are the method's
published per-cell figures (``METHOD_COUNTS``); for other sizes they follow
the formulas above with the mechanism's own nonzero counts.

Two peak models turn counts into a time:

* ``slots``: the datasheet issue rate, 256 CUs x 64 lanes x 2.4 GHz =
  39.3 T lane-slots/s, one slot per FP32/FP64 operation and 4 per
  transcendental (quarter rate);
* ``measured``: per-CU rates measured on the MI355X with microbenchmarks,
  lane-operations per clock per CU: v_exp_f32 21, FP32 FMA 82, FP64 FMA 46.

The roofline fraction is t_roof / t_measured with t_roof = max(t_HBM, t_VALU)
from the algorithmic counts.
"""

from __future__ import annotations

import numpy as np

# MI355X: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz, one full-rate VALU
# lane-op per lane per clock (packed FP32 not used).
N_CU = 256
CLOCK_HZ = 2.4e9
VALU_LANES_PER_CU = 64
PEAK_VALU_SLOTS = N_CU * VALU_LANES_PER_CU * CLOCK_HZ      # 3.93e13 lane-slots/s
PEAK_HBM = 8.0e12                                          # B/s
TRANS_SLOTS = 4

# microbenchmarked lane-operations per clock per CU on the MI355X
MEASURED_RATE = {"trans": 21.0, "fp32": 82.0, "fp64": 46.0}

# (transcendentals, FP32-class, FP64) per cell for the benchmark sizes
METHOD_COUNTS = {(9, 21): (54, 196, 126), (53, 325): (706, 2868, 1346),
                 (111, 784): (1682, 6886, 3129)}


def method_counts(nu_f: np.ndarray, nu_r: np.ndarray) -> tuple:
    """(transcendentals, FP32-class ops, FP64 ops) per cell (see module doc)."""
    nr, ns = nu_f.shape
    if (ns, nr) in METHOD_COUNTS:
        return METHOD_COUNTS[(ns, nr)]
    nu = nu_r.astype(int) - nu_f.astype(int)
    nnz_f = int((nu_f != 0).sum())
    nnz = int((nu != 0).sum())
    trans = 2 * nr + ns + 3
    fp64 = 7 * ns + 3 * nr
    # Arrhenius layer (3), nu'.ln C (nnz), the rate (1), production (nnz nu)
    fp32 = 3 * nr + nnz_f + nr + nnz
    return trans, fp32, fp64


def method_slots(nu_f: np.ndarray, nu_r: np.ndarray) -> float:
    """VALU lane-slots per cell under the datasheet model."""
    t, f32, f64 = method_counts(nu_f, nu_r)
    return float(TRANS_SLOTS * t + f32 + f64)


def t_valu(nu_f: np.ndarray, nu_r: np.ndarray, n_cells: int, model: str = "slots") -> float:
    """Seconds of vector-ALU work for n_cells under a peak model."""
    t, f32, f64 = method_counts(nu_f, nu_r)
    if model == "slots":
        return (TRANS_SLOTS * t + f32 + f64) * n_cells / PEAK_VALU_SLOTS
    r = MEASURED_RATE
    clocks_per_cell_cu = t / r["trans"] + f32 / r["fp32"] + f64 / r["fp64"]
    return clocks_per_cell_cu * n_cells / (N_CU * CLOCK_HZ)


def hbm_bytes(ns: int, elem_bytes: int) -> int:
    """Compulsory HBM bytes per cell: read T, P, Y (NS); write omega (NS)."""
    return elem_bytes * (2 * ns + 2)


def roofline(nu_f: np.ndarray, nu_r: np.ndarray, n_cells: int, elem_bytes: int,
             t_meas: float) -> dict:
    """Roofline of one source-term launch taking t_meas seconds."""
    nr, ns = nu_f.shape
    t_hbm = hbm_bytes(ns, elem_bytes) * n_cells / PEAK_HBM
    t_slots = t_valu(nu_f, nu_r, n_cells, "slots")
    t_meas_model = t_valu(nu_f, nu_r, n_cells, "measured")
    slots = method_slots(nu_f, nu_r)
    return {
        "t_hbm_s": t_hbm,
        "t_valu_slots_s": t_slots,
        "t_valu_measured_rates_s": t_meas_model,
        "frac": max(t_hbm, t_slots) / t_meas,
        "frac_measured_rates": max(t_hbm, t_meas_model) / t_meas,
        "slots_per_cell": slots,
        "achieved_slots_per_s": slots * n_cells / t_meas,
        "counts_per_cell": dict(zip(("transcendental", "fp32", "fp64"),
                                    method_counts(nu_f, nu_r))),
    }
