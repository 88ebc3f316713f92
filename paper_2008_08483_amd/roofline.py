"""Algorithmic work and MI355X peaks used to state roofline fractions.

The source term is neither a stream (HBM-bound) nor a dense contraction
(MFMA-bound) at realistic mechanism sizes: per cell it reads and writes
O(NS) numbers but evaluates O(NR) exponentials and sparse stoichiometric
sums.  The governing roof is the vector ALU issue rate.

Work is counted in VALU lane-slots: one slot is one lane of one full-rate
VALU instruction (FP32 or FP64 add/mul/FMA; on gfx950 FP64 FMA issues at the
same rate as unpacked FP32).  Transcendental instructions (exp, log,
reciprocal) issue at a quarter of that rate and count 4 slots.

``method_slots`` counts the paper's exact ANN form (Eqs. 2, 4, 6, 9-11)
evaluated sparsely, with the mechanism's own nonzero counts:

  per species: ln C_k (1 transcendental), C_k from Y (3 ops), Gibbs layer
               (7 FMAs over 6 features + bias), mu_k = ln C_k + Gt_k (1);
  per cell:    ln T and 1/T (2 transcendentals), T^2, T^3, T^4, ln C0 (4);
  per reaction j: Arrhenius layer (2 FMAs), x_f = nu'.lnC (nnz nu'_j),
               ln K_c = -nu.Gt (nnz nu_j), ln k_r = ln k_f - ln K_c (1),
               x_r = nu''.lnC (nnz nu''_j), two exponential activations
               (2 transcendentals), q_f - q_r (1), production
               omega += nu q (nnz nu_j).
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


def method_slots(nu_f: np.ndarray, nu_r: np.ndarray) -> float:
    """VALU lane-slots per cell for the paper's exact form (see module doc)."""
    nr, ns = nu_f.shape
    nu = nu_r.astype(int) - nu_f.astype(int)
    nnz_f = int((nu_f != 0).sum())
    nnz_r = int((nu_r != 0).sum())
    nnz = int((nu != 0).sum())
    per_species = TRANS_SLOTS + 3 + 7 + 1
    per_cell = 2 * TRANS_SLOTS + 4
    reactions = nr * (2 + 1 + 1) + nnz_f + nnz + nnz_r + nnz + nr * 2 * TRANS_SLOTS
    return float(ns * per_species + per_cell + reactions)


def hbm_bytes(ns: int, elem_bytes: int) -> int:
    """Compulsory HBM bytes per cell: read T, P, Y (NS); write omega (NS)."""
    return elem_bytes * (2 * ns + 2)
