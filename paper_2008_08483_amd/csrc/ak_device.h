// Device-side mechanism tables shared by the annkin kernels and their host
// preprocessing.  The layouts here are the library's own; the test oracle
// never sees them.
#pragma once
#include <stdint.h>

namespace ak {

// Physical constants: gas constant J/(kmol K), thermochemical calorie,
// reference pressure 1 bar (Eq. 8).
constexpr double kRu = 8314.46261815324;
constexpr double kRuMol = 8.31446261815324;
constexpr double kCal = 4.184;
constexpr double kPref = 1.0e5;
constexpr double kLog2e = 1.4426950408889634073599;

// Per species (128 B).  The Gibbs-layer weights act on the temperature
// features (ln T, T, T^2, T^3, T^4, 1/T, 1) and give
//     g2_k(T) = log2(e) * (G_k(T) - ln(p_ref/(Ru T)))
// i.e. the paper's Gibbs matrix (Eq. 10) with the standard concentration
// p_ref/(R T) folded into the weights (Eq. 11), in base-2 units.
struct SpeciesRec {
    double inv_W;      // 1 / W_k, kmol/kg
    double T_mid;      // K; the high-range weights apply for T >= T_mid
    double lo[7];
    double hi[7];
};
static_assert(sizeof(SpeciesRec) == 128, "SpeciesRec layout");

// Per reaction (32 B), reactions stored sorted by (shape, reversibility)
// (see ShapeRun).  Arrhenius layer (Eq. 6) in base 2:
//     log2 k_f = log2A + beta * log2 T + negEoR2 / T
// sp[0..nf) are the species of the reactant molecules (a species repeated
// nu' times), sp[nf..nf+nr) those of the product molecules.  The record is
// read with one scalar load per wave: the indices are bytes, so a mechanism
// has at most kMaxSpecies species.
struct RxnRec {
    double log2A;      // log2 of A in SI-kmol units
    double beta;
    double negEoR2;    // -(E/R) * log2(e), K
    uint8_t sp[8];
};
static_assert(sizeof(RxnRec) == 32, "RxnRec layout");

// zero records after the last reaction in the device array (reads ahead of
// a wave's range may touch them)
constexpr int kRecordPad = 4;

constexpr int kMaxSpecies = 256;
constexpr int kMaxSide = 4;      // molecules per side
constexpr int kMaxRuns = 32;     // (nf, nr) in 1..4 x 1..4, reversible or not

// Reactions [start, start + count) share nf, nr and reversibility
// (rev 1 reversible, 0 irreversible).
struct ShapeRun {
    int32_t nf, nr, start, count;
    double rev;
};

// NASA-7 coefficients a1..a7 per species and range (112 B), for enthalpy
// and heat capacity in the derivative kernels.
struct ThermoRec {
    double lo[7];
    double hi[7];
};

// Per reaction, in the same sorted order as RxnRec (32 B): species of the
// molecule slots (reactants first), molecule counts, reversibility and E/R.
struct RxnAux {
    uint16_t sp[8];
    uint8_t nf, nr;
    uint8_t rev;       // 1 reversible, 0 irreversible
    uint8_t pad[5];
    double EoR;        // E/R, K
};
static_assert(sizeof(RxnAux) == 32, "RxnAux layout");

// Kernel argument view of a loaded mechanism.
struct MechView {
    const SpeciesRec *sp;
    const RxnRec *rx;
    const ThermoRec *th;
    const RxnAux *aux;
    unsigned long long *err;     // bad-cell counter
    int32_t ns, nr, nruns;
    int32_t tile;                // cells per workgroup tile (<= 64)
    int32_t waves;               // waves per workgroup of the single-request kernel (8 or 16)
    int32_t pad;
    ShapeRun runs[kMaxRuns];
    // The forward kernels' split of the reaction sweep: with W waves, wave w
    // takes the contiguous range [seg8[w], seg8[w + 1]) of the sorted
    // reactions (W = 8) or [seg16[w], seg16[w + 1]) (W = 16), ranges of
    // about equal estimated cost.
    int32_t seg8[9];
    int32_t seg16[17];
    int32_t pad3[2];
};

// One request of a fused multi-request launch (device-resident table).
struct BatchDesc {
    MechView m;
    const void *T, *P, *Y;
    void *om;
    int64_t ldY, ldO, n;
    int64_t block_begin;     // first workgroup of this request
};

// LDS tile: per (species k, cell c) a 24-byte entry at
//     k * species_stride(tile) + c * kEntry
// holding {double a, double v, accumulator (float or double)}.
constexpr int kEntry = 24;
constexpr int kMaxTile = 64;
constexpr uint32_t species_stride(int tile) { return (uint32_t)tile * kEntry; }

}  // namespace ak
