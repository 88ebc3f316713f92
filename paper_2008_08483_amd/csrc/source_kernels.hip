// Fused source-term kernels for gfx950 (MI355X).
//
// One workgroup evaluates a tile of up to 64 cells (lane = cell).  All of its
// waves share an LDS tile that holds, per (species k, cell):
//     a_k   = C_k * exp(Gt_k)   (double)   -- exp of the chemical potential
//     v_k   = exp(-Gt_k)        (double)
//     w_k   = omega_k accumulator (double)
// with Gt_k = G_k - ln(p_ref/(R T)) the Gibbs-layer output (Eqs. 10-11).
// The exact ANN form of Eq. 4,
//     q_f = exp(nu'.lnC + ln k_f),  q_r = exp(nu''.lnC + ln k_f - ln K_c),
// is re-associated per reaction as
//     q_f - q_r = k_f * prod_reac v^nu' * (prod_reac a^nu' - prod_prod a^nu'')
// which is algebraically identical (ln K_c = -sum_k nu_kj Gt_k, Eq. 11), needs
// one exponential per (cell, reaction) instead of two, gives an exact zero for
// zero concentrations, and keeps the forward/reverse difference in double
// precision so that it does not cancel catastrophically near equilibrium.
// The production layer (Eq. 2) is a scatter of -q / +q per reactant / product
// molecule into the LDS accumulators.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ak_device.h"
#include "ak_internal.h"
#include "ak_math.h"

#ifndef AK_SOURCE_WAVES
#define AK_SOURCE_WAVES 8
#endif

namespace ak {

struct Cell {
    double log2T, invT;
};

// omega accumulators are double in both paths: LDS float atomics stall the
// LDS pipeline on gfx950 far more than double ones (measured), and double
// accumulation costs nothing in accuracy.

// Reaction records are wave-uniform and read with scalar loads into SGPRs.
// (Vector loads of a uniform address return the same 32 bytes to all 64
// lanes and saturate the texture data path; measured.)  A scalar load
// shares its wait counter with LDS instructions, but every wait for the next
// pair's records comes where the loop waits for its LDS reads anyway.

// One reaction's rate of progress q = q_f - q_r for this lane's cell, from
// the LDS tile.  Also returns the LDS addresses of its molecules' entries.
template <bool F64, int NF, int NR>
__device__ __forceinline__ double rate_of_progress(const RxnRec &R, double rev,
                                                   const unsigned char *lds, uint32_t lane_off,
                                                   uint32_t sstride, const Cell c,
                                                   uint32_t (&addr)[NF + NR])
{
    // Arrhenius layer, base 2 (Eq. 6)
    const double t = __builtin_fma(R.beta, c.log2T, __builtin_fma(R.negEoR2, c.invT, R.log2A));
    double Ar, Vr, Ap;
#pragma unroll
    for (int i = 0; i < NF; ++i) {
        addr[i] = lane_off + (uint32_t)R.sp[i] * sstride;
        const double *e = (const double *)(lds + addr[i]);
        const double a = e[0], v = e[1];
        Ar = i ? Ar * a : a;
        Vr = i ? Vr * v : v;
    }
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        addr[NF + i] = lane_off + (uint32_t)R.sp[NF + i] * sstride;
        const double a = *(const double *)(lds + addr[NF + i]);
        Ap = i ? Ap * a : a;
    }
    // prod_reac a^nu' - rev * prod_prod a^nu''  (double: no cancellation loss)
    const double D = __builtin_fma(-rev, Ap, Ar);
    if constexpr (F64) {
        return scale_exp2(Vr * D, t);
    } else {
        // 2^t = 2^n * 2^f with the reduction in double and 2^f, |f| <= 1/2,
        // on the transcendental unit (v_exp_f32)
        const double n = __builtin_rint(t);
        const float f = (float)(t - n);
        const float p = __builtin_amdgcn_exp2f(f);
        return __builtin_ldexp(Vr * D, (int)n) * (double)p;
    }
}

__device__ __forceinline__ void lds_add(double *p, double x)
{
    __hip_atomic_fetch_add(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Production layer (Eq. 2): -q into each reactant molecule's accumulator,
// +q into each product molecule's (nq = -q).
template <int NF, int NR>
__device__ __forceinline__ void scatter(unsigned char *lds, const uint32_t (&addr)[NF + NR],
                                        double q, double nq)
{
#pragma unroll
    for (int i = 0; i < NF; ++i) lds_add((double *)(lds + addr[i] + 16), nq);
#pragma unroll
    for (int i = 0; i < NR; ++i) lds_add((double *)(lds + addr[NF + i] + 16), q);
}

// An LDS atomic reads its data VGPRs when the LDS executes it, so the
// compiler waits for outstanding atomics before it reuses their data
// registers.  Keeping a group's q / -q registers allocated until the next
// group has waited for its own LDS reads (which drains the earlier atomics)
// removes those waits.  The asm statement emits nothing and passes x through
// unchanged; it is not volatile and touches no memory, so the record loads
// stay scalar.
__device__ __forceinline__ double hold(double x, const double (&h)[4])
{
    asm("" : "+v"(x) : "v"(h[0]), "v"(h[1]), "v"(h[2]), "v"(h[3]));
    return x;
}
__device__ __forceinline__ double hold(double x, const double (&h)[8])
{
    asm("" : "+v"(x) : "v"(h[0]), "v"(h[1]), "v"(h[2]), "v"(h[3]), "v"(h[4]), "v"(h[5]),
        "v"(h[6]), "v"(h[7]));
    return x;
}

#ifndef AK_REACTION_GROUP
#define AK_REACTION_GROUP 2
#endif
static_assert(2 * AK_REACTION_GROUP <= kRecordPad, "record reads ahead need the padding");

// The reactions of one run that lie in this wave's range [lo, hi) of the
// sorted list, U consecutive ones at a time so that their LDS reads overlap,
// with the next group's records requested while the current group computes.
template <bool F64, int NF, int NR, int U = AK_REACTION_GROUP>
__device__ __forceinline__ void reaction_run(const MechView &m, const ShapeRun run, int lo,
                                             int hi, unsigned char *lds, uint32_t lane_off,
                                             uint32_t sstride, const Cell c)
{
    const int end = run.start + run.count < hi ? run.start + run.count : hi;
    int j = run.start > lo ? run.start : lo;
    if (j >= end) return;
    const double rev = run.rev;
    // records through a running pointer: the array carries kRecordPad zero
    // records past the last reaction, so the reads ahead of the range need
    // no clamping (what they fetch past `end` is never used)
    const RxnRec *rp = m.rx + j;
    RxnRec r[U];
#pragma unroll
    for (int u = 0; u < U; ++u) r[u] = rp[u];
    double h[2 * U];
#pragma unroll
    for (int i = 0; i < 2 * U; ++i) h[i] = 0.0;
    for (; j < end; j += U, rp += U) {
        RxnRec nx[U];
#pragma unroll
        for (int u = 0; u < U; ++u) nx[u] = rp[U + u];
        uint32_t a[U][NF + NR];
        double q[U];
        q[0] = hold(rate_of_progress<F64, NF, NR>(r[0], rev, lds, lane_off, sstride, c, a[0]), h);
#pragma unroll
        for (int u = 1; u < U; ++u)
            q[u] = rate_of_progress<F64, NF, NR>(r[u], rev, lds, lane_off, sstride, c, a[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double nq = -q[u];
            if (u == 0 || j + u < end) scatter<NF, NR>(lds, a[u], q[u], nq);
            h[2 * u] = q[u];
            h[2 * u + 1] = nq;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) r[u] = nx[u];
    }
}

// This wave's share of the sweep: the contiguous range of the sorted
// reactions given by the mechanism's per-wave split, run by run.  (Taking
// every WAVES-th reaction of each run instead left each wave only a few
// reactions per run, and every run started its record pipeline afresh.)
template <bool F64, int WAVES>
__device__ __forceinline__ void all_reactions(const MechView &m, int wave, unsigned char *lds,
                                              uint32_t lane_off, uint32_t sstride, const Cell c)
{
    const int32_t *seg = WAVES == 16 ? m.seg16 : m.seg8;
    const int lo = seg[wave], hi = seg[wave + 1];
    for (int r = 0; r < m.nruns; ++r) {
        const ShapeRun run = m.runs[r];
        if (run.start >= hi) break;
        if (run.start + run.count <= lo) continue;
        const int s = (run.nf - 1) * 4 + (run.nr - 1);
#define AK_CASE(a, b)                                                                          \
    case (a - 1) * 4 + (b - 1):                                                                \
        reaction_run<F64, a, b>(m, run, lo, hi, lds, lane_off, sstride, c);                    \
        break;
        switch (s) {
            AK_CASE(1, 1) AK_CASE(1, 2) AK_CASE(1, 3) AK_CASE(1, 4)
            AK_CASE(2, 1) AK_CASE(2, 2) AK_CASE(2, 3) AK_CASE(2, 4)
            AK_CASE(3, 1) AK_CASE(3, 2) AK_CASE(3, 3) AK_CASE(3, 4)
            AK_CASE(4, 1) AK_CASE(4, 2) AK_CASE(4, 3) AK_CASE(4, 4)
            default: break;
        }
#undef AK_CASE
    }
}

// Gibbs-layer output in base 2 for one species and cell (Eqs. 10-11): the
// NASA range is chosen per cell (both polynomials are evaluated: a wave's
// cells straddle T_mid more often than not).
__device__ __forceinline__ double gibbs_g2(const SpeciesRec &sr, double T, double lnT, double T2,
                                           double T3, double T4, double invT)
{
    const double glo = sr.lo[0] * lnT + sr.lo[1] * T + sr.lo[2] * T2 + sr.lo[3] * T3 +
                       sr.lo[4] * T4 + sr.lo[5] * invT + sr.lo[6];
    const double ghi = sr.hi[0] * lnT + sr.hi[1] * T + sr.hi[2] * T2 + sr.hi[3] * T3 +
                       sr.hi[4] * T4 + sr.hi[5] * invT + sr.hi[6];
    return T >= sr.T_mid ? ghi : glo;
}

// Inputs of one tile, loaded into registers before any LDS work so that all
// of a wave's HBM reads are in flight at once: this wave's species
// k = wave + i * WAVES (i < KMAX, k < ns), and T, P.  Lanes past the last
// cell hold cell 0's state.
template <typename IO, int KMAX>
struct TileIn {
    IO y[KMAX];
    IO T, P;
};

template <typename IO, int KMAX, int WAVES>
__device__ __forceinline__ void load_tile(const MechView &m, const IO *__restrict__ T,
                                          const IO *__restrict__ P, const IO *__restrict__ Y,
                                          int64_t ldY, int64_t n, int64_t tile_idx, int lane,
                                          int wave, TileIn<IO, KMAX> &in)
{
    const int64_t cell = tile_idx * m.tile + lane;
    const bool valid = cell < n;
    // Every load is issued unconditionally, with no select after it: lanes
    // past the last cell read cell 0 (their results are never stored) and
    // slots past the last species read species 0 (never used).  A load under
    // a branch, or followed by a select of a default, made the compiler wait
    // for it right away, so the wave's loads went out one or two at a time
    // instead of all together.
    const int64_t c = valid ? cell : 0;
    in.T = T[c];
    in.P = P[c];
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
        const int k = wave + i * WAVES;
        in.y[i] = Y[(k < m.ns ? k : 0) * ldY + c];
    }
}

// One tile of m.tile cells starting at cell tile_idx * m.tile (IO: float for
// AK_FP32, double for AK_FP64); block = 64 * WAVES threads, lanes >= m.tile
// already gone; dynamic LDS = ns * m.tile * 24 B; ns <= KMAX * WAVES.
// `in` holds the tile's inputs (see load_tile).
template <typename IO, bool F64, int WAVES, int KMAX>
__device__ __forceinline__ void source_tile(const MechView &m, const IO *__restrict__ T,
                                            const IO *__restrict__ P,
                                            const IO *__restrict__ Y, int64_t ldY, int64_t n,
                                            IO *__restrict__ om, int64_t ldO, int64_t tile_idx,
                                            const TileIn<IO, KMAX> &in, unsigned char *lds)
{
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tile = m.tile;
    const int64_t cell = tile_idx * tile + lane;
    const bool valid = cell < n;                    // owns a real cell
    const uint32_t sstride = species_stride(tile);
    const uint32_t lane_off = (uint32_t)lane * kEntry;

    double Tc = (double)in.T;
    double Pc = (double)in.P;
    const bool tp_bad = !(Tc > 0.0) || !(Pc > 0.0) || !__builtin_isfinite(Tc) ||
                        !__builtin_isfinite(Pc);
    if (tp_bad) {
        Tc = 1000.0;
        Pc = 1.0e5;
    }
    const double lnT = log(Tc), invT = 1.0 / Tc;
    const double T2 = Tc * Tc, T3 = T2 * Tc, T4 = T3 * Tc;

    // (1) this wave's species k = wave + i * WAVES: y_k = max(Y_k, 0) / W_k
    //     and a partial mixture sum (NaN if any input is not finite).  With
    //     at most 8 species per wave the Gibbs layer (Eqs. 10-11) and the
    //     exponentials of the chemical potentials are evaluated here too, all
    //     species at once, so that their dependency chains overlap each other
    //     and the mass fractions still in flight; with more they wait for (3)
    //     and the exponentials are computed one species at a time.
    constexpr bool kEarly = KMAX <= 8;
    double w[KMAX], v[KMAX], yw[KMAX];
    double psum = 0.0;
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
        const int k = wave + i * WAVES;
        if (k < m.ns) {
            const SpeciesRec &sr = m.sp[k];
            if constexpr (kEarly)
                exp2_pair<F64 ? 12 : 10>(gibbs_g2(sr, Tc, lnT, T2, T3, T4, invT), w[i], v[i]);
            const double y = (double)in.y[i];
            yw[i] = __builtin_fmax(y, 0.0) * sr.inv_W;
            psum += __builtin_isfinite(y) ? yw[i] : __builtin_nan("");
            if constexpr (!kEarly) *(double *)(lds + (uint32_t)k * sstride + lane_off) = yw[i];
        }
    }
    if (wave < m.ns) *(double *)(lds + (uint32_t)wave * sstride + lane_off + 16) = psum;
    __syncthreads();
    // (2) mixture sum, same order in every wave
    double sigma = 0.0;
    const int nparts = m.ns < WAVES ? m.ns : WAVES;
    for (int p = 0; p < nparts; ++p)
        sigma += *(const double *)(lds + (uint32_t)p * sstride + lane_off + 16);
    __syncthreads();

    const bool bad = tp_bad || !(sigma > 0.0) || !__builtin_isfinite(sigma);
    if (bad) sigma = 1.0;
    const double rho_hat = Pc / (kRu * Tc * sigma);   // C_k = rho_hat * Y_k / W_k

    // (3) the LDS entries of this wave's species: a = C e^{Gt}, v = e^{-Gt},
    //     accumulator 0
    if constexpr (kEarly) {
#pragma unroll
        for (int i = 0; i < KMAX; ++i) {
            const int k = wave + i * WAVES;
            if (k < m.ns) {
                double *e = (double *)(lds + (uint32_t)k * sstride + lane_off);
                e[0] = rho_hat * (bad ? 0.0 : yw[i]) * w[i];
                e[1] = v[i];
                e[2] = 0.0;
            }
        }
    } else {
        for (int k = wave; k < m.ns; k += WAVES) {
            double wk, vk;
            exp2_pair<F64 ? 12 : 10>(gibbs_g2(m.sp[k], Tc, lnT, T2, T3, T4, invT), wk, vk);
            double *e = (double *)(lds + (uint32_t)k * sstride + lane_off);
            const double ywk = bad ? 0.0 : e[0];
            e[0] = rho_hat * ywk * wk;
            e[1] = vk;
            e[2] = 0.0;
        }
    }
    __syncthreads();

    // (4) rates of progress and production
    Cell cc;
    cc.log2T = lnT * kLog2e;
    cc.invT = invT;
    all_reactions<F64, WAVES>(m, wave, lds, lane_off, sstride, cc);
    __syncthreads();

    // (5) store omega (species-major, coalesced over cells)
    const IO nan = __builtin_nan("");
    for (int k = wave; k < m.ns; k += WAVES) {
        if (valid) {
            const double w = *(const double *)(lds + (uint32_t)k * sstride + lane_off + 16);
            om[k * ldO + cell] = bad ? nan : (IO)w;
        }
    }
    if (wave == 0 && valid && bad) atomicAdd(m.err, 1ull);
}

// Two 8-wave workgroups (or one of 16 waves) fill a CU with 4 waves per SIMD
// only if each wave fits in 128 VGPRs; without the cap the FP64
// instantiation takes a few more and drops to one 8-wave workgroup per CU.
// With 32 species per wave held in registers (more than 128 species in
// 8-wave workgroups, when the LDS holds one tile per CU anyway) the cap is
// relaxed to 256 VGPRs.
#define AK_TWO_TILES_PER_CU __attribute__((amdgpu_waves_per_eu(KMAX > 16 ? 2 : 4)))

// One tile per workgroup.  (A persistent variant that fetched the next
// tile's inputs during the reactions ran slower at 53/325: two resident
// workgroups per CU already overlap one tile's loads with the other's
// reactions, and the tile loop kept the kernel arguments live in SGPRs,
// which spilled inside the reaction loop.)
template <typename IO, bool F64, int WAVES, int KMAX>
__global__ __launch_bounds__(64 * WAVES) AK_TWO_TILES_PER_CU void
source_kernel(MechView m, const IO *__restrict__ T, const IO *__restrict__ P,
              const IO *__restrict__ Y, int64_t ldY, int64_t n, IO *__restrict__ om, int64_t ldO)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // Lanes past a tile narrower than 64 own no LDS column and leave at
    // once; every wave keeps lanes 0..tile-1, so every wave still reaches
    // each barrier, and no later branch has to mask the idle lanes.
    if (lane >= m.tile) return;
    TileIn<IO, KMAX> in;
    load_tile<IO, KMAX, WAVES>(m, T, P, Y, ldY, n, blockIdx.x, lane, wave, in);
    source_tile<IO, F64, WAVES, KMAX>(m, T, P, Y, ldY, n, om, ldO, blockIdx.x, in, lds);
}

// Several requests in one launch: request r owns workgroups
// [d[r].block_begin, d[r].block_begin + ceil(n_r / tile_r)); each workgroup
// finds its request in the descriptor table and runs that request's tile.
template <typename IO, bool F64, int WAVES, int KMAX>
__global__ __launch_bounds__(64 * WAVES) AK_TWO_TILES_PER_CU void
source_batch_kernel(const BatchDesc *__restrict__ d, int nreq)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    const int64_t b = blockIdx.x;
    int lo = 0, hi = nreq - 1;
    while (lo < hi) {                 // last r with block_begin <= b
        const int mid = (lo + hi + 1) >> 1;
        if (d[mid].block_begin <= b) lo = mid; else hi = mid - 1;
    }
    const BatchDesc &r = d[lo];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (lane >= r.m.tile) return;
    TileIn<IO, KMAX> in;
    load_tile<IO, KMAX, WAVES>(r.m, (const IO *)r.T, (const IO *)r.P, (const IO *)r.Y, r.ldY,
                               r.n, b - r.block_begin, lane, wave, in);
    source_tile<IO, F64, WAVES, KMAX>(r.m, (const IO *)r.T, (const IO *)r.P, (const IO *)r.Y,
                                      r.ldY, r.n, (IO *)r.om, r.ldO, b - r.block_begin, in, lds);
}

// ---------------------------------------------------------------------------
// host-side launchers

// species per wave held in registers: ns <= KMAX * WAVES
static int kmax_for(int ns, int waves = AK_SOURCE_WAVES)
{
    const int per = (ns + waves - 1) / waves;
    return per <= 2 ? 2 : per <= 8 ? 8 : per <= 16 ? 16 : 32;
}

template <typename IO, bool F64, int WAVES, int KMAX>
static hipError_t launch_source(const MechView &m, const void *T, const void *P, const void *Y,
                                int64_t ldY, int64_t n, void *om, int64_t ldO, hipStream_t st)
{
    const size_t lds = (size_t)m.ns * species_stride(m.tile);
    auto fn = source_kernel<IO, F64, WAVES, KMAX>;
    hipError_t e = allow_dynamic_lds((const void *)fn);
    if (e != hipSuccess) return e;
    const int64_t blocks = (n + m.tile - 1) / m.tile;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(64 * WAVES), lds, st, m,
                       (const IO *)T, (const IO *)P, (const IO *)Y, ldY, n, (IO *)om, ldO);
    return hipGetLastError();
}

template <typename IO, bool F64, int W>
static hipError_t launch_source_w(const MechView &m, const void *T, const void *P, const void *Y,
                                  int64_t ldY, int64_t n, void *om, int64_t ldO, hipStream_t st)
{
    switch (kmax_for(m.ns, W)) {
        case 2: return launch_source<IO, F64, W, 2>(m, T, P, Y, ldY, n, om, ldO, st);
        case 8: return launch_source<IO, F64, W, 8>(m, T, P, Y, ldY, n, om, ldO, st);
        case 16: return launch_source<IO, F64, W, 16>(m, T, P, Y, ldY, n, om, ldO, st);
        default:
            // 16 waves hold at most 16 species each (ns <= 256)
            if constexpr (W == 16) return hipErrorInvalidValue;
            else return launch_source<IO, F64, W, 32>(m, T, P, Y, ldY, n, om, ldO, st);
    }
}

template <typename IO, bool F64>
static hipError_t launch_source_k(const MechView &m, const void *T, const void *P, const void *Y,
                                  int64_t ldY, int64_t n, void *om, int64_t ldO, hipStream_t st)
{
    if (m.waves == 16) return launch_source_w<IO, F64, 16>(m, T, P, Y, ldY, n, om, ldO, st);
    return launch_source_w<IO, F64, AK_SOURCE_WAVES>(m, T, P, Y, ldY, n, om, ldO, st);
}

size_t source_lds_bytes(int ns, int tile) { return (size_t)ns * species_stride(tile); }

template <typename IO, bool F64, int KMAX>
static hipError_t launch_batch(const BatchDesc *d_desc, int nreq, int64_t blocks, size_t lds,
                               hipStream_t st)
{
    auto fn = source_batch_kernel<IO, F64, AK_SOURCE_WAVES, KMAX>;
    hipError_t e = allow_dynamic_lds((const void *)fn);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(64 * AK_SOURCE_WAVES), lds, st, d_desc,
                       nreq);
    return hipGetLastError();
}

hipError_t source_batch_launch(bool f64, const BatchDesc *d_desc, int nreq, int64_t blocks,
                               size_t lds, int max_ns, hipStream_t st)
{
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    const int k = kmax_for(max_ns);
    if (f64) {
        switch (k) {
            case 2: return launch_batch<double, true, 2>(d_desc, nreq, blocks, lds, st);
            case 8: return launch_batch<double, true, 8>(d_desc, nreq, blocks, lds, st);
            case 16: return launch_batch<double, true, 16>(d_desc, nreq, blocks, lds, st);
            default: return launch_batch<double, true, 32>(d_desc, nreq, blocks, lds, st);
        }
    }
    switch (k) {
        case 2: return launch_batch<float, false, 2>(d_desc, nreq, blocks, lds, st);
        case 8: return launch_batch<float, false, 8>(d_desc, nreq, blocks, lds, st);
        case 16: return launch_batch<float, false, 16>(d_desc, nreq, blocks, lds, st);
        default: return launch_batch<float, false, 32>(d_desc, nreq, blocks, lds, st);
    }
}

hipError_t source_launch(const MechView &m, bool f64, const void *T, const void *P,
                         const void *Y, int64_t ldY, int64_t n, void *om, int64_t ldO,
                         hipStream_t st)
{
    if (f64) return launch_source_k<double, true>(m, T, P, Y, ldY, n, om, ldO, st);
    return launch_source_k<float, false>(m, T, P, Y, ldY, n, om, ldO, st);
}

}  // namespace ak
