// Fused source-term kernels for gfx950 (MI355X).
//
// One workgroup evaluates a tile of up to 64 cells (lane = cell).  All of its
// waves share an LDS tile that holds, per (species k, cell):
//     a_k   = C_k * exp(Gt_k)   (double)   -- exp of the chemical potential
//     v_k   = exp(-Gt_k)        (double)
//     w_k   = omega_k accumulator (float in the FP32 path, double in FP64)
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

#ifndef AK_SOURCE_WAVES
#define AK_SOURCE_WAVES 4
#endif

namespace ak {

struct Cell {
    double log2T, invT;
};

template <bool F64>
struct AccT;
template <>
struct AccT<false> { using type = float; };
template <>
struct AccT<true> { using type = double; };

__device__ __forceinline__ void lds_add(float *p, float x)
{
    __hip_atomic_fetch_add(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_add(double *p, double x)
{
    __hip_atomic_fetch_add(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// One reaction's rate of progress q = q_f - q_r for this lane's cell, from
// the LDS tile.  Also returns the LDS addresses of its molecules' entries.
template <bool F64, int NF, int NR>
__device__ __forceinline__ typename AccT<F64>::type rate_of_progress(const RxnRec &R,
                                                                     const unsigned char *lds,
                                                                     uint32_t lane_off,
                                                                     const Cell c,
                                                                     uint32_t (&addr)[NF + NR])
{
    // Arrhenius layer, base 2 (Eq. 6)
    const double t = __builtin_fma(R.beta, c.log2T, __builtin_fma(R.negEoR2, c.invT, R.log2A));
    double Ar, Vr, Ap;
#pragma unroll
    for (int i = 0; i < NF; ++i) {
        addr[i] = lane_off + R.off[i];
        const double *e = (const double *)(lds + addr[i]);
        const double a = e[0], v = e[1];
        Ar = i ? Ar * a : a;
        Vr = i ? Vr * v : v;
    }
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        addr[NF + i] = lane_off + R.off[NF + i];
        const double a = *(const double *)(lds + addr[NF + i]);
        Ap = i ? Ap * a : a;
    }
    // prod_reac a^nu' - rev * prod_prod a^nu''  (double: no cancellation loss)
    const double D = __builtin_fma(-R.rev, Ap, Ar);
    if constexpr (F64) {
        return exp2(t) * (Vr * D);
    } else {
        // 2^t = 2^n * 2^f with the reduction in double and 2^f, |f| <= 1/2,
        // on the transcendental unit (v_exp_f32)
        const double n = __builtin_rint(t);
        const float f = (float)(t - n);
        const float p = __builtin_amdgcn_exp2f(f);
        return (float)__builtin_ldexp(Vr * D, (int)n) * p;
    }
}

// Production layer (Eq. 2): -q into each reactant molecule's accumulator,
// +q into each product molecule's.
template <bool F64, int NF, int NR>
__device__ __forceinline__ void scatter(unsigned char *lds, const uint32_t (&addr)[NF + NR],
                                        typename AccT<F64>::type q)
{
    using Acc = typename AccT<F64>::type;
#pragma unroll
    for (int i = 0; i < NF; ++i) lds_add((Acc *)(lds + addr[i] + 16), -q);
#pragma unroll
    for (int i = 0; i < NR; ++i) lds_add((Acc *)(lds + addr[NF + i] + 16), q);
}

// Reactions of one shape run: this wave takes reactions start+wave,
// start+wave+WAVES, ...; two at a time so that their loads overlap.
template <bool F64, int NF, int NR, int WAVES>
__device__ __forceinline__ void reaction_run(const MechView &m, const ShapeRun run, int wave,
                                             unsigned char *lds, uint32_t lane_off,
                                             const Cell c, bool active)
{
    const int end = run.start + run.count;
    for (int j = run.start + wave; j < end; j += 2 * WAVES) {
        const int j2 = j + WAVES;
        const bool two = j2 < end;
        uint32_t a1[NF + NR], a2[NF + NR];
        const auto q1 = rate_of_progress<F64, NF, NR>(m.rx[j], lds, lane_off, c, a1);
        const auto q2 = rate_of_progress<F64, NF, NR>(m.rx[two ? j2 : j], lds, lane_off, c, a2);
        if (active) {
            scatter<F64, NF, NR>(lds, a1, q1);
            if (two) scatter<F64, NF, NR>(lds, a2, q2);
        }
    }
}

template <bool F64, int WAVES>
__device__ __forceinline__ void all_reactions(const MechView &m, int wave, unsigned char *lds,
                                              uint32_t lane_off, const Cell c, bool active)
{
    for (int r = 0; r < m.nruns; ++r) {
        const ShapeRun run = m.runs[r];
        const int s = (run.nf - 1) * 4 + (run.nr - 1);
#define AK_CASE(a, b)                                                                  \
    case (a - 1) * 4 + (b - 1):                                                        \
        reaction_run<F64, a, b, WAVES>(m, run, wave, lds, lane_off, c, active);        \
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

// IO: float (AK_FP32) or double (AK_FP64).  Grid: one workgroup per tile of
// m.tile cells; block = 64 * WAVES threads; dynamic LDS = ns * m.tile * 24 B.
template <typename IO, bool F64, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void source_kernel(MechView m, const IO *__restrict__ T,
                                                           const IO *__restrict__ P,
                                                           const IO *__restrict__ Y, int64_t ldY,
                                                           int64_t n, IO *__restrict__ om,
                                                           int64_t ldO)
{
    using Acc = typename AccT<F64>::type;
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tile = m.tile;
    const bool active = lane < tile;               // owns an LDS column
    const int64_t cell = (int64_t)blockIdx.x * tile + lane;
    const bool valid = active && cell < n;          // owns a real cell
    const uint32_t sstride = species_stride(tile);

    double Tc = valid ? (double)T[cell] : 1000.0;
    double Pc = valid ? (double)P[cell] : 1.0e5;
    bool bad = !(Tc > 0.0) || !(Pc > 0.0) || !__builtin_isfinite(Tc) || !__builtin_isfinite(Pc);
    // mixture: sigma = sum_k max(Y_k, 0) / W_k (every wave, same order)
    double sigma = 0.0;
    for (int k = 0; k < m.ns; ++k) {
        const double y = valid ? (double)Y[k * ldY + cell] : 1.0;
        bad |= !__builtin_isfinite(y);
        sigma += __builtin_fmax(y, 0.0) * m.sp[k].inv_W;
    }
    bad |= !(sigma > 0.0);
    if (bad) {
        Tc = 1000.0;
        Pc = 1.0e5;
        sigma = 1.0;
    }
    const double lnT = log(Tc);
    const double invT = 1.0 / Tc;
    const double T2 = Tc * Tc, T3 = T2 * Tc, T4 = T3 * Tc;
    const double rho_hat = Pc / (kRu * Tc * sigma);   // C_k = rho_hat * Y_k / W_k
    // lanes past the tile read column 0 (harmless) and never write
    const uint32_t lane_off = active ? (uint32_t)lane * kEntry : 0u;

    // Gibbs layer (Eqs. 10-11) and the exponentials of the chemical
    // potentials for this wave's species
    for (int k = wave; k < m.ns; k += WAVES) {
        const SpeciesRec &s = m.sp[k];
        double y = valid ? (double)Y[k * ldY + cell] : 1.0;
        y = __builtin_fmax(y, 0.0) * s.inv_W;
        const double glo = s.lo[0] * lnT + s.lo[1] * Tc + s.lo[2] * T2 + s.lo[3] * T3 +
                           s.lo[4] * T4 + s.lo[5] * invT + s.lo[6];
        const double ghi = s.hi[0] * lnT + s.hi[1] * Tc + s.hi[2] * T2 + s.hi[3] * T3 +
                           s.hi[4] * T4 + s.hi[5] * invT + s.hi[6];
        const double g2 = (Tc >= s.T_mid) ? ghi : glo;
        if (active) {
            double *e = (double *)(lds + (uint32_t)k * sstride + lane_off);
            e[0] = rho_hat * y * exp2(g2);
            e[1] = exp2(-g2);
            *(Acc *)(e + 2) = (Acc)0;
        }
    }
    __syncthreads();

    Cell cc;
    cc.log2T = lnT * kLog2e;
    cc.invT = invT;
    all_reactions<F64, WAVES>(m, wave, lds, lane_off, cc, active);
    __syncthreads();

    const IO nan = __builtin_nan("");
    for (int k = wave; k < m.ns; k += WAVES) {
        if (valid) {
            const Acc w = *(const Acc *)(lds + (uint32_t)k * sstride + lane_off + 16);
            om[k * ldO + cell] = bad ? nan : (IO)w;
        }
    }
    if (wave == 0 && valid && bad) atomicAdd(m.err, 1ull);
}

// ---------------------------------------------------------------------------
// host-side launchers

template <typename IO, bool F64, int WAVES>
static hipError_t launch_source(const MechView &m, const void *T, const void *P, const void *Y,
                                int64_t ldY, int64_t n, void *om, int64_t ldO, hipStream_t st)
{
    const size_t lds = (size_t)m.ns * species_stride(m.tile);
    auto fn = source_kernel<IO, F64, WAVES>;
    hipError_t e = hipFuncSetAttribute((const void *)fn,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const int64_t blocks = (n + m.tile - 1) / m.tile;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(64 * WAVES), lds, st, m,
                       (const IO *)T, (const IO *)P, (const IO *)Y, ldY, n, (IO *)om, ldO);
    return hipGetLastError();
}

size_t source_lds_bytes(int ns, int tile) { return (size_t)ns * species_stride(tile); }

hipError_t source_launch(const MechView &m, bool f64, const void *T, const void *P,
                         const void *Y, int64_t ldY, int64_t n, void *om, int64_t ldO,
                         hipStream_t st)
{
    if (f64) return launch_source<double, true, AK_SOURCE_WAVES>(m, T, P, Y, ldY, n, om, ldO, st);
    return launch_source<float, false, AK_SOURCE_WAVES>(m, T, P, Y, ldY, n, om, ldO, st);
}

}  // namespace ak
