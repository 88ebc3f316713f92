// The equilibrium-constant layer on its own and its trained replacement
// (Sec. 2.3):
//  - ak_eval_lnkc: ln K_c of every reaction and cell from the Gibbs layer
//    (Eq. 10, with p_ref/(R T) folded into its bias, Eq. 11) followed by the
//    net stoichiometric layer: ln K_c,j = -sum_k nu_kj g_k;
//  - ak_eval_lnkc_net: the approximate network of Architecture 2, one input
//    (ln T, standardized), N_L hidden layers X_{l+1} = elu(X_l W_l + B_l)
//    (Eqs. 12 and 14), a linear readout to the N_R standardized outputs;
//  - ak_eval_source_lnkc: the source term (Eqs. 2-7) with a given ln K_c in
//    place of Eq. 8, the consumer of either;
//  - ak_eval_source_net: the two in sequence, the network as a drop-in for
//    the Gibbs and stoichiometric layers of the reverse rates.
// ln K_c is in (kmol m^-3)^dn, reaction-major and cell-minor:
// lnK[j * ldK + i] for reaction j (descriptor order) and cell i.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <vector>

#include "annkin.h"
#include "ak_device.h"
#include "ak_internal.h"
#include "ak_math.h"

struct ak_kcnet {
    int device = 0;
    int nl = 0, nh = 0, nhp = 0, nr = 0;   // hidden layers, width, padded width, outputs
    double x_mean = 0.0, x_std = 1.0;
    unsigned char *dev = nullptr;          // weights in double, then in float
    size_t n_elems = 0;                    // elements per precision
};

// Tuning: reaction rows per unrolled group in the two row loops, and how
// much hidden-layer recomputation (as a fraction 1/AK_KCNET_CHUNK_DIV of the
// readout's work) the output chunks may add.
#ifndef AK_KCNET_UNROLL
#define AK_KCNET_UNROLL 2
#endif
#ifndef AK_LNKC_UNROLL
#define AK_LNKC_UNROLL 8
#endif
#ifndef AK_KCNET_CHUNK_DIV
#define AK_KCNET_CHUNK_DIV 4
#endif
// Readout of networks of width >= 16 on the matrix cores (1) or the vector
// ALU (0), FP32 and FP64.  The FP64 matrix-core form
// (v_mfma_f64_16x16x4_f64, same operand layouts) differed from the float64
// oracle by about 4e-9 relative, a million times the rounding of the same
// sums on the vector ALU, so the FP64 path stays on the vector ALU (whose
// peak the FP64 matrix cores do not exceed on this device).
#ifndef AK_KCNET_MFMA
#define AK_KCNET_MFMA 1
#endif
#ifndef AK_KCNET_MFMA64
#define AK_KCNET_MFMA64 0
#endif

namespace ak {

// Per reaction, descriptor order (32 B): the distinct species of the
// reaction and their net coefficients nu_kj = nu''_kj - nu'_kj (nonzero).
struct KcRxn {
    uint16_t sp[8];
    int8_t nu[8];
    int32_t cnt;
    int32_t pad[1];
};
static_assert(sizeof(KcRxn) == 32, "KcRxn layout");

namespace {

constexpr double kLn2 = 0.693147180559945309417232121458;

// Both NASA ranges with uniform (scalar) coefficients, then the per-cell
// choice: a per-lane choice of coefficient address would make every load a
// vector load.
__device__ __forceinline__ double g2_of(const SpeciesRec &sr, double T, double lnT, double T2,
                                        double T3, double T4, double invT)
{
    const double glo = sr.lo[0] * lnT + sr.lo[1] * T + sr.lo[2] * T2 + sr.lo[3] * T3 +
                       sr.lo[4] * T4 + sr.lo[5] * invT + sr.lo[6];
    const double ghi = sr.hi[0] * lnT + sr.hi[1] * T + sr.hi[2] * T2 + sr.hi[3] * T3 +
                       sr.hi[4] * T4 + sr.hi[5] * invT + sr.hi[6];
    return T >= sr.T_mid ? ghi : glo;
}

// One 64-cell tile per workgroup (one wave), lane = cell; blockIdx.y picks
// a chunk of `rpc` reactions, so that a batch of few tiles still gives the
// chip enough waves.  Each lane keeps its cell's Gibbs-layer outputs
// g2_k = log2(e) (G_k - ln(p_ref/(R T))) in its own LDS column (no barrier
// needed); every reaction row is one coalesced store of 64 cells.  MAXT is
// the records' entry count (unused entries carry nu = 0), so the reaction
// loop has no data-dependent trip count and unrolls.
template <typename IO, int MAXT>
__global__ __launch_bounds__(64) void lnkc_kernel(MechView m, const KcRxn *__restrict__ kr,
                                                  int rpc, const IO *__restrict__ T, int64_t n,
                                                  IO *__restrict__ lnK, int64_t ldK)
{
    extern __shared__ double g2[];
    const int lane = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * 64 + lane;
    const bool live = i < n;
    const double t = (double)T[live ? i : n - 1];
    const bool bad = !(t > 0.0) || !__builtin_isfinite(t);
    const double Tc = bad ? 1000.0 : t;
    const double lnT = log(Tc), T2 = Tc * Tc, T3 = T2 * Tc, T4 = T3 * Tc, invT = 1.0 / Tc;
    for (int k = 0; k < m.ns; ++k) g2[k * 64 + lane] = g2_of(m.sp[k], Tc, lnT, T2, T3, T4, invT);
    const IO nan = (IO)__builtin_nan("");
    const int j0 = blockIdx.y * rpc, j1 = min(m.nr, j0 + rpc);
#pragma unroll AK_LNKC_UNROLL
    for (int j = j0; j < j1; ++j) {
        const KcRxn *r = &kr[j];
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < MAXT; ++q) acc += (double)r->nu[q] * g2[r->sp[q] * 64 + lane];
        if (live) lnK[(int64_t)j * ldK + i] = bad ? nan : (IO)(-acc * kLn2);
    }
    if (live && bad && blockIdx.y == 0) atomicAdd(m.err, 1ull);
}

// The same ln K_c with the two linear layers composed per reaction: over a
// temperature interval on which every species of reaction j keeps its NASA
// range, ln K_c,j = F(T) . w_j with F = (ln T, T, T^2, T^3, T^4, 1/T, 1) and
// w_j = -ln 2 sum_k nu_kj c_k (c_k the species' Gibbs-layer weights of that
// range).  A reaction has one interval per distinct T_mid of its species
// plus one (PM at most): its record holds the PM - 1 interval bounds, then
// PM weight vectors.  Lane = cell, no LDS; every weight is a scalar operand.
template <typename IO, int PM>
__global__ __launch_bounds__(256) void lnkc_fold_kernel(const double *__restrict__ fw, int nr,
                                                        int rpc, const IO *__restrict__ T,
                                                        int64_t n, IO *__restrict__ lnK,
                                                        int64_t ldK,
                                                        unsigned long long *err)
{
    constexpr int FS = (PM - 1) + 7 * PM;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double t = (double)T[i];
    const bool bad = !(t > 0.0) || !__builtin_isfinite(t);
    const double Tc = bad ? 1000.0 : t;
    const double F[7] = {log(Tc), Tc, Tc * Tc, Tc * Tc * Tc, (Tc * Tc) * (Tc * Tc), 1.0 / Tc, 1.0};
    const IO nan = (IO)__builtin_nan("");
    const int j0 = blockIdx.y * rpc, j1 = min(nr, j0 + rpc);
#pragma unroll 2
    for (int j = j0; j < j1; ++j) {
        const double *w = fw + (int64_t)j * FS;
        const double *v = w + (PM - 1);
        double acc = v[0] * F[0];
#pragma unroll
        for (int f = 1; f < 7; ++f) acc = __builtin_fma(v[f], F[f], acc);
#pragma unroll
        for (int q = 1; q < PM; ++q) {
            const double *u = v + 7 * q;
            double a2 = u[0] * F[0];
#pragma unroll
            for (int f = 1; f < 7; ++f) a2 = __builtin_fma(u[f], F[f], a2);
            acc = Tc >= w[q - 1] ? a2 : acc;
        }
        lnK[(int64_t)j * ldK + i] = bad ? nan : (IO)acc;
    }
    if (bad && blockIdx.y == 0) atomicAdd(err, 1ull);
}

// f(std::integral_constant<int, i>) for i = 0 .. N-1, unrolled at compile
// time so that register arrays indexed by i never go to scratch memory
template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// fused multiply-add in the element type (float stays float)
__device__ __forceinline__ float fma_e(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_e(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename E>
__device__ __forceinline__ E elu(E x)
{
    if constexpr (sizeof(E) == 8)
        return x >= 0.0 ? x : expm1(x);
    else
        return x >= 0.0f ? x : expm1f(x);
}

// The approximate network, lane = cell.  Weight layout (element type E,
// width NH padded with zero weights to the template width):
//   w0[NH], b0[NH];  per further hidden layer W^T[NH][NH] (output-major),
//   b[NH];  readout W^T[nr][NH] and b[nr], with the outputs' standard
//   deviation and mean folded in.
// Every weight index is uniform across the wave (scalar loads); the
// activations stay in registers.  Sums run in a fixed order.
// blockIdx.y picks a chunk of `rpc` outputs (each chunk recomputes the
// hidden layers of its cells: cheap next to the readout when it is chosen).
template <typename E, int NH>
__global__ __launch_bounds__(256) void kcnet_kernel(const E *__restrict__ w, int nl, int nr,
                                                    int rpc, double x_mean, double x_std,
                                                    const E *__restrict__ T, int64_t n,
                                                    E *__restrict__ lnK, int64_t ldK)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double t = (double)T[i];
    const bool bad = !(t > 0.0) || !__builtin_isfinite(t);
    const E z = (E)((log(bad ? 1.0 : t) - x_mean) / x_std);
    E h[NH];
    static_for<0, NH>([&](auto o) { h[o] = elu<E>(z * w[o] + w[NH + o]); });
    const E *p = w + 2 * NH;
    for (int l = 1; l < nl; ++l) {
        E g[NH];
        static_for<0, NH>([&](auto o) {
            E acc = p[NH * NH + o];
            static_for<0, NH>([&](auto q) { acc = fma_e(h[q], p[o * NH + q], acc); });
            g[o] = elu<E>(acc);
        });
        static_for<0, NH>([&](auto o) { h[o] = g[o]; });
        p += NH * NH + NH;
    }
    const E *bo = p + (int64_t)nr * NH;
    const E nan = (E)__builtin_nan("");
    const int j0 = blockIdx.y * rpc, j1 = min(nr, j0 + rpc);
#pragma unroll AK_KCNET_UNROLL
    for (int j = j0; j < j1; ++j) {
        const E *wj = p + (int64_t)j * NH;
        E acc = bo[j];
        static_for<0, NH>([&](auto q) { acc = fma_e(h[q], wj[q], acc); });
        lnK[(int64_t)j * ldK + i] = bad ? nan : acc;
    }
}

typedef float ak_f32x4 __attribute__((ext_vector_type(4)));
typedef double ak_f64x4 __attribute__((ext_vector_type(4)));

// One 16 x 16 x 4 matrix-core step D = A B + D in the element type
__device__ __forceinline__ ak_f32x4 mfma16x16x4(float a, float b, ak_f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ ak_f64x4 mfma16x16x4(double a, double b, ak_f64x4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// FP32 networks of width 16 and more: the hidden layers as in kcnet_kernel
// (lane = cell, activations in registers), then the readout, a
// [reactions x N_H] x [N_H x cells] product, on the matrix cores
// (v_mfma_f32_16x16x4_f32: 16 reactions x 16 cells per block, 4 hidden
// units per step).  Each wave of the 4 stages its 64 cells' activations in
// LDS (rows padded by one float against bank conflicts) and reads them back
// as the B operand; the A operand is the readout weights (reaction-major,
// standardization folded in); the bias is added to the result.  No lane
// leaves early (the matrix instructions need the whole wave): lanes past the
// last cell compute the last cell again and store nothing.  The k-steps run
// in a fixed order (bitwise repeatable).
template <typename E, int NH>
__global__ __launch_bounds__(256) void kcnet_mfma_kernel(const E *__restrict__ w, int nl, int nr,
                                                         int rpc, double x_mean, double x_std,
                                                         const E *__restrict__ T, int64_t n,
                                                         E *__restrict__ lnK, int64_t ldK)
{
    using V4 = typename std::conditional<sizeof(E) == 8, ak_f64x4, ak_f32x4>::type;
    constexpr int LDH = NH + 1;
    constexpr int KS = NH / 4;
    // dynamic LDS: per wave 64 rows of LDH elements, then 64 bad-cell flags
    extern __shared__ double kc_lds_d[];
    E *kc_lds = (E *)kc_lds_d;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    E *Hw = kc_lds + wave * 64 * LDH;
    E *badw = kc_lds + 4 * 64 * LDH + wave * 64;
    const int64_t c0 = (int64_t)blockIdx.x * 256 + wave * 64;
    const int64_t i = c0 + lane;
    const int64_t ic = i < n ? i : n - 1;
    const double t = (double)T[ic];
    const bool bad = !(t > 0.0) || !__builtin_isfinite(t);
    const E z = (E)((log(bad ? 1.0 : t) - x_mean) / x_std);
    E h[NH];
    static_for<0, NH>([&](auto o) { h[o] = elu<E>(z * w[o] + w[NH + o]); });
    const E *p = w + 2 * NH;
    for (int l = 1; l < nl; ++l) {
        E g[NH];
        static_for<0, NH>([&](auto o) {
            E acc = p[NH * NH + o];
            static_for<0, NH>([&](auto q) { acc = fma_e(h[q], p[o * NH + q], acc); });
            g[o] = elu<E>(acc);
        });
        static_for<0, NH>([&](auto o) { h[o] = g[o]; });
        p += NH * NH + NH;
    }
    static_for<0, NH>([&](auto q) { Hw[lane * LDH + q] = h[q]; });
    badw[lane] = bad ? (E)1 : (E)0;
    __syncthreads();
    // B operand: lane l holds H[cell 16 cb + l % 16][unit 4 kb + l / 16]
    const int lm = lane & 15, lk = lane >> 4;
    E bfr[4][KS];
    bool bcol[4];
    static_for<0, 4>([&](auto cb) {
        static_for<0, KS>([&](auto kb) { bfr[cb][kb] = Hw[(cb * 16 + lm) * LDH + kb * 4 + lk]; });
        bcol[cb] = badw[cb * 16 + lm] != (E)0;
    });
    const E *bo = p + (int64_t)nr * NH;
    const E nan = (E)__builtin_nan("");
    const int j0 = blockIdx.y * rpc, j1 = min(nr, j0 + rpc);
    for (int jb = j0; jb < j1; jb += 16) {
        // A operand: lane l holds W^T[reaction jb + l % 16][unit 4 kb + l / 16]
        const int ja = min(jb + lm, nr - 1);
        E afr[KS];
        static_for<0, KS>([&](auto kb) { afr[kb] = p[(int64_t)ja * NH + kb * 4 + lk]; });
        // this lane's result rows: reactions jb + 4 (l / 16) + v
        E bias[4];
        static_for<0, 4>([&](auto v) { bias[v] = bo[min(jb + 4 * lk + (int)v, nr - 1)]; });
        static_for<0, 4>([&](auto cb) {
            V4 acc = {(E)0, (E)0, (E)0, (E)0};
            static_for<0, KS>([&](auto kb) { acc = mfma16x16x4(afr[kb], bfr[cb][kb], acc); });
            const int64_t cell = c0 + cb * 16 + lm;
            static_for<0, 4>([&](auto v) {
                const int j = jb + 4 * lk + v;
                if (j < j1 && cell < n)
                    lnK[(int64_t)j * ldK + cell] = bcol[cb] ? nan : acc[decltype(v)::value] + bias[v];
            });
        });
    }
}

// One run of reactions of the same shape (NF reactant and NR product
// molecules, one reversibility) within [j, end): rates with the given ln K_c
// into this wave's accumulators.  The shape is a compile-time constant, so
// every loop unrolls and the next reactions' record loads can be issued
// while the current ones compute.
template <typename IO, int NF, int NR>
__device__ __forceinline__ void lnk_run(const MechView &m, const int32_t *__restrict__ order,
                                        int j, int end, double rev, const double *l2C,
                                        double *acc, int lane, const IO *__restrict__ lnK,
                                        int64_t ldK, int64_t c, double log2T, double invT)
{
#pragma unroll 2
    for (; j < end; ++j) {
        const RxnRec r = m.rx[j];
        const double t0 = r.log2A + r.beta * log2T + r.negEoR2 * invT;
        double tf = t0;
#pragma unroll
        for (int q = 0; q < NF; ++q) tf += l2C[r.sp[q] * 64 + lane];
        double qn = scale_exp2(1.0, tf);
        if (rev != 0.0) {
            double tr = t0 - (double)lnK[(int64_t)order[j] * ldK + c] * kLog2e;
#pragma unroll
            for (int q = 0; q < NR; ++q) tr += l2C[r.sp[NF + q] * 64 + lane];
            qn -= scale_exp2(1.0, tr);
        }
#pragma unroll
        for (int q = 0; q < NF; ++q) acc[r.sp[q] * 64 + lane] -= qn;
#pragma unroll
        for (int q = 0; q < NR; ++q) acc[r.sp[NF + q] * 64 + lane] += qn;
    }
}

// The source term with a given ln K_c, one 64-cell tile per workgroup of SW
// waves, lane = cell.  LDS holds the tile's log2 C_k (written by the waves
// in turn, species k = wave + SW i) and, per wave, omega_k accumulators for
// the contiguous share of the reactions the wave sweeps (its own region: no
// atomics).  The shares are added in wave order at the end, so every omega_k
// is a sum in a fixed order.  Reactions run in the library's sorted order;
// ln K_c is read at the descriptor index of each.
template <typename IO, int SW>
__global__ __launch_bounds__(64 * SW) void source_lnkc_kernel(MechView m,
                                                              const int32_t *__restrict__ order,
                                                              const IO *__restrict__ T,
                                                              const IO *__restrict__ P,
                                                              const IO *__restrict__ Y,
                                                              int64_t ldY, int64_t n,
                                                              const IO *__restrict__ lnK,
                                                              int64_t ldK, IO *__restrict__ om,
                                                              int64_t ldO)
{
    extern __shared__ double lds[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ns = m.ns;
    double *l2C = lds;
    double *acc = lds + (size_t)ns * 64 * (1 + wave);
    double *part = lds + (size_t)ns * 64 * (1 + SW);   // [SW][64]
    const int64_t i = (int64_t)blockIdx.x * 64 + lane;
    const bool live = i < n;
    const int64_t c = live ? i : n - 1;
    const double Tc = (double)T[c], Pc = (double)P[c];
    const bool tp_bad = !(Tc > 0.0) || !(Pc > 0.0) || !__builtin_isfinite(Tc) ||
                        !__builtin_isfinite(Pc);
    // mixture sum: a partial per wave, then the waves' partials in order (a
    // non-finite mass fraction makes it NaN)
    double ps = 0.0;
    for (int k = wave; k < ns; k += SW) {
        const double y = (double)Y[(int64_t)k * ldY + c];
        ps += __builtin_isfinite(y) ? (y > 0.0 ? y : 0.0) * m.sp[k].inv_W : __builtin_nan("");
    }
    part[wave * 64 + lane] = ps;
    __syncthreads();
    double sigma = 0.0;
    for (int w = 0; w < SW; ++w) sigma += part[w * 64 + lane];
    const bool bad = tp_bad || !(sigma > 0.0) || !__builtin_isfinite(sigma);
    const double Tu = bad ? 1000.0 : Tc;
    const double rh = bad ? 0.0 : Pc / (kRu * Tu * sigma);
    for (int k = wave; k < ns; k += SW) {
        const double y = (double)Y[(int64_t)k * ldY + c];
        const double C = rh * (y > 0.0 ? y : 0.0) * m.sp[k].inv_W;
        // an absent species: a floor far below any rate's range, so that
        // 2^t underflows to an exact 0 through the finite exponent path
        l2C[k * 64 + lane] = C > 0.0 ? log2(C) : -4096.0;
    }
    for (int k = 0; k < ns; ++k) acc[k * 64 + lane] = 0.0;
    __syncthreads();
    const double log2T = log2(Tu), invT = 1.0 / Tu;
    const int j0 = (int)((int64_t)m.nr * wave / SW), j1 = (int)((int64_t)m.nr * (wave + 1) / SW);
    // this wave's range, run by run (runs hold reactions of one shape)
    for (int rn = 0; rn < m.nruns; ++rn) {
        const ShapeRun run = m.runs[rn];
        const int a = run.start > j0 ? run.start : j0;
        const int b = run.start + run.count < j1 ? run.start + run.count : j1;
        if (a >= b) continue;
        const int shape = (run.nf - 1) * 4 + (run.nr - 1);
#define AK_LNK(F, R)                                                                         \
    case (F - 1) * 4 + (R - 1):                                                              \
        lnk_run<IO, F, R>(m, order, a, b, run.rev, l2C, acc, lane, lnK, ldK, c, log2T, invT); \
        break;
        switch (shape) {
            AK_LNK(1, 1) AK_LNK(1, 2) AK_LNK(1, 3) AK_LNK(1, 4)
            AK_LNK(2, 1) AK_LNK(2, 2) AK_LNK(2, 3) AK_LNK(2, 4)
            AK_LNK(3, 1) AK_LNK(3, 2) AK_LNK(3, 3) AK_LNK(3, 4)
            AK_LNK(4, 1) AK_LNK(4, 2) AK_LNK(4, 3) AK_LNK(4, 4)
            default: break;
        }
#undef AK_LNK
    }
    __syncthreads();
    // the waves' shares in wave order; this wave stores species k = wave + SW i
    bool nonfinite = false;
    const IO nan = (IO)__builtin_nan("");
    for (int k = wave; k < ns; k += SW) {
        double v = 0.0;
        for (int w = 0; w < SW; ++w) v += lds[(size_t)ns * 64 * (1 + w) + k * 64 + lane];
        if (!__builtin_isfinite(v)) nonfinite = true;
        if (live) om[(int64_t)k * ldO + i] = bad ? nan : (IO)v;
    }
    // one count per bad cell: the waves' flags meet in LDS
    part[wave * 64 + lane] = nonfinite ? 1.0 : 0.0;
    __syncthreads();
    if (wave == 0 && live) {
        bool any = bad;
        for (int w = 0; w < SW; ++w) any = any || part[w * 64 + lane] != 0.0;
        if (any) atomicAdd(m.err, 1ull);
    }
}

// ---------------------------------------------------------------------------
// host side

std::mutex g_kc_mu;   // guards the lazy tables of every mechanism
constexpr int kMaxPieces = 4;   // temperature intervals per reaction of the composed layers

// LDS of the given-ln K_c source term with `sw` sweep waves per tile
size_t source_lnkc_lds(int ns, int sw)
{
    return ((size_t)ns * 64 * (1 + sw) + (size_t)64 * sw) * sizeof(double);
}

// The most sweep waves (4, 2 or 1) whose LDS fits the device
int source_lnkc_waves(int ns, int lds_max)
{
    for (int sw = 4; sw > 1; sw /= 2)
        if (source_lnkc_lds(ns, sw) <= (size_t)lds_max) return sw;
    return 1;
}
size_t lnkc_lds(int ns) { return (size_t)ns * 64 * sizeof(double); }

// The descriptor-order reaction table and the sorted-to-descriptor index,
// uploaded at the first call that needs them.
int kc_tables(const ak_mechanism *m, const KcRxn **kr, const int32_t **order)
{
    std::lock_guard<std::mutex> l(g_kc_mu);
    if (!m->kc_dev) {
        const int nr = m->nr;
        std::vector<KcRxn> t(nr);
        for (int s = 0; s < nr; ++s) {
            const RxnAux &x = m->host_aux[s];
            KcRxn &r = t[m->rxn_order[s]];
            std::memset(&r, 0, sizeof r);
            int sp[8], nu[8], cnt = 0;
            for (int q = 0; q < x.nf + x.nr; ++q) {
                const int k = x.sp[q], d = q < x.nf ? -1 : 1;
                int a = 0;
                while (a < cnt && sp[a] != k) ++a;
                if (a == cnt) { sp[cnt] = k; nu[cnt] = 0; ++cnt; }
                nu[a] += d;
            }
            for (int a = 0; a < cnt; ++a)
                if (nu[a] != 0) {
                    r.sp[r.cnt] = (uint16_t)sp[a];
                    r.nu[r.cnt] = (int8_t)nu[a];
                    ++r.cnt;
                }
        }
        int maxcnt = 0;
        for (const KcRxn &r : t) maxcnt = std::max(maxcnt, (int)r.cnt);
        m->kc_wide = maxcnt > 4;
        // the composed layers: per reaction the distinct T_mid of its
        // species bound the intervals; the largest count sets the layout
        std::vector<std::vector<double>> thr(nr);
        int pm = 1;
        for (int j = 0; j < nr; ++j) {
            for (int q = 0; q < t[j].cnt; ++q) thr[j].push_back(m->host_species[t[j].sp[q]].T_mid);
            std::sort(thr[j].begin(), thr[j].end());
            thr[j].erase(std::unique(thr[j].begin(), thr[j].end()), thr[j].end());
            pm = std::max(pm, (int)thr[j].size() + 1);
        }
        std::vector<double> fold;
        if (pm <= kMaxPieces) {
            const int fs = (pm - 1) + 7 * pm;
            fold.assign((size_t)fs * nr, 0.0);
            for (int j = 0; j < nr; ++j) {
                double *w = &fold[(size_t)j * fs];
                const int np = (int)thr[j].size() + 1;
                for (int q = 0; q < pm - 1; ++q)
                    w[q] = q < np - 1 ? thr[j][q] : __builtin_inf();
                for (int q = 0; q < pm; ++q) {
                    double *v = w + (pm - 1) + 7 * q;
                    const int qq = std::min(q, np - 1);   // unused intervals repeat the last
                    for (int a = 0; a < t[j].cnt; ++a) {
                        const SpeciesRec &sr = m->host_species[t[j].sp[a]];
                        const bool hi = qq > 0 && sr.T_mid <= thr[j][qq - 1];
                        for (int f = 0; f < 7; ++f)
                            v[f] += (double)t[j].nu[a] * (hi ? sr.hi[f] : sr.lo[f]);
                    }
                    for (int f = 0; f < 7; ++f) v[f] *= -kLn2;
                }
            }
        }
        m->kc_pieces = fold.empty() ? 0 : pm;
        std::vector<int32_t> ord(m->rxn_order.begin(), m->rxn_order.end());
        const size_t o_ord = sizeof(KcRxn) * nr;
        const size_t o_fold = (o_ord + sizeof(int32_t) * nr + 255) & ~(size_t)255;
        const size_t bytes = o_fold + sizeof(double) * fold.size();
        unsigned char *d = nullptr;
        hipError_t e = hipMalloc(&d, bytes);
        if (e == hipSuccess) e = hipMemcpy(d, t.data(), sizeof(KcRxn) * nr, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(d + o_ord, ord.data(), sizeof(int32_t) * nr, hipMemcpyHostToDevice);
        if (e == hipSuccess && !fold.empty())
            e = hipMemcpy(d + o_fold, fold.data(), sizeof(double) * fold.size(),
                          hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            if (d) (void)hipFree(d);
            return hip_error(e, "ln K_c tables");
        }
        m->kc_dev = d;
        m->kc_fold_off = o_fold;
    }
    *kr = (const KcRxn *)m->kc_dev;
    *order = (const int32_t *)(m->kc_dev + sizeof(KcRxn) * m->nr);
    return AK_OK;
}

int check_prec(const char *fn, int prec)
{
    if (prec != AK_FP32 && prec != AK_FP64)
        return set_error(AK_EINVAL, "%s: bad precision %d", fn, prec);
    return AK_OK;
}

int check_cells(const char *fn, int64_t n)
{
    if (n < 0) return set_error(AK_EINVAL, "%s: n_cells < 0", fn);
    if (n > (int64_t)1 << 40) return set_error(AK_E2BIG, "%s: n_cells too large", fn);
    return AK_OK;
}

// Reaction (or output) chunks per tile: enough that the grid holds about
// `target` waves, at least `minr` rows per chunk, and at most `cap` chunks.
int chunks_for(int64_t tiles, int nr, int64_t target, int minr, int64_t cap)
{
    int64_t c = (target + tiles - 1) / tiles;
    c = std::min<int64_t>(c, std::max(1, nr / minr));
    c = std::min<int64_t>(c, std::max<int64_t>(1, cap));
    return (int)std::max<int64_t>(1, c);
}

constexpr int64_t kTargetWaves = 8192;   // 8 per SIMD
constexpr bool kMfmaReadout = AK_KCNET_MFMA != 0;
constexpr bool kMfmaReadout64 = AK_KCNET_MFMA64 != 0;

template <typename T>
struct Tag {
    using type = T;
};

template <typename E>
hipError_t launch_kcnet(const ak_kcnet *net, const E *w, const void *T, int64_t n, void *lnK,
                        int64_t ldK, hipStream_t st)
{
    const int64_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    // a chunk repeats the hidden layers: keep that below the readout's work
    const int64_t hidden = (int64_t)net->nhp * (1 + 8 * net->nl) +
                           (int64_t)(net->nl - 1) * net->nhp * net->nhp;
    const int64_t readout = (int64_t)net->nhp * net->nr;
    const int ch = chunks_for((n + 63) / 64, net->nr, kTargetWaves, 16,
                              readout / (hidden * AK_KCNET_CHUNK_DIV));
    int rpc = (net->nr + ch - 1) / ch;
    if (net->nhp >= 16 && (sizeof(E) == 4 ? kMfmaReadout : kMfmaReadout64)) {
        {
            // whole 16-reaction blocks per chunk
            rpc = (rpc + 15) & ~15;
            const dim3 g((unsigned)blocks, (unsigned)((net->nr + rpc - 1) / rpc)), b(256);
            auto go = [&](auto kern, int nh) {
                const size_t lds = ((size_t)4 * 64 * (nh + 1) + 4 * 64) * sizeof(E);
                hipError_t e = allow_dynamic_lds((const void *)kern);
                if (e != hipSuccess) return e;
                hipLaunchKernelGGL(kern, g, b, lds, st, w, net->nl, net->nr, rpc, net->x_mean,
                                   net->x_std, (const E *)T, n, (E *)lnK, ldK);
                return hipGetLastError();
            };
            switch (net->nhp) {
                case 16: return go(kcnet_mfma_kernel<E, 16>, 16);
                case 32: return go(kcnet_mfma_kernel<E, 32>, 32);
                case 64: return go(kcnet_mfma_kernel<E, 64>, 64);
                default: return hipErrorInvalidValue;
            }
        }
    }
    const dim3 g((unsigned)blocks, (unsigned)((net->nr + rpc - 1) / rpc)), b(256);
#define AK_KCNET(NH)                                                                         \
    hipLaunchKernelGGL((kcnet_kernel<E, NH>), g, b, 0, st, w, net->nl, net->nr, rpc,          \
                       net->x_mean, net->x_std, (const E *)T, n, (E *)lnK, ldK)
    switch (net->nhp) {
        case 8: AK_KCNET(8); break;
        case 16: AK_KCNET(16); break;
        case 32: AK_KCNET(32); break;
        case 64: AK_KCNET(64); break;
        default: return hipErrorInvalidValue;
    }
#undef AK_KCNET
    return hipGetLastError();
}

hipError_t kcnet_launch(const ak_kcnet *net, int prec, const void *T, int64_t n, void *lnK,
                        int64_t ldK, hipStream_t st)
{
    if (prec == AK_FP64) return launch_kcnet<double>(net, (const double *)net->dev, T, n, lnK, ldK, st);
    return launch_kcnet<float>(net, (const float *)(net->dev + net->n_elems * sizeof(double)), T, n,
                               lnK, ldK, st);
}

hipError_t source_lnkc_launch(const ak_mechanism *m, const int32_t *order, int prec,
                              const void *T, const void *P, const void *Y, int64_t ldY, int64_t n,
                              const void *lnK, int64_t ldK, void *om, int64_t ldO, hipStream_t st)
{
    const int64_t blocks = (n + 63) / 64;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    const int sw = source_lnkc_waves(m->ns, m->lds_max);
    const size_t lds = source_lnkc_lds(m->ns, sw);
    auto go = [&](auto kern, auto tag) {
        using IO = typename decltype(tag)::type;
        hipError_t e = allow_dynamic_lds((const void *)kern);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(64 * sw), lds, st, m->view, order,
                           (const IO *)T, (const IO *)P, (const IO *)Y, ldY, n,
                           (const IO *)lnK, ldK, (IO *)om, ldO);
        return hipGetLastError();
    };
    if (prec == AK_FP64) {
        if (sw == 4) return go(source_lnkc_kernel<double, 4>, Tag<double>{});
        if (sw == 2) return go(source_lnkc_kernel<double, 2>, Tag<double>{});
        return go(source_lnkc_kernel<double, 1>, Tag<double>{});
    }
    if (sw == 4) return go(source_lnkc_kernel<float, 4>, Tag<float>{});
    if (sw == 2) return go(source_lnkc_kernel<float, 2>, Tag<float>{});
    return go(source_lnkc_kernel<float, 1>, Tag<float>{});
}

int check_source(const char *fn, const ak_mechanism *m, int prec, const void *T, const void *P,
                 const void *Y, int64_t ldY, int64_t n, const void *om, int64_t ldO)
{
    if (!m) return set_error(AK_EINVAL, "%s: null mechanism", fn);
    int rc = check_prec(fn, prec);
    if (!rc) rc = check_cells(fn, n);
    if (rc) return rc;
    if (n > 0 && (!T || !P || !Y || !om)) return set_error(AK_EINVAL, "%s: null pointer", fn);
    if (n > 0 && (ldY < n || ldO < n))
        return set_error(AK_EINVAL, "%s: ldY=%lld ldO=%lld < n_cells=%lld", fn, (long long)ldY,
                         (long long)ldO, (long long)n);
    if (m->pdep)
        return set_error(AK_EUNSUPPORTED, "%s: third-body and falloff reactions are not "
                                          "supported with a given ln K_c", fn);
    if (source_lnkc_lds(m->ns, 1) > (size_t)m->lds_max)
        return set_error(AK_EUNSUPPORTED, "%s: %d species exceed the LDS", fn, m->ns);
    return AK_OK;
}

}  // namespace
}  // namespace ak

using namespace ak;

extern "C" {

int ak_eval_lnkc(const ak_mechanism *m, ak_precision prec, const void *T, int64_t n, void *lnK,
                 int64_t ldK, void *stream)
{
    const char *fn = "ak_eval_lnkc";
    if (!m) return set_error(AK_EINVAL, "%s: null mechanism", fn);
    int rc = check_prec(fn, prec);
    if (!rc) rc = check_cells(fn, n);
    if (rc) return rc;
    if (n == 0) return AK_OK;
    if (!T || !lnK) return set_error(AK_EINVAL, "%s: null pointer", fn);
    if (ldK < n)
        return set_error(AK_EINVAL, "%s: ldK=%lld < n_cells=%lld", fn, (long long)ldK,
                         (long long)n);
    DeviceGuard g(m->device);
    if (!g.ok) return set_error(AK_EDEVICE, "%s: cannot select device %d", fn, m->device);
    const KcRxn *kr;
    const int32_t *order;
    if ((rc = kc_tables(m, &kr, &order))) return rc;
    const int64_t blocks = (n + 63) / 64;
    if (blocks > 0x7fffffff) return set_error(AK_E2BIG, "%s: n_cells too large", fn);
    hipStream_t st = (hipStream_t)stream;
    if (m->kc_pieces > 0) {
        // the composed layers: no LDS, no repeated work per chunk
        const int64_t b256 = (n + 255) / 256;
        const int ch = chunks_for((n + 63) / 64, m->nr, kTargetWaves, 8, m->nr);
        const int rpc = (m->nr + ch - 1) / ch;
        const dim3 grid((unsigned)b256, (unsigned)((m->nr + rpc - 1) / rpc));
        const double *fw = (const double *)(m->kc_dev + m->kc_fold_off);
#define AK_FOLD(IO, PM)                                                                      \
    hipLaunchKernelGGL((lnkc_fold_kernel<IO, PM>), grid, dim3(256), 0, st, fw, m->nr, rpc,     \
                       (const IO *)T, n, (IO *)lnK, ldK, m->view.err)
        const bool f64 = prec == AK_FP64;
        switch (m->kc_pieces) {
            case 1: if (f64) AK_FOLD(double, 1); else AK_FOLD(float, 1); break;
            case 2: if (f64) AK_FOLD(double, 2); else AK_FOLD(float, 2); break;
            case 3: if (f64) AK_FOLD(double, 3); else AK_FOLD(float, 3); break;
            default: if (f64) AK_FOLD(double, 4); else AK_FOLD(float, 4); break;
        }
#undef AK_FOLD
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_error(e, "ak_eval_lnkc: launch");
        return AK_OK;
    }
    if (lnkc_lds(m->ns) > (size_t)m->lds_max)
        return set_error(AK_EUNSUPPORTED, "%s: %d species exceed the LDS", fn, m->ns);
    const size_t lds = lnkc_lds(m->ns);
    // each chunk repeats the Gibbs layer (14 ns FMAs per cell): at most as
    // many chunks as make that the stoichiometric layer's work (~4 per row)
    const int ch = chunks_for(blocks, m->nr, kTargetWaves, 16,
                              std::max(1, (4 * m->nr) / (14 * m->ns)) * 2);
    const int rpc = (m->nr + ch - 1) / ch;
    const dim3 grid((unsigned)blocks, (unsigned)((m->nr + rpc - 1) / rpc));
    hipError_t e;
    auto go = [&](auto kern, auto tp) {
        using IO = typename decltype(tp)::type;
        hipError_t r = allow_dynamic_lds((const void *)kern);
        if (r != hipSuccess) return r;
        hipLaunchKernelGGL(kern, grid, dim3(64), lds, st, m->view, kr, rpc, (const IO *)T, n,
                           (IO *)lnK, ldK);
        return hipGetLastError();
    };
    const bool wide = m->kc_wide;
    if (prec == AK_FP64)
        e = wide ? go(lnkc_kernel<double, 8>, Tag<double>{})
                 : go(lnkc_kernel<double, 4>, Tag<double>{});
    else
        e = wide ? go(lnkc_kernel<float, 8>, Tag<float>{})
                 : go(lnkc_kernel<float, 4>, Tag<float>{});
    if (e != hipSuccess) return hip_error(e, "ak_eval_lnkc: launch");
    return AK_OK;
}

int ak_load_kcnet(const ak_kcnet_desc *d, int device, ak_kcnet **out)
{
    const char *fn = "ak_load_kcnet";
    if (!d || !out) return set_error(AK_EINVAL, "%s: null argument", fn);
    *out = nullptr;
    const int nl = d->n_layers, nh = d->n_hidden, nr = d->n_out;
    if (nl < 1 || nl > AK_KCNET_MAX_LAYERS || nh < 1 || nh > AK_KCNET_MAX_HIDDEN || nr < 1)
        return set_error(AK_EINVAL, "%s: bad sizes (layers %d, hidden %d, outputs %d)", fn, nl,
                         nh, nr);
    if (!d->weights || !d->biases || !d->y_mean || !d->y_std)
        return set_error(AK_EINVAL, "%s: null array", fn);
    if (!(d->x_std > 0.0) || !std::isfinite(d->x_std) || !std::isfinite(d->x_mean))
        return set_error(AK_EINVAL, "%s: bad input standardization", fn);
    const size_t n_w = (size_t)nh + (size_t)(nl - 1) * nh * nh + (size_t)nh * nr;
    const size_t n_b = (size_t)nh * nl + (size_t)nr;
    for (size_t q = 0; q < n_w; ++q)
        if (!std::isfinite(d->weights[q])) return set_error(AK_EINVAL, "%s: non-finite weight", fn);
    for (size_t q = 0; q < n_b; ++q)
        if (!std::isfinite(d->biases[q])) return set_error(AK_EINVAL, "%s: non-finite bias", fn);
    for (int j = 0; j < nr; ++j)
        if (!std::isfinite(d->y_mean[j]) || !std::isfinite(d->y_std[j]))
            return set_error(AK_EINVAL, "%s: non-finite output standardization", fn);
    const int nhp = nh <= 8 ? 8 : nh <= 16 ? 16 : nh <= 32 ? 32 : 64;
    // device layout (kernel order), zero-padded to width nhp
    const size_t ne = 2 * (size_t)nhp + (size_t)(nl - 1) * (nhp * nhp + nhp) +
                      (size_t)nr * nhp + nr;
    std::vector<double> w(ne, 0.0);
    const double *W = d->weights, *B = d->biases;
    for (int o = 0; o < nh; ++o) {
        w[o] = W[o];
        w[nhp + o] = B[o];
    }
    size_t p = 2 * (size_t)nhp, iw = nh, ib = nh;
    for (int l = 1; l < nl; ++l) {
        for (int o = 0; o < nh; ++o)
            for (int q = 0; q < nh; ++q) w[p + (size_t)o * nhp + q] = W[iw + (size_t)q * nh + o];
        for (int o = 0; o < nh; ++o) w[p + (size_t)nhp * nhp + o] = B[ib + o];
        p += (size_t)nhp * nhp + nhp;
        iw += (size_t)nh * nh;
        ib += nh;
    }
    for (int j = 0; j < nr; ++j) {
        for (int q = 0; q < nh; ++q)
            w[p + (size_t)j * nhp + q] = W[iw + (size_t)q * nr + j] * d->y_std[j];
        w[p + (size_t)nr * nhp + j] = B[ib + j] * d->y_std[j] + d->y_mean[j];
    }
    std::vector<float> wf(ne);
    for (size_t q = 0; q < ne; ++q) wf[q] = (float)w[q];
    ak_kcnet *net = new ak_kcnet;
    net->device = device;
    net->nl = nl;
    net->nh = nh;
    net->nhp = nhp;
    net->nr = nr;
    net->x_mean = d->x_mean;
    net->x_std = d->x_std;
    net->n_elems = ne;
    DeviceGuard g(device);
    if (!g.ok) {
        delete net;
        return set_error(AK_EDEVICE, "%s: cannot select device %d", fn, device);
    }
    const size_t bytes = ne * (sizeof(double) + sizeof(float));
    hipError_t e = hipMalloc(&net->dev, bytes);
    if (e == hipSuccess) e = hipMemcpy(net->dev, w.data(), ne * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(net->dev + ne * sizeof(double), wf.data(), ne * sizeof(float),
                      hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (net->dev) (void)hipFree(net->dev);
        delete net;
        return hip_error(e, "ak_load_kcnet: upload");
    }
    *out = net;
    return AK_OK;
}

int ak_free_kcnet(ak_kcnet *net)
{
    if (!net) return AK_OK;
    DeviceGuard g(net->device);
    (void)hipFree(net->dev);
    delete net;
    return AK_OK;
}

int ak_kcnet_n_out(const ak_kcnet *net) { return net ? net->nr : -1; }

int ak_eval_lnkc_net(const ak_kcnet *net, ak_precision prec, const void *T, int64_t n, void *lnK,
                     int64_t ldK, void *stream)
{
    const char *fn = "ak_eval_lnkc_net";
    if (!net) return set_error(AK_EINVAL, "%s: null network", fn);
    int rc = check_prec(fn, prec);
    if (!rc) rc = check_cells(fn, n);
    if (rc) return rc;
    if (n == 0) return AK_OK;
    if (!T || !lnK) return set_error(AK_EINVAL, "%s: null pointer", fn);
    if (ldK < n)
        return set_error(AK_EINVAL, "%s: ldK=%lld < n_cells=%lld", fn, (long long)ldK,
                         (long long)n);
    DeviceGuard g(net->device);
    if (!g.ok) return set_error(AK_EDEVICE, "%s: cannot select device %d", fn, net->device);
    hipError_t e = kcnet_launch(net, prec, T, n, lnK, ldK, (hipStream_t)stream);
    if (e != hipSuccess) return hip_error(e, "ak_eval_lnkc_net: launch");
    return AK_OK;
}

int ak_eval_source_lnkc(const ak_mechanism *m, ak_precision prec, const void *T, const void *P,
                        const void *Y, int64_t ldY, int64_t n, const void *lnK, int64_t ldK,
                        void *omega, int64_t ldO, void *stream)
{
    const char *fn = "ak_eval_source_lnkc";
    int rc = check_source(fn, m, prec, T, P, Y, ldY, n, omega, ldO);
    if (rc) return rc;
    if (n == 0) return AK_OK;
    if (!lnK) return set_error(AK_EINVAL, "%s: null lnK", fn);
    if (ldK < n)
        return set_error(AK_EINVAL, "%s: ldK=%lld < n_cells=%lld", fn, (long long)ldK,
                         (long long)n);
    DeviceGuard g(m->device);
    if (!g.ok) return set_error(AK_EDEVICE, "%s: cannot select device %d", fn, m->device);
    const KcRxn *kr;
    const int32_t *order;
    if ((rc = kc_tables(m, &kr, &order))) return rc;
    hipError_t e = source_lnkc_launch(m, order, prec, T, P, Y, ldY, n, lnK, ldK, omega, ldO,
                                      (hipStream_t)stream);
    if (e != hipSuccess) return hip_error(e, "ak_eval_source_lnkc: launch");
    return AK_OK;
}

int ak_eval_source_net(const ak_mechanism *m, const ak_kcnet *net, ak_precision prec,
                       const void *T, const void *P, const void *Y, int64_t ldY, int64_t n,
                       void *omega, int64_t ldO, void *stream)
{
    const char *fn = "ak_eval_source_net";
    int rc = check_source(fn, m, prec, T, P, Y, ldY, n, omega, ldO);
    if (rc) return rc;
    if (!net) return set_error(AK_EINVAL, "%s: null network", fn);
    if (net->nr != m->nr)
        return set_error(AK_EINVAL, "%s: network has %d outputs, mechanism %d reactions", fn,
                         net->nr, m->nr);
    if (net->device != m->device)
        return set_error(AK_EINVAL, "%s: network on device %d, mechanism on %d", fn,
                         net->device, m->device);
    if (n == 0) return AK_OK;
    DeviceGuard g(m->device);
    if (!g.ok) return set_error(AK_EDEVICE, "%s: cannot select device %d", fn, m->device);
    const KcRxn *kr;
    const int32_t *order;
    if ((rc = kc_tables(m, &kr, &order))) return rc;
    hipStream_t st = (hipStream_t)stream;
    const size_t bytes = (size_t)m->nr * (size_t)n * (prec == AK_FP64 ? 8 : 4);
    void *lnK = nullptr;
    hipError_t e = hipMallocAsync(&lnK, bytes, st);
    if (e != hipSuccess)
        return set_error(AK_ENOMEM, "%s: scratch of %zu bytes: %s", fn, bytes,
                         hipGetErrorString(e));
    e = kcnet_launch(net, prec, T, n, lnK, n, st);
    if (e == hipSuccess)
        e = source_lnkc_launch(m, order, prec, T, P, Y, ldY, n, lnK, n, omega, ldO, st);
    const hipError_t ef = hipFreeAsync(lnK, st);
    if (e != hipSuccess) return hip_error(e, "ak_eval_source_net: launch");
    if (ef != hipSuccess) return hip_error(ef, "ak_eval_source_net: freeing the scratch");
    return AK_OK;
}

int ak_integrate_euler_net(const ak_mechanism *m, const ak_kcnet *net, ak_precision prec,
                           void *T, const void *P, void *Y, int64_t ldY, int64_t n, double dt,
                           int n_steps, void *stream)
{
    const char *fn = "ak_integrate_euler_net";
    int rc = check_source(fn, m, prec, T, P, Y, ldY, n, Y, ldY);
    if (rc) return rc;
    if (!net) return set_error(AK_EINVAL, "%s: null network", fn);
    if (net->nr != m->nr)
        return set_error(AK_EINVAL, "%s: network has %d outputs, mechanism %d reactions", fn,
                         net->nr, m->nr);
    if (net->device != m->device)
        return set_error(AK_EINVAL, "%s: network on device %d, mechanism on %d", fn,
                         net->device, m->device);
    if (!(dt > 0.0) || !std::isfinite(dt))
        return set_error(AK_EINVAL, "%s: dt must be positive and finite", fn);
    if (n_steps < 0) return set_error(AK_EINVAL, "%s: n_steps < 0", fn);
    if (n == 0 || n_steps == 0) return AK_OK;
    DeviceGuard g(m->device);
    if (!g.ok) return set_error(AK_EDEVICE, "%s: cannot select device %d", fn, m->device);
    const KcRxn *kr;
    const int32_t *order;
    if ((rc = kc_tables(m, &kr, &order))) return rc;
    hipStream_t st = (hipStream_t)stream;
    const size_t es = prec == AK_FP64 ? 8 : 4;
    const size_t kbytes = ((size_t)m->nr * (size_t)n * es + 255) & ~(size_t)255;
    const size_t obytes = (size_t)m->ns * (size_t)n * es;
    void *scratch = nullptr;
    hipError_t e = hipMallocAsync(&scratch, kbytes + obytes, st);
    if (e != hipSuccess)
        return set_error(AK_ENOMEM, "%s: scratch of %zu bytes: %s", fn, kbytes + obytes,
                         hipGetErrorString(e));
    void *lnK = scratch, *om = (unsigned char *)scratch + kbytes;
    for (int s = 0; s < n_steps && e == hipSuccess; ++s) {
        e = kcnet_launch(net, prec, T, n, lnK, n, st);
        if (e == hipSuccess)
            e = source_lnkc_launch(m, order, prec, T, P, Y, ldY, n, lnK, n, om, n, st);
        if (e == hipSuccess)
            e = euler_update_launch(m->view, prec == AK_FP64, T, P, Y, ldY, n, om, n, dt, st);
    }
    const hipError_t ef = hipFreeAsync(scratch, st);
    if (e != hipSuccess) return hip_error(e, "ak_integrate_euler_net: step");
    if (ef != hipSuccess) return hip_error(ef, "ak_integrate_euler_net: freeing the scratch");
    return AK_OK;
}

}  // extern "C"
