// Derivatives of the source term on gfx950: the dense state Jacobian and the
// vector-Jacobian product (VJP), both in double precision internally.
//
// State x = (Y_1..Y_NS, T) at fixed P; outputs omega_k (Eq. 2) and the
// constant-pressure temperature source omega_T = -sum_k h_k omega_k /
// sum_k C_k cp_k.  With a_k = C_k exp(Gt_k), v_k = exp(-Gt_k), w_k = 1/v_k
// (Gt the Gibbs-layer output, Eqs. 10-11) and E_j = k_f,j prod_reac v:
//     q_f = E prod_reac a,   q_r = rev E prod_prod a        (Eqs. 3-4, 7)
//     dq_f/dC_m = E w_m sum_{slots i of m} prod_{l != i} a_l    (same for q_r)
//     dC_l/dY_m = [Y_m >= 0] (delta_lm rho/W_m - C_l/(sigma W_m)),  dC_l/dT = -C_l/T
// so that, using the homogeneity sum_l C_l dq_f/dC_l = n_f q_f,
//     d omega_k/dY_m = [Y_m >= 0] (rho G_km - u_k/sigma) / W_m,
//     G_km = sum_j nu_kj dq_j/dC_m,  u_k = sum_j nu_kj (n_f q_f - n_r q_r)_j,
//     d omega_k/dT = sum_j nu_kj (dq_j/dT|_C - (n_f q_f - n_r q_r)_j / T),
//     d ln k_f/dT = (beta + E/RT)/T,  d ln K_c/dT = (dH/RT - dn)/T.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ak_device.h"
#include "ak_internal.h"
#include "ak_math.h"

namespace ak {


__device__ __forceinline__ void lds_addd(double *p, double x)
{
    __hip_atomic_fetch_add(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// x moved across lanes by one DPP pattern (both halves of the double);
// lanes with no source lane take 0
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x)
{
    int w[2];
    __builtin_memcpy(w, &x, 8);
    w[0] = __builtin_amdgcn_update_dpp(0, w[0], CTRL, 0xf, 0xf, false);
    w[1] = __builtin_amdgcn_update_dpp(0, w[1], CTRL, 0xf, 0xf, false);
    double r;
    __builtin_memcpy(&r, w, 8);
    return r;
}

// Sum over the 64 lanes of a wave (all lanes active), the same value in
// every lane and in every wave for the same inputs: scans within rows of 16
// lanes (row_shr 1, 2, 4, 8), then across rows (row_bcast 15, 31), which
// leaves the total in lane 63.  DPP moves stay in the vector registers, where
// a shuffle goes through the LDS crossbar.
__device__ __forceinline__ double wave_sum(double x)
{
    x += dpp_move<0x111>(x);
    x += dpp_move<0x112>(x);
    x += dpp_move<0x114>(x);
    x += dpp_move<0x118>(x);
    x += dpp_move<0x142>(x);
    x += dpp_move<0x143>(x);
    int w[2];
    __builtin_memcpy(w, &x, 8);
    w[0] = __builtin_amdgcn_readlane(w[0], 63);
    w[1] = __builtin_amdgcn_readlane(w[1], 63);
    double r;
    __builtin_memcpy(&r, w, 8);
    return r;
}

struct Thermo1 {
    double h, cp, dcp;   // h/RT, cp/R, d(cp/R)/dT
};

__device__ __forceinline__ Thermo1 nasa(const ThermoRec &t, double T, double T_mid)
{
    const double *a = (T >= T_mid) ? t.hi : t.lo;
    const double T2 = T * T, T3 = T2 * T, T4 = T3 * T;
    Thermo1 r;
    r.h = a[0] + a[1] * T / 2 + a[2] * T2 / 3 + a[3] * T3 / 4 + a[4] * T4 / 5 + a[5] / T;
    r.cp = a[0] + a[1] * T + a[2] * T2 + a[3] * T3 + a[4] * T4;
    r.dcp = a[1] + 2 * a[2] * T + 3 * a[3] * T2 + 4 * a[4] * T3;
    return r;
}

__device__ __forceinline__ double gibbs2(const SpeciesRec &s, double lnT, double T, double T2,
                                         double T3, double T4, double invT)
{
    const double *c = (T >= s.T_mid) ? s.hi : s.lo;
    return c[0] * lnT + c[1] * T + c[2] * T2 + c[3] * T3 + c[4] * T4 + c[5] * invT + c[6];
}

// ---------------------------------------------------------------------------
// Jacobian: one workgroup of kJacWaves waves per cell, thread = reaction.
//
// LDS per cell (doubles): J[(ns+1)^2] then per species C, a, v, w, h, cp,
// dcp, omega, u, y and s = [Y >= 0]/W, then 4 x 64 partial sums.  J holds
// G_km (and d omega_k/dT in the last column) during the reaction sweep and
// the finished Jacobian afterwards.  The per-cell LDS (28 KB at 53 species)
// lets several cells share a CU, and all of a workgroup's lanes share the
// sweep, the assembly and the store.  The cell's mass fractions are read
// from HBM once per workgroup (they lie NS cache lines apart).
constexpr int kJacWaves = 4;
constexpr int kJacThreads = 64 * kJacWaves;
constexpr int kJacSpeciesVecs = 11;

template <typename IO>
__global__ __launch_bounds__(kJacThreads) void jacobian_kernel(MechView m,
                                                               const IO *__restrict__ Tin,
                                                               const IO *__restrict__ Pin,
                                                               const IO *__restrict__ Y,
                                                               int64_t ldY, int64_t n,
                                                               IO *__restrict__ Jout,
                                                               int64_t ldJ)
{
    extern __shared__ __attribute__((aligned(16))) double jl[];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int ns = m.ns, nv = ns + 1;
    double *Jw = jl;
    double *sC = Jw + ((nv * nv + 1) & ~1), *sa = sC + ns, *sv = sa + ns, *sw = sv + ns,
           *sh = sw + ns, *scp = sh + ns, *sdcp = scp + ns, *som = sdcp + ns, *su = som + ns,
           *sy = su + ns, *ss = sy + ns;
    double *part = ss + ns;                       // [4][64]
    const int64_t cell = blockIdx.x;

    // the cell's state: Y once into LDS, then the mixture sum in every wave
    // (same order, lane = species)
    for (int k = tid; k < ns; k += kJacThreads) sy[k] = (double)Y[k * ldY + cell];
    for (int i = 2 * tid; i < nv * nv; i += 2 * kJacThreads) {
        if (i + 1 < nv * nv) *(double2 *)&Jw[i] = make_double2(0.0, 0.0);
        else Jw[i] = 0.0;
    }
    __syncthreads();
    double T = (double)Tin[cell];
    double P = (double)Pin[cell];
    bool bad = !(T > 0.0) || !(P > 0.0) || !__builtin_isfinite(T) || !__builtin_isfinite(P);
    double ysum = 0.0;
    bool ybad = false;
    for (int k = lane; k < ns; k += 64) {
        const double y = sy[k];
        ybad |= !__builtin_isfinite(y);
        ysum += __builtin_fmax(y, 0.0) * m.sp[k].inv_W;
    }
    double sigma = wave_sum(ysum);
    bad |= __any(ybad) || !(sigma > 0.0) || !__builtin_isfinite(sigma);
    if (bad) {
        T = 1000.0;
        P = 1.0e5;
        sigma = 1.0;
    }
    const double lnT = log(T), invT = 1.0 / T, T2 = T * T, T3 = T2 * T, T4 = T3 * T;
    const double rho = P / (kRu * T * sigma);
    for (int k = tid; k < ns; k += kJacThreads) {
        const SpeciesRec &s = m.sp[k];
        const double y = bad ? 0.0 : __builtin_fmax(sy[k], 0.0);
        const double C = rho * y * s.inv_W;
        const double g2 = gibbs2(s, lnT, T, T2, T3, T4, invT);
        double w, v;
        exp2_pair<12>(g2, w, v);
        const Thermo1 th = nasa(m.th[k], T, s.T_mid);
        sC[k] = C;
        sa[k] = C * w;
        sv[k] = v;
        sw[k] = w;
        sh[k] = th.h;
        scp[k] = th.cp;
        sdcp[k] = th.dcp;
        som[k] = 0.0;
        su[k] = 0.0;
        ss[k] = (sy[k] >= 0.0 ? 1.0 : 0.0) * s.inv_W;
    }
    __syncthreads();

    const double log2T = lnT * kLog2e;
    // reactions are sorted by molecule count, so walking them from the end
    // gives the first pass the expensive shapes and leaves the cheap ones for
    // the partial second pass (a wave's predicated loops run to the largest
    // molecule count among its lanes)
    for (int jr = tid; jr < m.nr; jr += kJacThreads) {
        const int j = m.nr - 1 - jr;
        const RxnRec R = m.rx[j];
        const RxnAux X = m.aux[j];
        const int nf = X.nf, nr = X.nr, nm = nf + nr;
        const double kf =
            scale_exp2(1.0, __builtin_fma(R.beta, log2T, __builtin_fma(R.negEoR2, invT, R.log2A)));
        double a[8], Ar = 1.0, Ap = 1.0, E = kf, dH = 0.0;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if (i < nm) {
                const int s = X.sp[i];
                a[i] = sa[s];
                if (i < nf) {
                    Ar *= a[i];
                    E *= sv[s];
                    dH -= sh[s];
                } else {
                    Ap *= a[i];
                    dH += sh[s];
                }
            }
        }
        const double rev = X.rev;
        const double qf = E * Ar, qr = rev * E * Ap;
        const double dlnkf = (R.beta + X.EoR * invT) * invT;
        const double dn = (double)(nr - nf);
        const double dqT = qf * (dlnkf - nf * invT) - qr * (dlnkf - (dH - dn) * invT - nr * invT);
        const double wu = nf * qf - nr * qr;
        const double qn = qf - qr;
        // d q_net / dC at each molecule slot: the product of the other
        // molecules of the same side, as prefix times suffix products
        double pre[8], suf[8];
        double p = 1.0;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if (i == nf) p = 1.0;
            pre[i] = p;
            if (i < nm) p *= a[i];
        }
        p = 1.0;
#pragma unroll
        for (int i = 7; i >= 0; --i) {
            if (i == nf - 1) p = 1.0;
            suf[i] = p;
            if (i < nm) p *= a[i];
        }
        double dq[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if (i < nm) {
                const double base = E * sw[X.sp[i]] * (pre[i] * suf[i]);
                dq[i] = i < nf ? base : -rev * base;
            }
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            if (r < nm) {
                const int k = X.sp[r];
                const double sg = r < nf ? -1.0 : 1.0;
                lds_addd(&som[k], sg * qn);
                lds_addd(&su[k], sg * wu);
                lds_addd(&Jw[k * nv + ns], sg * dqT);
#pragma unroll
                for (int c = 0; c < 8; ++c)
                    if (c < nm) lds_addd(&Jw[k * nv + X.sp[c]], sg * dq[c]);
            }
        }
    }
    __syncthreads();

    // assembly of the composition columns (the temperature column already
    // holds the full d omega_k/dT: dq/dT above includes -(n_f q_f - n_r q_r)/T)
    const double inv_sigma = 1.0 / sigma;
    const int wave = tid >> 6;
    for (int c0 = 0; c0 < ns; c0 += 64) {          // lane = column, rows k split by wave
        const int c = c0 + lane;
        if (c < ns) {
            const double ssc = ss[c];
#pragma unroll 4
            for (int k = wave; k < ns; k += kJacWaves) {
                double *jp = &Jw[k * nv + c];
                *jp = ssc * (rho * *jp - su[k] * inv_sigma);
            }
        }
    }
    // temperature-row sums: every wave, same order
    double num = 0.0, den = 0.0, omcp = 0.0, cdcp = 0.0;
    for (int k = lane; k < ns; k += 64) {
        num += kRu * T * sh[k] * som[k];
        den += sC[k] * kRu * scp[k];
        omcp += kRu * scp[k] * som[k];
        cdcp += sC[k] * kRu * sdcp[k];
    }
    num = wave_sum(num);
    den = wave_sum(den);
    omcp = wave_sum(omcp);
    cdcp = wave_sum(cdcp);
    __syncthreads();
    // temperature row: column c of d omega_T / dx; sum_k h_k J[k][c] in four
    // interleaved parts (thread = column c0 + lane, part = wave)
    for (int c0 = 0; c0 < nv; c0 += 64) {
        const int c = c0 + lane;
        double dn = 0.0;
        if (c < nv)
            for (int k = wave; k < ns; k += kJacWaves) dn += sh[k] * Jw[k * nv + c];
        part[wave * 64 + lane] = dn;
        __syncthreads();
        if (wave == 0 && c < nv) {
            double dnum = 0.0;
            for (int w = 0; w < kJacWaves; ++w) dnum += part[w * 64 + lane];
            dnum *= kRu * T;
            double dden;
            if (c < ns) {
                dden = ss[c] * (kRu * scp[c] * rho - den * inv_sigma);
            } else {
                dnum += omcp;
                dden = -den * invT + cdcp;
            }
            Jw[ns * nv + c] = -(dnum * den - num * dden) / (den * den);
        }
        __syncthreads();
    }
    // store, 16 bytes at a time where the row of this cell is 16-byte aligned
    const IO nan = __builtin_nan("");
    IO *o = Jout + cell * ldJ;
    const int nn = nv * nv;
    bool wide = false;
    if constexpr (sizeof(IO) == 8) wide = ((uintptr_t)o & 15) == 0;
    if (wide) {
        for (int i = 2 * tid; i < nn; i += 2 * kJacThreads) {
            if (i + 1 < nn) {
                const double2 x = *(const double2 *)&Jw[i];
                *(double2 *)(o + i) = bad ? make_double2(nan, nan) : x;
            } else {
                o[i] = bad ? nan : (IO)Jw[i];
            }
        }
    } else {
        for (int i = tid; i < nn; i += kJacThreads) o[i] = bad ? nan : (IO)Jw[i];
    }
    if (tid == 0 && bad) atomicAdd(m.err, 1ull);
}

// ---------------------------------------------------------------------------
// VJP: lane = cell, tile of `tile` cells shared by the workgroup's waves.
// LDS entry per (species, cell), 40 B: a, v, omega_bar, h/RT, a_bar.
// Reactions are walked in the forward kernel's (shape, reversibility) runs so
// that each molecule loop is unrolled for its shape.
constexpr int kVjpEntry = 40;
constexpr int kVjpWaves = 16;

struct VjpCell {
    double log2T, invT;
};

// One reaction's contribution: q_bar = sum_k nu_kj omega_bar_k; a_bar of each
// molecule slot += q_bar dq/da_slot (LDS atomics); s += q_bar (n_f q_f -
// n_r q_r); T_bar += q_bar dq/dT.
template <int NF, int NR>
__device__ __forceinline__ void vjp_reaction(const RxnRec &R, double rev, unsigned char *vl,
                                             uint32_t lane_off, uint32_t sstride,
                                             const VjpCell c, double &s_acc, double &tbar)
{
    constexpr int NM = NF + NR;
    const double t = __builtin_fma(R.beta, c.log2T, __builtin_fma(R.negEoR2, c.invT, R.log2A));
    double a[NM];
    double *e[NM];
    double Vr = 1.0, dH = 0.0, qbar = 0.0;
#pragma unroll
    for (int i = 0; i < NM; ++i) {
        e[i] = (double *)(vl + lane_off + (uint32_t)R.sp[i] * sstride);
        a[i] = e[i][0];
        if (i < NF) {
            Vr *= e[i][1];
            dH -= e[i][3];
            qbar -= e[i][2];
        } else {
            dH += e[i][3];
            qbar += e[i][2];
        }
    }
    double Ar = 1.0, Ap = 1.0;
#pragma unroll
    for (int i = 0; i < NM; ++i) {
        if (i < NF) Ar *= a[i]; else Ap *= a[i];
    }
    const double Ek = scale_exp2(Vr, t);         // k_f prod_reac v
    const double qf = Ek * Ar, qr = rev * Ek * Ap;
    const double EoR = -R.negEoR2 * 0.69314718055994530942;   // E/R
    const double dlnkf = (R.beta + EoR * c.invT) * c.invT;
    const double dqT = qf * (dlnkf - NF * c.invT) -
                       qr * (dlnkf - (dH - (double)(NR - NF)) * c.invT - NR * c.invT);
    s_acc += qbar * (NF * qf - NR * qr);
    tbar += qbar * dqT;
#pragma unroll
    for (int i = 0; i < NM; ++i) {
        double loo = 1.0;
#pragma unroll
        for (int l = 0; l < NM; ++l)
            if (l != i && ((l < NF) == (i < NF))) loo *= a[l];
        const double d = i < NF ? Ek * loo : -rev * Ek * loo;   // d q / d a_slot
        lds_addd(e[i] + 4, qbar * d);
    }
}

template <int NF, int NR>
__device__ __forceinline__ void vjp_run(const MechView &m, const ShapeRun run, int wave,
                                        unsigned char *vl, uint32_t lane_off, uint32_t sstride,
                                        const VjpCell c, double &s_acc, double &tbar)
{
    const int end = run.start + run.count;
    for (int j = run.start + wave; j < end; j += kVjpWaves)
        vjp_reaction<NF, NR>(m.rx[j], run.rev, vl, lane_off, sstride, c, s_acc, tbar);
}

// KV: species per wave held in registers (ns <= KV * kVjpWaves)
template <typename IO, int KV>
__global__ __launch_bounds__(64 * kVjpWaves) void vjp_kernel(MechView m, int tile,
                                                             const IO *__restrict__ Tin,
                                                             const IO *__restrict__ Pin,
                                                             const IO *__restrict__ Y,
                                                             int64_t ldY, int64_t n,
                                                             const IO *__restrict__ G,
                                                             int64_t ldG, IO *__restrict__ GY,
                                                             int64_t ldGY, IO *__restrict__ GT)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char vl[];
    __shared__ double partial[kVjpWaves][2][64];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // lanes past the tile own no LDS column; every wave keeps lanes 0..tile-1
    if (lane >= tile) return;
    const int64_t cell = (int64_t)blockIdx.x * tile + lane;
    const bool valid = cell < n;
    const uint32_t sstride = (uint32_t)tile * kVjpEntry;
    const uint32_t lane_off = (uint32_t)lane * kVjpEntry;
    auto E = [&](int k) { return (double *)(vl + (uint32_t)k * sstride + lane_off); };

    // all of this wave's inputs requested at once, with no branch or select
    // after the loads (which would make the compiler wait for each in turn):
    // lanes past the last cell read cell 0 and slots past the last species
    // read species 0, and neither result is stored
    const int64_t c0 = valid ? cell : 0;
    double T = (double)Tin[c0];
    double P = (double)Pin[c0];
    IO yv[KV], gv[KV];
#pragma unroll
    for (int i = 0; i < KV; ++i) {
        const int k = wave + i * kVjpWaves;
        const int64_t kk = k < m.ns ? k : 0;
        yv[i] = Y[kk * ldY + c0];
        gv[i] = G[kk * ldG + c0];
    }
    // this wave's species: y_k^+ / W_k into the a-slot, partial mixture sums
    // (NaN for a non-finite input) meeting in LDS
    double psum = 0.0;
#pragma unroll
    for (int i = 0; i < KV; ++i) {
        const int k = wave + i * kVjpWaves;
        if (k < m.ns) {
            const double y = (double)yv[i];
            const double yw = __builtin_fmax(y, 0.0) * m.sp[k].inv_W;
            psum += __builtin_isfinite(y) ? yw : __builtin_nan("");
            E(k)[0] = yw;
        }
    }
    partial[wave][0][lane] = psum;
    __syncthreads();
    double sigma = 0.0;
    for (int w = 0; w < kVjpWaves; ++w) sigma += partial[w][0][lane];
    bool bad = !(T > 0.0) || !(P > 0.0) || !__builtin_isfinite(T) || !__builtin_isfinite(P) ||
               !(sigma > 0.0) || !__builtin_isfinite(sigma);
    if (bad) {
        T = 1000.0;
        P = 1.0e5;
        sigma = 1.0;
    }
    const double lnT = log(T), invT = 1.0 / T, T2 = T * T, T3 = T2 * T, T4 = T3 * T;
    const double rho = P / (kRu * T * sigma);
#pragma unroll
    for (int i = 0; i < KV; ++i) {
        const int k = wave + i * kVjpWaves;
        if (k < m.ns) {
            const SpeciesRec &s = m.sp[k];
            const double g2 = gibbs2(s, lnT, T, T2, T3, T4, invT);
            const Thermo1 th = nasa(m.th[k], T, s.T_mid);
            double *e = E(k);
            const double yw = bad ? 0.0 : e[0];
            double w, v;
            exp2_pair<12>(g2, w, v);
            e[0] = rho * yw * w;
            e[1] = v;
            e[2] = (double)gv[i];
            e[3] = th.h;
            e[4] = 0.0;
        }
    }
    __syncthreads();      // also: every wave has read `partial` above

    // reverse sweep over reactions (this wave: every kVjpWaves-th reaction
    // of each run)
    VjpCell c;
    c.log2T = lnT * kLog2e;
    c.invT = invT;
    double s_acc = 0.0, tbar = 0.0;
    for (int r = 0; r < m.nruns; ++r) {
        const ShapeRun run = m.runs[r];
        const int sh = (run.nf - 1) * 4 + (run.nr - 1);
#define AK_VCASE(a, b)                                                                         \
    case (a - 1) * 4 + (b - 1):                                                                \
        vjp_run<a, b>(m, run, wave, vl, lane_off, sstride, c, s_acc, tbar);                     \
        break;
        switch (sh) {
            AK_VCASE(1, 1) AK_VCASE(1, 2) AK_VCASE(1, 3) AK_VCASE(1, 4)
            AK_VCASE(2, 1) AK_VCASE(2, 2) AK_VCASE(2, 3) AK_VCASE(2, 4)
            AK_VCASE(3, 1) AK_VCASE(3, 2) AK_VCASE(3, 3) AK_VCASE(3, 4)
            AK_VCASE(4, 1) AK_VCASE(4, 2) AK_VCASE(4, 3) AK_VCASE(4, 4)
            default: break;
        }
#undef AK_VCASE
    }
    partial[wave][0][lane] = s_acc;
    partial[wave][1][lane] = tbar;
    __syncthreads();
    double s_tot = 0.0, t_tot = 0.0;   // s = sum_j q_bar_j (n_f q_f - n_r q_r)_j
    for (int w = 0; w < kVjpWaves; ++w) {
        s_tot += partial[w][0][lane];
        t_tot += partial[w][1][lane];
    }
    const IO nan = __builtin_nan("");
    // Y_bar_m = [Y_m >= 0] (rho w_m a_bar_m - s/sigma) / W_m; T_bar = sum q_bar dq/dT
#pragma unroll
    for (int i = 0; i < KV; ++i) {
        const int k = wave + i * kVjpWaves;
        if (k < m.ns && valid) {
            const double *e = E(k);
            const double ycl = (double)yv[i] >= 0.0 ? 1.0 : 0.0;
            const double gy = ycl * (rho * e[4] / e[1] - s_tot / sigma) * m.sp[k].inv_W;
            GY[k * ldGY + cell] = bad ? nan : (IO)gy;
        }
    }
    if (wave == 0 && valid) {
        GT[cell] = bad ? nan : (IO)t_tot;
        if (bad) atomicAdd(m.err, 1ull);
    }
}

// ---------------------------------------------------------------------------
// launchers

static size_t jacobian_lds_per_cell(int ns)
{
    const size_t nv2 = ((size_t)(ns + 1) * (ns + 1) + 1) & ~(size_t)1;
    return (nv2 + kJacSpeciesVecs * (size_t)ns + 4 * 64) * sizeof(double);
}

// LDS of one cell's workgroup
size_t jacobian_lds_bytes(int ns) { return jacobian_lds_per_cell(ns); }

template <typename IO>
static hipError_t jacobian_launch_t(const MechView &m, const void *T, const void *P,
                                    const void *Y, int64_t ldY, int64_t n, void *J,
                                    int64_t ldJ, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    if (n > 0x7fffffff) return hipErrorInvalidValue;
    const size_t lds = jacobian_lds_per_cell(m.ns);
    auto fn = jacobian_kernel<IO>;
    hipError_t e = allow_dynamic_lds((const void *)fn);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3((unsigned)n), dim3(kJacThreads), lds, st, m, (const IO *)T,
                       (const IO *)P, (const IO *)Y, ldY, n, (IO *)J, ldJ);
    return hipGetLastError();
}

hipError_t jacobian_launch(const MechView &m, int lds_max, bool f64, const void *T,
                           const void *P, const void *Y, int64_t ldY, int64_t n, void *J,
                           int64_t ldJ, hipStream_t st)
{
    (void)lds_max;   // the caller checked jacobian_lds_bytes against it
    if (f64) return jacobian_launch_t<double>(m, T, P, Y, ldY, n, J, ldJ, st);
    return jacobian_launch_t<float>(m, T, P, Y, ldY, n, J, ldJ, st);
}

int vjp_tile(int ns, int lds_max)
{
    const int static_lds = kVjpWaves * 2 * 64 * (int)sizeof(double);
    int t = (lds_max - static_lds) / (ns * kVjpEntry);
    return t > 64 ? 64 : t;
}

template <typename IO, int KV>
static hipError_t vjp_launch_t(const MechView &m, int tile, const void *T, const void *P,
                               const void *Y, int64_t ldY, int64_t n, const void *G, int64_t ldG,
                               void *GY, int64_t ldGY, void *GT, int64_t blocks, hipStream_t st)
{
    const size_t lds = (size_t)m.ns * tile * kVjpEntry;
    auto fn = vjp_kernel<IO, KV>;
    hipError_t e = allow_dynamic_lds((const void *)fn);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(64 * kVjpWaves), lds, st, m, tile,
                       (const IO *)T, (const IO *)P, (const IO *)Y, ldY, n, (const IO *)G, ldG,
                       (IO *)GY, ldGY, (IO *)GT);
    return hipGetLastError();
}

hipError_t vjp_launch(const MechView &m, int tile, bool f64, const void *T, const void *P,
                      const void *Y, int64_t ldY, int64_t n, const void *G, int64_t ldG,
                      void *GY, int64_t ldGY, void *GT, hipStream_t st)
{
    const int64_t blocks = (n + tile - 1) / tile;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    const int per = (m.ns + kVjpWaves - 1) / kVjpWaves;   // ns <= 256: at most 16
    if (f64) {
        if (per <= 4) return vjp_launch_t<double, 4>(m, tile, T, P, Y, ldY, n, G, ldG, GY, ldGY, GT, blocks, st);
        if (per <= 8) return vjp_launch_t<double, 8>(m, tile, T, P, Y, ldY, n, G, ldG, GY, ldGY, GT, blocks, st);
        return vjp_launch_t<double, 16>(m, tile, T, P, Y, ldY, n, G, ldG, GY, ldGY, GT, blocks, st);
    }
    if (per <= 4) return vjp_launch_t<float, 4>(m, tile, T, P, Y, ldY, n, G, ldG, GY, ldGY, GT, blocks, st);
    if (per <= 8) return vjp_launch_t<float, 8>(m, tile, T, P, Y, ldY, n, G, ldG, GY, ldGY, GT, blocks, st);
    return vjp_launch_t<float, 16>(m, tile, T, P, Y, ldY, n, G, ldG, GY, ldGY, GT, blocks, st);
}

}  // namespace ak
