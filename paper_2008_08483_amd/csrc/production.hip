// The stoichiometric contraction omega = nu r on the matrix cores in split
// bfloat16 (the reduced-precision environments named as future work in
// Sec. 4; the contraction itself is Eq. 2 with the rates of progress given).
//
// nu = nu'' - nu' holds small integers, exact in bfloat16.  Each FP32 rate
// is cut into three bfloat16 parts h + m + l == r exactly (8 + 8 + 8
// significant bits, truncation leaves no remainder for normal numbers), so
// every product nu_kj * part is exact and the only rounding is the FP32
// accumulation inside v_mfma_f32_16x16x32_bf16.  The result carries the
// error of an FP32 dot product over 3 N_R terms.
//
// Layout: one wave owns 16 NCB cells, one workgroup 64 NCB (four waves), and a group
// of up to 16 blocks of 16 species (grid y; one group up to 256 species, so
// the rates are read once).  Per chunk of 32 reactions a
// lane loads the 8 rates of its (reaction octet, cell) pair straight from
// HBM (each load instruction covers 4 rows x 64 contiguous bytes), splits
// them, and issues three MFMAs per species block against the constant
// nu operand, which the host lays out in lane order once per mechanism; the
// next chunk's loads are in flight meanwhile.
// The work is HBM-bound: (N_R + N_S) x 4 bytes per cell against
// 2 N_S N_R x 3 dense MFMA flops.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "annkin.h"
#include "ak_device.h"
#include "ak_internal.h"

namespace ak {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

#ifndef AK_PROD_GROUP
#define AK_PROD_GROUP 16
#endif
constexpr int kGroup = AK_PROD_GROUP;   // species blocks of 16 per workgroup
constexpr int kChunk = 32;       // reactions per MFMA step
std::mutex g_prod_mu;

// x == h + m + l with each part's FP32 pattern in the high 16 bits (returned
// as the bfloat16 bit pattern)
__device__ __forceinline__ void split3(float x, unsigned &h, unsigned &m, unsigned &l)
{
    const unsigned hb = __float_as_uint(x) & 0xffff0000u;
    const float r1 = x - __uint_as_float(hb);
    const unsigned mb = __float_as_uint(r1) & 0xffff0000u;
    const float r2 = r1 - __uint_as_float(mb);
    h = hb >> 16;
    m = mb >> 16;
    l = __float_as_uint(r2) >> 16;
}

__device__ __forceinline__ bf16x8 pack8(const unsigned (&v)[8])
{
    u32x4 p;
    p[0] = v[0] | (v[1] << 16);
    p[1] = v[2] | (v[3] << 16);
    p[2] = v[4] | (v[5] << 16);
    p[3] = v[6] | (v[7] << 16);
    return __builtin_bit_cast(bf16x8, p);
}

// A: [kchunks][mbp][64 lanes] x 8 bfloat16 of nu, lane l holding species
// 16 b + l % 16 and reactions 32 c + 8 (l / 16) + 0..7 (the MFMA's A
// operand layout; the B operand uses the same reaction index per lane and
// slot, so the k order inside a chunk is immaterial).  Each wave owns NCB
// blocks of 16 cells, so a workgroup reads 256 NCB contiguous bytes of each
// rate row and every nu operand load feeds 3 NCB MFMAs.
template <int MB, int NCB>
__global__ __launch_bounds__(256) void production_kernel(const u32x4 *__restrict__ A,
                                                         int kchunks, int mbp,
                                                         const float *__restrict__ r,
                                                         int64_t ldr, int nr, int64_t n,
                                                         float *__restrict__ w, int64_t ldw,
                                                         int ns)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, kq = lane >> 4;
    const int64_t cell0 = (int64_t)blockIdx.x * (64 * NCB) + wave * (16 * NCB) + col;
    int64_t cc[NCB];
#pragma unroll
    for (int j = 0; j < NCB; ++j) cc[j] = cell0 + 16 * j < n ? cell0 + 16 * j : n - 1;
    const int g0 = blockIdx.y * MB;
    f32x4 acc[MB][NCB];
#pragma unroll
    for (int b = 0; b < MB; ++b)
#pragma unroll
        for (int j = 0; j < NCB; ++j) acc[b][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    // the next chunk's rates are loaded while this chunk's MFMAs run (rows
    // past the last reaction read the last row and are zeroed)
    float x[NCB][8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int k = kq * 8 + i;
        const float *row = r + (int64_t)(k < nr ? k : nr - 1) * ldr;
#pragma unroll
        for (int j = 0; j < NCB; ++j) x[j][i] = k < nr ? row[cc[j]] : 0.f;
    }
    for (int c = 0; c < kchunks; ++c) {
        float xn[NCB][8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int k = (c + 1) * kChunk + kq * 8 + i;
            const float *row = r + (int64_t)(k < nr ? k : nr - 1) * ldr;
#pragma unroll
            for (int j = 0; j < NCB; ++j) {
                xn[j][i] = row[cc[j]];
                if (k >= nr) xn[j][i] = 0.f;
            }
        }
        bf16x8 bh[NCB], bm[NCB], bl[NCB];
#pragma unroll
        for (int j = 0; j < NCB; ++j) {
            unsigned h[8], m[8], l[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) split3(x[j][i], h[i], m[i], l[i]);
            bh[j] = pack8(h);
            bm[j] = pack8(m);
            bl[j] = pack8(l);
        }
        const u32x4 *Ac = A + ((int64_t)c * mbp + g0) * 64 + lane;
#pragma unroll
        for (int b = 0; b < MB; ++b) {
            const bf16x8 a = __builtin_bit_cast(bf16x8, Ac[b * 64]);
#pragma unroll
            for (int j = 0; j < NCB; ++j) {
                acc[b][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bl[j], acc[b][j], 0, 0, 0);
                acc[b][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bm[j], acc[b][j], 0, 0, 0);
                acc[b][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bh[j], acc[b][j], 0, 0, 0);
            }
        }
#pragma unroll
        for (int j = 0; j < NCB; ++j)
#pragma unroll
            for (int i = 0; i < 8; ++i) x[j][i] = xn[j][i];
    }
    // output element (4 (l / 16) + v, l % 16) of each 16 x 16 block
#pragma unroll
    for (int j = 0; j < NCB; ++j) {
        const int64_t cell = cell0 + 16 * j;
        if (cell >= n) continue;
#pragma unroll
        for (int b = 0; b < MB; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int s = (g0 + b) * 16 + kq * 4 + v;
                if (s < ns) w[(int64_t)s * ldw + cell] = acc[b][j][v];
            }
    }
}

// The same contraction with nu staged in LDS: per stage of sc chunks the
// workgroup copies its nu blocks (sc x MB KB) once and its four waves read
// them from LDS, instead of each wave reading its MB KB per chunk from L2.
// Used for more than four species blocks, where those re-reads bound the
// register form (150/600 x 2^19: 1.06 -> 0.78 ms); at four blocks or fewer
// the register form is faster.
template <int MB, int NCB, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void production_lds_kernel(const u32x4 *__restrict__ A,
                                                             int kchunks, int mbp, int sc,
                                                             const float *__restrict__ r,
                                                             int64_t ldr, int nr, int64_t n,
                                                             float *__restrict__ w,
                                                             int64_t ldw, int ns)
{
    extern __shared__ u32x4 As[];   // sc chunks x MB blocks x 64 lanes
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, kq = lane >> 4;
    const int64_t cell0 = (int64_t)blockIdx.x * (16 * NCB * WAVES) + wave * (16 * NCB) + col;
    int64_t cc[NCB];
#pragma unroll
    for (int j = 0; j < NCB; ++j) cc[j] = cell0 + 16 * j < n ? cell0 + 16 * j : n - 1;
    const int g0 = blockIdx.y * MB;
    f32x4 acc[MB][NCB];
#pragma unroll
    for (int b = 0; b < MB; ++b)
#pragma unroll
        for (int j = 0; j < NCB; ++j) acc[b][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    float x[NCB][8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int k = kq * 8 + i;
        const float *row = r + (int64_t)(k < nr ? k : nr - 1) * ldr;
#pragma unroll
        for (int j = 0; j < NCB; ++j) x[j][i] = k < nr ? row[cc[j]] : 0.f;
    }
    for (int c0 = 0; c0 < kchunks; c0 += sc) {
        // this group's nu blocks for chunks c0 .. c0 + cn - 1 (the loop is
        // uniform over the workgroup: every wave reaches both barriers)
        const int cn = kchunks - c0 < sc ? kchunks - c0 : sc;
        __syncthreads();
        for (int t = threadIdx.x; t < cn * MB * 64; t += 64 * WAVES)
            As[t] = A[((int64_t)(c0 + t / (MB * 64)) * mbp + g0) * 64 + t % (MB * 64)];
        __syncthreads();
        for (int c = c0; c < c0 + cn; ++c) {
            float xn[NCB][8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int k = (c + 1) * kChunk + kq * 8 + i;
                const float *row = r + (int64_t)(k < nr ? k : nr - 1) * ldr;
#pragma unroll
                for (int j = 0; j < NCB; ++j) {
                    xn[j][i] = row[cc[j]];
                    if (k >= nr) xn[j][i] = 0.f;
                }
            }
            bf16x8 bh[NCB], bm[NCB], bl[NCB];
#pragma unroll
            for (int j = 0; j < NCB; ++j) {
                unsigned h[8], m[8], l[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) split3(x[j][i], h[i], m[i], l[i]);
                bh[j] = pack8(h);
                bm[j] = pack8(m);
                bl[j] = pack8(l);
            }
            const u32x4 *Ac = As + (c - c0) * MB * 64 + lane;
#pragma unroll
            for (int b = 0; b < MB; ++b) {
                const bf16x8 a = __builtin_bit_cast(bf16x8, Ac[b * 64]);
#pragma unroll
                for (int j = 0; j < NCB; ++j) {
                    acc[b][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bl[j], acc[b][j], 0, 0, 0);
                    acc[b][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bm[j], acc[b][j], 0, 0, 0);
                    acc[b][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bh[j], acc[b][j], 0, 0, 0);
                }
            }
#pragma unroll
            for (int j = 0; j < NCB; ++j)
#pragma unroll
                for (int i = 0; i < 8; ++i) x[j][i] = xn[j][i];
        }
    }
#pragma unroll
    for (int j = 0; j < NCB; ++j) {
        const int64_t cell = cell0 + 16 * j;
        if (cell >= n) continue;
#pragma unroll
        for (int b = 0; b < MB; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int s = (g0 + b) * 16 + kq * 4 + v;
                if (s < ns) w[(int64_t)s * ldw + cell] = acc[b][j][v];
            }
    }
}

// cell blocks per wave for MB species blocks.  Two blocks halve the
// re-reads of the nu operand (from L2, MB KB per wave and chunk); four push
// the wave past 160 registers and halve the waves per SIMD (53/325 x 2^20:
// 0.51 ms with one, 0.39 ms with two, 1.03 ms with four)
#ifndef AK_PROD_NCB
#define AK_PROD_NCB 0
#endif
constexpr int kProdLdsBytes = 32 * 1024;   // nu staged per workgroup
#ifndef AK_PROD_LDS_WAVES
#define AK_PROD_LDS_WAVES 4
#endif
constexpr int kLdsWaves = AK_PROD_LDS_WAVES;   // waves sharing each staged block

constexpr int ncb_for(int mb)
{
    return AK_PROD_NCB > 0 ? AK_PROD_NCB : mb <= 4 ? 2 : 1;
}

struct ProdShape {
    int kchunks, mbp, mb, groups;
};

ProdShape prod_shape(int ns, int nr)
{
    ProdShape p;
    const int mbt = (ns + 15) / 16;
    p.mb = std::min(mbt, kGroup);
    p.groups = (mbt + p.mb - 1) / p.mb;
    p.mbp = p.groups * p.mb;
    p.kchunks = (nr + kChunk - 1) / kChunk;
    return p;
}

// nu in the A operand's lane order, built from the reaction records at the
// first call and kept with the mechanism
int prod_table(const ak_mechanism *m, const ProdShape &p, const u32x4 **out)
{
    std::lock_guard<std::mutex> lk(g_prod_mu);
    if (!m->prod_dev) {
        std::vector<int> nu((size_t)m->ns * m->nr, 0);   // [species][descriptor reaction]
        for (int s = 0; s < m->nr; ++s) {
            const RxnAux &x = m->host_aux[s];
            const int j = m->rxn_order[s];
            for (int q = 0; q < x.nf + x.nr; ++q)
                nu[(size_t)x.sp[q] * m->nr + j] += q < x.nf ? -1 : 1;
        }
        const size_t words = (size_t)p.kchunks * p.mbp * 64 * 4;
        std::vector<uint32_t> t(words, 0);
        for (int c = 0; c < p.kchunks; ++c)
            for (int b = 0; b < p.mbp; ++b)
                for (int l = 0; l < 64; ++l)
                    for (int i = 0; i < 8; ++i) {
                        const int s = b * 16 + (l & 15), k = c * kChunk + 8 * (l >> 4) + i;
                        if (s >= m->ns || k >= m->nr) continue;
                        const float v = (float)nu[(size_t)s * m->nr + k];
                        uint32_t bits;
                        std::memcpy(&bits, &v, 4);
                        // |nu| <= 8: its float pattern has a zero low half
                        const uint32_t bf = bits >> 16;
                        t[(((size_t)c * p.mbp + b) * 64 + l) * 4 + i / 2] |= bf << (16 * (i & 1));
                    }
        void *d = nullptr;
        hipError_t e = hipMalloc(&d, words * 4);
        if (e != hipSuccess) return hip_error(e, "ak_eval_production: table allocation");
        e = hipMemcpy(d, t.data(), words * 4, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(d);
            return hip_error(e, "ak_eval_production: table upload");
        }
        m->prod_dev = (unsigned char *)d;
    }
    *out = (const u32x4 *)m->prod_dev;
    return AK_OK;
}

}  // namespace
}  // namespace ak

using namespace ak;

extern "C" {

int ak_eval_production(const ak_mechanism *m, const float *rates, int64_t ldR, int64_t n,
                       float *omega, int64_t ldO, void *stream)
{
    const char *fn = "ak_eval_production";
    if (!m) return set_error(AK_EINVAL, "%s: null mechanism", fn);
    if (n < 0) return set_error(AK_EINVAL, "%s: n_cells < 0", fn);
    if (n > (int64_t)1 << 40) return set_error(AK_E2BIG, "%s: n_cells too large", fn);
    if (n == 0) return AK_OK;
    if (!rates || !omega) return set_error(AK_EINVAL, "%s: null pointer", fn);
    if (ldR < n || ldO < n)
        return set_error(AK_EINVAL, "%s: ldR=%lld, ldO=%lld < n_cells=%lld", fn,
                         (long long)ldR, (long long)ldO, (long long)n);
    const ProdShape p = prod_shape(m->ns, m->nr);
    const int64_t cells_per_block = 16 * ncb_for(p.mb) * (p.mb <= 4 ? 4 : kLdsWaves);
    const int64_t blocks = (n + cells_per_block - 1) / cells_per_block;
    if (blocks > 0x7fffffff) return set_error(AK_E2BIG, "%s: n_cells too large", fn);
    DeviceGuard g(m->device);
    if (!g.ok) return set_error(AK_EDEVICE, "%s: cannot select device %d", fn, m->device);
    const u32x4 *A;
    int rc = prod_table(m, p, &A);
    if (rc) return rc;
    const dim3 grid((unsigned)blocks, (unsigned)p.groups);
    // chunks of nu per LDS stage (one 1 KB block per species block and chunk)
    const int sc = std::max(1, kProdLdsBytes / (p.mb * 1024));
    const size_t lds = (size_t)sc * p.mb * 1024;
    hipStream_t st = (hipStream_t)stream;
#define AK_PROD(MB)                                                                         \
    case MB:                                                                                \
        if (MB <= 4)                                                                        \
            hipLaunchKernelGGL((production_kernel<MB, ncb_for(MB)>), grid, dim3(256), 0, st,\
                               A, p.kchunks, p.mbp, rates, ldR, m->nr, n, omega, ldO, m->ns);\
        else                                                                                \
            hipLaunchKernelGGL((production_lds_kernel<MB, ncb_for(MB), kLdsWaves>), grid,   \
                               dim3(64 * kLdsWaves),                                        \
                               lds, st, A, p.kchunks, p.mbp, sc, rates, ldR, m->nr, n,      \
                               omega, ldO, m->ns);                                          \
        break
    switch (p.mb) {
        AK_PROD(1); AK_PROD(2); AK_PROD(3); AK_PROD(4);
        AK_PROD(5); AK_PROD(6); AK_PROD(7); AK_PROD(8);
#if AK_PROD_GROUP > 8
        AK_PROD(9); AK_PROD(10); AK_PROD(11); AK_PROD(12);
        AK_PROD(13); AK_PROD(14); AK_PROD(15); AK_PROD(16);
#endif
        default: return set_error(AK_EINVAL, "%s: species blocks %d", fn, p.mb);
    }
#undef AK_PROD
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "ak_eval_production: launch");
    return AK_OK;
}

}  // extern "C"
