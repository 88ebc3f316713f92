// State update of the 0-D constant-pressure reactor (the paper's 0-D ignition
// test, Sec. 3.1): one forward-Euler step of (T, Y) at fixed P from the
// production rates omega of Eq. 2 (evaluated by the source-term kernels
// into a scratch buffer before this kernel runs):
//     Y_k <- Y_k + dt W_k omega_k / rho,     T <- T + dt omega_T,
//     omega_T = -sum_k H_k omega_k / sum_k C_k cp_k,
// with rho = sum_k C_k W_k, and the molar enthalpy H_k and heat capacity cp_k
// from the NASA-7 polynomials (the high range for T >= T_mid).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>
#include <type_traits>

#include "annkin.h"
#include "ak_device.h"
#include "ak_internal.h"

namespace ak {

template <typename IO>
__global__ __launch_bounds__(256) void euler_update_kernel(MechView m, IO *__restrict__ T,
                                                           const IO *__restrict__ P,
                                                           IO *__restrict__ Y, int64_t ldY,
                                                           int64_t n,
                                                           const IO *__restrict__ om,
                                                           int64_t ldO, double dt)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double Ti = (double)T[i], Pi = (double)P[i];
        // mixture sum of the clamped mass fractions, then rho_hat = P / (Ru T sigma)
        double sg = 0.0;
        for (int k = 0; k < m.ns; ++k) {
            const double y = (double)Y[(int64_t)k * ldY + i];
            sg += (y > 0.0 ? y : 0.0) * m.sp[k].inv_W;
        }
        const double rh = Pi / (kRu * Ti * sg);
        const double T2 = Ti * Ti, T3 = T2 * Ti, T4 = T3 * Ti;
        double num = 0.0, den = 0.0, rho = 0.0;
        for (int k = 0; k < m.ns; ++k) {
            const double y = (double)Y[(int64_t)k * ldY + i];
            const double C = rh * (y > 0.0 ? y : 0.0) * m.sp[k].inv_W;
            const double *a = Ti >= m.sp[k].T_mid ? m.th[k].hi : m.th[k].lo;
            // H/(R T) and cp/R of the NASA-7 set
            const double hRT = a[0] + a[1] * Ti / 2.0 + a[2] * T2 / 3.0 + a[3] * T3 / 4.0 +
                               a[4] * T4 / 5.0 + a[5] / Ti;
            const double cpR = a[0] + a[1] * Ti + a[2] * T2 + a[3] * T3 + a[4] * T4;
            const double w = (double)om[(int64_t)k * ldO + i];
            num += kRu * Ti * hRT * w;
            den += C * kRu * cpR;
            rho += C / m.sp[k].inv_W;
        }
        const double omT = -num / den;
        for (int k = 0; k < m.ns; ++k) {
            const int64_t o = (int64_t)k * ldY + i;
            const double w = (double)om[(int64_t)k * ldO + i];
            Y[o] = (IO)((double)Y[o] + dt * w / (m.sp[k].inv_W * rho));
        }
        T[i] = (IO)(Ti + dt * omT);
    }
}

hipError_t euler_update_launch(const MechView &m, bool f64, void *T, const void *P, void *Y,
                               int64_t ldY, int64_t n, const void *om, int64_t ldO, double dt,
                               hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks64 = std::min<int64_t>((n + 255) / 256, 65536);
    const unsigned blocks = (unsigned)blocks64;
    if (f64)
        hipLaunchKernelGGL(euler_update_kernel<double>, dim3(blocks), dim3(256), 0, st, m,
                           (double *)T, (const double *)P, (double *)Y, ldY, n,
                           (const double *)om, ldO, dt);
    else
        hipLaunchKernelGGL(euler_update_kernel<float>, dim3(blocks), dim3(256), 0, st, m,
                           (float *)T, (const float *)P, (float *)Y, ldY, n, (const float *)om,
                           ldO, dt);
    return hipGetLastError();
}

namespace {

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

}  // namespace

// Linearly implicit Euler step of the same reactor (the stiff integration
// the paper names as the next step, Sec. 4): with x = (Y, T) and
//     f(x) = (W_k omega_k / rho, omega_T),
// solve (I - dt Jf) dx = dt f(x) and set x <- x + dx, where Jf has the rows
// (W_k / rho) d omega_k / dx and d omega_T / dx of the state Jacobian J
// (cell-major, J[i*ldJ + r*nv + c]) and rho is held at the step's start.
// One cell per workgroup of one wave.  The augmented matrix [A | b] sits in
// LDS column-major (A[c * ld + r], ld odd), lanes take rows: an elimination
// step reads the lane's own entries (consecutive across the wave) and the
// pivot row's by broadcast, with no dependent reads between columns.
// Gaussian elimination with partial pivoting (largest |A[r][k]|, ties to
// the lower row), then column-oriented back substitution.  Every reduction
// has a fixed order.
template <typename IO>
__global__ __launch_bounds__(64) void implicit_update_kernel(MechView m, IO *__restrict__ T,
                                                             const IO *__restrict__ P,
                                                             IO *__restrict__ Y, int64_t ldY,
                                                             const IO *__restrict__ om,
                                                             int64_t ldO,
                                                             const IO *__restrict__ J,
                                                             int64_t ldJ, double dt)
{
    extern __shared__ double A[];
    const int64_t i = blockIdx.x;
    const int lane = threadIdx.x;
    const int ns = m.ns, nv = ns + 1;
    const int ld = ((nv + 63) & ~63) + 1;
    const double Ti = (double)T[i], Pi = (double)P[i];
    bool bad = !(Ti > 0.0) || !(Pi > 0.0) || !__builtin_isfinite(Ti) || !__builtin_isfinite(Pi);
    double sg = 0.0;
    for (int k = lane; k < ns; k += 64) {
        const double y = (double)Y[(int64_t)k * ldY + i];
        sg += (y > 0.0 ? y : 0.0) * m.sp[k].inv_W;
    }
    sg = wave_sum(sg);
    if (!(sg > 0.0) || !__builtin_isfinite(sg)) bad = true;
    const double Tu = bad ? 1000.0 : Ti;
    const double rh = bad ? 0.0 : Pi / (kRu * Tu * sg);
    const double T2 = Tu * Tu, T3 = T2 * Tu, T4 = T3 * Tu;
    double num = 0.0, den = 0.0, rho = 0.0;
    for (int k = lane; k < ns; k += 64) {
        const double y = (double)Y[(int64_t)k * ldY + i];
        const double C = rh * (y > 0.0 ? y : 0.0) * m.sp[k].inv_W;
        const double *a = Tu >= m.sp[k].T_mid ? m.th[k].hi : m.th[k].lo;
        const double hRT = a[0] + a[1] * Tu / 2.0 + a[2] * T2 / 3.0 + a[3] * T3 / 4.0 +
                           a[4] * T4 / 5.0 + a[5] / Tu;
        const double cpR = a[0] + a[1] * Tu + a[2] * T2 + a[3] * T3 + a[4] * T4;
        num += kRu * Tu * hRT * (double)om[(int64_t)k * ldO + i];
        den += C * kRu * cpR;
        rho += C / m.sp[k].inv_W;
    }
    num = wave_sum(num);
    den = wave_sum(den);
    rho = wave_sum(rho);
    const double omT = -num / den;
    if (!(rho > 0.0)) bad = true;
    // [I - dt Jf | dt f]: the row scales W_r / rho first (column nv + 1),
    // then the cell's Jacobian as one flat, coalesced sweep whose loads are
    // independent of each other
    double *S = A + (nv + 1) * ld;
    for (int r = lane; r < nv; r += 64) {
        const double sr = r < ns ? 1.0 / (m.sp[r].inv_W * rho) : 1.0;
        S[r] = sr;
        A[nv * ld + r] = dt * (r < ns ? sr * (double)om[(int64_t)r * ldO + i] : omT);
    }
    __syncthreads();
    const IO *Jc = J + i * ldJ;
    const int nn = nv * nv;
#pragma unroll 8
    for (int e = lane; e < nn; e += 64) {
        const int r = e / nv, c = e - r * nv;
        A[c * ld + r] = (r == c ? 1.0 : 0.0) - dt * S[r] * (double)Jc[e];
    }
    __syncthreads();
    for (int k = 0; k < nv && !bad; ++k) {
        double best = -1.0;
        int bi = nv;
        for (int r = k + lane; r < nv; r += 64) {
            const double v = fabs(A[k * ld + r]);
            if (v > best) {
                best = v;
                bi = r;
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            const double ov = __shfl_xor(best, o);
            const int oi = __shfl_xor(bi, o);
            if (ov > best || (ov == best && oi < bi)) {
                best = ov;
                bi = oi;
            }
        }
        if (!(best > 0.0) || !__builtin_isfinite(best)) {
            bad = true;
            break;
        }
        if (bi != k)
            for (int c = k + lane; c <= nv; c += 64) {
                const double t = A[c * ld + k];
                A[c * ld + k] = A[c * ld + bi];
                A[c * ld + bi] = t;
            }
        __syncthreads();
        const double inv = 1.0 / A[k * ld + k];
        for (int r = k + 1 + lane; r < nv; r += 64) {
            const double l = A[k * ld + r] * inv;
#pragma unroll 4
            for (int c = k + 1; c <= nv; ++c) A[c * ld + r] -= l * A[c * ld + k];
        }
        __syncthreads();
    }
    // back substitution by columns: x_k = b_k / U_kk, then b_r -= U_rk x_k
    for (int k = nv - 1; k >= 0 && !bad; --k) {
        const double xk = A[nv * ld + k] / A[k * ld + k];
        for (int r = lane; r < k; r += 64) A[nv * ld + r] -= A[k * ld + r] * xk;
        __syncthreads();
        if (lane == 0) A[nv * ld + k] = xk;
        __syncthreads();
    }
    const IO nan = (IO)__builtin_nan("");
    for (int k = lane; k < ns; k += 64) {
        const int64_t o = (int64_t)k * ldY + i;
        Y[o] = bad ? nan : (IO)((double)Y[o] + A[nv * ld + k]);
    }
    if (lane == 0) {
        T[i] = bad ? nan : (IO)(Ti + A[nv * ld + ns]);
        if (bad) atomicAdd(m.err, 1ull);
    }
}

namespace {

template <typename T>
struct Tag {
    using type = T;
};

__device__ __forceinline__ double readlane_d_impl(double v, int lane)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = __builtin_amdgcn_readlane((unsigned)b, lane);
    const unsigned hi = __builtin_amdgcn_readlane((unsigned)(b >> 32), lane);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

template <int I, int N, typename F>
__device__ __forceinline__ void unrolled(F &&f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        unrolled<I + 1, N>(f);
    }
}

// x moved across lanes by one DPP pattern (both halves); lanes with no
// source lane take 0
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

// Maximum over the 64 lanes of values >= -1 (a lane without a candidate
// holds -1), the same in every lane: a max-scan within rows of 16 lanes
// (row_shr 1, 2, 4, 8), then across rows (row_bcast 15, 31), read from lane
// 63.  The shifted-in zeros only matter when every candidate is negative,
// i.e. when there is none, and the caller treats a maximum of 0 as singular
// either way.  DPP stays in the vector registers (no LDS crossbar).
__device__ __forceinline__ double wave_max_pivot(double x)
{
    x = fmax(x, dpp_move<0x111>(x));
    x = fmax(x, dpp_move<0x112>(x));
    x = fmax(x, dpp_move<0x114>(x));
    x = fmax(x, dpp_move<0x118>(x));
    x = fmax(x, dpp_move<0x142>(x));
    x = fmax(x, dpp_move<0x143>(x));
    return readlane_d_impl(x, 63);
}

__device__ __forceinline__ double readlane_d(double v, int lane) { return readlane_d_impl(v, lane); }

}  // namespace

// The same step for systems of at most 64 unknowns with the matrix in
// registers: lane r holds row r of [A | b], padded to 64 x 65 with the
// identity (padding rows never become pivots before the real ones are
// used up, and leave the solution unchanged).  Every column index is a
// compile-time constant.  Step k: the wave maximum of |A[r][k]| over rows
// not yet used as pivots (a DPP max-scan), the lowest such lane becomes the
// pivot (ballot);
// its row is read into scalar registers (readlane) and every other unused
// row subtracts its multiple of it.  No row moves: the pivot order is kept
// in the per-lane step index, and back substitution runs over the steps in
// reverse.  No LDS, no barriers.
template <typename IO, int N>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void implicit_update_reg_kernel(MechView m, IO *__restrict__ T,
                                                                 const IO *__restrict__ P,
                                                                 IO *__restrict__ Y, int64_t ldY,
                                                                 const IO *__restrict__ om,
                                                                 int64_t ldO,
                                                                 const IO *__restrict__ J,
                                                                 int64_t ldJ, double dt)
{
    const int64_t i = blockIdx.x;
    const int r = threadIdx.x;
    const int ns = m.ns, nv = ns + 1;
    const double Ti = (double)T[i], Pi = (double)P[i];
    bool bad = !(Ti > 0.0) || !(Pi > 0.0) || !__builtin_isfinite(Ti) || !__builtin_isfinite(Pi);
    // every index below is clamped into range: lanes past the last species
    // read species 0 and discard it
    const int rs = r < ns ? r : 0;
    const double y = r < ns ? (double)Y[(int64_t)rs * ldY + i] : 0.0;
    const double yc = y > 0.0 ? y : 0.0;
    const double invW = r < ns ? m.sp[rs].inv_W : 0.0;
    const double sg = wave_sum(yc * invW);
    if (!(sg > 0.0) || !__builtin_isfinite(sg)) bad = true;
    const double Tu = bad ? 1000.0 : Ti;
    const double rh = bad ? 0.0 : Pi / (kRu * Tu * sg);
    const double T2 = Tu * Tu, T3 = T2 * Tu, T4 = T3 * Tu;
    double hterm = 0.0, cterm = 0.0, mterm = 0.0, w = 0.0;
    if (r < ns) {
        const double C = rh * yc * invW;
        const double *a = Tu >= m.sp[rs].T_mid ? m.th[rs].hi : m.th[rs].lo;
        const double hRT = a[0] + a[1] * Tu / 2.0 + a[2] * T2 / 3.0 + a[3] * T3 / 4.0 +
                           a[4] * T4 / 5.0 + a[5] / Tu;
        const double cpR = a[0] + a[1] * Tu + a[2] * T2 + a[3] * T3 + a[4] * T4;
        w = (double)om[(int64_t)rs * ldO + i];
        hterm = kRu * Tu * hRT * w;
        cterm = C * kRu * cpR;
        mterm = C / invW;
    }
    const double num = wave_sum(hterm), den = wave_sum(cterm), rho = wave_sum(mterm);
    if (!(rho > 0.0) || !(den > 0.0)) bad = true;
    const double omT = -num / den;
    // row r of [I - dt Jf | dt f]
    const double sr = r < ns ? 1.0 / (invW * rho) : 1.0;
    const IO *Jr = J + i * ldJ + (int64_t)(r < nv ? r : 0) * nv;
    double a[N + 1];
    unrolled<0, N>([&](auto c) {
        const double jv = (r < nv && c < nv) ? (double)Jr[c < nv ? (int)c : 0] : 0.0;
        a[c] = (r == c ? 1.0 : 0.0) - dt * sr * jv;
    });
    a[N] = r < ns ? dt * sr * w : (r == ns ? dt * omT : 0.0);
    int step = N;                  // the step at which this row became the pivot
    bool singular = false;
    int pivot_of[N];
    unrolled<0, N>([&](auto k) {
        const double v = step == N ? fabs(a[k]) : -1.0;
        const double mx = wave_max_pivot(v);
        const unsigned long long hit = __ballot(v == mx);
        const int p = __builtin_ctzll(hit);
        pivot_of[k] = p;
        if (!(mx > 0.0) || !__builtin_isfinite(mx)) singular = true;
        const double piv = readlane_d(a[k], p);
        const double l = (step == N && r != p) ? a[k] / piv : 0.0;
        if (r == p) step = k;
        unrolled<k + 1, N + 1>([&](auto c) { a[c] = __builtin_fma(-l, readlane_d(a[c], p), a[c]); });
    });
    // back substitution over the steps in reverse: x_k from the row that
    // pivoted step k, then the rows of earlier steps drop its column
    double mine = 0.0;
    unrolled<0, N>([&](auto kk) {
        constexpr int k = N - 1 - decltype(kk)::value;
        const int p = pivot_of[k];
        const double xk = readlane_d(a[N], p) / readlane_d(a[k], p);
        if (step < k) a[N] = __builtin_fma(-a[k], xk, a[N]);
        if (r == k) mine = xk;
    });
    bad = bad || singular;
    const IO nan = (IO)__builtin_nan("");
    if (r < ns) Y[(int64_t)rs * ldY + i] = bad ? nan : (IO)(y + mine);
    if (r == ns) T[i] = bad ? nan : (IO)(Ti + mine);
    if (r == 0 && bad) atomicAdd(m.err, 1ull);
}

size_t implicit_lds_bytes(int ns)
{
    const size_t ld = (size_t)(((ns + 1 + 63) & ~63) + 1);
    return (size_t)(ns + 3) * ld * sizeof(double);
}

hipError_t implicit_update_launch(const MechView &m, bool f64, void *T, const void *P, void *Y,
                                  int64_t ldY, int64_t n, const void *om, int64_t ldO,
                                  const void *J, int64_t ldJ, double dt, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    if (n > 0x7fffffff) return hipErrorInvalidValue;
    if (m.ns + 1 <= 64) {
        // systems padded to 16, 32 or 64 unknowns
        auto go = [&](auto kern, auto tag) {
            using E = typename decltype(tag)::type;
            hipLaunchKernelGGL(kern, dim3((unsigned)n), dim3(64), 0, st, m, (E *)T,
                               (const E *)P, (E *)Y, ldY, (const E *)om, ldO, (const E *)J, ldJ,
                               dt);
        };
        const int nv = m.ns + 1;
        if (f64) {
            if (nv <= 16) go(implicit_update_reg_kernel<double, 16>, Tag<double>{});
            else if (nv <= 32) go(implicit_update_reg_kernel<double, 32>, Tag<double>{});
            else go(implicit_update_reg_kernel<double, 64>, Tag<double>{});
        } else {
            if (nv <= 16) go(implicit_update_reg_kernel<float, 16>, Tag<float>{});
            else if (nv <= 32) go(implicit_update_reg_kernel<float, 32>, Tag<float>{});
            else go(implicit_update_reg_kernel<float, 64>, Tag<float>{});
        }
        return hipGetLastError();
    }
    const size_t lds = implicit_lds_bytes(m.ns);
    hipError_t e;
    if (f64) {
        auto k = implicit_update_kernel<double>;
        if ((e = allow_dynamic_lds((const void *)k)) != hipSuccess) return e;
        hipLaunchKernelGGL(k, dim3((unsigned)n), dim3(64), lds, st, m, (double *)T,
                           (const double *)P, (double *)Y, ldY, (const double *)om, ldO,
                           (const double *)J, ldJ, dt);
    } else {
        auto k = implicit_update_kernel<float>;
        if ((e = allow_dynamic_lds((const void *)k)) != hipSuccess) return e;
        hipLaunchKernelGGL(k, dim3((unsigned)n), dim3(64), lds, st, m, (float *)T,
                           (const float *)P, (float *)Y, ldY, (const float *)om, ldO,
                           (const float *)J, ldJ, dt);
    }
    return hipGetLastError();
}

}  // namespace ak

// ---------------------------------------------------------------------------
// The integrator without allocations: its scratch (the production rates
// between the two kernels of a step) is this file-scope device array, one
// copy per GPU, held until the process ends.  Host code uses the address
// hipGetSymbolAddress returns for the current device, never the array's
// name.

namespace {

constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];   // device address of `scratch` per ordinal

// The scratch address on device `dev` (made current by the caller): looked
// up at the first call on that device and kept.
int scratch_on(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices)
        return ak::set_error(AK_EINVAL, "ak_integrate_euler_noalloc: device %d", dev);
    std::lock_guard<std::mutex> l(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return ak::hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                 "ak_integrate_euler_noalloc: scratch address");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return AK_OK;
}

}  // namespace

extern "C" int ak_integrate_euler_noalloc(const ak_mechanism *m, ak_precision prec, void *T,
                                          const void *P, void *Y, int64_t ldY, int64_t n,
                                          double dt, int n_steps, void *stream)
{
    int rc = ak::integrate_check("ak_integrate_euler_noalloc", m, prec, T, P, Y, ldY, n, dt,
                                 n_steps);
    if (rc) return rc;
    if (n == 0 || n_steps == 0) return AK_OK;
    const size_t bytes = (size_t)m->ns * (size_t)n * (prec == AK_FP64 ? 8 : 4);
    if (bytes > kNoAllocScratchBytes)
        return ak::set_error(AK_E2BIG,
                             "ak_integrate_euler_noalloc: %d species x %lld cells need %zu bytes "
                             "of scratch, at most %zu",
                             m->ns, (long long)n, bytes, kNoAllocScratchBytes);
    ak::DeviceGuard g(m->device);
    if (!g.ok)
        return ak::set_error(AK_EDEVICE, "ak_integrate_euler_noalloc: cannot select device %d",
                             m->device);
    void *omega = nullptr;
    if ((rc = scratch_on(m->device, &omega))) return rc;
    return ak::integrate_run(m, prec, T, P, Y, ldY, n, dt, n_steps, omega, stream);
}
