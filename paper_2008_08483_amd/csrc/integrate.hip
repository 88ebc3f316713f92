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
