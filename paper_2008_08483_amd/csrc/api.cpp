// C ABI of libannkin.so: argument checking, mechanism preprocessing and
// upload, launch dispatch.  See include/annkin.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "annkin.h"
#include "ak_device.h"
#include "ak_internal.h"
#include "ak_jit.h"

namespace ak {

static thread_local std::string g_last_error;

int set_error(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_error(hipError_t e, const char *what)
{
    return set_error(AK_EDEVICE, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

DeviceGuard::DeviceGuard(int dev) : prev(-1), ok(true)
{
    if (hipGetDevice(&prev) != hipSuccess) {
        ok = false;
        return;
    }
    if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
}
DeviceGuard::~DeviceGuard()
{
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
}

hipError_t allow_dynamic_lds(const void *fn)
{
    // Raised once per (kernel, device) to the device's whole LDS, never
    // lowered, so that concurrent launches of one kernel with different LDS
    // sizes cannot race on this process-wide attribute.
    static std::mutex mu;
    static std::map<std::pair<const void *, int>, bool> done;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> l(mu);
    if (done.count({fn, dev})) return hipSuccess;
    int lds_max = 0;
    if ((e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor,
                                   dev)) != hipSuccess)
        return e;
    lds_max = std::min(lds_max, 160 * 1024);
    // the kernel's static LDS comes out of the same budget
    hipFuncAttributes fa;
    if ((e = hipFuncGetAttributes(&fa, fn)) != hipSuccess) return e;
    const int dyn = lds_max - (int)fa.sharedSizeBytes;
    if (dyn <= 0) return hipErrorInvalidValue;
    if ((e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, dyn)) !=
        hipSuccess)
        return e;
    done[{fn, dev}] = true;
    return hipSuccess;
}

// Gibbs-layer weights on (ln T, T, T^2, T^3, T^4, 1/T, 1) for one NASA-7
// set a1..a7, scaled by log2(e):
//   G - ln(p_ref/(Ru T)) = (1 - a1) ln T - a2/2 T - a3/6 T^2 - a4/12 T^3
//                          - a5/20 T^4 + a6/T + a1 - a7 - ln(p_ref/Ru)
// (G = H/RT - S/R with the NASA-7 enthalpy and entropy, Eq. 10; the
// standard-concentration term of Eq. 9 folded into the ln T weight and the
// bias as Eq. 11 describes).
static void gibbs_weights(const double *a, double *c)
{
    c[0] = (1.0 - a[0]) * kLog2e;
    c[1] = -a[1] / 2.0 * kLog2e;
    c[2] = -a[2] / 6.0 * kLog2e;
    c[3] = -a[3] / 12.0 * kLog2e;
    c[4] = -a[4] / 20.0 * kLog2e;
    c[5] = a[5] * kLog2e;
    c[6] = (a[0] - a[6] - std::log(kPref / kRu)) * kLog2e;
}

static bool finite_all(const double *p, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

}  // namespace ak

using namespace ak;

extern "C" {

const char *ak_last_error(void) { return g_last_error.c_str(); }

const char *ak_version(void) { return "annkin 0.1 (gfx950)"; }

}  // extern "C"

namespace ak {

// Host-side preparation of a mechanism (no device needed): unit conversion,
// Gibbs-layer weights, reaction records sorted by shape, per-wave sweep
// ranges.  The device-dependent tile size is set by the caller.
struct Prepared {
    std::vector<SpeciesRec> sp;
    std::vector<RxnRec> rx;         // shape-sorted order
    std::vector<RxnAux> aux;        // same order
    std::vector<ThermoRec> th;
    std::vector<int> order;         // file index of each sorted reaction
    MechView view;                  // runs and sweep ranges filled in
    bool pdep = false;              // any third-body or falloff reaction
    std::vector<PdepRec> pd;        // [nr] sorted order (empty without pdep)
    std::vector<std::vector<double>> profiles;
};

static int prepare(const ak_mechanism_desc *d, Prepared &p)
{
    const int ns = d->n_species, nr = d->n_reactions;
    if (ns < 1 || nr < 1)
        return set_error(AK_EINVAL, "ak_load_mechanism: bad sizes ns=%d nr=%d", ns, nr);
    if (ns > kMaxSpecies)
        return set_error(AK_EUNSUPPORTED, "ak_load_mechanism: %d species, at most %d supported",
                         ns, kMaxSpecies);
    if (!d->W || !d->nu_f || !d->nu_r || !d->ln_A || !d->beta || !d->Ea || !d->nasa_low ||
        !d->nasa_high || !d->T_mid)
        return set_error(AK_EINVAL, "ak_load_mechanism: null array in descriptor");
    for (int k = 0; k < ns; ++k)
        if (!(d->W[k] > 0.0) || !std::isfinite(d->W[k]) || !std::isfinite(d->T_mid[k]))
            return set_error(AK_EINVAL, "ak_load_mechanism: bad W or T_mid of species %d", k);
    if (!finite_all(d->ln_A, nr) || !finite_all(d->beta, nr) || !finite_all(d->Ea, nr) ||
        !finite_all(d->nasa_low, 7 * (size_t)ns) || !finite_all(d->nasa_high, 7 * (size_t)ns))
        return set_error(AK_EINVAL, "ak_load_mechanism: non-finite parameter");

    p.sp.assign(ns, SpeciesRec{});
    for (int k = 0; k < ns; ++k) {
        p.sp[k].inv_W = 1.0 / d->W[k];
        p.sp[k].T_mid = d->T_mid[k];
        gibbs_weights(&d->nasa_low[7 * k], p.sp[k].lo);
        gibbs_weights(&d->nasa_high[7 * k], p.sp[k].hi);
    }
    // pressure-dependent reactions (Sec. 2.4)
    std::vector<PdepRec> pd(nr);
    if (d->rtype) {
        for (int j = 0; j < nr; ++j) {
            const int t = d->rtype[j];
            if (t > AK_RXN_TROE)
                return set_error(AK_EINVAL, "reaction %d: unknown reaction type %d", j, t);
            if (t == AK_RXN_ELEMENTARY) continue;
            p.pdep = true;
            PdepRec &r = pd[j];
            r.type = t;
            std::vector<double> e(ns, 1.0);
            if (d->efficiency)
                for (int k = 0; k < ns; ++k) {
                    e[k] = d->efficiency[(size_t)j * ns + k];
                    if (!std::isfinite(e[k]) || e[k] < 0.0)
                        return set_error(AK_EINVAL, "reaction %d: bad efficiency of species %d",
                                         j, k);
                }
            size_t q = 0;
            while (q < p.profiles.size() && p.profiles[q] != e) ++q;
            if (q == p.profiles.size()) p.profiles.push_back(e);
            r.profile = (int)q;
            if (t == AK_RXN_LINDEMANN || t == AK_RXN_TROE) {
                if (!d->low_ln_A || !d->low_beta || !d->low_Ea)
                    return set_error(AK_EINVAL, "reaction %d: falloff without low-pressure "
                                                "parameters", j);
                if (!std::isfinite(d->low_ln_A[j]) || !std::isfinite(d->low_beta[j]) ||
                    !std::isfinite(d->low_Ea[j]))
                    return set_error(AK_EINVAL, "reaction %d: non-finite low-pressure "
                                                "parameter", j);
                int order = 0;
                for (int k = 0; k < ns; ++k) order += d->nu_f[(size_t)j * ns + k];
                // k_0 carries one order more than the reaction
                r.log2A0 = (d->low_ln_A[j] + order * std::log(1e-3)) * kLog2e;
                r.beta0 = d->low_beta[j];
                r.negE0oR2 = -(d->low_Ea[j] * kCal / kRuMol) * kLog2e;
            }
            if (t == AK_RXN_TROE) {
                if (!d->troe) return set_error(AK_EINVAL, "reaction %d: Troe without parameters", j);
                const double *tp = &d->troe[4 * (size_t)j];
                if (!std::isfinite(tp[0]) || !(tp[1] > 0.0) || !(tp[2] > 0.0) ||
                    !std::isfinite(tp[1]) || !std::isfinite(tp[2]) || !std::isfinite(tp[3]) ||
                    tp[3] < 0.0)
                    return set_error(AK_EINVAL, "reaction %d: bad Troe parameters", j);
                r.alpha = tp[0];
                r.T3 = tp[1];
                r.T1 = tp[2];
                r.T2 = tp[3];
            }
        }
    }
    std::vector<RxnRec> rx(nr);
    std::vector<RxnAux> aux(nr);
    std::vector<int> shape(nr);
    for (int j = 0; j < nr; ++j) {
        RxnRec &r = rx[j];
        std::memset(&r, 0, sizeof r);
        int nf = 0, np = 0, order = 0;
        int reac[kMaxSide], prod[kMaxSide];
        for (int k = 0; k < ns; ++k) {
            const int a = d->nu_f[(size_t)j * ns + k], b = d->nu_r[(size_t)j * ns + k];
            if (a < 0 || b < 0)
                return set_error(AK_EINVAL, "reaction %d: negative stoichiometric coefficient", j);
            order += a;
            if (nf + a > kMaxSide || np + b > kMaxSide)
                return set_error(AK_EUNSUPPORTED,
                                 "reaction %d: more than %d molecules on one side", j, kMaxSide);
            for (int t = 0; t < a; ++t) reac[nf++] = k;
            for (int t = 0; t < b; ++t) prod[np++] = k;
        }
        if (nf == 0 || np == 0)
            return set_error(AK_EUNSUPPORTED, "reaction %d: empty reactant or product side", j);
        for (int t = 0; t < nf; ++t) r.sp[t] = (uint8_t)reac[t];
        for (int t = 0; t < np; ++t) r.sp[nf + t] = (uint8_t)prod[t];
        // Arrhenius parameters: A from (cm^3/mol)^(order-1)/s to (m^3/kmol)^(order-1)/s;
        // a third-body reaction's A counts [M] as one order more
        const int aorder = order + (pd[j].type == AK_RXN_THIRD_BODY ? 1 : 0);
        r.log2A = (d->ln_A[j] + (aorder - 1) * std::log(1e-3)) * kLog2e;
        r.beta = d->beta[j];
        r.negEoR2 = -(d->Ea[j] * kCal / kRuMol) * kLog2e;
        const bool rev = d->reversible == nullptr || d->reversible[j];
        // sort key: shape, then reversible before irreversible
        shape[j] = ((nf - 1) * kMaxSide + (np - 1)) * 2 + (rev ? 0 : 1);
        RxnAux &x = aux[j];
        std::memset(&x, 0, sizeof x);
        for (int t = 0; t < nf; ++t) x.sp[t] = (uint16_t)reac[t];
        for (int t = 0; t < np; ++t) x.sp[nf + t] = (uint16_t)prod[t];
        x.nf = (uint8_t)nf;
        x.nr = (uint8_t)np;
        x.rev = rev ? 1 : 0;
        x.EoR = d->Ea[j] * kCal / kRuMol;
    }
    // sort reactions by shape so that each wave of the table-driven kernels
    // runs one code path per run
    p.order.resize(nr);
    for (int j = 0; j < nr; ++j) p.order[j] = j;
    std::stable_sort(p.order.begin(), p.order.end(),
                     [&](int a, int b) { return shape[a] < shape[b]; });
    p.rx.resize(nr);
    p.aux.resize(nr);
    p.th.resize(ns);
    if (p.pdep) {
        p.pd.resize(nr);
        for (int i = 0; i < nr; ++i) p.pd[i] = pd[p.order[i]];
    }
    for (int k = 0; k < ns; ++k)
        for (int c = 0; c < 7; ++c) {
            p.th[k].lo[c] = d->nasa_low[7 * k + c];
            p.th[k].hi[c] = d->nasa_high[7 * k + c];
        }
    MechView &view = p.view;
    std::memset(&view, 0, sizeof view);
    view.ns = ns;
    view.nr = nr;
    for (int i = 0; i < nr; ++i) {
        p.rx[i] = rx[p.order[i]];
        p.aux[i] = aux[p.order[i]];
        const int s = shape[p.order[i]];
        if (i == 0 || shape[p.order[i - 1]] != s) {
            ShapeRun &run = view.runs[view.nruns++];
            run.nf = s / 2 / kMaxSide + 1;
            run.nr = s / 2 % kMaxSide + 1;
            run.rev = (s & 1) ? 0.0 : 1.0;
            run.start = i;
            run.count = 0;
        }
        view.runs[view.nruns - 1].count++;
    }
    // contiguous per-wave ranges of the sorted reactions, split by an
    // estimate of each reaction's sweep time: 16 + s^2 with s molecules (a
    // fit of measured per-wave sweep times; per-molecule costs grow with s
    // as the reaction's LDS reads and atomics contend)
    std::vector<double> cum(nr + 1, 0.0);
    for (int i = 0; i < nr; ++i) {
        const double s = p.aux[i].nf + p.aux[i].nr;
        cum[i + 1] = cum[i] + 16.0 + s * s;
    }
    auto split = [&](int32_t *seg, int w) {
        int i = 0;
        for (int k = 0; k <= w; ++k) {
            const double target = cum[nr] * k / w;
            while (i < nr && cum[i] < target) ++i;
            seg[k] = k == w ? nr : i;
        }
    };
    split(view.seg8, 8);
    split(view.seg16, 16);
    return AK_OK;
}

static JitMech jit_view(const Prepared &p)
{
    JitMech j;
    j.ns = (int)p.sp.size();
    j.nr = (int)p.rx.size();
    j.sp = p.sp.data();
    j.th = p.th.data();
    j.rx = p.rx.data();
    j.aux = p.aux.data();
    j.pd = p.pdep ? p.pd.data() : nullptr;
    j.profiles = &p.profiles;
    return j;
}

}  // namespace ak

extern "C" {

int ak_jit_source(const ak_mechanism_desc *d, ak_precision prec, char *buf, size_t cap,
                  size_t *needed)
{
    if (!d || !needed) return set_error(AK_EINVAL, "ak_jit_source: null argument");
    if (prec != AK_FP32 && prec != AK_FP64)
        return set_error(AK_EINVAL, "ak_jit_source: bad precision %d", (int)prec);
    Prepared p;
    int rc = prepare(d, p);
    if (rc) return rc;
    const std::string src = jit_generate(jit_view(p), prec == AK_FP64).src;
    *needed = src.size() + 1;
    if (buf && cap > 0) {
        const size_t n = std::min(cap - 1, src.size());
        std::memcpy(buf, src.data(), n);
        buf[n] = 0;
    }
    return AK_OK;
}

int ak_jit_tables(const ak_mechanism_desc *d, ak_precision prec, double *sp, size_t cap_sp,
                  double *rx, size_t cap_rx, size_t *n_sp, size_t *n_rx)
{
    if (!d || !n_sp || !n_rx) return set_error(AK_EINVAL, "ak_jit_tables: null argument");
    if (prec != AK_FP32 && prec != AK_FP64)
        return set_error(AK_EINVAL, "ak_jit_tables: bad precision %d", (int)prec);
    Prepared p;
    int rc = prepare(d, p);
    if (rc) return rc;
    const JitProgram prog = jit_generate(jit_view(p), prec == AK_FP64);
    *n_sp = prog.sp.size();
    *n_rx = prog.rx.size();
    if (sp) std::memcpy(sp, prog.sp.data(), sizeof(double) * std::min(cap_sp, prog.sp.size()));
    if (rx) std::memcpy(rx, prog.rx.data(), sizeof(double) * std::min(cap_rx, prog.rx.size()));
    return AK_OK;
}

int ak_jit_jacobian_source(const ak_mechanism_desc *d, ak_precision prec, int variant,
                           char *buf, size_t cap, size_t *needed)
{
    if (!d || !needed) return set_error(AK_EINVAL, "ak_jit_jacobian_source: null argument");
    if (prec != AK_FP32 && prec != AK_FP64)
        return set_error(AK_EINVAL, "ak_jit_jacobian_source: bad precision %d", (int)prec);
    Prepared p;
    int rc = prepare(d, p);
    if (rc) return rc;
    const JitMech jm = jit_view(p);
    if (!jac_suitable(jm))
        return set_error(AK_EUNSUPPORTED, "ak_jit_jacobian_source: no compiled Jacobian for this "
                                          "mechanism (pressure-dependent reactions or %d species)",
                         jm.ns);
    if (variant < 0 || variant > 2)
        return set_error(AK_EINVAL, "ak_jit_jacobian_source: bad variant %d", variant);
    const std::string src = variant == 2 ? jit_program_vjp(jm, prec == AK_FP64).src
                                         : jit_program_jac(jm, prec == AK_FP64, variant == 1).src;
    *needed = src.size() + 1;
    if (buf && cap > 0) {
        const size_t n = std::min(cap - 1, src.size());
        std::memcpy(buf, src.data(), n);
        buf[n] = 0;
    }
    return AK_OK;
}

int ak_jit_jacobian_tables(const ak_mechanism_desc *d, double *sp, size_t cap_sp, double *rx,
                           size_t cap_rx, size_t *n_sp, size_t *n_rx)
{
    if (!d || !n_sp || !n_rx) return set_error(AK_EINVAL, "ak_jit_jacobian_tables: null argument");
    Prepared p;
    int rc = prepare(d, p);
    if (rc) return rc;
    const JitMech jm = jit_view(p);
    if (!jac_suitable(jm))
        return set_error(AK_EUNSUPPORTED, "ak_jit_jacobian_tables: no compiled Jacobian for this "
                                          "mechanism");
    const JitProgram prog = jit_program_jac(jm, true);
    *n_sp = prog.sp.size();
    *n_rx = prog.rx.size();
    if (sp) std::memcpy(sp, prog.sp.data(), sizeof(double) * std::min(cap_sp, prog.sp.size()));
    if (rx) std::memcpy(rx, prog.rx.data(), sizeof(double) * std::min(cap_rx, prog.rx.size()));
    return AK_OK;
}

int ak_load_mechanism(const ak_mechanism_desc *d, int device, ak_mechanism **out)
{
    return ak_load_mechanism_ex(d, device, AK_KERNEL_AUTO, out);
}

int ak_load_mechanism_ex(const ak_mechanism_desc *d, int device, int kernels, ak_mechanism **out)
{
    if (!d || !out) return set_error(AK_EINVAL, "ak_load_mechanism: null argument");
    *out = nullptr;
    if (kernels != AK_KERNEL_AUTO && kernels != AK_KERNEL_TABLE)
        return set_error(AK_EINVAL, "ak_load_mechanism: bad kernel choice %d", kernels);
    Prepared p;
    int rc = prepare(d, p);
    if (rc) return rc;
    const int ns = p.view.ns, nr = p.view.nr;

    DeviceGuard g(device);
    if (!g.ok) return set_error(AK_EDEVICE, "ak_load_mechanism: cannot select device %d", device);
    // tile: cells per workgroup, as many as the LDS holds (at most 64)
    int lds_max = 0;
    if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor,
                              device) != hipSuccess || lds_max <= 0)
        return set_error(AK_EDEVICE, "ak_load_mechanism: cannot query LDS size of device %d",
                         device);
    lds_max = std::min(lds_max, 160 * 1024);
    const int tile = std::min<int>(kMaxTile, lds_max / (ns * kEntry));
    if (tile < 16)
        return set_error(AK_EUNSUPPORTED, "ak_load_mechanism: %d species do not fit the LDS tile",
                         ns);
    MechView view = p.view;
    view.tile = tile;
    // 8-wave workgroups when two tiles share a CU's LDS, else one tile of 16
    // waves, so that a CU runs 16 waves either way
    view.waves = 2 * (size_t)ns * tile * kEntry <= (size_t)lds_max ? 8 : 16;

    // the mechanism-compiled kernels (both precisions) where they fit
    std::vector<char> code[2];
    JitProgram prog[2];
    bool use_jit[2] = {false, false};
    for (int f = 0; f < 2; ++f) {
        const bool f64 = f == AK_FP64;   // index = ak_precision
        if (kernels != AK_KERNEL_AUTO || !jit_suitable(ns, f64)) continue;
        prog[f] = jit_generate(jit_view(p), f64);
        std::string log;
        rc = jit_compile(prog[f].src, code[f], log);
        if (rc) return set_error(rc, "ak_load_mechanism: compiling the mechanism's kernels "
                                     "failed: %s", log.c_str());
        use_jit[f] = true;
    }
    if (p.pdep && !use_jit[0] && !use_jit[1])
        return set_error(AK_EUNSUPPORTED,
                         "ak_load_mechanism: third-body and falloff reactions need the compiled "
                         "kernels (AK_KERNEL_AUTO and a mechanism of at most %d species)",
                         kJitMaxSpeciesFP32);

    ak_mechanism *m = new (std::nothrow) ak_mechanism();
    if (!m) return set_error(AK_ENOMEM, "ak_load_mechanism: out of host memory");
    m->device = device;
    m->ns = ns;
    m->nr = nr;
    m->lds_max = lds_max;
    m->vjp_tile = vjp_tile(ns, lds_max);
    hipError_t e;
    // one device allocation holds every table
    const size_t o_sp = 0;
    const size_t o_rx = o_sp + ((sizeof(SpeciesRec) * ns + 255) & ~(size_t)255);
    const size_t o_th = o_rx + ((sizeof(RxnRec) * (nr + kRecordPad) + 255) & ~(size_t)255);
    const size_t o_aux = o_th + ((sizeof(ThermoRec) * ns + 255) & ~(size_t)255);
    const size_t o_err = o_aux + ((sizeof(RxnAux) * nr + 255) & ~(size_t)255);
    // tables of the compiled kernels, per precision: species, reactions
    const size_t jsp_bytes = (sizeof(double) * 16 * ns + 255) & ~(size_t)255;
    // (falloff reactions carry more constants than the 3 of the others)
    const size_t jrx_bytes =
        (sizeof(double) * std::max(prog[0].rx.size(), prog[1].rx.size()) + 255) & ~(size_t)255;
    size_t o_jsp[2], o_jrx[2];
    o_jsp[0] = o_err + 256;
    o_jrx[0] = o_jsp[0] + jsp_bytes;
    o_jsp[1] = o_jrx[0] + jrx_bytes;
    o_jrx[1] = o_jsp[1] + jsp_bytes;
    const size_t bytes = o_jrx[1] + jrx_bytes;
    std::vector<unsigned char> host(bytes, 0);
    for (int f = 0; f < 2; ++f)
        if (use_jit[f]) {
            std::memcpy(&host[o_jsp[f]], prog[f].sp.data(), sizeof(double) * 16 * ns);
            std::memcpy(&host[o_jrx[f]], prog[f].rx.data(), sizeof(double) * prog[f].rx.size());
        }
    std::memcpy(&host[o_sp], p.sp.data(), sizeof(SpeciesRec) * ns);
    std::memcpy(&host[o_rx], p.rx.data(), sizeof(RxnRec) * nr);
    std::memcpy(&host[o_th], p.th.data(), sizeof(ThermoRec) * ns);
    std::memcpy(&host[o_aux], p.aux.data(), sizeof(RxnAux) * nr);
    unsigned char *dev = nullptr;
    if ((e = hipMalloc((void **)&dev, bytes)) != hipSuccess) {
        delete m;
        return set_error(AK_ENOMEM, "ak_load_mechanism: device allocation failed: %s",
                         hipGetErrorString(e));
    }
    if ((e = hipMemcpy(dev, host.data(), bytes, hipMemcpyHostToDevice)) != hipSuccess) {
        (void)hipFree(dev);
        delete m;
        return hip_error(e, "ak_load_mechanism: upload");
    }
    m->dev = dev;
    view.sp = (const SpeciesRec *)(dev + o_sp);
    view.rx = (const RxnRec *)(dev + o_rx);
    view.th = (const ThermoRec *)(dev + o_th);
    view.aux = (const RxnAux *)(dev + o_aux);
    view.err = (unsigned long long *)(dev + o_err);
    m->view = view;
    for (int f = 0; f < 2; ++f) {
        if (!use_jit[f]) continue;
        rc = jit_load(code[f], m->jit[f]);
        m->jit[f].threads = prog[f].threads;
        m->jit[f].sp = (const double *)(dev + o_jsp[f]);
        m->jit[f].rx = (const double *)(dev + o_jrx[f]);
        m->jit[f].T_lo = prog[f].T_lo;
        m->jit[f].T_hi = prog[f].T_hi;
        if (rc) {
            for (int q = 0; q < 2; ++q) jit_unload(m->jit[q]);
            (void)hipFree(dev);
            delete m;
            return rc;
        }
    }
    m->pdep = p.pdep;
    m->host_aux = p.aux;
    m->host_th = p.th;
    m->host_species = std::move(p.sp);
    m->host_rxn = std::move(p.rx);
    m->rxn_order = std::move(p.order);
    *out = m;
    return AK_OK;
}

int ak_free_mechanism(ak_mechanism *m)
{
    if (!m) return AK_OK;
    DeviceGuard g(m->device);
    for (int f = 0; f < 2; ++f) {
        jit_unload(m->jit[f]);
        jit_unload(m->jac[f][0]);
        jit_unload(m->jac[f][1]);
        jit_unload(m->vjp[f]);
    }
    if (m->jac_dev) (void)hipFree(m->jac_dev);
    if (m->kc_dev) (void)hipFree(m->kc_dev);
    if (m->prod_dev) (void)hipFree(m->prod_dev);
    (void)hipFree(m->dev);
    delete m;
    return AK_OK;
}

int ak_mechanism_n_species(const ak_mechanism *m) { return m ? m->ns : -1; }

int ak_mechanism_compiled(const ak_mechanism *m, ak_precision prec)
{
    if (!m || (prec != AK_FP32 && prec != AK_FP64))
        return set_error(AK_EINVAL, "ak_mechanism_compiled: bad argument");
    return m->jit[prec].src ? 1 : 0;
}
int ak_mechanism_n_reactions(const ak_mechanism *m) { return m ? m->nr : -1; }

int ak_eval_source(const ak_mechanism *m, ak_precision prec, const void *T, const void *P,
                   const void *Y, int64_t ldY, int64_t n, void *omega, int64_t ldO, void *stream)
{
    if (!m) return set_error(AK_EINVAL, "ak_eval_source: null mechanism");
    if (prec != AK_FP32 && prec != AK_FP64)
        return set_error(AK_EINVAL, "ak_eval_source: bad precision %d", (int)prec);
    if (n < 0) return set_error(AK_EINVAL, "ak_eval_source: n_cells < 0");
    if (n == 0) return AK_OK;
    if (!T || !P || !Y || !omega) return set_error(AK_EINVAL, "ak_eval_source: null pointer");
    if (ldY < n || ldO < n)
        return set_error(AK_EINVAL, "ak_eval_source: ldY=%lld ldO=%lld < n_cells=%lld",
                         (long long)ldY, (long long)ldO, (long long)n);
    if (n > (int64_t)1 << 40) return set_error(AK_E2BIG, "ak_eval_source: n_cells too large");
    DeviceGuard g(m->device);
    if (!g.ok) return set_error(AK_EDEVICE, "ak_eval_source: cannot select device %d", m->device);
    const JitKernels &jk = m->jit[prec];   // indexed by ak_precision
    if (!jk.src && m->pdep)
        return set_error(AK_EUNSUPPORTED, "ak_eval_source: third-body and falloff reactions "
                                          "need the compiled kernel, which this mechanism has "
                                          "not for %s", prec == AK_FP64 ? "AK_FP64" : "AK_FP32");
    hipError_t e = jk.src ? jit_launch(jk, T, P, Y, ldY, n, omega, ldO, m->view.err,
                                       (hipStream_t)stream)
                          : source_launch(m->view, prec == AK_FP64, T, P, Y, ldY, n, omega, ldO,
                                          (hipStream_t)stream);
    if (e != hipSuccess) return hip_error(e, "ak_eval_source: launch");
    return AK_OK;
}

static int check_state(const char *fn, const ak_mechanism *m, ak_precision prec, const void *T,
                       const void *P, const void *Y, int64_t ldY, int64_t n)
{
    if (!m) return set_error(AK_EINVAL, "%s: null mechanism", fn);
    if (prec != AK_FP32 && prec != AK_FP64)
        return set_error(AK_EINVAL, "%s: bad precision %d", fn, (int)prec);
    if (n < 0) return set_error(AK_EINVAL, "%s: n_cells < 0", fn);
    if (n > 0 && (!T || !P || !Y)) return set_error(AK_EINVAL, "%s: null state pointer", fn);
    if (n > 0 && ldY < n)
        return set_error(AK_EINVAL, "%s: ldY=%lld < n_cells=%lld", fn, (long long)ldY,
                         (long long)n);
    if (n > (int64_t)1 << 40) return set_error(AK_E2BIG, "%s: n_cells too large", fn);
    return AK_OK;
}

}  // extern "C"

namespace ak {

namespace {

JitMech jit_view(const ak_mechanism *m)
{
    JitMech j;
    j.ns = m->ns;
    j.nr = m->nr;
    j.sp = m->host_species.data();
    j.th = m->host_th.data();
    j.rx = m->host_rxn.data();
    j.aux = m->host_aux.data();
    return j;
}

bool jac_wanted()
{
    const char *e = std::getenv("AK_JIT_JACOBIAN");
    return !e || std::atoi(e) != 0;
}

bool jac_fits(const ak_mechanism *m) { return !m->pdep && jac_suitable(jit_view(m)); }

bool vjp_wanted()
{
    const char *e = std::getenv("AK_JIT_VJP");
    return !e || std::atoi(e) != 0;
}

// The compiled derivative kernel `which` (0 the cell-major Jacobian, 1 the
// interleaved one, 2 the VJP) of this precision, generated, compiled and
// loaded on the first call that uses it (the device is current; the caller
// has checked jac_fits).
int compiled_jacobian(const ak_mechanism *m, ak_precision prec, int which)
{
    std::lock_guard<std::mutex> l(m->jac_mu);
    int &state = which == 2 ? m->vjp_state[prec] : m->jac_state[prec][which];
    JitKernels &k = which == 2 ? m->vjp[prec] : m->jac[prec][which];
    if (state) return AK_OK;
    const JitMech jm = jit_view(m);
    const JitProgram prog = which == 2 ? jit_program_vjp(jm, prec == AK_FP64)
                                       : jit_program_jac(jm, prec == AK_FP64, which == 1);
    std::vector<char> code;
    std::string log;
    int rc = jit_compile(prog.src, code, log, jac_compile_options());
    if (rc) return set_error(rc, "compiling the mechanism's derivative kernel failed: %s",
                             log.c_str());
    if (!m->jac_dev) {
        // the tables are the same for both precisions and layouts
        const size_t o_rx = (sizeof(double) * prog.sp.size() + 255) & ~(size_t)255;
        const size_t bytes = o_rx + sizeof(double) * prog.rx.size();
        unsigned char *dev = nullptr;
        hipError_t e = hipMalloc((void **)&dev, bytes);
        if (e != hipSuccess)
            return set_error(AK_ENOMEM, "ak_eval_jacobian: device allocation failed: %s",
                             hipGetErrorString(e));
        std::vector<unsigned char> host(bytes, 0);
        std::memcpy(host.data(), prog.sp.data(), sizeof(double) * prog.sp.size());
        std::memcpy(host.data() + o_rx, prog.rx.data(), sizeof(double) * prog.rx.size());
        if ((e = hipMemcpy(dev, host.data(), bytes, hipMemcpyHostToDevice)) != hipSuccess) {
            (void)hipFree(dev);
            return hip_error(e, "ak_eval_jacobian: upload");
        }
        m->jac_dev = dev;
        for (int f = 0; f < 2; ++f) {
            for (int y = 0; y < 2; ++y) {
                m->jac[f][y].sp = (const double *)dev;
                m->jac[f][y].rx = (const double *)(dev + o_rx);
            }
            m->vjp[f].sp = (const double *)dev;
            m->vjp[f].rx = (const double *)(dev + o_rx);
        }
    }
    if ((rc = jit_load(code, k, which == 2 ? "ak_vjp" : "ak_jac", nullptr))) return rc;
    k.block = 64;
    k.threads = prog.threads;
    state = 1;
    return AK_OK;
}

}  // namespace

}  // namespace ak

extern "C" {

int ak_eval_jacobian(const ak_mechanism *m, ak_precision prec, const void *T, const void *P,
                     const void *Y, int64_t ldY, int64_t n, void *J, int64_t ldJ, void *stream)
{
    int rc = check_state("ak_eval_jacobian", m, prec, T, P, Y, ldY, n);
    if (rc) return rc;
    if (n == 0) return AK_OK;
    const int64_t nv = (int64_t)m->ns + 1;
    if (!J) return set_error(AK_EINVAL, "ak_eval_jacobian: null J");
    if (ldJ < nv * nv)
        return set_error(AK_EINVAL, "ak_eval_jacobian: ldJ=%lld < (NS+1)^2=%lld", (long long)ldJ,
                         (long long)(nv * nv));
    if (m->pdep)
        return set_error(AK_EUNSUPPORTED, "ak_eval_jacobian: third-body and falloff reactions "
                                          "are not differentiated");
    const bool compiled = jac_wanted() && jac_fits(m);
    if (jacobian_lds_bytes(m->ns) > (size_t)m->lds_max && !compiled)
        return set_error(AK_EUNSUPPORTED, "ak_eval_jacobian: %d species exceed the LDS", m->ns);
    DeviceGuard g(m->device);
    if (!g.ok) return set_error(AK_EDEVICE, "ak_eval_jacobian: cannot select device %d", m->device);
    if (compiled && (rc = compiled_jacobian(m, prec, 0))) return rc;
    hipError_t e;
    if (compiled)
        e = jit_launch(m->jac[prec][0], T, P, Y, ldY, n, J, ldJ, m->view.err, (hipStream_t)stream);
    else
        e = jacobian_launch(m->view, m->lds_max, prec == AK_FP64, T, P, Y, ldY, n, J, ldJ,
                            (hipStream_t)stream);
    if (e != hipSuccess) return hip_error(e, "ak_eval_jacobian: launch");
    return AK_OK;
}

int ak_mechanism_compiled_jacobian(const ak_mechanism *m, ak_precision prec)
{
    if (!m || (prec != AK_FP32 && prec != AK_FP64))
        return set_error(AK_EINVAL, "ak_mechanism_compiled_jacobian: bad argument");
    return jac_fits(m) ? 1 : 0;
}

int ak_eval_jacobian_interleaved(const ak_mechanism *m, ak_precision prec, const void *T,
                                 const void *P, const void *Y, int64_t ldY, int64_t n, void *J,
                                 int64_t ldJ, void *stream)
{
    int rc = check_state("ak_eval_jacobian_interleaved", m, prec, T, P, Y, ldY, n);
    if (rc) return rc;
    if (n == 0) return AK_OK;
    if (!J) return set_error(AK_EINVAL, "ak_eval_jacobian_interleaved: null J");
    if (ldJ < n)
        return set_error(AK_EINVAL, "ak_eval_jacobian_interleaved: ldJ=%lld < n_cells=%lld",
                         (long long)ldJ, (long long)n);
    if (!jac_fits(m))
        return set_error(AK_EUNSUPPORTED, "ak_eval_jacobian_interleaved: no compiled Jacobian for "
                                          "this mechanism (pressure-dependent reactions or %d "
                                          "species)", m->ns);
    DeviceGuard g(m->device);
    if (!g.ok)
        return set_error(AK_EDEVICE, "ak_eval_jacobian_interleaved: cannot select device %d",
                         m->device);
    if ((rc = compiled_jacobian(m, prec, 1))) return rc;
    hipError_t e = jit_launch(m->jac[prec][1], T, P, Y, ldY, n, J, ldJ, m->view.err,
                              (hipStream_t)stream);
    if (e != hipSuccess) return hip_error(e, "ak_eval_jacobian_interleaved: launch");
    return AK_OK;
}

int ak_eval_vjp(const ak_mechanism *m, ak_precision prec, const void *T, const void *P,
                const void *Y, int64_t ldY, int64_t n, const void *g_omega, int64_t ldG,
                void *g_Y, int64_t ldGY, void *g_T, void *stream)
{
    int rc = check_state("ak_eval_vjp", m, prec, T, P, Y, ldY, n);
    if (rc) return rc;
    if (n == 0) return AK_OK;
    if (!g_omega || !g_Y || !g_T) return set_error(AK_EINVAL, "ak_eval_vjp: null pointer");
    if (ldG < n || ldGY < n)
        return set_error(AK_EINVAL, "ak_eval_vjp: ldG=%lld ldGY=%lld < n_cells=%lld",
                         (long long)ldG, (long long)ldGY, (long long)n);
    if (m->pdep)
        return set_error(AK_EUNSUPPORTED, "ak_eval_vjp: third-body and falloff reactions are "
                                          "not differentiated");
    const bool compiled = vjp_wanted() && jac_fits(m);
    if (m->vjp_tile < 16 && !compiled)
        return set_error(AK_EUNSUPPORTED, "ak_eval_vjp: %d species exceed the LDS", m->ns);
    DeviceGuard g(m->device);
    if (!g.ok) return set_error(AK_EDEVICE, "ak_eval_vjp: cannot select device %d", m->device);
    if (compiled && (rc = compiled_jacobian(m, prec, 2))) return rc;
    hipError_t e = compiled ? jit_vjp_launch(m->vjp[prec], T, P, Y, ldY, n, g_omega, ldG, g_Y,
                                             ldGY, g_T, m->view.err, (hipStream_t)stream)
                            : vjp_launch(m->view, m->vjp_tile, prec == AK_FP64, T, P, Y, ldY, n,
                                         g_omega, ldG, g_Y, ldGY, g_T, (hipStream_t)stream);
    if (e != hipSuccess) return hip_error(e, "ak_eval_vjp: launch");
    return AK_OK;
}

}  // extern "C"

namespace ak {

int integrate_check(const char *fn, const ak_mechanism *m, int prec, const void *T,
                    const void *P, const void *Y, int64_t ldY, int64_t n, double dt,
                    int n_steps)
{
    int rc = check_state(fn, m, (ak_precision)prec, T, P, Y, ldY, n);
    if (rc) return rc;
    if (!(dt > 0.0) || !std::isfinite(dt))
        return set_error(AK_EINVAL, "%s: dt must be positive and finite", fn);
    if (n_steps < 0) return set_error(AK_EINVAL, "%s: n_steps < 0", fn);
    if (!m->jit[prec].src && m->pdep)
        return set_error(AK_EUNSUPPORTED, "%s: third-body and falloff reactions need the "
                                          "compiled kernel for this precision", fn);
    return AK_OK;
}

int integrate_run(const ak_mechanism *m, int prec, void *T, const void *P, void *Y,
                  int64_t ldY, int64_t n, double dt, int n_steps, void *omega, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    const JitKernels &jk = m->jit[prec];
    for (int s = 0; s < n_steps; ++s) {
        hipError_t e = jk.src ? jit_launch(jk, T, P, Y, ldY, n, omega, n, m->view.err, st)
                              : source_launch(m->view, prec == AK_FP64, T, P, Y, ldY, n, omega,
                                              n, st);
        if (e == hipSuccess)
            e = euler_update_launch(m->view, prec == AK_FP64, T, P, Y, ldY, n, omega, n, dt, st);
        if (e != hipSuccess) return hip_error(e, "integrator step");
    }
    return AK_OK;
}

}  // namespace ak

extern "C" {

int ak_integrate_euler(const ak_mechanism *m, ak_precision prec, void *T, const void *P,
                       void *Y, int64_t ldY, int64_t n, double dt, int n_steps, void *stream)
{
    int rc = integrate_check("ak_integrate_euler", m, prec, T, P, Y, ldY, n, dt, n_steps);
    if (rc) return rc;
    if (n == 0 || n_steps == 0) return AK_OK;
    DeviceGuard g(m->device);
    if (!g.ok) return set_error(AK_EDEVICE, "ak_integrate_euler: cannot select device %d",
                                m->device);
    hipStream_t st = (hipStream_t)stream;
    const size_t bytes = (size_t)m->ns * (size_t)n * (prec == AK_FP64 ? 8 : 4);
    void *omega = nullptr;
    hipError_t e = hipMallocAsync(&omega, bytes, st);
    if (e != hipSuccess)
        return set_error(AK_ENOMEM, "ak_integrate_euler: scratch of %zu bytes: %s", bytes,
                         hipGetErrorString(e));
    rc = integrate_run(m, prec, T, P, Y, ldY, n, dt, n_steps, omega, stream);
    e = hipFreeAsync(omega, st);
    if (rc) return rc;
    if (e != hipSuccess) return hip_error(e, "ak_integrate_euler: freeing the scratch");
    return AK_OK;
}

int ak_integrate_implicit(const ak_mechanism *m, ak_precision prec, void *T, const void *P,
                          void *Y, int64_t ldY, int64_t n, double dt, int n_steps, void *stream)
{
    const char *fn = "ak_integrate_implicit";
    int rc = integrate_check(fn, m, prec, T, P, Y, ldY, n, dt, n_steps);
    if (rc) return rc;
    if (m->pdep)
        return set_error(AK_EUNSUPPORTED, "%s: third-body and falloff reactions are not "
                                          "differentiated", fn);
    if (implicit_lds_bytes(m->ns) > (size_t)m->lds_max)
        return set_error(AK_EUNSUPPORTED, "%s: %d species exceed the LDS", fn, m->ns);
    if (n == 0 || n_steps == 0) return AK_OK;
    if (n > 0x7fffffff) return set_error(AK_E2BIG, "%s: n_cells too large", fn);
    DeviceGuard g(m->device);
    if (!g.ok) return set_error(AK_EDEVICE, "%s: cannot select device %d", fn, m->device);
    hipStream_t st = (hipStream_t)stream;
    const size_t es = prec == AK_FP64 ? 8 : 4;
    const int64_t nv = (int64_t)m->ns + 1;
    const size_t jbytes = (size_t)n * nv * nv * es, obytes = (size_t)m->ns * n * es;
    void *scratch = nullptr;
    hipError_t e = hipMallocAsync(&scratch, jbytes + obytes + 256, st);
    if (e != hipSuccess)
        return set_error(AK_ENOMEM, "%s: scratch of %zu bytes: %s", fn, jbytes + obytes,
                         hipGetErrorString(e));
    void *J = scratch;
    void *om = (unsigned char *)scratch + ((jbytes + 255) & ~(size_t)255);
    const JitKernels &jk = m->jit[prec];
    for (int s = 0; s < n_steps && !rc; ++s) {
        if ((rc = ak_eval_jacobian(m, prec, T, P, Y, ldY, n, J, nv * nv, stream))) break;
        e = jk.src ? jit_launch(jk, T, P, Y, ldY, n, om, n, m->view.err, st)
                   : source_launch(m->view, prec == AK_FP64, T, P, Y, ldY, n, om, n, st);
        if (e == hipSuccess)
            e = implicit_update_launch(m->view, prec == AK_FP64, T, P, Y, ldY, n, om, n, J,
                                       nv * nv, dt, st);
        if (e != hipSuccess) rc = hip_error(e, "ak_integrate_implicit: step");
    }
    e = hipFreeAsync(scratch, st);
    if (rc) return rc;
    if (e != hipSuccess) return hip_error(e, "ak_integrate_implicit: freeing the scratch");
    return AK_OK;
}

int ak_error_count(const ak_mechanism *m, void *stream, int64_t *n_bad)
{
    if (!m || !n_bad) return set_error(AK_EINVAL, "ak_error_count: null argument");
    DeviceGuard g(m->device);
    unsigned long long v = 0, zero = 0;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    if ((e = hipMemcpyAsync(&v, m->view.err, sizeof v, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipMemcpyAsync(m->view.err, &zero, sizeof zero, hipMemcpyHostToDevice, st)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_error(e, "ak_error_count");
    *n_bad = (int64_t)v;
    return AK_OK;
}

}  // extern "C"
