// Mechanism-compiled source-term kernels.
//
// The exact form of the paper (Eqs. 2, 4, 6, 7, 9-11) is evaluated with one
// lane per cell and the cell's whole state in registers: per species
//     a_k = C_k exp(Gt_k),  v_k = exp(-Gt_k)      (Gt: Gibbs-layer output)
// and an omega accumulator.  The stoichiometry of the mechanism is written
// into the kernel text, so every gather of a_k / v_k and every scatter into
// omega_k names a register: there is no index arithmetic, no LDS and no
// atomic, and the accumulation order of every omega_k is fixed by the text
// (results are bitwise reproducible and independent of the batch).  The
// numeric parameters (Gibbs-layer weights, Arrhenius layer) stay in the
// mechanism's device tables and are read with scalar loads at constant
// offsets.
//
// Per reaction (reactant molecules r, product molecules p, k_f from the
// Arrhenius layer in base 2, t = log2 k_f):
//     q_f - q_r = 2^t * prod_r v * (prod_r a - rev * prod_p a)
// which is Eq. 4 re-associated with ln K_c = -sum_k nu_kj Gt_k (Eq. 11).
// The FP32 path evaluates 2^t as 2^n * 2^f with the split in double and
// 2^f (|f| <= 1/2) on the transcendental unit, and accumulates omega in
// float; the FP64 path uses a degree-12 Taylor polynomial for 2^f and
// accumulates in double.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <iterator>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include <sys/stat.h>
#include <unistd.h>

#include "annkin.h"
#include "ak_internal.h"
#include "ak_jit.h"
#include "jit_text.h"

namespace ak {

bool jit_suitable(int ns, bool f64)
{
    // the tiled form keeps a (double) and v (float or double) of each
    // species and cell of a 64-cell tile in LDS and needs two tiles per CU;
    // the accumulators (one per species) stay within the register cap
    return tile_lds_bytes(ns, f64, kTileWaves) <= 80 * 1024;
}

size_t tile_lds_bytes(int ns, bool f64, int waves)
{
    const size_t v = f64 ? 8 : 4;   // FP32 path: v as float where its range allows
    return (size_t)64 * ns * (8 + v) + (size_t)64 * waves * (8 + (f64 ? 8 : 4));
}

namespace {

// Gibbs-layer output in base 2 (the device weights of one species) at T
double g2_host(const SpeciesRec &s, double T)
{
    const double *c = T >= s.T_mid ? s.hi : s.lo;
    return c[0] * std::log(T) + c[1] * T + c[2] * T * T + c[3] * T * T * T +
           c[4] * T * T * T * T + c[5] / T + c[6];
}

// Order of the reactions in the generated code.  A species' registers are
// live from its first reaction to its last, so the order is chosen greedily
// to open few new species and close many at each step (ties: lowest index).
std::vector<int> live_order(const JitMech &m, const std::vector<std::vector<int>> &rs)
{
    std::vector<int> left(m.ns, 0), order;
    std::vector<char> open(m.ns, 0), done(m.nr, 0);
    for (int j = 0; j < m.nr; ++j)
        for (int k : rs[j]) left[k]++;
    order.reserve(m.nr);
    for (int step = 0; step < m.nr; ++step) {
        int best = -1, bkey = 0, bclose = 0;
        for (int j = 0; j < m.nr; ++j) {
            if (done[j]) continue;
            int opens = 0, closes = 0;
            for (int k : rs[j]) {
                opens += !open[k];
                closes += left[k] == 1;
            }
            const int key = opens - closes;
            if (best < 0 || key < bkey || (key == bkey && closes > bclose)) {
                best = j;
                bkey = key;
                bclose = closes;
            }
        }
        done[best] = 1;
        order.push_back(best);
        for (int k : rs[best]) {
            open[k] = 1;
            left[k]--;
        }
    }
    return order;
}

}  // namespace

namespace {

// What both generators share: the FP32 path's per-species shifts of v and
// the species table.
struct Common {
    std::vector<int> h;        // integer shift of log2 v per species (FP32 path)
    std::vector<double> R;     // max |g_k - h_k| over the temperature interval
    std::vector<double> lw;    // log2 W_k
    bool vfloat = false;       // v stored as float
};

Common common_setup(const JitMech &m, bool f64, JitProgram &prog)
{
    const int ns = m.ns;
    Common cm;
    std::vector<int> &h = cm.h;
    std::vector<double> &R = cm.R;
    std::vector<double> &lw = cm.lw;
    bool &vfloat = cm.vfloat;
    h.assign(ns, 0);
    R.assign(ns, 0.0);
    lw.assign(ns, 0.0);
    // FP32 path: v'_k = 2^-(g'_k - h_k) stored as float, with h_k an integer
    // shift that centres it over a temperature interval [T_lo, T_hi] on which
    // |g_k - h_k| <= 60 for every species (so that a product of two stays
    // well inside float range); the shifts of a reaction's reactants are
    // folded into its log2 A.  Cells outside the interval are reported as
    // bad.  If no interval containing 300-3000 K qualifies, v stays double.
    if (!f64) {
        const double cand[2][2] = {{200.0, 6000.0}, {300.0, 3000.0}};
        for (const auto &iv : cand) {
            bool ok = true;
            for (int k = 0; k < ns && ok; ++k) {
                double lo = 1e300, hi = -1e300;
                for (int i = 0; i <= 600; ++i) {
                    const double T = iv[0] * std::pow(iv[1] / iv[0], i / 600.0);
                    const double g = g2_host(m.sp[k], T) + std::log2(m.sp[k].inv_W);
                    lo = std::min(lo, g);
                    hi = std::max(hi, g);
                }
                // both sides of T_mid near the switch
                for (double T : {m.sp[k].T_mid, std::nextafter(m.sp[k].T_mid, 0.0)})
                    if (T >= iv[0] && T <= iv[1]) {
                        const double g = g2_host(m.sp[k], T) + std::log2(m.sp[k].inv_W);
                        lo = std::min(lo, g);
                        hi = std::max(hi, g);
                    }
                h[k] = (int)std::lround(0.5 * (lo + hi));
                R[k] = std::max(hi - h[k], h[k] - lo) + 0.5;   // margin for the grid
                ok = std::isfinite(lo) && std::isfinite(hi) && R[k] <= 60.0;
            }
            if (ok) {
                vfloat = true;
                prog.T_lo = iv[0];
                prog.T_hi = iv[1];
                break;
            }
        }
        if (!vfloat) std::fill(h.begin(), h.end(), 0);
    }
    // Species table of the generated kernel: the Gibbs-layer weights with
    // log2(1/W_k) added to the bias, so that 2^g'_k = 2^{g_k} / W_k and
    // a_k = C_k 2^{g_k} = rho_hat max(Y_k, 0) 2^{g'_k} needs no 1/W_k.
    // Then v_k = 2^{-g_k} = 2^{-(g'_k - h_k)} 2^{-(h_k + log2 W_k)}, whose
    // constant factor joins the reaction's Arrhenius bias.
    prog.sp.resize(16 * (size_t)ns);
    for (int k = 0; k < ns; ++k) {
        std::memcpy(&prog.sp[16 * k], &m.sp[k], sizeof(SpeciesRec));
        lw[k] = -std::log2(m.sp[k].inv_W);   // log2 W_k
        prog.sp[16 * k + 8] -= lw[k];         // lo bias
        prog.sp[16 * k + 15] -= lw[k];        // hi bias
    }
    return cm;
}

}  // namespace

namespace {

// ---------------------------------------------------------------------------
// pieces shared by both generated forms

bool is_falloff(const JitMech &m, int j)
{
    return m.pd && (m.pd[j].type == AK_RXN_LINDEMANN || m.pd[j].type == AK_RXN_TROE);
}
bool is_pdep(const JitMech &m, int j) { return m.pd && m.pd[j].type != AK_RXN_ELEMENTARY; }

// log2 of the constant factor between the stored v'_k and v_k = 2^-g_k:
// v_k = v'_k 2^-(h_k + log2 W_k); a reaction's log2 A absorbs the factors of
// its reactants
double reactant_shift(const JitMech &m, const Common &cm, int j)
{
    double s = 0.0;
    for (int i = 0; i < m.aux[j].nf; ++i) s += cm.h[m.aux[j].sp[i]] + cm.lw[m.aux[j].sp[i]];
    return s;
}

// Constants of reaction j in the generated kernels' table: log2 A (shifted),
// beta, -E/R log2 e; for falloff 8 more: log2 A0, beta0, -E0/R log2 e (low-
// pressure limit), the shift, Troe alpha, log2(e)/T3, log2(e)/T1,
// T2 log2(e).
void push_rx(std::vector<double> &rx, const JitMech &m, const Common &cm, int j)
{
    const double sh = reactant_shift(m, cm, j);
    rx.push_back(m.rx[j].log2A - sh);
    rx.push_back(m.rx[j].beta);
    rx.push_back(m.rx[j].negEoR2);
    if (is_falloff(m, j)) {
        const PdepRec &d = m.pd[j];
        rx.push_back(d.log2A0);
        rx.push_back(d.beta0);
        rx.push_back(d.negE0oR2);
        rx.push_back(sh);
        rx.push_back(d.alpha);
        rx.push_back(d.type == AK_RXN_TROE ? kLog2e / d.T3 : 0.0);
        rx.push_back(d.type == AK_RXN_TROE ? kLog2e / d.T1 : 0.0);
        rx.push_back(d.T2 * kLog2e);
    }
}
int rx_size(const JitMech &m, int j) { return is_falloff(m, j) ? 11 : 3; }

// scalar loads of reaction p's constants from rxp[off..]
void emit_loads(Text &o, const char *ind, const JitMech &m, int p, int j, int off)
{
    o("%sconst double kA%d = rxp[%d], kB%d = rxp[%d], kE%d = rxp[%d];\n", ind, p, off, p,
      off + 1, p, off + 2);
    if (is_falloff(m, j))
        o("%sconst double kA0%d = rxp[%d], kB0%d = rxp[%d], kE0%d = rxp[%d], kS%d = rxp[%d], "
          "kal%d = rxp[%d], ki3%d = rxp[%d], ki1%d = rxp[%d], kt2%d = rxp[%d];\n",
          ind, p, off + 3, p, off + 4, p, off + 5, p, off + 6, p, off + 7, p, off + 8, p,
          off + 9, p, off + 10);
}

// Third-body concentration of efficiency profile q (Sec. 2.4, [M] = C E):
// Ctot + sum over species with efficiency != 1 of (eff - 1) C_k, where
// C(k) spells C_k and Ctot = P / (Ru T) is in scope.  Declares M<q> and,
// with `log`, lM<q> = log2 [M].
void emit_profile(Text &o, const char *ind, const JitMech &m, int q, bool log, bool f64,
                  const std::function<std::string(int)> &C)
{
    const std::vector<double> &e = (*m.profiles)[q];
    o("%sdouble M%d = Ctot;\n", ind, q);
    for (int k = 0; k < m.ns; ++k)
        if (e[k] != 1.0) o("%sM%d = __builtin_fma(%s, %s, M%d);\n", ind, q, lit(e[k] - 1.0).c_str(),
                           C(k).c_str(), q);
    if (log && f64) o("%sconst double lM%d = log2(M%d);\n", ind, q, q);
    else if (log) o("%sconst double lM%d = (double)__builtin_amdgcn_logf((float)M%d);\n", ind, q, q);
}

// Names of the third-body concentration of reaction j's profile: M<q>,
// lM<q> (in scope from emit_profile), or, with `local`, the names that
// emit_rate declares inside the reaction's block.

// The rate of progress of reaction j at position p of the generated code:
// declares q<p> (accumulator type) from
//     q = 2^t prod_r v (prod_r a - rev prod_p a) [x [M] | x Pr/(1+Pr) F]
// (Eq. 4 re-associated with ln K_c = -sum_k nu_kj Gt_k, Eq. 11; the
// pressure dependence of Sec. 2.4).  A(k) and V(k) spell a_k and v_k; the
// reaction's constants (emit_loads) and the M / lM of its profile are in
// scope.
void emit_rate(Text &o, const char *ind, const JitMech &m, const Common &cm, bool f64, int p,
               int j, const std::function<std::string(int)> &A,
               const std::function<std::string(int)> &V,
               const std::function<std::string(int)> *C = nullptr)
{
    const RxnAux &x = m.aux[j];
    const int nf = x.nf, np = x.nr;
    const char *AC = f64 ? "double" : "float";
    std::string Vr;
    if (f64 || !cm.vfloat) {
        for (int i = 0; i < nf; ++i) Vr += (i ? "*" : "") + V(x.sp[i]);
    } else {
        // float v's are multiplied in float while the product stays in
        // range, the partial products in double
        double acc = 0.0;
        std::string grp;
        for (int i = 0; i < nf; ++i) {
            const int k = x.sp[i];
            if (!grp.empty() && acc + cm.R[k] > 120.0) {
                Vr += (Vr.empty() ? "(double)(" : "*(double)(") + grp + ")";
                grp.clear();
                acc = 0.0;
            }
            grp += (grp.empty() ? "" : "*") + V(k);
            acc += cm.R[k];
        }
        Vr += (Vr.empty() ? "(double)(" : "*(double)(") + grp + ")";
    }
    std::string Ar, Ap;
    for (int i = 0; i < nf; ++i) Ar += (i ? "*" : "") + A(x.sp[i]);
    for (int i = 0; i < np; ++i) Ap += (i ? "*" : "") + A(x.sp[nf + i]);
    // one scalar operand per instruction (the constants sit in SGPRs)
    o("%s%s q%d;\n%s{\n", ind, AC, p, ind);
    o("%s  const double t = __builtin_fma(kB%d, L2T, kE%d * IT) + kA%d;\n", ind, p, p, p);
    if (x.rev) o("%s  double X = (%s) * ((%s) - (%s));\n", ind, Vr.c_str(), Ar.c_str(), Ap.c_str());
    else o("%s  double X = (%s) * (%s);\n", ind, Vr.c_str(), Ar.c_str());
    if (is_pdep(m, j)) {
        const PdepRec &d = m.pd[j];
        // with C given, the reaction's own third-body concentration is formed
        // here (short register live ranges), else the profile's is in scope
        if (C) {
            const std::string in = std::string(ind) + "  ";
            emit_profile(o, in.c_str(), m, d.profile, is_falloff(m, j), f64, *C);
        }
        if (d.type == AK_RXN_THIRD_BODY) {
            o("%s  X *= M%d;\n", ind, d.profile);
        } else {
            // log2 Pr = log2 k0 - log2 k_inf + log2 [M] (the Arrhenius layer
            // also evaluates the low-pressure limit); the falloff function is
            // a per-reaction epilogue outside the matrix form (Sec. 2.4)
            o("%s  const double lp = (__builtin_fma(kB0%d, L2T, kE0%d * IT) + kA0%d) - t - kS%d + "
              "lM%d;\n", ind, p, p, p, p, d.profile);
            const char *FT = f64 ? "double" : "float";
            // FP32 path: the hardware exp2 / log2 (about 1 ulp; the
            // arguments stay in the normal range); FP64 path: the library's
            const char *EX = f64 ? "exp2" : "__builtin_amdgcn_exp2f";
            const char *LG = f64 ? "log2" : "__builtin_amdgcn_logf";
            o("%s  %s r = (%s)1 / ((%s)1 + %s((%s)-lp));\n", ind, FT, FT, FT, EX, FT);
            if (d.type == AK_RXN_TROE) {
                o("%s  %s Fc = ((%s)1 - (%s)kal%d) * %s((%s)(-T * ki3%d)) + (%s)kal%d * "
                  "%s((%s)(-T * ki1%d))%s;\n", ind, FT, FT, FT, p, EX, FT, p, FT, p, EX, FT, p,
                  d.T2 != 0.0 ? (std::string(" + ") + EX + "((" + FT + ")(-kt2" +
                                 std::to_string(p) + " * IT))").c_str() : "");
                // log10 Fc, c, n, then F (Troe's broadening)
                o("%s  const %s lFc = %s(Fc) * (%s)%s;\n", ind, FT, LG, FT,
                  lit(std::log10(2.0)).c_str());
                o("%s  const %s xc = (%s)lp * (%s)%s + ((%s)-0.4 - (%s)0.67 * lFc);\n", ind, FT,
                  FT, FT, lit(std::log10(2.0)).c_str(), FT, FT);
                o("%s  const %s f1 = xc / (((%s)0.75 - (%s)1.27 * lFc) - (%s)0.14 * xc);\n", ind,
                  FT, FT, FT, FT);
                o("%s  r *= %s(lFc / ((%s)1 + f1 * f1) * (%s)%s);\n", ind, EX, FT, FT,
                  lit(std::log2(10.0)).c_str());
            }
            o("%s  X *= (double)r;\n", ind);
        }
    }
    o("%s  q%d = qrate(X, t);\n", ind, p);
}

}  // namespace

JitProgram jit_program(const JitMech &m, bool f64)
{
    // reactions per scheduling group
    int group = 8;
    if (const char *g = std::getenv("AK_JIT_GROUP")) group = std::max(1, std::atoi(g));
    const int ns = m.ns, nr = m.nr;
    const char *IO = f64 ? "double" : "float";
    const char *AC = f64 ? "double" : "float";   // omega accumulator type
    JitProgram prog;
    prog.threads = 64;
    const Common cm = common_setup(m, f64, prog);
    const std::vector<int> &h = cm.h;
    const bool vfloat = cm.vfloat;
    const std::vector<std::vector<int>> rs = reaction_species(m);
    const std::vector<int> order = live_order(m, rs);
    std::vector<int> first(ns, -1), last(ns, -1);
    for (int p = 0; p < nr; ++p)
        for (int k : rs[order[p]]) {
            if (first[k] < 0) first[k] = p;
            last[k] = p;
        }
    // per-reaction constants in the order of the generated code, so that
    // consecutive reactions' constants are adjacent
    std::vector<int> off(nr + 1, 0);
    prog.rx.clear();
    for (int p = 0; p < nr; ++p) {
        off[p] = (int)prog.rx.size();
        push_rx(prog.rx, m, cm, order[p]);
    }
    const char *VT = (f64 || !vfloat) ? "double" : "float";

    Text o;
    o("// generated by libannkin for a mechanism of %d species and %d reactions (%s path, "
      "one lane per cell)\n", ns, nr, f64 ? "FP64" : "FP32");
    o("typedef long long i64;\ntypedef unsigned long long u64;\n");
    const std::vector<double> c = exp2_taylor(12);
    if (f64) {
        // X * 2^t, degree-12 polynomial for 2^f
        o("__device__ __forceinline__ double qrate(double X, double t) {\n");
        o("  const double n = __builtin_rint(t), f = t - n;\n");
        o("  double p = %s;\n", lit(c[12]).c_str());
        for (int k = 11; k >= 0; --k) o("  p = __builtin_fma(p, f, %s);\n", lit(c[k]).c_str());
        o("  return __builtin_ldexp(X * p, (int)n);\n}\n");
    } else {
        o("__device__ __forceinline__ float qrate(double X, double t) {\n");
        o("  const double n = __builtin_rint(t);\n");
        o("  const float p = __builtin_amdgcn_exp2f((float)(t - n));\n");
        o("  return (float)__builtin_ldexp(X, (int)n) * p;\n}\n");
    }
    // omega_k of this lane's cell.  The row offset passes through an empty
    // volatile asm at the store, so that the compiler forms it there rather
    // than keeping every row's address in scalar registers from the start.
    o("__device__ __forceinline__ void store(%s *__restrict__ Ob, i64 ldO, int k, unsigned lane, "
      "%s x) {\n  i64 off = (i64)k * ldO;\n  asm volatile(\"\" : \"+s\"(off));\n"
      "  (Ob + off)[lane] = x;\n}\n", IO, IO);
    // the cell body: Tb, Pb, Yb, Ob point at the tile's first cell
    o("__device__ __forceinline__ void body(const %s *__restrict__ Tb, const %s *__restrict__ Pb,"
      " const %s *__restrict__ Yb, i64 ldY, %s *__restrict__ Ob, i64 ldO, unsigned lane,"
      " const double *__restrict__ SP, const double *__restrict__ RX, u64 *err) {\n",
      IO, IO, IO, IO);
    o("  const double T = (double)Tb[lane], P = (double)Pb[lane];\n");
    for (int k = 0; k < ns; ++k) o("  const %s y%d = (Yb + (i64)%d * ldY)[lane];\n", IO, k, k);
    o("  const double LNT = log(T), IT = 1.0 / T, T2 = T * T, T3 = T2 * T, T4 = T3 * T;\n");
    o("  const double L2T = LNT * %s;\n", lit(kLog2e).c_str());
    // mixture sum (Y <= 0 counts as 0); a non-finite mass fraction makes
    // chk non-finite
    o("  %s chk = 0;\n  double sg = 0;\n", IO);
    for (int k = 0; k < ns; ++k)
        o("  chk += y%d;\n  sg += __builtin_fmax((double)y%d, 0.0) * SP[%d];\n", k, k, 16 * k);
    o("  const bool bad = !(T > 0.0) || !(P > 0.0) || !__builtin_isfinite(T) || "
      "!__builtin_isfinite(P) || !__builtin_isfinite(chk) || !(sg > 0.0) || "
      "!__builtin_isfinite(sg)");
    if (vfloat) o(" || !(T >= %s) || !(T <= %s)", lit(prog.T_lo).c_str(), lit(prog.T_hi).c_str());
    o(";\n");
    o("  const double rh = P / (%s * T * sg);\n", lit(kRu).c_str());
    std::map<double, int> tmid;
    for (int k = 0; k < ns; ++k)
        if (!tmid.count(m.sp[k].T_mid)) {
            const int id = (int)tmid.size();
            tmid[m.sp[k].T_mid] = id;
            o("  const bool hi%d = T >= %s;\n", id, lit(m.sp[k].T_mid).c_str());
        }
    o("  const %s nan = __builtin_nan(\"\");\n", IO);
    // third-body concentrations of the efficiency profiles (while every
    // mass fraction is at hand): C_k = rho_hat max(Y_k, 0) / W_k
    if (m.pd) {
        o("  const double Ctot = rh * sg;\n");
        std::vector<char> used(m.profiles->size(), 0), logd(m.profiles->size(), 0);
        for (int j = 0; j < nr; ++j)
            if (is_pdep(m, j)) {
                used[m.pd[j].profile] = 1;
                if (is_falloff(m, j)) logd[m.pd[j].profile] = 1;
            }
        for (size_t q = 0; q < used.size(); ++q)
            if (used[q])
                emit_profile(o, "  ", m, (int)q, logd[q], f64, [&](int k) {
                    return "(rh * __builtin_fmax((double)y" + std::to_string(k) + ", 0.0) * SP[" +
                           std::to_string(16 * k) + "])";
                });
    }

    // 2^f, |f| <= 1/2: degree 12 (below one ulp) in the FP64 path; degree 8
    // (relative error below 3e-10) in the FP32 path
    const int pdeg = f64 ? 12 : 8;
    auto open_species = [&](int k) {
        const int b = 16 * k;
        auto poly = [&](int off) {
            // one scalar operand per instruction: the bias is added last
            char buf[512];
            snprintf(buf, sizeof buf,
                     "(__builtin_fma(spp[%d], LNT, __builtin_fma(spp[%d], T, "
                     "__builtin_fma(spp[%d], T2, __builtin_fma(spp[%d], T3, "
                     "__builtin_fma(spp[%d], T4, spp[%d] * IT))))) + spp[%d])",
                     b + off, b + off + 1, b + off + 2, b + off + 3, b + off + 4, b + off + 5,
                     b + off + 6);
            return std::string(buf);
        };
        o("  double a%d; %s v%d; %s w%d = 0;\n  {\n", k, VT, k, AC, k);
        // both ranges are evaluated and one is selected per lane; the empty
        // asm keeps the compiler from turning the select of the two
        // polynomials into a select of their coefficient addresses (which
        // would make the table reads per-lane vector loads) or into a branch
        o("    double glo = %s, ghi = %s;\n", poly(2).c_str(), poly(9).c_str());
        o("    asm(\"\" : \"+v\"(glo), \"+v\"(ghi));\n");
        o("    const double g = hi%d ? ghi : glo;\n", tmid[m.sp[k].T_mid]);
        // 2^g and 2^-g from the even and odd parts of one Taylor polynomial
        o("    const double n = __builtin_rint(g), f = g - n, f2 = f * f;\n");
        const int top_even = pdeg - (pdeg & 1), top_odd = (pdeg & 1) ? pdeg : pdeg - 1;
        o("    double E = %s;\n", lit(c[top_even]).c_str());
        for (int q = top_even - 2; q >= 0; q -= 2)
            o("    E = __builtin_fma(E, f2, %s);\n", lit(c[q]).c_str());
        o("    double O = %s;\n", lit(c[top_odd]).c_str());
        for (int q = top_odd - 2; q >= 1; q -= 2)
            o("    O = __builtin_fma(O, f2, %s);\n", lit(c[q]).c_str());
        o("    O *= f;\n    const int ni = (int)n;\n");
        // y passes through an empty asm so that the compiler does not keep
        // the mixture sum's converted copy of it live until here
        o("    %s yy = y%d;\n    asm(\"\" : \"+v\"(yy));\n", IO, k);
        o("    a%d = rh * __builtin_fmax((double)yy, 0.0) * __builtin_ldexp(E + O, ni);\n", k);
        if (f64 || !vfloat) o("    v%d = __builtin_ldexp(E - O, -ni);\n", k);
        else o("    v%d = (float)__builtin_ldexp(E - O, %d - ni);\n", k, h[k]);
        o("  }\n");
    };

    // species in no reaction: omega = 0
    for (int k = 0; k < ns; ++k)
        if (first[k] < 0) o("  store(Ob, ldO, %d, lane, bad ? nan : (%s)0);\n", k, IO);

    // The reactions are emitted in groups, separated by scheduling fences.
    // The group's table reads go through a pointer that an empty asm derives
    // from the previous group's last rate, so that they cannot move ahead of
    // it (left alone, the compiler reads every reaction's and species'
    // constants at the kernel entry and spills them); the next group's
    // constants are read one group ahead.  The pointers are in the constant
    // address space, so that the reads stay scalar.
    const int ngroups = (nr + group - 1) / group;
    auto load_group = [&](int g) {
        for (int p = g * group; p < std::min(nr, (g + 1) * group); ++p)
            emit_loads(o, "  ", m, p, order[p], off[p]);
    };
    o("  const __attribute__((address_space(4))) double *rxp = "
      "(const __attribute__((address_space(4))) double *)RX;\n"
      "  const __attribute__((address_space(4))) double *spp = "
      "(const __attribute__((address_space(4))) double *)SP;\n");
    load_group(0);
    auto A = [](int k) { return "a" + std::to_string(k); };
    auto V = [](int k) { return "v" + std::to_string(k); };
    for (int p = 0; p < nr; ++p) {
        const int j = order[p];
        const RxnAux &x = m.aux[j];
        const int nf = x.nf, np = x.nr;
        const int g = p / group;
        if (p % group == 0) {
            if (p > 0) o("  asm volatile(\"\" : \"+s\"(rxp), \"+s\"(spp) : \"v\"(q%d));\n", p - 1);
            if (g + 1 < ngroups) load_group(g + 1);
        }
        for (int k : rs[j])
            if (first[k] == p) open_species(k);
        emit_rate(o, "  ", m, cm, f64, p, j, A, V);
        o("    const %s q = q%d;\n", AC, p);
        // net coefficient of each species in this reaction (Eq. 2)
        for (int k : rs[j]) {
            int nu = 0;
            for (int i = 0; i < nf + np; ++i)
                if (x.sp[i] == k) nu += i < nf ? -1 : 1;
            if (nu == 1) o("    w%d += q;\n", k);
            else if (nu == -1) o("    w%d -= q;\n", k);
            else if (nu != 0)
                o("    w%d = %s((%s)%d, q, w%d);\n", k, f64 ? "__builtin_fma" : "__builtin_fmaf",
                  AC, nu, k);
        }
        o("  }\n");
        for (int k : rs[j])
            if (last[k] == p) o("  store(Ob, ldO, %d, lane, bad ? nan : (%s)w%d);\n", k, IO, k);
        if ((p + 1) % group == 0 || p + 1 == nr) o("  __builtin_amdgcn_sched_barrier(0);\n");
    }
    o("  if (bad) atomicAdd(err, 1ull);\n}\n");

    o("struct BD { const void *T, *P, *Y; void *om; i64 ldY, ldO, n, block_begin; };\n");
    o("extern \"C\" __global__ __launch_bounds__(64) void ak_src(const %s *__restrict__ T, "
      "const %s *__restrict__ P, const %s *__restrict__ Y, i64 ldY, i64 n, %s *__restrict__ om, "
      "i64 ldO, const double *__restrict__ SP, const double *__restrict__ RX, u64 *err) {\n",
      IO, IO, IO, IO);
    o("  const i64 c0 = (i64)blockIdx.x * 64;\n  const unsigned lane = threadIdx.x;\n");
    o("  if (c0 + lane >= n) return;\n");
    o("  body(T + c0, P + c0, Y + c0, ldY, om + c0, ldO, lane, SP, RX, err);\n}\n");
    o("extern \"C\" __global__ __launch_bounds__(64) void ak_src_batch(const BD *__restrict__ d, "
      "int nreq, const double *__restrict__ SP, const double *__restrict__ RX, u64 *err) {\n");
    o("  const i64 b = blockIdx.x;\n  int lo = 0, hi = nreq - 1;\n");
    o("  while (lo < hi) { const int mid = (lo + hi + 1) >> 1; "
      "if (d[mid].block_begin <= b) lo = mid; else hi = mid - 1; }\n");
    o("  const BD r = d[lo];\n  const i64 c0 = (b - r.block_begin) * 64;\n");
    o("  const unsigned lane = threadIdx.x;\n  if (c0 + lane >= r.n) return;\n");
    o("  body((const %s *)r.T + c0, (const %s *)r.P + c0, (const %s *)r.Y + c0, r.ldY, "
      "(%s *)r.om + c0, r.ldO, lane, SP, RX, err);\n}\n",
      IO, IO, IO, IO);
    prog.src = std::move(o.s);
    return prog;
}

// ---------------------------------------------------------------------------
// tiled form

namespace {

// Reactions split over the waves of a tile: each reaction goes to one of the
// waves whose estimated work is within a small slack of the least loaded,
// preferring the wave that already touches most of its species (fewer
// accumulators to reduce afterwards); then each wave's list is ordered so
// that consecutive reactions share species.
std::vector<std::vector<int>> split_reactions(const JitMech &m,
                                              const std::vector<std::vector<int>> &rs, int W)
{
    const int nr = m.nr;
    std::vector<double> cost(nr);
    double total = 0.0;
    for (int j = 0; j < nr; ++j) {
        cost[j] = 14.0 + 2.0 * (m.aux[j].nf + m.aux[j].nr) + 2.0 * rs[j].size();
        total += cost[j];
    }
    std::vector<double> load(W, 0.0);
    std::vector<std::vector<char>> touch(W, std::vector<char>(m.ns, 0));
    std::vector<std::vector<int>> part(W);
    const double slack = 2.0 * total / nr;
    for (int j = 0; j < nr; ++j) {
        const double lmin = *std::min_element(load.begin(), load.end());
        int best = -1, bov = -1;
        for (int w = 0; w < W; ++w) {
            if (load[w] > lmin + slack) continue;
            int ov = 0;
            for (int k : rs[j]) ov += touch[w][k];
            if (ov > bov || (ov == bov && load[w] < load[best])) {
                best = w;
                bov = ov;
            }
        }
        part[best].push_back(j);
        load[best] += cost[j];
        for (int k : rs[j]) touch[best][k] = 1;
    }
    // chain within each wave: next = the remaining reaction sharing most
    // species with the previous one (ties: list order)
    for (auto &pl : part) {
        std::vector<int> out;
        std::vector<char> used(pl.size(), 0);
        int prev = -1;
        for (size_t step = 0; step < pl.size(); ++step) {
            int bi = -1, bs = -1;
            for (size_t i = 0; i < pl.size(); ++i) {
                if (used[i]) continue;
                int sh = 0;
                if (prev >= 0)
                    for (int k : rs[pl[i]])
                        sh += std::find(rs[prev].begin(), rs[prev].end(), k) != rs[prev].end();
                if (sh > bs) {
                    bs = sh;
                    bi = (int)i;
                }
            }
            used[bi] = 1;
            prev = pl[bi];
            out.push_back(prev);
        }
        pl = out;
    }
    return part;
}

}  // namespace

JitProgram jit_program_tile(const JitMech &m, bool f64, int W)
{
    // reactions per scheduling group (measured best: 4 FP32, 3 FP64)
    int group = f64 ? 3 : 4;
    if (const char *g = std::getenv("AK_JIT_GROUP")) group = std::max(1, std::atoi(g));
    const bool ahead = !std::getenv("AK_JIT_PREFETCH") || std::atoi(std::getenv("AK_JIT_PREFETCH"));
    auto knob = [](const char *name, int def) {
        const char *v = std::getenv(name);
        return v ? std::atoi(v) : def;
    };
    const bool lsalias = knob("AK_JIT_LSALIAS", 1) != 0;
    const bool tree = knob("AK_JIT_TREE", 1) != 0;
    const int ns = m.ns, nr = m.nr;
    const char *IO = f64 ? "double" : "float";
    const char *AC = f64 ? "double" : "float";   // omega accumulator type
    JitProgram prog;
    prog.threads = 64 * W;
    const Common cm = common_setup(m, f64, prog);
    const std::vector<int> &h = cm.h;
    const bool vfloat = cm.vfloat;
    const char *VT = (f64 || !vfloat) ? "double" : "float";
    // waves per SIMD the kernel is built for: as many tiles as the LDS holds
    // (W waves each), within what the registers allow (one accumulator per
    // species, two registers each in the FP64 path, plus about 48 others)
    const size_t lds = (size_t)64 * ns * (8 + ((f64 || !vfloat) ? 8 : 4)) +
                       (lsalias ? 0 : (size_t)64 * W * (8 + (f64 ? 8 : 4)));
    const int tiles = std::max<int>(1, (int)(163840 / lds));
    const int wpe_lds = std::max(1, tiles * W / 4);
    const int wpe_reg = std::max(1, 512 / ((f64 ? 2 : 1) * ns + (m.pd ? 80 : 48)));
    const int wpe = knob(f64 ? "AK_JIT_WPE64" : "AK_JIT_WPE", std::min(wpe_lds, wpe_reg));

    const std::vector<std::vector<int>> rs = reaction_species(m);
    const std::vector<std::vector<int>> part = split_reactions(m, rs, W);
    // species owned by each wave (loads, the species layer, the stores)
    std::vector<std::vector<int>> own(W);
    for (int k = 0; k < ns; ++k) own[k % W].push_back(k);
    const int maxown = (ns + W - 1) / W;
    // the first wave (in the reduction order 0..W-1) that touches species k
    std::vector<int> first_w(ns, -1);
    for (int w = 0; w < W; ++w)
        for (int j : part[w])
            for (int k : rs[j])
                if (first_w[k] < 0 || first_w[k] > w) first_w[k] = w;
    // per-reaction constants in the order of the generated code: each
    // wave's segment, offsets within it
    std::vector<int> rxoff(W + 1, 0);
    std::vector<std::vector<int>> off(W);
    prog.rx.clear();
    for (int w = 0; w < W; ++w) {
        rxoff[w] = (int)prog.rx.size();
        for (int j : part[w]) {
            off[w].push_back((int)prog.rx.size() - rxoff[w]);
            push_rx(prog.rx, m, cm, j);
        }
    }
    rxoff[W] = (int)prog.rx.size();

    Text o;
    o("// generated by libannkin for a mechanism of %d species and %d reactions (%s path, "
      "%d waves per 64-cell tile)\n", ns, nr, f64 ? "FP64" : "FP32", W);
    o("typedef long long i64;\ntypedef unsigned long long u64;\n");
    const std::vector<double> c = exp2_taylor(12);
    if (f64) {
        o("__device__ __forceinline__ double qrate(double X, double t) {\n");
        o("  const double n = __builtin_rint(t), f = t - n;\n");
        o("  double p = %s;\n", lit(c[12]).c_str());
        for (int k = 11; k >= 0; --k) o("  p = __builtin_fma(p, f, %s);\n", lit(c[k]).c_str());
        o("  return __builtin_ldexp(X * p, (int)n);\n}\n");
    } else {
        o("__device__ __forceinline__ float qrate(double X, double t) {\n");
        o("  const double n = __builtin_rint(t);\n");
        o("  const float p = __builtin_amdgcn_exp2f((float)(t - n));\n");
        o("  return (float)__builtin_ldexp(X, (int)n) * p;\n}\n");
    }
    // LDS of a tile: a (double) and v per species and cell; after the sweep
    // the a area holds the accumulated rates
    o("__device__ __forceinline__ void tile(i64 c0, i64 n, const %s *__restrict__ Tg, "
      "const %s *__restrict__ Pg, const %s *__restrict__ Yg, i64 ldY, %s *__restrict__ Og, "
      "i64 ldO, const double *__restrict__ SP, const double *__restrict__ RX, u64 *err, "
      "double *LA, %s *LV, double *LS, %s *LC) {\n", IO, IO, IO, IO, VT, IO);
    o("  const unsigned lane = threadIdx.x & 63u;\n");
    o("  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));\n");
    o("  const bool live = c0 + (i64)lane < n;\n");
    o("  const i64 ci = live ? c0 + (i64)lane : n - 1;\n");
    o("  const double T = (double)Tg[ci], P = (double)Pg[ci];\n");
    o("  const double LNT = log(T), IT = 1.0 / T, T2 = T * T, T3 = T2 * T, T4 = T3 * T;\n");
    o("  const double L2T = LNT * %s;\n", lit(kLog2e).c_str());
    // phase 1: each wave loads its own species, partial mixture sums
    o("  %s ys[%d];\n  double sgp = 0;\n  %s chk = 0;\n", IO, maxown, IO);
    for (int w = 0; w < W; ++w) {
        o("  %sif (wave == %d) {\n", w ? "else " : "", w);
        for (size_t i = 0; i < own[w].size(); ++i)
            o("    ys[%d] = (Yg + (i64)%d * ldY)[ci];\n", (int)i, own[w][i]);
        for (size_t i = 0; i < own[w].size(); ++i)
            o("    chk += ys[%d];\n    sgp += __builtin_fmax((double)ys[%d], 0.0) * SP[%d];\n",
              (int)i, (int)i, 16 * own[w][i]);
        o("  }\n");
    }
    o("  LS[threadIdx.x] = sgp;\n  LC[threadIdx.x] = chk;\n  __syncthreads();\n");
    o("  double sg = LS[lane];\n  %s chkt = LC[lane];\n", IO);
    for (int w = 1; w < W; ++w) o("  sg += LS[%d + lane];\n  chkt += LC[%d + lane];\n", 64 * w, 64 * w);
    o("  const bool bad = !(T > 0.0) || !(P > 0.0) || !__builtin_isfinite(T) || "
      "!__builtin_isfinite(P) || !__builtin_isfinite(chkt) || !(sg > 0.0) || "
      "!__builtin_isfinite(sg)");
    if (vfloat) o(" || !(T >= %s) || !(T <= %s)", lit(prog.T_lo).c_str(), lit(prog.T_hi).c_str());
    o(";\n");
    o("  const double rh = P / (%s * T * sg);\n", lit(kRu).c_str());
    if (m.pd) o("  const double Ctot = rh * sg;\n");
    if (lsalias) o("  __syncthreads();\n");
    std::map<double, int> tmid;
    for (int k = 0; k < ns; ++k)
        if (!tmid.count(m.sp[k].T_mid)) {
            const int id = (int)tmid.size();
            tmid[m.sp[k].T_mid] = id;
            o("  const bool hi%d = T >= %s;\n", id, lit(m.sp[k].T_mid).c_str());
        }
    // phase 2: the species layer of each wave's own species into LDS
    // 2^f, |f| <= 1/2: degree 12 (below one ulp) in the FP64 path; degree 8
    // (relative error below 3e-10) in the FP32 path
    const int pdeg = f64 ? 12 : knob("AK_JIT_EXPDEG", 8);
    const int top_even = pdeg - (pdeg & 1), top_odd = (pdeg & 1) ? pdeg : pdeg - 1;
    for (int w = 0; w < W; ++w) {
        o("  %sif (wave == %d) {\n", w ? "else " : "", w);
        for (size_t i = 0; i < own[w].size(); ++i) {
            const int k = own[w][i], b = 16 * k;
            auto poly = [&](int off) {
                char buf[512];
                // one scalar operand per instruction: the bias is added last
                snprintf(buf, sizeof buf,
                         "(__builtin_fma(SP[%d], LNT, __builtin_fma(SP[%d], T, "
                         "__builtin_fma(SP[%d], T2, __builtin_fma(SP[%d], T3, "
                         "__builtin_fma(SP[%d], T4, SP[%d] * IT))))) + SP[%d])",
                         b + off, b + off + 1, b + off + 2, b + off + 3, b + off + 4,
                         b + off + 5, b + off + 6);
                return std::string(buf);
            };
            o("    {\n      double glo = %s, ghi = %s;\n", poly(2).c_str(), poly(9).c_str());
            o("      asm(\"\" : \"+v\"(glo), \"+v\"(ghi));\n");
            o("      const double g = hi%d ? ghi : glo;\n", tmid[m.sp[k].T_mid]);
            o("      const double nn = __builtin_rint(g), f = g - nn, f2 = f * f;\n");
            o("      double E = %s;\n", lit(c[top_even]).c_str());
            for (int q = top_even - 2; q >= 0; q -= 2)
                o("      E = __builtin_fma(E, f2, %s);\n", lit(c[q]).c_str());
            o("      double O = %s;\n", lit(c[top_odd]).c_str());
            for (int q = top_odd - 2; q >= 1; q -= 2)
                o("      O = __builtin_fma(O, f2, %s);\n", lit(c[q]).c_str());
            o("      O *= f;\n      const int ni = (int)nn;\n");
            o("      LA[%d + lane] = rh * __builtin_fmax((double)ys[%d], 0.0) * "
              "__builtin_ldexp(E + O, ni);\n", 64 * k, (int)i);
            if (f64 || !vfloat) o("      LV[%d + lane] = __builtin_ldexp(E - O, -ni);\n", 64 * k);
            else o("      LV[%d + lane] = (float)__builtin_ldexp(E - O, %d - ni);\n", 64 * k, h[k]);
            o("    }\n");
        }
        o("  }\n");
    }
    o("  __syncthreads();\n");
    // phase 3: each wave sweeps its reactions, rates accumulated in registers
    for (int k = 0; k < ns; ++k) o("  %s w%d = 0;\n", AC, k);
    for (int w = 0; w < W; ++w) {
        const std::vector<int> &pl = part[w];
        o("  %sif (wave == %d) {\n", w ? "else " : "", w);
        // the constants are read through a constant-address-space pointer, so
        // that the loads stay scalar after the pointer passes the asm fences
        o("    const __attribute__((address_space(4))) double *rxp = "
          "(const __attribute__((address_space(4))) double *)(RX + %d);\n"
          "    unsigned la8 = lane * 8u, lv8 = lane * (unsigned)sizeof(*LV);\n", rxoff[w]);
        const int cnt = (int)pl.size();
        const int ngroups = (cnt + group - 1) / group;
        std::vector<char> seen(ns, 0);
        // byte offsets passed through the group fences, so that each read
        // is a base register plus an immediate offset
        auto A = [&](int k) {
            return "*(const double *)((const char *)LA + la8 + " + std::to_string(512 * k) + ")";
        };
        auto V = [&](int k) {
            return std::string("*(const ") + VT + " *)((const char *)LV + lv8 + " +
                   std::to_string(64 * k * ((f64 || !vfloat) ? 8 : 4)) + ")";
        };
        // concentrations for third-body sums: C_k = a_k v_k 2^-(h_k + log2 W_k)
        const std::function<std::string(int)> Cf = [&](int k) {
            return "(" + A(k) + " * (double)" + V(k) + " * " +
                   lit(std::exp2(-(cm.h[k] + cm.lw[k]))) + ")";
        };
        auto load_group = [&](int g) {
            for (int p = g * group; p < std::min(cnt, (g + 1) * group); ++p)
                emit_loads(o, "    ", m, p, pl[p], off[w][p]);
        };
        if (ahead) load_group(0);
        for (int p = 0; p < cnt; ++p) {
            const int j = pl[p];
            const RxnAux &x = m.aux[j];
            const int nf = x.nf, np = x.nr;
            if (p % group == 0) {
                if (p > 0)
                    o("    asm volatile(\"\" : \"+s\"(rxp), \"+v\"(la8), \"+v\"(lv8) : \"v\"(q%d));\n",
                      p - 1);
                if (!ahead) load_group(p / group);
                else if (p / group + 1 < ngroups) load_group(p / group + 1);
            }
            emit_rate(o, "    ", m, cm, f64, p, j, A, V, &Cf);
            o("      const %s q = q%d;\n", AC, p);
            for (int k : rs[j]) {
                int nu = 0;
                for (int i = 0; i < nf + np; ++i)
                    if (x.sp[i] == k) nu += i < nf ? -1 : 1;
                if (nu == 0) continue;
                if (!seen[k]) {
                    // first term of this wave's sum for species k
                    if (nu == 1) o("      w%d = q;\n", k);
                    else if (nu == -1) o("      w%d = -q;\n", k);
                    else o("      w%d = (%s)%d * q;\n", k, AC, nu);
                    seen[k] = 1;
                } else if (nu == 1) o("      w%d += q;\n", k);
                else if (nu == -1) o("      w%d -= q;\n", k);
                else
                    o("      w%d = %s((%s)%d, q, w%d);\n", k,
                      f64 ? "__builtin_fma" : "__builtin_fmaf", AC, nu, k);
            }
            o("    }\n");
            if ((p + 1) % group == 0 || p + 1 == cnt) o("    __builtin_amdgcn_sched_barrier(0);\n");
        }
        o("  }\n");
    }
    o("  __syncthreads();\n");
    // phase 4: the waves' rates added in wave order into the a area
    o("  %s *LW = (%s *)LA;\n", AC, AC);
    std::vector<std::vector<char>> tw(W, std::vector<char>(ns, 0));
    for (int w = 0; w < W; ++w)
        for (int j : part[w])
            for (int k : rs[j]) tw[w][k] = 1;
    // fixed summation order per species: ((w0 + w1) + (w2 + w3)) for the tree,
    // (((w0 + w1) + w2) + w3) for the chain; untouched terms are left out
    std::vector<std::string> omega_expr(ns);
    if (tree && W == 4) {
        // two buffers: B0 (waves 0 + 1) at the start of the a area, B1 (waves
        // 2 + 3) after it in the FP32 path (floats take half of it) and in
        // the v area in the FP64 path (v is double there)
        const std::string lw1 = f64 ? "(double *)LV" : "LW + " + std::to_string(64 * ns);
        o("  %s *LW1 = %s;\n", AC, lw1.c_str());
        auto B = [&](int b, int k) {
            return std::string(b ? "LW1[" : "LW[") + std::to_string(64 * k) + " + lane]";
        };
        for (int half = 0; half < 2; ++half) {
            o("  if (wave == %d) {\n", 2 * half);
            for (int k = 0; k < ns; ++k)
                if (tw[2 * half][k]) o("    %s = w%d;\n", B(half, k).c_str(), k);
            o("  }\n");
        }
        o("  __syncthreads();\n");
        for (int half = 0; half < 2; ++half) {
            o("  if (wave == %d) {\n", 2 * half + 1);
            for (int k = 0; k < ns; ++k)
                if (tw[2 * half + 1][k])
                    o("    %s %s w%d;\n", B(half, k).c_str(), tw[2 * half][k] ? "+=" : "=", k);
            o("  }\n");
        }
        o("  __syncthreads();\n");
        for (int k = 0; k < ns; ++k) {
            const bool h0 = tw[0][k] || tw[1][k], h1 = tw[2][k] || tw[3][k];
            if (h0 && h1) omega_expr[k] = "(" + B(0, k) + " + " + B(1, k) + ")";
            else if (h0) omega_expr[k] = B(0, k);
            else if (h1) omega_expr[k] = B(1, k);
            else omega_expr[k] = "0";
        }
    } else {
        for (int w = 0; w < W; ++w) {
            o("  if (wave == %d) {\n", w);
            for (int k = 0; k < ns; ++k)
                if (tw[w][k])
                    o("    LW[%d + lane] %s w%d;\n", 64 * k, first_w[k] == w ? "=" : "+=", k);
            o("  }\n  __syncthreads();\n");
        }
        for (int k = 0; k < ns; ++k)
            omega_expr[k] = first_w[k] >= 0 ? "LW[" + std::to_string(64 * k) + " + lane]" : "0";
    }
    // phase 5: each wave stores its own species
    o("  if (live) {\n");
    for (int w = 0; w < W; ++w) {
        o("    %sif (wave == %d) {\n", w ? "else " : "", w);
        for (int k : own[w])
            o("      Og[(i64)%d * ldO + c0 + lane] = bad ? (%s)__builtin_nan(\"\") : (%s)(%s);\n",
              k, IO, IO, omega_expr[k].c_str());
        o("    }\n");
    }
    o("    if (wave == 0 && bad) atomicAdd(err, 1ull);\n  }\n}\n");

    o("struct BD { const void *T, *P, *Y; void *om; i64 ldY, ldO, n, block_begin; };\n");
    if (lsalias) {
        // the mixture-sum partials live in the v area until the species layer
        // writes it (a barrier separates the two)
        const size_t vbytes = (size_t)64 * ns * (f64 || !vfloat ? 8 : 4);
        const size_t need = (size_t)64 * W * 8 + (size_t)64 * W * (f64 ? 8 : 4);
        o("#define AK_TILE_LDS __shared__ double LA[%d]; __shared__ double LVD[%d]; "
          "%s *LV = (%s *)LVD; double *LS = LVD; %s *LC = (%s *)(LVD + %d);\n", 64 * ns,
          (int)((std::max(vbytes, need) + 7) / 8), VT, VT, IO, IO, 64 * W);
    } else {
        o("#define AK_TILE_LDS __shared__ double LA[%d]; __shared__ %s LV[%d]; "
          "__shared__ double LS[%d]; __shared__ %s LC[%d];\n", 64 * ns, VT, 64 * ns, 64 * W, IO,
          64 * W);
    }
    o("extern \"C\" __global__ __launch_bounds__(%d) __attribute__((amdgpu_waves_per_eu(%d))) "
      "void ak_src(const %s *__restrict__ T, const %s *__restrict__ P, "
      "const %s *__restrict__ Y, i64 ldY, i64 n, %s *__restrict__ om, i64 ldO, "
      "const double *__restrict__ SP, const double *__restrict__ RX, u64 *err) {\n",
      64 * W, wpe, IO, IO, IO, IO);
    o("  AK_TILE_LDS\n  tile((i64)blockIdx.x * 64, n, T, P, Y, ldY, om, ldO, SP, RX, err, "
      "LA, LV, LS, LC);\n}\n");
    o("extern \"C\" __global__ __launch_bounds__(%d) __attribute__((amdgpu_waves_per_eu(%d))) "
      "void ak_src_batch(const BD *__restrict__ d, int nreq, const double *__restrict__ SP, "
      "const double *__restrict__ RX, u64 *err) {\n", 64 * W, wpe);
    o("  AK_TILE_LDS\n  const i64 b = blockIdx.x;\n  int lo = 0, hi = nreq - 1;\n");
    o("  while (lo < hi) { const int mid = (lo + hi + 1) >> 1; "
      "if (d[mid].block_begin <= b) lo = mid; else hi = mid - 1; }\n");
    o("  const BD r = d[lo];\n");
    o("  tile((b - r.block_begin) * 64, r.n, (const %s *)r.T, (const %s *)r.P, "
      "(const %s *)r.Y, r.ldY, (%s *)r.om, r.ldO, SP, RX, err, LA, LV, LS, LC);\n}\n",
      IO, IO, IO, IO);
    prog.src = std::move(o.s);
    return prog;
}

JitProgram jit_generate(const JitMech &m, bool f64)
{
    // small mechanisms: the whole per-cell state in registers; larger ones:
    // the tiled form
    const char *mode = std::getenv("AK_JIT_MODE");
    bool lane = m.ns <= kLaneFormMaxSpecies;
    if (mode && std::strcmp(mode, "lane") == 0) lane = true;
    if (mode && std::strcmp(mode, "tile") == 0) lane = false;
    if (lane) return jit_program(m, f64);
    int waves = kTileWaves;
    if (const char *w = std::getenv(f64 ? "AK_JIT_WAVES64" : "AK_JIT_WAVES"))
        waves = std::max(1, std::min(16, std::atoi(w)));
    return jit_program_tile(m, f64, waves);
}

// ---------------------------------------------------------------------------
// compilation

namespace {

std::mutex g_cache_mu;
std::map<std::string, std::vector<char>> g_cache;   // source text -> code object

const char *const kOpts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17",
                             "-Xclang",              "-target-feature",
                             "-Xclang",              "-packed-fp32-ops"};

uint64_t fnv1a(const std::string &s, uint64_t h = 1469598103934665603ull)
{
    for (unsigned char ch : s) {
        h ^= ch;
        h *= 1099511628211ull;
    }
    return h;
}

// optional on-disk cache of code objects (AK_JIT_CACHE_DIR, else
// $HOME/.cache/annkin; "off" disables it)
std::string cache_path(const std::string &src, const std::vector<std::string> &extra)
{
    const char *dir = std::getenv("AK_JIT_CACHE_DIR");
    std::string d;
    if (dir && *dir) {
        if (std::strcmp(dir, "off") == 0) return "";
        d = dir;
    } else {
        const char *home = std::getenv("HOME");
        if (!home || !*home) return "";
        d = std::string(home) + "/.cache/annkin";
    }
    std::string key = src;
    for (const char *opt : kOpts) key += opt;
    for (const std::string &opt : extra) key += opt;
    int ver_major = 0, ver_minor = 0;
    hiprtcVersion(&ver_major, &ver_minor);
    key += std::to_string(ver_major) + "." + std::to_string(ver_minor);
    char name[64];
    snprintf(name, sizeof name, "/jit-%016llx.co", (unsigned long long)fnv1a(key));
    return d + name;
}

bool read_file(const std::string &p, std::vector<char> &out)
{
    FILE *f = std::fopen(p.c_str(), "rb");
    if (!f) return false;
    std::fseek(f, 0, SEEK_END);
    const long n = std::ftell(f);
    std::fseek(f, 0, SEEK_SET);
    bool ok = n > 0;
    if (ok) {
        out.resize(n);
        ok = std::fread(out.data(), 1, n, f) == (size_t)n;
    }
    std::fclose(f);
    return ok;
}

void write_file(const std::string &p, const std::vector<char> &data)
{
    const size_t slash = p.rfind('/');
    if (slash != std::string::npos) {
        // create the directory chain (ignore failures: the cache is optional)
        std::string dir = p.substr(0, slash);
        for (size_t i = 1; i <= dir.size(); ++i)
            if (i == dir.size() || dir[i] == '/') {
                std::string sub = dir.substr(0, i);
                (void)mkdir(sub.c_str(), 0755);
            }
    }
    char tmp_suffix[32];
    snprintf(tmp_suffix, sizeof tmp_suffix, ".tmp%d", (int)getpid());
    const std::string tmp = p + tmp_suffix;
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) return;
    const bool ok = std::fwrite(data.data(), 1, data.size(), f) == data.size();
    std::fclose(f);
    if (ok) std::rename(tmp.c_str(), p.c_str());
    else std::remove(tmp.c_str());
}

}  // namespace

int jit_compile(const std::string &src, std::vector<char> &code, std::string &log,
                const std::vector<std::string> &extra)
{
    std::string key = src;
    for (const std::string &opt : extra) key += "\n// " + opt;
    {
        std::lock_guard<std::mutex> l(g_cache_mu);
        auto it = g_cache.find(key);
        if (it != g_cache.end()) {
            code = it->second;
            return AK_OK;
        }
    }
    const std::string path = cache_path(src, extra);
    if (!path.empty() && read_file(path, code)) {
        std::lock_guard<std::mutex> l(g_cache_mu);
        g_cache[key] = code;
        return AK_OK;
    }
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "annkin_mechanism.hip", 0, nullptr, nullptr) !=
        HIPRTC_SUCCESS) {
        log = "hiprtcCreateProgram failed";
        return AK_EDEVICE;
    }
    std::vector<const char *> opts(std::begin(kOpts), std::end(kOpts));
    for (const std::string &opt : extra) opts.push_back(opt.c_str());
    const hiprtcResult r = hiprtcCompileProgram(prog, (int)opts.size(), opts.data());
    size_t ls = 0;
    if (hiprtcGetProgramLogSize(prog, &ls) == HIPRTC_SUCCESS && ls > 1) {
        std::vector<char> b(ls + 1, 0);
        if (hiprtcGetProgramLog(prog, b.data()) == HIPRTC_SUCCESS) log.assign(b.data());
    }
    if (r != HIPRTC_SUCCESS) {
        hiprtcDestroyProgram(&prog);
        if (log.empty()) log = hiprtcGetErrorString(r);
        return AK_EDEVICE;
    }
    size_t cs = 0;
    if (hiprtcGetCodeSize(prog, &cs) != HIPRTC_SUCCESS || cs == 0) {
        hiprtcDestroyProgram(&prog);
        log = "hiprtc produced no code";
        return AK_EDEVICE;
    }
    code.resize(cs);
    const hiprtcResult g = hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    if (g != HIPRTC_SUCCESS) {
        log = "hiprtcGetCode failed";
        return AK_EDEVICE;
    }
    if (!path.empty()) write_file(path, code);
    std::lock_guard<std::mutex> l(g_cache_mu);
    g_cache[key] = code;
    return AK_OK;
}

int jit_load(const std::vector<char> &code, JitKernels &out, const char *fn, const char *batch)
{
    hipError_t e = hipModuleLoadData(&out.mod, code.data());
    if (e != hipSuccess) return hip_error(e, "loading the mechanism's kernels");
    if ((e = hipModuleGetFunction(&out.src, out.mod, fn)) != hipSuccess ||
        (batch && (e = hipModuleGetFunction(&out.batch, out.mod, batch)) != hipSuccess)) {
        (void)hipModuleUnload(out.mod);
        out.mod = nullptr;
        return hip_error(e, "finding the mechanism's kernels");
    }
    out.block = 64;
    out.threads = 64;
    return AK_OK;
}

void jit_unload(JitKernels &k)
{
    if (k.mod) (void)hipModuleUnload(k.mod);
    k.mod = nullptr;
    k.src = k.batch = nullptr;
}

hipError_t jit_launch(const JitKernels &k, const void *T, const void *P, const void *Y,
                      int64_t ldY, int64_t n, void *om, int64_t ldO, unsigned long long *err,
                      hipStream_t st)
{
    const int64_t blocks = (n + k.block - 1) / k.block;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    const double *SP = k.sp, *RX = k.rx;
    void *args[] = {(void *)&T, (void *)&P,  (void *)&Y,  (void *)&ldY, (void *)&n,
                    (void *)&om, (void *)&ldO, (void *)&SP, (void *)&RX, (void *)&err};
    return hipModuleLaunchKernel(k.src, (unsigned)blocks, 1, 1, k.threads, 1, 1, 0, st, args,
                                 nullptr);
}

hipError_t jit_vjp_launch(const JitKernels &k, const void *T, const void *P, const void *Y,
                          int64_t ldY, int64_t n, const void *G, int64_t ldG, void *GY,
                          int64_t ldGY, void *GT, unsigned long long *err, hipStream_t st)
{
    const int64_t blocks = (n + k.block - 1) / k.block;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    const double *SP = k.sp, *RX = k.rx;
    void *args[] = {(void *)&T,  (void *)&P,    (void *)&Y,  (void *)&ldY, (void *)&n,
                    (void *)&G,  (void *)&ldG,  (void *)&GY, (void *)&ldGY, (void *)&GT,
                    (void *)&SP, (void *)&RX,   (void *)&err};
    return hipModuleLaunchKernel(k.src, (unsigned)blocks, 1, 1, k.threads, 1, 1, 0, st, args,
                                 nullptr);
}

hipError_t jit_batch_launch(const JitKernels &k, const JitBatchDesc *d_desc, int nreq,
                            int64_t blocks, unsigned long long *err, hipStream_t st)
{
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    const double *SP = k.sp, *RX = k.rx;
    void *args[] = {(void *)&d_desc, (void *)&nreq, (void *)&SP, (void *)&RX, (void *)&err};
    return hipModuleLaunchKernel(k.batch, (unsigned)blocks, 1, 1, k.threads, 1, 1, 0, st, args,
                                 nullptr);
}

}  // namespace ak
