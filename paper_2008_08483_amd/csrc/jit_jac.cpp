// The state Jacobian compiled for the mechanism.
//
// Rows omega_1..omega_NS (Eq. 2) and omega_T = -sum_k H_k omega_k /
// sum_k C_k cp_k (constant pressure); columns Y_1..Y_NS and T, at fixed P.
// With rho_hat = P / (Ru T sigma), sigma = sum_m max(Y_m, 0) / W_m and
// C_l = rho_hat max(Y_l, 0) / W_l,
//     dC_l / dY_c = f_c (rho_hat delta_lc - C_l / sigma),   f_c = [Y_c >= 0] / W_c
//     dC_l / dT   = -C_l / T
// so that, with G_kl = sum_j nu_kj dq_j / dC_l and (Euler's theorem for the
// mass-action products) sum_l G_kl C_l = sum_j nu_kj (n_f q_f - n_r q_r)_j:
//     J[k][c] = f_c (rho_hat G_kc - u_k / sigma),  u_k = sum_j nu_kj (n_f q_f - n_r q_r)_j
//     J[k][T] = sum_j nu_kj (dq_j/dT at fixed C - (n_f q_f - n_r q_r)_j / T)
// where dq_f/dT = q_f d ln k_f/dT (Arrhenius layer, Eq. 6) and dq_r/dT =
// q_r (d ln k_f/dT - d ln K_c/dT), d ln K_c/dT = (sum_k nu_k H_k/(R T) - dn)/T
// (Eq. 11 with the Gibbs layer's NASA-7 form).  The temperature row follows
// from the same sums weighted by dH_j = sum_k nu_kj H_k / (R T).
//
// The rates use the exact re-associated form of the source-term kernels,
// a_k = C_k exp(Gt_k), v_k = exp(-Gt_k), q_f = k_f prod_r v prod_r a,
// q_r = k_f prod_r v prod_p a; then dq_f/dC_l = k_f prod_r v w_l dA_f/da_l
// and dq_r/dC_l = k_f prod_r v w_l dA_p/da_l with w_l = exp(Gt_l).
//
// One 64-cell tile per workgroup (lane = cell), W waves.  The species values
// of the tile (a, v, w, H/RT and f) live in LDS.  Waves 0..WR-1 own
// contiguous blocks of rows: per row they walk the reactions that change the
// species and accumulate the row's nonzero columns in registers, then write
// the row.  The other waves walk all reactions once and accumulate the
// dH-weighted sums of the temperature row; the last of them writes it.  Every
// sum has a fixed order, so the result is bitwise reproducible.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <string>
#include <vector>

#include "annkin.h"
#include "ak_internal.h"
#include "ak_jit.h"
#include "jit_text.h"

namespace ak {

namespace {

constexpr int kJacWaves = 8;        // waves per tile
constexpr int kJacTempWaves = 2;    // of which build the temperature row
constexpr int kJacSpStride = 32;    // doubles per species in the table
constexpr int kJacRxStride = 4;     // doubles per reaction in the table

// molecule counts of species k on each side of reaction j
void side_counts(const JitMech &m, int j, int k, int &mf, int &mr)
{
    const RxnAux &x = m.aux[j];
    mf = mr = 0;
    for (int i = 0; i < x.nf; ++i) mf += x.sp[i] == k;
    for (int i = 0; i < x.nr; ++i) mr += x.sp[x.nf + i] == k;
}

// x * x * ... (p factors), "" for p == 0
std::string power(const std::string &x, int p)
{
    std::string s;
    for (int i = 0; i < p; ++i) s += (i ? " * " : "") + x;
    return s;
}

std::string times(const std::string &a, const std::string &b)
{
    if (a.empty()) return b;
    if (b.empty()) return a;
    return a + " * " + b;
}

// how the generated code spells the tile values of species k in a reaction
// block (locals declared by emit_jac_rxn)
std::string A(int k) { return "a_" + std::to_string(k); }
std::string V(int k) { return "v_" + std::to_string(k); }
std::string Wv(int k) { return "w_" + std::to_string(k); }
std::string H(int k) { return "h_" + std::to_string(k); }
std::string Gw(int k) { return "g_" + std::to_string(k); }

struct Lds {
    // LDS read of the value `q` (0 a, 1 v, 2 w, 3 h) of species k; the row
    // being built keeps its own species' values in registers
    int row = -1;
    std::string read(int q, int k) const
    {
        static const char *reg[4] = {"Ra", "Rv", "Rw", "Rh"};
        if (q == 4) {
            // the VJP's g_omega (in the place of the clamp flags)
            char b[64];
            snprintf(b, sizeof b, "LD(bf, %d)", 512 * k);
            return b;
        }
        if (k == row) return reg[q];
        // a and v' from the low base, w and h from the high one (two arrays
        // past it): every offset fits an LDS instruction's 16-bit immediate
        const char *base = q < 2 ? "bl" : "bh";
        char b[64];
        snprintf(b, sizeof b, "LD(%s, %d)", base, 512 * ((q & 1) * ns + k));
        return b;
    }
    int ns = 0;
};

// Derivatives of reaction j (position p of the wave's walk) at the lane's
// cell, as locals of the enclosing block: qf, qr, qn, uf (= n_f q_f - n_r
// q_r), dqT (= dq/dT at fixed Y), dH (= sum nu h, if `want_dH` or
// reversible), ga (= sum nu g_omega, if `want_gamma`), and for each species
// l of the reaction d<l> = |dq/dC_l| with sign s<l> (+1 / -1 / 0 when d<l>
// already carries its sign).
struct Deriv {
    std::vector<int> sp;      // species of the reaction
    std::vector<int> sign;    // sign of d<l> in dq/dC_l
};

Deriv emit_jac_rxn(Text &o, const char *ind, const JitMech &m, bool f64out, int p, int j,
                   const std::vector<int> &rsj, bool want_dH, const Lds &L,
                   bool want_gamma = false)
{
    const RxnAux &x = m.aux[j];
    const int nf = x.nf, np = x.nr;
    const bool rev = x.rev != 0;
    Deriv d;
    d.sp = rsj;
    std::vector<int> mf(rsj.size()), mr(rsj.size());
    for (size_t i = 0; i < rsj.size(); ++i) side_counts(m, j, rsj[i], mf[i], mr[i]);
    const bool need_h = want_dH || rev;
    // the tile values the reaction reads
    for (size_t i = 0; i < rsj.size(); ++i) {
        const int k = rsj[i];
        o("%sconst double %s = %s;\n", ind, A(k).c_str(), L.read(0, k).c_str());
        if (mf[i]) o("%sconst double %s = %s;\n", ind, V(k).c_str(), L.read(1, k).c_str());
        // w_l enters dq/dC_l of every species with a nonzero derivative
        const bool deriv = mf[i] || (rev && mr[i]);
        if (deriv) o("%sconst double %s = %s;\n", ind, Wv(k).c_str(), L.read(2, k).c_str());
        if (need_h && mf[i] != mr[i])
            o("%sconst double %s = %s;\n", ind, H(k).c_str(), L.read(3, k).c_str());
        if (want_gamma && mf[i] != mr[i])
            o("%sconst double %s = %s;\n", ind, Gw(k).c_str(), L.read(4, k).c_str());
    }
    if (want_gamma) {
        // the reaction's weight in the VJP: sum_k nu_kj g_omega_k
        std::string s;
        for (size_t i = 0; i < rsj.size(); ++i) {
            const int nu = mr[i] - mf[i];
            if (!nu) continue;
            if (s.empty()) s = nu == 1 ? Gw(rsj[i]) : nu == -1 ? "-" + Gw(rsj[i]) :
                               std::to_string(nu) + ".0 * " + Gw(rsj[i]);
            else s = "__builtin_fma(" + std::to_string(nu) + ".0, " + Gw(rsj[i]) + ", " + s + ")";
        }
        o("%sconst double ga = %s;\n", ind, s.empty() ? "0.0" : s.c_str());
    }
    // k_f prod_r v with the reactants' 1/W folded into the Arrhenius bias:
    // E' = 2^(t'), t' = log2 k_f - sum_r log2 W_r, and v' = W v
    o("%sconst double eIT = kE%d * IT;\n", ind, p);
    o("%sconst double t = __builtin_fma(kB%d, L2T, eIT) + kA%d;\n", ind, p, p);
    o("%sconst double Ep = ex2(t);\n", ind);
    std::string Vr, Af, Ap;
    for (size_t i = 0; i < rsj.size(); ++i) {
        Vr = times(Vr, power(V(rsj[i]), mf[i]));
        Af = times(Af, power(A(rsj[i]), mf[i]));
        Ap = times(Ap, power(A(rsj[i]), mr[i]));
    }
    o("%sconst double EV = Ep * (%s);\n", ind, Vr.c_str());
    o("%sconst double qf = EV * (%s);\n", ind, Af.c_str());
    if (rev) o("%sconst double qr = EV * (%s);\n", ind, Ap.c_str());
    else o("%sconst double qr = 0.0;\n", ind);
    o("%sconst double qn = qf - qr;\n", ind);
    if (!rev) o("%sconst double uf = %d.0 * qf;\n", ind, nf);
    else if (nf == np) o("%sconst double uf = %d.0 * qn;\n", ind, nf);
    else o("%sconst double uf = __builtin_fma(%d.0, qf, %d.0 * qr);\n", ind, nf, -np);
    // sum_k nu_k h_k (dH) and dlK = (dH - dn) / T
    if (need_h) {
        std::string s;
        for (size_t i = 0; i < rsj.size(); ++i) {
            const int nu = mr[i] - mf[i];
            if (!nu) continue;
            if (s.empty()) s = nu == 1 ? H(rsj[i]) : nu == -1 ? "-" + H(rsj[i]) :
                               std::to_string(nu) + ".0 * " + H(rsj[i]);
            else s = "__builtin_fma(" + std::to_string(nu) + ".0, " + H(rsj[i]) + ", " + s + ")";
        }
        if (s.empty()) s = "0.0";
        o("%sconst double dH = %s;\n", ind, s.c_str());
    }
    // dq/dT at fixed Y = q_n dlk + q_r dlK - uf / T with
    // dlk = (beta + (E/R)/T) / T, dlK = (dH - dn) / T
    o("%sconst double X = qn * IT;\n", ind);
    if (rev) {
        const int dn = np - nf;
        o("%sconst double dqT = __builtin_fma(kB%d, X, __builtin_fma(kR%d, X * IT, "
          "__builtin_fma(dH - %d.0, qr * IT, -uf * IT)));\n", ind, p, p, dn);
    } else {
        o("%sconst double dqT = __builtin_fma(kB%d, X, __builtin_fma(kR%d, X * IT, %d.0 * X));\n",
          ind, p, p, -nf);
    }
    // dq/dC_l = EV w_l (dA_f/da_l - rev dA_p/da_l)
    d.sign.assign(rsj.size(), 0);
    for (size_t i = 0; i < rsj.size(); ++i) {
        const int k = rsj[i];
        std::string dAf, dAp;
        const bool hf = mf[i] > 0, hr = rev && mr[i] > 0;
        if (!hf && !hr) continue;
        auto partial = [&](const std::vector<int> &mu) {
            // d/da_k of prod a^mu
            std::string s = mu[i] > 1 ? std::to_string(mu[i]) + ".0" : "";
            s = times(s, power(A(k), mu[i] - 1));
            for (size_t l = 0; l < rsj.size(); ++l)
                if (l != i) s = times(s, power(A(rsj[l]), mu[l]));
            return s;
        };
        if (hf) dAf = partial(mf);
        if (hr) dAp = partial(mr);
        const std::string Ew = "EV * " + Wv(k);
        if (hf && hr) {
            const std::string f = dAf.empty() ? "1.0" : dAf, r = dAp.empty() ? "1.0" : dAp;
            o("%sconst double d_%d = (%s) * (%s - %s);\n", ind, k, Ew.c_str(), f.c_str(), r.c_str());
            d.sign[i] = 2;   // signed
        } else {
            const std::string &s = hf ? dAf : dAp;
            o("%sconst double d_%d = (%s)%s%s;\n", ind, k, Ew.c_str(), s.empty() ? "" : " * ",
              s.c_str());
            d.sign[i] = hf ? 1 : -1;
        }
    }
    return d;
}

// accumulate coef * (sign * d) into acc
void accumulate(Text &o, const char *ind, const std::string &acc, int coef, int sign,
                const std::string &d)
{
    const int c = sign == 2 ? coef : coef * sign;
    if (c == 1) o("%s%s += %s;\n", ind, acc.c_str(), d.c_str());
    else if (c == -1) o("%s%s -= %s;\n", ind, acc.c_str(), d.c_str());
    else if (c != 0) o("%s%s = __builtin_fma(%d.0, %s, %s);\n", ind, acc.c_str(), c, d.c_str(),
                       acc.c_str());
}

// NASA-7 cp/R of species k at T: both ranges from scalar loads, then the one
// in use (selecting the values, not the addresses, keeps the loads scalar)
// (`ix` prefixes the table indices: "kz + " makes the loads vector loads)
void emit_cp(Text &o, const char *ind, const char *name, int k, const std::string &hiname,
             const char *ix = "")
{
    const int b = kJacSpStride * k;
    auto poly = [&](int off) {
        char s[400];
        snprintf(s, sizeof s,
                 "__builtin_fma(T, __builtin_fma(T, __builtin_fma(T, __builtin_fma(T, SP[%s%d], "
                 "SP[%s%d]), SP[%s%d]), SP[%s%d]), SP[%s%d])",
                 ix, b + off + 4, ix, b + off + 3, ix, b + off + 2, ix, b + off + 1, ix, b + off);
        return std::string(s);
    };
    o("%sdouble %s_l = %s, %s_h = %s;\n", ind, name, poly(16).c_str(), name, poly(23).c_str());
    o("%sasm(\"\" : \"+v\"(%s_l), \"+v\"(%s_h));\n", ind, name, name);
    o("%sconst double %s = %s ? %s_h : %s_l;\n", ind, name, hiname.c_str(), name, name);
}

}  // namespace

// doubles of the reaction-constant region (it first holds two per-wave
// partial sums of the mixture)
int jac_rx_doubles(int nr) { return std::max(kJacRxStride * nr, 2 * 64 * kJacWaves); }

size_t jac_lds_bytes(int ns, int nr)
{
    // a, v', w, h, f per species and cell; the reaction constants; three
    // per-wave partial sums
    return 8 * ((size_t)5 * 64 * ns + jac_rx_doubles(nr) + (size_t)3 * 64 * kJacWaves);
}

std::vector<std::string> jac_compile_options()
{
    const char *e = std::getenv("AK_JAC_SCHED");
    const std::string strat = e && *e ? e : "max-ilp";
    if (strat == "default") return {};
    return {"-mllvm", "-amdgpu-sched-strategy=" + strat};
}

bool jac_suitable(const JitMech &m)
{
    if (m.pd || !m.th) return false;
    // each LDS base covers two species arrays within a 16-bit offset
    return jac_lds_bytes(m.ns, m.nr) <= 160 * 1024 && 2 * 512 * m.ns <= 65536;
}

namespace {

// The Jacobian kernel, or with `vjp` the vector-Jacobian product of omega:
// g_Y[m] = sum_k g_k d omega_k/dY_m, g_T = sum_k g_k d omega_k/dT.  With
// gamma_j = sum_k nu_kj g_k these are the temperature row's sums with gamma_j
// in the place of dH_j:
//     g_Y[m] = f_m (rho_hat sum_j gamma_j dq_j/dC_m - sum_j gamma_j uf_j / sigma)
//     g_T    = sum_j gamma_j dq_j/dT
// so every wave sweeps a share of the reactions once, and the waves' sums are
// added in a fixed order.
JitProgram gen_deriv(const JitMech &m, bool f64out, bool interleaved, bool vjp)
{
    const int ns = m.ns, nr = m.nr, nv = ns + 1;
    const int W = kJacWaves;
    const int WT = vjp ? W : kJacTempWaves;   // waves that sweep all reactions
    const int WR = W - WT;
    int group = 3;
    if (const char *g = std::getenv("AK_JAC_GROUP")) group = std::max(1, std::atoi(g));
    // the temperature-row waves hold NS + 3 more sums: smaller groups
    bool xcd = true;
    if (const char *e = std::getenv("AK_JAC_XCD")) xcd = std::atoi(e) != 0;
    int tgroup = 2;
    if (const char *g = std::getenv("AK_JAC_TGROUP")) tgroup = std::max(1, std::atoi(g));
    const char *IO = f64out ? "double" : "float";
    const int SZ = f64out ? 8 : 4;
    JitProgram prog;
    prog.threads = 64 * W;

    // species table: the Gibbs-layer weights with log2(1/W) in the biases
    // (2^g' = w / W), the NASA-7 sets a1..a7 (low, high)
    prog.sp.assign((size_t)kJacSpStride * ns, 0.0);
    std::vector<double> lw(ns);
    for (int k = 0; k < ns; ++k) {
        double *s = &prog.sp[(size_t)kJacSpStride * k];
        std::memcpy(s, &m.sp[k], sizeof(SpeciesRec));
        lw[k] = -std::log2(m.sp[k].inv_W);
        s[8] -= lw[k];
        s[15] -= lw[k];
        for (int c = 0; c < 7; ++c) {
            s[16 + c] = m.th[k].lo[c];
            s[23 + c] = m.th[k].hi[c];
        }
    }
    // reactions: log2 A less the reactants' log2 W, beta, -(E/R) log2 e, E/R
    prog.rx.assign((size_t)kJacRxStride * nr, 0.0);
    for (int j = 0; j < nr; ++j) {
        double sh = 0.0;
        for (int i = 0; i < m.aux[j].nf; ++i) sh += lw[m.aux[j].sp[i]];
        prog.rx[kJacRxStride * j + 0] = m.rx[j].log2A - sh;
        prog.rx[kJacRxStride * j + 1] = m.rx[j].beta;
        prog.rx[kJacRxStride * j + 2] = m.rx[j].negEoR2;
        prog.rx[kJacRxStride * j + 3] = m.aux[j].EoR;
    }

    const std::vector<std::vector<int>> rs = reaction_species(m);
    // reactions that change species k, ascending
    std::vector<std::vector<int>> rx_of(ns);
    for (int j = 0; j < nr; ++j)
        for (int k : rs[j]) {
            int a, b;
            side_counts(m, j, k, a, b);
            if (a != b) rx_of[k].push_back(j);
        }
    // estimated cost of a row and of a temperature-row reaction
    auto rcost = [&](int j) { return 60.0 + 6.0 * rs[j].size(); };
    std::vector<double> rowc(ns, 20.0 + 4.0 * nv);
    for (int k = 0; k < ns; ++k)
        for (int j : rx_of[k]) rowc[k] += rcost(j);
    // the temperature-row reactions split between its waves by cost
    std::vector<std::vector<int>> trx(WT);
    double tcost = 0.0;
    for (int j = 0; j < nr; ++j) tcost += rcost(j) + 2.0 * rs[j].size();
    {
        double acc = 0.0;
        for (int j = 0; j < nr; ++j) {
            const int w = std::min(WT - 1, (int)(acc * WT / tcost));
            trx[w].push_back(j);
            acc += rcost(j) + 2.0 * rs[j].size();
        }
    }
    // contiguous row blocks: the waves of a workgroup sit on the four SIMDs in
    // turn (wave w on SIMD w % 4), so the row waves that share a SIMD with a
    // temperature-row wave get less
    std::vector<double> target(WR, 0.0);
    {
        double rtot = 0.0;
        for (int k = 0; k < ns; ++k) rtot += rowc[k];
        std::vector<double> simd(4, 0.0);
        std::vector<int> per(4, 0);
        for (int w = WR; w < W; ++w) simd[w % 4] += tcost / WT;
        for (int w = 0; w < WR; ++w) per[w % 4]++;
        const double X = (rtot + tcost) / 4.0;
        double sum = 0.0;
        for (int w = 0; w < WR; ++w) {
            target[w] = std::max(0.0, (X - simd[w % 4]) / per[w % 4]);
            sum += target[w];
        }
        for (int w = 0; w < WR; ++w) target[w] *= rtot / sum;
    }
    std::vector<int> rbeg(WR + 1, 0);
    {
        double acc = 0.0, goal = 0.0;
        int k = 0;
        for (int w = 0; w < WR; ++w) {
            rbeg[w] = k;
            goal += target[w];
            while (k < ns && (w == WR - 1 || acc + 0.5 * rowc[k] <= goal)) acc += rowc[k++];
        }
        rbeg[WR] = ns;
    }

    Text o;
    if (vjp)
        o("// generated by libannkin: vector-Jacobian product of the source term for a mechanism "
          "of %d species and %d reactions (%s states, one 64-cell tile per %d-wave workgroup)\n",
          ns, nr, f64out ? "FP64" : "FP32", W);
    else
        o("// generated by libannkin: state Jacobian for a mechanism of %d species and %d "
          "reactions (%s states and output, %s, one 64-cell tile per %d-wave workgroup)\n", ns,
          nr, f64out ? "FP64" : "FP32", interleaved ? "interleaved J" : "cell-major J", W);
    o("typedef long long i64;\ntypedef unsigned long long u64;\n");
    const std::vector<double> c = exp2_taylor(12);
    // 2^t: degree-12 Taylor polynomial of 2^f, |f| <= 1/2 (below one ulp of
    // double); with float output 2^f on the transcendental unit (about one
    // ulp of float)
    o("__device__ __forceinline__ double ex2(double t) {\n  const double nn = __builtin_rint(t);\n");
    if (f64out) {
        o("  const double f = t - nn;\n  double p = %s;\n", lit(c[12]).c_str());
        for (int q = 11; q >= 0; --q) o("  p = __builtin_fma(p, f, %s);\n", lit(c[q]).c_str());
        o("  return __builtin_ldexp(p, (int)nn);\n}\n");
    } else {
        o("  return __builtin_ldexp((double)__builtin_amdgcn_exp2f((float)(t - nn)), (int)nn);\n}\n");
    }
    // a tile value: byte offset `b` of the lane plus a constant
    o("#define LD(b, o) (*(const double *)((const char *)L + (b) + (o)))\n");
    // L (doubles): a | v' | w | h | f, [ns][64] each; the reaction constants
    // (first the mixture partials); per-wave partial sums of C cp, C dcp/dT
    // and cp omega
    const int LF = 4 * 64 * ns;
    const int LR = LF + 64 * ns;
    const int LX = LR + jac_rx_doubles(nr);
    o("#define AK_JAC_LDS __shared__ double L[%d];\n", LX + 3 * 64 * W);
    if (vjp)
        o("__device__ __forceinline__ void tile(i64 c0, i64 n, const %s *__restrict__ Tg, "
          "const %s *__restrict__ Pg, const %s *__restrict__ Yg, i64 ldY, "
          "const %s *__restrict__ Gg, i64 ldG, %s *__restrict__ GYg, i64 ldGY, "
          "%s *__restrict__ GTg, const double *__restrict__ SP, const double *__restrict__ RX, "
          "u64 *err, double *L) {\n", IO, IO, IO, IO, IO, IO);
    else
        o("__device__ __forceinline__ void tile(i64 c0, i64 n, const %s *__restrict__ Tg, "
          "const %s *__restrict__ Pg, const %s *__restrict__ Yg, i64 ldY, %s *__restrict__ Jg, "
          "i64 ldJ, const double *__restrict__ SP, const double *__restrict__ RX, u64 *err, "
          "double *L) {\n", IO, IO, IO, IO);
    // L: a [ns][64] | v' [ns][64] | w [ns][64] | h [ns][64] | f [ns][64] | partials
    o("  const unsigned lane = threadIdx.x & 63u;\n");
    o("  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));\n");
    o("  const bool live = c0 + (i64)lane < n;\n  const i64 ci = live ? c0 + (i64)lane : n - 1;\n");
    o("  const double T = (double)Tg[ci], P = (double)Pg[ci];\n");
    o("  const double LNT = log(T), IT = 1.0 / T, T2 = T * T, T3 = T2 * T, T4 = T3 * T;\n");
    o("  const double L2T = LNT * %s;\n", lit(kLog2e).c_str());
    o("  double *LXs = L + %d, *LXc = L + %d, *LXd = L + %d, *LXe = L + %d, *LXp = L + %d;\n", LR,
      LR + 64 * W, LX, LX + 64 * W, LX + 128 * W);
    // phase 1: the waves' own species (k = wave mod W), mixture sums
    std::vector<std::vector<int>> own(W);
    for (int k = 0; k < ns; ++k) own[k % W].push_back(k);
    const int maxown = (ns + W - 1) / W;
    o("  double ys[%d];\n  double sgp = 0.0, chk = 0.0;\n", std::max(1, maxown));
    if (vjp) o("  double gs[%d];\n", std::max(1, maxown));
    for (int w = 0; w < W; ++w) {
        if (own[w].empty()) continue;
        o("  %sif (wave == %d) {\n", w ? "else " : "", w);
        for (size_t i = 0; i < own[w].size(); ++i)
            o("    ys[%d] = (double)(Yg + (i64)%d * ldY)[ci];\n", (int)i, own[w][i]);
        if (vjp)
            for (size_t i = 0; i < own[w].size(); ++i)
                o("    gs[%d] = (double)(Gg + (i64)%d * ldG)[ci];\n", (int)i, own[w][i]);
        for (size_t i = 0; i < own[w].size(); ++i)
            o("    chk += ys[%d];\n    sgp += __builtin_fmax(ys[%d], 0.0) * SP[%d];\n", (int)i,
              (int)i, kJacSpStride * own[w][i]);
        o("  }\n");
    }
    o("  LXs[threadIdx.x] = sgp;\n  LXc[threadIdx.x] = chk;\n  __syncthreads();\n");
    o("  double sg = LXs[lane], chkt = LXc[lane];\n");
    for (int w = 1; w < W; ++w) o("  sg += LXs[%d + lane];\n  chkt += LXc[%d + lane];\n", 64 * w, 64 * w);
    // the reaction constants replace the mixture partials in LDS (read
    // there by every lane at the same address, in order with the other LDS
    // reads: scalar loads would share their wait counter)
    o("  __syncthreads();\n");
    o("  for (int i = threadIdx.x; i < %d; i += %d) L[%d + i] = RX[i];\n", kJacRxStride * nr, 64 * W,
      LR);
    o("  const bool bad = !(T > 0.0) || !(P > 0.0) || !__builtin_isfinite(T) || "
      "!__builtin_isfinite(P) || !__builtin_isfinite(chkt) || !(sg > 0.0) || "
      "!__builtin_isfinite(sg);\n");
    // a bad cell's whole matrix comes out NaN: rho_hat and 1/sigma carry it
    o("  const double nanb = bad ? __builtin_nan(\"\") : 0.0;\n");
    o("  const double rh = P / (%s * T * sg) + nanb, isg = 1.0 / sg + nanb;\n", lit(kRu).c_str());
    std::map<double, int> tmid;
    for (int k = 0; k < ns; ++k)
        if (!tmid.count(m.sp[k].T_mid)) {
            const int id = (int)tmid.size();
            tmid[m.sp[k].T_mid] = id;
            o("  const bool hi%d = T >= %s;\n", id, lit(m.sp[k].T_mid).c_str());
        }
    auto hiname = [&](int k) { return "hi" + std::to_string(tmid[m.sp[k].T_mid]); };
    // phase 2: a, w, v' = W v, H/RT and f of the own species into LDS;
    // partial sums of C cp and C dcp/dT
    o("  double denp = 0.0, ddp = 0.0;\n");
    for (int w = 0; w < W; ++w) {
        if (own[w].empty()) continue;
        o("  %sif (wave == %d) {\n", w ? "else " : "", w);
        for (size_t i = 0; i < own[w].size(); ++i) {
            const int k = own[w][i], b = kJacSpStride * k;
            auto gpoly = [&](int off) {
                char buf[512];
                snprintf(buf, sizeof buf,
                         "(__builtin_fma(SP[%d], LNT, __builtin_fma(SP[%d], T, "
                         "__builtin_fma(SP[%d], T2, __builtin_fma(SP[%d], T3, "
                         "__builtin_fma(SP[%d], T4, SP[%d] * IT))))) + SP[%d])",
                         b + off, b + off + 1, b + off + 2, b + off + 3, b + off + 4,
                         b + off + 5, b + off + 6);
                return std::string(buf);
            };
            // H/RT = a1 + a2 T/2 + a3 T^2/3 + a4 T^3/4 + a5 T^4/5 + a6/T
            auto hpoly = [&](int off) {
                char buf[640];
                snprintf(buf, sizeof buf,
                         "__builtin_fma(SP[%d], IT, __builtin_fma(T, __builtin_fma(T, "
                         "__builtin_fma(T, __builtin_fma(T, SP[%d] * 0.2, SP[%d] * 0.25), "
                         "SP[%d] * %s), SP[%d] * 0.5), SP[%d]))",
                         b + off + 5, b + off + 4, b + off + 3, b + off + 2,
                         lit(1.0 / 3.0).c_str(), b + off + 1, b + off);
                return std::string(buf);
            };
            auto dcpoly = [&](int off) {
                char buf[512];
                snprintf(buf, sizeof buf,
                         "__builtin_fma(T, __builtin_fma(T, __builtin_fma(T, SP[%d] * 4.0, "
                         "SP[%d] * 3.0), SP[%d] * 2.0), SP[%d])",
                         b + off + 4, b + off + 3, b + off + 2, b + off + 1);
                return std::string(buf);
            };
            o("    {\n      double glo = %s, ghi = %s;\n", gpoly(2).c_str(), gpoly(9).c_str());
            o("      asm(\"\" : \"+v\"(glo), \"+v\"(ghi));\n");
            o("      const double g = %s ? ghi : glo;\n", hiname(k).c_str());
            o("      const double nn = __builtin_rint(g), f = g - nn, f2 = f * f;\n");
            o("      double E = %s;\n", lit(c[12]).c_str());
            for (int q = 10; q >= 0; q -= 2) o("      E = __builtin_fma(E, f2, %s);\n", lit(c[q]).c_str());
            o("      double O = %s;\n", lit(c[11]).c_str());
            for (int q = 9; q >= 1; q -= 2) o("      O = __builtin_fma(O, f2, %s);\n", lit(c[q]).c_str());
            o("      O *= f;\n      const int ni = (int)nn;\n");
            o("      const double y = ys[%d], yp = __builtin_fmax(y, 0.0);\n", (int)i);
            o("      const double wp = __builtin_ldexp(E + O, ni);\n");   // 2^g' = w / W
            if (vjp)   // a, with the sign of zero keeping Y < 0 for the clamp
                o("      L[%d + lane] = y >= 0.0 ? rh * y * wp : -0.0;\n", 64 * k);
            else
                o("      L[%d + lane] = rh * yp * wp;\n", 64 * k);                    // a
            o("      L[%d + lane] = __builtin_ldexp(E - O, -ni);\n", 64 * (ns + k));  // v' = W v
            o("      L[%d + lane] = wp * %s;\n", 64 * (2 * ns + k),                  // w
              lit(1.0 / m.sp[k].inv_W).c_str());
            o("      double hl = %s, hh = %s;\n", hpoly(16).c_str(), hpoly(23).c_str());
            o("      asm(\"\" : \"+v\"(hl), \"+v\"(hh));\n");
            o("      L[%d + lane] = %s ? hh : hl;\n", 64 * (3 * ns + k), hiname(k).c_str());
            if (vjp) {
                o("      L[%d + lane] = gs[%d];\n    }\n", LF + 64 * k, (int)i);     // g_omega
                continue;
            }
            o("      L[%d + lane] = y >= 0.0 ? SP[%d] : 0.0;\n", LF + 64 * k, b);   // f = [Y >= 0] / W
            o("      const double C = rh * yp * SP[%d];\n", b);
            emit_cp(o, "      ", "cp", k, hiname(k));
            o("      denp = __builtin_fma(C, cp, denp);\n");
            o("      double dl = %s, dh = %s;\n", dcpoly(16).c_str(), dcpoly(23).c_str());
            o("      asm(\"\" : \"+v\"(dl), \"+v\"(dh));\n");
            o("      ddp = __builtin_fma(C, %s ? dh : dl, ddp);\n    }\n", hiname(k).c_str());
        }
        o("  }\n");
    }
    o("  LXd[threadIdx.x] = denp;\n  LXe[threadIdx.x] = ddp;\n  __syncthreads();\n");
    // the last wave keeps the sums of C cp and C dcp/dT; then the staging
    // slots are free
    // where this lane's cell's matrix goes: cell-major (J[cell][row][col])
    // or interleaved (J[row * nv + col][cell]); the lanes past the end write
    // the last cell's again, bit for bit
    if (vjp) {
    } else if (interleaved) {
        o("  const i64 ldJb = ldJ * %d;\n", SZ);
        o("  char *Jb = (char *)(Jg + c0) + (unsigned)(ci - c0) * %du;\n", SZ);
    } else {
        o("  %s *Jc = Jg + ci * ldJ;\n", IO);
    }

    // phase 3: rows and the temperature-row sums
    o("  double cpw = 0.0;\n");
    // the temperature-row sums (set only in the waves that build it)
    o("  double ");
    for (int cc = 0; cc < nv; ++cc) o("St%d, ", cc);
    o("SU, SN;\n");
    Lds lds;
    lds.ns = ns;
    // J[row][col] of this lane's cell
    auto put = [&](const char *ind, int row, int col, const std::string &v) {
        if (interleaved)
            o("%s*(%s *)(Jb + %d * ldJb) = (%s)(%s);\n", ind, IO, row * nv + col, IO, v.c_str());
        else
            o("%sJc[%d] = (%s)(%s);\n", ind, row * nv + col, IO, v.c_str());
    };
    // the walks: (row, reaction) pairs of the row waves, reactions of the
    // temperature-row waves
    for (int w = 0; w < W; ++w) {
        const bool trow = w >= WR;
        std::vector<std::pair<int, int>> walk;
        if (!trow) {
            for (int k = rbeg[w]; k < rbeg[w + 1]; ++k)
                for (int j : rx_of[k]) walk.push_back({k, j});
        } else {
            for (int j : trx[w - WR]) walk.push_back({-1, j});
        }
        o("  %sif (wave == %d) {\n", w ? "else " : "", w);
        o("    unsigned bl = lane * 8u, bh = lane * 8u + %du, bf = lane * 8u + %du, bk = %du;\n",
          2 * 512 * ns, 8 * LF, 8 * LR);
        o("    double zz = 0.0;\n");
        if (trow) {
            for (int cc = 0; cc < nv; ++cc) o("    St%d = 0.0;\n", cc);
            o("    SU = 0.0;\n    SN = 0.0;\n");
        }
        const int cnt = (int)walk.size();
        // scheduling groups of at most `group` walk entries, none across a
        // row boundary
        std::vector<std::pair<int, int>> groups;
        const int gsize = trow ? tgroup : group;
        for (int q = 0; q < cnt;) {
            int e = q + 1;
            while (e < cnt && e - q < gsize && walk[e].first == walk[q].first) ++e;
            groups.push_back({q, e});
            q = e;
        }
        auto loads = [&](int g) {
            for (int q = groups[g].first; q < groups[g].second; ++q) {
                const int j = walk[q].second;
                o("    const double kA%d = LD(bk, %d), kB%d = LD(bk, %d), kE%d = LD(bk, %d), "
                  "kR%d = LD(bk, %d);\n", q, 8 * kJacRxStride * j, q, 8 * kJacRxStride * j + 8, q,
                  8 * kJacRxStride * j + 16, q, 8 * kJacRxStride * j + 24);
            }
        };
        const int ngroups = (int)groups.size();
        std::vector<int> cols;        // nonzero columns of the row being built
        auto finish_row = [&](int k) {
            // J[k][c] = f_c (rho_hat G_kc - u / sigma), J[k][T] = Tc; stores
            // without a branch: one here would let the compiler sink the
            // row's whole accumulation into it
            o("    {\n      const double us = u%d * isg;\n", k);
            for (int cc = 0; cc < ns; ++cc) {
                const bool has = std::find(cols.begin(), cols.end(), cc) != cols.end();
                // the flag through the fenced base: a value kept from an
                // earlier row would hold a register for the whole walk
                const std::string f = "LD(bf, " + std::to_string(512 * cc) + ")";
                put("      ", k, cc, has ? f + " * __builtin_fma(rh, G" + std::to_string(k) + "_" +
                                            std::to_string(cc) + ", -us)"
                                      : "-(" + f + " * us)");
            }
            put("      ", k, ns, "Tc" + std::to_string(k) + " + nanb");
            emit_cp(o, "      ", "cp", k, hiname(k));
            o("      cpw = __builtin_fma(cp, om%d, cpw);\n    }\n", k);
            o("    __builtin_amdgcn_sched_barrier(0);\n");
        };
        for (int g = 0; g < ngroups; ++g) {
            const int q0 = groups[g].first, q1 = groups[g].second;
            const int k = walk[q0].first;
            if (g > 0)
                o("    asm volatile(\"\" : \"+v\"(bl), \"+v\"(bh), \"+v\"(bf), \"+v\"(bk) : \"v\"(zz));\n");
            loads(g);
            if (!trow && (g == 0 || walk[groups[g - 1].first].first != k)) {
                // a new row: its own species' values in registers, zeroed sums
                cols.clear();
                for (int jj : rx_of[k])
                    for (int l : rs[jj])
                        if (std::find(cols.begin(), cols.end(), l) == cols.end()) cols.push_back(l);
                std::sort(cols.begin(), cols.end());
                o("    const double Ra%d = %s, Rv%d = %s, Rw%d = %s, Rh%d = %s;\n", k,
                  lds.read(0, k).c_str(), k, lds.read(1, k).c_str(), k, lds.read(2, k).c_str(), k,
                  lds.read(3, k).c_str());
                for (int l : cols) o("    double G%d_%d = 0.0;\n", k, l);
                o("    double u%d = 0.0, Tc%d = 0.0, om%d = 0.0;\n", k, k, k);
            }
            for (int q = q0; q < q1; ++q) {
                const int j = walk[q].second;
                Lds rl = lds;
                rl.row = trow ? -1 : k;
                o("    {\n");
                if (!trow)
                    o("      const double Ra = Ra%d, Rv = Rv%d, Rw = Rw%d, Rh = Rh%d;\n", k, k, k, k);
                const Deriv d = emit_jac_rxn(o, "      ", m, f64out, q, j, rs[j], trow && !vjp, rl,
                                             vjp);
                if (!trow) {
                    int a, b;
                    side_counts(m, j, k, a, b);
                    const int nu = b - a;
                    for (size_t i = 0; i < d.sp.size(); ++i)
                        if (d.sign[i])
                            accumulate(o, "      ",
                                       "G" + std::to_string(k) + "_" + std::to_string(d.sp[i]),
                                       nu, d.sign[i], "d_" + std::to_string(d.sp[i]));
                    accumulate(o, "      ", "Tc" + std::to_string(k), nu, 2, "dqT");
                    accumulate(o, "      ", "u" + std::to_string(k), nu, 2, "uf");
                    accumulate(o, "      ", "om" + std::to_string(k), nu, 2, "qn");
                } else {
                    // the weight: dH_j for the temperature row, gamma_j for the VJP
                    const char *wt = vjp ? "ga" : "dH";
                    for (size_t i = 0; i < d.sp.size(); ++i) {
                        if (!d.sign[i]) continue;
                        const int l = d.sp[i];
                        if (d.sign[i] == -1)
                            o("      St%d = __builtin_fma(-%s, d_%d, St%d);\n", l, wt, l, l);
                        else o("      St%d = __builtin_fma(%s, d_%d, St%d);\n", l, wt, l, l);
                    }
                    o("      St%d = __builtin_fma(%s, dqT, St%d);\n", ns, wt, ns);
                    o("      SU = __builtin_fma(%s, uf, SU);\n", wt);
                    if (!vjp) o("      SN = __builtin_fma(dH, qn, SN);\n");
                }
                o("      zz = dqT;\n    }\n");
            }
            o("    __builtin_amdgcn_sched_barrier(0);\n");
            if (!trow && (g + 1 == ngroups || walk[groups[g + 1].first].first != k)) finish_row(k);
        }
        // the wave's share of sum_k cp_k omega_k, in the first 64 doubles of
        // its staging slot
        if (!trow) o("    LXp[threadIdx.x] = cpw;\n");
        o("  }\n");
    }
    // every wave is done with the tile values
    o("  __syncthreads();\n");
    if (vjp) {
        // the eight waves' sums (St_0..St_NS, SU) added in the fixed order
        // ((w0 + w1) + (w2 + w3)) + ((w4 + w5) + (w6 + w7)) through two LDS
        // slots past the a area (a keeps the clamp in its sign)
        const int S0 = 64 * ns, S1 = S0 + 64 * (nv + 1);
        const int stages[4][4] = {{1, 0, 3, 2}, {5, 4, 7, 6}, {2, 0, 6, 4}, {4, 0, -1, -1}};
        for (const auto &st : stages) {
            for (int h = 0; h < 2; ++h) {
                if (st[2 * h] < 0) continue;
                o("  if (wave == %d) {\n", st[2 * h]);
                for (int cc = 0; cc < nv; ++cc) o("    L[%d + lane] = St%d;\n", (h ? S1 : S0) + 64 * cc, cc);
                o("    L[%d + lane] = SU;\n  }\n", (h ? S1 : S0) + 64 * nv);
            }
            o("  __syncthreads();\n");
            for (int h = 0; h < 2; ++h) {
                if (st[2 * h] < 0) continue;
                o("  if (wave == %d) {\n", st[2 * h + 1]);
                for (int cc = 0; cc < nv; ++cc)
                    o("    St%d += L[%d + lane];\n", cc, (h ? S1 : S0) + 64 * cc);
                o("    SU += L[%d + lane];\n  }\n", (h ? S1 : S0) + 64 * nv);
            }
            o("  __syncthreads();\n");
        }
        // g_Y[m] = f_m (rho_hat St_m - SU / sigma), g_T = St_NS; the lanes past
        // the end write the last cell's again
        o("  if (wave == 0) {\n    const double us = SU * isg;\n");
        for (int cc = 0; cc < ns; ++cc)
            o("    GYg[(i64)%d * ldGY + ci] = (%s)((__builtin_signbit(L[%d + lane]) ? 0.0 : %s) * "
              "__builtin_fma(rh, St%d, -us));\n", cc, IO, 64 * cc, lit(m.sp[cc].inv_W).c_str(), cc);
        o("    GTg[ci] = (%s)(St%d + nanb);\n", IO, ns);
        o("    if (live && bad) atomicAdd(err, 1ull);\n  }\n}\n");
        o("extern \"C\" __global__ __launch_bounds__(%d) void ak_vjp(const %s *__restrict__ T, "
          "const %s *__restrict__ P, const %s *__restrict__ Y, i64 ldY, i64 n, "
          "const %s *__restrict__ G, i64 ldG, %s *__restrict__ GY, i64 ldGY, %s *__restrict__ GT, "
          "const double *__restrict__ SP, const double *__restrict__ RX, u64 *err) {\n", 64 * W,
          IO, IO, IO, IO, IO, IO);
        o("  AK_JAC_LDS\n  const unsigned nb = gridDim.x, per = nb / 8u, b = blockIdx.x;\n"
          "  const unsigned t = %s;\n"
          "  tile((i64)t * 64, n, T, P, Y, ldY, G, ldG, GY, ldGY, GT, SP, RX, err, L);\n}\n",
          xcd ? "b < per * 8u ? (b % 8u) * per + b / 8u : b" : "b");
        prog.src = std::move(o.s);
        return prog;
    }
    // the first temperature-row wave's sums go to LDS, the last one adds its
    // own (fixed order)
    if (WT == 2) {
        o("  if (wave == %d) {\n", WR);
        for (int cc = 0; cc < nv; ++cc) o("    L[%d + lane] = St%d;\n", 64 * cc, cc);
        o("    L[%d + lane] = SU;\n    L[%d + lane] = SN;\n  }\n", 64 * nv, 64 * (nv + 1));
    }
    o("  __syncthreads();\n");
    // the temperature row, written by the last wave:
    // omega_T = -num/den, num = Ru T sum_j dH_j q_j, den = Ru sum C cp
    o("  if (wave == %d) {\n", W - 1);
    o("    double denr = LXd[lane], ddr = LXe[lane], cpwt = LXp[lane];\n");
    for (int w = 1; w < W; ++w) o("    denr += LXd[%d + lane];\n    ddr += LXe[%d + lane];\n", 64 * w, 64 * w);
    for (int w = 1; w < WR; ++w) o("    cpwt += LXp[%d + lane];\n", 64 * w);
    o("    const double SUt = L[%d + lane] + SU, SNt = L[%d + lane] + SN;\n", 64 * nv, 64 * (nv + 1));
    o("    const double num = %s * T * SNt, den = %s * denr;\n", lit(kRu).c_str(), lit(kRu).c_str());
    o("    const double iden2 = 1.0 / (den * den) + nanb;\n");
    for (int cc = 0; cc < ns; ++cc) {
        o("    {\n      const double fc = L[%d + lane];\n", LF + 64 * cc);
        o("      const double dnum = %s * T * fc * __builtin_fma(rh, L[%d + lane] + St%d, -SUt * isg);\n",
          lit(kRu).c_str(), 64 * cc, cc);
        emit_cp(o, "      ", "cp", cc, hiname(cc));
        o("      const double dden = %s * fc * __builtin_fma(rh, cp, -denr * isg);\n",
          lit(kRu).c_str());
        put("      ", ns, cc, "-(dnum * den - num * dden) * iden2");
        o("    }\n");
    }
    o("    {\n      const double dnum = %s * (cpwt + T * (L[%d + lane] + St%d));\n", lit(kRu).c_str(),
      64 * ns, ns);
    o("      const double dden = -den * IT + %s * ddr;\n", lit(kRu).c_str());
    put("      ", ns, ns, "-(dnum * den - num * dden) * iden2");
    o("    }\n    if (live && bad) atomicAdd(err, 1ull);\n  }\n}\n");
    o("extern \"C\" __global__ __launch_bounds__(%d) void ak_jac(const %s *__restrict__ T, "
      "const %s *__restrict__ P, const %s *__restrict__ Y, i64 ldY, i64 n, %s *__restrict__ J, "
      "i64 ldJ, const double *__restrict__ SP, const double *__restrict__ RX, u64 *err) {\n",
      64 * W, IO, IO, IO, IO);
    if (xcd) {
        // workgroups go to the eight XCDs in turn: give each XCD a contiguous
        // range of tiles, so that the tiles sharing an L2 write neighbouring
        // cells (the rest, fewer than eight, keep their own index)
        o("  AK_JAC_LDS\n  const unsigned nb = gridDim.x, per = nb / 8u, b = blockIdx.x;\n"
          "  const unsigned t = b < per * 8u ? (b %% 8u) * per + b / 8u : b;\n"
          "  tile((i64)t * 64, n, T, P, Y, ldY, J, ldJ, SP, RX, err, L);\n}\n");
    } else {
        o("  AK_JAC_LDS\n  tile((i64)blockIdx.x * 64, n, T, P, Y, ldY, J, ldJ, SP, RX, err, L);\n}\n");
    }
    prog.src = std::move(o.s);
    return prog;
}

}  // namespace

JitProgram jit_program_jac(const JitMech &m, bool f64out, bool interleaved)
{
    return gen_deriv(m, f64out, interleaved, false);
}

JitProgram jit_program_vjp(const JitMech &m, bool f64out)
{
    return gen_deriv(m, f64out, false, true);
}

}  // namespace ak
