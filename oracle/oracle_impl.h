/*
 * Test oracle body, instantiated twice by oracle.c: once with REAL = double
 * (suffix _f64) and once with REAL = long double (suffix _ld).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load or call this code.
 *
 * It computes the *plain definition* of the chemical source term
 * (Barwey & Raman, Sec. 2): the classical law of mass action with products
 * of concentrations, Arrhenius rate constants, and equilibrium constants from
 * enthalpy and entropy changes.  It deliberately does NOT use the paper's
 * log-space matrix ("ANN") re-association.
 *
 * Expects the including file to define REAL, SFX(name), EXP, LOG, POW, FABS.
 */

/* NASA-7 enthalpy, entropy and heat capacity of one species at T (McBride,
 * Gordon & Reno, NASA TM-4513; the paper's "NASA polynomials", Sec. 2.2,
 * Eq. 10).  The high-range set applies for T >= T_mid. */
static void SFX(thermo1)(const ora_mech *m, int k, REAL T, REAL *h_RT, REAL *s_R,
                         REAL *cp_R, REAL *dcp_R)
{
    const double *a = (T >= (REAL)m->T_mid[k]) ? &m->nasa_high[7 * k] : &m->nasa_low[7 * k];
    REAL a1 = a[0], a2 = a[1], a3 = a[2], a4 = a[3], a5 = a[4], a6 = a[5], a7 = a[6];
    REAL T2 = T * T, T3 = T2 * T, T4 = T3 * T;
    if (h_RT) *h_RT = a1 + a2 * T / 2 + a3 * T2 / 3 + a4 * T3 / 4 + a5 * T4 / 5 + a6 / T;
    if (s_R)  *s_R  = a1 * LOG(T) + a2 * T + a3 * T2 / 2 + a4 * T3 / 3 + a5 * T4 / 4 + a7;
    if (cp_R) *cp_R = a1 + a2 * T + a3 * T2 + a4 * T3 + a5 * T4;
    if (dcp_R) *dcp_R = a2 + 2 * a3 * T + 3 * a4 * T2 + 4 * a5 * T3;
}

/* Arrhenius rate constant A T^beta exp(-E/(R T)) in SI-kmol units (Eq. 5),
 * from A in cgs units of the given order, (cm^3/mol)^(order-1)/s, and E in
 * cal/mol. */
static REAL SFX(arrhenius)(double ln_A, double beta, double Ea, int order, REAL T)
{
    REAL A_si = EXP((REAL)ln_A) * POW((REAL)1e-3L, (REAL)(order - 1));
    REAL E_R = (REAL)Ea * (REAL)ORA_CAL / (REAL)ORA_RU_MOL;
    return A_si * POW(T, (REAL)beta) * EXP(-E_R / T);
}

static int SFX(rtype1)(const ora_mech *m, int j) { return m->rtype ? m->rtype[j] : 0; }

/* Forward rate constant of reaction j (Eq. 5), with the pressure dependence
 * of Sec. 2.4 for third-body and falloff reactions:
 *   third body:  k_f = k [M], [M] = sum_k eff_kj C_k (the paper's M = C E);
 *   falloff:     k_f = k_inf Pr/(1 + Pr) F, Pr = k_0 [M] / k_inf, with F = 1
 *                (Lindemann) or the Troe broadening
 *                log10 F = log10 Fc / (1 + ((log10 Pr + c)/(n - 0.14 (log10 Pr + c)))^2),
 *                c = -0.4 - 0.67 log10 Fc, n = 0.75 - 1.27 log10 Fc,
 *                Fc = (1 - alpha) exp(-T/T3) + alpha exp(-T/T1) + exp(-T2/T)
 *                (Gilbert, Luther & Troe 1983; T3, T1, T2 are the usual T***,
 *                T* and T**). */
static REAL SFX(kf1)(const ora_mech *m, int j, REAL T, const REAL *C)
{
    int order = 0;
    for (int k = 0; k < m->ns; ++k) order += m->nu_f[j * m->ns + k];
    const int type = SFX(rtype1)(m, j);
    if (type == ORA_ELEMENTARY)
        return SFX(arrhenius)(m->ln_A[j], m->beta[j], m->Ea[j], order, T);
    REAL M = 0;
    for (int k = 0; k < m->ns; ++k) M += (m->eff ? (REAL)m->eff[j * m->ns + k] : 1) * C[k];
    if (type == ORA_THIRD_BODY)
        return SFX(arrhenius)(m->ln_A[j], m->beta[j], m->Ea[j], order + 1, T) * M;
    REAL kinf = SFX(arrhenius)(m->ln_A[j], m->beta[j], m->Ea[j], order, T);
    REAL k0 = SFX(arrhenius)(m->low_ln_A[j], m->low_beta[j], m->low_Ea[j], order + 1, T);
    REAL Pr = k0 * M / kinf;
    REAL F = 1;
    if (type == ORA_TROE && Pr > 0) {
        const double *tp = &m->troe[4 * j];
        REAL Fc = (1 - (REAL)tp[0]) * EXP(-T / (REAL)tp[1]) + (REAL)tp[0] * EXP(-T / (REAL)tp[2]);
        if (tp[3] != 0) Fc += EXP(-(REAL)tp[3] / T);
        REAL lFc = LOG10(Fc);
        REAL c = (REAL)-0.4L - (REAL)0.67L * lFc, nn = (REAL)0.75L - (REAL)1.27L * lFc;
        REAL x = LOG10(Pr) + c;
        REAL f1 = x / (nn - (REAL)0.14L * x);
        F = POW((REAL)10, lFc / (1 + f1 * f1));
    }
    return kinf * (Pr / (1 + Pr)) * F;
}

/* Concentrations from the ideal-gas state: C_k = P/(Ru T) * (Y_k/W_k)/sum_l(Y_l/W_l),
 * with negative mass fractions clamped to zero. */
static REAL SFX(concentrations)(const ora_mech *m, REAL T, REAL P, const REAL *Y, REAL *C)
{
    REAL sum = 0;
    for (int k = 0; k < m->ns; ++k) {
        REAL y = Y[k] > 0 ? Y[k] : 0;
        C[k] = y / (REAL)m->W[k];
        sum += C[k];
    }
    REAL rho_hat = P / ((REAL)ORA_RU * T * sum);
    for (int k = 0; k < m->ns; ++k) C[k] *= rho_hat;
    return sum;
}

/* integer power by repeated multiplication */
static REAL SFX(ipow)(REAL x, int n)
{
    REAL r = 1;
    for (int i = 0; i < n; ++i) r *= x;
    return r;
}

/* Equilibrium constant in concentration units of reaction j (Eq. 8):
 *   K_c = (p_ref/(Ru T))^dn exp(dS/R - dH/(R T)),  dn = sum_k nu_kj. */
static REAL SFX(kc1)(const ora_mech *m, int j, REAL T, const REAL *h_RT, const REAL *s_R)
{
    const int ns = m->ns;
    const int8_t *nf = &m->nu_f[j * ns], *nr = &m->nu_r[j * ns];
    REAL dn = 0, dS = 0, dH = 0;
    for (int k = 0; k < ns; ++k) {
        int nu = nr[k] - nf[k];
        if (!nu) continue;
        dn += nu;
        dS += nu * s_R[k];
        dH += nu * h_RT[k];
    }
    return POW((REAL)ORA_PREF / ((REAL)ORA_RU * T), dn) * EXP(dS - dH);
}

/* Per-reaction quantities for one cell at given concentrations:
 * kf (Eq. 5), Kc (Eq. 8), kr = kf/Kc (Eq. 7, zero for irreversible
 * reactions), qf and qr (Eq. 3).  h_RT and s_R are the species values at T.
 * With lnK not NULL, *lnK is used as ln K_c instead of Eq. 8 (a trained
 * approximation of ln K_c as a drop-in, Sec. 2.3). */
static void SFX(reaction_kc)(const ora_mech *m, int j, REAL T, const REAL *C,
                             const REAL *h_RT, const REAL *s_R, const REAL *lnK,
                             REAL *kf, REAL *Kc, REAL *qf, REAL *qr)
{
    const int ns = m->ns;
    const int8_t *nf = &m->nu_f[j * ns], *nr = &m->nu_r[j * ns];
    REAL k_f = SFX(kf1)(m, j, T, C);
    REAL K_c = lnK ? EXP(*lnK) : SFX(kc1)(m, j, T, h_RT, s_R);
    REAL k_r = (m->reversible == 0 || m->reversible[j]) ? k_f / K_c : 0;
    REAL pf = 1, pr = 1;
    for (int k = 0; k < ns; ++k) {
        if (nf[k]) pf *= SFX(ipow)(C[k], nf[k]);
        if (nr[k]) pr *= SFX(ipow)(C[k], nr[k]);
    }
    *kf = k_f;
    *Kc = K_c;
    *qf = k_f * pf;
    *qr = k_r * pr;
}

static void SFX(reaction1)(const ora_mech *m, int j, REAL T, const REAL *C,
                           const REAL *h_RT, const REAL *s_R,
                           REAL *kf, REAL *Kc, REAL *qf, REAL *qr)
{
    SFX(reaction_kc)(m, j, T, C, h_RT, s_R, 0, kf, Kc, qf, qr);
}

/* ln K_c (Eq. 8) of every reaction at each of n temperatures:
 * lnK[j*ldK + i] for reaction j (file order) and temperature T[i]. */
int SFX(ora_lnkc)(const ora_mech *m, int64_t n, const double *T, REAL *lnK, int64_t ldK)
{
    const int ns = m->ns;
    REAL *h = (REAL *)malloc(sizeof(REAL) * 2 * ns);
    if (!h) return -1;
    REAL *s = h + ns;
    for (int64_t i = 0; i < n; ++i) {
        REAL Ti = T[i];
        for (int k = 0; k < ns; ++k) SFX(thermo1)(m, k, Ti, &h[k], &s[k], 0, 0);
        for (int j = 0; j < m->nr; ++j) lnK[j * ldK + i] = LOG(SFX(kc1)(m, j, Ti, h, s));
    }
    free(h);
    return 0;
}

int SFX(ora_thermo)(const ora_mech *m, double T, REAL *h_RT, REAL *s_R, REAL *cp_R)
{
    for (int k = 0; k < m->ns; ++k)
        SFX(thermo1)(m, k, (REAL)T, h_RT ? &h_RT[k] : 0, s_R ? &s_R[k] : 0,
                     cp_R ? &cp_R[k] : 0, 0);
    return 0;
}

/* One cell: concentrations and per-reaction kf, Kc, qf, qr (arrays of NR). */
int SFX(ora_rates)(const ora_mech *m, double T, double P, const double *Y,
                   REAL *C, REAL *kf, REAL *Kc, REAL *qf, REAL *qr)
{
    const int ns = m->ns;
    if (ns <= 0) return -1;
    REAL *Yr = (REAL *)malloc(sizeof(REAL) * 3 * ns);
    if (!Yr) return -1;
    REAL *h = Yr + ns, *s = h + ns;
    for (int k = 0; k < ns; ++k) Yr[k] = Y[k];
    SFX(concentrations)(m, T, P, Yr, C);
    for (int k = 0; k < ns; ++k) SFX(thermo1)(m, k, T, &h[k], &s[k], 0, 0);
    for (int j = 0; j < m->nr; ++j)
        SFX(reaction1)(m, j, T, C, h, s, &kf[j], &Kc[j], &qf[j], &qr[j]);
    free(Yr);
    return 0;
}

/* Net molar production rates (Eq. 2) for n cells.
 * Y is species-major with leading dimension ldY (Y[k*ldY + i]); omega, S and
 * N likewise with ldO.  S_ik = sum_j |nu_kj| (qf + qr) is the gross rate
 * scale and N_ik = sum_j |nu_kj| |qf - qr| the net rate scale (used to grade
 * rounding error); either may be NULL. */
static int SFX(source_body)(const ora_mech *m, int64_t n, const double *T, const double *P,
                           const double *Y, int64_t ldY, const double *lnKin, int64_t ldK,
                           REAL *omega, REAL *S, REAL *N, int64_t ldO, int n_threads);

int SFX(ora_source)(const ora_mech *m, int64_t n, const double *T, const double *P,
                    const double *Y, int64_t ldY, REAL *omega, REAL *S, REAL *N,
                    int64_t ldO, int n_threads)
{
    return SFX(source_body)(m, n, T, P, Y, ldY, 0, 0, omega, S, N, ldO, n_threads);
}

/* As ora_source, with ln K_c of reaction j in cell i taken from
 * lnK[j*ldK + i] instead of Eq. 8 (the drop-in of a trained ln K_c,
 * Sec. 2.3); the forward rates, and so the irreversible reactions, are
 * unchanged. */
int SFX(ora_source_lnkc)(const ora_mech *m, int64_t n, const double *T, const double *P,
                         const double *Y, int64_t ldY, const double *lnK, int64_t ldK,
                         REAL *omega, REAL *S, REAL *N, int64_t ldO, int n_threads)
{
    if (!lnK) return -1;
    return SFX(source_body)(m, n, T, P, Y, ldY, lnK, ldK, omega, S, N, ldO, n_threads);
}

static int SFX(source_body)(const ora_mech *m, int64_t n, const double *T, const double *P,
                           const double *Y, int64_t ldY, const double *lnKin, int64_t ldK,
                           REAL *omega, REAL *S, REAL *N, int64_t ldO, int n_threads)
{
    const int ns = m->ns, nr = m->nr;
    int err = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel
#endif
    {
        REAL *buf = (REAL *)malloc(sizeof(REAL) * 7 * ns);
        if (!buf) {
            err = -1;
        } else {
            REAL *Yc = buf, *C = Yc + ns, *h = C + ns, *s = h + ns, *om = s + ns, *sg = om + ns,
                 *sn = sg + ns;
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
            for (int64_t i = 0; i < n; ++i) {
                REAL Ti = T[i], Pi = P[i];
                for (int k = 0; k < ns; ++k) {
                    Yc[k] = Y[k * ldY + i];
                    om[k] = sg[k] = sn[k] = 0;
                }
                SFX(concentrations)(m, Ti, Pi, Yc, C);
                for (int k = 0; k < ns; ++k) SFX(thermo1)(m, k, Ti, &h[k], &s[k], 0, 0);
                for (int j = 0; j < nr; ++j) {
                    REAL kf, Kc, qf, qr, lk = lnKin ? (REAL)lnKin[j * ldK + i] : 0;
                    SFX(reaction_kc)(m, j, Ti, C, h, s, lnKin ? &lk : 0, &kf, &Kc, &qf, &qr);
                    REAL qn = qf - qr;
                    const int8_t *nf = &m->nu_f[j * ns], *nrr = &m->nu_r[j * ns];
                    for (int k = 0; k < ns; ++k) {
                        int nu = nrr[k] - nf[k];
                        if (!nu) continue;
                        om[k] += nu * qn;
                        sg[k] += FABS((REAL)nu) * (qf + qr);
                        sn[k] += FABS((REAL)nu) * FABS(qn);
                    }
                }
                for (int k = 0; k < ns; ++k) {
                    omega[k * ldO + i] = om[k];
                    if (S) S[k * ldO + i] = sg[k];
                    if (N) N[k * ldO + i] = sn[k];
                }
            }
            free(buf);
        }
    }
    return err;
}

/* Constant-pressure temperature source  omega_T = -sum_k h_k omega_k / sum_k C_k cp_k
 * in K/s, with h_k = Ru T (h/RT)_k the molar enthalpy and cp_k = Ru (cp/R)_k.
 * (Not part of the paper's method; it is the last row of the state Jacobian
 * an implicit integrator of (Y, T) needs.) */
int SFX(ora_temp_source)(const ora_mech *m, int64_t n, const double *T, const double *P,
                         const double *Y, int64_t ldY, REAL *omega_T, int n_threads)
{
    const int ns = m->ns;
    REAL *om = (REAL *)malloc(sizeof(REAL) * ns * n);
    if (!om) return -1;
    int rc = SFX(ora_source)(m, n, T, P, Y, ldY, om, 0, 0, n, n_threads);
    if (rc) { free(om); return rc; }
    REAL *C = (REAL *)malloc(sizeof(REAL) * 2 * ns);
    if (!C) { free(om); return -1; }
    REAL *Yc = C + ns;
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k < ns; ++k) Yc[k] = Y[k * ldY + i];
        SFX(concentrations)(m, T[i], P[i], Yc, C);
        REAL num = 0, den = 0;
        for (int k = 0; k < ns; ++k) {
            REAL h, cp;
            SFX(thermo1)(m, k, T[i], &h, 0, &cp, 0);
            num += (REAL)ORA_RU * T[i] * h * om[k * n + i];
            den += C[k] * (REAL)ORA_RU * cp;
        }
        omega_T[i] = -num / den;
    }
    free(C);
    free(om);
    return 0;
}

/* Analytic Jacobian of (omega_1..omega_NS, omega_T) with respect to
 * x = (Y_1..Y_NS, T) at fixed P, in the classical (product) form.
 * J is [n][NS+1][NS+1] row-major per cell, cells outermost, cell stride ldJ.
 * dC_l/dY_m = (rho_hat/W_m) delta_lm - C_l/(sigma W_m) with sigma = sum Y/W,
 * dC_l/dT = -C_l/T, d ln kf/dT = (beta + E/RT)/T,
 * d ln Kc/dT = (dH/RT - dn)/T, and dq/dC_l by differentiating each power
 * C_l^nu directly (defined at C_l = 0).  For Y_m < 0 the clamp makes
 * dC/dY_m zero; at Y_m = 0 the right derivative is used. */
int SFX(ora_jacobian)(const ora_mech *m, int64_t n, const double *T, const double *P,
                      const double *Y, int64_t ldY, REAL *J, int64_t ldJ, int n_threads)
{
    return SFX(ora_jacobian_scaled)(m, n, T, P, Y, ldY, J, 0, ldJ, n_threads);
}

/* As ora_jacobian, and (if Jabs is not NULL) the gross scale of every entry,
 * the rounding-error scale for grading a Jacobian computed another way:
 *   rows k < NS:  S^J_kc = sum_j |nu_kj| (|d q_f,j / d x_c| + |d q_r,j / d x_c|)
 * with d/dx_c the total derivative with respect to x_c = Y_c or T (the
 * forward and reverse rates kept apart, so that their cancellation does not
 * shrink the scale);
 *   row NS (omega_T = -num/den): (|d num| |den| + |num| |d den|) / den^2 with
 *   |d num| = sum_k |Ru T h_k| S^J_kc (+ sum_k |Ru cp_k omega_k| for c = T) and
 *   |d den| = sum_k |Ru cp_k dC_k/dx_c| (+ sum_k |C_k Ru dcp_k| for c = T). */
int SFX(ora_jacobian_scaled)(const ora_mech *m, int64_t n, const double *T, const double *P,
                             const double *Y, int64_t ldY, REAL *J, REAL *Jabs, int64_t ldJ,
                             int n_threads)
{
    const int ns = m->ns, nr = m->nr, nv = ns + 1;
    int err = 0;
    /* the derivatives of [M] and of the falloff form are not implemented */
    for (int j = 0; j < nr; ++j)
        if (SFX(rtype1)(m, j) != ORA_ELEMENTARY) return -2;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel
#endif
    {
        REAL *buf = (REAL *)malloc(sizeof(REAL) * (10 * ns + 2 * ns * nv + 2 * nv * nv));
        if (!buf) {
            err = -1;
        } else {
            REAL *Yc = buf, *C = Yc + ns, *h = C + ns, *s = h + ns, *cp = s + ns, *dcp = cp + ns,
                 *om = dcp + ns, *dqdC = om + ns;     /* dqdC: [ns] per reaction */
            REAL *dCdx = dqdC + ns;                   /* [ns][nv] */
            REAL *Jc = dCdx + ns * nv;                /* [nv][nv] */
            REAL *Ja = Jc + nv * nv;                  /* [nv][nv] gross scale */
            REAL *dqfdC = Ja + nv * nv;               /* [ns] dq_f/dC_l */
            REAL *dqrdC = dqfdC + ns;                 /* [ns] dq_r/dC_l */
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
            for (int64_t i = 0; i < n; ++i) {
                REAL Ti = T[i], Pi = P[i];
                for (int k = 0; k < ns; ++k) { Yc[k] = Y[k * ldY + i]; om[k] = 0; }
                REAL sigma = SFX(concentrations)(m, Ti, Pi, Yc, C);
                REAL rho_hat = Pi / ((REAL)ORA_RU * Ti * sigma);
                for (int k = 0; k < ns; ++k)
                    SFX(thermo1)(m, k, Ti, &h[k], &s[k], &cp[k], &dcp[k]);
                /* dC_l/dx_c */
                for (int l = 0; l < ns; ++l) {
                    for (int c = 0; c < ns; ++c) {
                        REAL clamp_c = Yc[c] >= 0 ? 1 : 0;
                        REAL v = -C[l] / (sigma * (REAL)m->W[c]);
                        if (l == c) v += rho_hat / (REAL)m->W[c];
                        dCdx[l * nv + c] = v * clamp_c;
                    }
                    dCdx[l * nv + ns] = -C[l] / Ti;
                }
                for (int a = 0; a < nv * nv; ++a) Jc[a] = Ja[a] = 0;
                for (int j = 0; j < nr; ++j) {
                    REAL kf, Kc, qf, qr;
                    SFX(reaction1)(m, j, Ti, C, h, s, &kf, &Kc, &qf, &qr);
                    const int8_t *nf = &m->nu_f[j * ns], *nrr = &m->nu_r[j * ns];
                    int rev = (m->reversible == 0 || m->reversible[j]);
                    REAL kr = rev ? kf / Kc : 0;
                    REAL dn = 0, dH = 0;
                    for (int k = 0; k < ns; ++k) {
                        int nu = nrr[k] - nf[k];
                        dn += nu;
                        dH += nu * h[k];
                    }
                    REAL E_R = (REAL)m->Ea[j] * (REAL)ORA_CAL / (REAL)ORA_RU_MOL;
                    REAL dlnkf = ((REAL)m->beta[j] + E_R / Ti) / Ti;
                    REAL dlnKc = (dH - dn) / Ti;
                    /* explicit temperature dependence at fixed C */
                    REAL dqfdT = qf * dlnkf;
                    REAL dqrdT = rev ? qr * (dlnkf - dlnKc) : 0;
                    /* dq_f/dC_l and dq_r/dC_l, product rule on each power */
                    for (int l = 0; l < ns; ++l) {
                        dqfdC[l] = dqrdC[l] = 0;
                        if (nf[l]) {
                            REAL p = kf * (REAL)nf[l] * SFX(ipow)(C[l], nf[l] - 1);
                            for (int mm = 0; mm < ns; ++mm)
                                if (mm != l && nf[mm]) p *= SFX(ipow)(C[mm], nf[mm]);
                            dqfdC[l] = p;
                        }
                        if (nrr[l] && rev) {
                            REAL p = kr * (REAL)nrr[l] * SFX(ipow)(C[l], nrr[l] - 1);
                            for (int mm = 0; mm < ns; ++mm)
                                if (mm != l && nrr[mm]) p *= SFX(ipow)(C[mm], nrr[mm]);
                            dqrdC[l] = p;
                        }
                        dqdC[l] = dqfdC[l] - dqrdC[l];
                    }
                    REAL qn = qf - qr;
                    for (int k = 0; k < ns; ++k) {
                        int nu = nrr[k] - nf[k];
                        if (!nu) continue;
                        om[k] += nu * qn;
                        for (int c = 0; c < nv; ++c) {
                            /* total derivatives of q_f and q_r along x_c */
                            REAL gf = (c == ns) ? dqfdT : 0;
                            REAL gr = (c == ns) ? dqrdT : 0;
                            for (int l = 0; l < ns; ++l) {
                                if (dqfdC[l] != 0) gf += dqfdC[l] * dCdx[l * nv + c];
                                if (dqrdC[l] != 0) gr += dqrdC[l] * dCdx[l * nv + c];
                            }
                            Jc[k * nv + c] += nu * (gf - gr);
                            Ja[k * nv + c] += FABS((REAL)nu) * (FABS(gf) + FABS(gr));
                        }
                    }
                }
                /* last row: omega_T = -num/den */
                REAL num = 0, den = 0;
                for (int k = 0; k < ns; ++k) {
                    num += (REAL)ORA_RU * Ti * h[k] * om[k];
                    den += C[k] * (REAL)ORA_RU * cp[k];
                }
                for (int c = 0; c < nv; ++c) {
                    REAL dnum = 0, dden = 0, dnuma = 0, ddena = 0;
                    for (int k = 0; k < ns; ++k) {
                        dnum += (REAL)ORA_RU * Ti * h[k] * Jc[k * nv + c];
                        dden += (REAL)ORA_RU * cp[k] * dCdx[k * nv + c];
                        dnuma += FABS((REAL)ORA_RU * Ti * h[k]) * Ja[k * nv + c];
                        ddena += FABS((REAL)ORA_RU * cp[k] * dCdx[k * nv + c]);
                    }
                    if (c == ns) {
                        for (int k = 0; k < ns; ++k) {
                            dnum += (REAL)ORA_RU * cp[k] * om[k];   /* d h_k/dT = cp_k */
                            dden += C[k] * (REAL)ORA_RU * dcp[k];
                            dnuma += FABS((REAL)ORA_RU * cp[k] * om[k]);
                            ddena += FABS(C[k] * (REAL)ORA_RU * dcp[k]);
                        }
                    }
                    Jc[ns * nv + c] = -(dnum * den - num * dden) / (den * den);
                    Ja[ns * nv + c] = (dnuma * FABS(den) + FABS(num) * ddena) / (den * den);
                }
                REAL *Jo = &J[i * ldJ];
                for (int a = 0; a < nv * nv; ++a) Jo[a] = Jc[a];
                if (Jabs) {
                    REAL *Jao = &Jabs[i * ldJ];
                    for (int a = 0; a < nv * nv; ++a) Jao[a] = Ja[a];
                }
            }
            free(buf);
        }
    }
    return err;
}

/* 0-D constant-pressure adiabatic reactor, forward Euler (the paper's 0-D
 * ignition test, Sec. 3.1): per step, with omega from Eq. 2 and
 * omega_T = -sum_k H_k omega_k / sum_k C_k cp_k (molar enthalpy and heat
 * capacity from the NASA-7 polynomials),
 *     Y_k <- Y_k + dt W_k omega_k / rho,   T <- T + dt omega_T,
 * rho = sum_k C_k W_k the mass density.  T and Y are updated in place
 * (double in, the step evaluated in REAL, rounded back to double). */
int SFX(ora_integrate_euler)(const ora_mech *m, int64_t n, double *T, const double *P,
                             double *Y, int64_t ldY, double dt, int n_steps, int n_threads)
{
    const int ns = m->ns, nr = m->nr;
    int err = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel
#endif
    {
        REAL *buf = (REAL *)malloc(sizeof(REAL) * 5 * ns);
        if (!buf) {
            err = -1;
        } else {
            REAL *Yc = buf, *C = Yc + ns, *h = C + ns, *s = h + ns, *om = s + ns;
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
            for (int64_t i = 0; i < n; ++i) {
                REAL Ti = T[i];
                const REAL Pi = P[i];
                for (int k = 0; k < ns; ++k) Yc[k] = Y[k * ldY + i];
                for (int step = 0; step < n_steps; ++step) {
                    SFX(concentrations)(m, Ti, Pi, Yc, C);
                    for (int k = 0; k < ns; ++k) {
                        SFX(thermo1)(m, k, Ti, &h[k], &s[k], 0, 0);
                        om[k] = 0;
                    }
                    for (int j = 0; j < nr; ++j) {
                        REAL kf, Kc, qf, qr;
                        SFX(reaction1)(m, j, Ti, C, h, s, &kf, &Kc, &qf, &qr);
                        const int8_t *nf = &m->nu_f[j * ns], *nrr = &m->nu_r[j * ns];
                        for (int k = 0; k < ns; ++k) {
                            int nu = nrr[k] - nf[k];
                            if (nu) om[k] += nu * (qf - qr);
                        }
                    }
                    REAL num = 0, den = 0, rho = 0;
                    for (int k = 0; k < ns; ++k) {
                        REAL cp;
                        SFX(thermo1)(m, k, Ti, 0, 0, &cp, 0);
                        num += (REAL)ORA_RU * Ti * h[k] * om[k];
                        den += C[k] * (REAL)ORA_RU * cp;
                        rho += C[k] * (REAL)m->W[k];
                    }
                    const REAL omT = -num / den;
                    for (int k = 0; k < ns; ++k) Yc[k] += (REAL)dt * (REAL)m->W[k] * om[k] / rho;
                    Ti += (REAL)dt * omT;
                }
                T[i] = (double)Ti;
                for (int k = 0; k < ns; ++k) Y[k * ldY + i] = (double)Yc[k];
            }
            free(buf);
        }
    }
    return err;
}

/* Solve A x = b in place for one dense system of order nv (A row-major,
 * overwritten), Gaussian elimination with partial pivoting (the largest
 * remaining |A[i][k]| in column k becomes the pivot); b becomes x.
 * Returns -1 for a zero pivot. */
static int SFX(gauss_solve)(int nv, REAL *A, REAL *b)
{
    for (int k = 0; k < nv; ++k) {
        int p = k;
        for (int i = k + 1; i < nv; ++i)
            if (FABS(A[i * nv + k]) > FABS(A[p * nv + k])) p = i;
        if (A[p * nv + k] == 0) return -1;
        if (p != k) {
            for (int c = 0; c < nv; ++c) {
                REAL t = A[k * nv + c];
                A[k * nv + c] = A[p * nv + c];
                A[p * nv + c] = t;
            }
            REAL t = b[k];
            b[k] = b[p];
            b[p] = t;
        }
        for (int i = k + 1; i < nv; ++i) {
            REAL l = A[i * nv + k] / A[k * nv + k];
            if (l == 0) continue;
            for (int c = k; c < nv; ++c) A[i * nv + c] -= l * A[k * nv + c];
            b[i] -= l * b[k];
        }
    }
    for (int k = nv - 1; k >= 0; --k) {
        REAL v = b[k];
        for (int c = k + 1; c < nv; ++c) v -= A[k * nv + c] * b[c];
        b[k] = v / A[k * nv + k];
    }
    return 0;
}

/* 0-D constant-pressure reactor, linearly implicit Euler steps (the stiff
 * integration the paper names as the next step, Sec. 4): with x = (Y, T),
 *     f(x) = (W_k omega_k / rho, omega_T),
 *     (I - dt Jf) dx = dt f(x),   x <- x + dx,
 * where Jf has the rows (W_k / rho) d omega_k / dx and d omega_T / dx from
 * the analytic Jacobian (ora_jacobian), rho held at its value at x (a
 * W-method: the step is first-order accurate with any such matrix, and with
 * Jf exact it is one Newton iteration of backward Euler).  P is fixed; the
 * state is carried in double between steps.  Cells run one after another.
 * Returns -2 for mechanisms the Jacobian does not cover, -3 for a singular
 * system. */
int SFX(ora_integrate_implicit)(const ora_mech *m, int64_t n, double *T, const double *P,
                                double *Y, int64_t ldY, double dt, int n_steps)
{
    const int ns = m->ns, nv = ns + 1;
    REAL *J = (REAL *)malloc(sizeof(REAL) * (nv * nv * 2 + 4 * nv));
    double *Yc = (double *)malloc(sizeof(double) * ns);
    if (!J || !Yc) { free(J); free(Yc); return -1; }
    REAL *A = J + nv * nv, *b = A + nv * nv, *om = b + nv, *C = om + nv;
    int rc = 0;
    for (int64_t i = 0; i < n && !rc; ++i) {
        double Ti = T[i], Pi = P[i];
        for (int k = 0; k < ns; ++k) Yc[k] = Y[k * ldY + i];
        for (int step = 0; step < n_steps && !rc; ++step) {
            REAL omT;
            if ((rc = SFX(ora_jacobian)(m, 1, &Ti, &Pi, Yc, 1, J, nv * nv, 1))) break;
            if ((rc = SFX(ora_source)(m, 1, &Ti, &Pi, Yc, 1, om, 0, 0, 1, 1))) break;
            if ((rc = SFX(ora_temp_source)(m, 1, &Ti, &Pi, Yc, 1, &omT, 1))) break;
            /* rho = sum_k C_k W_k at the current state */
            REAL rho = 0, sum = 0;
            for (int k = 0; k < ns; ++k) {
                REAL y = Yc[k] > 0 ? (REAL)Yc[k] : 0;
                sum += y / (REAL)m->W[k];
            }
            for (int k = 0; k < ns; ++k) {
                REAL y = Yc[k] > 0 ? (REAL)Yc[k] : 0;
                C[k] = (REAL)Pi / ((REAL)ORA_RU * (REAL)Ti * sum) * y / (REAL)m->W[k];
                rho += C[k] * (REAL)m->W[k];
            }
            for (int r = 0; r < nv; ++r) {
                REAL s = r < ns ? (REAL)m->W[r] / rho : 1;
                for (int c = 0; c < nv; ++c)
                    A[r * nv + c] = (r == c ? 1 : 0) - (REAL)dt * s * J[r * nv + c];
                b[r] = (REAL)dt * (r < ns ? s * om[r] : omT);
            }
            if (SFX(gauss_solve)(nv, A, b)) { rc = -3; break; }
            for (int k = 0; k < ns; ++k) Yc[k] = (double)((REAL)Yc[k] + b[k]);
            Ti = (double)((REAL)Ti + b[ns]);
        }
        T[i] = Ti;
        for (int k = 0; k < ns; ++k) Y[k * ldY + i] = Yc[k];
    }
    free(J);
    free(Yc);
    return rc;
}
