/*
 * Test oracle for the batched chemical source term of Barwey & Raman,
 * "A Neural Network Inspired Formulation of Chemical Kinetics" (Sec. 2).
 *
 * TEST INFRASTRUCTURE ONLY: a plain, slow, per-cell CPU evaluation of the
 * law-of-mass-action definition, used to check the HIP library.  Only the
 * tests, the smoke check and the CPU-baseline leg of the benchmark may load
 * it; the library never does, and the two share no code.
 *
 * Every function exists twice: *_f64 computes in double, *_ld in x86
 * extended precision (long double), the reference for grading the FP64 GPU
 * path.  Inputs are always double.
 */
#ifndef ORACLE_H
#define ORACLE_H
#include <stdint.h>

/* Gas constant in J/(kmol K) and J/(mol K); thermochemical calorie in J;
 * reference pressure 1 bar in Pa (the paper states p_ref = 1 bar, Eq. 8). */
#define ORA_RU 8314.46261815324L
#define ORA_RU_MOL 8.31446261815324L
#define ORA_CAL 4.184L
#define ORA_PREF 1.0e5L

/* Mechanism as a mechanism file carries it (all arrays host, row-major):
 *   W[ns] kg/kmol; nu_f, nu_r [nr][ns] (entry [j][k] = nu'_kj, nu''_kj);
 *   ln_A[nr] natural log of A in cgs units (cm^3/mol)^(order-1)/s;
 *   beta[nr]; Ea[nr] cal/mol; nasa_low, nasa_high [ns][7] a1..a7;
 *   T_mid[ns] K; reversible[nr] (NULL = all reversible);
 * pressure-dependent reactions (Sec. 2.4), all NULL for none:
 *   rtype[nr] 0 elementary, 1 third body (+M), 2 falloff (Lindemann),
 *     3 falloff (Troe); eff[nr][ns] third-body efficiencies (NULL = all 1);
 *   for types 2 and 3 the arrays ln_A, beta, Ea give the high-pressure limit
 *   and low_ln_A, low_beta, low_Ea the low-pressure limit k0 (A in cgs units
 *   of one order more); troe[nr][4] = alpha, T3, T1, T2 (the usual T-triple-
 *   star, T-star, T-double-star; T2 = 0: the third term is absent).  Third-body reactions carry A in cgs units of
 *   order sum nu' + 1. */
typedef struct {
    int ns, nr;
    const double *W;
    const int8_t *nu_f, *nu_r;
    const double *ln_A, *beta, *Ea;
    const double *nasa_low, *nasa_high, *T_mid;
    const uint8_t *reversible;
    const uint8_t *rtype;
    const double *eff;
    const double *low_ln_A, *low_beta, *low_Ea;
    const double *troe;
} ora_mech;

#define ORA_ELEMENTARY 0
#define ORA_THIRD_BODY 1
#define ORA_LINDEMANN 2
#define ORA_TROE 3

#define ORA_DECL(R, S)                                                                        \
    int ora_thermo_##S(const ora_mech *m, double T, R *h_RT, R *s_R, R *cp_R);                \
    int ora_rates_##S(const ora_mech *m, double T, double P, const double *Y, R *C, R *kf,    \
                      R *Kc, R *qf, R *qr);                                                   \
    int ora_source_##S(const ora_mech *m, int64_t n, const double *T, const double *P,       \
                       const double *Y, int64_t ldY, R *omega, R *S, R *N, int64_t ldO,       \
                       int n_threads);                                                        \
    int ora_temp_source_##S(const ora_mech *m, int64_t n, const double *T, const double *P,  \
                            const double *Y, int64_t ldY, R *omega_T, int n_threads);          \
    int ora_jacobian_##S(const ora_mech *m, int64_t n, const double *T, const double *P,     \
                         const double *Y, int64_t ldY, R *J, int64_t ldJ, int n_threads);      \
    int ora_integrate_euler_##S(const ora_mech *m, int64_t n, double *T, const double *P,      \
                                double *Y, int64_t ldY, double dt, int n_steps, int n_threads); \
    int ora_jacobian_scaled_##S(const ora_mech *m, int64_t n, const double *T,                 \
                                const double *P, const double *Y, int64_t ldY, R *J, R *Jabs,  \
                                int64_t ldJ, int n_threads);                                   \
    int ora_lnkc_##S(const ora_mech *m, int64_t n, const double *T, R *lnK, int64_t ldK);       \
    int ora_source_lnkc_##S(const ora_mech *m, int64_t n, const double *T, const double *P,    \
                            const double *Y, int64_t ldY, const double *lnK, int64_t ldK,      \
                            R *omega, R *S, R *N, int64_t ldO, int n_threads);          \
    int ora_integrate_implicit_##S(const ora_mech *m, int64_t n, double *T, const double *P,   \
                                   double *Y, int64_t ldY, double dt, int n_steps);

ORA_DECL(double, f64)
ORA_DECL(long double, ld)

#endif
