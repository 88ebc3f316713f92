/*
 * annkin: batched chemical source terms on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libannkin.so.  The library evaluates, for a batch of N_C
 * reacting cells, the net molar production rates of Barwey & Raman,
 * "A Neural Network Inspired Formulation of Chemical Kinetics":
 *
 *   omega_k = sum_j nu_kj (q_f,j - q_r,j)                        (Eq. 2)
 *   q_f,j = exp(sum_k nu'_kj ln C_k + ln k_f,j),
 *   q_r,j = exp(sum_k nu''_kj ln C_k + ln k_f,j - ln K_c,j)      (Eq. 4, Eq. 7)
 *   ln k_f,j = ln A_j + beta_j ln T - (E_j/R)/T                  (Eq. 6)
 *   ln K_c,j = -sum_k nu_kj (G_k - ln(p_ref/(R T)))              (Eqs. 9-11)
 *
 * with G_k = H_k/(RT) - S_k/R from NASA 7-coefficient polynomials (Eq. 10)
 * and p_ref = 1 bar.  The batch dimension N_C is the leading (fastest)
 * dimension of every per-cell array (Sec. 2.1).
 *
 * Conventions for every entry point:
 *  - Return 0 on success or a negative AK_E* code; ak_last_error() then
 *    returns a message for the calling thread.
 *  - State and result pointers are DEVICE pointers on the mechanism's
 *    device, owned by the caller, of the element type the precision
 *    selects (AK_FP32: float, AK_FP64: double).
 *  - Calls are asynchronous on `stream` (a hipStream_t passed as void*;
 *    NULL is the null stream).  Argument errors are reported synchronously,
 *    before anything is enqueued.  Concurrent calls on different streams
 *    are allowed.
 *  - Units: T in K, P in Pa, Y mass fractions (need not sum to one;
 *    negative values count as zero), omega in kmol m^-3 s^-1.
 *  - Layout: Y[k*ldY + i] for species k and cell i (ldY >= n_cells), and
 *    likewise for omega with ldO.
 *  - A cell with non-finite input, T <= 0 or P <= 0 gets NaN outputs and is
 *    counted on the mechanism's device-side error counter (ak_error_count).
 *  - n_cells == 0 is a no-op.
 */
#ifndef ANNKIN_H
#define ANNKIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AK_OK 0
#define AK_EINVAL (-1)       /* bad argument (null pointer, size, enum, layout) */
#define AK_EDEVICE (-2)      /* HIP runtime error; message in ak_last_error() */
#define AK_ENOMEM (-3)       /* device or host allocation failed */
#define AK_E2BIG (-4)        /* request larger than a configured limit */
#define AK_ETIMEDOUT (-5)    /* wait timed out */
#define AK_ECANCELED (-6)    /* request was cancelled */
#define AK_EUNSUPPORTED (-7) /* mechanism feature outside what the kernels handle */

typedef enum { AK_FP64 = 0, AK_FP32 = 1 } ak_precision;

typedef struct ak_mechanism ak_mechanism; /* opaque; owns its device tables */

/*
 * Mechanism as a CHEMKIN-style file carries it (Sec. 2, Eq. 1; Eq. 5;
 * Eq. 10; Sec. 2.4 for the pressure-dependent reactions).  All pointers are
 * HOST arrays owned by the caller and copied during ak_load_mechanism;
 * row-major.
 *   W          [NS]      molecular weights, kg/kmol (> 0)
 *   nu_f, nu_r [NR][NS]  reactant / product stoichiometric coefficients
 *                        nu'_kj, nu''_kj at [j*NS + k] (>= 0)
 *   ln_A       [NR]      ln of the pre-exponential factor in cgs units,
 *                        (cm^3/mol)^(order-1)/s, order = sum_k nu'_kj (one
 *                        more for a third-body reaction); for a falloff
 *                        reaction the high-pressure limit
 *   beta       [NR]      temperature exponent
 *   Ea         [NR]      activation energy, cal/mol
 *   nasa_low, nasa_high [NS][7]  NASA-7 coefficients a1..a7 below / at and
 *                        above T_mid
 *   T_mid      [NS]      range switch temperature, K
 *   reversible [NR]      1 = reversible, 0 = irreversible (the indicator of
 *                        Sec. 2.4); NULL means all reversible
 *   rtype      [NR]      AK_RXN_* (Sec. 2.4); NULL means all elementary
 *   efficiency [NR][NS]  third-body efficiencies eff_kj of the third-body
 *                        concentration [M]_j = sum_k eff_kj C_k (the paper's
 *                        M = C E); read for rows with rtype != 0; NULL means
 *                        all 1.  Finite and >= 0.
 *   low_ln_A, low_beta, low_Ea [NR]  low-pressure limit k_0 of falloff
 *                        reactions (A in cgs units of order sum nu' + 1);
 *                        read for rows with rtype AK_RXN_LINDEMANN or
 *                        AK_RXN_TROE (may be NULL if there are none)
 *   troe       [NR][4]   Troe parameters alpha, T3, T1, T2 (the usual T***,
 *                        T*, T**; T3, T1 > 0; T2 = 0 leaves the exp(-T2/T)
 *                        term out); read for AK_RXN_TROE rows
 * Falloff rate constants are k = k_inf Pr/(1 + Pr) F with
 * Pr = k_0 [M] / k_inf and F = 1 (Lindemann) or the Troe broadening
 * log10 F = log10 Fc / (1 + ((log10 Pr + c)/(n - 0.14 (log10 Pr + c)))^2),
 * c = -0.4 - 0.67 log10 Fc, n = 0.75 - 1.27 log10 Fc,
 * Fc = (1 - alpha) exp(-T/T3) + alpha exp(-T/T1) + exp(-T2/T).
 * Third-body and falloff reactions are evaluated by the compiled kernels
 * only: a mechanism with them needs AK_KERNEL_AUTO and a size the compiled
 * kernels take, and ak_eval_jacobian / ak_eval_vjp return AK_EUNSUPPORTED
 * for it.
 * Limits: NS >= 1 and NR >= 1 (else AK_EINVAL); NS <= 256, at most 4
 * reactant and 4 product molecules per reaction counting multiplicity
 * (sum of nu' <= 4, sum of nu'' <= 4), and a 16-cell LDS tile of
 * 24 * NS bytes per cell must fit the device (NS <= 426 on gfx950);
 * otherwise AK_EUNSUPPORTED.
 */
#define AK_RXN_ELEMENTARY 0
#define AK_RXN_THIRD_BODY 1 /* k [M] */
#define AK_RXN_LINDEMANN 2  /* falloff, F = 1 */
#define AK_RXN_TROE 3       /* falloff, Troe broadening */

typedef struct {
    int32_t n_species;
    int32_t n_reactions;
    const double *W;
    const int8_t *nu_f;
    const int8_t *nu_r;
    const double *ln_A;
    const double *beta;
    const double *Ea;
    const double *nasa_low;
    const double *nasa_high;
    const double *T_mid;
    const uint8_t *reversible;
    const uint8_t *rtype;
    const double *efficiency;
    const double *low_ln_A;
    const double *low_beta;
    const double *low_Ea;
    const double *troe;
} ak_mechanism_desc;

/* Thread-local message describing the last error on this thread. */
const char *ak_last_error(void);

/* Library version string. */
const char *ak_version(void);

/*
 * Convert and upload a mechanism to `device` (HIP ordinal): rate parameters
 * to SI-kmol units and base-2 logarithms, NASA coefficients to the
 * Gibbs-layer weights of Eq. 11 with the standard concentration folded in,
 * and the stoichiometry to per-reaction factor lists.  Where the mechanism
 * is small enough for one lane to hold a cell's whole state in registers
 * (NS <= 64 for AK_FP32, NS <= 53 for AK_FP64), its source-term kernels are
 * also generated with the stoichiometry written into the code and compiled
 * for the device (hiprtc; a few seconds per precision, cached by text in
 * the process and on disk under $AK_JIT_CACHE_DIR or $HOME/.cache/annkin,
 * "off" disables the disk cache).  Larger mechanisms use the table-driven
 * kernels.  The call is synchronous.  On success *out owns device memory
 * until ak_free_mechanism.
 * Errors: AK_EINVAL (null/invalid desc), AK_EUNSUPPORTED, AK_EDEVICE
 * (including a failed compilation), AK_ENOMEM.
 */
int ak_load_mechanism(const ak_mechanism_desc *desc, int device, ak_mechanism **out);

/* Kernel choice of ak_load_mechanism_ex. */
#define AK_KERNEL_AUTO 0   /* mechanism-compiled kernels where they fit (the default) */
#define AK_KERNEL_TABLE 1  /* the table-driven kernels only (no compilation) */

/* ak_load_mechanism with an explicit kernel choice (AK_KERNEL_*). */
int ak_load_mechanism_ex(const ak_mechanism_desc *desc, int device, int kernels,
                         ak_mechanism **out);

/* 1 if ak_eval_source runs the mechanism-compiled kernel for this
 * precision, 0 if the table-driven one, negative on bad arguments. */
int ak_mechanism_compiled(const ak_mechanism *mech, ak_precision prec);

/* 1 if the mechanism has a compiled state Jacobian (what
 * ak_eval_jacobian_interleaved needs and ak_eval_jacobian runs unless the
 * environment variable AK_JIT_JACOBIAN=0 is set), 0 if not, negative on
 * bad arguments.  The same for both precisions. */
int ak_mechanism_compiled_jacobian(const ak_mechanism *mech, ak_precision prec);

/*
 * Diagnostic, no device needed: the HIP source text the library generates
 * for a mechanism and precision (what ak_load_mechanism compiles).  Writes
 * at most cap bytes including the terminating NUL into buf (buf may be NULL
 * with cap 0) and the full size including the NUL into *needed.
 * Errors: as ak_load_mechanism's argument checks.
 */
int ak_jit_source(const ak_mechanism_desc *desc, ak_precision prec, char *buf, size_t cap,
                  size_t *needed);

/*
 * Diagnostic, no device needed: the constant tables the generated kernels
 * of ak_jit_source read (per species 16 doubles: 1/W, T_mid, the low- and
 * high-range Gibbs-layer weights; per reaction the Arrhenius layer and, for
 * falloff reactions, the low-pressure and Troe constants, in the order of
 * the generated code).  Copies at most cap_sp / cap_rx doubles into sp / rx
 * (either may be NULL with cap 0) and the full counts into *n_sp / *n_rx.
 * Errors: as ak_jit_source.
 */
int ak_jit_tables(const ak_mechanism_desc *desc, ak_precision prec, double *sp, size_t cap_sp,
                  double *rx, size_t cap_rx, size_t *n_sp, size_t *n_rx);

/*
 * Diagnostic, no device needed: the HIP source text of a derivative kernel
 * compiled for a mechanism, what the first call for the mechanism and
 * precision compiles: variant 0 ak_eval_jacobian's, 1
 * ak_eval_jacobian_interleaved's, 2 ak_eval_vjp's.  Same buffer convention
 * as ak_jit_source.  Errors: as ak_jit_source, plus AK_EINVAL for another
 * variant and AK_EUNSUPPORTED for a mechanism without compiled derivatives
 * (third-body or falloff reactions, more species than the compiled form
 * takes).
 */
int ak_jit_jacobian_source(const ak_mechanism_desc *desc, ak_precision prec, int variant,
                           char *buf, size_t cap, size_t *needed);

/*
 * Diagnostic, no device needed: the constant tables of that kernel (the same
 * for both precisions): per species 32 doubles (1/W, T_mid, the Gibbs-layer
 * weights of both ranges with log2(1/W) in the biases, the NASA-7 sets
 * a1..a7 low then high, two zeros); per reaction 4 doubles (log2 A less the
 * reactants' log2 W, beta, -(E/R) log2 e, E/R).  Buffer convention and
 * errors as ak_jit_tables / ak_jit_jacobian_source.
 */
int ak_jit_jacobian_tables(const ak_mechanism_desc *desc, double *sp, size_t cap_sp, double *rx,
                           size_t cap_rx, size_t *n_sp, size_t *n_rx);

/* Free a mechanism.  The caller must ensure no enqueued work still uses it
 * (synchronise the streams first).  NULL is a no-op. */
int ak_free_mechanism(ak_mechanism *mech);

/* Number of species / reactions of a loaded mechanism (or -1 for NULL). */
int ak_mechanism_n_species(const ak_mechanism *mech);
int ak_mechanism_n_reactions(const ak_mechanism *mech);

/*
 * Net production rates omega (Eq. 2 with the rates of Eq. 4) for n_cells
 * cells.  T[n_cells], P[n_cells], Y[NS][ldY] in; omega[NS][ldO] out.
 * AK_FP32 takes float states and returns float omega; internally the
 * chemical potentials and the forward/reverse difference are evaluated in
 * double precision and the rate exponentials in single precision.
 * AK_FP64 is double throughout.
 * Errors: AK_EINVAL (null pointers with n_cells > 0, n_cells < 0,
 * ldY or ldO < n_cells, bad precision), AK_EDEVICE (launch failure).
 */
int ak_eval_source(const ak_mechanism *mech, ak_precision prec, const void *T, const void *P,
                   const void *Y, int64_t ldY, int64_t n_cells, void *omega, int64_t ldO,
                   void *stream);

/*
 * Dense Jacobian of the state source with respect to x = (Y_1..Y_NS, T) at
 * fixed P, per cell: rows 0..NS-1 are d omega_k / dx (kmol m^-3 s^-1 per unit
 * mass fraction, per K), row NS is d omega_T / dx with
 * omega_T = -sum_k h_k omega_k / sum_k C_k cp_k (K/s) the constant-pressure
 * temperature source (h_k molar enthalpy, cp_k molar heat capacity from the
 * NASA-7 polynomials).  This is the matrix an implicit integrator of the
 * paper's source term (Eq. 2) needs.  Output J is [n_cells][NS+1][NS+1],
 * row-major per cell, cells outermost with stride ldJ >= (NS+1)^2 elements;
 * float for AK_FP32, double for AK_FP64 (both evaluate in double).  Where
 * Y_m < 0 the column of Y_m is zero (the clamp); at Y_m = 0 the one-sided
 * derivative from above is returned.
 * Mechanisms of elementary reactions that fit one 64-cell tile's LDS (see
 * ak_eval_jacobian_interleaved; 53 species and 325 reactions do) use a kernel
 * compiled for the mechanism (one 64-cell tile per workgroup, every sum in
 * a fixed order: results are bitwise reproducible); it is generated and
 * compiled at the first call for the mechanism and precision (seconds; the
 * code object is cached like the source-term kernels'), which also makes
 * one small device allocation for its tables, freed with the mechanism.
 * Larger mechanisms, or the environment variable AK_JIT_JACOBIAN=0, use the
 * table-driven kernel (one cell per workgroup, LDS atomics: the summation
 * order, and so the last bits, may vary between runs).
 * Errors: as ak_eval_source, plus AK_EINVAL for ldJ < (NS+1)^2,
 * AK_EUNSUPPORTED when neither kernel takes the mechanism (the table-driven
 * one needs (NS+1)^2 + 11 NS + 257 doubles in one workgroup's LDS: NS <= 135
 * on gfx950), AK_EDEVICE / AK_ENOMEM when compiling or loading the compiled
 * kernel fails.
 */
int ak_eval_jacobian(const ak_mechanism *mech, ak_precision prec, const void *T, const void *P,
                     const void *Y, int64_t ldY, int64_t n_cells, void *J, int64_t ldJ,
                     void *stream);

/*
 * The same Jacobian in the interleaved (cell-minor) layout a batched solver
 * with one lane per cell reads: entry (r, c) of cell i at
 * J[(r * (NS+1) + c) * ldJ + i], ldJ >= n_cells, like Y and omega (species
 * outermost).  Consecutive cells are adjacent, so the kernel's stores are
 * contiguous across a wavefront; the cell-major layout of ak_eval_jacobian
 * scatters them by the cell stride, which caps its write bandwidth.  Always
 * the kernel compiled for the mechanism (generated and compiled at the first
 * call for the mechanism and precision, as for ak_eval_jacobian), bitwise
 * the same values as ak_eval_jacobian's compiled kernel.
 * Errors: as ak_eval_source, plus AK_EINVAL for ldJ < n_cells,
 * AK_EUNSUPPORTED for a mechanism without a compiled Jacobian (third-body or
 * falloff reactions; more species than fit one 64-cell tile's LDS:
 * 5 * 512 NS + 8 max(4 NR, 1024) + 12288 bytes <= 160 KB, and NS <= 64),
 * AK_EDEVICE / AK_ENOMEM when compiling or loading it fails.
 */
int ak_eval_jacobian_interleaved(const ak_mechanism *mech, ak_precision prec, const void *T,
                                 const void *P, const void *Y, int64_t ldY, int64_t n_cells,
                                 void *J, int64_t ldJ, void *stream);

/*
 * Vector-Jacobian product of omega (Eq. 2) with respect to (Y, T) at fixed P:
 * given g_omega [NS][ldG], returns g_Y[m] = sum_k g_omega_k d omega_k / dY_m
 * ([NS][ldGY]) and g_T = sum_k g_omega_k d omega_k / dT ([n_cells]), without
 * forming the Jacobian.  Same clamp convention as ak_eval_jacobian.
 * Mechanisms with a compiled Jacobian (ak_mechanism_compiled_jacobian) use a
 * kernel compiled the same way: with gamma_j = sum_k g_omega_k nu_kj every
 * wave of a 64-cell tile sweeps a share of the reactions once and the
 * waves' sums are added in a fixed order, so results are bitwise
 * reproducible (compiled at the first call, as for ak_eval_jacobian).
 * Others, or AK_JIT_VJP=0, use the table-driven kernel (LDS atomics).
 * Errors: as ak_eval_source, plus AK_EINVAL for ldG or ldGY < n_cells,
 * AK_EDEVICE / AK_ENOMEM when compiling or loading the compiled kernel fails.
 */
int ak_eval_vjp(const ak_mechanism *mech, ak_precision prec, const void *T, const void *P,
                const void *Y, int64_t ldY, int64_t n_cells, const void *g_omega, int64_t ldG,
                void *g_Y, int64_t ldGY, void *g_T, void *stream);

/*
 * 0-D constant-pressure adiabatic reactor (the paper's 0-D ignition test,
 * Sec. 3.1): advances every cell's (T, Y) in place by n_steps forward-Euler
 * steps of dt seconds at its fixed P,
 *     Y_k <- Y_k + dt W_k omega_k / rho,   T <- T + dt omega_T,
 * with omega from Eq. 2 (the same kernels as ak_eval_source), rho the mass
 * density and omega_T = -sum_k H_k omega_k / sum_k C_k cp_k (molar enthalpy
 * and heat capacity from the NASA-7 polynomials).  T[n], P[n] and
 * Y[NS][ldY] are device arrays of the precision's type; T and Y are
 * overwritten.  Forward Euler is stable only for dt below the fastest
 * chemical time scale (1/|largest Jacobian eigenvalue|).  Uses a scratch
 * buffer of NS * n_cells elements for omega, allocated and freed
 * stream-ordered (hipMallocAsync) within the call.  Asynchronous on stream.
 * Errors: as ak_eval_source, plus AK_EINVAL for dt <= 0 or non-finite and
 * n_steps < 0, AK_ENOMEM.
 */
int ak_integrate_euler(const ak_mechanism *mech, ak_precision prec, void *T, const void *P,
                       void *Y, int64_t ldY, int64_t n_cells, double dt, int n_steps,
                       void *stream);

/*
 * The same reactor advanced by n_steps linearly implicit Euler steps (the
 * stiff integration Sec. 4 calls for), each using the state Jacobian: with
 * x = (Y, T) and f(x) = (W_k omega_k / rho, omega_T),
 *     (I - dt Jf) dx = dt f(x),   x <- x + dx,
 * where Jf has the rows (W_k / rho) d omega_k / dx and d omega_T / dx
 * (ak_eval_jacobian) and rho is held at the step's start.  A step stays
 * bounded far beyond the explicit stability limit and conserves total mass
 * fraction and elements.  Per step: the Jacobian and omega into scratch
 * (n_cells ((NS+1)^2 + NS) elements, allocated and freed stream-ordered),
 * then one workgroup per cell solves its (NS+1) x (NS+1) system in LDS
 * (Gaussian elimination with partial pivoting, fixed reduction order).  A
 * cell whose system is singular or whose state is bad gets NaN and is
 * counted (ak_error_count).  Errors: as ak_integrate_euler, AK_EUNSUPPORTED
 * for mechanisms ak_eval_jacobian does not take (third-body or falloff
 * reactions) or systems larger than the LDS, AK_ENOMEM.
 */
int ak_integrate_implicit(const ak_mechanism *mech, ak_precision prec, void *T, const void *P,
                          void *Y, int64_t ldY, int64_t n_cells, double dt, int n_steps,
                          void *stream);

/*
 * ak_integrate_euler without any allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid it).  Same arguments, results and errors; the
 * scratch for omega is a 64 MiB device array inside the library, one per GPU
 * (present from the library's load until the process ends), so
 * NS * n_cells * element size may not exceed 64 MiB (else AK_E2BIG; e.g.
 * 158,275 cells at 53 species FP64).  Every call on one GPU uses that GPU's
 * array: calls that overlap on one GPU (other threads or streams) race and
 * must be serialised by the caller.  The array needs no clearing: each step
 * overwrites it before reading it.
 */
int ak_integrate_euler_noalloc(const ak_mechanism *mech, ak_precision prec, void *T,
                               const void *P, void *Y, int64_t ldY, int64_t n_cells, double dt,
                               int n_steps, void *stream);

/*
 * Read and reset the number of bad cells (non-finite input, T <= 0 or
 * P <= 0) seen by all evaluations with this mechanism since the last call.
 * Synchronises `stream`.  Errors: AK_EINVAL, AK_EDEVICE.
 */
int ak_error_count(const ak_mechanism *mech, void *stream, int64_t *n_bad_cells);

/* ------------------------------------------------------------------------
 * The equilibrium constant on its own, and a trained network in its place
 * (Sec. 2.3).  ln K_c is in natural-log units of (kmol m^-3)^dn, stored
 * reaction-major and cell-minor: lnK[j*ldK + i] for reaction j (descriptor
 * order) and cell i, ldK >= n_cells, of the precision's element type.
 */

/*
 * ln K_c of every reaction from the Gibbs layer and the net stoichiometric
 * layer (Eqs. 9-11): ln K_c,j = -sum_k nu_kj (G_k - ln(p_ref/(R T))), with
 * the NASA-7 range chosen per species and cell.  The two linear layers are
 * composed per reaction and temperature interval (the intervals between the
 * distinct T_mid of its species; at most 3 such T_mid per reaction, else
 * the layers run separately, the Gibbs outputs in LDS).  The arithmetic is
 * double in both precisions (AK_FP32 rounds the result).  A cell with
 * T <= 0 or non-finite T gets NaN and is counted (ak_error_count).
 * Errors: AK_EINVAL, AK_EUNSUPPORTED (the separate form with more species
 * than the LDS holds: 8 * 64 bytes each), AK_EDEVICE.
 */
int ak_eval_lnkc(const ak_mechanism *mech, ak_precision prec, const void *T, int64_t n_cells,
                 void *lnK, int64_t ldK, void *stream);

#define AK_KCNET_MAX_LAYERS 16
#define AK_KCNET_MAX_HIDDEN 64

/*
 * The approximate ln K_c network of Sec. 2.3, Architecture 2 (Fig. 2): input
 * the standardized log temperature x = (ln T - x_mean) / x_std, then n_layers
 * hidden layers of n_hidden neurons, X_{l+1} = elu(X_l W_l + B_l) (Eqs. 12
 * and 14), then a linear readout to n_out standardized outputs y, and
 * ln K_c,j = y_j y_std[j] + y_mean[j].  Row-major matrices, input index
 * first (X W):
 *   weights = W_0 [1][n_hidden], W_1 .. W_{n_layers-1} [n_hidden][n_hidden],
 *             W_{n_layers} [n_hidden][n_out], concatenated;
 *   biases  = B_0 .. B_{n_layers-1} [n_hidden], B_{n_layers} [n_out].
 * Host arrays, read during ak_load_kcnet only.
 */
typedef struct {
    int32_t n_layers;   /* N_L hidden layers, 1 .. AK_KCNET_MAX_LAYERS */
    int32_t n_hidden;   /* N_H neurons per hidden layer, 1 .. AK_KCNET_MAX_HIDDEN */
    int32_t n_out;      /* N_R outputs, one per reaction */
    int32_t pad;
    const double *weights;
    const double *biases;
    double x_mean, x_std;              /* standardization of ln T (x_std > 0) */
    const double *y_mean, *y_std;      /* [n_out] standardization of ln K_c */
} ak_kcnet_desc;

typedef struct ak_kcnet ak_kcnet; /* opaque; owns its device weights */

/*
 * Copy a network's weights to `device` (in double and in float; widths
 * below 64 are padded with zero weights to 8, 16, 32 or 64).  The output
 * standardization is folded into the readout.  Errors: AK_EINVAL (sizes,
 * non-finite values, x_std <= 0), AK_EDEVICE.
 */
int ak_load_kcnet(const ak_kcnet_desc *desc, int device, ak_kcnet **out);
int ak_free_kcnet(ak_kcnet *net);
int ak_kcnet_n_out(const ak_kcnet *net);

/*
 * ln K_c from the network for n_cells temperatures, one cell per lane with
 * its activations in registers.  AK_FP64 evaluates in double; AK_FP32 in
 * float (ln T in double, then standardized and rounded).  Each output is a
 * sum in a fixed order, so repeated calls agree bitwise.  A cell with
 * T <= 0 or non-finite T gets NaN (there is no counter for networks).
 * Errors: AK_EINVAL, AK_EDEVICE.
 */
int ak_eval_lnkc_net(const ak_kcnet *net, ak_precision prec, const void *T, int64_t n_cells,
                     void *lnK, int64_t ldK, void *stream);

/*
 * The source term (Eqs. 2-7) with ln K_c of reaction j in cell i taken from
 * lnK[j*ldK + i] in place of Eq. 8: q_r = k_f exp(-ln K_c) prod C^nu''.
 * Irreversible reactions do not read lnK.  Arguments otherwise as
 * ak_eval_source.  The arithmetic is double in both precisions; the
 * accumulation order is fixed (bitwise reproducible).  Errors: AK_EINVAL,
 * AK_EUNSUPPORTED (third-body or falloff reactions; more species than the
 * LDS holds: 16 * 64 bytes each), AK_EDEVICE.
 */
int ak_eval_source_lnkc(const ak_mechanism *mech, ak_precision prec, const void *T,
                        const void *P, const void *Y, int64_t ldY, int64_t n_cells,
                        const void *lnK, int64_t ldK, void *omega, int64_t ldO, void *stream);

/*
 * ak_eval_lnkc_net into a scratch buffer of N_R x n_cells elements
 * (allocated and freed stream-ordered on `stream`), then
 * ak_eval_source_lnkc: the network as a drop-in for ln K_c.  The network's
 * n_out must equal the mechanism's reaction count, and both must live on
 * the same device.  Errors: as the two calls, AK_ENOMEM.
 */
int ak_eval_source_net(const ak_mechanism *mech, const ak_kcnet *net, ak_precision prec,
                       const void *T, const void *P, const void *Y, int64_t ldY,
                       int64_t n_cells, void *omega, int64_t ldO, void *stream);

/*
 * The 0-D reactor of ak_integrate_euler with the network's ln K_c in place
 * of Eq. 8 at every step (the a-posteriori use of Sec. 3.1): per step
 * ak_eval_lnkc_net, ak_eval_source_lnkc, then the same state update.
 * Scratch of (N_R + NS) x n_cells elements, stream-ordered.  Errors: as
 * ak_eval_source_net and ak_integrate_euler.
 */
int ak_integrate_euler_net(const ak_mechanism *mech, const ak_kcnet *net, ak_precision prec,
                           void *T, const void *P, void *Y, int64_t ldY, int64_t n_cells,
                           double dt, int n_steps, void *stream);

/*
 * Net production rates from given rates of progress, omega = nu r (Eq. 2,
 * nu = nu'' - nu'), with the contraction on the matrix cores in split
 * bfloat16: the reduced-precision environment Sec. 4 names as future work.
 * nu is exact in bfloat16; each rate is cut exactly into three bfloat16
 * parts, so every product is exact and only the FP32 accumulation rounds
 * (the error of an FP32 dot product over 3 N_R terms; rates below about
 * 1e-33 in magnitude lose their lowest part).
 *   rates  device, FP32, [N_R][ldR]: r_j = q_f,j - q_r,j of reaction j
 *          (descriptor order) in cell i at rates[j*ldR + i]; finite (a
 *          non-finite rate makes its species' outputs non-finite)
 *   omega  device, FP32, [NS][ldO], written for i < n_cells only
 * The caller owns both buffers.  The first call uploads nu in the operand
 * order (a few hundred KB, kept with the mechanism).  Errors: AK_EINVAL
 * (null pointers, ldR or ldO < n_cells), AK_E2BIG, AK_EDEVICE, AK_ENOMEM.
 */
int ak_eval_production(const ak_mechanism *mech, const float *rates, int64_t ldR,
                       int64_t n_cells, float *omega, int64_t ldO, void *stream);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of many callers' source-term requests.
 *
 * The paper's use is an MPI rank offloading its cells to the GPU (Sec. 1,
 * Sec. 3.2).  A server accepts such offloads from many host threads at once:
 * requests are queued FIFO and admitted while their bytes fit a device arena
 * and fewer than max_inflight batches are on the device; consecutive small
 * requests (at most small_request_cells cells each) form one batch, which is
 * copied in and evaluated by ONE fused launch per precision covering all its
 * requests (mechanisms may differ); larger requests run alone.  Each request
 * completes, and frees its arena range, as soon as its own result is copied
 * back, while later requests keep being admitted as memory and batch slots
 * free up.  With batching = 0 every request is its own batch (one launch per
 * request), for comparison.
 * Results equal ak_eval_source's up to the rounding order of the omega
 * accumulation.
 */
typedef struct ak_server ak_server;   /* opaque */
typedef struct ak_request ak_request; /* opaque */

typedef struct {
    int32_t device;             /* HIP device of the server (mechanisms must match) */
    int32_t max_inflight;       /* batches on the device at once (0: 3; at most 16) */
    int32_t max_batch_requests; /* requests per batch (0: 64; at most 4096) */
    int32_t batching;           /* 1: continuous batching, 0: one launch per request */
    int64_t max_batch_cells;    /* cells per batch (0: 2^16) */
    size_t arena_bytes;         /* device arena for staged requests (0: 1 GiB) */
    int64_t small_request_cells; /* larger requests are never fused (0: 4096) */
    void *arena;                /* NULL: the server allocates the arena; else a caller-owned
                                   device buffer of arena_bytes (> 0) bytes on `device`,
                                   256-byte aligned, that the caller keeps and does not
                                   touch until ak_server_destroy has returned */
} ak_server_config;

typedef struct {
    int64_t submitted, completed, cancelled, failed; /* requests since the last reset */
    int64_t batches, launches, cells;                /* device work since the last reset */
    int64_t queue_depth;                             /* queued now */
    int32_t inflight, pad;                           /* batches on the device now */
    size_t arena_bytes, arena_used;
    double p50_ms, p99_ms, mean_ms, max_ms;          /* submit -> host-visible result */
    double cells_per_s;                              /* cells / (last completion - first submit) */
} ak_server_stats;

/* Create a server: allocates the device arena (unless the caller passes one
 * in cfg->arena), max_inflight streams (default priority) and descriptor
 * tables, and starts the batcher and completion threads.  Errors: AK_EINVAL
 * (also for a caller arena that is not device memory of cfg->device, not
 * 256-byte aligned, or has arena_bytes 0), AK_ENOMEM, AK_EDEVICE. */
int ak_server_create(const ak_server_config *cfg, ak_server **out);

/*
 * Submit one request: n_cells states in HOST memory (T[n], P[n], Y[NS][ldY];
 * float or double by `prec`), results written to HOST omega[NS][ldO] before
 * the request completes.  Page-locked host buffers give asynchronous copies.
 * The buffers must stay valid until the request has completed or been
 * cancelled.  Returns at once.  Errors: AK_EINVAL (null, n_cells <= 0,
 * ld < n_cells, mechanism on another device), AK_E2BIG (request larger than
 * the arena), AK_ENOMEM.
 */
int ak_server_submit(ak_server *srv, const ak_mechanism *mech, ak_precision prec, const void *T,
                     const void *P, const void *Y, int64_t ldY, int64_t n_cells, void *omega,
                     int64_t ldO, ak_request **out);

/* Wait for a request: 0 when its results are in omega; AK_ETIMEDOUT after
 * timeout_s seconds (< 0: no limit); AK_ECANCELED; AK_EDEVICE if its batch
 * failed. */
int ak_request_wait(ak_request *req, double timeout_s);

/* Cancel a request that is still queued: 0 if cancelled, 1 if it was
 * already admitted to the device (it then completes normally). */
int ak_request_cancel(ak_request *req);

/* Free a completed, failed or cancelled request (AK_EINVAL while pending). */
int ak_request_free(ak_request *req);

/* Counters and latency percentiles since the last reset. */
int ak_server_get_stats(ak_server *srv, ak_server_stats *out);
int ak_server_reset_stats(ak_server *srv);

/* Stop the server: queued requests are cancelled, admitted ones complete,
 * then device resources are released.  Requests stay valid for
 * ak_request_wait / ak_request_free. */
int ak_server_destroy(ak_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* ANNKIN_H */
