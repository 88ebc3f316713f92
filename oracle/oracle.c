/*
 * Test oracle (TEST INFRASTRUCTURE ONLY; see oracle.h).  The body in
 * oracle_impl.h is compiled twice, in double and in long double.
 */
#include <math.h>
#include <stdlib.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include "oracle.h"

#define REAL double
#define SFX(x) x##_f64
#define EXP exp
#define LOG log
#define POW pow
#define FABS fabs
#define LOG10 log10
#include "oracle_impl.h"
#undef REAL
#undef SFX
#undef EXP
#undef LOG
#undef POW
#undef FABS
#undef LOG10

#define REAL long double
#define SFX(x) x##_ld
#define EXP expl
#define LOG logl
#define POW powl
#define FABS fabsl
#define LOG10 log10l
#include "oracle_impl.h"
