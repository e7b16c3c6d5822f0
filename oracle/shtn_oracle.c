/*
 * Reference (oracle) spherical harmonic transform -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain C, compiled with gcc -O2 -fopenmp (no -ffast-math, no intrinsics).
 * Two instantiations of the same body: suffix _d computes in double, suffix
 * _ld in long double (used to measure the double-precision floor and to check
 * the underflow guard of the GPU path at large degree).  All public arrays are
 * double; complex arrays are interleaved (re, im).
 *
 * Only tests, the package smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It shares no source with the GPU library.
 */
#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define REAL double
#define OR_SUFFIX _d
#define OR_PI 3.14159265358979323846264338327950288L
#define OR_EPS DBL_EPSILON
#define OR_SQRT sqrt
#define OR_COS cos
#define OR_SIN sin
#define OR_FABS fabs
#include "shtn_oracle_body.h"
#undef REAL
#undef OR_SUFFIX
#undef OR_EPS
#undef OR_SQRT
#undef OR_COS
#undef OR_SIN
#undef OR_FABS

#define REAL long double
#define OR_SUFFIX _ld
#define OR_EPS LDBL_EPSILON
#define OR_SQRT sqrtl
#define OR_COS cosl
#define OR_SIN sinl
#define OR_FABS fabsl
#include "shtn_oracle_body.h"

/* Number of spectral coefficients of the (L, M) triangular truncation. */
long oracle_nlm(int L, int M) { return (long)(M + 1) * (L + 1) - (long)M * (M + 1) / 2; }
