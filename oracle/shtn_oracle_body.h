/*
 * Reference (oracle) spherical harmonic transform -- TEST INFRASTRUCTURE ONLY.
 *
 * This body is included twice by shtn_oracle.c, once with REAL = double and
 * once with REAL = long double.  It is a plain, slow, obviously-correct CPU
 * implementation of the Gauss-Legendre spherical harmonic transform of
 * Schaeffer, "Efficient Spherical Harmonic Transforms aimed at pseudo-spectral
 * numerical simulations" (arXiv 1202.6522).  It shares no code, table or
 * helper with the GPU library; only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may call it.
 *
 * Conventions (the paper is silent on these; the readings are fixed here):
 *  - spectral arrays are complex, interleaved (re, im), in "m-major"
 *    triangular order idx(n,m) = m(2L+1-m)/2 + n, 0 <= m <= M, m <= n <= L;
 *  - grids are [nlat][nphi] doubles, row i = colatitude theta_i increasing
 *    (Gauss node x_i = cos theta_i decreasing), column k = phi_k = 2 pi k/nphi;
 *  - the real-field reconstruction is f = Re F_0 + 2 Re sum_{m>=1} F_m e^{im phi}
 *    (Hermitian symmetry, Sec. 2.2); Im Q_n^0 is ignored on input and is
 *    returned as exactly 0 by the analysis;
 *  - the phi integral of the analysis (Sec. 2.3) is the trapezoidal sum,
 *    i.e. a DFT scaled by 2 pi / nphi; the synthesis sum is unscaled.
 *
 * Summation order is fixed (ascending n, then i, then k) with plain "+=", so
 * the results do not depend on the thread count.  Threads split the orders m
 * cyclically (thread t takes m = t, t+p, ...), the work split of Sec. 3.3.
 */

#define OR_CAT2(a, b) a##b
#define OR_CAT(a, b) OR_CAT2(a, b)
#define OR_FN(name) OR_CAT(name, OR_SUFFIX)

/* ------------------------------------------------------------------------ */
/* Legendre polynomials P_N and Gauss nodes/weights (Sec. 2.1 recurrence,    */
/* Sec. 2.3 quadrature).                                                     */
/* ------------------------------------------------------------------------ */

/* Bonnet recurrence of Sec. 2.1: P_0 = 1, P_1 = x,
 * n P_n = (2n-1) x P_{n-1} - (n-1) P_{n-2}.  Returns P_N(x), and P_{N-1}(x)
 * through *pnm1. */
static REAL OR_FN(or_legendre_pn)(int N, REAL x, REAL* pnm1)
{
    REAL p0 = 1, p1 = x;
    if (N == 0) { *pnm1 = 0; return 1; }
    for (int n = 2; n <= N; n++) {
        REAL p2 = ((2 * n - 1) * x * p1 - (n - 1) * p0) / n;
        p0 = p1;
        p1 = p2;
    }
    *pnm1 = p0;
    return p1;
}

/* Gauss-Legendre nodes (roots of P_nlat) and weights, x decreasing.
 * Newton iteration x <- x - P_N(x)/P_N'(x) from the classical initial guess
 * cos(pi (i+3/4)/(N+1/2)), with P_N'(x) = N (x P_N - P_{N-1})/((x-1)(x+1))
 * (the factored form avoids cancellation near the poles);
 * w_i = 2 / ((1-x_i)(1+x_i) P_N'(x_i)^2).  The north half is computed and
 * mirrored; for odd N the middle node is exactly 0. */
int OR_FN(oracle_gauss)(int nlat, double* xout, double* wout)
{
    if (nlat < 1 || !xout || !wout) return -1;
    const int N = nlat;
    const REAL pi = OR_PI;
    for (int i = 0; i < (N + 1) / 2; i++) {
        REAL x;
        if ((N & 1) && i == N / 2) {
            x = 0;
        } else {
            x = OR_COS(pi * ((REAL)i + (REAL)0.75) / ((REAL)N + (REAL)0.5));
            int settled = 0;
            for (int it = 0; it < 200; it++) {
                REAL pm1;
                REAL p = OR_FN(or_legendre_pn)(N, x, &pm1);
                REAL dp = N * (x * p - pm1) / ((x - 1) * (x + 1));
                REAL dx = p / dp;
                x -= dx;
                if (settled) break;
                if (OR_FABS(dx) <= 2 * OR_EPS * OR_FABS(x)) settled = 1;
            }
        }
        REAL pm1;
        REAL p = OR_FN(or_legendre_pn)(N, x, &pm1);
        REAL dp = N * (x * p - pm1) / ((x - 1) * (x + 1));
        REAL w = 2 / ((1 - x) * (1 + x) * dp * dp);
        xout[i] = (double)x;
        wout[i] = (double)w;
        xout[N - 1 - i] = (double)(-x);
        wout[N - 1 - i] = (double)w;
    }
    if (N & 1) xout[N / 2] = 0.0;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Orthonormal associated Legendre functions P_n^m (Sec. 2.1 definition,     */
/* computed with the recurrence of Sec. 3.2, eq. rec), including the         */
/* (-1)^m Condon-Shortley factor of the definition.                          */
/* ------------------------------------------------------------------------ */

/* Fills p[n - m] = P_n^m(x) for n = m..L.  s = sqrt((1-x)(1+x)).
 * P_m^m = (-1)^m a_m^m s^m with a_m^m = sqrt(prod_{k=1}^m (2k+1)/(2k) / 4pi),
 * built by repeated multiplication (it may underflow to a denormal or to 0;
 * no rescaling is done here).  P_{m+1}^m = a_{m+1}^m x P_m^m and
 * P_n^m = a_n^m x P_{n-1}^m + b_n^m P_{n-2}^m with
 * a_n^m = sqrt((4n^2-1)/(n^2-m^2)),
 * b_n^m = -sqrt((2n+1)/(2n-3) ((n-1)^2-m^2)/(n^2-m^2)). */
static void OR_FN(or_plm_column)(int L, int m, REAL x, REAL* p)
{
    const REAL pi = OR_PI;
    REAL s = OR_SQRT((1 - x) * (1 + x));
    REAL pmm = OR_SQRT(1 / (4 * pi));
    for (int k = 1; k <= m; k++) pmm *= -OR_SQRT((REAL)(2 * k + 1) / (REAL)(2 * k)) * s;
    if (m > L) return;
    p[0] = pmm;
    if (m + 1 <= L) {
        REAL a = OR_SQRT((REAL)(4 * (m + 1) * (m + 1) - 1) / (REAL)((m + 1) * (m + 1) - m * m));
        p[1] = a * x * pmm;
    }
    for (int n = m + 2; n <= L; n++) {
        REAL nn = (REAL)n * n, mm = (REAL)m * m, n1 = (REAL)(n - 1) * (n - 1);
        REAL a = OR_SQRT((4 * nn - 1) / (nn - mm));
        REAL b = -OR_SQRT((REAL)(2 * n + 1) / (REAL)(2 * n - 3) * (n1 - mm) / (nn - mm));
        p[n - m] = a * x * p[n - m - 1] + b * p[n - m - 2];
    }
}

#ifndef OR_COMMON_HELPERS
#define OR_COMMON_HELPERS
static long or_idx(int L, int n, int m) { return (long)m * (2 * L + 1 - m) / 2 + n; }

static int or_in_list(int m, int nm, const int* mlist)
{
    if (!mlist) return 1;
    for (int t = 0; t < nm; t++)
        if (mlist[t] == m) return 1;
    return 0;
}

static int or_check(int L, int M, int nlat, int nphi, int nfields)
{
    if (L < 0 || M < 0 || M > L || nlat < 1 || nphi < 1 || nfields < 1) return -1;
    if (nphi <= 2 * M) return -1;
    return 0;
}
#endif

/* out[idx(n,m) * nx + j] = P_n^m(x_j) for 0 <= m <= M, m <= n <= L. */
int OR_FN(oracle_plm)(int L, int M, int nx, const double* x, double* out)
{
    if (L < 0 || M < 0 || M > L || nx < 0 || (nx && (!x || !out))) return -1;
    REAL* col = (REAL*)malloc(sizeof(REAL) * (size_t)(L + 1));
    if (!col) return -2;
    for (int m = 0; m <= M; m++)
        for (int j = 0; j < nx; j++) {
            OR_FN(or_plm_column)(L, m, (REAL)x[j], col);
            for (int n = m; n <= L; n++) out[or_idx(L, n, m) * nx + j] = (double)col[n - m];
        }
    free(col);
    return 0;
}

/* The same values left in the working type REAL (no rounding to double), for
 * the orders in mlist only: out[(t * (L+1) + n) * nx + j] = P_n^m(x_j) with
 * m = mlist[t] (entries n < m are set to 0).  Lets the long-double
 * instantiation be compared with a high-precision reference below the
 * rounding of double, and where P_n^m lies outside the range of double. */
int OR_FN(oracle_plm_raw)(int L, int nm, const int* mlist, int nx, const double* x, REAL* out)
{
    if (L < 0 || nm < 0 || nx < 0 || (nm && !mlist) || (nx && nm && (!x || !out))) return -1;
    for (int t = 0; t < nm; t++)
        if (mlist[t] < 0 || mlist[t] > L) return -1;
    REAL* col = (REAL*)malloc(sizeof(REAL) * (size_t)(L + 1));
    if (!col) return -2;
    for (int t = 0; t < nm; t++) {
        const int m = mlist[t];
        for (int j = 0; j < nx; j++) {
            OR_FN(or_plm_column)(L, m, (REAL)x[j], col);
            for (int n = 0; n <= L; n++)
                out[((size_t)t * (L + 1) + n) * nx + j] = n < m ? (REAL)0 : col[n - m];
        }
    }
    free(col);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* DFT tables: c_j = cos(2 pi j / nphi), s_j = sin(2 pi j / nphi); the       */
/* argument of e^{i m phi_k} is reduced exactly as j = (m k) mod nphi.       */
/* ------------------------------------------------------------------------ */
static void OR_FN(or_dft_tables)(int nphi, REAL* c, REAL* s)
{
    const REAL pi = OR_PI;
    for (int j = 0; j < nphi; j++) {
        REAL t = 2 * pi * (REAL)j / (REAL)nphi;
        c[j] = OR_COS(t);
        s[j] = OR_SIN(t);
    }
}

/* ------------------------------------------------------------------------ */
/* Synthesis (Sec. 2.2, eq. synth_direct, then the Fourier sum in m), and   */
/* its adjoint-of-analysis variant.                                          */
/* ------------------------------------------------------------------------ */

/* Legendre synthesis for one field: F[m][i] = sum_{n=m}^{L} Q_n^m P_n^m(x_i)
 * (complex), for every order in the list (others left at 0). */
static void OR_FN(or_legendre_synth)(int L, int M, int nlat, const REAL* x, const double* Q,
                                     REAL* F, int nm, const int* mlist, int nthreads)
{
    (void)nthreads;
#pragma omp parallel for schedule(static, 1) num_threads(nthreads)
    for (int m = 0; m <= M; m++) {
        if (!or_in_list(m, nm, mlist)) continue;
        REAL* col = (REAL*)malloc(sizeof(REAL) * (size_t)(L + 1));
        for (int i = 0; i < nlat; i++) {
            OR_FN(or_plm_column)(L, m, x[i], col);
            REAL re = 0, im = 0;
            for (int n = m; n <= L; n++) {
                long id = or_idx(L, n, m);
                re += (REAL)Q[2 * id] * col[n - m];
                im += (REAL)Q[2 * id + 1] * col[n - m];
            }
            F[2 * ((long)m * nlat + i)] = re;
            F[2 * ((long)m * nlat + i) + 1] = im;
        }
        free(col);
    }
}

/* Fourier synthesis of the listed rows:
 * f_ik = scale_i * ( Re F_0(i) + sum_{m>=1} wm (Re F_m c_{mk} - Im F_m s_{mk}) ),
 * with wm = 2 for the synthesis (Hermitian symmetry) and wm = 1 for the
 * adjoint of the analysis. */
static void OR_FN(or_fourier_synth)(int M, int nlat, int nphi, const REAL* F, const REAL* c,
                                    const REAL* s, REAL wm, const REAL* rowscale, int nrows,
                                    const int* rows, double* out, int nthreads)
{
    (void)nthreads;
    int nr = rows ? nrows : nlat;
#pragma omp parallel for schedule(static, 1) num_threads(nthreads)
    for (int r = 0; r < nr; r++) {
        int i = rows ? rows[r] : r;
        for (int k = 0; k < nphi; k++) {
            REAL acc = F[2 * ((long)0 * nlat + i)];
            for (int m = 1; m <= M; m++) {
                int j = (int)(((long)m * k) % nphi);
                const REAL* f = F + 2 * ((long)m * nlat + i);
                acc += wm * (f[0] * c[j] - f[1] * s[j]);
            }
            if (rowscale) acc *= rowscale[i];
            out[(long)r * nphi + k] = (double)acc;
        }
    }
}

/* Fourier analysis of every row: F[m][i] = scale * sum_k f_ik (c_{mk} - i s_{mk}). */
static void OR_FN(or_fourier_analys)(int M, int nlat, int nphi, const double* grid, const REAL* c,
                                     const REAL* s, REAL scale, REAL* F, int nm, const int* mlist,
                                     int nthreads)
{
    (void)nthreads;
#pragma omp parallel for schedule(static, 1) num_threads(nthreads)
    for (int i = 0; i < nlat; i++) {
        for (int m = 0; m <= M; m++) {
            if (!or_in_list(m, nm, mlist)) continue;
            REAL re = 0, im = 0;
            for (int k = 0; k < nphi; k++) {
                int j = (int)(((long)m * k) % nphi);
                REAL v = (REAL)grid[(long)i * nphi + k];
                re += v * c[j];
                im -= v * s[j];
            }
            F[2 * ((long)m * nlat + i)] = scale * re;
            F[2 * ((long)m * nlat + i) + 1] = scale * im;
        }
    }
}

/* Legendre analysis (eq. gauss): Q_n^m = cm * sum_i wt_i P_n^m(x_i) F_m(theta_i).
 * cm = 1 for the analysis; for the adjoint of the synthesis wt = 1 and
 * cm = 1 (m = 0) or 2 (m >= 1).  Im Q_n^0 is set to 0. */
static void OR_FN(or_legendre_analys)(int L, int M, int nlat, const REAL* x, const REAL* wt,
                                      const REAL* F, REAL cm0, REAL cm1, double* Q, int nm,
                                      const int* mlist, int nthreads)
{
    (void)nthreads;
#pragma omp parallel for schedule(static, 1) num_threads(nthreads)
    for (int m = 0; m <= M; m++) {
        long base = or_idx(L, m, m);
        if (!or_in_list(m, nm, mlist)) {
            for (int n = m; n <= L; n++) Q[2 * (base + n - m)] = Q[2 * (base + n - m) + 1] = 0.0;
            continue;
        }
        REAL* col = (REAL*)malloc(sizeof(REAL) * (size_t)(L + 1));
        REAL* acc = (REAL*)calloc((size_t)(2 * (L + 1)), sizeof(REAL));
        for (int i = 0; i < nlat; i++) {
            OR_FN(or_plm_column)(L, m, x[i], col);
            REAL fr = F[2 * ((long)m * nlat + i)] * wt[i];
            REAL fi = F[2 * ((long)m * nlat + i) + 1] * wt[i];
            for (int n = m; n <= L; n++) {
                acc[2 * (n - m)] += col[n - m] * fr;
                acc[2 * (n - m) + 1] += col[n - m] * fi;
            }
        }
        REAL cm = m == 0 ? cm0 : cm1;
        for (int n = m; n <= L; n++) {
            Q[2 * (base + n - m)] = (double)(cm * acc[2 * (n - m)]);
            Q[2 * (base + n - m) + 1] = m == 0 ? 0.0 : (double)(cm * acc[2 * (n - m) + 1]);
        }
        free(col);
        free(acc);
    }
}

/* Common driver for the two grid-producing maps (synthesis and the adjoint of
 * the analysis).  adjoint = 0: f = S Q.  adjoint = 1: f = A^T h. */
static int OR_FN(or_to_grid)(int adjoint, int L, int M, int nlat, int nphi, int nfields,
                             const double* Q, double* grid, int nm, const int* mlist, int nrows,
                             const int* rows, int nthreads)
{
    if (or_check(L, M, nlat, nphi, nfields) || !Q || !grid) return -1;
    if (nthreads < 1) nthreads = 1;
    const REAL pi = OR_PI;
    double* xd = (double*)malloc(sizeof(double) * nlat);
    double* wd = (double*)malloc(sizeof(double) * nlat);
    REAL* x = (REAL*)malloc(sizeof(REAL) * nlat);
    REAL* rs = (REAL*)malloc(sizeof(REAL) * nlat);
    REAL* c = (REAL*)malloc(sizeof(REAL) * nphi);
    REAL* s = (REAL*)malloc(sizeof(REAL) * nphi);
    REAL* F = (REAL*)malloc(sizeof(REAL) * 2 * (size_t)(M + 1) * nlat);
    OR_FN(oracle_gauss)(nlat, xd, wd);
    for (int i = 0; i < nlat; i++) {
        x[i] = (REAL)xd[i];
        rs[i] = 2 * pi / (REAL)nphi * (REAL)wd[i];
    }
    OR_FN(or_dft_tables)(nphi, c, s);
    long nlm = (long)(M + 1) * (L + 1) - (long)M * (M + 1) / 2;
    int nr = rows ? nrows : nlat;
    for (int f = 0; f < nfields; f++) {
        memset(F, 0, sizeof(REAL) * 2 * (size_t)(M + 1) * nlat);
        OR_FN(or_legendre_synth)(L, M, nlat, x, Q + 2 * nlm * f, F, nm, mlist, nthreads);
        OR_FN(or_fourier_synth)(M, nlat, nphi, F, c, s, adjoint ? (REAL)1 : (REAL)2,
                                adjoint ? rs : NULL, nrows, rows, grid + (long)nr * nphi * f,
                                nthreads);
    }
    free(xd); free(wd); free(x); free(rs); free(c); free(s); free(F);
    return 0;
}

/* Common driver for the two spectrum-producing maps (analysis and the adjoint
 * of the synthesis).  adjoint = 0: Q = A f.  adjoint = 1: Q = S^T g. */
static int OR_FN(or_to_spec)(int adjoint, int L, int M, int nlat, int nphi, int nfields,
                             const double* grid, double* Q, int nm, const int* mlist,
                             int nthreads)
{
    if (or_check(L, M, nlat, nphi, nfields) || !Q || !grid) return -1;
    if (nthreads < 1) nthreads = 1;
    const REAL pi = OR_PI;
    double* xd = (double*)malloc(sizeof(double) * nlat);
    double* wd = (double*)malloc(sizeof(double) * nlat);
    REAL* x = (REAL*)malloc(sizeof(REAL) * nlat);
    REAL* wt = (REAL*)malloc(sizeof(REAL) * nlat);
    REAL* c = (REAL*)malloc(sizeof(REAL) * nphi);
    REAL* s = (REAL*)malloc(sizeof(REAL) * nphi);
    REAL* F = (REAL*)malloc(sizeof(REAL) * 2 * (size_t)(M + 1) * nlat);
    OR_FN(oracle_gauss)(nlat, xd, wd);
    for (int i = 0; i < nlat; i++) {
        x[i] = (REAL)xd[i];
        wt[i] = adjoint ? (REAL)1 : (REAL)wd[i];
    }
    OR_FN(or_dft_tables)(nphi, c, s);
    long nlm = (long)(M + 1) * (L + 1) - (long)M * (M + 1) / 2;
    REAL scale = adjoint ? (REAL)1 : 2 * pi / (REAL)nphi;
    for (int f = 0; f < nfields; f++) {
        memset(F, 0, sizeof(REAL) * 2 * (size_t)(M + 1) * nlat);
        OR_FN(or_fourier_analys)(M, nlat, nphi, grid + (long)nlat * nphi * f, c, s, scale, F, nm,
                                 mlist, nthreads);
        OR_FN(or_legendre_analys)(L, M, nlat, x, wt, F, 1, adjoint ? (REAL)2 : (REAL)1,
                                  Q + 2 * nlm * f, nm, mlist, nthreads);
    }
    free(xd); free(wd); free(x); free(wt); free(c); free(s); free(F);
    return 0;
}

/* Synthesis S: Q (nfields x nlm complex) -> grid (nfields x nrows x nphi).
 * mlist (nm entries) restricts the sum to the listed orders (the caller
 * guarantees Q vanishes elsewhere); NULL means all orders.  rows (nrows
 * entries) selects output latitudes; NULL means all nlat rows. */
int OR_FN(oracle_synth)(int L, int M, int nlat, int nphi, int nfields, const double* Q,
                        double* grid, int nm, const int* mlist, int nrows, const int* rows,
                        int nthreads)
{
    return OR_FN(or_to_grid)(0, L, M, nlat, nphi, nfields, Q, grid, nm, mlist, nrows, rows,
                             nthreads);
}

/* Analysis A: grid (nfields x nlat x nphi) -> Q; only listed orders are
 * computed (others are written as 0). */
int OR_FN(oracle_analys)(int L, int M, int nlat, int nphi, int nfields, const double* grid,
                         double* Q, int nm, const int* mlist, int nthreads)
{
    return OR_FN(or_to_spec)(0, L, M, nlat, nphi, nfields, grid, Q, nm, mlist, nthreads);
}

/* Adjoint of the synthesis, S^T: grid -> Q-shaped,
 * (S^T g)_n^m = c_m sum_i P_n^m(x_i) sum_k g_ik e^{-i m phi_k}, c_0 = 1, c_m = 2. */
int OR_FN(oracle_synth_adj)(int L, int M, int nlat, int nphi, int nfields, const double* grid,
                            double* Q, int nm, const int* mlist, int nthreads)
{
    return OR_FN(or_to_spec)(1, L, M, nlat, nphi, nfields, grid, Q, nm, mlist, nthreads);
}

/* Adjoint of the analysis, A^T: Q-shaped -> grid,
 * (A^T h)_ik = (2 pi/nphi) w_i [Re H_0 + sum_{m>=1} Re(H_m e^{i m phi_k})],
 * H_m(theta_i) = sum_n h_n^m P_n^m(x_i). */
int OR_FN(oracle_analys_adj)(int L, int M, int nlat, int nphi, int nfields, const double* Q,
                             double* grid, int nm, const int* mlist, int nrows, const int* rows,
                             int nthreads)
{
    return OR_FN(or_to_grid)(1, L, M, nlat, nphi, nfields, Q, grid, nm, mlist, nrows, rows,
                             nthreads);
}

#undef OR_FN
#undef OR_CAT
#undef OR_CAT2
