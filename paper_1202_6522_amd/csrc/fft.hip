// Longitude stage of the SHT on gfx950: batched real FFTs in FP64 (Sec. 3.1,
// "use the FFT" and Hermitian symmetry of real data).
//
// A real transform of length N = 2K is computed as a complex FFT of length K
// on z_k = f_{2k} + i f_{2k+1}, with an O(K) pre/post-pass that separates the
// even and odd samples.  The complex FFT is a Stockham autosort with radix-16
// passes (a 16-point DFT in registers as 4 x 4) and one radix-4 or radix-2
// pass for the remaining factor: three passes through LDS at K = 1024.
//
// A workgroup holds rows x K <= 4096 complex points in LDS with one thread
// per 16 points (one to four waves), so several workgroups share a CU; the
// twiddles come from a two-level table of at most 128 entries in LDS.  Every
// thread owns 16 points of every pass (16/R butterflies of radix R); all
// index arithmetic is shifts and masks (K is a power of two).  Row blocks are
// spread over the XCDs so that neighbouring blocks share an L2.
#include <hip/hip_runtime.h>

#include "shtn_internal.h"

namespace shtn {

constexpr int kFftMaxThreads = 256;           // at most four waves
constexpr int kFftPoints = 4096;              // complex points per workgroup at most (LDS)
constexpr int kFftPerThread = 16;             // points per thread: one radix-16 butterfly per pass
constexpr int kTwEntries = 128;               // two-level twiddle table, K <= 4096

// Twiddle tables are read through global-address-space pointers (the plan
// descriptor holds them as generic pointers, which would compile to flat
// loads).
typedef const __attribute__((address_space(1))) double* gdp;


__device__ __forceinline__ double2 ld2(gdp t, int i) { return make_double2(t[2 * i], t[2 * i + 1]); }

// LDS slot of point x: one pad slot after every 16 points, so the strided
// writes of a radix-16 pass spread over the banks.
__device__ __forceinline__ int at(int x) { return x + (x >> 4); }
constexpr int lds_points(int p) { return p + p / 16; }

struct FftArgs {
    const DevPlan* plans;
    const int* rowblocks;  // per block {field, plan, row0, nrows}, or null for plan calls
    const long* g_off;     // per field grid offset in doubles, or null (f * nlat * nphi)
    const long* f_off;     // per field F offset in doubles, or null (f * 2 f_size)
    const double* in;
    double* out;
    int nfields;
    int rows_per_block;
    double scale;
};

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
// multiply by +i (s = +1) or -i (s = -1)
__device__ __forceinline__ double2 cmuli(double2 a, int s)
{
    return s > 0 ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x);
}

// In-place DFT_4 of v[o], v[o+st], v[o+2st], v[o+3st] with e^{dir 2 pi i jk/4}.
template <int N>
__device__ __forceinline__ void dft4(double2 (&v)[N], int o, int st, int dir)
{
    const double2 a0 = cadd(v[o], v[o + 2 * st]), a1 = csub(v[o], v[o + 2 * st]);
    const double2 b0 = cadd(v[o + st], v[o + 3 * st]), b1 = cmuli(csub(v[o + st], v[o + 3 * st]), dir);
    v[o] = cadd(a0, b0);
    v[o + 2 * st] = csub(a0, b0);
    v[o + st] = cadd(a1, b1);
    v[o + 3 * st] = csub(a1, b1);
}

// In-place 16-point DFT with e^{dir 2 pi i jk/16}: index j = 4 j1 + j2,
// k = k1 + 4 k2.  Four DFT_4 over j1, twiddles e^{dir 2 pi i j2 k1/16}, four
// DFT_4 over j2.  The result X[k1 + 4 k2] is left in v[4 k1 + k2]
// (digit-reversed order; out_slot maps it back at no cost).
__device__ __forceinline__ void dft16(double2 (&v)[16], int dir)
{
    // cos and sin of 2 pi p / 16: p = 1 (c1, s1), p = 2 (c2, c2)
    constexpr double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173;
    constexpr double c2 = 0.70710678118654752440;
#pragma unroll
    for (int j2 = 0; j2 < 4; j2++) dft4(v, j2, 4, dir);  // v[4 k1 + j2] = A[k1][j2]
    const double sd = dir;
    // twiddle A[k1][j2] by w^{j2 k1}, w = e^{dir 2 pi i / 16}
    const double2 w1 = make_double2(c1, sd * s1), w2 = make_double2(c2, sd * c2);
    const double2 w3 = make_double2(s1, sd * c1), w6 = make_double2(-c2, sd * c2);
    const double2 w9 = make_double2(-c1, -sd * s1);
    // v[4 k1 + j2] *= w^{k1 j2}
    v[5] = cmul(v[5], w1);
    v[6] = cmul(v[6], w2);
    v[7] = cmul(v[7], w3);
    v[9] = cmul(v[9], w2);
    v[10] = cmuli(v[10], dir);  // w^4 = dir i
    v[11] = cmul(v[11], w6);
    v[13] = cmul(v[13], w3);
    v[14] = cmul(v[14], w6);
    v[15] = cmul(v[15], w9);
#pragma unroll
    for (int k1 = 0; k1 < 4; k1++) dft4(v, 4 * k1, 1, dir);  // v[4 k1 + k2] = X[k1 + 4 k2]
}

// Register holding output q of dft_r<R>: the radix-16 DFT leaves X[k1 + 4 k2]
// in v[4 k1 + k2]; the others are in natural order.
template <int R>
__device__ __forceinline__ constexpr int out_slot(int q)
{
    return R == 16 ? 4 * (q & 3) + (q >> 2) : q;
}

template <int R>
__device__ __forceinline__ void dft_r(double2 (&v)[R], int dir)
{
    if constexpr (R == 16) {
        dft16(v, dir);
    } else if constexpr (R == 4) {
        dft4(v, 0, 1, dir);
    } else {
        const double2 a = v[0], c = v[1];
        v[0] = cadd(a, c);
        v[1] = csub(a, c);
    }
}

// Twiddle e^{-2 pi i t/K} (0 <= t < K = 2^lgK) from the two-level table in
// LDS: t = hi 2^lo + lo_part with lo = ceil(lgK/2); entries [0, 2^lo) hold
// e^{-2 pi i b/K}, entries [2^lo, 2^lo + 2^(lgK-lo)) hold e^{-2 pi i a 2^lo/K}.
__device__ __forceinline__ double2 tw_at(const double2* twl, int t, int lgK)
{
    const int lo = (lgK + 1) >> 1;
    return cmul(twl[t & ((1 << lo) - 1)], twl[(1 << lo) + (t >> lo)]);
}

// One Stockham pass of radix R over the rows held in buf (npts = rows x K
// points, K = 2^lgK); Ns = 2^lgNs = product of the radices of the previous
// passes; twl = the two-level twiddle table in LDS.  Each thread reads
// its 16/R butterflies, the workgroup synchronises, then they are written
// back in place.  dir = -1 forward (e^{-2 pi i}), +1 inverse.
template <int R, int LGR>
__device__ __forceinline__ void stockham_pass(double2* buf, const double2* twl, int lgK, int npts, int lgNs,
                                              int dir)
{
    constexpr int NB = 16 / R;
    const int lgKR = lgK - LGR;
    const int nb = npts >> LGR;
    const int KR = 1 << lgKR;
    double2 v[NB][R];
    int dst[NB];
#pragma unroll
    for (int i = 0; i < NB; i++) {
        const int b = threadIdx.x + i * blockDim.x;
        dst[i] = -1;
        if (b < nb) {
            const int r = b >> lgKR, jj = b & (KR - 1);
            const int js = jj & ((1 << lgNs) - 1);
            const int rowb = r << lgK;
#pragma unroll
            for (int q = 0; q < R; q++) v[i][q] = buf[at(rowb + jj + q * KR)];
            if (lgNs > 0) {  // the first pass has js = 0: all twiddles are 1
                // twiddle index q js K / (Ns R)
                const int tstep = js << (lgK - lgNs - LGR);
#pragma unroll
                for (int q = 1; q < R; q++) {
                    double2 w = tw_at(twl, q * tstep, lgK);
                    if (dir > 0) w = cconj(w);
                    v[i][q] = cmul(v[i][q], w);
                }
            }
            dft_r<R>(v[i], dir);
            dst[i] = rowb + (((jj >> lgNs) << (lgNs + LGR)) | js);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NB; i++) {
        if (dst[i] >= 0) {
#pragma unroll
            for (int q = 0; q < R; q++) buf[at(dst[i] + (q << lgNs))] = v[i][out_slot<R>(q)];
        }
    }
    __syncthreads();
}

// Complex FFT of length K = 2^lgK on every row held in buf: radix 16 while
// four or more factors of 2 remain, then one radix-4 and/or radix-2 pass.
__device__ __forceinline__ void complex_fft(double2* buf, const double2* twl, int lgK, int npts, int dir)
{
    int lgNs = 0;
    while (lgK - lgNs >= 4) {
        stockham_pass<16, 4>(buf, twl, lgK, npts, lgNs, dir);
        lgNs += 4;
    }
    if (lgK - lgNs >= 2) {
        stockham_pass<4, 2>(buf, twl, lgK, npts, lgNs, dir);
        lgNs += 2;
    }
    if (lgK - lgNs == 1) stockham_pass<2, 1>(buf, twl, lgK, npts, lgNs, dir);
}

// Builds the two-level twiddle table (see tw_at) from the K-entry table
// e^{-2 pi i t/K} in global memory.
__device__ __forceinline__ void stage_twiddles(double2* twl, gdp tw, int lgK)
{
    const int lo = (lgK + 1) >> 1, nlo = 1 << lo, n = nlo + (1 << (lgK - lo));
    for (int t = threadIdx.x; t < n; t += blockDim.x) twl[t] = ld2(tw, t < nlo ? t : (t - nlo) << lo);
}

struct RowBlock {
    int field, plan, row0, nrows;
};

__device__ __forceinline__ RowBlock row_block(const FftArgs& a, int nlat)
{
    RowBlock rb;
    if (a.rowblocks) {
        const int* q = a.rowblocks + 4 * blockIdx.x;
        rb.field = q[0];
        rb.plan = q[1];
        rb.row0 = q[2];
        rb.nrows = q[3];
    } else {
        // XCD-aware: workgroup b runs on XCD b % 8; give each XCD a
        // contiguous range of row blocks
        const int nb = gridDim.x, b = blockIdx.x;
        const int x = b % kXcds, q = nb / kXcds, rem = nb % kXcds;
        const int blk = x * q + min(x, rem) + b / kXcds;
        rb.field = blockIdx.y;
        rb.plan = 0;
        rb.row0 = blk * a.rows_per_block;
        rb.nrows = min(a.rows_per_block, nlat - rb.row0);
    }
    return rb;
}

// F_m of latitude row0 + r for all (m <= M, r < nrows) <-> LDS rows of K
// points.  When the block is a power-of-two run of rows aligned inside the
// tiles (whole tiles, or an aligned part of one), every order contributes
// one contiguous run per tile, read or written by consecutive threads;
// otherwise point by point.
template <bool LOAD>
__device__ __forceinline__ void move_f(double2* buf, const double* Fin, double* Fout, long ts, int M,
                                       int lgK, int row0, int nrows)
{
    const int run = nrows < kFTile ? nrows : kFTile;  // rows per tile in the block
    const bool pow2 = (run & (run - 1)) == 0;
    if (LOAD && pow2 && nrows <= kFTile && (row0 & (nrows - 1)) == 0) {
        // The block is one aligned run inside a tile: entry e is order
        // e >> lg, row e & (nrows - 1).  Every thread owns at most
        // kFftPerThread entries (nrows (M+1) <= nrows K <= kFftPerThread
        // threads), all loaded, from valid addresses, before any LDS write:
        // one memory round trip instead of one per entry.
        const int lg = __builtin_ctz(nrows);
        const int n = nrows * (M + 1);
        const long tb = (long)(row0 >> kFTileLg) * ts + (row0 & (kFTile - 1));
        double2 v[kFftPerThread];
#pragma unroll
        for (int k = 0; k < kFftPerThread; k++) {
            const int e = threadIdx.x + k * blockDim.x;
            const int ec = e < n ? e : 0;
            v[k] = *(const double2*)(Fin + 2 * (tb + ((long)(ec >> lg) << kFTileLg) + (ec & (nrows - 1))));
        }
#pragma unroll
        for (int k = 0; k < kFftPerThread; k++) {
            const int e = threadIdx.x + k * blockDim.x;
            const int m = e >> lg, r = e & (nrows - 1);
            if (e < n) buf[at((r << lgK) + m)] = make_double2(v[k].x, m == 0 ? 0.0 : v[k].y);
        }
        return;
    }
    if (!LOAD && pow2 && nrows <= kFTile && (row0 & (nrows - 1)) == 0) {
        // store side of the same run: all LDS reads first, then the stores
        const int lg = __builtin_ctz(nrows);
        const int n = nrows * (M + 1);
        const long tb = (long)(row0 >> kFTileLg) * ts + (row0 & (kFTile - 1));
        double2 v[kFftPerThread];
#pragma unroll
        for (int k = 0; k < kFftPerThread; k++) {
            const int e = threadIdx.x + k * blockDim.x;
            const int ec = e < n ? e : 0;
            v[k] = buf[at(((ec & (nrows - 1)) << lgK) + (ec >> lg))];
        }
#pragma unroll
        for (int k = 0; k < kFftPerThread; k++) {
            const int e = threadIdx.x + k * blockDim.x;
            if (e < n)
                *(double2*)(Fout + 2 * (tb + ((long)(e >> lg) << kFTileLg) + (e & (nrows - 1)))) = v[k];
        }
        return;
    }
    if (pow2 && (row0 & (run - 1)) == 0 && (nrows & (run - 1)) == 0) {
        const int lgrun = __builtin_ctz(run);
        const int per_tile = (M + 1) << lgrun;
        for (int t = 0; t < nrows >> lgrun; t++) {
            const int i0 = row0 + (t << lgrun);  // first latitude of this run
            const long tb = (long)(i0 >> kFTileLg) * ts + (i0 & (kFTile - 1));
            for (int e = threadIdx.x; e < per_tile; e += blockDim.x) {
                const int m = e >> lgrun, r = (t << lgrun) + (e & (run - 1));
                const long off = tb + ((long)m << kFTileLg) + (e & (run - 1));
                if (LOAD) {
                    double2 y = *(const double2*)(Fin + 2 * off);
                    if (m == 0) y.y = 0.0;
                    buf[at((r << lgK) + m)] = y;
                } else {
                    *(double2*)(Fout + 2 * off) = buf[at((r << lgK) + m)];
                }
            }
        }
    } else {
        const int n = nrows * (M + 1);
        for (int e = threadIdx.x; e < n; e += blockDim.x) {
            const int r = e % nrows, m = e / nrows;
            const int i = row0 + r;
            const long off = (long)(i >> kFTileLg) * ts + ((long)m << kFTileLg) + (i & (kFTile - 1));
            if (LOAD) {
                double2 y = *(const double2*)(Fin + 2 * off);
                if (m == 0) y.y = 0.0;
                buf[at((r << lgK) + m)] = y;
            } else {
                *(double2*)(Fout + 2 * off) = buf[at((r << lgK) + m)];
            }
        }
    }
}

// Fourier synthesis of rows: f_ik = Re F_0 + 2 Re sum_{m=1}^{M} F_m e^{2 pi i m k / N}.
__global__ void __launch_bounds__(kFftMaxThreads) k_c2r(FftArgs a)
{
    extern __shared__ double2 lds[];  // points (16 per thread), then the twiddle table
    double2* buf = lds;
    double2* twl = lds + lds_points(blockDim.x * kFftPerThread);
    const int pl = a.rowblocks ? a.rowblocks[4 * blockIdx.x + 1] : 0;
    const DevPlan& D = a.plans[pl];
    const RowBlock rb = row_block(a, D.nlat);
    if (rb.field >= a.nfields || rb.nrows <= 0) return;
    const int K = D.K, M = D.M, nlat = D.nlat, nphi = D.nphi;
    const int lgK = __builtin_ctz(K);
    const gdp tw = (gdp)D.tw;
    const gdp rtw = (gdp)D.rtw;
    const double* F = a.in + (a.f_off ? a.f_off[rb.field] : (long)rb.field * 2 * D.f_size);
    double* g = a.out + (a.g_off ? a.g_off[rb.field] : (long)rb.field * nlat * nphi);
    const int npts = rb.nrows << lgK;

    stage_twiddles(twl, tw, lgK);
    // w^m of this thread's points, loaded while the rows arrive
    double2 rw[kFftPerThread];
#pragma unroll
    for (int e = 0; e < kFftPerThread; e++)
        rw[e] = ld2(rtw, (threadIdx.x + e * blockDim.x) & (K - 1));
    // Y_m (Y_0 = Re F_0, Y_m = F_m for 1 <= m <= M, 0 above) row by row
    for (int idx = threadIdx.x; idx < npts; idx += blockDim.x)
        if ((idx & (K - 1)) > M) buf[at(idx)] = make_double2(0.0, 0.0);
    move_f<true>(buf, F, nullptr, D.f_ts, M, lgK, rb.row0, rb.nrows);
    __syncthreads();
    // Z_m = (Y_m + conj Y_{K-m}) + i w^m (Y_m - conj Y_{K-m}), w = e^{i pi/K},
    // Y_K = 0 (M < K)
    double2 z[kFftPerThread];
#pragma unroll
    for (int e = 0; e < kFftPerThread; e++) {
        const int idx = threadIdx.x + e * blockDim.x;
        z[e] = make_double2(0.0, 0.0);
        if (idx < npts) {
            const int m = idx & (K - 1);
            const double2 ym = buf[at(idx)];
            const double2 yc = m == 0 ? make_double2(0.0, 0.0) : buf[at(idx - m + (K - m))];
            const double2 s = cadd(ym, cconj(yc)), d = csub(ym, cconj(yc));
            z[e] = cadd(s, cmuli(cmul(rw[e], d), 1));
        }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kFftPerThread; e++) {
        const int idx = threadIdx.x + e * blockDim.x;
        if (idx < npts) buf[at(idx)] = z[e];
    }
    __syncthreads();
    complex_fft(buf, twl, lgK, npts, +1);
#pragma unroll
    for (int e = 0; e < kFftPerThread; e++) {
        const int idx = threadIdx.x + e * blockDim.x;
        if (idx < npts) {
            const int r = idx >> lgK, k = idx & (K - 1);
            *(double2*)(g + (size_t)(rb.row0 + r) * nphi + 2 * k) = buf[at(idx)];
        }
    }
}

// Fourier analysis of rows: F_m(theta_i) = scale * sum_k f_ik e^{-2 pi i m k / N}, m <= M.
__global__ void __launch_bounds__(kFftMaxThreads) k_r2c(FftArgs a)
{
    extern __shared__ double2 lds[];  // points (16 per thread), then the twiddle table
    double2* buf = lds;
    double2* twl = lds + lds_points(blockDim.x * kFftPerThread);
    const int pl = a.rowblocks ? a.rowblocks[4 * blockIdx.x + 1] : 0;
    const DevPlan& D = a.plans[pl];
    const RowBlock rb = row_block(a, D.nlat);
    if (rb.field >= a.nfields || rb.nrows <= 0) return;
    const int K = D.K, M = D.M, nlat = D.nlat, nphi = D.nphi;
    const int lgK = __builtin_ctz(K);
    const gdp tw = (gdp)D.tw;
    const gdp rtw = (gdp)D.rtw;
    const double* g = a.in + (a.g_off ? a.g_off[rb.field] : (long)rb.field * nlat * nphi);
    double* F = a.out + (a.f_off ? a.f_off[rb.field] : (long)rb.field * 2 * D.f_size);
    const int npts = rb.nrows << lgK;
    stage_twiddles(twl, tw, lgK);
    // Straight-line loads from valid addresses, then LDS writes without
    // branches (idx < 16 blockDim stays inside the point buffer; slots past
    // npts are never read), so every load is issued before the first wait.
    double2 v[kFftPerThread];
#pragma unroll
    for (int e = 0; e < kFftPerThread; e++) {
        const int idx = threadIdx.x + e * blockDim.x;
        const int ic = idx < npts ? idx : 0;
        const int r = ic >> lgK, k = ic & (K - 1);
        v[e] = *(const double2*)(g + (size_t)(rb.row0 + r) * nphi + 2 * k);
    }
#pragma unroll
    for (int e = 0; e < kFftPerThread; e++) buf[at(threadIdx.x + e * blockDim.x)] = v[e];

    __syncthreads();
    complex_fft(buf, twl, lgK, npts, -1);
    // w^m of this thread's points for the post-pass
    double2 rw[kFftPerThread];
#pragma unroll
    for (int e = 0; e < kFftPerThread; e++)
        rw[e] = ld2(rtw, (threadIdx.x + e * blockDim.x) & (K - 1));
    // scale <= 0: the analysis scale 2 pi / nphi of each field's plan
    const double sc = a.scale > 0.0 ? a.scale : 2.0 * 3.14159265358979323846 / nphi;
    // X_m from Z_m and Z_{K-m}, computed in registers, then written over the
    // buffer so that F leaves in tile order
    // (straight-line: every index below stays inside the point buffer, a
    // row of K points lying within its 16 blockDim slots; points past npts
    // are computed from unused slots and never read back)
    double2 x[kFftPerThread];
#pragma unroll
    for (int e = 0; e < kFftPerThread; e++) {
        const int idx = threadIdx.x + e * blockDim.x;
        const int m = idx & (K - 1);
        const double2 zm = buf[at(idx)];
        const double2 zc = cconj(buf[at(idx - m + ((K - m) & (K - 1)))]);
        const double2 A = make_double2(0.5 * (zm.x + zc.x), 0.5 * (zm.y + zc.y));
        const double2 Dd = csub(zm, zc);
        const double2 B = make_double2(0.5 * Dd.y, -0.5 * Dd.x);  // (Z_m - conj Z_{K-m}) / (2i)
        double2 X = cadd(A, cmul(cconj(rw[e]), B));
        X.x *= sc;
        X.y = m == 0 ? 0.0 : X.y * sc;
        x[e] = X;
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kFftPerThread; e++) buf[at(threadIdx.x + e * blockDim.x)] = x[e];
    __syncthreads();
    move_f<false>(buf, nullptr, F, D.f_ts, M, lgK, rb.row0, rb.nrows);
}

static FftArgs fft_args(const FftLaunch& l)
{
    FftArgs a{l.plans, l.rowblocks, l.g_off, l.f_off, l.in, l.out, l.nfields, l.rows_per_block,
              l.scale};
    return a;
}

int fft_rows_cap(int K) { return K <= kFftPoints ? kFftPoints / K : 1; }

// Threads of a launch whose largest block holds `points` complex points: one
// per 16 points, whole waves, one to four.
static int fft_threads(int points)
{
    const int t = (points + kFftPerThread - 1) / kFftPerThread;
    return t < 64 ? 64 : (t > kFftMaxThreads ? kFftMaxThreads : (t + 63) / 64 * 64);
}

// Dynamic LDS for that thread count: 16 points per thread plus the twiddles.
static size_t fft_lds_bytes(int threads)
{
    return sizeof(double2) * ((size_t)lds_points(threads * kFftPerThread) + kTwEntries);
}

// Allows the largest dynamic LDS of these kernels (above the 64 KB default).
static int allow_lds()
{
    static const int rc = [] {
        const int bytes = (int)fft_lds_bytes(kFftMaxThreads);
        hipError_t e = hipFuncSetAttribute((const void*)k_c2r, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)k_r2c, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        return (int)e;
    }();
    return rc;
}

int launch_c2r(const FftLaunch& l, void* stream)
{
    if (l.K < 1 || l.K > kFftPoints || l.points < l.K || l.points > kFftPoints) return (int)hipErrorInvalidValue;
    if (int e = allow_lds()) return e;
    const int nt = fft_threads(l.points);
    hipLaunchKernelGGL(k_c2r, dim3(l.nblocks, l.grid_y), dim3(nt), fft_lds_bytes(nt),
                       (hipStream_t)stream, fft_args(l));
    return (int)hipGetLastError();
}

int launch_r2c(const FftLaunch& l, void* stream)
{
    if (l.K < 1 || l.K > kFftPoints || l.points < l.K || l.points > kFftPoints) return (int)hipErrorInvalidValue;
    if (int e = allow_lds()) return e;
    const int nt = fft_threads(l.points);
    hipLaunchKernelGGL(k_r2c, dim3(l.nblocks, l.grid_y), dim3(nt), fft_lds_bytes(nt),
                       (hipStream_t)stream, fft_args(l));
    return (int)hipGetLastError();
}

}  // namespace shtn
