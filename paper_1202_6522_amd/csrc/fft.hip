// Longitude stage of the SHT on gfx950: batched real FFTs in FP64 (Sec. 3.1,
// "use the FFT" and Hermitian symmetry of real data).
//
// A real transform of length N = 2K is computed as a complex FFT of length K
// on z_k = f_{2k} + i f_{2k+1}, with an O(K) pre/post-pass that separates the
// even and odd samples.  The complex FFT is a Stockham autosort with radix-P
// passes (P points per thread: 4, 8 or 16; the 16-point DFT runs in
// registers as 4 x 4, the 8-point one as 2 x 4) and one radix-4 and/or
// radix-2 pass for the remaining factors.
//
// The longitude stage moves every byte of F and of the grid once and does
// little arithmetic, so it is bound by memory latency and bandwidth: a launch
// needs many waves in flight, on every SIMD.  A workgroup holds rows x K <=
// 4096 points in LDS (whole rows; at lmax 1023 four rows, so that the reads
// of F, stored in tiles of eight latitudes per order, come in 64-byte runs;
// 71 KB with the padding against bank conflicts), with one thread per P
// points: P = 8 up to K = 2048 (512 threads: at lmax 1023 2048 waves, two
// per SIMD), 16 at K = 4096.  Rows of K >= 1024 points read the K twiddles
// e^{-2 pi i t/K} from the plan's table in global memory; shorter rows copy
// them to LDS while their points arrive.  Every thread owns P points of every
// pass (P/R butterflies of radix R); all index arithmetic is shifts and masks
// (K is a power of two).  The rows and the pre/post-pass twiddles are
// requested before anything waits for memory.  Both directions load the points of each thread's
// butterfly of the first radix-P pass straight into registers and run that
// pass there; with P = 8 the last radix-8 pass and a radix-2 pass after it
// share one LDS round trip, and the c2r stores the grid rows from it.  Row
// blocks are spread over the XCDs so that neighbouring blocks share an L2.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "shtn_internal.h"

namespace shtn {

constexpr int kFftPoints = 4096;  // complex points per workgroup at most (LDS)

// Points per thread for rows of K points (see above), and the most threads a
// workgroup of that kind has.
__host__ __device__ constexpr int fft_pts(int K) { return K <= 2048 ? 8 : 16; }
__host__ __device__ constexpr int fft_max_threads(int P) { return kFftPoints / P; }
// Kernels built for rows of 2^lgk >= 1024 points read their twiddles from
// global memory (see tw_get); the others, and the general kernels (lgk = 0),
// from a copy in LDS.
__host__ __device__ constexpr bool fft_global_tw(int lgk) { return lgk >= 10; }

// Twiddle tables are read through global-address-space pointers (the plan
// descriptor holds them as generic pointers, which would compile to flat
// loads).
typedef const __attribute__((address_space(1))) double* gdp;


__device__ __forceinline__ double2 ld2(gdp t, int i) { return make_double2(t[2 * i], t[2 * i + 1]); }

// LDS slot of point x: one pad slot after every 16 points, so the strided
// writes of a radix-16 pass spread over the banks, and two more after every
// row of 2^rs >= 64 points (rs = 31: none), so that the same order of
// neighbouring rows, which the F loads and stores touch together, falls in
// different banks.
__device__ __forceinline__ int at(int x, int rs) { return x + (x >> 4) + ((x >> rs) << 1); }
// row shift for rows of 2^lgK points
__device__ __forceinline__ int row_shift(int lgK) { return lgK >= 6 ? lgK : 31; }
// slots for p points, whatever the row length
constexpr int lds_points(int p) { return p + p / 16 + p / 32; }
// twiddle t of the K-entry table in LDS, padded like the points: the
// strided reads of a pass's twiddles spread over the banks
__device__ __forceinline__ int tw_at(int t) { return t + (t >> 4); }
constexpr int tw_slots(int K) { return K + K / 16; }

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

// In-place 8-point DFT with e^{dir 2 pi i jk/8}: index j = 4 j1 + j2, k = k1
// + 2 k2.  Four DFT_2 over j1, twiddles e^{dir 2 pi i j2 k1/8}, two DFT_4
// over j2.  The result X[k1 + 2 k2] is left in v[4 k1 + k2].
__device__ __forceinline__ void dft8(double2 (&v)[8], int dir)
{
    constexpr double c = 0.70710678118654752440;
#pragma unroll
    for (int j2 = 0; j2 < 4; j2++) {
        const double2 a = v[j2], b = v[4 + j2];
        v[j2] = cadd(a, b);
        v[4 + j2] = csub(a, b);
    }
    const double sd = dir;
    v[5] = cmul(v[5], make_double2(c, sd * c));   // w^1
    v[6] = cmuli(v[6], dir);                      // w^2 = dir i
    v[7] = cmul(v[7], make_double2(-c, sd * c));  // w^3
    dft4(v, 0, 1, dir);
    dft4(v, 4, 1, dir);
}

// Register holding output q of dft_r<R>: the radix-16 DFT leaves X[k1 + 4 k2]
// in v[4 k1 + k2], the radix-8 one X[k1 + 2 k2] in v[4 k1 + k2]; the others
// are in natural order.
template <int R>
__device__ __forceinline__ constexpr int out_slot(int q)
{
    return R == 16 ? 4 * (q & 3) + (q >> 2) : (R == 8 ? 4 * (q & 1) + (q >> 1) : q);
}

template <int R>
__device__ __forceinline__ void dft_r(double2 (&v)[R], int dir)
{
    if constexpr (R == 16) {
        dft16(v, dir);
    } else if constexpr (R == 8) {
        dft8(v, dir);
    } else if constexpr (R == 4) {
        dft4(v, 0, 1, dir);
    } else {
        const double2 a = v[0], c = v[1];
        v[0] = cadd(a, c);
        v[1] = csub(a, c);
    }
}

// Twiddle e^{-2 pi i t/K}: from the LDS copy (padded slots), or with GT
// straight from the plan's table in global memory, where it stays in cache:
// for long rows the copy costs more than it saves (its staging, and LDS that
// at 2048 and 4096 points keeps a second workgroup off the CU).
template <bool GT>
__device__ __forceinline__ double2 tw_get(const double2* twl, gdp twg, int t)
{
    if constexpr (GT)
        return ld2(twg, t);
    else
        return twl[tw_at(t)];
}

// One Stockham pass of radix R over the rows held in buf (npts = rows x K
// points, K = 2^lgK); Ns = 2^lgNs = product of the radices of the previous
// passes; twl = the K twiddles e^{-2 pi i t/K} in LDS.  Each thread reads
// its P/R butterflies, the workgroup synchronises, then they are written
// back in place.  dir = -1 forward (e^{-2 pi i}), +1 inverse.
// ZIN (first pass of the synthesis only): buf holds Y_m and the pass reads
// Z_m = (Y_m + conj Y_{K-m}) + i w^m (Y_m - conj Y_{K-m}) instead, Y_K = 0,
// with w^m of each of the thread's points in zw.
template <int P, int R, int LGR, bool ZIN = false, bool GT = false>
__device__ __forceinline__ void stockham_pass(double2* buf, const double2* twl, int lgK, int npts, int lgNs,
                                              int dir, const double2 (*zw)[R] = nullptr, gdp twg = nullptr)
{
    const int rs = row_shift(lgK);
    static_assert(R <= P, "a thread holds whole butterflies");
    constexpr int NB = P / R;
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
            if constexpr (ZIN) {
#pragma unroll
                for (int q = 0; q < R; q++) {
                    const int m = jj + q * KR;
                    const double2 ym = buf[at(rowb + m, rs)];
                    const double2 yc = m == 0 ? make_double2(0.0, 0.0) : buf[at(rowb + (1 << lgK) - m, rs)];
                    const double2 sm = cadd(ym, cconj(yc)), d = csub(ym, cconj(yc));
                    v[i][q] = cadd(sm, cmuli(cmul(zw[i][q], d), 1));
                }
            } else {
                // jj < KR and q KR have no bit in common, and stay in the
                // row: the slots are the first one plus fixed offsets
                const int rd = at(rowb + jj, rs);
#pragma unroll
                for (int q = 0; q < R; q++) v[i][q] = buf[rd + q * KR + ((q * KR) >> 4)];
            }
            if (lgNs > 0) {  // the first pass has js = 0: all twiddles are 1
                // twiddle q is w^q, w = table entry js K / (Ns R): one read,
                // the powers by products at most four deep
                double2 w[R];
                w[1] = tw_get<GT>(twl, twg, js << (lgK - lgNs - LGR));
                if (dir > 0) w[1] = cconj(w[1]);
#pragma unroll
                for (int q = 2; q < R; q++) w[q] = cmul(w[q >> 1], w[q - (q >> 1)]);
#pragma unroll
                for (int q = 1; q < R; q++) v[i][q] = cmul(v[i][q], w[q]);
            }
            dft_r<R>(v[i], dir);
            dst[i] = rowb + (((jj >> lgNs) << (lgNs + LGR)) | js);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NB; i++) {
        if (dst[i] >= 0) {
            // dst has no bit in [lgNs, lgNs + LGR), where q << lgNs lies
            const int wr = at(dst[i], rs);
#pragma unroll
            for (int q = 0; q < R; q++) buf[wr + (q << lgNs) + ((q << lgNs) >> 4)] = v[i][out_slot<R>(q)];
        }
    }
    __syncthreads();
}

// v of the neighbouring lane (lanes 2i and 2i + 1 swap; DPP quad_perm
// [1,0,3,2]; every lane takes part).
__device__ __forceinline__ double swap_pair(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp((int)b, (int)b, 0xB1, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(b >> 32), (int)(b >> 32), 0xB1, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double2 swap_pair(double2 v) { return make_double2(swap_pair(v.x), swap_pair(v.y)); }

// The last radix-P pass (stage Ns = K/(2P)) and the radix-2 pass after it in
// one LDS round trip.  The outputs of radix-P butterflies js and js + Ns
// land K/2 apart, which is what the radix-2 pass pairs; they run on lanes 2i
// and 2i + 1, which swap half of their outputs and finish the radix-2
// butterflies of the even (lane 2i) and odd (lane 2i + 1) output slots.
// One butterfly per thread (P points), as stockham_pass<P, P, ...>.  With
// gout the results go straight to global memory (row r of the block at
// gout + r gstride, point p as the doubles 2p, 2p + 1) instead of buf.
template <int P, int LGP, bool GT = false>
__device__ __forceinline__ void stockham_last2(double2* buf, const double2* twl, int lgK, int npts, int dir,
                                               double* gout, size_t gstride, gdp twg = nullptr)
{
    const int rs = row_shift(lgK);
    const int lgNs = lgK - LGP - 1, Ns = 1 << lgNs;
    const int lgKR = lgK - LGP, KR = 1 << lgKR;  // 2 Ns radix-P butterflies per row
    const int nb = npts >> LGP;                 // even: lanes 2i and 2i + 1 are valid together
    const bool valid = (int)threadIdx.x < nb;
    const int bc = valid ? (int)threadIdx.x : 0;
    const int r = bc >> lgKR, u = bc & (KR - 1);
    const int half = u & 1, js = u >> 1;
    const int rowb = r << lgK;
    double2 v[P];
    const int rd = at(rowb + (half << lgNs) + js, rs);
#pragma unroll
    for (int q = 0; q < P; q++) v[q] = buf[rd + q * KR + ((q * KR) >> 4)];
    if (lgNs > 0) {
        double2 w[P];
        w[1] = tw_get<GT>(twl, twg, js << (lgK - lgNs - LGP));
        if (dir > 0) w[1] = cconj(w[1]);
#pragma unroll
        for (int q = 2; q < P; q++) w[q] = cmul(w[q >> 1], w[q - (q >> 1)]);
#pragma unroll
        for (int q = 1; q < P; q++) v[q] = cmul(v[q], w[q]);
    }
    dft_r<P>(v, dir);
    // output slot q of this lane's butterfly: v[out_slot<P>(q)], at js + q Ns
    // of its half of the row
    double2 lo[P / 2], hi[P / 2];
#pragma unroll
    for (int k = 0; k < P / 2; k++) {
        // (fixed register indices, the lane's choice by selects)
        const double2 ev = v[out_slot<P>(2 * k)], od = v[out_slot<P>(2 * k + 1)];
        const double2 mine = half ? od : ev;
        const double2 got = swap_pair(half ? ev : od);
        const double2 a = half ? got : mine, b = half ? mine : got;
        double2 w = tw_get<GT>(twl, twg, js + (2 * k + half) * Ns);
        if (dir > 0) w = cconj(w);
        const double2 t = cmul(w, b);
        lo[k] = cadd(a, t);
        hi[k] = csub(a, t);
    }
    const int K2 = 1 << (lgK - 1);
    if (gout) {
        if (valid) {
            double* row = gout + (size_t)r * gstride + 2 * js;
#pragma unroll
            for (int k = 0; k < P / 2; k++) {
                const int o = (2 * k + half) * Ns;
                *(double2*)(row + 2 * o) = lo[k];
                *(double2*)(row + 2 * (K2 + o)) = hi[k];
            }
        }
        return;
    }
    __syncthreads();
    if (valid) {
        const int wr = at(rowb + js, rs);
#pragma unroll
        for (int k = 0; k < P / 2; k++) {
            const int o = (2 * k + half) * Ns;  // js + o and K/2 + js + o: no bit of js in o
            buf[wr + o + (o >> 4)] = lo[k];
            buf[wr + K2 + o + ((K2 + o) >> 4)] = hi[k];
        }
    }
    __syncthreads();
}

// Complex FFT of length K = 2^lgK on every row held in buf: radix P while
// lg P or more factors of 2 remain, then one radix-4 and/or radix-2 pass
// (with eight points per thread a last radix-2 pass joins the radix-8 one
// before it).
template <int P>
constexpr int lg_pts() { return P == 16 ? 4 : (P == 8 ? 3 : 2); }

// zw non-null: the first pass is of radix P (lgK >= lg P) and forms the
// synthesis's Z from Y in buf (see stockham_pass).  gout non-null: when the
// last passes are the joined radix-8 and radix-2 ones, they store the result
// there (see stockham_last2) and the call returns true; else it is in buf.
template <int P, bool GT = false>
__device__ __forceinline__ bool complex_fft(double2* buf, const double2* twl, int lgK, int npts, int dir,
                                            const double2 (*zw)[P] = nullptr, double* gout = nullptr,
                                            size_t gstride = 0, int lgNs0 = 0, gdp twg = nullptr)
{
    constexpr int LGP = lg_pts<P>();
    int lgNs = lgNs0;
    if (zw) {
        stockham_pass<P, P, LGP, true, GT>(buf, twl, lgK, npts, 0, dir, zw, twg);
        lgNs = LGP;
    }
    while (lgK - lgNs >= LGP) {
        if (P == 8 && lgK - lgNs == LGP + 1) {
            stockham_last2<P, LGP, GT>(buf, twl, lgK, npts, dir, gout, gstride, twg);
            return gout != nullptr;
        }
        stockham_pass<P, P, LGP, false, GT>(buf, twl, lgK, npts, lgNs, dir, nullptr, twg);
        lgNs += LGP;
    }
    if (P > 4 && lgK - lgNs >= 2) {
        stockham_pass<P, 4, 2, false, GT>(buf, twl, lgK, npts, lgNs, dir, nullptr, twg);
        lgNs += 2;
    }
    if (lgK - lgNs == 1) stockham_pass<P, 2, 1, false, GT>(buf, twl, lgK, npts, lgNs, dir, nullptr, twg);
    return false;
}

// Copies the K-entry table e^{-2 pi i t/K} from global memory to LDS.
__device__ __forceinline__ void stage_twiddles(double2* twl, gdp tw, int K)
{
    for (int t = threadIdx.x; t < K; t += blockDim.x) twl[tw_at(t)] = ld2(tw, t);
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
template <int P, bool LOAD>
__device__ __forceinline__ void move_f(double2* buf, const double* Fin, double* Fout, long ts, int M,
                                       int lgK, int row0, int nrows)
{
    const int rs = row_shift(lgK);
    const int run = nrows < kFTile ? nrows : kFTile;  // rows per tile in the block
    const bool pow2 = (run & (run - 1)) == 0;
    if (LOAD && pow2 && nrows <= kFTile && (row0 & (nrows - 1)) == 0) {
        // The block is one aligned run inside a tile: entry e is order
        // e >> lg, row e & (nrows - 1).  Every thread owns at most
        // P entries (nrows (M+1) <= nrows K <= P
        // threads), all loaded, from valid addresses, before any LDS write:
        // one memory round trip instead of one per entry.
        const int lg = __builtin_ctz(nrows);
        const int n = nrows * (M + 1);
        const long tb = (long)(row0 >> kFTileLg) * ts + (row0 & (kFTile - 1));
        double2 v[P];
#pragma unroll
        for (int k = 0; k < P; k++) {
            const int e = threadIdx.x + k * blockDim.x;
            const int ec = e < n ? e : 0;
            v[k] = *(const double2*)(Fin + 2 * (tb + ((long)(ec >> lg) << kFTileLg) + (ec & (nrows - 1))));
        }
#pragma unroll
        for (int k = 0; k < P; k++) {
            const int e = threadIdx.x + k * blockDim.x;
            const int m = e >> lg, r = e & (nrows - 1);
            if (e < n) buf[at((r << lgK) + m, rs)] = make_double2(v[k].x, m == 0 ? 0.0 : v[k].y);
        }
        return;
    }
    if (!LOAD && pow2 && nrows <= kFTile && (row0 & (nrows - 1)) == 0) {
        // store side of the same run: all LDS reads first, then the stores
        const int lg = __builtin_ctz(nrows);
        const int n = nrows * (M + 1);
        const long tb = (long)(row0 >> kFTileLg) * ts + (row0 & (kFTile - 1));
        double2 v[P];
#pragma unroll
        for (int k = 0; k < P; k++) {
            const int e = threadIdx.x + k * blockDim.x;
            const int ec = e < n ? e : 0;
            v[k] = buf[at(((ec & (nrows - 1)) << lgK) + (ec >> lg), rs)];
        }
#pragma unroll
        for (int k = 0; k < P; k++) {
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
                    buf[at((r << lgK) + m, rs)] = y;
                } else {
                    *(double2*)(Fout + 2 * off) = buf[at((r << lgK) + m, rs)];
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
                buf[at((r << lgK) + m, rs)] = y;
            } else {
                *(double2*)(Fout + 2 * off) = buf[at((r << lgK) + m, rs)];
            }
        }
    }
}

// Fourier synthesis of rows: f_ik = Re F_0 + 2 Re sum_{m=1}^{M} F_m e^{2 pi i m k / N}.
// LGK > 0: every row of the launch has K = 2^LGK points, so the passes and
// all index arithmetic are fixed at compile time; LGK = 0: K per block.
template <int P, int LGK>
__global__ void __launch_bounds__(fft_max_threads(P)) k_c2r(FftArgs a)
{
    extern __shared__ double2 lds[];  // points (P per thread), then the twiddle table
    double2* buf = lds;
    constexpr bool GT = fft_global_tw(LGK);
    double2* twl = lds + lds_points(blockDim.x * P);  // unused with GT
    const int pl = a.rowblocks ? a.rowblocks[4 * blockIdx.x + 1] : 0;
    const DevPlan& D = a.plans[pl];
    const RowBlock rb = row_block(a, D.nlat);
    if (rb.field >= a.nfields || rb.nrows <= 0) return;
    const int K = LGK > 0 ? 1 << LGK : D.K, M = D.M, nlat = D.nlat, nphi = D.nphi;
    const int lgK = LGK > 0 ? LGK : __builtin_ctz(K), rs = row_shift(lgK);
    const gdp tw = (gdp)D.tw;
    const gdp rtw = (gdp)D.rtw;
    const double* F = a.in + (a.f_off ? a.f_off[rb.field] : (long)rb.field * 2 * D.f_size);
    double* g = a.out + (a.g_off ? a.g_off[rb.field] : (long)rb.field * nlat * nphi);
    const int npts = rb.nrows << lgK;

    // Z_m = (Y_m + conj Y_{K-m}) + i w^m (Y_m - conj Y_{K-m}), w = e^{i pi/K},
    // Y_K = 0 (M < K): formed by the first radix-P pass as it reads Y, when
    // there is one (lgK >= lg P), else by a pass of its own.
    constexpr int LGP = lg_pts<P>();
    const bool fused = lgK >= LGP;
    double* grow = g + (size_t)rb.row0 * nphi;  // the block's first grid row
    // When the block is a power-of-two run of two or more rows aligned inside
    // an F tile (the usual case), each thread loads the points of its
    // butterfly of the first pass, Y_m for m = jj + q K/P and their mirrors
    // Y_{K-m}, straight from F (rows fastest over the threads: four threads
    // read one 64-byte run of a tile), forms Z and runs that pass in
    // registers: Y never goes through LDS.  A block of one row (K = 4096)
    // would read every F value twice in 16-byte pieces; it goes through LDS.
    if (fused && rb.nrows >= 2 && (rb.nrows & (rb.nrows - 1)) == 0 && rb.nrows <= kFTile &&
        (rb.row0 & (rb.nrows - 1)) == 0) {
        const int lgr = __builtin_ctz(rb.nrows);
        const int lgKR = lgK - LGP;
        const int nb = npts >> LGP;
        const int bc = (int)threadIdx.x < nb ? (int)threadIdx.x : 0;
        const int r = bc & (rb.nrows - 1), jj = bc >> lgr;
        const double* Fr = F + 2 * ((long)(rb.row0 >> kFTileLg) * D.f_ts + (rb.row0 & (kFTile - 1)) + r);
        // straight-line loads from valid addresses (orders above M read
        // order 0 and are replaced by 0 below)
        double2 ym[P], yc[P], rw[P];
#pragma unroll
        for (int q = 0; q < P; q++) {
            const int m = jj + (q << lgKR), mc = K - m;  // mc = K only for m = 0
            ym[q] = *(const double2*)(Fr + 2 * ((long)(m <= M ? m : 0) << kFTileLg));
            yc[q] = *(const double2*)(Fr + 2 * ((long)(mc <= M ? mc : 0) << kFTileLg));
            rw[q] = ld2(rtw, m);
        }
        if (!GT) stage_twiddles(twl, tw, K);
        double2 v[P];
#pragma unroll
        for (int q = 0; q < P; q++) {
            const int m = jj + (q << lgKR), mc = K - m;
            const double2 y = m > M ? make_double2(0.0, 0.0) : make_double2(ym[q].x, m == 0 ? 0.0 : ym[q].y);
            const double2 c = mc > M ? make_double2(0.0, 0.0) : yc[q];
            const double2 sm = cadd(y, cconj(c)), d = csub(y, cconj(c));
            v[q] = cadd(sm, cmuli(cmul(rw[q], d), 1));
        }
        // the first pass (Ns = 1, no twiddles): outputs to slots
        // (jj << lg P) + q of the row
        dft_r<P>(v, +1);
        if ((int)threadIdx.x < nb) {
            const int wr = at((r << lgK) + (jj << LGP), rs);  // jj << lg P has no bit below lg P
#pragma unroll
            for (int q = 0; q < P; q++) buf[wr + q + (q >> 4)] = v[out_slot<P>(q)];
        }
        __syncthreads();
        if (complex_fft<P, GT>(buf, twl, lgK, npts, +1, nullptr, grow, nphi, LGP, tw)) return;
#pragma unroll
        for (int e = 0; e < P; e++) {
            const int idx = threadIdx.x + e * blockDim.x;
            if (idx < npts) {
                const int rr = idx >> lgK, k = idx & (K - 1);
                *(double2*)(grow + (size_t)rr * nphi + 2 * k) = buf[at(idx, rs)];
            }
        }
        return;
    }
    // w^m of the points this thread forms Z for, loaded while the rows arrive
    double2 rw[P];
    if (fused) {
        const int jj = threadIdx.x & ((K >> LGP) - 1);
#pragma unroll
        for (int q = 0; q < P; q++) rw[q] = ld2(rtw, jj + q * (K >> LGP));
    } else {
#pragma unroll
        for (int e = 0; e < P; e++) rw[e] = ld2(rtw, (threadIdx.x + e * blockDim.x) & (K - 1));
    }
    // Y_m (Y_0 = Re F_0, Y_m = F_m for 1 <= m <= M, 0 above) row by row
    for (int idx = threadIdx.x; idx < npts; idx += blockDim.x)
        if ((idx & (K - 1)) > M) buf[at(idx, rs)] = make_double2(0.0, 0.0);
    move_f<P, true>(buf, F, nullptr, D.f_ts, M, lgK, rb.row0, rb.nrows);
    if (!GT) stage_twiddles(twl, tw, K);
    __syncthreads();
    bool stored;
    if (fused) {
        const double2(*zw)[P] = (const double2(*)[P])rw;
        stored = complex_fft<P, GT>(buf, twl, lgK, npts, +1, zw, grow, nphi, 0, tw);
    } else {
        double2 z[P];
#pragma unroll
        for (int e = 0; e < P; e++) {
            const int idx = threadIdx.x + e * blockDim.x;
            z[e] = make_double2(0.0, 0.0);
            if (idx < npts) {
                const int m = idx & (K - 1);
                const double2 ym = buf[at(idx, rs)];
                const double2 yc = m == 0 ? make_double2(0.0, 0.0) : buf[at(idx - m + (K - m), rs)];
                const double2 s = cadd(ym, cconj(yc)), d = csub(ym, cconj(yc));
                z[e] = cadd(s, cmuli(cmul(rw[e], d), 1));
            }
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < P; e++) {
            const int idx = threadIdx.x + e * blockDim.x;
            if (idx < npts) buf[at(idx, rs)] = z[e];
        }
        __syncthreads();
        stored = complex_fft<P, GT>(buf, twl, lgK, npts, +1, nullptr, grow, nphi, 0, tw);
    }
    if (stored) return;
#pragma unroll
    for (int e = 0; e < P; e++) {
        const int idx = threadIdx.x + e * blockDim.x;
        if (idx < npts) {
            const int r = idx >> lgK, k = idx & (K - 1);
            *(double2*)(grow + (size_t)r * nphi + 2 * k) = buf[at(idx, rs)];
        }
    }
}

// Fourier analysis of rows: F_m(theta_i) = scale * sum_k f_ik e^{-2 pi i m k / N}, m <= M
// (LGK as for k_c2r).
template <int P, int LGK>
__global__ void __launch_bounds__(fft_max_threads(P)) k_r2c(FftArgs a)
{
    extern __shared__ double2 lds[];  // points (P per thread), then the twiddle table
    double2* buf = lds;
    constexpr bool GT = fft_global_tw(LGK);
    double2* twl = lds + lds_points(blockDim.x * P);  // unused with GT
    const int pl = a.rowblocks ? a.rowblocks[4 * blockIdx.x + 1] : 0;
    const DevPlan& D = a.plans[pl];
    const RowBlock rb = row_block(a, D.nlat);
    if (rb.field >= a.nfields || rb.nrows <= 0) return;
    const int K = LGK > 0 ? 1 << LGK : D.K, M = D.M, nlat = D.nlat, nphi = D.nphi;
    const int lgK = LGK > 0 ? LGK : __builtin_ctz(K), rs = row_shift(lgK);
    const gdp tw = (gdp)D.tw;
    const gdp rtw = (gdp)D.rtw;
    const double* g = a.in + (a.g_off ? a.g_off[rb.field] : (long)rb.field * nlat * nphi);
    double* F = a.out + (a.f_off ? a.f_off[rb.field] : (long)rb.field * 2 * D.f_size);
    const int npts = rb.nrows << lgK;
    // Straight-line loads from valid addresses, then LDS writes without
    // branches (idx < P blockDim stays inside the point buffer; slots past
    // npts are never read), so every load is issued before the first wait.
    double2 v[P];
    // With lgK >= lg P the thread loads the P points of its butterfly of the
    // first radix-P pass (jj + q K/P of its row), which then runs in
    // registers; else the points idx = tid + e blockDim, put in LDS as they are.
    constexpr int LGP = lg_pts<P>();
    const bool first_in_regs = lgK >= LGP;
    const int lgKR = lgK - LGP;
    const int nb = npts >> LGP;
    const int bc = (int)threadIdx.x < nb ? (int)threadIdx.x : 0;
#pragma unroll
    for (int e = 0; e < P; e++) {
        int r, k;
        if (first_in_regs) {
            r = bc >> lgKR;
            k = (bc & ((1 << lgKR) - 1)) + (e << lgKR);
        } else {
            const int idx = threadIdx.x + e * blockDim.x;
            const int ic = idx < npts ? idx : 0;
            r = ic >> lgK;
            k = ic & (K - 1);
        }
        v[e] = *(const double2*)(g + (size_t)(rb.row0 + r) * nphi + 2 * k);
    }
    // When the block is a power-of-two run of rows aligned inside an F tile
    // (the usual case), each thread computes the outputs X_m it stores,
    // straight from Z in LDS (entry e: order e >> lg, row e & (nrows - 1));
    // otherwise a post-pass writes X over the buffer first.
    const bool direct = (rb.nrows & (rb.nrows - 1)) == 0 && rb.nrows <= kFTile && (rb.row0 & (rb.nrows - 1)) == 0;
    const int lgr = __builtin_ctz(rb.nrows);
    const int nout = rb.nrows * (M + 1);
    // w^m of this thread's outputs for the post-pass, requested with the rows
    double2 rw[P];
#pragma unroll
    for (int e = 0; e < P; e++) {
        const int idx = threadIdx.x + e * blockDim.x;
        rw[e] = ld2(rtw, direct ? ((idx < nout ? idx : 0) >> lgr) : (idx & (K - 1)));
    }
    if (!GT) stage_twiddles(twl, tw, K);
    if (first_in_regs) {
        // the first pass (Ns = 1, no twiddles): DFT of the loaded points,
        // outputs to slots (jj << lg P) + q of the row
        dft_r<P>(v, -1);
        if ((int)threadIdx.x < nb) {
            const int r = bc >> lgKR, jj = bc & ((1 << lgKR) - 1);
            const int wr = at((r << lgK) + (jj << LGP), rs);  // jj << lg P has no bit below lg P
#pragma unroll
            for (int q = 0; q < P; q++) buf[wr + q + (q >> 4)] = v[out_slot<P>(q)];
        }
        __syncthreads();
        complex_fft<P, GT>(buf, twl, lgK, npts, -1, nullptr, nullptr, 0, LGP, tw);
    } else {
#pragma unroll
        for (int e = 0; e < P; e++) buf[at(threadIdx.x + e * blockDim.x, rs)] = v[e];
        __syncthreads();
        complex_fft<P, GT>(buf, twl, lgK, npts, -1, nullptr, nullptr, 0, 0, tw);
    }
    // scale <= 0: the analysis scale 2 pi / nphi of each field's plan
    const double sc = a.scale > 0.0 ? a.scale : 2.0 * 3.14159265358979323846 / nphi;
    // X_m = (Z_m + conj Z_{K-m}) / 2 + conj(w^m) (Z_m - conj Z_{K-m}) / (2i),
    // scaled; Im X_0 = 0
    auto post = [&](double2 zm, double2 zc, double2 w, int m) {
        const double2 A = make_double2(0.5 * (zm.x + zc.x), 0.5 * (zm.y + zc.y));
        const double2 Dd = csub(zm, zc);
        const double2 B = make_double2(0.5 * Dd.y, -0.5 * Dd.x);
        double2 X = cadd(A, cmul(cconj(w), B));
        X.x *= sc;
        X.y = m == 0 ? 0.0 : X.y * sc;
        return X;
    };
    if (direct) {
        const long tb = (long)(rb.row0 >> kFTileLg) * D.f_ts + (rb.row0 & (kFTile - 1));
        double2 x[P];
#pragma unroll
        for (int e = 0; e < P; e++) {
            const int idx = threadIdx.x + e * blockDim.x;
            const int ec = idx < nout ? idx : 0;
            const int m = ec >> lgr, rbase = (ec & (rb.nrows - 1)) << lgK;
            x[e] = post(buf[at(rbase + m, rs)], cconj(buf[at(rbase + ((K - m) & (K - 1)), rs)]), rw[e], m);
        }
#pragma unroll
        for (int e = 0; e < P; e++) {
            const int idx = threadIdx.x + e * blockDim.x;
            if (idx < nout)
                *(double2*)(F + 2 * (tb + ((long)(idx >> lgr) << kFTileLg) + (idx & (rb.nrows - 1)))) = x[e];
        }
        return;
    }
    // X_m from Z_m and Z_{K-m}, computed in registers, then written over the
    // buffer so that F leaves in tile order
    // (straight-line: every index below stays inside the point buffer, a
    // row of K points lying within its P blockDim slots; points past npts
    // are computed from unused slots and never read back)
    double2 x[P];
#pragma unroll
    for (int e = 0; e < P; e++) {
        const int idx = threadIdx.x + e * blockDim.x;
        const int m = idx & (K - 1);
        x[e] = post(buf[at(idx, rs)], cconj(buf[at(idx - m + ((K - m) & (K - 1)), rs)]), rw[e], m);
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < P; e++) buf[at(threadIdx.x + e * blockDim.x, rs)] = x[e];
    __syncthreads();
    move_f<P, false>(buf, nullptr, F, D.f_ts, M, lgK, rb.row0, rb.nrows);
}

static FftArgs fft_args(const FftLaunch& l)
{
    FftArgs a{l.plans, l.rowblocks, l.g_off, l.f_off, l.in, l.out, l.nfields, l.rows_per_block,
              l.scale};
    return a;
}

int fft_rows_cap(int K) { return K <= kFftPoints ? kFftPoints / K : 1; }

// Threads of a launch whose largest block holds `points` complex points: one
// per P points, whole waves.
static int fft_threads(int points, int P)
{
    const int t = (points + P - 1) / P;
    return t < 64 ? 64 : std::min(fft_max_threads(P), (t + 63) / 64 * 64);
}

// Dynamic LDS for that thread count and row length: P points per thread
// plus the K twiddles.
static size_t fft_lds_bytes(int threads, int P, int K, bool global_tw)
{
    return sizeof(double2) * ((size_t)lds_points(threads * P) + (global_tw ? 0 : tw_slots(K)));
}

// Allows the largest dynamic LDS of these kernels (above the 64 KB default).
template <int P, int LGK>
static int allow_lds()
{
    static const int rc = [] {
        const int bytes = (int)fft_lds_bytes(fft_max_threads(P), P, kFftPoints, fft_global_tw(LGK));
        hipError_t e =
            hipFuncSetAttribute((const void*)k_c2r<P, LGK>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)k_r2c<P, LGK>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        return (int)e;
    }();
    return rc;
}

template <int P, int LGK, bool C2R>
static int launch_fft_t(const FftLaunch& l, void* stream)
{
    if (int e = allow_lds<P, LGK>()) return e;
    const int nt = fft_threads(l.points, P);
    if (nt * P < l.points) return (int)hipErrorInvalidValue;
    const size_t lds = fft_lds_bytes(nt, P, l.K, fft_global_tw(LGK));
    if (C2R)
        hipLaunchKernelGGL((k_c2r<P, LGK>), dim3(l.nblocks, l.grid_y), dim3(nt), lds, (hipStream_t)stream,
                           fft_args(l));
    else
        hipLaunchKernelGGL((k_r2c<P, LGK>), dim3(l.nblocks, l.grid_y), dim3(nt), lds, (hipStream_t)stream,
                           fft_args(l));
    return (int)hipGetLastError();
}

// One points-per-thread variant per launch, chosen by its longest rows; when
// every row has the same K = 64 ... 4096 points, the variant built for it.
template <bool C2R>
static int launch_fft(const FftLaunch& l, void* stream)
{
    if (l.K < 1 || l.K > kFftPoints || l.points < l.K || l.points > kFftPoints) return (int)hipErrorInvalidValue;
    if (l.uniform_k) {
        switch (l.K) {
        case 64: return launch_fft_t<8, 6, C2R>(l, stream);
        case 128: return launch_fft_t<8, 7, C2R>(l, stream);
        case 256: return launch_fft_t<8, 8, C2R>(l, stream);
        case 512: return launch_fft_t<8, 9, C2R>(l, stream);
        case 1024: return launch_fft_t<8, 10, C2R>(l, stream);
        case 2048: return launch_fft_t<8, 11, C2R>(l, stream);
        case 4096: return launch_fft_t<16, 12, C2R>(l, stream);
        default: break;
        }
    }
    return fft_pts(l.K) == 8 ? launch_fft_t<8, 0, C2R>(l, stream) : launch_fft_t<16, 0, C2R>(l, stream);
}

int launch_c2r(const FftLaunch& l, void* stream) { return launch_fft<true>(l, stream); }

int launch_r2c(const FftLaunch& l, void* stream) { return launch_fft<false>(l, stream); }

}  // namespace shtn
