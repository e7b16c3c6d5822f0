// Longitude stage of the SHT on gfx950: batched real FFTs in FP64 (Sec. 3.1,
// "use the FFT" and Hermitian symmetry of real data).
//
// A real transform of length N = 2K is computed as a complex FFT of length K
// on z_k = f_{2k} + i f_{2k+1}, with an O(K) pre/post-pass that separates the
// even and odd samples.  The complex FFT is a radix-4 (+ one radix-2 stage when
// log2 K is odd) Stockham autosort in LDS: each stage reads its operands into
// registers, synchronises, and writes them back in place.  A workgroup handles
// several latitude rows (up to 4096 complex points = 64 KB of LDS); the
// Fourier coefficients F_m(theta_i) are stored order-major ([m][latitude]) so
// the Legendre kernels access them with unit stride, and the rows of one
// workgroup are adjacent latitudes so those reads coalesce here too.
#include <hip/hip_runtime.h>

#include "shtn_internal.h"

namespace shtn {

constexpr int kFftThreads = 256;
constexpr int kFftPoints = 4096;  // complex points per workgroup

struct FftArgs {
    const DevPlan* plans;
    const int* rowblocks;  // per block {field, plan, row0, nrows}, or null for plan calls
    const long* g_off;     // per field grid offset in doubles, or null (f * nlat * nphi)
    const long* f_off;     // per field F offset in doubles, or null (f * 2 (M+1) nlat)
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

// One Stockham stage of radix R over `nrows` rows of length K held in buf.
// dir = -1: forward (e^{-2 pi i}), +1: inverse.
template <int R>
__device__ void stockham_stage(double2* buf, const double2* tw, int K, int nrows, int Ns, int dir)
{
    constexpr int MAXB = kFftPoints / (R * kFftThreads);
    const int KR = K / R;
    const int nb = nrows * KR;
    double2 v[MAXB][R];
    int dst[MAXB];
#pragma unroll
    for (int i = 0; i < MAXB; i++) {
        const int b = threadIdx.x + i * kFftThreads;
        if (b < nb) {
            const int r = b / KR, jj = b - r * KR;
            const int js = jj % Ns;
            double2* row = buf + r * K;
#pragma unroll
            for (int q = 0; q < R; q++) v[i][q] = row[jj + q * KR];
            const int tstep = js * (K / (Ns * R));
#pragma unroll
            for (int q = 1; q < R; q++) {
                double2 w = tw[q * tstep];
                if (dir > 0) w = cconj(w);
                v[i][q] = cmul(v[i][q], w);
            }
            if (R == 2) {
                const double2 a = v[i][0], c = v[i][1];
                v[i][0] = cadd(a, c);
                v[i][1] = csub(a, c);
            } else {
                // DFT_4 with e^{dir 2 pi i rk / 4}
                const double2 a0 = cadd(v[i][0], v[i][2]), a1 = csub(v[i][0], v[i][2]);
                const double2 b0 = cadd(v[i][1], v[i][3]), b1 = cmuli(csub(v[i][1], v[i][3]), dir);
                v[i][0] = cadd(a0, b0);
                v[i][2] = csub(a0, b0);
                v[i][1] = cadd(a1, b1);
                v[i][3] = csub(a1, b1);
            }
            dst[i] = r * K + (jj / Ns) * Ns * R + js;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXB; i++) {
        const int b = threadIdx.x + i * kFftThreads;
        if (b < nb) {
#pragma unroll
            for (int q = 0; q < R; q++) buf[dst[i] + q * Ns] = v[i][q];
        }
    }
    __syncthreads();
}

__device__ void complex_fft(double2* buf, const double2* tw, int K, int nrows, int dir)
{
    int Ns = 1;
    while (Ns < K) {
        if (K / Ns >= 4) {
            stockham_stage<4>(buf, tw, K, nrows, Ns, dir);
            Ns *= 4;
        } else {
            stockham_stage<2>(buf, tw, K, nrows, Ns, dir);
            Ns *= 2;
        }
    }
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
        rb.field = blockIdx.y;
        rb.plan = 0;
        rb.row0 = blockIdx.x * a.rows_per_block;
        rb.nrows = min(a.rows_per_block, nlat - rb.row0);
    }
    return rb;
}

// Fourier synthesis of rows: f_ik = Re F_0 + 2 Re sum_{m=1}^{M} F_m e^{2 pi i m k / N}.
__global__ void __launch_bounds__(kFftThreads) k_c2r(FftArgs a)
{
    __shared__ double2 buf[kFftPoints];
    const int pl = a.rowblocks ? a.rowblocks[4 * blockIdx.x + 1] : 0;
    const DevPlan& P = a.plans[pl];
    const RowBlock rb = row_block(a, P.nlat);
    if (rb.field >= a.nfields || rb.nrows <= 0) return;
    const int K = P.K, M = P.M, nlat = P.nlat, nphi = P.nphi;
    const double2* tw = (const double2*)P.tw;
    const double2* rtw = (const double2*)P.rtw;
    const double* F = a.in + (a.f_off ? a.f_off[rb.field] : (long)rb.field * 2 * (M + 1) * nlat);
    double* g = a.out + (a.g_off ? a.g_off[rb.field] : (long)rb.field * nlat * nphi);
    const int nr = rb.nrows;

    // Z_m = (Y_m + conj Y_{K-m}) + i w^m (Y_m - conj Y_{K-m}), Y_0 = Re F_0,
    // Y_m = F_m (1 <= m <= M), 0 otherwise (M < K).
    const int half = K / 2;
    for (int idx = threadIdx.x; idx < nr * (half + 1); idx += kFftThreads) {
        const int r = idx % nr, m = idx / nr;
        const int i = rb.row0 + r;
        const int mc = K - m;
        double2 ym = make_double2(0.0, 0.0), yc = make_double2(0.0, 0.0);
        if (m <= M) ym = *(const double2*)(F + 2 * ((size_t)m * nlat + i));
        if (m == 0) ym.y = 0.0;
        if (mc <= M && mc < K) yc = *(const double2*)(F + 2 * ((size_t)mc * nlat + i));
        const double2 s = cadd(ym, cconj(yc)), d = csub(ym, cconj(yc));
        const double2 zm = cadd(s, cmuli(cmul(rtw[m], d), 1));
        buf[r * K + (m % K)] = zm;
        if (m != 0 && mc != m) {
            // Z_{K-m} from the same pair: roles swapped, w^{K-m} = -conj(w^m)
            const double2 s2 = cadd(yc, cconj(ym)), d2 = csub(yc, cconj(ym));
            const double2 wc = make_double2(-rtw[m].x, rtw[m].y);
            buf[r * K + mc] = cadd(s2, cmuli(cmul(wc, d2), 1));
        }
    }
    __syncthreads();
    complex_fft(buf, tw, K, nr, +1);
    for (int idx = threadIdx.x; idx < nr * K; idx += kFftThreads) {
        const int r = idx / K, kk = idx - r * K;
        *(double2*)(g + (size_t)(rb.row0 + r) * nphi + 2 * kk) = buf[r * K + kk];
    }
}

// Fourier analysis of rows: F_m(theta_i) = scale * sum_k f_ik e^{-2 pi i m k / N}, m <= M.
__global__ void __launch_bounds__(kFftThreads) k_r2c(FftArgs a)
{
    __shared__ double2 buf[kFftPoints];
    const int pl = a.rowblocks ? a.rowblocks[4 * blockIdx.x + 1] : 0;
    const DevPlan& P = a.plans[pl];
    const RowBlock rb = row_block(a, P.nlat);
    if (rb.field >= a.nfields || rb.nrows <= 0) return;
    const int K = P.K, M = P.M, nlat = P.nlat, nphi = P.nphi;
    const double2* tw = (const double2*)P.tw;
    const double2* rtw = (const double2*)P.rtw;
    const double* g = a.in + (a.g_off ? a.g_off[rb.field] : (long)rb.field * nlat * nphi);
    double* F = a.out + (a.f_off ? a.f_off[rb.field] : (long)rb.field * 2 * (M + 1) * nlat);
    const int nr = rb.nrows;
    for (int idx = threadIdx.x; idx < nr * K; idx += kFftThreads) {
        const int r = idx / K, kk = idx - r * K;
        buf[r * K + kk] = *(const double2*)(g + (size_t)(rb.row0 + r) * nphi + 2 * kk);
    }
    __syncthreads();
    complex_fft(buf, tw, K, nr, -1);
    // scale <= 0: the analysis scale 2 pi / nphi of each field's plan
    const double sc = a.scale > 0.0 ? a.scale : 2.0 * 3.14159265358979323846 / nphi;
    for (int idx = threadIdx.x; idx < nr * (M + 1); idx += kFftThreads) {
        const int r = idx % nr, m = idx / nr;
        const double2 zm = buf[r * K + m];
        const double2 zc = cconj(buf[r * K + (K - m) % K]);
        const double2 A = make_double2(0.5 * (zm.x + zc.x), 0.5 * (zm.y + zc.y));
        const double2 D = csub(zm, zc);
        const double2 B = make_double2(0.5 * D.y, -0.5 * D.x);  // (Z_m - conj Z_{K-m}) / (2i)
        double2 X = cadd(A, cmul(cconj(rtw[m]), B));
        X.x *= sc;
        X.y = m == 0 ? 0.0 : X.y * sc;
        *(double2*)(F + 2 * ((size_t)m * nlat + rb.row0 + r)) = X;
    }
}

static FftArgs fft_args(const FftLaunch& l)
{
    FftArgs a{l.plans, l.rowblocks, l.g_off, l.f_off, l.in, l.out, l.nfields, l.rows_per_block,
              l.scale};
    return a;
}

int launch_c2r(const FftLaunch& l, void* stream)
{
    hipLaunchKernelGGL(k_c2r, dim3(l.nblocks, l.grid_y), dim3(kFftThreads), 0, (hipStream_t)stream,
                       fft_args(l));
    return (int)hipGetLastError();
}

int launch_r2c(const FftLaunch& l, void* stream)
{
    hipLaunchKernelGGL(k_r2c, dim3(l.nblocks, l.grid_y), dim3(kFftThreads), 0, (hipStream_t)stream,
                       fft_args(l));
    return (int)hipGetLastError();
}

}  // namespace shtn
