// Vector (spheroidal / toroidal) transforms on top of the scalar stages.
//
// A tangent field V = grad S + curl(T r) on the unit sphere has
//   V_theta = dS/dtheta - (1/sin) dT/dphi,  V_phi = (1/sin) dS/dphi + dT/dtheta.
// With sin(theta) dP_n^m/dtheta = n x P_n^m - c_n P_{n-1}^m,
// c_n = sqrt((2n+1)(n^2-m^2)/(2n-1)) (orthonormal P, x = cos theta), each
// order of each component is a combination of scalar Legendre sums:
//   sin Vt_m = x Syn(n S) - Syn(c_{n+1} S_{n+1} + i m T),
//   sin Vp_m = x Syn(n T) - Syn(c_{n+1} T_{n+1} - i m S),
// where Syn(Q)_m(theta) = sum_n Q_n^m P_n^m(x).  So the synthesis forms four
// spectra per field (k_vec_spec_in), runs the scalar Legendre synthesis on
// them as one 4-field call, and combines per (order, latitude)
// (k_vec_f_out) before the two longitude syntheses.  The analysis mirrors
// it: with A(g)_n = sum_i w_i g_i P_n^m(x_i),
//   n(n+1) S_n = n A(x Ft/s)_n - c_n A(Ft/s)_{n-1} - i m A(Fp/s)_n,
//   n(n+1) T_n = i m A(Ft/s)_n + n A(x Fp/s)_n - c_n A(Fp/s)_{n-1},
// the four weighted inputs formed by k_vec_f_in, the combination by
// k_vec_spec_out.  sin(theta) is taken as sqrt((1-x)(1+x)) of the node x the
// Legendre stage uses.
//
// Adjoints (the same kernels, `nn` selects the n(n+1) scaling): the
// transpose of the synthesis is the analysis combination without the
// division by n(n+1), fed by the scalar stages in their adjoint mode (unit
// weights, c_m, unnormalised longitude DFT); the transpose of the analysis
// forms the synthesis spectra from (S, T) / (n(n+1)) and runs the scalar
// synthesis in its adjoint mode.  Degree 0 and Im of order 0 carry nothing
// in either direction.
#include <hip/hip_runtime.h>

#include "shtn_internal.h"

namespace shtn {

__device__ __forceinline__ long vec_base(int L, int m) { return (long)m * (2 * L + 1 - m) / 2 + m; }

// c_n for order m (0 when n = m).
__device__ __forceinline__ double vec_c(int n, int m)
{
    return n > m ? sqrt((2.0 * n + 1) * ((double)n * n - (double)m * m) / (2.0 * n - 1)) : 0.0;
}

// 1/(n(n+1)), 0 at degree 0.
__device__ __forceinline__ double inv_nn(int n) { return n > 0 ? 1.0 / ((double)n * (n + 1.0)) : 0.0; }

// Q4[4f + k] from S[f], T[f]: k = 0: n S, 1: c_{n+1} S_{n+1} + i m T,
// 2: n T, 3: c_{n+1} T_{n+1} - i m S; with nn, S and T are first divided by
// n(n+1) (adjoint of the analysis).  One thread per (degree, order, field).
__global__ void __launch_bounds__(256) k_vec_spec_in(const DevPlan* plan, const double* S, const double* T,
                                                      double* Q4, int nfields, int nn)
{
    const DevPlan& P = *plan;
    const int m = blockIdx.y, f = blockIdx.z;
    const int n = m + blockIdx.x * 256 + threadIdx.x;
    if (n > P.L || f >= nfields) return;
    const long nlm = P.nlm;
    const long i = vec_base(P.L, m) + (n - m);
    const double2* s2 = (const double2*)(S + 2 * (long)f * nlm);
    const double2* t2 = (const double2*)(T + 2 * (long)f * nlm);
    const double w0 = nn ? inv_nn(n) : 1.0;
    double2 s = s2[i], t = t2[i];
    s = make_double2(w0 * s.x, w0 * s.y);
    t = make_double2(w0 * t.x, w0 * t.y);
    double2 sn = make_double2(0.0, 0.0), tn = sn;
    double c = 0.0;
    if (n < P.L) {
        sn = s2[i + 1];
        tn = t2[i + 1];
        c = vec_c(n + 1, m) * (nn ? inv_nn(n + 1) : 1.0);
    }
    const double dn = n, dm = m;
    double2* q = (double2*)(Q4 + 2 * (long)(4 * f) * nlm);
    q[i] = make_double2(dn * s.x, dn * s.y);
    q[nlm + i] = make_double2(c * sn.x - dm * t.y, c * sn.y + dm * t.x);
    q[2 * nlm + i] = make_double2(dn * t.x, dn * t.y);
    q[3 * nlm + i] = make_double2(c * tn.x + dm * s.y, c * tn.y - dm * s.x);
}

// Latitude and order of the e-th complex entry of a field's F (tiles of
// kFTile latitudes, see f_layout); false for the padding of the last tile.
__device__ __forceinline__ bool f_entry(const DevPlan& P, long e, int& m, int& lat)
{
    const long tile = e / P.f_ts, r = e % P.f_ts;
    m = (int)(r / kFTile);
    lat = (int)(tile * kFTile + r % kFTile);
    return lat < P.nlat;
}

__device__ __forceinline__ void node(const DevPlan& P, int lat, double& x, double& s)
{
    const bool north = lat < P.npair;
    const double xp = P.xp[north ? lat : P.nlat - 1 - lat];
    x = north ? xp : -xp;
    s = sqrt((1.0 - xp) * (1.0 + xp));
}

// Vt[f] = (x F4[4f] - F4[4f+1]) / s, Vp[f] = (x F4[4f+2] - F4[4f+3]) / s.
__global__ void __launch_bounds__(256) k_vec_f_out(const DevPlan* plan, const double* F4, double* Fv, int nfields)
{
    const DevPlan& P = *plan;
    const int f = blockIdx.y;
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    if (e >= P.f_size || f >= nfields) return;
    int m, lat;
    if (!f_entry(P, e, m, lat)) return;
    double x, s;
    node(P, lat, x, s);
    const double r = 1.0 / s;
    const long fs = P.f_size;
    const double2* a = (const double2*)F4 + (long)(4 * f) * fs + e;
    const double2 a0 = a[0], a1 = a[fs], a2 = a[2 * fs], a3 = a[3 * fs];
    double2* vt = (double2*)Fv + (long)f * fs + e;
    double2* vp = (double2*)Fv + (long)(nfields + f) * fs + e;
    *vt = make_double2((x * a0.x - a1.x) * r, (x * a0.y - a1.y) * r);
    *vp = make_double2((x * a2.x - a3.x) * r, (x * a2.y - a3.y) * r);
}

// F4[4f] = x Ft / s, F4[4f+1] = Ft / s, F4[4f+2] = x Fp / s, F4[4f+3] = Fp / s
// with Ft = Fv[f], Fp = Fv[nfields + f].
__global__ void __launch_bounds__(256) k_vec_f_in(const DevPlan* plan, const double* Fv, double* F4, int nfields)
{
    const DevPlan& P = *plan;
    const int f = blockIdx.y;
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    if (e >= P.f_size || f >= nfields) return;
    int m, lat;
    if (!f_entry(P, e, m, lat)) return;
    double x, s;
    node(P, lat, x, s);
    const double r = 1.0 / s;
    const long fs = P.f_size;
    const double2 t = ((const double2*)Fv)[(long)f * fs + e];
    const double2 p = ((const double2*)Fv)[(long)(nfields + f) * fs + e];
    double2* o = (double2*)F4 + (long)(4 * f) * fs + e;
    o[0] = make_double2(x * t.x * r, x * t.y * r);
    o[fs] = make_double2(t.x * r, t.y * r);
    o[2 * fs] = make_double2(x * p.x * r, x * p.y * r);
    o[3 * fs] = make_double2(p.x * r, p.y * r);
}

// S, T from the four analyses A4[4f + k] (k: x Ft/s, Ft/s, x Fp/s, Fp/s),
// divided by n(n+1) when nn (the analysis), not otherwise (the adjoint of
// the synthesis); 0 at degree 0.
__global__ void __launch_bounds__(256) k_vec_spec_out(const DevPlan* plan, const double* A4, double* S, double* T,
                                                       int nfields, int nn)
{
    const DevPlan& P = *plan;
    const int m = blockIdx.y, f = blockIdx.z;
    const int n = m + blockIdx.x * 256 + threadIdx.x;
    if (n > P.L || f >= nfields) return;
    const long nlm = P.nlm;
    const long i = vec_base(P.L, m) + (n - m);
    const double2* a = (const double2*)(A4 + 2 * (long)(4 * f) * nlm);
    const double2 a1 = a[i], a2 = a[nlm + i], a3 = a[2 * nlm + i], a4 = a[3 * nlm + i];
    double2 a2p = make_double2(0.0, 0.0), a4p = a2p;
    if (n > m) {
        a2p = a[nlm + i - 1];
        a4p = a[3 * nlm + i - 1];
    }
    const double c = vec_c(n, m), dn = n, dm = m;
    const double inv = n == 0 ? 0.0 : (nn ? inv_nn(n) : 1.0);
    // n A1 - c A2(n-1) - i m A4 ;  i m A2 + n A3 - c A4(n-1)
    double2 sv = make_double2((dn * a1.x - c * a2p.x + dm * a4.y) * inv, (dn * a1.y - c * a2p.y - dm * a4.x) * inv);
    double2 tv = make_double2((-dm * a2.y + dn * a3.x - c * a4p.x) * inv, (dm * a2.x + dn * a3.y - c * a4p.y) * inv);
    if (m == 0) {
        sv.y = 0.0;
        tv.y = 0.0;
    }
    ((double2*)(S + 2 * (long)f * nlm))[i] = sv;
    ((double2*)(T + 2 * (long)f * nlm))[i] = tv;
}

int launch_vec_spec_in(const DevPlan* plan, int L, int M, const double* S, const double* T, double* Q4, int nfields,
                       int nn, void* stream)
{
    hipLaunchKernelGGL(k_vec_spec_in, dim3((L + 256) / 256, M + 1, nfields), dim3(256), 0, (hipStream_t)stream,
                       plan, S, T, Q4, nfields, nn);
    return (int)hipGetLastError();
}

int launch_vec_f_out(const DevPlan* plan, long f_size, const double* F4, double* Fv, int nfields, void* stream)
{
    hipLaunchKernelGGL(k_vec_f_out, dim3((unsigned)((f_size + 255) / 256), nfields), dim3(256), 0,
                       (hipStream_t)stream, plan, F4, Fv, nfields);
    return (int)hipGetLastError();
}

int launch_vec_f_in(const DevPlan* plan, long f_size, const double* Fv, double* F4, int nfields, void* stream)
{
    hipLaunchKernelGGL(k_vec_f_in, dim3((unsigned)((f_size + 255) / 256), nfields), dim3(256), 0,
                       (hipStream_t)stream, plan, Fv, F4, nfields);
    return (int)hipGetLastError();
}

int launch_vec_spec_out(const DevPlan* plan, int L, int M, const double* A4, double* S, double* T, int nfields,
                        int nn, void* stream)
{
    hipLaunchKernelGGL(k_vec_spec_out, dim3((L + 256) / 256, M + 1, nfields), dim3(256), 0, (hipStream_t)stream,
                       plan, A4, S, T, nfields, nn);
    return (int)hipGetLastError();
}

}  // namespace shtn
