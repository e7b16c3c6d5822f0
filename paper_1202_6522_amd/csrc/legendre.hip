// Legendre stage of the Gauss-Legendre SHT on gfx950: FP64 vector ALUs.
//
// Synthesis (Sec. 2.2, eq. synth_direct) and analysis (Sec. 2.3, eq. gauss)
// with P_n^m generated on the fly by the three-term recurrence of Sec. 3.2
// (eq. rec), the equatorial mirror symmetry of Sec. 3.1 folded in (one lane
// carries the pair of latitudes x and -x: even degrees n-m add, odd degrees
// subtract), and the scaled-exponent underflow guard of Sec. 3.5.
//
// The recurrence runs in the rescaled form u_n = x u_{n-1} + beta_n u_{n-2}
// (two FP64 operations per step: one multiply by an SGPR coefficient and one
// FMA), with P_n^m = gamma_n u_n; gamma is folded into the spectrum before the
// synthesis and applied after the reduction in the analysis.  Recurrence
// coefficients and spectra are wave-uniform and are read with scalar loads
// into SGPRs, so every lane's FMAs take them as operands for free.
//
// One work unit = one wave of 64 lanes, LP latitude pairs per lane and FW
// fields that share the plan.
#include <hip/hip_runtime.h>

#include "shtn_internal.h"

namespace shtn {

typedef const __attribute__((address_space(4))) double* cdp;
typedef const __attribute__((address_space(4))) int* cip;
typedef const __attribute__((address_space(4))) long* clp;
typedef const __attribute__((address_space(4))) DevPlan* cplan;

struct LegArgs {
    const DevPlan* plans;
    const int* units;
    const long* q_off;  // per field: spectrum offset in doubles (null: f * 2 nlm)
    const long* f_off;  // per field: F offset in doubles (null: f * 2 (M+1) nlat)
    const double* in;
    double* out;
    int nfields;
    int adjoint;
};

__device__ __forceinline__ long field_q_off(const LegArgs& a, int f, long nlm)
{
    return a.q_off ? ((clp)a.q_off)[f] : (long)f * 2 * nlm;
}

__device__ __forceinline__ long field_f_off(const LegArgs& a, int f, int M, int nlat)
{
    return a.f_off ? ((clp)a.f_off)[f] : (long)f * 2 * (M + 1) * nlat;
}

__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0; }

// ---------------------------------------------------------------------------
// Spectrum rescaling: Qs = gamma * Q (complex), per field.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_prescale(const DevPlan* plans, const long* q_off, const long* s_off, const int* fplan,
           const double* Q, double* Qs, int nfields)
{
    const int f = blockIdx.y;
    if (f >= nfields) return;
    const int pi = fplan ? fplan[f] : 0;
    const DevPlan& P = plans[pi];
    const long qo = q_off ? q_off[f] : (long)f * 2 * P.nlm;
    const long so = s_off ? s_off[f] : (long)f * 2 * P.nlm;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < P.nlm;
         i += (long)gridDim.x * blockDim.x) {
        const double g = P.gamma[i];
        const double2 q = *(const double2*)(Q + qo + 2 * i);
        *(double2*)(Qs + so + 2 * i) = make_double2(g * q.x, g * q.y);
    }
}

// ---------------------------------------------------------------------------
// Synthesis: F_m(theta) for one order, LP pairs per lane, FW fields.
// ---------------------------------------------------------------------------
template <int LP, int FW>
struct SynthState {
    double x[LP], ua[LP], ub[LP];
    int k[LP];
    double er[LP][FW], ei[LP][FW], orr[LP][FW], oi[LP][FW];
};

// One even step (degree n = m + j) and one odd step (n + 1), unmasked.
template <int LP, int FW>
__device__ __forceinline__ void synth_pair_step(SynthState<LP, FW>& s, double b0, double b1,
                                                const double (&q0)[FW][2],
                                                const double (&q1)[FW][2], bool odd)
{
#pragma unroll
    for (int p = 0; p < LP; p++) s.ua[p] = fma(s.x[p], s.ub[p], b0 * s.ua[p]);
#pragma unroll
    for (int p = 0; p < LP; p++)
#pragma unroll
        for (int f = 0; f < FW; f++) {
            s.er[p][f] = fma(q0[f][0], s.ua[p], s.er[p][f]);
            s.ei[p][f] = fma(q0[f][1], s.ua[p], s.ei[p][f]);
        }
    if (odd) {
#pragma unroll
        for (int p = 0; p < LP; p++) s.ub[p] = fma(s.x[p], s.ua[p], b1 * s.ub[p]);
#pragma unroll
        for (int p = 0; p < LP; p++)
#pragma unroll
            for (int f = 0; f < FW; f++) {
                s.orr[p][f] = fma(q1[f][0], s.ub[p], s.orr[p][f]);
                s.oi[p][f] = fma(q1[f][1], s.ub[p], s.oi[p][f]);
            }
    }
}

// Same, with lanes whose guard exponent k > 0 contributing zero.
template <int LP, int FW>
__device__ __forceinline__ void synth_pair_step_masked(SynthState<LP, FW>& s, double b0,
                                                       double b1, const double (&q0)[FW][2],
                                                       const double (&q1)[FW][2], bool odd)
{
#pragma unroll
    for (int p = 0; p < LP; p++) s.ua[p] = fma(s.x[p], s.ub[p], b0 * s.ua[p]);
#pragma unroll
    for (int p = 0; p < LP; p++) {
        const double v = s.k[p] ? 0.0 : s.ua[p];
#pragma unroll
        for (int f = 0; f < FW; f++) {
            s.er[p][f] = fma(q0[f][0], v, s.er[p][f]);
            s.ei[p][f] = fma(q0[f][1], v, s.ei[p][f]);
        }
    }
    if (odd) {
#pragma unroll
        for (int p = 0; p < LP; p++) s.ub[p] = fma(s.x[p], s.ua[p], b1 * s.ub[p]);
#pragma unroll
        for (int p = 0; p < LP; p++) {
            const double v = s.k[p] ? 0.0 : s.ub[p];
#pragma unroll
            for (int f = 0; f < FW; f++) {
                s.orr[p][f] = fma(q1[f][0], v, s.orr[p][f]);
                s.oi[p][f] = fma(q1[f][1], v, s.oi[p][f]);
            }
        }
    }
}

template <int LP, int FW>
__device__ __forceinline__ void guard_check(SynthState<LP, FW>& s)
{
    const double down = 0x1p-256;
#pragma unroll
    for (int p = 0; p < LP; p++) {
        const bool big = fabs(s.ua[p]) >= 1.0 || fabs(s.ub[p]) >= 1.0;
        if (s.k[p] > 0 && big) {
            s.ua[p] *= down;
            s.ub[p] *= down;
            s.k[p] -= 1;
        }
    }
}

template <int LP, int FW>
__device__ __forceinline__ bool any_scaled(const SynthState<LP, FW>& s)
{
    bool any = false;
#pragma unroll
    for (int p = 0; p < LP; p++) any |= s.k[p] > 0;
    return wave_any(any);
}

template <int LP, int FW>
__global__ void __launch_bounds__(64) k_legendre_synth(LegArgs a)
{
    cip U = (cip)a.units + (size_t)blockIdx.x * kUnitInts;
    const int field0 = U[U_FIELD] + blockIdx.y * FW;
    if (field0 >= a.nfields) return;
    const int nf = min(U[U_NF], a.nfields - field0);
    cplan P = (cplan)a.plans + U[U_PLAN];
    const int L = P->L, M = P->M, nlat = P->nlat, npair = P->npair;
    const long nlm = P->nlm;
    const int lane = threadIdx.x;
    const int pb = U[U_PB];

    long qoff[FW];
    long foff[FW];
#pragma unroll
    for (int f = 0; f < FW; f++) {
        const int ff = field0 + min(f, nf - 1);
        qoff[f] = field_q_off(a, ff, nlm);
        foff[f] = field_f_off(a, ff, M, nlat);
    }

    for (int pass = 0; pass < 2; pass++) {
        const int m = pass == 0 ? U[U_M0] : U[U_M1];
        if (m < 0) break;
        const long base = (long)m * (2 * L + 1 - m) / 2 + m;
        const int nj = L - m + 1;
        cdp bet = (cdp)P->beta + base;
        cdp qs[FW];
#pragma unroll
        for (int f = 0; f < FW; f++) qs[f] = (cdp)(a.in + qoff[f]) + 2 * base;
        cip segexp = (cip)P->segexp + ((cip)P->segoff)[m];

        SynthState<LP, FW> s;
#pragma unroll
        for (int p = 0; p < LP; p++) {
            const int pair = pb + p * 64 + lane;
            const bool act = pair < npair;
            const int pc = act ? pair : 0;
            s.x[p] = act ? P->xp[pc] : 0.0;
            s.ua[p] = act ? P->start_y[(size_t)m * npair + pc] : 0.0;
            s.ub[p] = 0.0;
            s.k[p] = act ? P->start_k[(size_t)m * npair + pc] : 0;
#pragma unroll
            for (int f = 0; f < FW; f++) s.er[p][f] = s.ei[p][f] = s.orr[p][f] = s.oi[p][f] = 0.0;
        }
        bool guard = any_scaled(s);

        for (int js = 0; js < nj; js += kSegLen) {
            const int je = min(js + kSegLen, nj);
            if (js > 0) {
                const double sc = __builtin_amdgcn_ldexp(1.0, segexp[js / kSegLen]);
#pragma unroll
                for (int p = 0; p < LP; p++) {
                    s.ua[p] *= sc;
                    s.ub[p] *= sc;
                }
            }
            if (guard) {
                for (int j = js; j < je; j += 2) {
                    if ((j & (kGuardEvery - 1)) == 0) guard_check(s);
                    double q0[FW][2], q1[FW][2];
                    const bool odd = j + 1 < je;
                    const int jn = odd ? j + 1 : j;  // never index past the order's last degree
#pragma unroll
                    for (int f = 0; f < FW; f++) {
                        q0[f][0] = qs[f][2 * j];
                        q0[f][1] = qs[f][2 * j + 1];
                        q1[f][0] = qs[f][2 * jn];
                        q1[f][1] = qs[f][2 * jn + 1];
                    }
                    synth_pair_step_masked(s, bet[j], bet[jn], q0, q1, odd);
                }
                guard = any_scaled(s);
            } else if (je - js == kSegLen) {
#pragma unroll 4
                for (int j = js; j < je; j += 8) {
                    double b[8];
                    double q[FW][8][2];
#pragma unroll
                    for (int t = 0; t < 8; t++) {
                        b[t] = bet[j + t];
#pragma unroll
                        for (int f = 0; f < FW; f++) {
                            q[f][t][0] = qs[f][2 * (j + t)];
                            q[f][t][1] = qs[f][2 * (j + t) + 1];
                        }
                    }
#pragma unroll
                    for (int t = 0; t < 8; t += 2) {
                        double q0[FW][2], q1[FW][2];
#pragma unroll
                        for (int f = 0; f < FW; f++) {
                            q0[f][0] = q[f][t][0];
                            q0[f][1] = q[f][t][1];
                            q1[f][0] = q[f][t + 1][0];
                            q1[f][1] = q[f][t + 1][1];
                        }
                        synth_pair_step(s, b[t], b[t + 1], q0, q1, true);
                    }
                }
            } else {
                for (int j = js; j < je; j += 2) {
                    double q0[FW][2], q1[FW][2];
                    const bool odd = j + 1 < je;
                    const int jn = odd ? j + 1 : j;
#pragma unroll
                    for (int f = 0; f < FW; f++) {
                        q0[f][0] = qs[f][2 * j];
                        q0[f][1] = qs[f][2 * j + 1];
                        q1[f][0] = qs[f][2 * jn];
                        q1[f][1] = qs[f][2 * jn + 1];
                    }
                    synth_pair_step(s, bet[j], bet[jn], q0, q1, odd);
                }
            }
        }

        // Mirror fold: north = E + O, south = E - O.  For the adjoint of the
        // analysis the output carries (2 pi/nphi) w_i / c_m.
        const double cm = a.adjoint ? (2.0 * M_PI / P->nphi) * (m == 0 ? 1.0 : 0.5) : 1.0;
#pragma unroll
        for (int p = 0; p < LP; p++) {
            const int pair = pb + p * 64 + lane;
            if (pair >= npair) continue;
            const double sc = a.adjoint ? cm * P->wfull[pair] : 1.0;
            const int is = nlat - 1 - pair;
#pragma unroll
            for (int f = 0; f < FW; f++) {
                if (f >= nf) continue;
                double* F = a.out + foff[f] + 2 * ((size_t)m * nlat);
                *(double2*)(F + 2 * pair) =
                    make_double2(sc * (s.er[p][f] + s.orr[p][f]), sc * (s.ei[p][f] + s.oi[p][f]));
                if (is != pair)
                    *(double2*)(F + 2 * is) = make_double2(sc * (s.er[p][f] - s.orr[p][f]),
                                                           sc * (s.ei[p][f] - s.oi[p][f]));
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Analysis: Q_n^m = gamma_n sum_pairs u_n (w (F_N +- F_S)), one wave covers all
// latitude pairs of one order (64 LP >= npair) for a range of degrees.
// ---------------------------------------------------------------------------
template <int LP, int FW>
__global__ void __launch_bounds__(64) k_legendre_analys(LegArgs a)
{
    constexpr int C = kChunk;
    constexpr int NV = 2 * C * FW;  // reduced values per chunk: 32 or 64
    static_assert(NV == 32 || NV == 64, "chunk/field combination");
    __shared__ double red[NV][65];

    cip U = (cip)a.units + (size_t)blockIdx.x * kUnitInts;
    const int field0 = U[U_FIELD] + blockIdx.y * FW;
    if (field0 >= a.nfields) return;
    const int nf = min(U[U_NF], a.nfields - field0);
    cplan P = (cplan)a.plans + U[U_PLAN];
    const int L = P->L, M = P->M, nlat = P->nlat, npair = P->npair;
    const long nlm = P->nlm;
    const int lane = threadIdx.x;
    const int m = U[U_M0];
    const int j0 = U[U_PB], j1 = U[U_J1], rst = U[U_RST];
    const long base = (long)m * (2 * L + 1 - m) / 2 + m;
    cdp bet = (cdp)P->beta + base;
    cip segexp = (cip)P->segexp + ((cip)P->segoff)[m];

    long qoff[FW];
    long foff[FW];
#pragma unroll
    for (int f = 0; f < FW; f++) {
        const int ff = field0 + min(f, nf - 1);
        qoff[f] = field_q_off(a, ff, nlm);
        foff[f] = field_f_off(a, ff, M, nlat);
    }

    // per-pair inputs: folded, weighted Fourier coefficients
    double x[LP], ua[LP], ub[LP];
    int k[LP];
    double fer[LP][FW], fei[LP][FW], for_[LP][FW], foi[LP][FW];
#pragma unroll
    for (int p = 0; p < LP; p++) {
        const int pair = p * 64 + lane;
        const bool act = pair < npair;
        const int pc = act ? pair : 0;
        const bool middle = (nlat & 1) && pc == npair - 1;
        const double wt = !act ? 0.0 : (a.adjoint ? (middle ? 0.5 : 1.0) : P->wq[pc]);
        x[p] = act ? P->xp[pc] : 0.0;
        if (rst < 0) {
            ua[p] = act ? P->start_y[(size_t)m * npair + pc] : 0.0;
            ub[p] = 0.0;
            k[p] = act ? P->start_k[(size_t)m * npair + pc] : 0;
        } else {
            const double2 st = *(const double2*)(P->rst_y + 2 * ((size_t)rst * npair + pc));
            ua[p] = act ? st.x : 0.0;
            ub[p] = act ? st.y : 0.0;
            k[p] = act ? P->rst_k[(size_t)rst * npair + pc] : 0;
        }
#pragma unroll
        for (int f = 0; f < FW; f++) {
            const double* F = a.in + foff[f] + 2 * ((size_t)m * nlat);
            const double2 fn = *(const double2*)(F + 2 * pc);
            const double2 fs = *(const double2*)(F + 2 * (nlat - 1 - pc));
            fer[p][f] = wt * (fn.x + fs.x);
            fei[p][f] = wt * (fn.y + fs.y);
            for_[p][f] = wt * (fn.x - fs.x);
            foi[p][f] = wt * (fn.y - fs.y);
        }
    }
    bool anyk = false;
#pragma unroll
    for (int p = 0; p < LP; p++) anyk |= k[p] > 0;
    bool guard = wave_any(anyk);
    const double cm0 = 1.0, cm1 = a.adjoint ? 2.0 : 1.0;
    const double cm = m == 0 ? cm0 : cm1;
    const double down = 0x1p-256;

    for (int c = j0; c < j1; c += C) {
        double acc[C][FW][2];
#pragma unroll
        for (int t = 0; t < C; t++)
#pragma unroll
            for (int f = 0; f < FW; f++) acc[t][f][0] = acc[t][f][1] = 0.0;

#pragma unroll
        for (int t = 0; t < C; t++) {
            const int j = c + t;
            if (j < j1) {
                if ((t & 1) == 0) {
                    if (j > 0 && (j % kSegLen) == 0) {
                        const double sc = __builtin_amdgcn_ldexp(1.0, segexp[j / kSegLen]);
#pragma unroll
                        for (int p = 0; p < LP; p++) {
                            ua[p] *= sc;
                            ub[p] *= sc;
                        }
                    }
                    if (guard && (j & (kGuardEvery - 1)) == 0) {
                        bool any = false;
#pragma unroll
                        for (int p = 0; p < LP; p++) {
                            const bool big = fabs(ua[p]) >= 1.0 || fabs(ub[p]) >= 1.0;
                            if (k[p] > 0 && big) {
                                ua[p] *= down;
                                ub[p] *= down;
                                k[p] -= 1;
                            }
                            any |= k[p] > 0;
                        }
                        guard = wave_any(any);
                    }
                }
                const double b = bet[j];
                if ((t & 1) == 0) {
#pragma unroll
                    for (int p = 0; p < LP; p++) {
                        ua[p] = fma(x[p], ub[p], b * ua[p]);
                        const double v = k[p] ? 0.0 : ua[p];
#pragma unroll
                        for (int f = 0; f < FW; f++) {
                            acc[t][f][0] = fma(fer[p][f], v, acc[t][f][0]);
                            acc[t][f][1] = fma(fei[p][f], v, acc[t][f][1]);
                        }
                    }
                } else {
#pragma unroll
                    for (int p = 0; p < LP; p++) {
                        ub[p] = fma(x[p], ua[p], b * ub[p]);
                        const double v = k[p] ? 0.0 : ub[p];
#pragma unroll
                        for (int f = 0; f < FW; f++) {
                            acc[t][f][0] = fma(for_[p][f], v, acc[t][f][0]);
                            acc[t][f][1] = fma(foi[p][f], v, acc[t][f][1]);
                        }
                    }
                }
            }
        }

        // cross-lane reduction of the chunk through LDS
#pragma unroll
        for (int t = 0; t < C; t++)
#pragma unroll
            for (int f = 0; f < FW; f++) {
                red[(t * FW + f) * 2 + 0][lane] = acc[t][f][0];
                red[(t * FW + f) * 2 + 1][lane] = acc[t][f][1];
            }
        __syncthreads();
        double sum = 0.0;
        int v;
        if (NV == 32) {
            v = lane & 31;
            const int h = (lane >> 5) * 32;
#pragma unroll 8
            for (int r = 0; r < 32; r++) sum += red[v][h + r];
            sum += __shfl_xor(sum, 32);
        } else {
            v = lane;
#pragma unroll 8
            for (int r = 0; r < 64; r++) sum += red[v][r];
        }
        __syncthreads();
        const int t = v / (2 * FW);
        const int f = (v / 2) % FW;
        const int comp = v & 1;
        const int j = c + t;
        if (lane < NV && j < j1 && f < nf) {
            const long idx = base + j;
            double val = P->gamma[idx] * sum * cm;
            if (m == 0 && comp == 1) val = 0.0;
            a.out[qoff[f] + 2 * idx + comp] = val;
        }
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int launch_prescale(const DevPlan* plans, const long* q_off, const long* s_off, const int* fplan,
                    const double* Q, double* Qs, long max_nlm, int nfields, void* stream)
{
    const int blocks = (int)std::min<long>(1024, (max_nlm + 255) / 256);
    dim3 grid(std::max(1, blocks), nfields);
    hipLaunchKernelGGL(k_prescale, grid, dim3(256), 0, (hipStream_t)stream, plans, q_off, s_off,
                       fplan, Q, Qs, nfields);
    return (int)hipGetLastError();
}

template <int LP, int FW>
static int launch_synth_t(const LegLaunch& l, void* stream)
{
    LegArgs a{l.plans, l.units, l.q_off, l.f_off, l.in, l.out, l.nfields, l.adjoint};
    hipLaunchKernelGGL((k_legendre_synth<LP, FW>), dim3(l.nunits, l.grid_y), dim3(64), 0,
                       (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

template <int LP, int FW>
static int launch_analys_t(const LegLaunch& l, void* stream)
{
    LegArgs a{l.plans, l.units, l.q_off, l.f_off, l.in, l.out, l.nfields, l.adjoint};
    hipLaunchKernelGGL((k_legendre_analys<LP, FW>), dim3(l.nunits, l.grid_y), dim3(64), 0,
                       (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

int launch_legendre_synth(const LegLaunch& l, void* stream)
{
    if (l.nunits <= 0) return 0;
#define SHTN_S(LPV, FWV) \
    if (l.lp == LPV && l.fw == FWV) return launch_synth_t<LPV, FWV>(l, stream);
    SHTN_S(1, 1) SHTN_S(2, 1) SHTN_S(4, 1) SHTN_S(8, 1)
    SHTN_S(1, 2) SHTN_S(2, 2) SHTN_S(4, 2)
    SHTN_S(1, 4) SHTN_S(2, 4)
#undef SHTN_S
    return (int)hipErrorInvalidValue;
}

int launch_legendre_analys(const LegLaunch& l, void* stream)
{
    if (l.nunits <= 0) return 0;
#define SHTN_A(LPV, FWV) \
    if (l.lp == LPV && l.fw == FWV) return launch_analys_t<LPV, FWV>(l, stream);
    SHTN_A(1, 1) SHTN_A(2, 1) SHTN_A(4, 1) SHTN_A(8, 1)
    SHTN_A(1, 2) SHTN_A(2, 2) SHTN_A(4, 2)
#undef SHTN_A
    return (int)hipErrorInvalidValue;
}

}  // namespace shtn
