// Legendre stage of the Gauss-Legendre SHT on gfx950: FP64 vector ALUs.
//
// Synthesis (Sec. 2.2, eq. synth_direct) and analysis (Sec. 2.3, eq. gauss)
// with P_n^m generated on the fly by the three-term recurrence of Sec. 3.2
// (eq. rec), the equatorial mirror symmetry of Sec. 3.1 folded in (one lane
// carries the pair of latitudes x and -x: even degrees n-m add, odd degrees
// subtract), and the underflow guard of Sec. 3.5 with the polar threshold of
// Sec. 3.1 resolved at plan time: every lane starts at the step where its
// |P_n^m| first matters, from a state stored by the plan, and a wave skips
// the steps in which none of its lanes has started.
//
// The recurrence runs in the rescaled form u_n = x u_{n-1} + beta_n u_{n-2}
// (two FP64 operations per step: one multiply by an SGPR coefficient and one
// FMA), with P_n^m = gamma_n u_n; gamma is folded into the spectrum before the
// synthesis and applied after the reduction in the analysis.  Recurrence
// coefficients and spectra are wave-uniform and are read with scalar loads
// into SGPRs, in blocks of several degrees, so every lane's FMAs take them as
// operands for free.  The tables are padded past their last entry so a block
// load at the end of an order stays in bounds.
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
    const long* f_off;  // per field: F offset in doubles (null: f * 2 f_size)
    const double* in;
    double* out;
    int nfields;
    int adjoint;
    int nunits;
    int wpg;  // waves (units) per workgroup
};

__device__ __forceinline__ long field_q_off(const LegArgs& a, int f, long nlm)
{
    return a.q_off ? ((clp)a.q_off)[f] : (long)f * 2 * nlm;
}

__device__ __forceinline__ long field_f_off(const LegArgs& a, int f, long fsize)
{
    return a.f_off ? ((clp)a.f_off)[f] : (long)f * 2 * fsize;
}

__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0; }

// Complex offset of F_m(theta_i) in a field's longitude coefficients (tiles
// of kFTile latitudes, see f_layout).
__device__ __forceinline__ long f_index(long ts, int m, int i)
{
    return (long)(i >> kFTileLg) * ts + m * kFTile + (i & (kFTile - 1));
}

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
    // two coefficients per thread, both loads issued before the stores
    const long i0 = (long)blockIdx.x * (2 * blockDim.x) + threadIdx.x;
    const long i1 = i0 + blockDim.x;
    const bool v0 = i0 < P.nlm, v1 = i1 < P.nlm;
    double g0 = 0.0, g1 = 0.0;
    double2 q0 = make_double2(0.0, 0.0), q1 = q0;
    if (v0) { g0 = P.gamma[i0]; q0 = *(const double2*)(Q + qo + 2 * i0); }
    if (v1) { g1 = P.gamma[i1]; q1 = *(const double2*)(Q + qo + 2 * i1); }
    if (v0) *(double2*)(Qs + so + 2 * i0) = make_double2(g0 * q0.x, g0 * q0.y);
    if (v1) *(double2*)(Qs + so + 2 * i1) = make_double2(g1 * q1.x, g1 * q1.y);
}

// Per-lane vector loads that warm L2 ahead of the scalar loads (synthesis).
constexpr int kPrefetchSlots = 2;

// Blocks of scalar operands.
struct D4 {
    double v[4];
};
struct D8 {
    double v[8];
};
struct D16 {
    double v[16];
};
typedef const __attribute__((address_space(4))) D4* cd4p;
typedef const __attribute__((address_space(4))) D8* cd8p;
typedef const __attribute__((address_space(4))) D16* cd16p;

// ---------------------------------------------------------------------------
// Lane starts (shared by both directions).
// ---------------------------------------------------------------------------
// Per lane and pair: the step at which the lane starts and the state
// (u_{j-2}, u_{j-1}) entering it; before that step the lane holds 0.
template <int LP>
struct Starts {
    int j[LP];
    double ya[LP], yb[LP];
};

template <int LP>
__device__ __forceinline__ void load_starts(Starts<LP>& st, cplan P, int m, int pb, int nj)
{
    const int lane = threadIdx.x & 63;
    const int npair = P->npair;
#pragma unroll
    for (int p = 0; p < LP; p++) {
        const int pair = pb + p * 64 + lane;
        const bool act = pair < npair;
        const size_t q = (size_t)m * npair + (act ? pair : 0);
        const double2 y = *(const double2*)(P->inj_y + 2 * q);
        st.j[p] = act ? P->inj_j[q] : nj;
        st.ya[p] = y.x;
        st.yb[p] = y.y;
    }
}

// Lanes whose start step is j take their stored state (a select per state).
template <int LP>
__device__ __forceinline__ void start_lanes(double (&ua)[LP], double (&ub)[LP], const Starts<LP>& st, int j)
{
#pragma unroll
    for (int p = 0; p < LP; p++) {
        const bool go = st.j[p] == j;
        ua[p] = go ? st.ya[p] : ua[p];
        ub[p] = go ? st.yb[p] : ub[p];
    }
}

template <int LP>
__device__ __forceinline__ void rescale(double (&ua)[LP], double (&ub)[LP], int sh)
{
#pragma unroll
    for (int p = 0; p < LP; p++) {
        ua[p] = __builtin_amdgcn_ldexp(ua[p], sh);
        ub[p] = __builtin_amdgcn_ldexp(ub[p], sh);
    }
}

// ---------------------------------------------------------------------------
// Synthesis: F_m(theta) for one order, LP pairs per lane, FW fields.
// ---------------------------------------------------------------------------
template <int LP, int FW>
struct SynthState {
    double x[LP], ua[LP], ub[LP];
    double er[LP][FW], ei[LP][FW], orr[LP][FW], oi[LP][FW];
};

// beta and the rescaled spectrum (re, im per field) for four degrees
template <int FW>
struct SBlock {
    D4 b;
    D8 q[FW];
};

template <int FW>
__device__ __forceinline__ void load_block(SBlock<FW>& B, cdp bet, const cdp (&qs)[FW], int j)
{
    cd4p pb = (cd4p)(bet + j);
#pragma unroll
    for (int i = 0; i < 4; i++) B.b.v[i] = pb->v[i];
#pragma unroll
    for (int f = 0; f < FW; f++) {
        cd8p pq = (cd8p)(qs[f] + 2 * j);
#pragma unroll
        for (int i = 0; i < 8; i++) B.q[f].v[i] = pq->v[i];
    }
}

// Step t of a block (degree offset j + t).  Even t advance ua and feed the
// even (E) sums, odd t advance ub and feed the odd (O) sums.
template <int LP, int FW>
__device__ __forceinline__ void synth_step(SynthState<LP, FW>& s, const SBlock<FW>& B, int t)
{
    const double b = B.b.v[t];
    if ((t & 1) == 0) {
#pragma unroll
        for (int p = 0; p < LP; p++) s.ua[p] = fma(s.x[p], s.ub[p], b * s.ua[p]);
#pragma unroll
        for (int p = 0; p < LP; p++) {
#pragma unroll
            for (int f = 0; f < FW; f++) {
                s.er[p][f] = fma(B.q[f].v[2 * t], s.ua[p], s.er[p][f]);
                s.ei[p][f] = fma(B.q[f].v[2 * t + 1], s.ua[p], s.ei[p][f]);
            }
        }
    } else {
#pragma unroll
        for (int p = 0; p < LP; p++) s.ub[p] = fma(s.x[p], s.ua[p], b * s.ub[p]);
#pragma unroll
        for (int p = 0; p < LP; p++) {
#pragma unroll
            for (int f = 0; f < FW; f++) {
                s.orr[p][f] = fma(B.q[f].v[2 * t], s.ub[p], s.orr[p][f]);
                s.oi[p][f] = fma(B.q[f].v[2 * t + 1], s.ub[p], s.oi[p][f]);
            }
        }
    }
}

// Four steps; `lim` = number of valid steps (4 for a full block).
template <int LP, int FW>
__device__ __forceinline__ void synth_block4(SynthState<LP, FW>& s, const SBlock<FW>& B, int lim)
{
#pragma unroll
    for (int t = 0; t < 4; t++)
        if (t < lim) synth_step(s, B, t);
}

// Eight steps from j (bounded by nj).
template <int LP, int FW>
__device__ __forceinline__ void synth_block8(SynthState<LP, FW>& s, cdp bet, const cdp (&qs)[FW], int j, int nj)
{
    SBlock<FW> b0, b1;
    load_block(b0, bet, qs, j);
    load_block(b1, bet, qs, j + 4);
    if (j + 8 <= nj) {
        synth_block4(s, b0, 4);
        synth_block4(s, b1, 4);
    } else {
        synth_block4(s, b0, nj - j);
        if (j + 4 < nj) synth_block4(s, b1, nj - j - 4);
    }
}

// One wave per unit; a workgroup holds `wpg` consecutive units: the latitude
// blocks of one order (they share scalar-cache lines), or of the orders m and
// M-m together so that every workgroup carries the same work.
template <int LP, int FW>
constexpr int synth_max_threads() { return LP == 1 && FW == 1 ? 1024 : 512; }

template <int LP, int FW>
__global__ void __launch_bounds__((synth_max_threads<LP, FW>())) k_legendre_synth(LegArgs a)
{
    // wave-uniform for the compiler, so unit data and coefficients stay in SGPRs
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int unit = blockIdx.x * a.wpg + wave;
    if (unit >= a.nunits) return;
    cip U = (cip)a.units + (size_t)unit * kUnitInts;
    const int m = U[U_M];
    if (m < 0) return;
    const int field0 = U[U_FIELD] + blockIdx.y * FW;
    if (field0 >= a.nfields) return;
    const int nf = min(U[U_NF], a.nfields - field0);
    cplan P = (cplan)a.plans + U[U_PLAN];
    const int L = P->L, nlat = P->nlat, npair = P->npair;
    const long fts = P->f_ts;
    const long nlm = P->nlm;
    const int pb = U[U_PB];
    long qoff[FW];
    long foff[FW];
#pragma unroll
    for (int f = 0; f < FW; f++) {
        const int ff = field0 + min(f, nf - 1);
        qoff[f] = field_q_off(a, ff, nlm);
        foff[f] = field_f_off(a, ff, P->f_size);
    }

    if (U[U_ZERO]) {
        // no latitude of the block reaches the polar threshold: F_m = 0 there
#pragma unroll
        for (int p = 0; p < LP; p++) {
            const int pair = pb + p * 64 + lane;
            if (pair >= npair) continue;
            const int is = nlat - 1 - pair;
#pragma unroll
            for (int f = 0; f < FW; f++) {
                if (f >= nf) continue;
                double* F = a.out + foff[f];
                *(double2*)(F + 2 * f_index(fts, m, pair)) = make_double2(0.0, 0.0);
                *(double2*)(F + 2 * f_index(fts, m, is)) = make_double2(0.0, 0.0);
            }
        }
        return;
    }
    const int jstart = U[U_JS], jwin = U[U_JW];
    const long base = (long)m * (2 * L + 1 - m) / 2 + m;
    const int nj = L - m + 1;
    cdp bet = (cdp)P->beta + base;
    cdp qs[FW];
#pragma unroll
    for (int f = 0; f < FW; f++) qs[f] = (cdp)(a.in + qoff[f]) + 2 * base;
    cip segexp = (cip)P->segexp + ((cip)P->segoff)[m];

    SynthState<LP, FW> s;
    Starts<LP> st;
    load_starts(st, P, m, pb, nj);
#pragma unroll
    for (int p = 0; p < LP; p++) {
        const int pair = pb + p * 64 + lane;
        const bool act = pair < npair;
        s.x[p] = act ? P->xp[act ? pair : 0] : 0.0;
        s.ua[p] = 0.0;
        s.ub[p] = 0.0;
#pragma unroll
        for (int f = 0; f < FW; f++) s.er[p][f] = s.ei[p][f] = s.orr[p][f] = s.oi[p][f] = 0.0;
    }

    // Warm L2 with this order's beta and spectrum from the first step on: the
    // waves of the order's latitude blocks touch one word per 64-byte line
    // with vector loads into registers that are consumed only after the order
    // is done.  They are issued after the start values above have arrived and
    // no other vector load follows before the end, so no wave waits on them
    // (the scalar loads are counted apart).  The scalar loads then find these
    // lines in L2.
    __builtin_amdgcn_sched_barrier(0);
    unsigned pf[kPrefetchSlots];
    {
        const int nblk_m = (npair + 64 * LP - 1) / (64 * LP);
        const int nthr = nblk_m * 64;
        const int gi = (pb / (64 * LP)) * 64 + lane;
        const int nrem = nj - jstart;
        const int lb = (nrem * 8 + 63) / 64;   // beta lines
        const int lq = (nrem * 16 + 63) / 64;  // spectrum lines per field
        const char* b0 = (const char*)(P->beta + base + jstart);
#pragma unroll
        for (int k = 0; k < kPrefetchSlots; k++) {
            int li = gi + k * nthr;
            const char* addr = b0;
            if (li < lb) {
                addr = b0 + li * 64;
            } else {
                li -= lb;
#pragma unroll
                for (int f = 0; f < FW; f++) {
                    if (li >= 0 && li < lq) addr = (const char*)(a.in + qoff[f] + 2 * (base + jstart)) + li * 64;
                    li -= lq;
                }
            }
            pf[k] = *(const unsigned*)addr;
        }
    }

    // Start window: blocks of kInject steps from the first start, lanes
    // joining at block boundaries, up to the segment boundary after the last
    // start.  (The shift is 0 off segment boundaries: an unconditional
    // ldexp, not a branch, which the compiler would turn into selects.)
    static_assert(kInject == 8, "the start window advances in blocks of 8 steps");
    int j = jstart;
    while (j < nj && (j <= jwin || j % kSegLen != 0)) {
        rescale(s.ua, s.ub, (j > jstart && j % kSegLen == 0) ? segexp[j / kSegLen] : 0);
        start_lanes(s.ua, s.ub, st, j);
        synth_block8(s, bet, qs, j, nj);
        j += 8;
    }
    // Every lane has started: whole segments, straight-line.
    for (int js = j; js < nj; js += kSegLen) {
        const int je = min(js + kSegLen, nj);
        rescale(s.ua, s.ub, segexp[js / kSegLen]);
        if (je - js == kSegLen) {
#pragma unroll
            for (int bk = 0; bk < kSegLen; bk += 8) {
                SBlock<FW> b0, b1;
                load_block(b0, bet, qs, js + bk);
                load_block(b1, bet, qs, js + bk + 4);
                synth_block4(s, b0, 4);
                synth_block4(s, b1, 4);
            }
        } else {
            // last, partial segment of the order
            for (int jj = js; jj < je; jj += 8) synth_block8(s, bet, qs, jj, nj);
        }
    }

    unsigned sink = 0;
#pragma unroll
    for (int k = 0; k < kPrefetchSlots; k++) sink ^= pf[k];

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
            double* F = a.out + foff[f];
            *(double2*)(F + 2 * f_index(fts, m, pair)) =
                make_double2(sc * (s.er[p][f] + s.orr[p][f]), sc * (s.ei[p][f] + s.oi[p][f]));
            if (is != pair)
                *(double2*)(F + 2 * f_index(fts, m, is)) = make_double2(sc * (s.er[p][f] - s.orr[p][f]),
                                                                        sc * (s.ei[p][f] - s.oi[p][f]));
        }
    }
    // keeps the prefetch loads alive; nfields is never negative
    if (a.nfields < 0) a.out[lane] = (double)sink;
}

// ---------------------------------------------------------------------------
// Analysis: Q_n^m = gamma_n sum_pairs u_n (w (F_N +- F_S)), one wave covers all
// latitude pairs of one order (64 LP >= npair) for a range of degrees.
// ---------------------------------------------------------------------------
template <int LP, int FW>
struct AState {
    double x[LP], ua[LP], ub[LP];
    // folded, weighted inputs w (F_N + F_S), w (F_N - F_S)
    double ger[LP][FW], gei[LP][FW], gor[LP][FW], goi[LP][FW];
};

// Loads the folded inputs of every lane.  A lane that has not started holds a
// zero state, so it adds exactly 0 whatever its inputs.
template <int LP, int FW>
__device__ __forceinline__ void analys_inputs(AState<LP, FW>& s, const double* const (&F)[FW], int nlat,
                                              long fts, int m, int pb, int npair, int adjoint,
                                              const double* wq)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int p = 0; p < LP; p++) {
        const int pair = pb + p * 64 + lane;
        const bool act = pair < npair;
        const int pc = act ? pair : 0;
        const bool middle = (nlat & 1) && pc == npair - 1;
        const double wt = !act ? 0.0 : (adjoint ? (middle ? 0.5 : 1.0) : wq[pc]);
#pragma unroll
        for (int f = 0; f < FW; f++) {
            const double2 vn = *(const double2*)(F[f] + 2 * f_index(fts, m, pc));
            const double2 vs = *(const double2*)(F[f] + 2 * f_index(fts, m, nlat - 1 - pc));
            s.ger[p][f] = wt * (vn.x + vs.x);
            s.gei[p][f] = wt * (vn.y + vs.y);
            s.gor[p][f] = wt * (vn.x - vs.x);
            s.goi[p][f] = wt * (vn.y - vs.y);
        }
    }
}

// One recurrence step (even t: ua and the even inputs, odd t: ub and the odd
// inputs); returns this lane's partial sum over its pairs, per field.
template <int LP, int FW>
__device__ __forceinline__ void analys_step(AState<LP, FW>& s, int t, double b,
                                            double (&sr)[FW], double (&si)[FW])
{
#pragma unroll
    for (int f = 0; f < FW; f++) sr[f] = si[f] = 0.0;
    if ((t & 1) == 0) {
#pragma unroll
        for (int p = 0; p < LP; p++) {
            s.ua[p] = fma(s.x[p], s.ub[p], b * s.ua[p]);
#pragma unroll
            for (int f = 0; f < FW; f++) {
                sr[f] = fma(s.ger[p][f], s.ua[p], sr[f]);
                si[f] = fma(s.gei[p][f], s.ua[p], si[f]);
            }
        }
    } else {
#pragma unroll
        for (int p = 0; p < LP; p++) {
            s.ub[p] = fma(s.x[p], s.ua[p], b * s.ub[p]);
#pragma unroll
            for (int f = 0; f < FW; f++) {
                sr[f] = fma(s.gor[p][f], s.ub[p], sr[f]);
                si[f] = fma(s.goi[p][f], s.ub[p], si[f]);
            }
        }
    }
}

// Each lane's partial sums go straight to LDS, one row per (degree, field,
// re/im) with a column per thread of the workgroup; every 16/FW degrees one
// pass sums the 32 rows (2W threads per row, padded rows).  No accumulators
// stay in registers.  A workgroup of W waves covers 64 LP W latitude pairs:
// wave w takes pairs [64 LP w, 64 LP (w + 1)); a wave none of whose
// latitudes has started writes zero rows instead of computing.
template <int LP, int FW, int W>
__global__ void __launch_bounds__(64 * W) k_legendre_analys(LegArgs a)
{
    constexpr int C = kChunk;       // degrees per beta block load
    constexpr int SC = kChunk / FW; // degrees per reduction
    constexpr int NV = 2 * SC * FW; // rows reduced per pass
    constexpr int NT = 64 * W;      // threads = columns
    constexpr int PR = 2 * W;       // threads per row
    static_assert(NV * PR == NT, "the threads cover the rows");
    static_assert(kSegLen % C == 0, "chunks tile a segment");
    static_assert(SC % kInject == 0, "lanes start at reduction-block boundaries or inside them");
    __shared__ double red[NV][NT + 1];

    cip U = (cip)a.units + (size_t)blockIdx.x * kUnitInts;
    const int m = U[U_M];
    if (m < 0) return;
    const int field0 = U[U_FIELD] + blockIdx.y * FW;
    if (field0 >= a.nfields) return;
    const int nf = min(U[U_NF], a.nfields - field0);
    cplan P = (cplan)a.plans + U[U_PLAN];
    const int L = P->L, nlat = P->nlat, npair = P->npair;
    const long fts = P->f_ts;
    const long nlm = P->nlm;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int pb = wv * 64 * LP;  // first latitude pair of this wave
    const int j0 = U[U_PB], j1 = U[U_J1], js0 = U[U_JS], jwin = U[U_JW], rst = U[U_RST];
    const long base = (long)m * (2 * L + 1 - m) / 2 + m;
    const int nj = L - m + 1;
    cdp bet = (cdp)P->beta + base;
    cip segexp = (cip)P->segexp + ((cip)P->segoff)[m];

    long qoff[FW];
    long foff[FW];
#pragma unroll
    for (int f = 0; f < FW; f++) {
        const int ff = field0 + min(f, nf - 1);
        qoff[f] = field_q_off(a, ff, nlm);
        foff[f] = field_f_off(a, ff, P->f_size);
    }

    // degrees before the first started lane: every term is dropped
    for (int j = j0 + (tid >> 1); j < js0; j += NT / 2) {
#pragma unroll
        for (int f = 0; f < FW; f++)
            if (f < nf) a.out[qoff[f] + 2 * (base + j) + (tid & 1)] = 0.0;
    }
    if (js0 >= j1) return;

    AState<LP, FW> s;
    Starts<LP> st;
    load_starts(st, P, m, pb, nj);
    const bool from_rst = rst >= 0 && js0 == j0;
    int first = nj;  // first step at which a lane of this wave is live
#pragma unroll
    for (int p = 0; p < LP; p++) {
        const int pair = pb + p * 64 + lane;
        const bool act = pair < npair;
        const int pc = act ? pair : 0;
        s.x[p] = act ? P->xp[pc] : 0.0;
        s.ua[p] = 0.0;
        s.ub[p] = 0.0;
        if (from_rst) {
            const double2 r = *(const double2*)(P->rst_y + 2 * ((size_t)rst * npair + pc));
            s.ua[p] = act ? r.x : 0.0;
            s.ub[p] = act ? r.y : 0.0;
        }
        const bool live0 = from_rst && st.j[p] < j0;
        first = min(first, live0 ? js0 : st.j[p]);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) first = min(first, __shfl_xor(first, o));
    first = __builtin_amdgcn_readfirstlane(first);
    {
        const double* F[FW];
#pragma unroll
        for (int f = 0; f < FW; f++) F[f] = a.in + foff[f];
        analys_inputs(s, F, nlat, fts, m, pb, npair, a.adjoint, P->wq);
    }

    // Warm L2 with the beta entries of this unit (one word per 64-byte line
    // per lane, consumed at the end; see the synthesis kernel).
    __builtin_amdgcn_sched_barrier(0);
    unsigned pf;
    {
        const int nbytes = (j1 - js0 + C) * 8;
        const int off = lane * 64;
        pf = *(const unsigned*)((const char*)(P->beta + base + js0) + (off < nbytes ? off : 0));
    }
    const double cm = (m == 0 || !a.adjoint) ? 1.0 : 2.0;
    const int v = tid / PR;   // reduction row of this thread
    const int h = tid % PR;   // its part of the row
    const int comp = v & 1;
    const int t_out = (v >> 1) / FW;
    const int f_out = (v >> 1) % FW;
    const int col = wv * 64 + lane;  // this thread's column

    // js0 is a segment start (the plan rounds it down)
    for (int js = js0; js < j1; js += kSegLen) {
        rescale(s.ua, s.ub, js > js0 ? segexp[js / kSegLen] : 0);
        const int je = min(js + kSegLen, j1);
        for (int c = js; c < je; c += C) {
            // beta for the chunk in one block load (the table is padded).  A
            // partial last chunk runs all C steps: the extra degrees belong to
            // no output (their results are not written) and the unit ends here.
            D16 b;
            cd16p pbk = (cd16p)(bet + c);
#pragma unroll
            for (int i = 0; i < C; i++) b.v[i] = pbk->v[i];
            const bool window = c <= jwin;
            const bool idle = c + C <= first;  // wave-uniform: no lane live in the chunk
#pragma unroll
            for (int c0 = 0; c0 < C; c0 += SC) {
                // this thread's output scale, loaded ahead of the steps
                // (clamped index: rows past the unit's end write nothing)
                const int j_out = c + c0 + t_out;
                const double gam = P->gamma[base + min(j_out, je - 1)] * cm;
                if (idle) {
#pragma unroll
                    for (int t = 0; t < NV; t++) red[t][col] = 0.0;
                } else if (window) {
#pragma unroll
                    for (int t = 0; t < SC; t++) {
                        if ((c0 + t) % kInject == 0) start_lanes(s.ua, s.ub, st, c + c0 + t);
                        double sr[FW], si[FW];
                        analys_step(s, c0 + t, b.v[c0 + t], sr, si);
#pragma unroll
                        for (int f = 0; f < FW; f++) {
                            red[2 * (t * FW + f)][col] = sr[f];
                            red[2 * (t * FW + f) + 1][col] = si[f];
                        }
                    }
                } else {
#pragma unroll
                    for (int t = 0; t < SC; t++) {
                        double sr[FW], si[FW];
                        analys_step(s, c0 + t, b.v[c0 + t], sr, si);
#pragma unroll
                        for (int f = 0; f < FW; f++) {
                            red[2 * (t * FW + f)][col] = sr[f];
                            red[2 * (t * FW + f) + 1][col] = si[f];
                        }
                    }
                }
                // row v summed over the NT columns by PR threads (columns
                // r PR + h), four independent partial sums each
                __syncthreads();
                double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
                for (int r = 0; r < 32; r += 4) {
                    s0 += red[v][(r + 0) * PR + h];
                    s1 += red[v][(r + 1) * PR + h];
                    s2 += red[v][(r + 2) * PR + h];
                    s3 += red[v][(r + 3) * PR + h];
                }
                double sum = (s0 + s1) + (s2 + s3);
#pragma unroll
                for (int o = 1; o < PR; o <<= 1) sum += __shfl_xor(sum, o);
                __syncthreads();
                if (h == 0 && j_out < je && f_out < nf) {
                    const long idx = base + j_out;
                    double val = gam * sum;
                    if (m == 0 && comp == 1) val = 0.0;
                    a.out[qoff[f_out] + 2 * idx + comp] = val;
                }
            }
        }
    }
    // keeps the prefetch load alive; nfields is never negative
    if (a.nfields < 0) a.out[lane] = (double)pf;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int launch_prescale(const DevPlan* plans, const long* q_off, const long* s_off, const int* fplan,
                    const double* Q, double* Qs, long max_nlm, int nfields, void* stream)
{
    const int blocks = (int)((max_nlm + 511) / 512);
    dim3 grid(std::max(1, blocks), nfields);
    hipLaunchKernelGGL(k_prescale, grid, dim3(256), 0, (hipStream_t)stream, plans, q_off, s_off,
                       fplan, Q, Qs, nfields);
    return (int)hipGetLastError();
}

template <int LP, int FW>
static int launch_synth_t(const LegLaunch& l, void* stream)
{
    const int wpg = std::max(1, std::min(l.wpg, synth_max_threads<LP, FW>() / 64));
    LegArgs a{l.plans, l.units, l.q_off, l.f_off, l.in, l.out, l.nfields, l.adjoint, l.nunits, wpg};
    hipLaunchKernelGGL((k_legendre_synth<LP, FW>), dim3((l.nunits + wpg - 1) / wpg, l.grid_y),
                       dim3(64 * wpg), 0, (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

template <int LP, int FW, int W>
static int launch_analys_t(const LegLaunch& l, void* stream)
{
    LegArgs a{l.plans, l.units, l.q_off, l.f_off, l.in, l.out, l.nfields, l.adjoint, l.nunits, 1};
    hipLaunchKernelGGL((k_legendre_analys<LP, FW, W>), dim3(l.nunits, l.grid_y), dim3(64 * W), 0,
                       (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

int launch_legendre_synth(const LegLaunch& l, void* stream)
{
    if (l.nunits <= 0) return 0;
#define SHTN_S(LPV, FWV) \
    if (l.lp == LPV && l.fw == FWV) return launch_synth_t<LPV, FWV>(l, stream);
    SHTN_S(1, 1) SHTN_S(2, 1) SHTN_S(4, 1)
    SHTN_S(1, 2) SHTN_S(2, 2) SHTN_S(4, 2)
#undef SHTN_S
    return (int)hipErrorInvalidValue;
}

int launch_legendre_analys(const LegLaunch& l, void* stream)
{
    if (l.nunits <= 0) return 0;
#define SHTN_A(LPV, FWV, WV) \
    if (l.lp == LPV && l.fw == FWV && l.waves == WV) return launch_analys_t<LPV, FWV, WV>(l, stream);
    SHTN_A(1, 1, 1) SHTN_A(2, 1, 1) SHTN_A(4, 1, 1) SHTN_A(8, 1, 1)
    SHTN_A(1, 2, 1) SHTN_A(2, 2, 1) SHTN_A(4, 2, 1)
    SHTN_A(2, 1, 2) SHTN_A(4, 1, 2) SHTN_A(8, 1, 2)
    SHTN_A(2, 2, 2) SHTN_A(4, 2, 2)
    SHTN_A(4, 1, 4) SHTN_A(8, 1, 4)
#undef SHTN_A
    return (int)hipErrorInvalidValue;
}

}  // namespace shtn
