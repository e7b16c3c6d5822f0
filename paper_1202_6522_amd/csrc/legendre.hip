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
template <int N>
struct DN {
    double v[N];
};

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

// Analysis: the start steps stay in registers and the stored states in this
// lane's slots in LDS (read back only at the checkpoints of the start
// window, so they hold no registers through the degree loop).
template <int LP>
__device__ __forceinline__ void start_lanes_lds(double (&ua)[LP], double (&ub)[LP], const int (&sj)[LP],
                                                const double2 (*sy)[64], int j)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int p = 0; p < LP; p++) {
        const double2 y = sy[p][lane];
        const bool go = sj[p] == j;
        ua[p] = go ? y.x : ua[p];
        ub[p] = go ? y.y : ub[p];
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

// Degrees per block of scalar operands: four, two with four fields, so that
// a block (beta and the spectra of all fields) fits the scalar registers.
// Blocks start at even offsets and hold an even number of steps, so a step's
// parity within its block is the parity of its degree offset.
template <int FW>
constexpr int block_steps() { return FW >= 4 ? 2 : 4; }

// beta and the rescaled spectrum (re, im per field) for NS = block_steps degrees
template <int FW>
struct SBlock {
    static constexpr int NS = block_steps<FW>();
    static_assert(NS % 2 == 0, "blocks keep the step parity");
    DN<NS> b;
    DN<2 * NS> q[FW];
};

template <int FW>
__device__ __forceinline__ void load_block(SBlock<FW>& B, cdp bet, const cdp (&qs)[FW], int j)
{
    constexpr int NS = SBlock<FW>::NS;
    typedef const __attribute__((address_space(4))) DN<NS>* cbp;
    typedef const __attribute__((address_space(4))) DN<2 * NS>* cqp;
    cbp pb = (cbp)(bet + j);
#pragma unroll
    for (int i = 0; i < NS; i++) B.b.v[i] = pb->v[i];
#pragma unroll
    for (int f = 0; f < FW; f++) {
        cqp pq = (cqp)(qs[f] + 2 * j);
#pragma unroll
        for (int i = 0; i < 2 * NS; i++) B.q[f].v[i] = pq->v[i];
    }
}

// Step t of a block (degree offset j + t, j even).  Even t advance ua and
// feed the even (E) sums, odd t advance ub and feed the odd (O) sums.
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

// The steps of one block; `lim` = number of valid steps.
template <int LP, int FW>
__device__ __forceinline__ void synth_block(SynthState<LP, FW>& s, const SBlock<FW>& B, int lim)
{
#pragma unroll
    for (int t = 0; t < SBlock<FW>::NS; t++)
        if (t < lim) synth_step(s, B, t);
}

// Eight steps from j (bounded by nj; the operand tables are padded, so the
// loads stay in bounds past nj).  One field: both 4-step blocks are loaded
// before either is used; with several fields two blocks would not fit the
// scalar registers, so each block is loaded where it is used.
template <int LP, int FW>
__device__ __forceinline__ void synth_block8(SynthState<LP, FW>& s, cdp bet, const cdp (&qs)[FW], int j, int nj)
{
    constexpr int NS = SBlock<FW>::NS;
    if (FW == 1) {
        SBlock<FW> b0, b1;
        load_block(b0, bet, qs, j);
        load_block(b1, bet, qs, j + NS);
        if (j + 2 * NS <= nj) {
            synth_block(s, b0, NS);
            synth_block(s, b1, NS);
        } else {
            synth_block(s, b0, nj - j);
            if (j + NS < nj) synth_block(s, b1, nj - j - NS);
        }
        return;
    }
#pragma unroll
    for (int k = 0; k < 8; k += NS) {
        if (j + k >= nj) break;
        SBlock<FW> b0;
        load_block(b0, bet, qs, j + k);
        synth_block(s, b0, nj - j - k);
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
    // Every lane has started: whole segments, straight-line.  One field: the
    // scalar operands of each 4-step block are loaded one block ahead; with
    // several fields each block is loaded where it is used.
    SBlock<FW> cur;
    if (FW == 1) load_block(cur, bet, qs, j);
    int shn = j < nj ? segexp[j / kSegLen] : 0;
    for (int js = j; js < nj; js += kSegLen) {
        const int je = min(js + kSegLen, nj);
        rescale(s.ua, s.ub, shn);
        shn = js + kSegLen < nj ? segexp[js / kSegLen + 1] : 0;
        if (je - js == kSegLen) {
            constexpr int NS = SBlock<FW>::NS;
            // operands of the segment from one base pointer per table, so
            // that the block loads take fixed offsets
            const cdp bseg = bet + js;
            cdp qseg[FW];
#pragma unroll
            for (int f = 0; f < FW; f++) qseg[f] = qs[f] + 2 * js;
#pragma unroll
            for (int bk = 0; bk < kSegLen; bk += NS) {
                if (FW == 1) {
                    SBlock<FW> nxt;
                    load_block(nxt, bseg, qseg, bk + NS);
                    synth_block(s, cur, NS);
                    cur = nxt;
                } else {
                    SBlock<FW> b0;
                    load_block(b0, bseg, qseg, bk);
                    synth_block(s, b0, NS);
                }
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
    // folded, weighted inputs: even-degree (w (F_N + F_S)) and odd-degree
    // (w (F_N - F_S)) parts, the component this lane keeps (k) and the one it
    // hands to its neighbour lane (s): even lanes keep the real part, odd
    // lanes the imaginary part
    double ek[LP][FW], es[LP][FW], ok[LP][FW], os[LP][FW];
};

// v of the neighbouring lane (lanes 2i and 2i+1 swap; DPP quad_perm [1,0,3,2]).
__device__ __forceinline__ double swap_lane_pair(double v)
{
    const long long b = __double_as_longlong(v);
    // every lane is active here, so the "old" operand is never used; passing
    // the source itself saves the moves that would initialise it
    const int lo = __builtin_amdgcn_update_dpp((int)b, (int)b, 0xB1, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(b >> 32), (int)(b >> 32), 0xB1, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Two recurrence steps, an even one (ua and the even inputs) and the odd one
// after it (ub and the odd inputs), on the pair slots PF..LP-1; the slots
// below PF belong to latitude blocks none of whose lanes has started, hold 0
// and would add exactly 0.  Both steps advance the recurrence first, then
// their four sums (kept and handed-over component of each step) are
// accumulated side by side over the slots, so four independent chains of
// fused multiply-adds share the latency.  Returns per field and step the
// lane pair's partial sum over its pairs of the kept component: real part on
// even lanes, imaginary part on odd lanes.
template <int LP, int FW, int PF>
__device__ __forceinline__ void analys_step_pair(AState<LP, FW>& s, double b0, double b1, double (&out0)[FW],
                                                 double (&out1)[FW])
{
#pragma unroll
    for (int p = PF; p < LP; p++) s.ua[p] = fma(s.x[p], s.ub[p], b0 * s.ua[p]);
#pragma unroll
    for (int p = PF; p < LP; p++) s.ub[p] = fma(s.x[p], s.ua[p], b1 * s.ub[p]);
    double sk0[FW], ss0[FW], sk1[FW], ss1[FW];
#pragma unroll
    for (int f = 0; f < FW; f++) sk0[f] = ss0[f] = sk1[f] = ss1[f] = 0.0;
#pragma unroll
    for (int p = PF; p < LP; p++) {
#pragma unroll
        for (int f = 0; f < FW; f++) {
            sk0[f] = fma(s.ek[p][f], s.ua[p], sk0[f]);
            ss0[f] = fma(s.es[p][f], s.ua[p], ss0[f]);
            sk1[f] = fma(s.ok[p][f], s.ub[p], sk1[f]);
            ss1[f] = fma(s.os[p][f], s.ub[p], ss1[f]);
        }
    }
#pragma unroll
    for (int f = 0; f < FW; f++) {
        out0[f] = sk0[f] + swap_lane_pair(ss0[f]);
        out1[f] = sk1[f] + swap_lane_pair(ss1[f]);
    }
}

template <int N>
struct DBlk {
    double v[N];
};

template <int N>
struct DBlk2u {
    unsigned v[N];
};

// A block of N wave-uniform 32-bit words through the scalar cache.
template <int N>
__device__ __forceinline__ void load_u32(DBlk2u<N>& d, cip src)
{
    typedef const __attribute__((address_space(4))) DBlk2u<N>* cbp;
    cbp p = (cbp)src;
#pragma unroll
    for (int i = 0; i < N; i++) d.v[i] = p->v[i];
}

// A block of N wave-uniform doubles through the scalar cache.
template <int N>
__device__ __forceinline__ void load_blk(DBlk<N>& d, cdp src)
{
    typedef const __attribute__((address_space(4))) DBlk<N>* cbp;
    cbp p = (cbp)src;
#pragma unroll
    for (int i = 0; i < N; i++) d.v[i] = p->v[i];
}

// kInject steps (one start checkpoint to the next) on slots PF..LP-1, the
// rows of steps t0 .. t0 + kInject - 1 of the pass written to LDS (PF = LP:
// no slot live, zero rows).  t0 is even, so a step's parity is that of t.
template <int LP, int FW, int PF, int RS>
__device__ __forceinline__ void analys_half(AState<LP, FW>& s, const double (&b)[kInject], double* rows, int t0)
{
#pragma unroll
    for (int t = 0; t < kInject; t += 2) {
        double v0[FW], v1[FW];
        if (PF < LP) {
            analys_step_pair<LP, FW, PF>(s, b[t], b[t + 1], v0, v1);
        } else {
#pragma unroll
            for (int f = 0; f < FW; f++) v0[f] = v1[f] = 0.0;
        }
#pragma unroll
        for (int f = 0; f < FW; f++) {
            rows[((t0 + t) * FW + f) * RS] = v0[f];
            rows[((t0 + t + 1) * FW + f) * RS] = v1[f];
        }
    }
}

// The half for the first live slot pf (wave-uniform).
template <int LP, int FW, int RS>
__device__ __forceinline__ void analys_half_from(int pf, AState<LP, FW>& s, const double (&b)[kInject],
                                                 double* rows, int t0)
{
    // (pf <= LP; a case k >= LP is the no-live-slot variant: zero rows)
    switch (pf) {
    case 0: analys_half<LP, FW, 0, RS>(s, b, rows, t0); break;
    case 1: analys_half<LP, FW, (1 < LP ? 1 : LP), RS>(s, b, rows, t0); break;
    case 2: analys_half<LP, FW, (2 < LP ? 2 : LP), RS>(s, b, rows, t0); break;
    case 3: analys_half<LP, FW, (3 < LP ? 3 : LP), RS>(s, b, rows, t0); break;
    case 4: analys_half<LP, FW, (4 < LP ? 4 : LP), RS>(s, b, rows, t0); break;
    case 5: analys_half<LP, FW, (5 < LP ? 5 : LP), RS>(s, b, rows, t0); break;
    case 6: analys_half<LP, FW, (6 < LP ? 6 : LP), RS>(s, b, rows, t0); break;
    case 7: analys_half<LP, FW, (7 < LP ? 7 : LP), RS>(s, b, rows, t0); break;
    default: analys_half<LP, FW, LP, RS>(s, b, rows, t0); break;
    }
}

// Start checkpoint cc: in the slots whose block has a lane starting there
// (bits of mk, wave-uniform), the lanes whose start step is cc take their
// stored state (kept in this lane's slots in LDS).
template <int LP>
__device__ __forceinline__ void start_slots(double (&ua)[LP], double (&ub)[LP], const int (&sj)[LP],
                                            const double2 (*sy)[64], unsigned mk, int cc)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int p = 0; p < LP; p++) {
        if (mk & (1u << p)) {
            const double2 y = sy[p][lane];
            const bool go = sj[p] == cc;
            ua[p] = go ? y.x : ua[p];
            ub[p] = go ? y.y : ub[p];
        }
    }
}

// The degrees of a unit run in passes of SC = kChunk / FW degrees.  In a pass
// each lane pair's partial sums (one row per degree and field, one column
// per thread: real parts in even columns, imaginary parts in odd ones) go to
// LDS, while the sums of the previous pass are read back, added over the
// columns (2W threads per output, padded rows) and stored.  The rows live in
// one buffer: one wave executes its LDS operations in order, so with W = 1
// the reads of the previous pass, issued before this pass's writes, need no
// barrier; with several waves a barrier after the reads lets every wave
// finish reading before any wave writes, and one at the end of the pass
// makes the rows visible.  (Two alternating buffers would save the first
// barrier, but at W = 2 and 4 their LDS halves the workgroups a CU holds:
// lmax 2047 and 4095 ran 14% and 33% slower that way.)
// A workgroup of W waves covers 64 LP W latitude pairs: wave w takes pairs
// [64 LP w, 64 LP (w + 1)), pair slot p of its lanes being the 64-pair block
// LP w + p.  A pass runs as halves of kInject steps; each half first injects
// the start states of the blocks with lanes starting at its checkpoint, then
// runs only the slots from the first one whose block has started (the polar
// optimisation of Sec. 3.1 at the granularity of 64 latitudes).
template <int LP, int FW, int W>
struct AnalysGeom {
    static constexpr int SC = kChunk / FW;  // degrees per pass
    static constexpr int NR = SC * FW;      // rows per pass
    static constexpr int NT = 64 * W;       // threads = columns
    static constexpr int PR = 2 * W;        // threads per output (row, component)
    static constexpr int NK = NT / 2 / PR;  // columns each of them adds
    // row stride NT + 2 PR doubles: a thread's PR-wide column groups of
    // consecutive rows start 4 PR banks apart, so the 32 lanes of a half-wave
    // read distinct banks
    static constexpr int RS = NT + 2 * PR;
    static constexpr int NH = SC / kInject;  // halves per pass
};

// One unit: degrees [j0, j1) of one order for all latitude pairs (the
// workgroup's W waves), the outputs stored; uniform over the workgroup.
template <int LP, int FW, int W>
__device__ __forceinline__ void analys_unit(
    const LegArgs& a, int ui,
    double (&red)[AnalysGeom<LP, FW, W>::NR][AnalysGeom<LP, FW, W>::RS],
    double2 (&start_y)[W][LP][64])
{
    using G = AnalysGeom<LP, FW, W>;
    constexpr int SC = G::SC, NR = G::NR, NT = G::NT, PR = G::PR, NK = G::NK, RS = G::RS, NH = G::NH;
    static_assert(2 * NR * PR == NT, "the threads cover the outputs");
    static_assert(kSegLen % SC == 0, "passes tile a segment");
    static_assert(SC % kInject == 0, "passes are whole halves");
    static_assert(kInject % 2 == 0, "halves keep the step parity");
    static_assert(LP <= 8 && LP * W <= kMaxMaskBlocks, "one mask word covers the unit's blocks");

    cip U = (cip)a.units + (size_t)ui * kUnitInts;
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
    const int wb = wv * LP;       // its first 64-pair block
    const int j0 = U[U_PB], j1 = U[U_J1], js0 = U[U_JS], jwin = U[U_JW], rst = U[U_RST];
    const long base = (long)m * (2 * L + 1 - m) / 2 + m;
    const int nj = L - m + 1;
    cdp bet = (cdp)P->beta + base;
    cip segexp = (cip)P->segexp + ((cip)P->segoff)[m];
    // per checkpoint: blocks with lanes starting there, blocks started
    cip ckm = (cip)P->ck_mask + (size_t)m * P->nck * 2;

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

    // Unit setup.  Every global load is issued before any of them is used
    // (indices clamped to valid entries, inactive lanes masked afterwards),
    // so the setup costs one memory round trip.
    AState<LP, FW> s;
    int sj[LP];
    const bool from_rst = rst >= 0 && js0 == j0;
    // no lane starts inside the unit (window -1): its start states are not
    // needed, all lanes come live from the restart state
    const bool starts = jwin >= js0;
    {
        const bool odd = lane & 1;
        int pc[LP], jv[LP];
        bool act[LP];
        double xv[LP], wl[LP];
        double2 y[LP], r[LP], fn[LP][FW], fsth[LP][FW];
#pragma unroll
        for (int p = 0; p < LP; p++) {
            const int pair = pb + p * 64 + lane;
            act[p] = pair < npair;
            pc[p] = act[p] ? pair : 0;
            const size_t q = (size_t)m * npair + pc[p];
            xv[p] = P->xp[pc[p]];
            wl[p] = P->wq[pc[p]];
            if (starts) {
                y[p] = *(const double2*)(P->inj_y + 2 * q);
                jv[p] = P->inj_j[q];
            } else {
                y[p] = make_double2(0.0, 0.0);
                jv[p] = nj;
            }
#pragma unroll
            for (int f = 0; f < FW; f++) {
                const double* F = a.in + foff[f];
                fn[p][f] = *(const double2*)(F + 2 * f_index(fts, m, pc[p]));
                fsth[p][f] = *(const double2*)(F + 2 * f_index(fts, m, nlat - 1 - pc[p]));
            }
        }
        if (from_rst) {
#pragma unroll
            for (int p = 0; p < LP; p++)
                r[p] = *(const double2*)(P->rst_y + 2 * ((size_t)rst * npair + pc[p]));
        } else {
#pragma unroll
            for (int p = 0; p < LP; p++) r[p] = make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int p = 0; p < LP; p++) {
            // lane starts: steps in registers, stored states in LDS
            start_y[wv][p][lane] = y[p];
            sj[p] = act[p] ? jv[p] : nj;
            s.x[p] = act[p] ? xv[p] : 0.0;
            s.ua[p] = act[p] ? r[p].x : 0.0;
            s.ub[p] = act[p] ? r[p].y : 0.0;
            // folded, weighted inputs; a lane that has not started holds a
            // zero state, so it adds exactly 0 whatever its inputs
            const bool middle = (nlat & 1) && pc[p] == npair - 1;
            const double wt = !act[p] ? 0.0 : (a.adjoint ? (middle ? 0.5 : 1.0) : wl[p]);
#pragma unroll
            for (int f = 0; f < FW; f++) {
                const double2 vn = fn[p][f], vs = fsth[p][f];
                const double er = wt * (vn.x + vs.x), ei = wt * (vn.y + vs.y);
                const double orr = wt * (vn.x - vs.x), oi = wt * (vn.y - vs.y);
                s.ek[p][f] = odd ? ei : er;
                s.es[p][f] = odd ? er : ei;
                s.ok[p][f] = odd ? oi : orr;
                s.os[p][f] = odd ? orr : oi;
            }
        }
    }

    // Warm L2 with the beta entries of this unit (one word per 64-byte line
    // per lane, consumed at the end; see the synthesis kernel).
    __builtin_amdgcn_sched_barrier(0);
    unsigned pf_sink;
    {
        const int nbytes = (j1 - js0 + 2 * SC) * 8;
        const int off = lane * 64;
        pf_sink = *(const unsigned*)((const char*)(P->beta + base + js0) + (off < nbytes ? off : 0));
    }
    const double cm = (m == 0 || !a.adjoint) ? 1.0 : 2.0;
    const int o = tid / PR;        // output of this thread: (row, component)
    const int h = tid % PR;        // its part of the columns
    const int row = o >> 1, comp = o & 1;
    const int t_out = row / FW;
    const int f_out = row % FW;
    const int col = wv * 64 + lane;  // this thread's column
    cdp gam_tab = (cdp)P->gamma + base;

    // beta is loaded one half ahead (the second half's while the first
    // runs, the next pass's first half's after an explicit wait for the
    // second), the segment shift and the start masks one pass ahead; the
    // tables are padded past the last order.  Each explicit lgkmcnt(0) wait
    // comes before the next scalar load is issued, so no wait drains a load
    // just issued (scalar loads return out of order: a wait is always for
    // all of them).  A partial last pass runs all SC steps: the extra
    // degrees belong to no output and are not stored.
    static_assert(NH == 1 || NH == 2, "one or two halves per pass");
    DBlk<kInject> bh0, bh1;
    load_blk(bh0, bet + js0);
    DBlk2u<2 * NH> mkw;
    load_u32(mkw, ckm + 2 * (js0 / kInject));
    int shn = 0;        // js0 is a segment start (the plan rounds it down)
    for (int c = js0; c < j1 + SC; c += SC) {
        const bool compute = c < j1;
        const int sh = shn;
        // The scalar loads above have arrived before the LDS reads of the
        // previous pass's sums are issued (one counter covers both kinds), so
        // the steps below wait on neither and the reads complete under them.
        __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
        __builtin_amdgcn_sched_barrier(0);
        // this wave's slots: starting at each checkpoint, started by it
        unsigned mk[NH], lv[NH];
#pragma unroll
        for (int hh = 0; hh < NH; hh++) {
            mk[hh] = (mkw.v[2 * hh] >> wb) & ((1u << LP) - 1u);
            lv[hh] = (mkw.v[2 * hh + 1] >> wb) & ((1u << LP) - 1u);
        }
        double part[NK];
#pragma unroll
        for (int k = 0; k < NK; k++) part[k] = red[row][2 * (k * PR + h) + comp];
        // gamma of this thread's output in that pass, needed after the steps
        const double gl = gam_tab[min(max(c - SC, js0) + t_out, j1 - 1)];
        // several waves: every wave has read the previous pass's rows before
        // any wave writes this pass's (before the next scalar loads are
        // issued, so that the barrier's wait does not drain them)
        if (W > 1 && compute) __syncthreads();
        if (compute) {
            const int cn = c + SC;
            // two halves: the second half's beta; one half: the next pass's
            load_blk(bh1, bet + c + kInject);
            load_u32(mkw, ckm + 2 * (cn / kInject));
            shn = (cn < j1 && cn % kSegLen == 0) ? segexp[cn / kSegLen] : 0;
            __builtin_amdgcn_sched_barrier(0);
            if (sh != 0) rescale(s.ua, s.ub, sh);
            if (mk[0] != 0u && c <= jwin) start_slots(s.ua, s.ub, sj, start_y[wv], mk[0], c);
            analys_half_from<LP, FW, RS>(lv[0] ? __builtin_ctz(lv[0]) : LP, s, bh0.v, &red[0][col], 0);
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (NH == 2) {
                __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): bh1, the masks, the shift
                __builtin_amdgcn_sched_barrier(0);
                load_blk(bh0, bet + cn);
                __builtin_amdgcn_sched_barrier(0);
                const int c1 = c + kInject;
                if (mk[1] != 0u && c1 <= jwin) start_slots(s.ua, s.ub, sj, start_y[wv], mk[1], c1);
                analys_half_from<LP, FW, RS>(lv[1] ? __builtin_ctz(lv[1]) : LP, s, bh1.v, &red[0][col], kInject);
            } else {
                bh0 = bh1;
            }
        }
        if (c > js0) {
            double s0 = part[0], s1 = part[1], s2 = part[2], s3 = part[3];
#pragma unroll
            for (int k = 4; k < NK; k += 4) {
                s0 += part[k];
                s1 += part[k + 1];
                s2 += part[k + 2];
                s3 += part[k + 3];
            }
            double sum = (s0 + s1) + (s2 + s3);
#pragma unroll
            for (int q = 1; q < PR; q <<= 1) sum += __shfl_xor(sum, q);
            const int j_out = c - SC + t_out;
            if (h == 0 && j_out < j1 && f_out < nf) {
                double val = cm * gl * sum;
                if (m == 0 && comp == 1) val = 0.0;
                a.out[qoff[f_out] + 2 * (base + j_out) + comp] = val;
            }
        }
        if (W > 1) __syncthreads();
    }
    // keeps the prefetch load alive; nfields is never negative
    if (a.nfields < 0) a.out[lane] = (double)pf_sink;
}

// One workgroup per unit.
template <int LP, int FW, int W>
__global__ void __launch_bounds__(64 * W) k_legendre_analys(LegArgs a)
{
    using G = AnalysGeom<LP, FW, W>;
    __shared__ double red[G::NR][G::RS];
    __shared__ double2 start_y[W][LP][64];  // stored lane start states
    analys_unit<LP, FW, W>(a, blockIdx.x, red, start_y);
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
    SHTN_S(1, 4) SHTN_S(2, 4)
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
