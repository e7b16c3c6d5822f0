// Stored-P Legendre stage (Sec. 3.1, precomputed P_n^m; the runtime choice
// between the two algorithms is the tuning of Sec. 3.2).
//
// The table holds P_n^m(x_i) for every order m, degree n and northern
// latitude pair i, as doubles, split by the parity of j = n - m (the mirror
// fold of Sec. 3.1 pairs even j with F_N + F_S and odd j with F_N - F_S).
// Per (m, parity q) the degrees j = 2 jq + q form rows jq, the pairs form
// columns; both are padded to multiples of 16 with zeros and cut into 16 x 16
// blocks (2 KB), laid out block row by block row.  Inside a block, entry
// (jl, pl) sits at
//     (jl / 4) 64 + (pl / 4) 16 + (jl % 4) 4 + pl % 4,
// so that the 4 degrees x 16 pairs the synthesis feeds one matrix
// instruction, and the 16 degrees x 4 pairs the analysis feeds one, are each
// four whole 128-byte lines.
//
// With several fields of the same shape the Legendre stage is then a dense
// contraction per order: synthesis F[pair][col] = sum_j P[j][pair] Q[j][col],
// analysis Q[j][col] = sum_pair P[j][pair] G[pair][col], where a column is
// (field, re/im).  Both run on the FP64 matrix cores
// (v_mfma_f64_16x16x4_f64: D[16x16] += A[16x4] B[4x16]).  The table is built
// on the device from the plan's own recurrence tables (lane starts, segment
// shifts), so an entry is 0 exactly where the on-the-fly kernels drop the
// term (the polar cut), and equals gamma_n u_n elsewhere.
#include <hip/hip_runtime.h>

#include "shtn_internal.h"

namespace shtn {

typedef double d4 __attribute__((ext_vector_type(4)));

// m-major index of (n = m, m): the first coefficient of order m.
__device__ __forceinline__ long order_base(int L, int m) { return (long)m * (2 * L + 1 - m) / 2 + m; }

// XCD-aware placement: workgroup b of a launch runs on XCD b % kXcds.  The
// nu units of order m all go to XCD m % kXcds, one after another in that
// XCD's share of the launch (orders ascending, longest first), so they share
// its L2 for the order's inputs.  False past the last order.
__device__ __forceinline__ bool xcd_unit(int nu, int M, int& u, int& m)
{
    const int b = blockIdx.x;
    const int slot = b / kXcds;
    const int k = slot / nu;
    u = slot - k * nu;
    m = b % kXcds + kXcds * k;
    return m <= M;
}

__device__ __forceinline__ int ptab_in_block(int jl, int pl)
{
    return (jl >> 2) * 64 + (pl >> 2) * 16 + (jl & 3) * 4 + (pl & 3);
}

// ---------------------------------------------------------------------------
// Builder: one thread per (order, pair column, padded to whole blocks).  The
// recurrence is the synthesis kernel's (same steps, same segment shifts, same
// lane starts), so a lane is 0 before its start step.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64) k_ptable_build(const DevPlan* plan, const long* boff, double* tab, int npt)
{
    const DevPlan& P = *plan;
    const int m = blockIdx.y;
    const int pair = blockIdx.x * 64 + threadIdx.x;
    if (pair >= npt * 16) return;
    const int L = P.L, npair = P.npair;
    const int nj = L - m + 1;
    const long base = order_base(L, m);
    const bool act = pair < npair;
    const size_t q = (size_t)m * npair + (act ? pair : 0);
    const int jst = act ? P.inj_j[q] : nj;
    const double2 y = act ? *(const double2*)(P.inj_y + 2 * q) : make_double2(0.0, 0.0);
    const double x = act ? P.xp[pair] : 0.0;
    const int* segexp = P.segexp + P.segoff[m];
    const int pt = pair >> 4, pl = pair & 15;
    double* t0 = tab + boff[2 * m] * 256;
    double* t1 = tab + boff[2 * m + 1] * 256;
    auto at = [&](double* t, int jq) -> double& {
        return t[((long)(jq >> 4) * npt + pt) * 256 + ptab_in_block(jq & 15, pl)];
    };
    double ua = 0.0, ub = 0.0;
    for (int j = 0; j < nj; j += 2) {
        if (j > 0 && j % kSegLen == 0) {
            const int d = segexp[j / kSegLen];
            ua = ldexp(ua, d);
            ub = ldexp(ub, d);
        }
        if (j == jst) {  // start steps are multiples of kInject, hence even
            ua = y.x;
            ub = y.y;
        }
        ua = fma(x, ub, P.beta[base + j] * ua);
        at(t0, j >> 1) = j >= jst ? P.gamma[base + j] * ua : 0.0;
        if (j + 1 < nj) {
            ub = fma(x, ua, P.beta[base + j + 1] * ub);
            at(t1, j >> 1) = j + 1 >= jst ? P.gamma[base + j + 1] * ub : 0.0;
        }
    }
    // zero rows up to the end of the last block row of each parity
    const int c0 = (nj + 1) >> 1, c1 = nj >> 1;
    for (int jq = c0; jq < ((c0 + 15) & ~15); jq++) at(t0, jq) = 0.0;
    for (int jq = c1; jq < ((c1 + 15) & ~15); jq++) at(t1, jq) = 0.0;
}

// ---------------------------------------------------------------------------
// Synthesis (or the adjoint of the analysis): one wave per (order, group of
// RT pair tiles, group of CT column tiles).  Lane l feeds A[pair l%16][degree
// l/16] and B[degree l/16][column l%16] and holds D[pair l/16 + 4 r][column
// l%16], r < 4.  Even and odd degrees accumulate apart; the fold north =
// E + O, south = E - O is then lane-local.
// ---------------------------------------------------------------------------
template <int RT, int CT>
__global__ void __launch_bounds__(64) k_sp_synth(PtabArgs a)
{
    const DevPlan& P = *a.plan;
    const int npg = (a.npt + RT - 1) / RT;
    int pg, m;
    if (!xcd_unit(npg, P.M, pg, m)) return;
    const int L = P.L, nlat = P.nlat, npair = P.npair;
    const int npt = a.npt;
    const int nj = L - m + 1;
    const long base = order_base(L, m);
    const int lane = threadIdx.x;
    const int col = lane & 15, kk = lane >> 4;
    const int comp = col & 1;

    // Every address, plan value and weight the epilogue needs is read here,
    // before the first store: the output may alias them for all the compiler
    // knows, so reads placed between the stores would each wait on memory.
    const long ts = P.f_ts;
    const double* qp[CT];
    double* fo[CT];
    bool fv[CT];
#pragma unroll
    for (int c = 0; c < CT; c++) {
        const int f = (blockIdx.y * CT + c) * 8 + (col >> 1);
        fv[c] = f < a.nfields;
        const int fc = fv[c] ? f : 0;
        qp[c] = a.in + (a.q_off ? a.q_off[fc] : (long)fc * 2 * P.nlm) + 2 * base + comp;
        fo[c] = a.out + (a.f_off ? a.f_off[fc] : (long)fc * 2 * P.f_size) + comp;
    }
    // pair tiles past the last one read tile pg RT (always present): their
    // output rows are never stored
    int tr[RT];
#pragma unroll
    for (int r = 0; r < RT; r++) tr[r] = pg * RT + r < npt ? r : 0;
    const int a_off = ptab_in_block(kk, lane & 15);  // + 64 s for step s of a block

    d4 acc[2][RT][CT];
#pragma unroll
    for (int q = 0; q < 2; q++)
#pragma unroll
        for (int r = 0; r < RT; r++)
#pragma unroll
            for (int c = 0; c < CT; c++) acc[q][r][c] = d4{0.0, 0.0, 0.0, 0.0};

    // Step br covers block row br of both parities (the odd parity has as
    // many rows as the even one, or one fewer: its missing row reloads the
    // even row).  All operands of a step are loaded before its first matrix
    // instruction, every load unconditional from a valid address (one memory
    // round trip per step; the waves resident on a SIMD overlap them).  Only
    // the contraction index needs a mask: degrees past the order's last
    // (among them the whole missing odd row) get a factor 0 on B (the clamped
    // coefficient belongs to the same order, so this can only turn an output
    // that already involves a non-finite input into NaN; every table entry is
    // finite).  Operands of pair rows past the last and of field columns past
    // the last are left as loaded: they only reach outputs that are never
    // stored.
    const int nbr0 = (((nj + 1) >> 1) + 15) >> 4, nbr1 = ((nj >> 1) + 15) >> 4;
    const double* t0 = a.tab + a.boff[2 * m] * 256 + (long)pg * RT * 256 + a_off;
    const double* t1 = a.tab + a.boff[2 * m + 1] * 256 + (long)pg * RT * 256 + a_off;
    struct Ops {
        double a[2][4][RT];
        double b[2][4][CT];
    };
    auto load = [&](Ops& o, int br) {
#pragma unroll
        for (int q = 0; q < 2; q++) {
            const double* tb = (q && br < nbr1 ? t1 : t0) + (long)br * npt * 256;
#pragma unroll
            for (int s = 0; s < 4; s++) {
#pragma unroll
                for (int r = 0; r < RT; r++) o.a[q][s][r] = tb[tr[r] * 256 + s * 64];
                const int j = min(2 * (br * 16 + s * 4 + kk) + q, nj - 1);
#pragma unroll
                for (int c = 0; c < CT; c++) o.b[q][s][c] = qp[c][2 * j];
            }
        }
    };
    auto run = [&](const Ops& o, int br) {
#pragma unroll
        for (int q = 0; q < 2; q++) {
#pragma unroll
            for (int s = 0; s < 4; s++) {
                const double mj = 2 * (br * 16 + s * 4 + kk) + q < nj ? 1.0 : 0.0;
                double bv[CT];
#pragma unroll
                for (int c = 0; c < CT; c++) bv[c] = o.b[q][s][c] * mj;
#pragma unroll
                for (int r = 0; r < RT; r++)
#pragma unroll
                    for (int c = 0; c < CT; c++)
                        acc[q][r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(o.a[q][s][r], bv[c], acc[q][r][c], 0, 0, 0);
            }
        }
    };
    for (int br = 0; br < nbr0; br++) {
        Ops o;
        load(o, br);
        run(o, br);
    }

    // For the adjoint of the analysis the output carries (2 pi/nphi) w_i / c_m.
    const double cm = a.adjoint ? (2.0 * M_PI / P.nphi) * (m == 0 ? 1.0 : 0.5) : 1.0;
    double sc[RT][4];
#pragma unroll
    for (int r = 0; r < RT; r++)
#pragma unroll
        for (int i = 0; i < 4; i++)
            sc[r][i] = a.adjoint ? cm * P.wfull[min((pg * RT + r) * 16 + kk + 4 * i, npair - 1)] : 1.0;
#pragma unroll
    for (int r = 0; r < RT; r++) {
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int pair = (pg * RT + r) * 16 + kk + 4 * i;
            if (pair >= npair) continue;
            const int is = nlat - 1 - pair;
#pragma unroll
            for (int c = 0; c < CT; c++) {
                if (!fv[c]) continue;
                const double e = acc[0][r][c][i], o = acc[1][r][c][i];
                fo[c][2 * f_index(ts, m, pair)] = sc[r][i] * (e + o);
                if (is != pair) fo[c][2 * f_index(ts, m, is)] = sc[r][i] * (e - o);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Analysis (or the adjoint of the synthesis): one wave per (order, group of
// JT block rows of each parity, group of CT column tiles); the contraction
// runs over all pairs, 4 per step.  Lane l feeds A[degree l%16][pair l/16]
// and B[pair l/16][column l%16] = the folded, weighted longitude
// coefficients, and holds D[degree l/16 + 4 r][column l%16].
// ---------------------------------------------------------------------------
template <int JT, int CT>
__global__ void __launch_bounds__(64) k_sp_analys(PtabArgs a)
{
    const DevPlan& P = *a.plan;
    int g, m;
    if (!xcd_unit(a.nu, P.M, g, m)) return;
    const int L = P.L, nlat = P.nlat, npair = P.npair;
    const int npt = a.npt;
    const int nj = L - m + 1;
    const int nbr0 = (((nj + 1) >> 1) + 15) >> 4, nbr1 = ((nj >> 1) + 15) >> 4;
    if (g * JT >= nbr0) return;  // nbr0 >= nbr1
    const long base = order_base(L, m);
    const int lane = threadIdx.x;
    const int col = lane & 15, kk = lane >> 4;
    const int comp = col & 1;

    // Output bases are read here, before the first store (which, for all the
    // compiler knows, may alias them).
    const double* fp[CT];
    double* qo[CT];
    bool fv[CT];
#pragma unroll
    for (int c = 0; c < CT; c++) {
        const int f = (blockIdx.y * CT + c) * 8 + (col >> 1);
        fv[c] = f < a.nfields;
        const int fc = fv[c] ? f : 0;
        fp[c] = a.in + (a.f_off ? a.f_off[fc] : (long)fc * 2 * P.f_size) + comp;
        qo[c] = a.out + (a.q_off ? a.q_off[fc] : (long)fc * 2 * P.nlm) + 2 * base + comp;
    }
    bool rv[2][JT];
    const double* tq[2][JT];
#pragma unroll
    for (int q = 0; q < 2; q++)
#pragma unroll
        for (int t = 0; t < JT; t++) {
            const int br = g * JT + t;
            rv[q][t] = br < (q ? nbr1 : nbr0);
            // a block row past the last of its parity (the odd parity of
            // order lmax has none) reads the first even one: its accumulator
            // rows are degrees past the order's last, never stored
            const long blk = rv[q][t] ? a.boff[2 * m + q] + (long)br * npt : a.boff[2 * m];
            tq[q][t] = a.tab + blk * 256 + ptab_in_block(lane & 15, kk);  // + 256 pt + 16 (step % 4)
        }

    d4 acc[2][JT][CT];
#pragma unroll
    for (int q = 0; q < 2; q++)
#pragma unroll
        for (int t = 0; t < JT; t++)
#pragma unroll
            for (int c = 0; c < CT; c++) acc[q][t][c] = d4{0.0, 0.0, 0.0, 0.0};

    // Per pair tile (4 steps of 4 pairs) every operand is loaded before the
    // first matrix instruction, unconditionally from valid addresses (pairs
    // past the last read the last pair with weight 0): one memory round trip
    // per tile, overlapped across the waves resident on a SIMD.
    for (int pt = 0; pt < npt; pt++) {
        double pa[4][2][JT], vn[4][CT], vs[4][CT], wv[4];
#pragma unroll
        for (int s = 0; s < 4; s++) {
            const int pc = min(pt * 16 + s * 4 + kk, npair - 1);
            wv[s] = P.wq[pc];
#pragma unroll
            for (int c = 0; c < CT; c++) {
                vn[s][c] = fp[c][2 * f_index(P.f_ts, m, pc)];
                vs[s][c] = fp[c][2 * f_index(P.f_ts, m, nlat - 1 - pc)];
            }
#pragma unroll
            for (int q = 0; q < 2; q++)
#pragma unroll
                for (int t = 0; t < JT; t++) pa[s][q][t] = tq[q][t][pt * 256 + s * 16];
        }
        // keep every load of the tile ahead of its matrix instructions: left
        // alone, the scheduler interleaves them with one wait per group
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int s = 0; s < 4; s++) {
            const int pair = pt * 16 + s * 4 + kk;
            const bool middle = (nlat & 1) && pair == npair - 1;
            const double wt = pair >= npair ? 0.0 : (a.adjoint ? (middle ? 0.5 : 1.0) : wv[s]);
            double ge[CT], go[CT];
#pragma unroll
            for (int c = 0; c < CT; c++) {
                ge[c] = wt * (vn[s][c] + vs[s][c]);
                go[c] = wt * (vn[s][c] - vs[s][c]);
            }
#pragma unroll
            for (int t = 0; t < JT; t++)
#pragma unroll
                for (int c = 0; c < CT; c++) {
                    acc[0][t][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[s][0][t], ge[c], acc[0][t][c], 0, 0, 0);
                    acc[1][t][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[s][1][t], go[c], acc[1][t][c], 0, 0, 0);
                }
        }
    }

    const double cm = (m == 0 || !a.adjoint) ? 1.0 : 2.0;
#pragma unroll
    for (int q = 0; q < 2; q++)
#pragma unroll
        for (int t = 0; t < JT; t++)
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int j = 2 * ((g * JT + t) * 16 + kk + 4 * i) + q;
                if (j >= nj) continue;
#pragma unroll
                for (int c = 0; c < CT; c++) {
                    if (!fv[c]) continue;
                    const double v = (m == 0 && comp == 1) ? 0.0 : cm * acc[q][t][c][i];
                    qo[c][2 * j] = v;
                }
            }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
int launch_ptable_build(const DevPlan* plan, const long* boff, double* tab, int npt, int M, void* stream)
{
    hipLaunchKernelGGL(k_ptable_build, dim3((npt * 16 + 63) / 64, M + 1), dim3(64), 0, (hipStream_t)stream,
                       plan, boff, tab, npt);
    return (int)hipGetLastError();
}

template <int RT, int CT>
static int launch_sp_synth_t(const PtabArgs& a, int M, void* stream)
{
    const int npg = (a.npt + RT - 1) / RT;
    const int nfg = (a.nfields + 8 * CT - 1) / (8 * CT);
    const int nx = kXcds * ((M + kXcds) / kXcds) * npg;
    hipLaunchKernelGGL((k_sp_synth<RT, CT>), dim3(nx, nfg), dim3(64), 0, (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

template <int JT, int CT>
static int launch_sp_analys_t(const PtabArgs& a, int M, int nbr_max, void* stream)
{
    const int ng = (nbr_max + JT - 1) / JT;
    const int nfg = (a.nfields + 8 * CT - 1) / (8 * CT);
    const int nx = kXcds * ((M + kXcds) / kXcds) * ng;
    PtabArgs b = a;
    b.nu = ng;
    hipLaunchKernelGGL((k_sp_analys<JT, CT>), dim3(nx, nfg), dim3(64), 0, (hipStream_t)stream, b);
    return (int)hipGetLastError();
}

// A call of at most 8 fields fills one column tile: a second would only
// add columns that are never stored.
int launch_sp_synth(const PtabArgs& a, int M, int rt, int ct, void* stream)
{
    if (a.nfields <= 8) ct = 1;
#define SHTN_SP(RV, CV) \
    if (rt == RV && ct == CV) return launch_sp_synth_t<RV, CV>(a, M, stream);
    SHTN_SP(1, 1) SHTN_SP(2, 1) SHTN_SP(4, 1) SHTN_SP(1, 2) SHTN_SP(2, 2) SHTN_SP(4, 2)
#undef SHTN_SP
    return (int)hipErrorInvalidValue;
}

int launch_sp_analys(const PtabArgs& a, int M, int nbr_max, int jt, int ct, void* stream)
{
    if (a.nfields <= 8) ct = 1;
#define SHTN_SP(JV, CV) \
    if (jt == JV && ct == CV) return launch_sp_analys_t<JV, CV>(a, M, nbr_max, stream);
    SHTN_SP(1, 1) SHTN_SP(2, 1) SHTN_SP(4, 1) SHTN_SP(1, 2) SHTN_SP(2, 2) SHTN_SP(4, 2)
#undef SHTN_SP
    return (int)hipErrorInvalidValue;
}

}  // namespace shtn
