// Host-side plan construction: Gauss grid, recurrence tables, start values
// with scaled exponents, analysis restart states, FFT twiddles and the work
// unit lists.  Host code only.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <thread>

#include "shtn_internal.h"

namespace shtn {

typedef long double ld;
static const ld kPi = 3.141592653589793238462643383279502884L;

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Legendre P_N and P_{N-1} at x by the Bonnet recurrence (Sec. 2.1).
static void legendre_pair(int N, ld x, ld& pn, ld& pn1)
{
    ld p0 = 1, p1 = x;
    if (N == 0) { pn = 1; pn1 = 0; return; }
    for (int n = 2; n <= N; n++) {
        ld p2 = ((2 * n - 1) * x * p1 - (n - 1) * p0) / n;
        p0 = p1;
        p1 = p2;
    }
    pn = p1;
    pn1 = p0;
}

// Gauss-Legendre rule (Sec. 2.3, eq. gauss) by Newton iteration on the
// colatitude theta (long double): f(theta) = P_N(cos theta),
// f'(theta) = -N (P_{N-1} - x P_N) / sin theta.  Working in theta keeps
// sin(theta) accurate at the poles, where it sets the P_m^m start values.
// Weight w = 2 sin^2 / (N^2 (P_{N-1} - x P_N)^2) (= 2/((1-x^2) P_N'^2)).
static void gauss_rule(int N, std::vector<ld>& theta, std::vector<ld>& w)
{
    theta.assign(N, 0);
    w.assign(N, 0);
    for (int i = 0; i < (N + 1) / 2; i++) {
        ld t;
        if ((N & 1) && i == N / 2) {
            t = kPi / 2;
        } else {
            t = kPi * ((ld)i + 0.75L) / ((ld)N + 0.5L);
            for (int it = 0; it < 100; it++) {
                ld x = cosl(t), s = sinl(t), pn, pn1;
                legendre_pair(N, x, pn, pn1);
                ld d = -N * (pn1 - x * pn) / s;
                ld dt = pn / d;
                t -= dt;
                if (fabsl(dt) <= 4 * LDBL_EPSILON * t) {
                    x = cosl(t); s = sinl(t);
                    legendre_pair(N, x, pn, pn1);
                    d = -N * (pn1 - x * pn) / s;
                    t -= pn / d;
                    break;
                }
            }
        }
        ld x = cosl(t), s = sinl(t), pn, pn1;
        if ((N & 1) && i == N / 2) x = 0;
        legendre_pair(N, x, pn, pn1);
        ld dd = N * (pn1 - x * pn);
        ld wi = 2 * s * s / (dd * dd);
        theta[i] = t;
        w[i] = wi;
        theta[N - 1 - i] = kPi - t;
        w[N - 1 - i] = wi;
    }
}

static int log2_floor(ld v)
{
    int e;
    frexpl(v, &e);  // v = f 2^e, f in [0.5, 1)
    return e - 1;
}

// Lane starts (Sec. 3.5 guard and Sec. 3.1 polar threshold, at plan time).
// For each (order, latitude pair) the recurrence is followed from n = m in the
// scaled form u = w 2^{-256 k} with the kernels' own steps (same segment
// shifts, same fused multiply-adds), so values far below the range of double
// are tracked exactly.
//
// A lane's own start is the checkpoint (multiple of kInject) that opens the
// first block of kInject steps in which |P_n^m| reaches 2^polar_log2 (nj =
// lmax - m + 1 if it never does).  The latitudes of one 64-pair block run in
// the same pair slot of a wave, so a block is live from the earliest own
// start among its lanes; every lane of the block starts there too, from its
// exact state at that step, as long as that state is a normal double with
// margin (each component 0 or of magnitude at least 2^kStartFloor), and
// otherwise at the first later checkpoint where it is (no later than its
// own start).  Starting early only adds terms below the threshold, and it
// leaves most lanes of a block starting together: the kernels inject start
// states at few checkpoints.
constexpr int kStartFloor = -900;

// Follows lane (m, i) and returns at the first checkpoint c >= c_lo where
// `own` (the block of kInject steps from c reaches the threshold) or, if
// !own, the entering state is representable; jst = nj if none.
static void lane_walk(const Plan& p, int m, int i, int c_lo, bool own, int& jst, double& ya, double& yb)
{
    const int nj = p.L - m + 1;
    const long base = lm_index(p.L, m, m);
    const double down = std::ldexp(1.0, -kGuardUnit);
    const double floor_v = std::ldexp(1.0, kStartFloor);
    const double x = p.xp[i];
    double ua = p.start_y[(size_t)m * p.npair + i], ub = 0.0;
    int k = p.start_k[(size_t)m * p.npair + i];
    jst = nj;
    ya = yb = 0.0;
    for (int c = 0; c < nj; c += kInject) {
        if (c > 0 && c % kSegLen == 0) {
            const int d = p.segexp[p.segoff[m] + c / kSegLen];
            ua = std::ldexp(ua, d);
            ub = std::ldexp(ub, d);
        }
        const double sa = ua, sb = ub;
        const int sk = k;
        if (!own && c >= c_lo) {
            const double va = std::ldexp(sa, -kGuardUnit * sk), vb = std::ldexp(sb, -kGuardUnit * sk);
            const bool ok_a = va == 0.0 || std::fabs(va) >= floor_v, ok_b = vb == 0.0 || std::fabs(vb) >= floor_v;
            if (ok_a && ok_b && (va != 0.0 || vb != 0.0)) {
                jst = c;
                ya = va;
                yb = vb;
                return;
            }
        }
        bool sig = false;
        for (int j = c; j < std::min(c + kInject, nj); j += 2) {
            if (j % kGuardEvery == 0 && k > 0 && (std::fabs(ua) >= 1.0 || std::fabs(ub) >= 1.0)) {
                ua *= down;
                ub *= down;
                k -= 1;
            }
            ua = std::fma(x, ub, p.beta[base + j] * ua);
            if (j + 1 < nj) ub = std::fma(x, ua, p.beta[base + j + 1] * ub);
            // |P| = |u| gamma 2^{-256 k}
            const double v = std::max(std::fabs(ua) * p.gamma[base + j],
                                      j + 1 < nj ? std::fabs(ub) * p.gamma[base + j + 1] : 0.0);
            if (v > 0.0) {
                int e;
                std::frexp(v, &e);
                if (e - (long)kGuardUnit * k >= p.polar_log2) sig = true;
            }
        }
        if (own && sig) {
            jst = c;
            ya = std::ldexp(sa, -kGuardUnit * sk);
            yb = std::ldexp(sb, -kGuardUnit * sk);
            return;
        }
    }
}

void lane_starts(Plan& p)
{
    const int M = p.M, np = p.npair;
    const int nb = (np + kBlkPairs - 1) / kBlkPairs;
    p.inj_j.assign((size_t)(M + 1) * np, 0);
    p.inj_y.assign((size_t)(M + 1) * np * 2, 0.0);
    p.first_pair.assign(M + 1, 0);
    std::vector<double> own_min(M + 1, 0.0);
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (unsigned tid = 0; tid < nth; tid++) {
        pool.emplace_back([&, tid]() {
            std::vector<int> own(np);
            for (int m = (int)tid; m <= M; m += (int)nth) {
                const int nj = p.L - m + 1;
                // own starts (the threshold), the first kept pair, and the
                // smallest nonzero state there
                int first = np;
                double lo = 0.0;
                for (int i = 0; i < np; i++) {
                    double ya, yb;
                    lane_walk(p, m, i, 0, true, own[i], ya, yb);
                    if (own[i] < nj && first == np) first = i;
                    for (double v : {ya, yb}) {
                        const double a = std::fabs(v);
                        if (a > 0.0 && (lo == 0.0 || a < lo)) lo = a;
                    }
                }
                p.first_pair[m] = first;
                own_min[m] = lo;
                // block starts: each lane from its block's first own start
                for (int b = 0; b < nb; b++) {
                    const int i0 = b * kBlkPairs, i1 = std::min(np, i0 + kBlkPairs);
                    int bfirst = nj;
                    for (int i = i0; i < i1; i++) bfirst = std::min(bfirst, own[i]);
                    for (int i = i0; i < i1; i++) {
                        const size_t q = (size_t)m * np + i;
                        if (bfirst >= nj) {
                            p.inj_j[q] = nj;
                            p.inj_y[2 * q] = p.inj_y[2 * q + 1] = 0.0;
                        } else {
                            lane_walk(p, m, i, bfirst, false, p.inj_j[q], p.inj_y[2 * q], p.inj_y[2 * q + 1]);
                        }
                    }
                }
            }
        });
    }
    for (auto& th : pool) th.join();
    p.min_own_state = 0.0;
    for (double v : own_min)
        if (v > 0.0 && (p.min_own_state == 0.0 || v < p.min_own_state)) p.min_own_state = v;
    // per 64-pair block: first start step and the checkpoints with starts
    // (the mask holds 32 blocks; plans with more pairs leave it 0 beyond,
    // the kernels that read it cover at most kMaxMaskBlocks blocks)
    const int nck = (p.L + 2 * kChunk) / kInject + 2;  // checkpoints of order 0, padded for loads a pass ahead
    p.nblk = nb;
    p.nck = nck;
    p.blk_first.assign((size_t)(M + 1) * nb, 0);
    p.ck_mask.assign((size_t)(M + 1) * nck * 2, 0u);
    for (int m = 0; m <= M; m++) {
        const int nj = p.L - m + 1;
        unsigned* ck = &p.ck_mask[(size_t)m * nck * 2];
        for (int b = 0; b < nb; b++) {
            int first = nj;
            for (int i = b * kBlkPairs; i < std::min(np, (b + 1) * kBlkPairs); i++) {
                const int j = p.inj_j[(size_t)m * np + i];
                if (j >= nj) continue;
                first = std::min(first, j);
                if (b < kMaxMaskBlocks) ck[2 * (j / kInject)] |= 1u << b;
            }
            p.blk_first[(size_t)m * nb + b] = first;
            if (b < kMaxMaskBlocks && first < nj)
                for (int k = first / kInject; k < nck; k++) ck[2 * k + 1] |= 1u << b;
        }
    }
}

double min_start_state(const Plan& p) { return p.min_own_state; }

Plan* build_plan(int L, int M, int nlat, int nphi, std::string& err)
{
    if (L < 0 || M < 0 || M > L) { err = "need 0 <= mmax <= lmax"; return nullptr; }
    if (nlat < 1) { err = "need nlat >= 1"; return nullptr; }
    if (nphi < 1 || nphi <= 2 * M) { err = "need nphi > 2*mmax (no aliasing of order mmax)"; return nullptr; }
    if (L > 16383 || nlat > 32768 || nphi > (1 << 16)) { err = "size beyond the supported range"; return nullptr; }
    Plan* p = new Plan();
    p->L = L; p->M = M; p->nlat = nlat; p->nphi = nphi;
    p->npair = (nlat + 1) / 2;
    p->K = nphi / 2 > 0 ? nphi / 2 : 1;
    p->nlm = (long)(M + 1) * (L + 1) - (long)M * (M + 1) / 2;
    const int np = p->npair;

    // ---- grid ----
    std::vector<ld> th, wl;
    gauss_rule(nlat, th, wl);
    p->x.resize(nlat); p->w.resize(nlat);
    for (int i = 0; i < nlat; i++) {
        p->x[i] = (double)((nlat & 1) && i == nlat / 2 ? 0.0L : cosl(th[i]));
        p->w[i] = (double)wl[i];
    }
    p->xp.resize(np); p->sp.resize(np); p->wq.resize(np); p->wfull.resize(np);
    for (int i = 0; i < np; i++) {
        p->xp[i] = p->x[i];
        p->sp[i] = (double)sinl(th[i]);
        p->wfull[i] = p->w[i];
        bool middle = (nlat & 1) && i == nlat / 2;
        p->wq[i] = middle ? 0.5 * p->w[i] : p->w[i];
    }

    // ---- rescaled recurrence tables (Sec. 3.2, eq. rec) ----
    p->beta.resize(p->nlm); p->gamma.resize(p->nlm);
    p->segoff.resize(M + 2);
    int nseg_total = 0;
    for (int m = 0; m <= M; m++) {
        p->segoff[m] = nseg_total;
        nseg_total += (L - m + 1 + kSegLen - 1) / kSegLen;
    }
    p->segoff[M + 1] = nseg_total;
    p->segexp.assign(nseg_total, 0);
    for (int m = 0; m <= M; m++) {
        long base = lm_index(L, m, m);
        ld alpha = 1;
        int E = 0;
        for (int n = m; n <= L; n++) {
            int j = n - m;
            if (n > m) {
                ld a = sqrtl((ld)(4.0L * n * n - 1) / ((ld)n * n - (ld)m * m));
                alpha *= a;
            }
            if (j > 0 && j % kSegLen == 0) {
                int En = log2_floor(alpha);
                p->segexp[p->segoff[m] + j / kSegLen] = En - E;
                E = En;
            }
            double b;
            if (j == 0) b = 1.0;        // u_m = 1 * (start value) with u_{m-1} = 0
            else if (j == 1) b = 0.0;   // u_{m+1} = x u_m
            else {
                long long num = (long long)(n - 1 - m) * (n - 1 + m);
                long long den = (long long)(2 * n - 1) * (2 * n - 3);
                b = (double)(-(ld)num / (ld)den);
            }
            p->beta[base + j] = b;
            p->gamma[base + j] = (double)ldexpl(alpha, -E);
        }
    }

    // ---- P_m^m start values with scaled exponents (Sec. 3.2 and 3.5) ----
    // P_m^m(x) = (-1)^m sqrt(prod_{k<=m}(2k+1)/(2k) / (4 pi)) sin^m(theta),
    // kept as mantissa * 2^e (long double, renormalised every step), then
    // split as w * 2^{-256 k} with k >= 0 minimal such that |w| >= 2^-256.
    p->start_y.assign((size_t)(M + 1) * np, 0.0);
    p->start_k.assign((size_t)(M + 1) * np, 0);
    for (int i = 0; i < np; i++) {
        ld s = sinl(th[i]);
        ld v = sqrtl(1.0L / (4 * kPi));
        long e = 0;
        for (int m = 0; m <= M; m++) {
            if (m > 0) {
                v *= -sqrtl((ld)(2 * m + 1) / (ld)(2 * m)) * s;
                int ei;
                v = frexpl(v, &ei);
                e += ei;
            }
            // value = v 2^e, |v| in [0.5, 1) (or exactly 1/sqrt(4 pi) at m = 0)
            long k = 0;
            long ee = e;
            // |value| < 2^{e}; need |value| 2^{256 k} >= 2^{-256} for the minimal k
            while (ee + (long)kGuardUnit * k < -(long)kGuardUnit + 1) k++;
            p->start_y[(size_t)m * np + i] = (double)ldexpl(v, (int)(ee + (long)kGuardUnit * k));
            p->start_k[(size_t)m * np + i] = (int)k;
        }
    }

    // ---- lane starts: guard and polar threshold at plan time ----
    lane_starts(*p);

    // ---- FFT twiddles ----
    const int K = p->K;
    p->tw.resize(2 * (size_t)K);
    for (int t = 0; t < K; t++) {
        ld a = 2 * kPi * (ld)t / (ld)K;
        p->tw[2 * t] = (double)cosl(a);
        p->tw[2 * t + 1] = (double)(-sinl(a));
    }
    p->rtw.resize(2 * (size_t)(K + 1));
    for (int m = 0; m <= K; m++) {
        ld a = kPi * (ld)m / (ld)K;  // 2 pi m / (2K)
        p->rtw[2 * m] = (double)cosl(a);
        p->rtw[2 * m + 1] = (double)sinl(a);
    }

    // default tiling: one pair per synthesis lane, orders unpaired (measured
    // fastest at lmax 1023); one analysis wave covers every pair of its order
    p->tiling.synth_lp = 1;
    p->tiling.m_pairing = 0;
    analys_shape(np, p->tiling.analys_lp, p->tiling.analys_waves);
    if (rebuild_units(*p, err)) { delete p; return nullptr; }
    build_image(*p);
    ptable_layout(*p);
    return p;
}

// Analysis restart states: the kernels' recurrence (same operations, same
// order, fused multiply-adds) run per lane from its start step up to each
// listed restart step, giving the state entering that step after its segment
// shift.  Lanes that start at or after a restart step hold 0 there.
static void restart_states(const Plan& p, int m, const std::vector<int>& j_list, std::vector<double>& ys)
{
    const int np = p.npair;
    const int nj = p.L - m + 1;
    const long base = lm_index(p.L, m, m);
    ys.assign(j_list.size() * np * 2, 0.0);
    for (int i = 0; i < np; i++) {
        const size_t q = (size_t)m * np + i;
        const int js = p.inj_j[q];
        if (js >= nj) continue;
        const double x = p.xp[i];
        double ua = p.inj_y[2 * q], ub = p.inj_y[2 * q + 1];
        int j = js;
        for (size_t r = 0; r < j_list.size(); r++) {
            const int jr = j_list[r];
            if (jr <= js) continue;  // the lane starts by itself in that unit
            for (; j < jr; j += 2) {
                if (j > js && j % kSegLen == 0) {
                    const int d = p.segexp[p.segoff[m] + j / kSegLen];
                    ua = std::ldexp(ua, d);
                    ub = std::ldexp(ub, d);
                }
                ua = std::fma(x, ub, p.beta[base + j] * ua);
                if (j + 1 < nj) ub = std::fma(x, ua, p.beta[base + j + 1] * ub);
            }
            // entering jr (a segment start): apply its shift
            const int d = p.segexp[p.segoff[m] + jr / kSegLen];
            ys[(r * np + i) * 2] = std::ldexp(ua, d);
            ys[(r * np + i) * 2 + 1] = std::ldexp(ub, d);
        }
    }
}

// First / last start step of the lanes [i0, i1) of order m that start in
// [lo, hi); returns false if none does.
bool start_range(const Plan& p, int m, int i0, int i1, int lo, int hi, int& jmin, int& jmax)
{
    jmin = hi;
    jmax = lo;
    bool any = false;
    for (int i = i0; i < i1; i++) {
        const int j = p.inj_j[(size_t)m * p.npair + i];
        if (j < lo || j >= hi) continue;
        any = true;
        jmin = std::min(jmin, j);
        jmax = std::max(jmax, j);
    }
    return any;
}

// Time of an analysis unit covering steps [js, j1) of order m, in ns on
// MI355X (two waves per SIMD), as measured per unit: about 4.6 us of set-up,
// then per half pass (kInject steps) 0.32 us plus 0.1 us per live pair slot
// (slots whose 64-pair block has started) plus 0.46 us when start states are
// injected.  The waves of a unit keep pace, so the busiest one counts.  Used
// to order the pieces and to deal the orders to the XCDs.
static long analys_unit_cost(const Plan& p, int m, int js, int j1)
{
    const int lp = p.tiling.analys_lp, waves = p.tiling.analys_waves;
    const int* bf = &p.blk_first[(size_t)m * p.nblk];
    const unsigned* ck = &p.ck_mask[(size_t)m * p.nck * 2];
    const unsigned wmask = lp >= 32 ? ~0u : (1u << lp) - 1u;
    long cost = 4600;
    for (int c = js; c < j1; c += kInject) {
        long worst = 0;
        for (int w = 0; w < waves; w++) {
            int k = 0;
            for (int q = 0; q < lp; q++) {
                const int b = w * lp + q;
                if (b < p.nblk && bf[b] <= c) k++;
            }
            const bool inj = ((ck[2 * (c / kInject)] >> (w * lp)) & wmask) != 0u;
            worst = std::max(worst, 320L + 100L * k + (inj ? 460L : 0L));
        }
        cost += worst;
    }
    return cost;
}

int rebuild_units(Plan& p, std::string& err)
{
    const Tiling& t = p.tiling;
    const int np = p.npair, L = p.L, M = p.M;
    // ---- synthesis units: order x latitude-pair block ----
    // m_pairing 0: one workgroup per order (its latitude blocks);
    // 1: orders m and M-m in the same workgroup (equal work per workgroup).
    p.synth_units.clear();
    const int blk = 64 * t.synth_lp;
    const int nblk = (np + blk - 1) / blk;
    const int max_wpg = t.synth_lp == 1 && t.fw == 1 ? 16 : 8;
    auto emit = [&](int m, int b) {
        int u[kUnitInts] = {0, t.fw, 0, -1, 0, 0, b * blk, 0, -1, 0, 0, 0};
        if (m >= 0) {
            const int nj = L - m + 1;
            int jmin, jmax;
            u[U_M] = m;
            if (start_range(p, m, b * blk, std::min((b + 1) * blk, np), 0, nj, jmin, jmax)) {
                u[U_JS] = jmin;
                u[U_JW] = jmax;
            } else {
                u[U_ZERO] = 1;  // every lane of the block is below the polar threshold
            }
        }
        p.synth_units.insert(p.synth_units.end(), u, u + kUnitInts);
    };
    if (t.m_pairing && 2 * nblk <= max_wpg) {
        for (int m = 0; 2 * m <= M; m++) {
            const int m2 = M - m;
            for (int b = 0; b < nblk; b++) emit(m, b);
            for (int b = 0; b < nblk; b++) emit(m2 != m ? m2 : -1, b);
        }
        p.synth_wpg = 2 * nblk;
    } else {
        for (int m = 0; m <= M; m++)
            for (int b = 0; b < nblk; b++) emit(m, b);
        // the latitude blocks of one order, or an equal share of them
        int wpg = std::min(nblk, max_wpg);
        while (nblk % wpg) wpg--;
        p.synth_wpg = wpg;
    }

    // ---- analysis units: (m, degree range) pieces of S degrees ----
    // Workgroup b runs on XCD b % kXcds.  All pieces of one order go to one
    // XCD, so the inputs and start states they share come from that XCD's
    // L2; orders are dealt largest first to the XCD with the least work so
    // far, each XCD runs its pieces longest first (the hardware hands the
    // next piece to the first free slot, so the short ones fill the tail),
    // and the shorter XCD queues are padded with units without work.
    int S = t.split;
    if (S <= 0) {
        // about two pieces per SIMD at large sizes (256 at lmax 1023)
        const long target = p.nlm / 2048;
        S = (int)std::max<long>(64, (target / kSegLen) * kSegLen);
    }
    if (S % kSegLen) { err = "split must be a multiple of 32"; return -1; }
    p.split_used = S;
    struct AU { int m, j0, j1, js, jw, rst; long cost; };
    std::vector<std::vector<int>> rj(M + 1);  // restart steps of each order, ascending
    auto make_piece = [&](int m, int j0, int j1) {
        int jmin, jmax;
        // lanes started before j0 are live from the restart state; the piece
        // may skip ahead (in whole segments) to its first start
        const bool live0 = start_range(p, m, 0, np, 0, j0 + (j0 == 0 ? 1 : 0), jmin, jmax);
        int js, jw;
        // jw: the last start step inside the piece, -1 if no lane starts in it
        if (live0) {
            js = j0;
            jw = start_range(p, m, 0, np, j0, j1, jmin, jmax) ? jmax : -1;
        } else if (start_range(p, m, 0, np, j0, j1, jmin, jmax)) {
            js = j0 + ((jmin - j0) / kSegLen) * kSegLen;
            jw = jmax;
        } else {
            js = j1;  // nothing starts: the piece only writes zeros
            jw = -1;
        }
        int r = -1;
        if (j0 > 0) {
            r = (int)rj[m].size();
            rj[m].push_back(j0);
        }
        return AU{m, j0, j1, js, jw, r, js < j1 ? analys_unit_cost(p, m, js, j1) : 0};
    };
    std::vector<std::vector<AU>> pieces(M + 1);
    std::vector<long> mcost(M + 1, 0);
    for (int m = 0; m <= M; m++) {
        const int nj = L - m + 1;
        for (int j0 = 0; j0 < nj; j0 += S) {
            pieces[m].push_back(make_piece(m, j0, std::min(j0 + S, nj)));
            mcost[m] += pieces[m].back().cost;
        }
    }
    std::vector<int> ms(M + 1);
    for (int m = 0; m <= M; m++) ms[m] = m;
    std::stable_sort(ms.begin(), ms.end(), [&](int a, int b) { return mcost[a] > mcost[b]; });
    std::vector<std::vector<AU>> xq(kXcds);
    {
        long xload[kXcds] = {0};
        for (int m : ms) {
            int x = 0;
            for (int k = 1; k < kXcds; k++)
                if (xload[k] < xload[x]) x = k;
            xload[x] += mcost[m];
            xq[x].insert(xq[x].end(), pieces[m].begin(), pieces[m].end());
        }
    }
    for (auto& q : xq)
        std::stable_sort(q.begin(), q.end(), [](const AU& a, const AU& b) { return a.cost > b.cost; });
    // restart slots: order by order, each order's restart steps ascending
    int nrst = 0;
    std::vector<int> rbase(M + 1, 0);
    for (int m = 0; m <= M; m++) {
        rbase[m] = nrst;
        nrst += (int)rj[m].size();
    }
    p.analys_units.clear();
    size_t qlen = 0;
    for (auto& q : xq) qlen = std::max(qlen, q.size());
    for (size_t k = 0; k < qlen; k++) {
        for (int x = 0; x < kXcds; x++) {
            int u[kUnitInts] = {0, t.fw, 0, -1, 0, 0, 0, 0, -1, 0, 0, 0};
            if (k < xq[x].size()) {
                const AU& a = xq[x][k];
                const int v[kUnitInts] = {0, t.fw, 0, a.m, a.js, a.jw, a.j0, a.j1,
                                          a.rst >= 0 ? rbase[a.m] + a.rst : -1, 0, 0, 0};
                std::copy(v, v + kUnitInts, u);
            }
            p.analys_units.insert(p.analys_units.end(), u, u + kUnitInts);
        }
    }
    p.rst_y.assign((size_t)nrst * np * 2, 0.0);
    // restart states, orders split over host threads
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (unsigned tid = 0; tid < nth; tid++) {
        pool.emplace_back([&, tid]() {
            std::vector<double> ys;
            for (int m = (int)tid; m <= M; m += (int)nth) {
                if (rj[m].empty()) continue;
                restart_states(p, m, rj[m], ys);
                std::memcpy(&p.rst_y[(size_t)rbase[m] * np * 2], ys.data(), ys.size() * sizeof(double));
            }
        });
    }
    for (auto& th : pool) th.join();
    return 0;
}

template <typename T>
static size_t put(std::vector<unsigned char>& img, size_t off, const std::vector<T>& v)
{
    size_t bytes = v.size() * sizeof(T);
    if (img.size() < off + bytes) img.resize(off + bytes);
    if (bytes) std::memcpy(img.data() + off, v.data(), bytes);
    return align256(off + bytes);
}

// Stored-P table geometry: per order m (nj = lmax - m + 1 degrees) the even
// offsets j = n - m give ceil(nj/2) rows and the odd ones floor(nj/2); each
// parity takes ceil(rows/16) block rows of npt blocks.
void ptable_layout(Plan& p)
{
    PTable& t = p.ptab;
    t.npt = (p.npair + 15) / 16;
    t.boff.assign((size_t)(p.M + 1) * 2, 0);
    long cur = 0;
    for (int m = 0; m <= p.M; m++) {
        const int nj = p.L - m + 1;
        const int rows[2] = {(nj + 1) / 2, nj / 2};
        for (int q = 0; q < 2; q++) {
            t.boff[2 * m + q] = cur;
            cur += (long)((rows[q] + 15) / 16) * t.npt;
        }
    }
    t.nblocks = cur;
    t.head_bytes = align256(t.boff.size() * sizeof(long));
}

void build_image(Plan& p)
{
    p.image.clear();
    p.table_off.assign(TB_COUNT, 0);
    size_t off = align256(sizeof(DevPlan));
    p.image.resize(off, 0);
    auto place = [&](int tb, const auto& v) {
        p.table_off[tb] = off;
        off = put(p.image, off, v);
    };
    place(TB_XP, p.xp);
    place(TB_WQ, p.wq);
    place(TB_WFULL, p.wfull);
    {
        // padded: the kernels load beta in blocks that may run past the end
        std::vector<double> bpad(p.beta);
        bpad.resize(p.beta.size() + kTablePad, 0.0);
        place(TB_BETA, bpad);
    }
    place(TB_GAMMA, p.gamma);
    place(TB_INJ_J, p.inj_j);
    place(TB_INJ_Y, p.inj_y);
    place(TB_SEGEXP, p.segexp);
    place(TB_SEGOFF, p.segoff);
    place(TB_RST_Y, p.rst_y);
    place(TB_TW, p.tw);
    place(TB_RTW, p.rtw);
    place(TB_SYNTH_UNITS, p.synth_units);
    place(TB_ANALYS_UNITS, p.analys_units);
    place(TB_CK_MASK, p.ck_mask);
    p.image.resize(off, 0);
}

WorkLayout work_layout(const Plan& p, int nfields)
{
    WorkLayout w;
    w.f_bytes = align256((size_t)nfields * f_layout(p.M, p.nlat).size * 16);
    w.q_bytes = align256(((size_t)nfields * p.nlm + kTablePad) * 16);  // padded for block loads
    w.total = w.f_bytes + w.q_bytes;
    return w;
}

}  // namespace shtn
