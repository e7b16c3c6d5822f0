// Internal structures shared by the host plan code, the C-ABI layer and the
// HIP kernels.  Not part of the public interface (include/shtn.h).
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace shtn {

// Rescaled recurrence (Sec. 3.2, eq. rec, divided through by
// alpha_n = prod_{j=m+1}^{n} a_j^m):
//   y_n = x y_{n-1} + beta_n y_{n-2},  beta_n = -((n-1)^2 - m^2)/((2n-1)(2n-3)),
//   P_n^m(x) = alpha_n y_n.
// The kernels carry u_n = y_n 2^{E_s} where E_s is constant over a segment of
// kSegLen consecutive degrees, so u stays within the range of P; at a segment
// start both recurrence states are multiplied by 2^{E_s - E_{s-1}} (exact).
// gamma_n = alpha_n 2^{-E_s} maps u back to P.
constexpr int kSegLen = 32;
// Underflow guard (Sec. 3.5), run at plan time: the host follows every
// (order, latitude pair) recurrence from n = m in a scaled form
// u = w 2^{-kGuardUnit k} (every kGuardEvery steps a value with k > 0 and
// |w| >= 1 is multiplied by 2^{-kGuardUnit} and k decremented), so values far
// below the double range are tracked exactly.
constexpr int kGuardUnit = 256;
constexpr int kGuardEvery = 4;
// Polar threshold (Sec. 3.1, polar optimisation): contributions with
// |P_n^m| < 2^kPolarLog2 are dropped (the default; a plan may raise the
// threshold, trading accuracy for work, see Plan::polar_log2).  A lane starts at the first checkpoint
// (a multiple of kInject steps) of the block of kInject steps in which its
// |P_n^m| first reaches 2^kPolarLog2 -- or earlier, at the first start of
// its 64-pair block, when its state there is a normal double (see
// lane_starts); before its start the lane holds 0, so it adds exactly 0 and
// the kernels carry no exponent.  The host stores the state (u_{j-2},
// u_{j-1}) entering that step as plain doubles.  A block none of whose
// latitudes reaches the threshold for an order never starts.
constexpr int kPolarLog2 = -200;
constexpr int kInject = 8;
// Analysis accumulates kChunk consecutive degrees per lane before a
// cross-lane reduction.
constexpr int kChunk = 16;
// Entries of zero padding after the tables that the kernels read in blocks
// (beta, the rescaled spectrum): a block starting at an order's last degree
// stays in bounds.
constexpr int kTablePad = 32;
// Pairs per lane and waves of an analysis unit covering npair latitude pairs
// (the smallest power-of-two coverage, up to 8 pairs per lane first).
inline void analys_shape(int npair, int& lp, int& waves)
{
    lp = 1;
    waves = 1;
    while (64 * lp * waves < npair) {
        if (lp < 8) lp *= 2;
        else waves *= 2;
    }
}
// Largest latitude-pair count one analysis unit covers (4 waves x 64 lanes x
// 8 pairs).
constexpr int kMaxAnalysPairs = 2048;

// One work unit of a Legendre kernel = one wave (kUnitInts ints).  Steps j
// count degrees from the order: n = m + j.
enum UnitField {
    U_FIELD = 0,  // first field of the unit (relative; plus blockIdx.y * fw for plan calls)
    U_NF = 1,     // number of fields in the unit (<= fw)
    U_PLAN = 2,   // plan index (batch) or 0
    U_M = 3,      // order m, or -1 for a unit without work
    U_JS = 4,     // first step executed (lanes start there or later)
    U_JW = 5,     // last step at which a lane of the unit starts (injection window; analysis: -1 if none)
    U_PB = 6,     // synthesis: first latitude pair of the block; analysis: first output step j0
    U_J1 = 7,     // analysis: one past the last output step
    U_RST = 8,    // analysis: restart slot of j0 or -1 (j0 = 0)
    U_ZERO = 9,   // synthesis: 1 if no lane of the block ever starts (F written as 0)
};
constexpr int kUnitInts = 12;

// Tables of a plan's device buffer, in buffer order (Plan::table_off).
enum DevTable {
    TB_XP = 0,
    TB_WQ,
    TB_WFULL,
    TB_BETA,
    TB_GAMMA,
    TB_INJ_J,
    TB_INJ_Y,
    TB_SEGEXP,
    TB_SEGOFF,
    TB_RST_Y,
    TB_TW,
    TB_RTW,
    TB_SYNTH_UNITS,
    TB_ANALYS_UNITS,
    TB_CK_MASK,
    TB_COUNT
};

// Lane-start summaries per block of 64 latitude pairs (the pair slot of a
// wave lane: pairs [64 b, 64 b + 64) form block b).  blk_first[m][b]: the
// first start step of the block's lanes of order m (nj if none starts; host
// only).  ck_mask[m][2 k]: bit b set iff some lane of block b starts at the
// checkpoint j = kInject k; ck_mask[m][2 k + 1]: bit b set iff some lane of
// block b has started at or before it.  A kernel skips the slots whose block
// has not started and injects start states only into the blocks whose bit is
// set.
constexpr int kBlkPairs = 64;
constexpr int kMaxMaskBlocks = 32;  // blocks one 32-bit mask covers (2048 pairs)

// Device-resident view of a plan (stored at the start of its device buffer).
struct DevPlan {
    const double* xp;      // [npair] x = cos(theta) of the northern node of each pair
    const double* wq;      // [npair] analysis weight per pair (middle node of odd nlat halved)
    const double* wfull;   // [npair] Gauss weight per pair
    const double* beta;    // [nlm] rescaled recurrence coefficient, m-major
    const double* gamma;   // [nlm] output scale gamma_n
    const int* inj_j;      // [(M+1) * npair] step at which the lane starts (n = m + j), or > lmax - m
    const double* inj_y;   // [(M+1) * npair * 2] state (u_{j-2}, u_{j-1}) entering that step
    const int* segexp;     // per (m, segment s >= 1): E_s - E_{s-1}
    const int* segoff;     // [M+2] index of (m, s=0) in segexp
    const double* rst_y;   // [nrst * npair * 2] analysis restart states (ua, ub), 0 before a lane starts
    const double* tw;      // [K] complex e^{-2 pi i t / K}
    const double* rtw;     // [K+1] complex e^{+2 pi i m / (2K)}
    const int* synth_units;
    const int* analys_units;
    const unsigned* ck_mask;  // [(M+1) * nck * 2] per checkpoint: blocks starting there, blocks started
    int nblk, nck;
    int L, M, nlat, nphi, npair, K;
    long nlm;
    int n_synth_units, n_analys_units;
    int synth_lp, analys_lp, fw, pad0;
    // Longitude coefficients of one field: tile stride and size (complex).
    long f_ts, f_size;
};

struct Tiling {
    int synth_lp = 1;
    int analys_lp = 8;
    int analys_waves = 1;  // waves per analysis unit
    int fw = 1;
    int m_pairing = 0;  // synthesis: 1 = orders m and M-m share a workgroup
    int split = 0;     // analysis: pieces of this many degrees, 0 = automatic
    int fft_rows = 0;  // latitude rows per FFT workgroup, 0 = automatic
};

// Stored-P table of a plan (Sec. 3, precomputed P_n^m; ptable.hip): P_n^m
// at the northern latitude pairs per (order, parity of n - m) in 16 x 16
// blocks of (degree row, pair), rows and pairs zero-padded to 16.  The device
// buffer holds the block offsets (boff) first, then the blocks.
struct PTable {
    int npt = 0;              // pair tiles of 16
    std::vector<long> boff;   // [(M+1) * 2] first block of (order, parity)
    long nblocks = 0;
    size_t head_bytes = 0;    // boff, padded to 256 bytes
    void* dev = nullptr;      // caller's buffer once built
    bool built = false;       // matches the plan's current lane starts
    int synth_rt = 4, synth_ct = 2;    // synthesis: pair tiles, column tiles per wave
    int analys_jt = 4, analys_ct = 2;  // analysis: block rows per parity, column tiles per wave
};

struct Plan {
    int L = 0, M = 0, nlat = 0, nphi = 0, npair = 0, K = 0;
    long nlm = 0;
    Tiling tiling;
    int split_used = 0;
    int synth_wpg = 1;  // waves per synthesis workgroup for the unit order
    int polar_log2 = kPolarLog2;  // lanes start where |P_n^m| first reaches 2^polar_log2
    // host tables
    std::vector<double> x, w;                 // full grid
    std::vector<double> xp, sp, wq, wfull;    // per pair
    std::vector<double> beta, gamma;          // nlm
    std::vector<double> start_y;              // (M+1) x npair: P_m^m mantissa (host emulation only)
    std::vector<int> start_k;                 // its scaled exponent
    std::vector<int> inj_j;                   // (M+1) x npair: lane start step
    std::vector<double> inj_y;                // (M+1) x npair x 2: state entering it
    std::vector<int> segexp, segoff;
    std::vector<double> rst_y;
    std::vector<double> tw, rtw;
    std::vector<int> synth_units, analys_units;
    std::vector<int> first_pair;              // per m: first latitude pair kept by the polar cut
    double min_own_state = 0.0;               // see min_start_state
    std::vector<int> blk_first;               // (M+1) x nblk, see TB_BLK_FIRST
    std::vector<unsigned> ck_mask;            // (M+1) x nck x 2, see TB_CK_MASK
    int nblk = 0, nck = 0;
    // device image
    std::vector<unsigned char> image;  // staged device buffer contents
    std::vector<size_t> table_off;     // byte offsets of each table inside the image
    void* dev = nullptr;               // caller's device buffer after upload
    bool uploaded = false;
    PTable ptab;
    int algo = 0;  // Legendre stage: 0 on-the-fly recurrence, 1 stored P
    // Bumped by every change that moves the plan's device state or its lane
    // starts (upload, tiling, polar threshold, stored-P build or release):
    // batches that copied the plan's device descriptor or built unit tables
    // from its lane starts compare it to refuse stale copies.
    unsigned long gen = 0;
};
// Smallest nonzero |state| at the lanes' own threshold starts, or 0 if
// none: below DBL_MIN a start state at the threshold would be a denormal
// that has lost precision (the threshold is then too low for the plan).
double min_start_state(const Plan& p);
void ptable_layout(Plan& p);  // geometry of the stored-P table

// Error reporting shared by the C-ABI sources (api.cpp): sets the detail
// string of shtn_last_error_detail and returns the code.
int set_error(int code, const std::string& msg);

// A device byte range a call touches; `written` when the call writes it.
struct Range {
    const char* what;
    const void* p;
    size_t bytes;
    bool written;
};
// SHTN_OK, or SHTN_EINVAL when a written range shares a byte with any
// other range of the list (read-only ranges may overlap); the message names
// the first such pair in list order.
int check_disjoint(const std::vector<Range>& r);
// Fields of a transform: spectra (nlm complex each) or grids (nlat x nphi).
enum class Data { spec, grid };
// Appends the device memory a plan's transforms read: its uploaded image
// and, when built, its stored-P table.
void plan_ranges(const Plan& p, std::vector<Range>& r);
int hip_error(int e, const char* where);
int rows_per_block(const Plan& p);  // FFT rows per workgroup for a plan

// Host plan construction (plan.cpp).
Plan* build_plan(int L, int M, int nlat, int nphi, std::string& err);
int rebuild_units(Plan& p, std::string& err);     // units + restart states for the tiling
void lane_starts(Plan& p);                        // start step and state of every (order, pair) lane
// First / last start step of the lanes [i0, i1) of order m that start in
// [lo, hi); false if none does.
bool start_range(const Plan& p, int m, int i0, int i1, int lo, int hi, int& jmin, int& jmax);
void build_image(Plan& p);                        // lays out the device buffer
inline long lm_index(int L, int n, int m) { return (long)m * (2 * L + 1 - m) / 2 + n; }
// Layout of the longitude coefficients F_m(theta_i) of one field: tiles of
// kFTile consecutive latitudes, each tile order-major with the kFTile values
// of one order adjacent:
//   offset(m, i) = (i / kFTile) f_ts + m kFTile + i % kFTile,  f_ts = (mmax+1) kFTile.
// The Legendre kernels' lanes (consecutive latitudes of one order) touch
// whole 128-byte lines, and an FFT workgroup moves its rows in contiguous
// runs (half a tile per order at K = 1024).
constexpr int kFTile = 8;
constexpr int kFTileLg = 3;
struct FLayout {
    long ts, size;  // tile stride and values per field (complex)
};
#ifdef __HIPCC__
// Complex offset of F_m(theta_i) in a field's longitude coefficients.
__device__ __forceinline__ long f_index(long ts, int m, int i)
{
    return (long)(i >> kFTileLg) * ts + m * kFTile + (i & (kFTile - 1));
}
#endif
inline FLayout f_layout(int M, int nlat)
{
    const long ts = (long)(M + 1) * kFTile;
    return {ts, ts * ((nlat + kFTile - 1) / kFTile)};
}
// XCDs of the chip: workgroup b of a launch runs on XCD b % kXcds.
constexpr int kXcds = 8;
size_t align256(size_t v);

// Workspace layout of a plan call with nfields fields.
struct WorkLayout {
    size_t f_bytes;   // F: nfields x f_layout().size complex
    size_t q_bytes;   // rescaled spectrum: nfields x nlm complex
    size_t total;
};
WorkLayout work_layout(const Plan& p, int nfields);

// Fields per wave of the analysis kernel for a (pairs per lane, waves) class:
// the largest count <= fw among the built kernels (two fields with lp <= 4
// and waves <= 2, else one).  Four-field analysis passes were slower than
// two-field ones in every class that can hold them.
inline int analys_fw(int fw, int lp, int waves)
{
    return fw >= 2 && lp <= 4 && waves <= 2 ? 2 : 1;
}

// Kernel launchers (legendre.hip, fft.hip).  Return a hipError_t as int.
struct LegLaunch {
    const DevPlan* plans;  // device array of plans
    const int* units;      // device unit array
    int nunits;
    int grid_y;            // blockIdx.y extent (field groups), 1 for batches
    const long* q_off;     // per-field offset (doubles) of the spectrum, or null (f * 2 nlm)
    const long* f_off;     // per-field offset (doubles) of F, or null (f * 2 (M+1) nlat)
    const double* in;
    double* out;
    int nfields;
    int adjoint;           // 0 forward transform, 1 adjoint variant
    int lp, fw;            // template selection
    int waves = 1;         // analysis: waves per unit (latitude pairs 64 lp waves)
    int wpg;               // synthesis: waves (consecutive units) per workgroup
};
// Qs = gamma * Q per field; q_off/s_off/fplan per field (device) or null.
int launch_prescale(const DevPlan* plans, const long* q_off, const long* s_off, const int* fplan,
                    const double* Q, double* Qs, long max_nlm, int nfields, void* stream);
// Stored-P kernels (ptable.hip).
struct PtabArgs {
    const DevPlan* plan;
    const long* boff;    // device copy of PTable::boff
    const double* tab;   // the blocks
    const double* in;    // synthesis: spectra (nfields x nlm complex); analysis: F
    double* out;         // synthesis: F; analysis: spectra
    int nfields;
    int adjoint;
    int npt;
    int nu;              // analysis: units (groups of block rows) per order, set by the launcher
    const long* q_off = nullptr;  // per-field spectrum offset (doubles), or null (f * 2 nlm)
    const long* f_off = nullptr;  // per-field F offset (doubles), or null (f * 2 f_size)
};
int launch_ptable_build(const DevPlan* plan, const long* boff, double* tab, int npt, int M, void* stream);
int launch_sp_synth(const PtabArgs& a, int M, int rt, int ct, void* stream);
int launch_sp_analys(const PtabArgs& a, int M, int nbr_max, int jt, int ct, void* stream);
// Vector transforms (vector.hip): spectral and latitude combinations around
// the scalar stages.
int launch_vec_spec_in(const DevPlan* plan, int L, int M, const double* S, const double* T, double* Q4, int nfields,
                       int nn, void* stream);
int launch_vec_f_out(const DevPlan* plan, long f_size, const double* F4, double* Fv, int nfields, void* stream);
int launch_vec_f_in(const DevPlan* plan, long f_size, const double* Fv, double* F4, int nfields, void* stream);
int launch_vec_spec_out(const DevPlan* plan, int L, int M, const double* A4, double* S, double* T, int nfields,
                        int nn, void* stream);
int launch_legendre_synth(const LegLaunch& a, void* stream);
int launch_legendre_analys(const LegLaunch& a, void* stream);

struct FftLaunch {
    const DevPlan* plans;     // device plan array
    const int* rowblocks;     // device: per block {field, plan, row0, nrows} or null
    int nblocks;
    int grid_y;
    int K;                    // longest rows of the launch
    int points;               // most complex points in one block (rows x K <= 4096): sizes
                              // the workgroup (one thread per 4, 8 or 16 points) and its LDS
    int rows_per_block;
    const long* g_off;        // per-field grid offset (doubles) or null
    const long* f_off;        // per-field F offset (doubles) or null
    const double* in;
    double* out;
    int nfields;
    double scale;             // r2c: output scale (2 pi/nphi or 1)
    int uniform_k = 0;        // 1: every row of the launch has K points
};
int launch_c2r(const FftLaunch& a, void* stream);
int fft_rows_cap(int K);     // rows of K complex points held by one FFT workgroup
int launch_r2c(const FftLaunch& a, void* stream);

}  // namespace shtn

// Opaque handle behind shtn_plan_t.
struct shtn_plan_s {
    shtn::Plan* p;
};

namespace shtn {
// shtn_synth's checks and launches with `work` as the workspace (api.cpp).
int synth_on_work(shtn_plan_s* plan, const double* Q, double* grid, int nfields, void* work, void* stream);
}  // namespace shtn
