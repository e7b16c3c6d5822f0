// C-ABI of libshtn (declared in include/shtn.h): validation, plan upload and
// the launch sequences of the four transforms.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "shtn.h"
#include "shtn_internal.h"
#include "shtn_profile.h"

using namespace shtn;

namespace {
thread_local std::string g_detail;
}  // namespace

namespace shtn {
int set_error(int code, const std::string& msg)
{
    g_detail = msg;
    return code;
}

int hip_error(int e, const char* where)
{
    g_detail = std::string(where) + ": " + hipGetErrorString((hipError_t)e);
    return SHTN_EHIP;
}

int check_disjoint(const std::vector<Range>& r)
{
    for (size_t i = 0; i < r.size(); i++)
        for (size_t j = i + 1; j < r.size(); j++) {
            if (!r[i].written && !r[j].written) continue;
            const uintptr_t a = (uintptr_t)r[i].p, b = (uintptr_t)r[j].p;
            if (r[i].bytes && r[j].bytes && a < b + r[j].bytes && b < a + r[i].bytes)
                return set_error(SHTN_EINVAL, std::string(r[i].what) + " overlaps " + r[j].what);
        }
    return SHTN_OK;
}

// Device memory the plan reads during a transform: its uploaded image and,
// when built, its stored-P table.
void plan_ranges(const Plan& p, std::vector<Range>& r)
{
    r.push_back({"the plan's device buffer", p.dev, p.image.size(), false});
    if (p.ptab.dev)
        r.push_back({"the plan's stored-P buffer", p.ptab.dev,
                     p.ptab.head_bytes + (size_t)p.ptab.nblocks * 256 * sizeof(double), false});
}

int rows_per_block(const Plan& p)
{
    // rows of K points that fill one FFT workgroup (4096 points)
    const int cap = fft_rows_cap(p.K);
    int r = p.tiling.fft_rows > 0 ? p.tiling.fft_rows : cap;
    if (r > cap) r = cap;
    if (r > p.nlat) r = p.nlat;
    return r;
}
}  // namespace shtn

namespace {
int fail(int code, const std::string& msg) { return set_error(code, msg); }
int hip_fail(int e, const char* where) { return hip_error(e, where); }

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

const DevPlan* dplan(const Plan& p) { return (const DevPlan*)p.dev; }
const int* dev_table_int(const Plan& p, int t) { return (const int*)((char*)p.dev + p.table_off[t]); }

size_t data_bytes(const Plan& p, Data k, int nfields)
{
    return k == Data::spec ? (size_t)nfields * (size_t)p.nlm * 16 : (size_t)nfields * (size_t)p.nlat * (size_t)p.nphi * 8;
}


// A scalar call reading nfields fields of kind kin at `in` and writing
// fields of kind kout at `out`, with the workspace at `work`.
int check_call(shtn_plan_t plan, const void* in, Data kin, const void* out, Data kout, int nfields, const void* work)
{
    if (!plan || !plan->p) return fail(SHTN_EINVAL, "null plan");
    if (nfields < 1 || nfields > SHTN_MAX_FIELDS)
        return fail(SHTN_EINVAL, "nfields must be in [1, SHTN_MAX_FIELDS = 65535]: split the call");
    if (!plan->p->uploaded) return fail(SHTN_ESTATE, "plan not uploaded (call shtn_plan_upload)");
    if (!in || !out || !work) return fail(SHTN_EINVAL, "null data or workspace pointer");
    const Plan& p = *plan->p;
    std::vector<Range> r{{"the input", in, data_bytes(p, kin, nfields), false},
                         {"the output", out, data_bytes(p, kout, nfields), true},
                         {"the workspace", work, work_layout(p, nfields).total, true}};
    plan_ranges(p, r);
    return check_disjoint(r);
}

// Which passes of an algorithm choice read the stored table.
bool stored_synth(int algo) { return algo == SHTN_ALGO_STORED || algo == SHTN_ALGO_STORED_SYNTH; }
bool stored_analys(int algo) { return algo == SHTN_ALGO_STORED || algo == SHTN_ALGO_STORED_ANALYS; }

// Stored-P kernel arguments; ESTATE when the plan has no current table.
int sp_args(const Plan& p, const double* in, double* out, int nfields, int adjoint, PtabArgs& a)
{
    if (!p.ptab.built) return fail(SHTN_ESTATE, "stored-P table not built for the current plan (shtn_ptable_build)");
    a = PtabArgs{dplan(p), (const long*)p.ptab.dev, (const double*)((char*)p.ptab.dev + p.ptab.head_bytes),
                 in, out, nfields, adjoint, p.ptab.npt, 0};
    return SHTN_OK;
}

// Legendre synthesis-type stage (synthesis or adjoint of the analysis):
// spectra Q -> longitude coefficients F.  Qs is the scratch of the rescaled
// spectra (on-the-fly algorithm), nfields x nlm complex plus padding.
int leg_to_f(const Plan& p, const double* Q, double* F, double* Qs, int nfields, int adjoint, void* stream)
{
    int e;
    if (stored_synth(p.algo)) {
        PtabArgs a;
        int rc = sp_args(p, Q, F, nfields, adjoint, a);
        if (rc) return rc;
        {
            ProfScope ps(PK_LEG_SYNTH, stream);
            e = launch_sp_synth(a, p.M, p.ptab.synth_rt, p.ptab.synth_ct, stream);
        }
        if (e) return hip_fail(e, "stored-P synthesis launch");
        return SHTN_OK;
    }
    {
        ProfScope ps(PK_PRESCALE, stream);
        e = launch_prescale(dplan(p), nullptr, nullptr, nullptr, Q, Qs, p.nlm, nfields, stream);
    }
    if (e) return hip_fail(e, "prescale launch");
    LegLaunch l{};
    l.plans = dplan(p);
    l.units = dev_table_int(p, TB_SYNTH_UNITS);
    l.nunits = (int)(p.synth_units.size() / kUnitInts);
    l.grid_y = (nfields + p.tiling.fw - 1) / p.tiling.fw;
    l.in = Qs;
    l.out = F;
    l.nfields = nfields;
    l.adjoint = adjoint;
    l.lp = p.tiling.synth_lp;
    l.fw = p.tiling.fw;
    l.wpg = p.synth_wpg;
    {
        ProfScope ps(PK_LEG_SYNTH, stream);
        e = launch_legendre_synth(l, stream);
    }
    if (e) return hip_fail(e, "legendre synthesis launch");
    return SHTN_OK;
}

FftLaunch fft_launch(const Plan& p, const double* in, double* out, int nfields, double scale)
{
    FftLaunch f{};
    f.plans = dplan(p);
    f.rows_per_block = rows_per_block(p);
    f.nblocks = (p.nlat + f.rows_per_block - 1) / f.rows_per_block;
    f.points = f.rows_per_block * p.K;
    f.grid_y = nfields;
    f.K = p.K;
    f.uniform_k = 1;
    f.in = in;
    f.out = out;
    f.nfields = nfields;
    f.scale = scale;
    return f;
}

// Longitude synthesis: F -> grid (c2r).
int f_to_grid(const Plan& p, const double* F, double* grid, int nfields, void* stream)
{
    int e;
    {
        ProfScope ps(PK_C2R, stream);
        e = launch_c2r(fft_launch(p, F, grid, nfields, 1.0), stream);
    }
    return e ? hip_fail(e, "c2r launch") : SHTN_OK;
}

// Longitude analysis: grid -> F (r2c), F scaled by `scale`.
int grid_to_f(const Plan& p, const double* grid, double* F, int nfields, double scale, void* stream)
{
    int e;
    {
        ProfScope ps(PK_R2C, stream);
        e = launch_r2c(fft_launch(p, grid, F, nfields, scale), stream);
    }
    return e ? hip_fail(e, "r2c launch") : SHTN_OK;
}

// Checks that the analysis-type stage can run with the plan's algorithm.
int check_analys_stage(const Plan& p)
{
    if (!stored_analys(p.algo) && p.npair > kMaxAnalysPairs)
        return fail(SHTN_EUNSUPPORTED, "on-the-fly analysis supports at most 4096 latitudes");
    if (stored_analys(p.algo) && !p.ptab.built)
        return fail(SHTN_ESTATE, "stored-P table not built for the current plan (shtn_ptable_build)");
    return SHTN_OK;
}

// Legendre analysis-type stage (analysis or adjoint of the synthesis): F -> Q.
int f_to_leg(const Plan& p, const double* F, double* Q, int nfields, int adjoint, void* stream)
{
    int e;
    if (stored_analys(p.algo)) {
        PtabArgs a;
        int rc = sp_args(p, F, Q, nfields, adjoint, a);
        if (rc) return rc;
        const int nbr_max = ((p.L + 2) / 2 + 15) / 16;  // block rows of order 0, even parity
        {
            ProfScope ps(PK_LEG_ANALYS, stream);
            e = launch_sp_analys(a, p.M, nbr_max, p.ptab.analys_jt, p.ptab.analys_ct, stream);
        }
        if (e) return hip_fail(e, "stored-P analysis launch");
        return SHTN_OK;
    }
    LegLaunch l{};
    l.plans = dplan(p);
    l.units = dev_table_int(p, TB_ANALYS_UNITS);
    l.nunits = (int)(p.analys_units.size() / kUnitInts);
    l.lp = p.tiling.analys_lp;
    l.waves = p.tiling.analys_waves;
    l.fw = analys_fw(p.tiling.fw, l.lp, l.waves);
    l.grid_y = (nfields + l.fw - 1) / l.fw;
    l.in = F;
    l.out = Q;
    l.nfields = nfields;
    l.adjoint = adjoint;
    {
        ProfScope ps(PK_LEG_ANALYS, stream);
        e = launch_legendre_analys(l, stream);
    }
    if (e) return hip_fail(e, "legendre analysis launch");
    return SHTN_OK;
}

// Workspace of the vector transforms of nfields fields: F of the four scalar
// passes, F of the two components, the four spectra, the rescaled spectra.
struct VecLayout {
    size_t f4, fv, q4, qs, total;
};
VecLayout vec_layout(const Plan& p, int nfields)
{
    const size_t fs = (size_t)f_layout(p.M, p.nlat).size * 16;
    VecLayout v;
    v.f4 = 0;
    v.fv = v.f4 + align256(4 * (size_t)nfields * fs);
    v.q4 = v.fv + align256(2 * (size_t)nfields * fs);
    v.qs = v.q4 + align256(4 * (size_t)nfields * p.nlm * 16);
    v.total = v.qs + align256((4 * (size_t)nfields * p.nlm + kTablePad) * 16);
    return v;
}

// A vector call reading nfields fields of kind kin at a and b and writing
// fields of kind kout at c and d, with the workspace at `work`.
int check_vec_call(shtn_plan_t plan, const void* a, const void* b, Data kin, const void* c, const void* d, Data kout,
                   int nfields, const void* work)
{
    if (!plan || !plan->p) return fail(SHTN_EINVAL, "null plan");
    if (nfields < 1 || nfields > SHTN_MAX_VEC_FIELDS)
        return fail(SHTN_EINVAL, "nfields must be in [1, SHTN_MAX_VEC_FIELDS = 16383]: split the call");
    if (!plan->p->uploaded) return fail(SHTN_ESTATE, "plan not uploaded (call shtn_plan_upload)");
    if (!a || !b || !c || !d || !work) return fail(SHTN_EINVAL, "null data or workspace pointer");
    const Plan& p = *plan->p;
    const size_t ni = data_bytes(p, kin, nfields), no = data_bytes(p, kout, nfields);
    std::vector<Range> r{{"the first input", a, ni, false},
                         {"the second input", b, ni, false},
                         {"the first output", c, no, true},
                         {"the second output", d, no, true},
                         {"the workspace", work, vec_layout(p, nfields).total, true}};
    plan_ranges(p, r);
    return check_disjoint(r);
}

// Legendre synthesis-type pass (synthesis or adjoint of the analysis) then c2r.
int to_grid(shtn_plan_t plan, const double* Q, double* grid, int nfields, void* work, void* stream,
            int adjoint)
{
    int rc = check_call(plan, Q, Data::spec, grid, Data::grid, nfields, work);
    if (rc) return rc;
    const Plan& p = *plan->p;
    WorkLayout wl = work_layout(p, nfields);
    double* F = (double*)work;
    double* Qs = (double*)((char*)work + wl.f_bytes);
    if ((rc = leg_to_f(p, Q, F, Qs, nfields, adjoint, stream))) return rc;
    return f_to_grid(p, F, grid, nfields, stream);
}

// r2c then Legendre analysis-type pass (analysis or adjoint of the synthesis).
int to_spec(shtn_plan_t plan, const double* grid, double* Q, int nfields, void* work, void* stream,
            int adjoint)
{
    int rc = check_call(plan, grid, Data::grid, Q, Data::spec, nfields, work);
    if (rc) return rc;
    const Plan& p = *plan->p;
    if ((rc = check_analys_stage(p))) return rc;
    double* F = (double*)work;
    if ((rc = grid_to_f(p, grid, F, nfields, adjoint ? 1.0 : 2.0 * 3.14159265358979323846 / p.nphi, stream)))
        return rc;
    return f_to_leg(p, F, Q, nfields, adjoint, stream);
}

}  // namespace

namespace shtn {
// The synthesis call sequence on a workspace chosen by the caller (noalloc.hip).
int synth_on_work(shtn_plan_t plan, const double* Q, double* grid, int nfields, void* work, void* stream)
{
    return to_grid(plan, Q, grid, nfields, work, stream, 0);
}
}  // namespace shtn

extern "C" {

shtn_plan_t shtn_plan(int lmax, int mmax, int nlat, int nphi)
{
    try {
        if (nphi >= 1 && !is_pow2(nphi)) {
            g_detail = "nphi must be a power of two";
            return nullptr;
        }
        if (nphi < 2) {
            g_detail = "nphi must be >= 2";
            return nullptr;
        }
        if (nphi > 8192) {
            g_detail = "nphi > 8192 is not supported";
            return nullptr;
        }
        if (lmax > 8191) {
            g_detail = "lmax > 8191 is not supported";
            return nullptr;
        }
        std::string err;
        Plan* p = build_plan(lmax, mmax, nlat, nphi, err);
        if (!p) {
            g_detail = err;
            return nullptr;
        }
        shtn_plan_s* h = new shtn_plan_s;
        h->p = p;
        return h;
    } catch (const std::bad_alloc&) {
        g_detail = "out of host memory";
        return nullptr;
    } catch (...) {
        g_detail = "internal error";
        return nullptr;
    }
}

void shtn_plan_destroy(shtn_plan_t plan)
{
    if (!plan) return;
    delete plan->p;
    delete plan;
}

size_t shtn_plan_device_bytes(shtn_plan_t plan)
{
    if (!plan || !plan->p) return 0;
    return plan->p->image.size();
}

int shtn_plan_upload(shtn_plan_t plan, void* dev_buf, void* stream)
{
    if (!plan || !plan->p) return fail(SHTN_EINVAL, "null plan");
    if (!dev_buf) return fail(SHTN_EINVAL, "null device buffer");
    if ((uintptr_t)dev_buf % 256) return fail(SHTN_EINVAL, "device buffer must be 256-byte aligned");
    Plan& p = *plan->p;
    char* base = (char*)dev_buf;
    DevPlan d{};
    auto at = [&](int tb) { return (const void*)(base + p.table_off[tb]); };
    d.xp = (const double*)at(TB_XP);
    d.wq = (const double*)at(TB_WQ);
    d.wfull = (const double*)at(TB_WFULL);
    d.beta = (const double*)at(TB_BETA);
    d.gamma = (const double*)at(TB_GAMMA);
    d.inj_j = (const int*)at(TB_INJ_J);
    d.inj_y = (const double*)at(TB_INJ_Y);
    d.segexp = (const int*)at(TB_SEGEXP);
    d.segoff = (const int*)at(TB_SEGOFF);
    d.rst_y = (const double*)at(TB_RST_Y);
    d.tw = (const double*)at(TB_TW);
    d.rtw = (const double*)at(TB_RTW);
    d.synth_units = (const int*)at(TB_SYNTH_UNITS);
    d.analys_units = (const int*)at(TB_ANALYS_UNITS);
    d.ck_mask = (const unsigned*)at(TB_CK_MASK);
    d.nblk = p.nblk;
    d.nck = p.nck;
    d.L = p.L;
    d.M = p.M;
    d.nlat = p.nlat;
    d.nphi = p.nphi;
    d.npair = p.npair;
    d.K = p.K;
    d.nlm = p.nlm;
    d.n_synth_units = (int)(p.synth_units.size() / kUnitInts);
    d.n_analys_units = (int)(p.analys_units.size() / kUnitInts);
    d.synth_lp = p.tiling.synth_lp;
    d.analys_lp = p.tiling.analys_lp;
    d.fw = p.tiling.fw;
    const FLayout fl = f_layout(p.M, p.nlat);
    d.f_ts = fl.ts;
    d.f_size = fl.size;
    std::memcpy(p.image.data(), &d, sizeof(DevPlan));
    hipError_t e = hipMemcpyAsync(dev_buf, p.image.data(), p.image.size(), hipMemcpyHostToDevice,
                                  (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail((int)e, "plan upload copy");
    e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail((int)e, "plan upload sync");
    p.dev = dev_buf;
    p.uploaded = true;
    p.gen++;
    return SHTN_OK;
}

size_t shtn_work_bytes(shtn_plan_t plan, int nfields)
{
    if (!plan || !plan->p || nfields < 1) return 0;
    return work_layout(*plan->p, nfields).total;
}

int shtn_synth(shtn_plan_t plan, const double* Q, double* grid, int nfields, void* work, void* stream)
{
    return to_grid(plan, Q, grid, nfields, work, stream, 0);
}

int shtn_analys_adj(shtn_plan_t plan, const double* Q, double* grid, int nfields, void* work,
                    void* stream)
{
    return to_grid(plan, Q, grid, nfields, work, stream, 1);
}

int shtn_analys(shtn_plan_t plan, const double* grid, double* Q, int nfields, void* work, void* stream)
{
    return to_spec(plan, grid, Q, nfields, work, stream, 0);
}

int shtn_synth_adj(shtn_plan_t plan, const double* grid, double* Q, int nfields, void* work,
                   void* stream)
{
    return to_spec(plan, grid, Q, nfields, work, stream, 1);
}

long shtn_nlm(shtn_plan_t plan)
{
    if (!plan || !plan->p) return fail(SHTN_EINVAL, "null plan");
    return plan->p->nlm;
}

long shtn_lm_index(shtn_plan_t plan, int n, int m)
{
    if (!plan || !plan->p) return -1;
    const Plan& p = *plan->p;
    if (m < 0 || m > p.M || n < m || n > p.L) return -1;
    return lm_index(p.L, n, m);
}

int shtn_get_grid(shtn_plan_t plan, double* x_host, double* w_host)
{
    if (!plan || !plan->p) return fail(SHTN_EINVAL, "null plan");
    const Plan& p = *plan->p;
    if (x_host) std::memcpy(x_host, p.x.data(), sizeof(double) * p.nlat);
    if (w_host) std::memcpy(w_host, p.w.data(), sizeof(double) * p.nlat);
    return SHTN_OK;
}

double shtn_legendre_flops(shtn_plan_t plan)
{
    if (!plan || !plan->p) return 0.0;
    return 8.0 * (double)plan->p->npair * (double)plan->p->nlm;
}

long shtn_plan_table(shtn_plan_t plan, int which, void* dst, size_t bytes)
{
    if (!plan || !plan->p) return fail(SHTN_EINVAL, "null plan");
    const Plan& p = *plan->p;
    const void* src = nullptr;
    size_t n = 0;
    int tiling[9] = {p.tiling.synth_lp, p.tiling.analys_lp, p.tiling.fw, p.tiling.m_pairing,
                     p.split_used, rows_per_block(p), p.tiling.analys_waves, kInject, p.polar_log2};
    switch (which) {
    case 0: src = p.xp.data(); n = p.xp.size() * 8; break;
    case 1: src = p.sp.data(); n = p.sp.size() * 8; break;
    case 2: src = p.wq.data(); n = p.wq.size() * 8; break;
    case 3: src = p.beta.data(); n = p.beta.size() * 8; break;
    case 4: src = p.gamma.data(); n = p.gamma.size() * 8; break;
    case 5: src = p.start_y.data(); n = p.start_y.size() * 8; break;
    case 6: src = p.start_k.data(); n = p.start_k.size() * 4; break;
    case 7: src = p.segexp.data(); n = p.segexp.size() * 4; break;
    case 8: src = p.segoff.data(); n = p.segoff.size() * 4; break;
    case 9: src = p.rst_y.data(); n = p.rst_y.size() * 8; break;
    case 10: src = nullptr; n = 0; break;  // no longer used (restart states carry no exponent)
    case 11: src = p.analys_units.data(); n = p.analys_units.size() * 4; break;
    case 12: src = p.synth_units.data(); n = p.synth_units.size() * 4; break;
    case 13: src = tiling; n = sizeof(tiling); break;
    case 14: src = p.first_pair.data(); n = p.first_pair.size() * 4; break;
    case 15: src = p.inj_j.data(); n = p.inj_j.size() * 4; break;
    case 16: src = p.inj_y.data(); n = p.inj_y.size() * 8; break;
    case 17: src = p.blk_first.data(); n = p.blk_first.size() * 4; break;
    case 18: src = p.ck_mask.data(); n = p.ck_mask.size() * 4; break;
    default: return fail(SHTN_EINVAL, "unknown table");
    }
    if (dst && bytes >= n && n) std::memcpy(dst, src, n);
    return (long)n;
}

int shtn_plan_set_tiling(shtn_plan_t plan, int synth_lp, int analys_lp, int analys_waves, int fw,
                         int m_pairing, int split, int fft_rows)
{
    if (!plan || !plan->p) return fail(SHTN_EINVAL, "null plan");
    Plan& p = *plan->p;
    auto okl = [](int v) { return v == 1 || v == 2 || v == 4 || v == 8; };
    if (!okl(synth_lp) || !okl(analys_lp)) return fail(SHTN_EINVAL, "lp must be 1, 2, 4 or 8");
    if (synth_lp > 4) return fail(SHTN_EINVAL, "synth_lp must be 1, 2 or 4");
    if (!(analys_waves == 1 || analys_waves == 2 || analys_waves == 4))
        return fail(SHTN_EINVAL, "analys_waves must be 1, 2 or 4");
    // analysis kernels built: waves 1 (lp 1-8), 2 (lp 2-8), 4 (lp 4, 8); the
    // analysis takes analys_fw(fw, lp, waves) fields per wave
    if ((analys_waves == 2 && analys_lp < 2) || (analys_waves == 4 && analys_lp < 4))
        return fail(SHTN_EINVAL, "analys_lp too small for analys_waves");
    if (!(fw == 1 || fw == 2 || fw == 4)) return fail(SHTN_EINVAL, "fw must be 1, 2 or 4");
    if (fw == 4 && synth_lp > 2) return fail(SHTN_EINVAL, "fw=4 needs synth_lp <= 2");
    if (64 * analys_lp * analys_waves < p.npair && p.npair <= kMaxAnalysPairs)
        return fail(SHTN_EINVAL, "analysis unit too small: 64 analys_lp analys_waves must cover all latitude pairs");
    if (m_pairing < 0 || m_pairing > 1) return fail(SHTN_EINVAL, "m_pairing must be 0 or 1");
    if (split < 0 || split % kSegLen) return fail(SHTN_EINVAL, "split must be a multiple of 32");
    if (fft_rows < 0) return fail(SHTN_EINVAL, "fft_rows must be >= 0");
    Tiling old = p.tiling;
    p.tiling.synth_lp = synth_lp;
    p.tiling.analys_lp = analys_lp;
    p.tiling.analys_waves = analys_waves;
    p.tiling.fw = fw;
    p.tiling.m_pairing = m_pairing;
    p.tiling.split = split;
    p.tiling.fft_rows = fft_rows;
    std::string err;
    if (rebuild_units(p, err)) {
        p.tiling = old;
        rebuild_units(p, err);
        build_image(p);
        return fail(SHTN_EINVAL, err);
    }
    build_image(p);
    p.uploaded = false;
    p.dev = nullptr;
    p.gen++;
    return SHTN_OK;
}

int shtn_plan_set_polar(shtn_plan_t plan, int log2_threshold)
{
    if (!plan || !plan->p) return fail(SHTN_EINVAL, "null plan");
    if (log2_threshold < -1000 || log2_threshold > -1)
        return fail(SHTN_EINVAL, "polar threshold exponent must lie in [-1000, -1]");
    Plan& p = *plan->p;
    if (log2_threshold == p.polar_log2) return SHTN_OK;
    const int old = p.polar_log2;
    p.polar_log2 = log2_threshold;
    try {
        lane_starts(p);
    } catch (const std::bad_alloc&) {
        p.polar_log2 = old;
        lane_starts(p);
        return fail(SHTN_ENOMEM, "polar threshold: out of host memory");
    }
    // The stored start states must stay normal doubles: a denormal start has
    // lost bits, and the recurrence would carry that error to where P_n^m
    // grows to O(1).  How low a threshold keeps them normal depends on the
    // plan (about -900 at lmax 1023).
    const double lo = min_start_state(p);
    if (lo > 0.0 && lo < DBL_MIN) {
        p.polar_log2 = old;
        lane_starts(p);
        return fail(SHTN_EINVAL, "polar threshold too low for this plan: lane start states fall below the "
                                 "normal double range");
    }
    std::string err;
    if (rebuild_units(p, err)) {
        p.polar_log2 = old;
        lane_starts(p);
        rebuild_units(p, err);
        build_image(p);
        return fail(SHTN_EINVAL, err);
    }
    build_image(p);
    p.uploaded = false;
    p.dev = nullptr;
    p.ptab.built = false;  // the table follows the lane starts
    p.gen++;
    return SHTN_OK;
}

size_t shtn_vec_work_bytes(shtn_plan_t plan, int nfields)
{
    if (!plan || !plan->p || nfields < 1) return 0;
    return vec_layout(*plan->p, nfields).total;
}

}  // extern "C"

namespace {
// Vector synthesis-type sequence: spectra (S, T) -> grids (Vt, Vp).  adjoint:
// the adjoint of the vector analysis ((S, T) / n(n+1), scalar stages in
// their adjoint mode).
int vec_to_grid(shtn_plan_t plan, const double* S, const double* T, double* Vt, double* Vp, int nfields,
                void* work, void* stream, int adjoint)
{
    int rc = check_vec_call(plan, S, T, Data::spec, Vt, Vp, Data::grid, nfields, work);
    if (rc) return rc;
    const Plan& p = *plan->p;
    const VecLayout v = vec_layout(p, nfields);
    char* w = (char*)work;
    double* F4 = (double*)(w + v.f4);
    double* Fv = (double*)(w + v.fv);
    double* Q4 = (double*)(w + v.q4);
    double* Qs = (double*)(w + v.qs);
    const long fs = f_layout(p.M, p.nlat).size;
    int e = launch_vec_spec_in(dplan(p), p.L, p.M, S, T, Q4, nfields, adjoint, stream);
    if (e) return hip_fail(e, "vector spectra launch");
    if ((rc = leg_to_f(p, Q4, F4, Qs, 4 * nfields, adjoint, stream))) return rc;
    if ((e = launch_vec_f_out(dplan(p), fs, F4, Fv, nfields, stream))) return hip_fail(e, "vector combine launch");
    if ((rc = f_to_grid(p, Fv, Vt, nfields, stream))) return rc;
    return f_to_grid(p, Fv + 2 * (size_t)nfields * fs, Vp, nfields, stream);
}

// Vector analysis-type sequence: grids (Vt, Vp) -> spectra (S, T).  adjoint:
// the adjoint of the vector synthesis (unnormalised DFT, scalar stages in
// their adjoint mode, no division by n(n+1)).
int vec_to_spec(shtn_plan_t plan, const double* Vt, const double* Vp, double* S, double* T, int nfields,
                void* work, void* stream, int adjoint)
{
    int rc = check_vec_call(plan, Vt, Vp, Data::grid, S, T, Data::spec, nfields, work);
    if (rc) return rc;
    const Plan& p = *plan->p;
    if ((rc = check_analys_stage(p))) return rc;
    const VecLayout v = vec_layout(p, nfields);
    char* w = (char*)work;
    double* F4 = (double*)(w + v.f4);
    double* Fv = (double*)(w + v.fv);
    double* Q4 = (double*)(w + v.q4);
    const long fs = f_layout(p.M, p.nlat).size;
    const double sc = adjoint ? 1.0 : 2.0 * 3.14159265358979323846 / p.nphi;
    if ((rc = grid_to_f(p, Vt, Fv, nfields, sc, stream))) return rc;
    if ((rc = grid_to_f(p, Vp, Fv + 2 * (size_t)nfields * fs, nfields, sc, stream))) return rc;
    int e = launch_vec_f_in(dplan(p), fs, Fv, F4, nfields, stream);
    if (e) return hip_fail(e, "vector weights launch");
    if ((rc = f_to_leg(p, F4, Q4, 4 * nfields, adjoint, stream))) return rc;
    if ((e = launch_vec_spec_out(dplan(p), p.L, p.M, Q4, S, T, nfields, !adjoint, stream)))
        return hip_fail(e, "vector spectra launch");
    return SHTN_OK;
}
}  // namespace

extern "C" {

int shtn_vec_synth(shtn_plan_t plan, const double* S, const double* T, double* Vt, double* Vp, int nfields,
                   void* work, void* stream)
{
    return vec_to_grid(plan, S, T, Vt, Vp, nfields, work, stream, 0);
}

int shtn_vec_analys(shtn_plan_t plan, const double* Vt, const double* Vp, double* S, double* T, int nfields,
                    void* work, void* stream)
{
    return vec_to_spec(plan, Vt, Vp, S, T, nfields, work, stream, 0);
}

int shtn_vec_synth_adj(shtn_plan_t plan, const double* Vt, const double* Vp, double* S, double* T, int nfields,
                       void* work, void* stream)
{
    return vec_to_spec(plan, Vt, Vp, S, T, nfields, work, stream, 1);
}

int shtn_vec_analys_adj(shtn_plan_t plan, const double* S, const double* T, double* Vt, double* Vp, int nfields,
                        void* work, void* stream)
{
    return vec_to_grid(plan, S, T, Vt, Vp, nfields, work, stream, 1);
}

long shtn_ptable_bytes(shtn_plan_t plan)
{
    if (!plan || !plan->p) return fail(SHTN_EINVAL, "null plan");
    const PTable& t = plan->p->ptab;
    return (long)(t.head_bytes + (size_t)t.nblocks * 256 * sizeof(double));
}

int shtn_ptable_build(shtn_plan_t plan, void* dev_buf, size_t bytes, void* stream)
{
    if (!plan || !plan->p) return fail(SHTN_EINVAL, "null plan");
    Plan& p = *plan->p;
    if (!p.uploaded) return fail(SHTN_ESTATE, "plan not uploaded (call shtn_plan_upload)");
    if (!dev_buf) return fail(SHTN_EINVAL, "null device buffer");
    if ((uintptr_t)dev_buf % 256) return fail(SHTN_EINVAL, "device buffer must be 256-byte aligned");
    const size_t need = p.ptab.head_bytes + (size_t)p.ptab.nblocks * 256 * sizeof(double);
    if (bytes < need) return fail(SHTN_EINVAL, "stored-P buffer smaller than shtn_ptable_bytes");
    p.ptab.built = false;
    p.gen++;
    hipError_t e = hipMemcpyAsync(dev_buf, p.ptab.boff.data(), p.ptab.boff.size() * sizeof(long),
                                  hipMemcpyHostToDevice, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail((int)e, "stored-P offsets copy");
    const int k = launch_ptable_build(dplan(p), (const long*)dev_buf,
                                      (double*)((char*)dev_buf + p.ptab.head_bytes), p.ptab.npt, p.M, stream);
    if (k) return hip_fail(k, "stored-P build launch");
    e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail((int)e, "stored-P build sync");
    p.ptab.dev = dev_buf;
    p.ptab.built = true;
    p.gen++;
    return SHTN_OK;
}

int shtn_ptable_release(shtn_plan_t plan)
{
    if (!plan || !plan->p) return fail(SHTN_EINVAL, "null plan");
    plan->p->ptab.dev = nullptr;
    plan->p->ptab.built = false;
    plan->p->algo = SHTN_ALGO_ONTHEFLY;
    plan->p->gen++;
    return SHTN_OK;
}

int shtn_ptable_set_tiling(shtn_plan_t plan, int synth_rt, int synth_ct, int analys_jt, int analys_ct)
{
    if (!plan || !plan->p) return fail(SHTN_EINVAL, "null plan");
    auto ok_t = [](int v) { return v == 1 || v == 2 || v == 4; };
    auto ok_c = [](int v) { return v == 1 || v == 2; };
    if (!ok_t(synth_rt) || !ok_t(analys_jt)) return fail(SHTN_EINVAL, "synth_rt and analys_jt must be 1, 2 or 4");
    if (!ok_c(synth_ct) || !ok_c(analys_ct)) return fail(SHTN_EINVAL, "synth_ct and analys_ct must be 1 or 2");
    PTable& t = plan->p->ptab;
    t.synth_rt = synth_rt;
    t.synth_ct = synth_ct;
    t.analys_jt = analys_jt;
    t.analys_ct = analys_ct;
    return SHTN_OK;
}

int shtn_ptable_get_tiling(shtn_plan_t plan, int* tiling4)
{
    if (!plan || !plan->p || !tiling4) return fail(SHTN_EINVAL, "null plan or output");
    const PTable& t = plan->p->ptab;
    tiling4[0] = t.synth_rt;
    tiling4[1] = t.synth_ct;
    tiling4[2] = t.analys_jt;
    tiling4[3] = t.analys_ct;
    return SHTN_OK;
}

int shtn_plan_set_algorithm(shtn_plan_t plan, int algo)
{
    if (!plan || !plan->p) return fail(SHTN_EINVAL, "null plan");
    if (algo < SHTN_ALGO_ONTHEFLY || algo > SHTN_ALGO_STORED_ANALYS)
        return fail(SHTN_EINVAL, "algorithm must be one of SHTN_ALGO_*");
    if (algo != SHTN_ALGO_ONTHEFLY && !plan->p->ptab.built)
        return fail(SHTN_ESTATE, "stored-P table not built for the current plan (shtn_ptable_build)");
    plan->p->algo = algo;
    return SHTN_OK;
}

int shtn_plan_get_algorithm(shtn_plan_t plan)
{
    if (!plan || !plan->p) return fail(SHTN_EINVAL, "null plan");
    return plan->p->algo;
}

int shtn_plan_tune_algorithm(shtn_plan_t plan, const double* Q, double* grid, double* Qout, int nfields,
                             void* work, void* stream, int reps, float* us4)
{
    int rc = check_call(plan, Q, Data::spec, grid, Data::grid, nfields, work);
    if (rc) return rc;
    if (!Qout) return fail(SHTN_EINVAL, "null Qout");
    if ((rc = check_call(plan, grid, Data::grid, Qout, Data::spec, nfields, work))) return rc;
    {
        const size_t sb = data_bytes(*plan->p, Data::spec, nfields);
        if ((rc = check_disjoint({{"Q", Q, sb, false}, {"Qout", Qout, sb, true}}))) return rc;
    }
    if (reps < 1) reps = 5;
    Plan& p = *plan->p;
    const int keep = p.algo;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            for (auto& f : ev)
                if (f) (void)hipEventDestroy(f);
            return hip_fail((int)hipGetLastError(), "tuner events");
        }
    // t[pass][algo]: mean synthesis (pass 0) and analysis (pass 1) times
    float t[2][2] = {{-1.f, -1.f}, {-1.f, -1.f}};
    hipStream_t st = (hipStream_t)stream;
    for (int algo = 0; algo < 2 && !rc; algo++) {
        if (algo == 1 && !p.ptab.built) break;
        p.algo = algo;
        // one untimed round trip, then reps synthesis calls and reps analysis calls
        rc = to_grid(plan, Q, grid, nfields, work, stream, 0);
        if (!rc) rc = to_spec(plan, grid, Qout, nfields, work, stream, 0);
        if (!rc && hipEventRecord(ev[0], st) != hipSuccess) rc = hip_fail((int)hipGetLastError(), "tuner event");
        for (int r = 0; r < reps && !rc; r++) rc = to_grid(plan, Q, grid, nfields, work, stream, 0);
        if (!rc && hipEventRecord(ev[1], st) != hipSuccess) rc = hip_fail((int)hipGetLastError(), "tuner event");
        for (int r = 0; r < reps && !rc; r++) rc = to_spec(plan, grid, Qout, nfields, work, stream, 0);
        if (!rc && hipEventRecord(ev[2], st) != hipSuccess) rc = hip_fail((int)hipGetLastError(), "tuner event");
        if (!rc && hipEventSynchronize(ev[2]) != hipSuccess) rc = hip_fail((int)hipGetLastError(), "tuner sync");
        float ms0 = 0.f, ms1 = 0.f;
        if (!rc && (hipEventElapsedTime(&ms0, ev[0], ev[1]) != hipSuccess ||
                    hipEventElapsedTime(&ms1, ev[1], ev[2]) != hipSuccess))
            rc = hip_fail((int)hipGetLastError(), "tuner elapsed time");
        if (!rc) {
            t[0][algo] = 1e3f * ms0 / reps;
            t[1][algo] = 1e3f * ms1 / reps;
        }
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    if (rc) {
        p.algo = keep;
        return rc;
    }
    const bool ss = t[0][1] >= 0.f && t[0][1] < t[0][0];
    const bool sa = t[1][1] >= 0.f && t[1][1] < t[1][0];
    p.algo = ss ? (sa ? SHTN_ALGO_STORED : SHTN_ALGO_STORED_SYNTH) : (sa ? SHTN_ALGO_STORED_ANALYS : SHTN_ALGO_ONTHEFLY);
    if (us4) {
        us4[0] = t[0][0];
        us4[1] = t[0][1];
        us4[2] = t[1][0];
        us4[3] = t[1][1];
    }
    return SHTN_OK;
}


const char* shtn_strerror(int code)
{
    switch (code) {
    case SHTN_OK: return "success";
    case SHTN_EINVAL: return "invalid argument";
    case SHTN_EUNSUPPORTED: return "unsupported configuration";
    case SHTN_ESTATE: return "plan not uploaded";
    case SHTN_EHIP: return "HIP runtime error";
    case SHTN_ENOMEM: return "out of host memory";
    default: return "unknown error";
    }
}

const char* shtn_last_error_detail(void) { return g_detail.c_str(); }

}  // extern "C"
