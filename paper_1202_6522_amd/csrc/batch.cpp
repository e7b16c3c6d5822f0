// Batches of fields with different truncations (include/shtn.h, shtn_batch_*):
// every stage of a batched transform is one launch over all fields (the
// analysis stage one launch per pairs-per-lane class), optionally captured in
// a hipGraph, with the tiling chosen by a timing autotuner.
//
// Work units of all fields go into one list per stage.  A unit names its
// field slot and its plan, so one launch serves fields of any truncation; the
// per-plan tables (recurrence coefficients, start values, restart states,
// twiddles) stay in the plans' own device buffers and are reached through a
// copy of each plan's device descriptor.  Units are ordered longest first so
// the tail of a launch is made of short units (the greedy longest-processing-
// time order of the paper's work split over threads, Sec. 3.3, applied to
// waves).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <array>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "shtn.h"
#include "shtn_internal.h"
#include "shtn_profile.h"

using namespace shtn;

namespace {

struct BatchTiling {
    int synth_lp = 1;      // latitude pairs per synthesis lane (block of 64 lp pairs per wave)
    int fw = 1;            // fields per wave (fields of the same plan)
    int m_pairing = 0;     // synthesis unit order: 1 = long and short units alternate
    int analys_merge = 0;  // analysis: 1 = a single launch at the largest pairs-per-lane class
    int stored = 0;        // 1 = plans with a current stored-P table use the stored kernels
};

struct AnalysClass {
    int lp, waves, fw;
    size_t first;  // first unit (index into analys_units / kUnitInts)
    int count;
};

// analysis class of a plan: (pairs per lane, waves), encoded as lp * 16 + waves
int analys_class(int npair)
{
    int lp, w;
    analys_shape(npair, lp, w);
    return lp * 16 + w;
}

}  // namespace

struct shtn_batch_s {
    int nfields = 0;
    std::vector<shtn_plan_t> field_plan;  // per user field
    std::vector<Plan*> plans;             // distinct plans
    std::vector<int> slot_field;          // slot -> user field (slots grouped by plan)
    std::vector<int> slot_plan;           // slot -> distinct plan index
    std::vector<size_t> q_off, g_off;     // per user field (+ total), in doubles
    std::vector<long> slot_q, slot_g, slot_f, slot_s;  // per slot offsets in doubles
    size_t work_f_doubles = 0, work_total_bytes = 0;
    long max_nlm = 0;
    BatchTiling tiling;
    // unit tables of the current tiling
    std::vector<int> synth_units, analys_units, rowblocks;
    // plans whose slots run the stored-P kernels: {plan index, first slot, slots}
    std::vector<std::array<int, 3>> stored_runs;
    std::vector<AnalysClass> classes;
    int synth_wpg = 1;
    int fft_points = 1;  // most complex points in one FFT row block
    int fft_kmax = 1;  // longest FFT rows of the batch (sizes the FFT's LDS)
    // device image
    std::vector<unsigned char> image;
    size_t off_plans = 0, off_slot_plan = 0, off_q = 0, off_g = 0, off_f = 0, off_s = 0,
           off_su = 0, off_au = 0, off_rb = 0;
    size_t max_image = 0;
    void* dev = nullptr;
    bool uploaded = false;
    // generation of every distinct plan when the unit tables were built and
    // when the batch was uploaded (Plan::gen): a plan changed since either
    // makes the batch's copies stale
    std::vector<unsigned long> tables_gen, upload_gen;
    // captured graphs: 0 synthesis, 1 analysis
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t exec[2] = {nullptr, nullptr};
};

namespace {

size_t put_bytes(std::vector<unsigned char>& img, size_t off, const void* src, size_t bytes)
{
    if (img.size() < off + bytes) img.resize(off + bytes);
    if (bytes) std::memcpy(img.data() + off, src, bytes);
    return align256(off + bytes);
}

template <typename T>
size_t put_vec(std::vector<unsigned char>& img, size_t off, const std::vector<T>& v)
{
    return put_bytes(img, off, v.data(), v.size() * sizeof(T));
}

std::vector<unsigned long> plan_gens(const shtn_batch_s& b)
{
    std::vector<unsigned long> g;
    for (auto* p : b.plans) g.push_back(p->gen);
    return g;
}

// Builds the unit tables and the device image for tiling t.
void build_tables(shtn_batch_s& b, const BatchTiling& t)
{
    b.tables_gen = plan_gens(b);
    const int ns = (int)b.slot_field.size();
    // slot ranges per plan (slots of one plan are consecutive)
    std::vector<std::pair<int, int>> range(b.plans.size(), {ns, 0});
    for (int s = 0; s < ns; s++) {
        auto& r = range[b.slot_plan[s]];
        r.first = std::min(r.first, s);
        r.second = std::max(r.second, s + 1);
    }
    // plans served by the stored-P kernels: no on-the-fly units for their slots
    std::vector<char> stored(b.plans.size(), 0);
    b.stored_runs.clear();
    for (size_t pi = 0; pi < b.plans.size(); pi++)
        if (t.stored && b.plans[pi]->ptab.built && range[pi].first < range[pi].second) {
            stored[pi] = 1;
            b.stored_runs.push_back({(int)pi, range[pi].first, range[pi].second - range[pi].first});
        }

    // ---- synthesis units ----
    struct SU {
        long cost;
        int u[kUnitInts];
    };
    std::vector<SU> su;
    int maxblk = 1;
    for (size_t pi = 0; pi < b.plans.size(); pi++) {
        if (stored[pi]) continue;
        const Plan& p = *b.plans[pi];
        const int blk = 64 * t.synth_lp;
        const int nblk = (p.npair + blk - 1) / blk;
        maxblk = std::max(maxblk, nblk);
        for (int fg = range[pi].first; fg < range[pi].second; fg += t.fw) {
            const int nf = std::min(t.fw, range[pi].second - fg);
            for (int m = 0; m <= p.M; m++) {
                const int nj = p.L - m + 1;
                for (int k = 0; k < nblk; k++) {
                    int jmin, jmax;
                    SU x{0, {fg, nf, (int)pi, m, 0, 0, k * blk, 0, -1, 0, 0, 0}};
                    if (start_range(p, m, k * blk, std::min((k + 1) * blk, p.npair), 0, nj, jmin, jmax)) {
                        x.u[U_JS] = jmin;
                        x.u[U_JW] = jmax;
                        x.cost = (long)(nj - jmin) * t.synth_lp * nf;
                    } else {
                        x.u[U_ZERO] = 1;
                    }
                    su.push_back(x);
                }
            }
        }
    }
    // longest first; with m_pairing, long and short units alternate instead
    std::stable_sort(su.begin(), su.end(), [](const SU& a, const SU& c) { return a.cost > c.cost; });
    if (t.m_pairing) {
        std::vector<SU> alt;
        alt.reserve(su.size());
        for (size_t lo = 0, hi = su.size(); lo < hi;) {
            alt.push_back(su[lo++]);
            if (lo < hi) alt.push_back(su[--hi]);
        }
        su.swap(alt);
    }
    b.synth_units.clear();
    for (auto& x : su) b.synth_units.insert(b.synth_units.end(), x.u, x.u + kUnitInts);
    b.synth_wpg = std::min(t.synth_lp == 1 && t.fw == 1 ? 16 : 8, maxblk);

    // ---- analysis units, per (pairs per lane, waves) class ----
    int cls_max = 0, npair_max = 0;
    for (auto* p : b.plans)
        if (p->npair > npair_max) {
            npair_max = p->npair;
            cls_max = analys_class(p->npair);
        }
    std::vector<int> classes;
    if (t.analys_merge) {
        classes.push_back(cls_max);
    } else {
        for (auto* p : b.plans) {
            const int c = analys_class(p->npair);
            if (std::find(classes.begin(), classes.end(), c) == classes.end()) classes.push_back(c);
        }
        std::sort(classes.rbegin(), classes.rend());
    }
    b.analys_units.clear();
    b.classes.clear();
    for (int cl : classes) {
        const int lp = cl / 16, waves = cl % 16;
        const int fw = analys_fw(t.fw, lp, waves);
        std::vector<SU> au;
        for (size_t pi = 0; pi < b.plans.size(); pi++) {
            const Plan& p = *b.plans[pi];
            if (stored[pi]) continue;
            if (!t.analys_merge && analys_class(p.npair) != cl) continue;
            for (int fg = range[pi].first; fg < range[pi].second; fg += fw) {
                const int nf = std::min(fw, range[pi].second - fg);
                const size_t nu = p.analys_units.size() / kUnitInts;
                for (size_t i = 0; i < nu; i++) {
                    const int* pu = &p.analys_units[i * kUnitInts];
                    if (pu[U_M] < 0) continue;  // padding of the plan's XCD queues
                    SU x{(long)(pu[U_J1] - pu[U_JS] + 4) * nf, {}};
                    std::copy(pu, pu + kUnitInts, x.u);
                    x.u[U_FIELD] = fg;
                    x.u[U_NF] = nf;
                    x.u[U_PLAN] = (int)pi;
                    au.push_back(x);
                }
            }
        }
        std::stable_sort(au.begin(), au.end(), [](const SU& a, const SU& c) { return a.cost > c.cost; });
        AnalysClass c{lp, waves, fw, b.analys_units.size() / kUnitInts, (int)au.size()};
        for (auto& x : au) b.analys_units.insert(b.analys_units.end(), x.u, x.u + kUnitInts);
        b.classes.push_back(c);
    }

    // ---- FFT row blocks: {slot, plan, first row, rows} ----
    b.fft_kmax = 1;
    b.fft_points = 1;
    for (auto* p : b.plans) {
        b.fft_kmax = std::max(b.fft_kmax, p->K);
        b.fft_points = std::max(b.fft_points, rows_per_block(*p) * p->K);
    }
    b.rowblocks.clear();
    for (int s = 0; s < ns; s++) {
        const Plan& p = *b.plans[b.slot_plan[s]];
        const int rpb = rows_per_block(p);
        for (int r0 = 0; r0 < p.nlat; r0 += rpb) {
            int rb[4] = {s, b.slot_plan[s], r0, std::min(rpb, p.nlat - r0)};
            b.rowblocks.insert(b.rowblocks.end(), rb, rb + 4);
        }
    }

    // ---- device image ----
    b.image.clear();
    size_t off = 0;
    b.off_plans = off;
    off = align256(off + b.plans.size() * sizeof(DevPlan));
    b.image.resize(off, 0);
    b.off_slot_plan = off; off = put_vec(b.image, off, b.slot_plan);
    b.off_q = off; off = put_vec(b.image, off, b.slot_q);
    b.off_g = off; off = put_vec(b.image, off, b.slot_g);
    b.off_f = off; off = put_vec(b.image, off, b.slot_f);
    b.off_s = off; off = put_vec(b.image, off, b.slot_s);
    b.off_su = off; off = put_vec(b.image, off, b.synth_units);
    b.off_au = off; off = put_vec(b.image, off, b.analys_units);
    b.off_rb = off; off = put_vec(b.image, off, b.rowblocks);
    b.image.resize(off, 0);
}

template <typename T>
T* dev_at(const shtn_batch_s& b, size_t off)
{
    return (T*)((char*)b.dev + off);
}

void drop_graphs(shtn_batch_s& b)
{
    for (auto& e : b.exec) {
        if (e) (void)hipGraphExecDestroy(e);
        e = nullptr;
    }
}

size_t packed_bytes(const shtn_batch_s& b, Data k)
{
    return (k == Data::spec ? b.q_off.back() : b.g_off.back()) * sizeof(double);
}

// A batch call reading packed fields of kind kin at `in` and writing packed
// fields of kind kout at `out`, with the workspace at `work`.
// 1 if every plan of the batch has rows of the same length.
int uniform_k(const shtn_batch_s& b)
{
    for (const Plan* p : b.plans)
        if (p->K != b.fft_kmax) return 0;
    return 1;
}

int check_batch(const shtn_batch_s* b, const void* in, Data kin, const void* out, Data kout, const void* work)
{
    if (!b) return set_error(SHTN_EINVAL, "null batch");
    if (!b->uploaded) return set_error(SHTN_ESTATE, "batch not uploaded (call shtn_batch_upload)");
    if (!in || !out || !work) return set_error(SHTN_EINVAL, "null data or workspace pointer");
    for (auto* p : b->plans)
        if (!p->uploaded) return set_error(SHTN_ESTATE, "a plan of the batch is no longer uploaded");
    std::vector<Range> r{{"the input", in, packed_bytes(*b, kin), false},
                         {"the output", out, packed_bytes(*b, kout), true},
                         {"the batch's device buffer", b->dev, b->image.size(), false},
                         {"the workspace", work, b->work_total_bytes, true}};
    for (auto* p : b->plans) plan_ranges(*p, r);
    if (int rc = check_disjoint(r)) return rc;
    if (plan_gens(*b) != b->upload_gen)
        return set_error(SHTN_ESTATE, "a plan of the batch changed since the batch upload (upload, tiling, polar "
                                      "threshold or stored-P table): call shtn_batch_upload again");
    for (const auto& r : b->stored_runs)
        if (!b->plans[r[0]]->ptab.built)
            return set_error(SHTN_ESTATE, "a stored-P table of the batch is no longer current (set the algorithm again)");
    return SHTN_OK;
}

// Stored-P launches of the batch's stored plans (fields addressed through
// the per-slot offset tables).
int run_stored(const shtn_batch_s& b, const double* in, double* out, int synth, void* stream)
{
    const DevPlan* plans = dev_at<const DevPlan>(b, b.off_plans);
    for (const auto& r : b.stored_runs) {
        const Plan& p = *b.plans[r[0]];
        PtabArgs a{plans + r[0], (const long*)p.ptab.dev,
                   (const double*)((const char*)p.ptab.dev + p.ptab.head_bytes), in, out, r[2], 0, p.ptab.npt, 0};
        a.q_off = dev_at<const long>(b, b.off_q) + r[1];
        a.f_off = dev_at<const long>(b, b.off_f) + r[1];
        int e;
        if (synth) {
            ProfScope ps(PK_LEG_SYNTH, stream);
            e = launch_sp_synth(a, p.M, p.ptab.synth_rt, p.ptab.synth_ct, stream);
        } else {
            ProfScope ps(PK_LEG_ANALYS, stream);
            e = launch_sp_analys(a, p.M, ((p.L + 2) / 2 + 15) / 16, p.ptab.analys_jt, p.ptab.analys_ct, stream);
        }
        if (e) return hip_error(e, "batch stored-P launch");
    }
    return SHTN_OK;
}

int run_synth(const shtn_batch_s& b, const double* Q, double* grid, void* work, void* stream)
{
    const int ns = (int)b.slot_field.size();
    double* F = (double*)work;
    double* Qs = F + b.work_f_doubles;
    const DevPlan* plans = dev_at<const DevPlan>(b, b.off_plans);
    int e;
    {
        ProfScope ps(PK_PRESCALE, stream);
        e = launch_prescale(plans, dev_at<const long>(b, b.off_q), dev_at<const long>(b, b.off_s),
                            dev_at<const int>(b, b.off_slot_plan), Q, Qs, b.max_nlm, ns, stream);
    }
    if (e) return hip_error(e, "batch prescale launch");
    LegLaunch l{};
    l.plans = plans;
    l.units = dev_at<const int>(b, b.off_su);
    l.nunits = (int)(b.synth_units.size() / kUnitInts);
    l.grid_y = 1;
    l.q_off = dev_at<const long>(b, b.off_s);
    l.f_off = dev_at<const long>(b, b.off_f);
    l.in = Qs;
    l.out = F;
    l.nfields = ns;
    l.adjoint = 0;
    l.lp = b.tiling.synth_lp;
    l.fw = b.tiling.fw;
    l.wpg = b.synth_wpg;
    {
        ProfScope ps(PK_LEG_SYNTH, stream);
        e = launch_legendre_synth(l, stream);
    }
    if (e) return hip_error(e, "batch legendre synthesis launch");
    int rc = run_stored(b, Q, F, 1, stream);
    if (rc) return rc;
    FftLaunch f{};
    f.plans = plans;
    f.rowblocks = dev_at<const int>(b, b.off_rb);
    f.K = b.fft_kmax;
    f.uniform_k = uniform_k(b);
    f.points = b.fft_points;
    f.nblocks = (int)(b.rowblocks.size() / 4);
    f.grid_y = 1;
    f.g_off = dev_at<const long>(b, b.off_g);
    f.f_off = dev_at<const long>(b, b.off_f);
    f.in = F;
    f.out = grid;
    f.nfields = ns;
    f.scale = 1.0;
    {
        ProfScope ps(PK_C2R, stream);
        e = launch_c2r(f, stream);
    }
    if (e) return hip_error(e, "batch c2r launch");
    return SHTN_OK;
}

int run_analys(const shtn_batch_s& b, const double* grid, double* Q, void* work, void* stream)
{
    const int ns = (int)b.slot_field.size();
    double* F = (double*)work;
    const DevPlan* plans = dev_at<const DevPlan>(b, b.off_plans);
    FftLaunch f{};
    f.plans = plans;
    f.rowblocks = dev_at<const int>(b, b.off_rb);
    f.K = b.fft_kmax;
    f.uniform_k = uniform_k(b);
    f.points = b.fft_points;
    f.nblocks = (int)(b.rowblocks.size() / 4);
    f.grid_y = 1;
    f.g_off = dev_at<const long>(b, b.off_g);
    f.f_off = dev_at<const long>(b, b.off_f);
    f.in = grid;
    f.out = F;
    f.nfields = ns;
    f.scale = 0.0;  // each field's 2 pi / nphi
    int e;
    {
        ProfScope ps(PK_R2C, stream);
        e = launch_r2c(f, stream);
    }
    if (e) return hip_error(e, "batch r2c launch");
    for (const auto& c : b.classes) {
        LegLaunch l{};
        l.plans = plans;
        l.units = dev_at<const int>(b, b.off_au) + c.first * kUnitInts;
        l.nunits = c.count;
        l.grid_y = 1;
        l.q_off = dev_at<const long>(b, b.off_q);
        l.f_off = dev_at<const long>(b, b.off_f);
        l.in = F;
        l.out = Q;
        l.nfields = ns;
        l.adjoint = 0;
        l.lp = c.lp;
        l.waves = c.waves;
        l.fw = c.fw;
        {
            ProfScope ps(PK_LEG_ANALYS, stream);
            e = launch_legendre_analys(l, stream);
        }
        if (e) return hip_error(e, "batch legendre analysis launch");
    }
    return run_stored(b, F, Q, 0, stream);
}

int upload(shtn_batch_s& b, void* dev_buf, void* stream)
{
    for (auto* p : b.plans)
        if (!p->uploaded) return set_error(SHTN_ESTATE, "plan of the batch not uploaded");
    // unit tables built from an earlier state of a plan (lane starts, tiling,
    // stored-P table): rebuild them for the current one
    if (plan_gens(b) != b.tables_gen) {
        try {
            build_tables(b, b.tiling);
        } catch (const std::bad_alloc&) {
            return set_error(SHTN_ENOMEM, "out of host memory");
        }
        if (b.image.size() > b.max_image)
            return set_error(SHTN_ESTATE, "the batch's plans changed so that its tables no longer fit the buffer "
                                          "sized by shtn_batch_device_bytes: create the batch again");
    }
    // descriptors of the plans as uploaded (device pointers to their tables)
    for (size_t i = 0; i < b.plans.size(); i++) {
        const Plan& p = *b.plans[i];
        DevPlan d;
        std::memcpy(&d, p.image.data(), sizeof(DevPlan));
        std::memcpy(b.image.data() + b.off_plans + i * sizeof(DevPlan), &d, sizeof(DevPlan));
    }
    hipError_t e = hipMemcpyAsync(dev_buf, b.image.data(), b.image.size(), hipMemcpyHostToDevice,
                                  (hipStream_t)stream);
    if (e != hipSuccess) return hip_error((int)e, "batch upload copy");
    e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_error((int)e, "batch upload sync");
    b.dev = dev_buf;
    b.uploaded = true;
    b.upload_gen = plan_gens(b);
    drop_graphs(b);
    return SHTN_OK;
}

int capture(shtn_batch_s& b, int which, const double* in, double* out, void* work)
{
    if (which != 0 && which != 1) return set_error(SHTN_EINVAL, "which must be 0 (synthesis) or 1 (analysis)");
    int rc = which == 0 ? check_batch(&b, in, Data::spec, out, Data::grid, work)
                        : check_batch(&b, in, Data::grid, out, Data::spec, work);
    if (rc) return rc;
    if (!b.cap_stream) {
        hipError_t e = hipStreamCreateWithFlags(&b.cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_error((int)e, "capture stream");
    }
    if (b.exec[which]) {
        (void)hipGraphExecDestroy(b.exec[which]);
        b.exec[which] = nullptr;
    }
    hipError_t e = hipStreamBeginCapture(b.cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_error((int)e, "begin capture");
    prof_set_capturing(true);
    rc = which == 0 ? run_synth(b, in, out, work, b.cap_stream) : run_analys(b, in, out, work, b.cap_stream);
    prof_set_capturing(false);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b.cap_stream, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return hip_error((int)e, "end capture");
    e = hipGraphInstantiate(&b.exec[which], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        b.exec[which] = nullptr;
        return hip_error((int)e, "graph instantiate");
    }
    return SHTN_OK;
}

// Tuner cache key: format version, the GPU's architecture name (a tiling
// tuned on one chip is no answer for another) and the field shapes.
std::string cache_key(const shtn_batch_s& b)
{
    std::ostringstream os;
    os << "shtn-batch-v2";
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        std::string arch(prop.gcnArchName);
        for (char& c : arch)
            if (c == ' ' || c == '|') c = '_';
        os << ' ' << arch;
    } else {
        os << " unknown-arch";
    }
    for (int f = 0; f < b.nfields; f++) {
        const Plan& p = *b.field_plan[f]->p;
        os << ' ' << p.L << ',' << p.M << ',' << p.nlat << ',' << p.nphi;
    }
    return os.str();
}

int validate(const BatchTiling& t)
{
    if (t.synth_lp != 1 && t.synth_lp != 2 && t.synth_lp != 4)
        return set_error(SHTN_EINVAL, "synth_lp must be 1, 2 or 4");
    if (t.fw != 1 && t.fw != 2 && t.fw != 4) return set_error(SHTN_EINVAL, "fw must be 1, 2 or 4");
    if (t.fw == 4 && t.synth_lp > 2) return set_error(SHTN_EINVAL, "fw=4 needs synth_lp <= 2");
    if (t.m_pairing != 0 && t.m_pairing != 1) return set_error(SHTN_EINVAL, "m_pairing must be 0 or 1");
    if (t.analys_merge != 0 && t.analys_merge != 1)
        return set_error(SHTN_EINVAL, "analys_merge must be 0 or 1");
    if (t.stored != 0 && t.stored != 1) return set_error(SHTN_EINVAL, "stored must be 0 or 1");
    return SHTN_OK;
}

// A cached tiling for key, or false.  Entries that do not parse or that name
// a tiling outside the built kernels (a damaged or foreign cache file) are
// treated as misses, so the tuner times the candidates instead.
bool cache_lookup(const char* path, const std::string& key, BatchTiling& t)
{
    if (!path) return false;
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line)) {
        if (line.size() <= key.size() || line.compare(0, key.size(), key) != 0 || line[key.size()] != '|')
            continue;
        std::istringstream is(line.substr(key.size() + 1));
        BatchTiling c;
        if (is >> c.synth_lp >> c.fw >> c.m_pairing >> c.analys_merge) {
            if (!(is >> c.stored)) c.stored = 0;
            if (validate(c) != SHTN_OK) continue;
            t = c;
            return true;
        }
    }
    return false;
}


}  // namespace

extern "C" {

shtn_batch_t shtn_batch(int nfields, const shtn_plan_t* plans)
{
    if (nfields < 1 || !plans) {
        set_error(SHTN_EINVAL, "nfields must be >= 1 and plans non-null");
        return nullptr;
    }
    try {
        auto* b = new shtn_batch_s;
        b->nfields = nfields;
        b->field_plan.assign(plans, plans + nfields);
        std::vector<int> fpi(nfields);
        for (int f = 0; f < nfields; f++) {
            if (!plans[f] || !plans[f]->p) {
                delete b;
                set_error(SHTN_EINVAL, "null plan in batch");
                return nullptr;
            }
            Plan* p = plans[f]->p;
            if (p->npair > kMaxAnalysPairs) {
                delete b;
                set_error(SHTN_EUNSUPPORTED, "batch fields support at most 4096 latitudes");
                return nullptr;
            }
            auto it = std::find(b->plans.begin(), b->plans.end(), p);
            if (it == b->plans.end()) {
                fpi[f] = (int)b->plans.size();
                b->plans.push_back(p);
            } else {
                fpi[f] = (int)(it - b->plans.begin());
            }
        }
        // packed layout in user field order
        b->q_off.assign(nfields + 1, 0);
        b->g_off.assign(nfields + 1, 0);
        for (int f = 0; f < nfields; f++) {
            const Plan& p = *plans[f]->p;
            b->q_off[f + 1] = b->q_off[f] + 2 * (size_t)p.nlm;
            b->g_off[f + 1] = b->g_off[f] + (size_t)p.nlat * p.nphi;
        }
        // slots grouped by plan
        for (size_t pi = 0; pi < b->plans.size(); pi++)
            for (int f = 0; f < nfields; f++)
                if (fpi[f] == (int)pi) {
                    b->slot_field.push_back(f);
                    b->slot_plan.push_back((int)pi);
                }
        // workspace: F then the rescaled spectra, per slot, 256-byte aligned
        size_t fo = 0;
        for (int s = 0; s < nfields; s++) {
            const Plan& p = *b->plans[b->slot_plan[s]];
            b->slot_q.push_back((long)b->q_off[b->slot_field[s]]);
            b->slot_g.push_back((long)b->g_off[b->slot_field[s]]);
            b->slot_f.push_back((long)fo);
            fo += align256((size_t)f_layout(p.M, p.nlat).size * 16) / 8;
            b->max_nlm = std::max(b->max_nlm, p.nlm);
        }
        b->work_f_doubles = fo;
        size_t so = 0;
        for (int s = 0; s < nfields; s++) {
            const Plan& p = *b->plans[b->slot_plan[s]];
            b->slot_s.push_back((long)so);
            so += align256((size_t)p.nlm * 16) / 8;
        }
        so += 2 * (size_t)kTablePad;  // block loads may run past the last field
        b->work_total_bytes = align256((fo + so) * 8);
        // the largest image over the tiling space (one field per wave, one
        // order and one pair per lane, separate analysis classes)
        BatchTiling worst;
        build_tables(*b, worst);
        b->max_image = b->image.size();
        build_tables(*b, b->tiling);
        b->max_image = std::max(b->max_image, b->image.size());
        return b;
    } catch (const std::bad_alloc&) {
        set_error(SHTN_ENOMEM, "out of host memory");
        return nullptr;
    } catch (...) {
        set_error(SHTN_EINVAL, "internal error");
        return nullptr;
    }
}

void shtn_batch_destroy(shtn_batch_t batch)
{
    if (!batch) return;
    drop_graphs(*batch);
    if (batch->cap_stream) (void)hipStreamDestroy(batch->cap_stream);
    delete batch;
}

int shtn_batch_offsets(shtn_batch_t batch, size_t* q_off, size_t* grid_off)
{
    if (!batch) return set_error(SHTN_EINVAL, "null batch");
    if (q_off) std::memcpy(q_off, batch->q_off.data(), batch->q_off.size() * sizeof(size_t));
    if (grid_off) std::memcpy(grid_off, batch->g_off.data(), batch->g_off.size() * sizeof(size_t));
    return SHTN_OK;
}

size_t shtn_batch_device_bytes(shtn_batch_t batch) { return batch ? batch->max_image : 0; }

size_t shtn_batch_work_bytes(shtn_batch_t batch) { return batch ? batch->work_total_bytes : 0; }

int shtn_batch_upload(shtn_batch_t batch, void* dev_buf, void* stream)
{
    if (!batch) return set_error(SHTN_EINVAL, "null batch");
    if (!dev_buf) return set_error(SHTN_EINVAL, "null device buffer");
    if ((uintptr_t)dev_buf % 256) return set_error(SHTN_EINVAL, "device buffer must be 256-byte aligned");
    return upload(*batch, dev_buf, stream);
}

int shtn_batch_synth(shtn_batch_t batch, const double* Qpacked, double* gridpacked, void* work,
                     void* stream)
{
    int rc = check_batch(batch, Qpacked, Data::spec, gridpacked, Data::grid, work);
    if (rc) return rc;
    return run_synth(*batch, Qpacked, gridpacked, work, stream);
}

int shtn_batch_analys(shtn_batch_t batch, const double* gridpacked, double* Qpacked, void* work,
                      void* stream)
{
    int rc = check_batch(batch, gridpacked, Data::grid, Qpacked, Data::spec, work);
    if (rc) return rc;
    return run_analys(*batch, gridpacked, Qpacked, work, stream);
}

int shtn_batch_set_tiling(shtn_batch_t batch, int synth_lp, int fw, int m_pairing, int analys_merge)
{
    if (!batch) return set_error(SHTN_EINVAL, "null batch");
    BatchTiling t{synth_lp, fw, m_pairing, analys_merge, batch->tiling.stored};
    int rc = validate(t);
    if (rc) return rc;
    try {
        batch->tiling = t;
        build_tables(*batch, t);
    } catch (const std::bad_alloc&) {
        return set_error(SHTN_ENOMEM, "out of host memory");
    }
    batch->uploaded = false;  // the unit tables changed: upload again
    drop_graphs(*batch);
    return SHTN_OK;
}

int shtn_batch_set_algorithm(shtn_batch_t batch, int algo)
{
    if (!batch) return set_error(SHTN_EINVAL, "null batch");
    if (algo != SHTN_ALGO_ONTHEFLY && algo != SHTN_ALGO_STORED)
        return set_error(SHTN_EINVAL, "batch algorithm must be SHTN_ALGO_ONTHEFLY or SHTN_ALGO_STORED");
    BatchTiling t = batch->tiling;
    t.stored = algo == SHTN_ALGO_STORED;
    try {
        batch->tiling = t;
        build_tables(*batch, t);
    } catch (const std::bad_alloc&) {
        return set_error(SHTN_ENOMEM, "out of host memory");
    }
    batch->uploaded = false;
    drop_graphs(*batch);
    return SHTN_OK;
}

int shtn_batch_get_algorithm(shtn_batch_t batch)
{
    if (!batch) return set_error(SHTN_EINVAL, "null batch");
    return batch->tiling.stored ? SHTN_ALGO_STORED : SHTN_ALGO_ONTHEFLY;
}

int shtn_batch_get_tiling(shtn_batch_t batch, int* tiling4)
{
    if (!batch || !tiling4) return set_error(SHTN_EINVAL, "null argument");
    tiling4[0] = batch->tiling.synth_lp;
    tiling4[1] = batch->tiling.fw;
    tiling4[2] = batch->tiling.m_pairing;
    tiling4[3] = batch->tiling.analys_merge;
    return SHTN_OK;
}

int shtn_batch_capture(shtn_batch_t batch, int which, const double* in, double* out, void* work)
{
    if (!batch) return set_error(SHTN_EINVAL, "null batch");
    return capture(*batch, which, in, out, work);
}

int shtn_batch_replay(shtn_batch_t batch, int which, void* stream)
{
    if (!batch) return set_error(SHTN_EINVAL, "null batch");
    if (which != 0 && which != 1) return set_error(SHTN_EINVAL, "which must be 0 or 1");
    if (!batch->uploaded || !batch->exec[which])
        return set_error(SHTN_ESTATE, "no captured graph (call shtn_batch_capture after the upload)");
    if (plan_gens(*batch) != batch->upload_gen)
        return set_error(SHTN_ESTATE, "a plan of the batch changed since the graphs were captured: upload and "
                                      "capture again");
    hipError_t e = hipGraphLaunch(batch->exec[which], (hipStream_t)stream);
    if (e != hipSuccess) return hip_error((int)e, "graph launch");
    return SHTN_OK;
}

int shtn_batch_tune(shtn_batch_t batch, const double* Qpacked, double* gridpacked, double* Qout,
                    void* work, void* stream, int reps, const char* cache_path, float* best_us)
{
    int rc = check_batch(batch, Qpacked, Data::spec, gridpacked, Data::grid, work);
    if (rc) return rc;
    if (!Qout) return set_error(SHTN_EINVAL, "null Qout");
    if ((rc = check_batch(batch, gridpacked, Data::grid, Qout, Data::spec, work))) return rc;
    {
        const size_t sb = packed_bytes(*batch, Data::spec);
        if ((rc = check_disjoint({{"Qpacked", Qpacked, sb, false}, {"Qout", Qout, sb, true}}))) return rc;
    }
    if (reps < 1) reps = 10;
    shtn_batch_s& b = *batch;
    void* dev = b.dev;
    const std::string key = cache_key(b);
    BatchTiling best = b.tiling;
    float best_t = -1.f;
    if (!cache_lookup(cache_path, key, best)) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
            return hip_error((int)hipGetLastError(), "tuner events");
        bool any_table = false;
        for (auto* p : b.plans) any_table = any_table || p->ptab.built;
        std::vector<BatchTiling> cands;
        for (int st = 0; st <= (any_table ? 1 : 0); st++)
            for (int lp : {1, 2})
                for (int fw : {1, 2, 4})
                    for (int mp : {0, 1})
                        for (int merge : {0, 1}) cands.push_back(BatchTiling{lp, fw, mp, merge, st});
        for (const BatchTiling& t : cands) {
            build_tables(b, t);
            b.tiling = t;
            if ((rc = upload(b, dev, stream))) break;
            if ((rc = capture(b, 0, Qpacked, gridpacked, work))) break;
            if ((rc = capture(b, 1, gridpacked, Qout, work))) break;
            for (int w = 0; w < 2; w++) {
                (void)hipGraphLaunch(b.exec[0], (hipStream_t)stream);
                (void)hipGraphLaunch(b.exec[1], (hipStream_t)stream);
            }
            (void)hipEventRecord(e0, (hipStream_t)stream);
            for (int r = 0; r < reps; r++) {
                (void)hipGraphLaunch(b.exec[0], (hipStream_t)stream);
                (void)hipGraphLaunch(b.exec[1], (hipStream_t)stream);
            }
            (void)hipEventRecord(e1, (hipStream_t)stream);
            hipError_t he = hipEventSynchronize(e1);
            float ms = 0.f;
            if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
            if (he != hipSuccess) {
                rc = hip_error((int)he, "tuner timing");
                break;
            }
            const float us = 1000.f * ms / reps;
            if (best_t < 0.f || us < best_t) {
                best_t = us;
                best = t;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (rc) return rc;
        if (cache_path) {
            std::ofstream out(cache_path, std::ios::app);
            out << key << '|' << best.synth_lp << ' ' << best.fw << ' ' << best.m_pairing << ' '
                << best.analys_merge << ' ' << best.stored << '\n';
        }
    }
    build_tables(b, best);
    b.tiling = best;
    if ((rc = upload(b, dev, stream))) return rc;
    if ((rc = capture(b, 0, Qpacked, gridpacked, work))) return rc;
    if ((rc = capture(b, 1, gridpacked, Qout, work))) return rc;
    if (best_us) *best_us = best_t;
    return SHTN_OK;
}

}  // extern "C"
