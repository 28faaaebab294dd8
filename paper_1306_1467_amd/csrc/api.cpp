// C ABI of libvjboost: argument checks, workspace layout, context lifetime,
// round launches (direct or replayed from a captured HIP graph) and timing.
#include <math.h>
#include <string.h>

#include <string>
#include <vector>

#include "launch.h"

namespace vjb {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
const char* get_error() { return g_err.c_str(); }

constexpr int64_t kMaxFp64N = 20000;   // FP64 weight table must fit in LDS

bool valid_options(const boost_options* o) {
    if (!o) return false;
    if (o->precision < BOOST_PREC_FP32 || o->precision > BOOST_PREC_FP32_WIDE) return false;
    if (o->on_perfect != BOOST_ON_PERFECT_CLAMP && o->on_perfect != BOOST_ON_PERFECT_STOP) return false;
    if (!(o->eps_floor > 0.0) || !(o->eps_floor < 0.5)) return false;
    if (o->schedule_id != BOOST_SCHEDULE_AUTO && (o->schedule_id < 0 || o->schedule_id >= scan_schedule_count()))
        return false;
    if (o->flags & ~(BOOST_FLAG_TIMING | BOOST_FLAG_NO_GRAPH)) return false;
    return true;
}

static size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
    size_t keys, ii, ftab, sorder, defer, w, wtmp, wpart, st, ring, perm, inv, wgbest, cls, pad, scratch, total;
};

static bool make_layout(int64_t n, const boost_feature_set* fs, Layout& L) {
    const int64_t F = host_feature_count(fs);
    if (F <= 0) return false;
    const KeyGeom g = make_geom(n, 64);
    const int64_t P = (int64_t)(fs->window_w + 1) * (fs->window_h + 1);
    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t o = off; off += a256(bytes); return o; };
    L.keys = take((size_t)F * (size_t)g.row_units * 16);
    L.ii = take((size_t)P * (size_t)ii_stride_of(n) * 4);
    L.ftab = take((size_t)F * 4);
    L.sorder = take((size_t)F * 4);
    L.defer = take(n > kNarrowMaxN ? (size_t)(F + 16) * 4 : 0);
    L.w = take((size_t)n * 16);
    L.wtmp = take((size_t)n * 8);
    L.wpart = take((size_t)kMaxPart * 8);
    L.st = take(sizeof(JobState));
    L.ring = take((size_t)kRing * sizeof(boost_stump));
    L.perm = take((size_t)n * 4);
    L.inv = take((size_t)n * 4);
    L.wgbest = take((size_t)kMaxScanGrid * sizeof(WgBest));
    L.cls = take((size_t)kMaxClassifyT * sizeof(StumpDev));
    L.pad = take(16);
    L.scratch = take(sort_scratch_bytes(n));
    L.total = off;
    return true;
}

int check_job_args(int64_t n, const boost_feature_set* fs, const boost_options* o) {
    if (n < 2 || n > kMaxN) { set_error("n must be in 2..32767"); return BOOST_E_INVALID; }
    if (!valid_feature_set(fs)) { set_error("invalid feature set (window 1..32, non-empty 5-bit type mask)"); return BOOST_E_INVALID; }
    if (!valid_options(o)) { set_error("invalid options"); return BOOST_E_INVALID; }
    if (host_feature_count(fs) <= 0) { set_error("the feature set has no feature that fits the window"); return BOOST_E_INVALID; }
    if (o->precision == BOOST_PREC_FP64 && n > kMaxFp64N) {
        set_error("FP64 precision supports at most 20000 windows (the weight table lives in LDS)");
        return BOOST_E_INVALID;
    }
    return BOOST_OK;
}

size_t job_bytes(int64_t n, const boost_feature_set* fs) {
    Layout L;
    if (!make_layout(n, fs, L)) return 0;
    return L.total;
}

static int sync_state(hipStream_t s, const JobState* d_st, JobState& st) {
    VJB_HIP(hipStreamSynchronize(s));
    VJB_HIP(hipMemcpy(&st, d_st, sizeof(JobState), hipMemcpyDeviceToHost));
    return BOOST_OK;
}

// Lays one job out in ws (job_bytes(n, fs) bytes) and runs its one-time
// preparation: ingest, integral images, per-feature evaluate + sort + keys,
// initial weights.  Synchronises (label validation needs the count).
int setup_job(JobHost& h, char* ws, int64_t n, const boost_feature_set* fs, const boost_options* o,
              const uint8_t* d_images, const uint8_t* d_labels, int num_cu, hipStream_t s, const ExtendSrc* ext) {
    Layout L;
    make_layout(n, fs, L);
    JobDev& jd = h.jd;
    jd = JobDev{};
    jd.keys = (const uint4*)(ws + L.keys);
    jd.ii = (const int32_t*)(ws + L.ii);
    jd.ftab = (const uint32_t*)(ws + L.ftab);
    jd.w = (double*)(ws + L.w);
    jd.wpart = (double*)(ws + L.wpart);
    jd.wgb = (WgBest*)(ws + L.wgbest);
    jd.pad = (const uint4*)(ws + L.pad);
    jd.st = (JobState*)(ws + L.st);
    jd.ring = (boost_stump*)(ws + L.ring);
    jd.perm = (const int32_t*)(ws + L.perm);
    jd.inv = (const int32_t*)(ws + L.inv);
    jd.g = make_geom(n, scan_schedule_lanes(o->schedule_id < 0 ? 0 : o->schedule_id));
    jd.F = host_feature_count(fs);
    jd.ii_stride = ii_stride_of(n);
    jd.W = fs->window_w;
    jd.H = fs->window_h;
    jd.precision = o->precision;
    jd.on_perfect = o->on_perfect;
    jd.n_part = (int32_t)((n + kUpdWg - 1) / kUpdWg);
    jd.unused = 0;
    jd.eps_floor = o->eps_floor;
    h.wtmp = (double*)(ws + L.wtmp);
    h.merged = false;
    h.cls = (StumpDev*)(ws + L.cls);
    h.scratch = sort_scratch_bytes(n) ? (uint64_t*)(ws + L.scratch) : nullptr;

    h.sorder = (const uint32_t*)(ws + L.sorder);
    h.defer = n > kNarrowMaxN ? (uint32_t*)(ws + L.defer) : nullptr;
    std::vector<uint32_t> ftab((size_t)jd.F), sorder((size_t)jd.F);
    host_feature_table(fs, ftab.data());
    host_sort_order(ftab.data(), jd.F, sorder.data());
    const uint32_t pd = pad_dword(jd.g);
    const uint32_t pad_unit[4] = {pd, pd, pd, pd};
    VJB_HIP(hipMemcpyAsync((void*)jd.ftab, ftab.data(), ftab.size() * 4, hipMemcpyHostToDevice, s));
    VJB_HIP(hipMemcpyAsync((void*)h.sorder, sorder.data(), sorder.size() * 4, hipMemcpyHostToDevice, s));
    VJB_HIP(hipMemcpyAsync((void*)jd.pad, pad_unit, 16, hipMemcpyHostToDevice, s));
    VJB_HIP(hipMemsetAsync(jd.st, 0, sizeof(JobState), s));
    int rc;
    if (ext != nullptr) {
        // the union's labels (old windows first) go through the same ingest;
        // the weight scratch holds them until then
        uint8_t* ul = (uint8_t*)h.wtmp;
        if ((rc = union_labels_launch(*ext->old, ext->l0, d_labels, n - ext->old->g.n, ul, s)) != BOOST_OK) return rc;
        d_labels = ul;
    }
    if ((rc = ingest_launch(jd, d_labels, n, s)) != BOOST_OK) return rc;
    JobState st;
    if ((rc = sync_state(s, jd.st, st)) != BOOST_OK) return rc;   // also retires the host copies above
    if (st.label_error) { set_error("labels must be 0 or 1"); return BOOST_E_INVALID; }
    if (st.n_pos == 0 || st.n_pos == n) {
        set_error("both classes need at least one window (1/(2l) and 1/(2m) must exist)");
        return BOOST_E_INVALID;
    }
    h.n_pos = st.n_pos;
    if (ext == nullptr) {
        if ((rc = integral_launch(jd, d_images, s)) != BOOST_OK) return rc;
        if ((rc = sort_launch(jd, h.sorder, h.scratch, h.defer, num_cu, s)) != BOOST_OK) return rc;
    } else {
        const JobDev& old = *ext->old;
        if ((rc = extend_ii_launch(jd, old, d_images, s)) != BOOST_OK) return rc;
        const int64_t lm = st.n_pos - ext->l0;
        h.merged = n > kMergeMinN && n <= kMergeMaxN && n - old.g.n <= kMergeMaxM && old.g.narrow &&
                   old.g.lanes == jd.g.lanes;
        if (h.merged) rc = merge_launch(jd, h.sorder, old.keys, old.g, (int)ext->l0, (int)lm, num_cu, s);
        else rc = sort_launch(jd, h.sorder, h.scratch, h.defer, num_cu, s);
        if (rc != BOOST_OK) return rc;
    }
    if ((rc = init_weights_launch(jd, s)) != BOOST_OK) return rc;
    return BOOST_OK;
}

}  // namespace vjb

using namespace vjb;

struct boost_ctx {
    JobDev jd;
    double* wtmp = nullptr;
    StumpDev* cls = nullptr;
    uint64_t* scratch = nullptr;
    int device = 0, num_cu = 0;
    hipStream_t stream = nullptr;
    boost_options opts;
    boost_feature_set fs;
    int64_t n = 0, F = 0, n_pos = 0;
    bool merged = false;   // keys merged from an extended job's (boost_extend)
    ScanPlan plan;
    int schedule = 0;
    std::vector<double> tune_ms;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    std::vector<hipEvent_t> ev;
    double t_scan = 0, t_fin = 0, rounds_timed = 0, scans_timed = 0;
    int64_t launched = 0;   // scan launches so far (= device ring cursor)
};

extern "C" {

int boost_version(void) { return 10000; }

const char* boost_last_error(void) { return get_error(); }

int boost_options_default(boost_options* o) {
    if (!o) { set_error("options pointer is NULL"); return BOOST_E_INVALID; }
    o->precision = BOOST_PREC_FP32_WIDE;
    o->on_perfect = BOOST_ON_PERFECT_CLAMP;
    o->eps_floor = 1e-10;
    o->schedule_id = 0;
    o->flags = 0;
    o->stream = nullptr;
    return BOOST_OK;
}

int64_t boost_feature_count(const boost_feature_set* fs) { return host_feature_count(fs); }

int boost_feature_desc(const boost_feature_set* fs, int64_t j, boost_feature* out) {
    const int64_t F = host_feature_count(fs);
    if (F < 0 || !out || j < 0 || j >= F) { set_error("invalid feature set, index or output"); return BOOST_E_INVALID; }
    return host_feature_desc(fs, j, out);
}

int boost_schedule_count(int32_t precision) {
    (void)precision;
    return scan_schedule_count();
}

int boost_probe_stream(boost_ctx* c, int32_t reps, double* best_ms) {
    if (!c || !best_ms || reps < 1) { set_error("NULL context or output, or reps < 1"); return BOOST_E_INVALID; }
    // the per-workgroup candidate records (one per scan workgroup) take the
    // probe's words; the next round's scan rewrites them
    uint32_t* sink = (uint32_t*)c->jd.wgb;
    static_assert(sizeof(WgBest) >= sizeof(uint32_t), "one probe word per scan workgroup record");
    return time_launches(c->stream, reps, [&]() { return probe_launch(c->plan, c->schedule, c->jd, sink, c->stream); },
                         *best_ms);
}

int boost_get_schedule(const boost_ctx* c, double* ms_out, int32_t cap) {
    if (!c) { set_error("NULL context"); return BOOST_E_INVALID; }
    if (ms_out)
        for (int k = 0; k < cap && k < (int)c->tune_ms.size(); ++k) ms_out[k] = c->tune_ms[(size_t)k];
    return c->schedule;
}

size_t boost_workspace_bytes(int64_t n, const boost_feature_set* fs, const boost_options* o) {
    if (check_job_args(n, fs, o) != BOOST_OK) return 0;
    return job_bytes(n, fs);
}

static int sync_and_state(boost_ctx* c, JobState& st) { return sync_state(c->stream, c->jd.st, st); }

// Shared by boost_init and boost_extend: a context over n windows of
// d_images / d_labels, or (ext) over the union of an old job and them.
static int init_context(boost_ctx** out, const uint8_t* d_images, const uint8_t* d_labels, int64_t n,
                        const boost_feature_set* fs, const boost_options* o, void* d_workspace,
                        size_t workspace_bytes, const ExtendSrc* ext) {
    int rc = check_job_args(n, fs, o);
    if (rc != BOOST_OK) return rc;
    const size_t need = job_bytes(n, fs);
    if (workspace_bytes < need) {
        set_error("workspace too small: need " + std::to_string(need) + " bytes");
        return BOOST_E_NOMEM;
    }
    boost_ctx* c = new boost_ctx();
    c->opts = *o;
    c->fs = *fs;
    c->n = n;
    c->F = host_feature_count(fs);
    c->stream = (hipStream_t)o->stream;
    // on failure, work already queued on the stream finishes before the call
    // returns: the caller may free the workspace right away
    auto fail = [&](int code) {
        if (c->stream) (void)hipStreamSynchronize(c->stream); else (void)hipDeviceSynchronize();
        delete c;
        return code;
    };
    if (hipGetDevice(&c->device) != hipSuccess ||
        hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess) {
        set_error("no HIP device");
        return fail(BOOST_E_DEVICE);
    }
    JobHost h;
    if ((rc = setup_job(h, (char*)d_workspace, n, fs, o, d_images, d_labels, c->num_cu, c->stream, ext)) !=
        BOOST_OK)
        return fail(rc);
    c->jd = h.jd;
    c->n_pos = h.n_pos;
    c->merged = h.merged;
    c->wtmp = h.wtmp;
    c->cls = h.cls;
    c->scratch = h.scratch;
    c->schedule = o->schedule_id;
    c->tune_ms.assign((size_t)scan_schedule_count(), -1.0);
    if (o->schedule_id == BOOST_SCHEDULE_AUTO &&
        (rc = tune_single(c->jd, o->precision, c->num_cu, c->device, c->stream, c->tune_ms.data(), c->schedule)) !=
            BOOST_OK)
        return fail(rc);
    if ((rc = scan_plan(c->plan, o->precision, c->jd.g.narrow != 0, c->schedule, n, c->F, c->num_cu)) != BOOST_OK)
        return fail(rc);
    if (hipStreamSynchronize(c->stream) != hipSuccess) { set_error("device error during init"); return fail(BOOST_E_DEVICE); }
    *out = c;
    return BOOST_OK;
}

int boost_init(boost_ctx** out, const uint8_t* d_images, const uint8_t* d_labels, int64_t n,
               const boost_feature_set* fs, const boost_options* o, void* d_workspace, size_t workspace_bytes) {
    if (!out || !d_images || !d_labels || !d_workspace) { set_error("NULL pointer argument"); return BOOST_E_INVALID; }
    *out = nullptr;
    return init_context(out, d_images, d_labels, n, fs, o, d_workspace, workspace_bytes, nullptr);
}

size_t boost_extend_workspace_bytes(const boost_ctx* c, int64_t m) {
    if (!c || m < 1) return 0;
    return boost_workspace_bytes(c->n + m, &c->fs, &c->opts);
}

int boost_extend(boost_ctx** out, const boost_ctx* c, const uint8_t* d_images, const uint8_t* d_labels, int64_t m,
                 void* d_workspace, size_t workspace_bytes) {
    if (!out || !c || !d_images || !d_labels || !d_workspace) { set_error("NULL pointer argument"); return BOOST_E_INVALID; }
    *out = nullptr;
    if (m < 1 || c->n + m > kMaxN) { set_error("m must be >= 1 with n + m <= 32767"); return BOOST_E_INVALID; }
    if (c->stream) VJB_HIP(hipStreamSynchronize(c->stream));   // the old job's preparation is complete
    const ExtendSrc ext{&c->jd, c->n_pos};
    return init_context(out, d_images, d_labels, c->n + m, &c->fs, &c->opts, d_workspace, workspace_bytes, &ext);
}

int boost_extend_merged(const boost_ctx* c) {
    if (!c) { set_error("NULL context"); return BOOST_E_INVALID; }
    return c->merged ? 1 : 0;
}

static int launch_round(boost_ctx* c, double* d_feature_err, hipEvent_t e0, hipEvent_t e1, hipEvent_t e2) {
    int rc;
    if (e0) VJB_HIP(hipEventRecord(e0, c->stream));
    if ((rc = scan_launch(c->plan, c->jd, (double2*)d_feature_err, c->stream)) != BOOST_OK) return rc;
    if (e1) VJB_HIP(hipEventRecord(e1, c->stream));
    if ((rc = update_launch(c->jd, c->plan.grid, c->stream)) != BOOST_OK) return rc;
    if (e2) VJB_HIP(hipEventRecord(e2, c->stream));
    c->launched++;
    return BOOST_OK;
}

static int ensure_events(boost_ctx* c, size_t count) {
    while (c->ev.size() < count) {
        hipEvent_t e;
        VJB_HIP(hipEventCreate(&e));
        c->ev.push_back(e);
    }
    return BOOST_OK;
}

// Sums the elapsed times of the first `rounds` event triples.
static int collect_timing(boost_ctx* c, int rounds) {
    if (rounds <= 0) return BOOST_OK;
    VJB_HIP(hipEventSynchronize(c->ev[3 * (rounds - 1) + 2]));
    for (int r = 0; r < rounds; ++r) {
        float a = 0, b = 0;
        VJB_HIP(hipEventElapsedTime(&a, c->ev[3 * r], c->ev[3 * r + 1]));
        VJB_HIP(hipEventElapsedTime(&b, c->ev[3 * r + 1], c->ev[3 * r + 2]));
        c->t_scan += a;
        c->t_fin += b;
    }
    c->rounds_timed += rounds;
    c->scans_timed += rounds;
    return BOOST_OK;
}

static int copy_records(boost_ctx* c, int64_t first_launch, int count, boost_stump* dst) {
    // records of launches first_launch .. first_launch+count-1 (count <= kRing)
    int done = 0;
    while (done < count) {
        const int64_t slot = (first_launch + done) % kRing;
        int m = (int)(kRing - slot);
        if (m > count - done) m = count - done;
        VJB_HIP(hipMemcpyAsync(dst + done, c->jd.ring + slot, (size_t)m * sizeof(boost_stump), hipMemcpyDeviceToHost,
                               c->stream));
        done += m;
    }
    VJB_HIP(hipStreamSynchronize(c->stream));
    return BOOST_OK;
}

int boost_round(boost_ctx* c, boost_stump* out_host, double* d_feature_err) {
    if (!c) { set_error("NULL context"); return BOOST_E_INVALID; }
    int rc;
    const bool timing = (c->opts.flags & BOOST_FLAG_TIMING) != 0;
    const int64_t first = c->launched;
    if (timing) {
        if ((rc = ensure_events(c, 3)) != BOOST_OK) return rc;
        if ((rc = launch_round(c, d_feature_err, c->ev[0], c->ev[1], c->ev[2])) != BOOST_OK) return rc;
        if ((rc = collect_timing(c, 1)) != BOOST_OK) return rc;
    } else if ((rc = launch_round(c, d_feature_err, nullptr, nullptr, nullptr)) != BOOST_OK) {
        return rc;
    }
    if (out_host) {
        if ((rc = copy_records(c, first, 1, out_host)) != BOOST_OK) return rc;
        JobState st;
        if ((rc = sync_and_state(c, st)) != BOOST_OK) return rc;
        if (st.stopped) { set_error("eps reached the floor with the STOP policy"); return BOOST_E_DEGENERATE; }
    }
    return BOOST_OK;
}

static int ensure_graph(boost_ctx* c) {
    if (c->gexec) return BOOST_OK;
    VJB_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    int rc = scan_launch(c->plan, c->jd, nullptr, c->stream);
    if (rc == BOOST_OK) rc = update_launch(c->jd, c->plan.grid, c->stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->stream, &g);
    if (rc != BOOST_OK) { if (g) (void)hipGraphDestroy(g); return rc; }
    if (e != hipSuccess) { set_error(std::string("graph capture: ") + hipGetErrorString(e)); return BOOST_E_DEVICE; }
    c->graph = g;
    VJB_HIP(hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0));
    return BOOST_OK;
}

int boost_train(boost_ctx* c, int32_t rounds, boost_stump* out_host) {
    if (!c) { set_error("NULL context"); return BOOST_E_INVALID; }
    if (rounds < 0) { set_error("rounds must be >= 0"); return BOOST_E_INVALID; }
    int rc;
    const bool timing = (c->opts.flags & BOOST_FLAG_TIMING) != 0;
    const bool graph = !timing && !(c->opts.flags & BOOST_FLAG_NO_GRAPH) && c->stream != nullptr;
    if (graph && (rc = ensure_graph(c)) != BOOST_OK) return rc;
    const int chunk_max = timing ? 1024 : kRing;
    int32_t done = 0;
    while (done < rounds) {
        const int chunk = (rounds - done) < chunk_max ? (rounds - done) : chunk_max;
        const int64_t first = c->launched;
        if (timing && (rc = ensure_events(c, 3 * (size_t)chunk)) != BOOST_OK) return rc;
        for (int r = 0; r < chunk; ++r) {
            if (graph) {
                VJB_HIP(hipGraphLaunch(c->gexec, c->stream));
                c->launched++;
            } else if (timing) {
                if ((rc = launch_round(c, nullptr, c->ev[3 * r], c->ev[3 * r + 1], c->ev[3 * r + 2])) != BOOST_OK) return rc;
            } else if ((rc = launch_round(c, nullptr, nullptr, nullptr, nullptr)) != BOOST_OK) {
                return rc;
            }
        }
        if (timing && (rc = collect_timing(c, chunk)) != BOOST_OK) return rc;
        if (out_host && (rc = copy_records(c, first, chunk, out_host + done)) != BOOST_OK) return rc;
        done += chunk;
    }
    if (out_host || timing) {
        JobState st;
        if ((rc = sync_and_state(c, st)) != BOOST_OK) return rc;
        if (st.stopped) { set_error("eps reached the floor with the STOP policy"); return BOOST_E_DEGENERATE; }
    }
    return BOOST_OK;
}

int boost_get_weights(boost_ctx* c, double* d_w) {
    if (!c || !d_w) { set_error("NULL argument"); return BOOST_E_INVALID; }
    return get_weights_launch(c->jd, d_w, c->stream);
}

int boost_set_weights(boost_ctx* c, const double* d_w) {
    if (!c || !d_w) { set_error("NULL argument"); return BOOST_E_INVALID; }
    int rc = set_weights_launch(c->jd, d_w, c->wtmp, c->stream);
    if (rc != BOOST_OK) return rc;
    JobState st;
    if ((rc = sync_and_state(c, st)) != BOOST_OK) return rc;
    if (st.weight_error) { set_error("weights must be finite, >= 0 and not all zero"); return BOOST_E_INVALID; }
    return BOOST_OK;
}

int boost_rounds_done(boost_ctx* c, int32_t* out_rounds) {
    if (!c || !out_rounds) { set_error("NULL argument"); return BOOST_E_INVALID; }
    JobState st;
    int rc = sync_and_state(c, st);
    if (rc != BOOST_OK) return rc;
    *out_rounds = st.round;
    return BOOST_OK;
}

int boost_get_timing(boost_ctx* c, double out[4]) {
    if (!c || !out) { set_error("NULL argument"); return BOOST_E_INVALID; }
    VJB_HIP(hipStreamSynchronize(c->stream));
    out[0] = c->t_scan; out[1] = c->t_fin; out[2] = c->rounds_timed; out[3] = c->scans_timed;
    return BOOST_OK;
}

int boost_reset_timing(boost_ctx* c) {
    if (!c) { set_error("NULL context"); return BOOST_E_INVALID; }
    c->t_scan = c->t_fin = c->rounds_timed = c->scans_timed = 0;
    return BOOST_OK;
}

int boost_get_feature_values(boost_ctx* c, int64_t j0, int64_t nf, int32_t* d_out) {
    if (!c || !d_out || j0 < 0 || nf < 0 || j0 + nf > c->F) { set_error("invalid feature range or output"); return BOOST_E_INVALID; }
    if (nf == 0) return BOOST_OK;
    return feature_values_launch(c->jd, j0, nf, d_out, c->stream);
}

int boost_get_integral(boost_ctx* c, int32_t* d_out) {
    if (!c || !d_out) { set_error("NULL argument"); return BOOST_E_INVALID; }
    return integral_out_launch(c->jd, d_out, c->stream);
}

int boost_get_sorted(boost_ctx* c, int64_t j0, int64_t nf, int32_t* d_order, uint8_t* d_run_end) {
    if (!c || !d_order || !d_run_end || j0 < 0 || nf < 0 || j0 + nf > c->F) {
        set_error("invalid feature range or output");
        return BOOST_E_INVALID;
    }
    if (nf == 0) return BOOST_OK;
    return sorted_out_launch(c->jd, j0, nf, d_order, d_run_end, c->stream);
}

static int classify_train(boost_ctx* c, const boost_stump* stumps, int32_t T, uint8_t* d_out, double* d_score,
                          int32_t* d_err_curve) {
    if (T < 0 || (T > 0 && !stumps)) { set_error("invalid arguments"); return BOOST_E_INVALID; }
    if (T > kMaxClassifyT) { set_error("at most 4096 stumps"); return BOOST_E_INVALID; }
    std::vector<StumpDev> h((size_t)(T > 0 ? T : 1));
    for (int t = 0; t < T; ++t) {
        const boost_stump& s = stumps[t];
        boost_feature f;
        if (s.feature < 0 || s.feature >= c->F || host_feature_desc(&c->fs, s.feature, &f) != BOOST_OK ||
            (s.polarity != 1 && s.polarity != -1) || !isfinite(s.alpha)) {
            set_error("invalid stump record " + std::to_string(t));
            return BOOST_E_INVALID;
        }
        h[t].desc = pack_feature(f.type, f.x, f.y, f.cell_w, f.cell_h);
        h[t].polarity = s.polarity;
        h[t].theta = s.threshold;
        h[t].pad = 0;
        h[t].alpha = s.alpha;
    }
    if (T > 0) VJB_HIP(hipMemcpyAsync(c->cls, h.data(), (size_t)T * sizeof(StumpDev), hipMemcpyHostToDevice, c->stream));
    int rc = classify_any_launch(c->jd.ii, c->jd.ii_stride, c->jd.W, c->n, c->cls, T, c->jd.perm, nullptr,
                                 d_err_curve ? (int64_t)c->n_pos : -1, d_out, d_score, d_err_curve, c->stream);
    if (rc != BOOST_OK) return rc;
    VJB_HIP(hipStreamSynchronize(c->stream));   // the host array h is read by the copy
    return BOOST_OK;
}

int boost_classify_train(boost_ctx* c, const boost_stump* stumps, int32_t T, uint8_t* d_out, double* d_score) {
    if (!c || !d_out) { set_error("invalid arguments"); return BOOST_E_INVALID; }
    return classify_train(c, stumps, T, d_out, d_score, nullptr);
}

int boost_classify_train_curve(boost_ctx* c, const boost_stump* stumps, int32_t T, int32_t* d_err_curve) {
    if (!c || !d_err_curve) { set_error("invalid arguments"); return BOOST_E_INVALID; }
    return classify_train(c, stumps, T, nullptr, nullptr, d_err_curve);
}

void boost_destroy(boost_ctx* c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream); else (void)hipDeviceSynchronize();
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    delete c;
}

}  // extern "C"
