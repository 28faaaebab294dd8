// C ABI of batched jobs: layout of many jobs in one workspace, the segment
// schedule of the persistent scan, and round launches (direct or replayed
// from a captured HIP graph).
#include <math.h>

#include <algorithm>
#include <string>
#include <vector>

#include "batch.h"

using namespace vjb;

namespace vjb {

static size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

struct BatchLayout {
    std::vector<size_t> job_off;
    size_t jobs, segs, next_seg, job_seg, seg_best, upd_job, upd_part, gather, total;
    size_t max_segs;
    int64_t n_upd;
};

static int check_batch(int32_t n_jobs, const boost_job* jobs, const boost_options* o) {
    if (n_jobs < 1 || n_jobs > kMaxJobs || !jobs) { set_error("1..4096 jobs required"); return BOOST_E_INVALID; }
    for (int k = 0; k < n_jobs; ++k) {
        const int rc = check_job_args(jobs[k].n, &jobs[k].fs, o);
        if (rc != BOOST_OK) { set_error("job " + std::to_string(k) + ": " + get_error()); return rc; }
    }
    return BOOST_OK;
}

static void batch_layout(int32_t n_jobs, const boost_job* jobs, BatchLayout& L) {
    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t o = off; off += a256(bytes); return o; };
    L.n_upd = 0;
    for (int k = 0; k < n_jobs; ++k) {
        L.job_off.push_back(take(job_bytes(jobs[k].n, &jobs[k].fs)));
        L.n_upd += (jobs[k].n + kUpdWg - 1) / kUpdWg;
    }
    // per launch at most about grid * segments per workgroup (rounding of the
    // segment length adds under 2 %) plus one per job
    const size_t max_segs = (size_t)2 * 2 * kMaxScanGrid * kMaxSegsPerWg + (size_t)n_jobs;
    L.max_segs = max_segs;
    L.jobs = take((size_t)n_jobs * sizeof(JobDev));
    L.segs = take(max_segs * sizeof(BatchSeg));
    L.next_seg = take(8);
    L.job_seg = take((size_t)n_jobs * 8);
    L.seg_best = take(max_segs * sizeof(WgBest));
    L.upd_job = take((size_t)L.n_upd * 4);
    L.upd_part = take((size_t)L.n_upd * 4);
    L.gather = take((size_t)kGatherRounds * (size_t)n_jobs * sizeof(boost_stump));
    L.total = off;
}

// Launch configuration of one key format's scan.
struct PartCfg {
    int schedule = -1, wg = 0, unroll = 0, spw = kSegsPerWg, grid = 0;
    const void* kernel = nullptr;
};

static int part_config(PartCfg& pc, int precision, bool narrow, int schedule, int num_cu) {
    pc.schedule = schedule;
    pc.wg = scan_schedule_wg(schedule);
    pc.unroll = scan_schedule_unroll(schedule);
    pc.kernel = batch_scan_kernel(precision, narrow, schedule);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pc.kernel, pc.wg, 0) != hipSuccess || per_cu < 1) {
        set_error("batched scan kernel does not fit on a compute unit");
        return BOOST_E_INVALID;
    }
    int64_t grid = (int64_t)per_cu * num_cu;
    if (grid > kMaxScanGrid) grid = kMaxScanGrid;
    pc.grid = (int)grid;
    return BOOST_OK;
}

// Cuts every job's features into segments of about the same cost for the
// work queues: about grid * spw segments per launch.  A feature of job k
// costs the key units its lanes walk (padding of the tail batch included)
// plus about two units per lane for the group epilogue.  The 14-bit-key jobs'
// segments come first (launch 0), then the 15-bit ones' (launch 1).
static void build_segments(const std::vector<JobHost>& jobs, const PartCfg part[2], std::vector<BatchSeg>& segs,
                           std::vector<int32_t>& job_seg, int32_t& split) {
    const int n_jobs = (int)jobs.size();
    std::vector<double> cost(n_jobs);
    double total[2] = {0, 0};
    for (int k = 0; k < n_jobs; ++k) {
        const KeyGeom& g = jobs[k].jd.g;
        const int pk = g.narrow ? 0 : 1;
        const int64_t unroll = part[pk].unroll > 0 ? part[pk].unroll : 8;
        const int64_t per = g.q + (g.rem > 0 ? 1 : 0), rest = per % unroll;
        const int64_t walked =
            per <= unroll ? unroll : per - rest + (rest == 0 ? 0 : rest <= unroll / 2 ? unroll / 2 : unroll);
        cost[k] = (double)(walked + 2) * g.lanes;
        total[pk] += cost[k] * (double)jobs[k].jd.F;
    }
    segs.clear();
    job_seg.assign((size_t)2 * n_jobs, 0);
    for (int pk = 0; pk < 2; ++pk) {
        if (pk == 1) split = (int32_t)segs.size();
        if (part[pk].grid <= 0) continue;
        const double target = total[pk] / ((double)part[pk].grid * part[pk].spw);
        for (int k = 0; k < n_jobs; ++k) {
            if ((jobs[k].jd.g.narrow ? 0 : 1) != pk) continue;
            job_seg[2 * k] = (int32_t)segs.size();
            const int64_t F = jobs[k].jd.F;
            int64_t per = (int64_t)(target / cost[k]);
            if (per < 64) per = 64;
            for (int64_t f = 0; f < F; f += per) segs.push_back(BatchSeg{k, 0, f, f + per < F ? f + per : F});
            job_seg[2 * k + 1] = (int32_t)segs.size();
        }
    }
}

}  // namespace vjb

struct boost_batch {
    int n_jobs = 0;
    std::vector<JobHost> jobs;
    BatchDev bd;
    boost_stump* gather = nullptr;
    PartCfg part[2];
    int num_cu = 0, device = 0;
    size_t max_segs = 0;
    int64_t n_upd = 0;
    hipStream_t stream = nullptr;
    boost_options opts;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    std::vector<hipEvent_t> ev;
    double t_scan = 0, t_upd = 0, rounds_timed = 0;
    int64_t launched = 0;
};

// Builds the segment tables for the current part configurations and copies
// them to the device (stream-ordered).
static int upload_segments(boost_batch* b) {
    std::vector<BatchSeg> segs;
    std::vector<int32_t> job_seg;
    int32_t split = 0;
    build_segments(b->jobs, b->part, segs, job_seg, split);
    if (segs.size() > b->max_segs) { set_error("segment table overflow"); return BOOST_E_INVALID; }
    b->bd.n_segs = (int32_t)segs.size();
    b->bd.seg_split = split;
    VJB_HIP(hipMemcpyAsync((void*)b->bd.segs, segs.data(), segs.size() * sizeof(BatchSeg), hipMemcpyHostToDevice,
                           b->stream));
    VJB_HIP(hipMemcpyAsync((void*)b->bd.job_seg, job_seg.data(), job_seg.size() * 4, hipMemcpyHostToDevice, b->stream));
    VJB_HIP(hipStreamSynchronize(b->stream));   // the host vectors end here
    return BOOST_OK;
}

static int launch_part(boost_batch* b, int p) {
    return batch_scan_launch(b->part[p].kernel, b->part[p].grid, b->part[p].wg, b->bd, p, b->stream);
}

// Measured choice for one key format, by successive halving: every schedule
// (default segment granularity) is timed once, the three fastest twice more,
// then the winner with the other segment granularities (twice each).  Each
// configuration first runs a short untimed launch over its last `grid`
// segments (instruction cache and first-launch costs); the minimum counts.
static int tune_part(boost_batch* b, int p) {
    std::string key = "batch/" + tune_device_tag(b->device) + "/" + std::to_string(b->opts.precision) + "/" +
                      std::to_string(p);
    for (const JobHost& h : b->jobs)
        if ((h.jd.g.narrow ? 0 : 1) == p) key += "/" + std::to_string(h.jd.g.n) + "x" + std::to_string(h.jd.F);
    std::vector<int> hit;
    int rc;
    PartCfg cached;
    if (tune_cache_get(key, hit) && hit.size() == 2 && hit[0] >= 0 && hit[0] < scan_schedule_count() &&
        scan_schedule_lanes(hit[0]) == scan_schedule_lanes(b->part[p].schedule) && hit[1] >= 1 &&
        hit[1] <= kMaxSegsPerWg && part_config(cached, b->opts.precision, p == 0, hit[0], b->num_cu) == BOOST_OK) {
        cached.spw = hit[1];   // entries that do not fit are ignored and re-tuned
        b->part[p] = cached;
        return upload_segments(b);
    }
    auto time_cfg = [&](const PartCfg& pc, int reps, double& ms) -> int {
        b->part[p] = pc;
        int r = upload_segments(b);
        if (r != BOOST_OK) return r;
        VJB_HIP(hipMemsetAsync(b->bd.next_seg + p, 0, 4, b->stream));
        if ((r = batch_scan_launch(pc.kernel, pc.grid, pc.wg, b->bd, p, b->stream, pc.grid)) != BOOST_OK) return r;
        return time_launches(b->stream, reps, [&]() -> int {
            VJB_HIP(hipMemsetAsync(b->bd.next_seg + p, 0, 4, b->stream));
            return launch_part(b, p);
        }, ms, false);
    };
    struct Cand { PartCfg pc; double ms; };
    std::vector<Cand> cands;
    const int lanes = scan_schedule_lanes(b->part[p].schedule);
    for (int k = 0; k < scan_schedule_count(); ++k) {
        if (scan_schedule_lanes(k) != lanes) continue;
        Cand c;
        if (part_config(c.pc, b->opts.precision, p == 0, k, b->num_cu) != BOOST_OK) continue;
        if ((rc = time_cfg(c.pc, 1, c.ms)) != BOOST_OK) return rc;
        cands.push_back(c);
    }
    if (cands.empty()) { set_error("no batched scan schedule fits"); return BOOST_E_INVALID; }
    std::stable_sort(cands.begin(), cands.end(), [](const Cand& x, const Cand& y) { return x.ms < y.ms; });
    if (cands.size() > 3) cands.resize(3);
    for (Cand& c : cands) {
        double ms = 0;
        if ((rc = time_cfg(c.pc, 2, ms)) != BOOST_OK) return rc;
        if (ms < c.ms) c.ms = ms;
    }
    Cand best = *std::min_element(cands.begin(), cands.end(), [](const Cand& x, const Cand& y) { return x.ms < y.ms; });
    static const int kSpw[] = {4, 8, 32};   // besides the default kSegsPerWg
    const PartCfg winner = best.pc;
    for (int spw : kSpw) {
        PartCfg pc = winner;
        pc.spw = spw;
        double ms = 0;
        if ((rc = time_cfg(pc, 2, ms)) != BOOST_OK) return rc;
        if (ms < best.ms) { best.ms = ms; best.pc = pc; }
    }
    b->part[p] = best.pc;
    tune_cache_put(key, {best.pc.schedule, best.pc.spw});
    return upload_segments(b);
}

extern "C" {

size_t boost_batch_workspace_bytes(int32_t n_jobs, const boost_job* jobs, const boost_options* o) {
    if (check_batch(n_jobs, jobs, o) != BOOST_OK) return 0;
    BatchLayout L;
    batch_layout(n_jobs, jobs, L);
    return L.total;
}

int boost_batch_init(boost_batch** out, int32_t n_jobs, const boost_job* jobs, const boost_options* o,
                     void* d_workspace, size_t workspace_bytes) {
    if (!out || !d_workspace) { set_error("NULL pointer argument"); return BOOST_E_INVALID; }
    *out = nullptr;
    int rc = check_batch(n_jobs, jobs, o);
    if (rc != BOOST_OK) return rc;
    for (int k = 0; k < n_jobs; ++k)
        if (!jobs[k].d_images || !jobs[k].d_labels) { set_error("NULL job input"); return BOOST_E_INVALID; }
    BatchLayout L;
    batch_layout(n_jobs, jobs, L);
    if (workspace_bytes < L.total) {
        set_error("workspace too small: need " + std::to_string(L.total) + " bytes");
        return BOOST_E_NOMEM;
    }
    boost_batch* b = new boost_batch();
    // on failure, work already queued on the stream finishes before the call
    // returns: the caller may free the workspace right away
    auto fail = [&](int code) {
        if (b->stream) (void)hipStreamSynchronize(b->stream); else (void)hipDeviceSynchronize();
        delete b;
        return code;
    };
    b->n_jobs = n_jobs;
    b->opts = *o;
    b->stream = (hipStream_t)o->stream;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&b->num_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        set_error("no HIP device");
        return fail(BOOST_E_DEVICE);
    }
    b->device = dev;
    char* ws = (char*)d_workspace;
    b->jobs.resize(n_jobs);
    for (int k = 0; k < n_jobs; ++k) {
        rc = setup_job(b->jobs[k], ws + L.job_off[k], jobs[k].n, &jobs[k].fs, o, jobs[k].d_images, jobs[k].d_labels,
                       b->num_cu, b->stream);
        if (rc != BOOST_OK) { set_error("job " + std::to_string(k) + ": " + get_error()); return fail(rc); }
    }
    // device tables
    std::vector<JobDev> hj(n_jobs);
    for (int k = 0; k < n_jobs; ++k) hj[k] = b->jobs[k].jd;
    std::vector<int32_t> upd_job, upd_part;
    for (int k = 0; k < n_jobs; ++k)
        for (int p = 0; p < b->jobs[k].jd.n_part; ++p) { upd_job.push_back(k); upd_part.push_back(p); }
    b->n_upd = (int64_t)upd_job.size();
    b->max_segs = L.max_segs;
    BatchDev& bd = b->bd;
    bd.jobs = (const JobDev*)(ws + L.jobs);
    bd.segs = (const BatchSeg*)(ws + L.segs);
    bd.next_seg = (uint32_t*)(ws + L.next_seg);
    bd.job_seg = (const int32_t*)(ws + L.job_seg);
    bd.seg_best = (WgBest*)(ws + L.seg_best);
    bd.upd_job = (const int32_t*)(ws + L.upd_job);
    bd.upd_part = (const int32_t*)(ws + L.upd_part);
    b->gather = (boost_stump*)(ws + L.gather);
    if (hipMemcpyAsync((void*)bd.jobs, hj.data(), hj.size() * sizeof(JobDev), hipMemcpyHostToDevice, b->stream) != hipSuccess ||
        hipMemsetAsync(bd.next_seg, 0, 8, b->stream) != hipSuccess ||
        hipMemcpyAsync((void*)bd.upd_job, upd_job.data(), upd_job.size() * 4, hipMemcpyHostToDevice, b->stream) != hipSuccess ||
        hipMemcpyAsync((void*)bd.upd_part, upd_part.data(), upd_part.size() * 4, hipMemcpyHostToDevice, b->stream) != hipSuccess) {
        set_error("copying the batch tables failed");
        return fail(BOOST_E_DEVICE);
    }
    // one scan launch per key format present, with its schedule
    bool present[2] = {false, false};
    for (int k = 0; k < n_jobs; ++k) present[b->jobs[k].jd.g.narrow ? 0 : 1] = true;
    const int sched0 = o->schedule_id == BOOST_SCHEDULE_AUTO ? 0 : o->schedule_id;
    for (int p = 0; p < 2; ++p)
        if (present[p] && (rc = part_config(b->part[p], o->precision, p == 0, sched0, b->num_cu)) != BOOST_OK)
            return fail(rc);
    if ((rc = upload_segments(b)) != BOOST_OK) return fail(rc);
    if (o->schedule_id == BOOST_SCHEDULE_AUTO)
        for (int p = 0; p < 2; ++p)
            if (present[p] && (rc = tune_part(b, p)) != BOOST_OK) return fail(rc);
    if (hipMemsetAsync(bd.next_seg, 0, 8, b->stream) != hipSuccess || hipStreamSynchronize(b->stream) != hipSuccess) {
        set_error("device error during batch init");
        return fail(BOOST_E_DEVICE);
    }
    *out = b;
    return BOOST_OK;
}

static int batch_launch(boost_batch* b, hipEvent_t e0, hipEvent_t e1, hipEvent_t e2) {
    int rc;
    if (e0) VJB_HIP(hipEventRecord(e0, b->stream));
    for (int p = 0; p < 2; ++p)
        if (b->part[p].kernel && (rc = launch_part(b, p)) != BOOST_OK) return rc;
    if (e1) VJB_HIP(hipEventRecord(e1, b->stream));
    if ((rc = batch_update_launch(b->opts.precision, (int)b->n_upd, b->bd, b->stream)) != BOOST_OK) return rc;
    if (e2) VJB_HIP(hipEventRecord(e2, b->stream));
    b->launched++;
    return BOOST_OK;
}

static int batch_graph(boost_batch* b) {
    if (b->gexec) return BOOST_OK;
    VJB_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    int rc = BOOST_OK;
    for (int p = 0; p < 2 && rc == BOOST_OK; ++p)
        if (b->part[p].kernel) rc = launch_part(b, p);
    if (rc == BOOST_OK) rc = batch_update_launch(b->opts.precision, (int)b->n_upd, b->bd, b->stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (rc != BOOST_OK) { if (g) (void)hipGraphDestroy(g); return rc; }
    if (e != hipSuccess) { set_error(std::string("graph capture: ") + hipGetErrorString(e)); return BOOST_E_DEVICE; }
    b->graph = g;
    VJB_HIP(hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0));
    return BOOST_OK;
}

static int batch_copy_records(boost_batch* b, int64_t first, int count, boost_stump* dst) {
    int rc = batch_gather_launch(b->bd, b->n_jobs, first, count, b->gather, b->stream);
    if (rc != BOOST_OK) return rc;
    VJB_HIP(hipMemcpyAsync(dst, b->gather, (size_t)count * b->n_jobs * sizeof(boost_stump), hipMemcpyDeviceToHost,
                           b->stream));
    VJB_HIP(hipStreamSynchronize(b->stream));
    return BOOST_OK;
}

int boost_batch_train(boost_batch* b, int32_t rounds, boost_stump* out_host) {
    if (!b) { set_error("NULL batch"); return BOOST_E_INVALID; }
    if (rounds < 0) { set_error("rounds must be >= 0"); return BOOST_E_INVALID; }
    int rc;
    const bool timing = (b->opts.flags & BOOST_FLAG_TIMING) != 0;
    const bool graph = !timing && !(b->opts.flags & BOOST_FLAG_NO_GRAPH) && b->stream != nullptr;
    if (graph && (rc = batch_graph(b)) != BOOST_OK) return rc;
    int32_t done = 0;
    while (done < rounds) {
        const int chunk = (rounds - done) < kGatherRounds ? (rounds - done) : kGatherRounds;
        const int64_t first = b->launched;
        while (timing && b->ev.size() < 3 * (size_t)chunk) {
            hipEvent_t e;
            VJB_HIP(hipEventCreate(&e));
            b->ev.push_back(e);
        }
        for (int r = 0; r < chunk; ++r) {
            if (graph) {
                VJB_HIP(hipGraphLaunch(b->gexec, b->stream));
                b->launched++;
            } else if ((rc = batch_launch(b, timing ? b->ev[3 * r] : nullptr, timing ? b->ev[3 * r + 1] : nullptr,
                                          timing ? b->ev[3 * r + 2] : nullptr)) != BOOST_OK) {
                return rc;
            }
        }
        if (timing) {
            VJB_HIP(hipEventSynchronize(b->ev[3 * (chunk - 1) + 2]));
            for (int r = 0; r < chunk; ++r) {
                float x = 0, y = 0;
                VJB_HIP(hipEventElapsedTime(&x, b->ev[3 * r], b->ev[3 * r + 1]));
                VJB_HIP(hipEventElapsedTime(&y, b->ev[3 * r + 1], b->ev[3 * r + 2]));
                b->t_scan += x;
                b->t_upd += y;
            }
            b->rounds_timed += chunk;
        }
        if (out_host && (rc = batch_copy_records(b, first, chunk, out_host + (size_t)done * b->n_jobs)) != BOOST_OK)
            return rc;
        done += chunk;
    }
    return BOOST_OK;
}

int boost_batch_round(boost_batch* b, boost_stump* out_host) { return boost_batch_train(b, 1, out_host); }

int boost_batch_get_weights(boost_batch* b, int32_t job, double* d_w) {
    if (!b || !d_w || job < 0 || job >= b->n_jobs) { set_error("invalid batch, job or output"); return BOOST_E_INVALID; }
    return get_weights_launch(b->jobs[job].jd, d_w, b->stream);
}

int boost_batch_get_schedule(const boost_batch* b, int32_t key_format, int32_t* schedule, int32_t* segs_per_wg) {
    if (!b || !schedule || key_format < 0 || key_format > 1) {
        set_error("invalid batch, key format or output");
        return BOOST_E_INVALID;
    }
    const PartCfg& pc = b->part[key_format];
    *schedule = pc.kernel ? pc.schedule : -1;
    if (segs_per_wg) *segs_per_wg = pc.kernel ? pc.spw : 0;
    return BOOST_OK;
}

int boost_batch_get_timing(boost_batch* b, double out[4]) {
    if (!b || !out) { set_error("NULL argument"); return BOOST_E_INVALID; }
    VJB_HIP(hipStreamSynchronize(b->stream));
    out[0] = b->t_scan; out[1] = b->t_upd; out[2] = b->rounds_timed; out[3] = b->rounds_timed;
    return BOOST_OK;
}

void boost_batch_destroy(boost_batch* b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream); else (void)hipDeviceSynchronize();
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (hipEvent_t e : b->ev) (void)hipEventDestroy(e);
    delete b;
}

}  // extern "C"
