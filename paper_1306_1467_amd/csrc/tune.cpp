// Measured choice of launch schedules (BOOST_SCHEDULE_AUTO).
//
// A scan launch only reads the keys and the current weights and rewrites the
// same per-round scratch (workgroup records, the state's sums), so it can be
// repeated before the first update without changing any result.  The tuner
// times each candidate on the job's own keys with HIP events and keeps the
// fastest; results are cached per process by workload shape so that jobs of
// the same shape are tuned once.
#include <map>
#include <mutex>
#include <string>

#include "launch.h"

namespace vjb {

int time_launches(hipStream_t s, int reps, const std::function<int()>& launch, double& best_ms, bool warm) {
    hipEvent_t e[2];
    VJB_HIP(hipEventCreate(&e[0]));
    if (hipEventCreate(&e[1]) != hipSuccess) {
        (void)hipEventDestroy(e[0]);
        set_error("hipEventCreate failed");
        return BOOST_E_DEVICE;
    }
    int rc = warm ? launch() : BOOST_OK;   // untimed: first-touch and instruction-cache warm-up
    best_ms = 1e300;
    for (int r = 0; r < reps && rc == BOOST_OK; ++r) {
        float ms = 0;
        if (hipEventRecord(e[0], s) != hipSuccess) { rc = BOOST_E_DEVICE; break; }
        if ((rc = launch()) != BOOST_OK) break;
        if (hipEventRecord(e[1], s) != hipSuccess || hipEventSynchronize(e[1]) != hipSuccess ||
            hipEventElapsedTime(&ms, e[0], e[1]) != hipSuccess) {
            rc = BOOST_E_DEVICE;
            break;
        }
        if (ms < best_ms) best_ms = ms;
    }
    if (rc == BOOST_E_DEVICE) set_error("timing a candidate schedule failed");
    (void)hipEventDestroy(e[0]);
    (void)hipEventDestroy(e[1]);
    return rc;
}

static std::mutex g_tune_mu;
static std::map<std::string, std::vector<int>> g_tune_cache;

bool tune_cache_get(const std::string& key, std::vector<int>& choice) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it == g_tune_cache.end()) return false;
    choice = it->second;
    return true;
}

void tune_cache_put(const std::string& key, const std::vector<int>& choice) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = choice;
}

void tune_cache_clear() {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache.clear();
}

int tune_single(const JobDev& jd, int precision, int num_cu, int device, hipStream_t s, double* ms_out,
                int& chosen) {
    const int lanes = jd.g.lanes;
    const std::string key = "job/" + std::to_string(device) + "/" + std::to_string(precision) + "/" +
                            std::to_string(lanes) + "/" + std::to_string(jd.g.n) + "/" + std::to_string(jd.F);
    for (int k = 0; k < scan_schedule_count(); ++k) ms_out[k] = -1.0;
    std::vector<int> hit;
    if (tune_cache_get(key, hit)) { chosen = hit[0]; return BOOST_OK; }
    std::vector<int> ids;
    std::vector<ScanPlan> plans;
    for (int k = 0; k < scan_schedule_count(); ++k) {
        if (scan_schedule_lanes(k) != lanes) continue;
        ScanPlan p;
        if (scan_plan(p, precision, jd.g.narrow != 0, k, jd.g.n, jd.F, num_cu) != BOOST_OK) continue;   // does not fit
        ids.push_back(k);
        plans.push_back(p);
    }
    if (ids.empty()) { set_error("no launch schedule fits this job"); return BOOST_E_INVALID; }
    // candidates are timed in turn, kTuneReps rounds over all of them, in
    // alternating order, so that slow drifts of the clock (it is still rising
    // in the first rounds) do not favour one; each keeps its fastest launch.
    // Round 0 only warms every candidate up (one untimed launch).  After two
    // timed rounds, candidates more than kTunePrune slower than the fastest
    // are not timed again (run-to-run noise is about 1 %).
    std::vector<double> best(ids.size(), 1e300);
    std::vector<char> alive(ids.size(), 1);
    int rc;
    for (int rep = 0; rep <= kTuneReps; ++rep) {
        for (size_t i = 0; i < ids.size(); ++i) {
            const size_t c = rep % 2 ? i : ids.size() - 1 - i;
            if (!alive[c]) continue;
            double ms = 0;
            if ((rc = time_launches(s, rep == 0 ? 0 : 1, [&]() { return scan_launch(plans[c], jd, nullptr, s); }, ms,
                                    rep == 0)) != BOOST_OK)
                return rc;
            if (rep > 0 && ms < best[c]) best[c] = ms;
        }
        if (rep == 2) {
            double bmin = 1e300;
            for (size_t c = 0; c < ids.size(); ++c) bmin = best[c] < bmin ? best[c] : bmin;
            for (size_t c = 0; c < ids.size(); ++c) alive[c] = best[c] <= bmin * kTunePrune;
        }
    }
    size_t win = 0;
    for (size_t c = 0; c < ids.size(); ++c) {
        ms_out[ids[c]] = best[c];
        if (best[c] < best[win]) win = c;
    }
    chosen = ids[win];
    tune_cache_put(key, {chosen});
    return BOOST_OK;
}

}  // namespace vjb

extern "C" void boost_tune_cache_clear(void) { vjb::tune_cache_clear(); }
