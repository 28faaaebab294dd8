// Measured choice of launch schedules (BOOST_SCHEDULE_AUTO).
//
// A scan launch only reads the keys and the current weights and rewrites the
// same per-round scratch (workgroup records, the state's sums), so it can be
// repeated before the first update without changing any result.  The tuner
// times each candidate on the job's own keys with HIP events and keeps the
// fastest; results are cached by workload shape (per process, and in a file
// when VJBOOST_TUNE_CACHE names one) so that jobs of the same shape are tuned
// once.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

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

// The cache: in process memory, and, when the environment variable
// VJBOOST_TUNE_CACHE names a file, also in that file (one "key value ..."
// line per choice, appended as choices are made; read on the first lookup
// that misses in memory).  Keys name the device by its architecture and
// compute-unit count, and the library's schedule table by its size and a
// revision number, so a file can be shared between processes and boxes of
// the same kind; a later line for the same key wins.
static std::mutex g_tune_mu;
static std::map<std::string, std::vector<int>> g_tune_cache;
static bool g_file_loaded = false;
constexpr int kTuneRevision = 2;   // bump when the schedules' meaning changes

static const char* cache_path() {
    const char* p = getenv("VJBOOST_TUNE_CACHE");
    return p != nullptr && p[0] != 0 ? p : nullptr;
}

static void load_file_locked() {
    if (g_file_loaded) return;
    g_file_loaded = true;
    const char* path = cache_path();
    if (!path) return;
    FILE* f = fopen(path, "r");
    if (!f) return;
    char line[1024];
    while (fgets(line, sizeof line, f)) {
        char* save = nullptr;
        char* tok = strtok_r(line, " \t\r\n", &save);
        if (!tok || tok[0] == '#') continue;
        std::string key = tok;
        std::vector<int> v;
        bool ok = true;
        while ((tok = strtok_r(nullptr, " \t\r\n", &save)) != nullptr) {
            char* end = nullptr;
            const long x = strtol(tok, &end, 10);
            if (end == tok || *end != 0 || x < -1000000 || x > 1000000) { ok = false; break; }
            v.push_back((int)x);
        }
        if (ok && !v.empty()) g_tune_cache[key] = v;
    }
    fclose(f);
}

std::string tune_device_tag(int device) {
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    int cus = 0;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        arch = prop.gcnArchName;
        cus = prop.multiProcessorCount;
        for (char& ch : arch)
            if (ch == ' ' || ch == '/' || ch == '\t') ch = '_';
    }
    return "r" + std::to_string(kTuneRevision) + "/s" + std::to_string(scan_schedule_count()) + "/" + arch + "/" +
           std::to_string(cus);
}

bool tune_cache_get(const std::string& key, std::vector<int>& choice) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it == g_tune_cache.end()) {
        load_file_locked();
        it = g_tune_cache.find(key);
        if (it == g_tune_cache.end()) return false;
    }
    choice = it->second;
    return true;
}

void tune_cache_put(const std::string& key, const std::vector<int>& choice) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = choice;
    const char* path = cache_path();
    if (!path) return;
    std::string line = key;
    for (int v : choice) line += " " + std::to_string(v);
    line += "\n";
    FILE* f = fopen(path, "a");   // one short append per choice; a failure only loses persistence
    if (!f) return;
    fputs(line.c_str(), f);
    fclose(f);
}

void tune_cache_clear() {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache.clear();
    g_file_loaded = false;   // the next miss reads the file again
}

int tune_single(const JobDev& jd, int precision, int num_cu, int device, hipStream_t s, double* ms_out,
                int& chosen) {
    const int lanes = jd.g.lanes;
    const std::string key = "job/" + tune_device_tag(device) + "/" + std::to_string(precision) + "/" +
                            std::to_string(lanes) + "/" + std::to_string(jd.g.n) + "/" + std::to_string(jd.F);
    for (int k = 0; k < scan_schedule_count(); ++k) ms_out[k] = -1.0;
    std::vector<int> hit;
    ScanPlan probe;
    if (tune_cache_get(key, hit) && hit.size() == 1 && hit[0] >= 0 && hit[0] < scan_schedule_count() &&
        scan_schedule_lanes(hit[0]) == lanes &&
        scan_plan(probe, precision, jd.g.narrow != 0, hit[0], jd.g.n, jd.F, num_cu) == BOOST_OK) {
        chosen = hit[0];   // a choice from the cache (entries that do not fit are ignored and re-tuned)
        return BOOST_OK;
    }
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
