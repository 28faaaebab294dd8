// Host launchers of the library's kernels (one translation unit per kernel family).
#pragma once

#include <functional>
#include <string>
#include <vector>

#include "common.h"

namespace vjb {

constexpr int kMaxScanGrid = 8192;   // upper bound of scan workgroups (per-workgroup records)
constexpr int kMaxClassifyT = 4096;  // stumps per classifier call
constexpr int kMaxSortGrid = 1024;   // upper bound of sort workgroups (fallback scratch)
constexpr int kMaxPart = (int)((kMaxN + kUpdWg - 1) / kUpdWg);   // update workgroups of the largest job (<= 128)
static_assert(kMaxPart <= 128, "weight_sum reads at most 128 partials");

struct StumpDev { uint32_t desc; int32_t polarity; int32_t theta; int32_t pad; double alpha; };

struct ScanPlan {
    const void* kernel = nullptr;
    int wg = 0;
    int grid = 0;
    size_t lds = 0;
};

// api.cpp: one job's layout and one-time preparation (shared by the batch)
struct JobHost {
    JobDev jd;
    double* wtmp;
    StumpDev* cls;
    uint64_t* scratch;       // the 64-bit sort path's scratch (n > kNarrowMaxN), else NULL
    const uint32_t* sorder;  // the order the one-time preparation visits the features
    uint32_t* defer;         // features left to the 64-bit sort path (n > kNarrowMaxN), else NULL
    int64_t n_pos;
    bool merged;
};
// A prepared job that a new job extends: the new job's windows are the old
// job's (in its caller order) followed by the new ones.
struct ExtendSrc { const JobDev* old; int64_t l0; };
// A union of more than kMergeMinN and at most kMergeMaxN windows that adds
// at most kMergeMaxM merges the old keys with the sorted new windows; any
// other is sorted in full, which is faster there: the merge still evaluates
// every window, its ranking of the new windows grows as m^2, and below
// kMergeMinN the sort's smaller workgroup shapes beat its 1,024 x 11 slots
// (measured crossovers: about 250 new windows at 10,000 and 14,500 old ones;
// none at 2,000).
constexpr int64_t kMergeMinN = 1024 * 7;
constexpr int64_t kMergeMaxN = 1024 * 15;
constexpr int64_t kMergeMaxM = 256;
int check_job_args(int64_t n, const boost_feature_set* fs, const boost_options* o);
size_t job_bytes(int64_t n, const boost_feature_set* fs);
// ext == NULL: a job of d_images / d_labels (n windows).  Otherwise the union
// of ext's job and the n - ext->old->g.n windows of d_images / d_labels.
int setup_job(JobHost& h, char* ws, int64_t n, const boost_feature_set* fs, const boost_options* o,
              const uint8_t* d_images, const uint8_t* d_labels, int num_cu, hipStream_t s,
              const ExtendSrc* ext = nullptr);

// k_scan.hip
int scan_schedule_count();
int scan_schedule_wg(int schedule);
int scan_schedule_lanes(int schedule);
int scan_schedule_unroll(int schedule);
int64_t scan_table_capacity(int precision, bool narrow);
int scan_plan(ScanPlan& p, int precision, bool narrow, int schedule, int64_t n, int64_t F, int num_cu);
int scan_launch(const ScanPlan& p, const JobDev& jd, double2* ferr, hipStream_t s);
int update_launch(const JobDev& jd, int n_wg, hipStream_t s);

// k_probe.hip: reads every key with the scan's access pattern and no arithmetic
// (one word per workgroup to sink[grid])
int probe_launch(const ScanPlan& p, int schedule, const JobDev& jd, uint32_t* sink, hipStream_t s);

// tune.cpp: measured schedule choice
constexpr int kTuneReps = 5;        // timed launches per candidate of a single job (the minimum counts)
constexpr double kTunePrune = 1.03;  // a single job's candidates this much slower than the best stop after two rounds
// Runs launch() once untimed (when warm), then `reps` times each bracketed by
// HIP events on s; best_ms is the fastest.
int time_launches(hipStream_t s, int reps, const std::function<int()>& launch, double& best_ms, bool warm = true);
std::string tune_device_tag(int device);   // architecture, compute units, schedule table revision
bool tune_cache_get(const std::string& key, std::vector<int>& choice);
void tune_cache_put(const std::string& key, const std::vector<int>& choice);
// Times every schedule with the job's lane count; ms_out[k] = -1 for schedules
// not tried (or when the choice came from the cache).
int tune_single(const JobDev& jd, int precision, int num_cu, int device, hipStream_t s, double* ms_out, int& chosen);

// k_prep.hip
int ingest_launch(const JobDev& jd, const uint8_t* d_labels, int64_t n, hipStream_t s);
int integral_launch(const JobDev& jd, const uint8_t* d_images, hipStream_t s);
int init_weights_launch(const JobDev& jd, hipStream_t s);
int set_weights_launch(const JobDev& jd, const double* d_w, double* tmp, hipStream_t s);
int get_weights_launch(const JobDev& jd, double* d_out, hipStream_t s);
int feature_values_launch(const JobDev& jd, int64_t j0, int64_t nf, int32_t* d_out, hipStream_t s);
int integral_out_launch(const JobDev& jd, int32_t* d_out, hipStream_t s);
int sorted_out_launch(const JobDev& jd, int64_t j0, int64_t nf, int32_t* d_order, uint8_t* d_flags, hipStream_t s);
// integral images of n windows (images n x H x W row-major; window perm[i] at
// sample i, or window i when perm is NULL) into ii[(H+1)(W+1)][S]
int integral_raw_launch(const uint8_t* d_images, const int32_t* perm, int64_t n, int W, int H, int32_t* ii, int64_t S,
                        hipStream_t s);

// k_classify.hip: the strong classifier over n windows of sample-minor
// integral images; labels (caller order) or, when NULL and l >= 0, y = [i < l];
// perm maps sample i to the caller's index (NULL: identity).  d_curve[t] =
// windows misclassified by the first t + 1 stumps (needs labels or l >= 0).
int classify_any_launch(const int32_t* ii, int64_t S, int W, int64_t n, const StumpDev* d_stumps, int T,
                        const int32_t* perm, const uint8_t* labels, int64_t l, uint8_t* d_out, double* d_score,
                        int32_t* d_curve, hipStream_t s);

// extending a job by m windows (the union's caller order: old windows, then new)
int union_labels_launch(const JobDev& old, int64_t l0, const uint8_t* d_new_labels, int64_t m, uint8_t* d_out,
                        hipStream_t s);
int extend_ii_launch(const JobDev& jd, const JobDev& old, const uint8_t* d_new_images, hipStream_t s);
// keys of the union from the old keys (union <= 15,360 windows, old keys narrow)
int merge_launch(const JobDev& jd, const uint32_t* sorder, const uint4* old_keys, const KeyGeom& og, int l0, int lm, int num_cu,
                 hipStream_t s);

// k_sort.hip
int64_t sort_pow2(int64_t n);
size_t sort_scratch_bytes(int64_t n);
// defer: F + 16 words for jobs of more than kNarrowMaxN windows (the features
// the counting sort leaves to the 64-bit path), NULL otherwise.
int sort_launch(const JobDev& jd, const uint32_t* sorder, uint64_t* scratch, uint32_t* defer, int num_cu,
                hipStream_t s);

}  // namespace vjb
