// Batched jobs: device tables and launchers shared by batch.cpp and k_batch.hip.
#pragma once

#include "launch.h"

namespace vjb {

// A contiguous feature range [f0, f1) of one job, scanned by one workgroup.
struct BatchSeg {
    int32_t job;
    int32_t pad;
    int64_t f0, f1;
};

struct BatchDev {
    const JobDev* jobs;      // [n_jobs]
    const BatchSeg* segs;    // [n_segs]: the 14-bit-key jobs' segments, then the 15-bit ones; per job in feature order
    uint32_t* next_seg;      // [2] work-queue counters of the two scan launches (reset by the update launch)
    int32_t seg_split;       // segments [0, seg_split) are 14-bit-key jobs', [seg_split, n_segs) 15-bit
    int32_t n_segs;
    const int32_t* job_seg;  // [2 * n_jobs]: segments of job k are job_seg[2k] .. job_seg[2k+1]-1
    WgBest* seg_best;        // [n_segs]
    const int32_t* upd_job;  // [n_upd]: job of each update workgroup
    const int32_t* upd_part; // [n_upd]: its index within the job
};

constexpr int kGatherRounds = 256;   // records gathered per copy
constexpr int kSegsPerWg = 16;       // work-queue granularity without tuning: segments per scan workgroup on average
constexpr int kMaxSegsPerWg = 32;    // the largest granularity the tuner tries
constexpr int kMaxJobs = 4096;

const void* batch_scan_kernel(int precision, bool narrow, int schedule);
// part 0: the 14-bit-key jobs' segments, part 1: the 15-bit ones
// last > 0: only the part's last `last` segments (a short warm-up launch of
// the tuner; the other segments' results are left as they were).
int batch_scan_launch(const void* kernel, int grid, int wg, const BatchDev& b, int part, hipStream_t s,
                      int last = 0);
int batch_update_launch(int precision, int n_upd, const BatchDev& b, hipStream_t s);
int batch_gather_launch(const BatchDev& b, int n_jobs, int64_t first, int count, boost_stump* out, hipStream_t s);

}  // namespace vjb
