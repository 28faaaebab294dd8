// Batched rounds: many independent jobs (own windows, labels, feature sets)
// advance one boosting round with one persistent scan launch per key format
// (jobs with 14-bit keys, jobs with 15-bit keys) and one update launch for
// all of them.
//
// The scan's work is cut into segments (job, feature range) of about the same
// cost; workgroups take segments from a work queue (an atomic counter; every
// workgroup stops once the counter passes the last segment), refilling the
// LDS weight table when the segment's job differs from the previous one
// (normalisation, Section 2.3 step 1), and leave one candidate per segment.
// The update launch runs one workgroup per 256 windows of every job; each
// takes the argmin over its job's segment candidates (Section 3.3.2 step 4a)
// and updates its windows (Section 2.3 step 4).  Per job, the arithmetic is
// that of the single-job kernels, so the stumps equal those of the job run
// alone.
#include "batch.h"
#include "update_core.h"

namespace vjb {

// One launch per key format: NARROW selects the 14-bit-key jobs (64 KiB
// table, two workgroups per compute unit) or the 15-bit ones (128 KiB).
// Segments [s_begin, s_end) belong to this launch; the counter counts from 0.
template <int PREC, bool NARROW, int WG, int UNROLL, int LPF, bool RING>
__global__ __launch_bounds__(WG, (ScanOccupancy<PREC, NARROW, WG, UNROLL, true, RING>::waves_per_eu)) void k_scan_batch(
    const JobDev* __restrict__ jobs, const BatchSeg* __restrict__ segs, uint32_t* __restrict__ next_seg, int s_begin,
    int s_end, const int32_t* __restrict__ job_seg, WgBest* __restrict__ seg_best) {
    using Wt = typename ScanTypes<PREC>::W;
    constexpr int NG = (WG / 64) * (64 / LPF);
    __shared__ ScanLds<Wt, TabCap<PREC, NARROW>::value, NG> lds;
    __shared__ int32_t s_next;
    Wt* tab = lds.tab;
    const int tid = threadIdx.x, wv = tid >> 6;
    int cur_job = -1;
    double tp = 0.0, tn = 0.0;
    while (true) {
        if (tid == 0) s_next = s_begin + (int32_t)atomicAdd(next_seg, 1u);
        __syncthreads();
        const int s = __builtin_amdgcn_readfirstlane(s_next);   // uniform: descriptor loads stay scalar
        if (s >= s_end) break;
        const BatchSeg sg = segs[s];
        const JobDev& jd = jobs[sg.job];   // fields read on demand (scalar loads)
        WgBest best{DBL_MAX, -1, 0, -1};
        if (!jd.st->stopped) {
            if (sg.job != cur_job) {
                const int par = jd.st->wpar;
                const double S = weight_sum(jd);
                fill_table<PREC>(jd, weights(jd, par), tab, 1.0 / S, WG, lds.sh, tp, tn);
                if (s == job_seg[2 * sg.job] && tid == 0) {
                    jd.st->sum_w = S; jd.st->t_pos = tp; jd.st->t_neg = tn; jd.st->cur = par;
                }
                cur_job = sg.job;
            }
            best = scan_range<PREC, NARROW, UNROLL, LPF, RING>(jd, tab, sg.f0, sg.f1, wv, WG / 64, tp, tn, nullptr);
        }
        const WgBest b = block_best<NG>(lds.wb, best, LPF);
        if (tid == 0) seg_best[s] = b;
        __syncthreads();   // s_next and the per-group records are reused
    }
}

template <int PREC>
__global__ __launch_bounds__(kUpdWg) void k_update_batch(const JobDev* __restrict__ jobs,
                                                         uint32_t* __restrict__ next_seg,
                                                         const int32_t* __restrict__ upd_job,
                                                         const int32_t* __restrict__ upd_part,
                                                         const int32_t* __restrict__ job_seg,
                                                         const WgBest* __restrict__ seg_best) {
    if (blockIdx.x == 0 && threadIdx.x < 2) next_seg[threadIdx.x] = 0u;   // the next round's scan queues
    const int k = upd_job[blockIdx.x];
    const JobDev& jd = jobs[k];
    const int s0 = job_seg[2 * k], s1 = job_seg[2 * k + 1];
    update_body<PREC>(jd, seg_best + s0, s1 - s0, upd_part[blockIdx.x]);
}

// Records of launches first .. first+count-1 of every job into out[r][job].
__global__ void k_gather_records(const JobDev* __restrict__ jobs, int n_jobs, int64_t first, int count,
                                 boost_stump* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n_jobs * count) return;
    const int r = (int)(t / n_jobs), k = (int)(t % n_jobs);
    out[t] = jobs[k].ring[(first + r) % kRing];
}

// ---------------------------------------------------------------- launchers
template <int PREC, bool NARROW>
static const void* batch_kernel_ptr(int schedule) {
    switch (schedule) {
    case 1: return (const void*)k_scan_batch<PREC, NARROW, 512, 10, 16, false>;
    case 2: return (const void*)k_scan_batch<PREC, NARROW, 512, 6, 16, false>;
    case 3: return (const void*)k_scan_batch<PREC, NARROW, 512, 4, 16, false>;
    case 4: return (const void*)k_scan_batch<PREC, NARROW, 1024, 8, 16, false>;
    case 5: return (const void*)k_scan_batch<PREC, NARROW, 512, 8, 32, false>;
    case 6: return (const void*)k_scan_batch<PREC, NARROW, 512, 10, 64, false>;
    case 7: return (const void*)k_scan_batch<PREC, NARROW, 256, 8, 16, false>;
    case 8: return (const void*)k_scan_batch<PREC, NARROW, 1024, 4, 16, false>;
    case 9: return (const void*)k_scan_batch<PREC, NARROW, 512, 4, 16, true>;
    case 10: return (const void*)k_scan_batch<PREC, NARROW, 1024, 4, 16, true>;
    default: return (const void*)k_scan_batch<PREC, NARROW, 512, 8, 16, false>;
    }
}

const void* batch_scan_kernel(int precision, bool narrow, int schedule) {
    switch (precision) {
    case BOOST_PREC_FP32: return narrow ? batch_kernel_ptr<BOOST_PREC_FP32, true>(schedule) : batch_kernel_ptr<BOOST_PREC_FP32, false>(schedule);
    case BOOST_PREC_FP32_KAHAN: return narrow ? batch_kernel_ptr<BOOST_PREC_FP32_KAHAN, true>(schedule) : batch_kernel_ptr<BOOST_PREC_FP32_KAHAN, false>(schedule);
    case BOOST_PREC_FP64: return narrow ? batch_kernel_ptr<BOOST_PREC_FP64, true>(schedule) : batch_kernel_ptr<BOOST_PREC_FP64, false>(schedule);
    default: return narrow ? batch_kernel_ptr<BOOST_PREC_FP32_WIDE, true>(schedule) : batch_kernel_ptr<BOOST_PREC_FP32_WIDE, false>(schedule);
    }
}

int batch_scan_launch(const void* kernel, int grid, int wg, const BatchDev& b, int part, hipStream_t s, int last) {
    uint32_t* ctr = b.next_seg + part;
    int s_begin = part == 0 ? 0 : b.seg_split;
    int s_end = part == 0 ? b.seg_split : b.n_segs;
    if (last > 0 && s_end - last > s_begin) s_begin = s_end - last;
    void* args[] = {(void*)&b.jobs, (void*)&b.segs, (void*)&ctr, (void*)&s_begin, (void*)&s_end, (void*)&b.job_seg,
                    (void*)&b.seg_best};
    VJB_HIP(hipLaunchKernel(kernel, dim3((unsigned)grid), dim3((unsigned)wg), args, 0, s));
    return BOOST_OK;
}

int batch_update_launch(int precision, int n_upd, const BatchDev& b, hipStream_t s) {
    const void* k;
    switch (precision) {
    case BOOST_PREC_FP32: k = (const void*)k_update_batch<BOOST_PREC_FP32>; break;
    case BOOST_PREC_FP32_KAHAN: k = (const void*)k_update_batch<BOOST_PREC_FP32_KAHAN>; break;
    case BOOST_PREC_FP64: k = (const void*)k_update_batch<BOOST_PREC_FP64>; break;
    default: k = (const void*)k_update_batch<BOOST_PREC_FP32_WIDE>; break;
    }
    void* args[] = {(void*)&b.jobs, (void*)&b.next_seg, (void*)&b.upd_job, (void*)&b.upd_part, (void*)&b.job_seg,
                    (void*)&b.seg_best};
    VJB_HIP(hipLaunchKernel(k, dim3((unsigned)n_upd), dim3(kUpdWg), args, 0, s));
    return BOOST_OK;
}

int batch_gather_launch(const BatchDev& b, int n_jobs, int64_t first, int count, boost_stump* out, hipStream_t s) {
    const int64_t tot = (int64_t)n_jobs * count;
    hipLaunchKernelGGL(k_gather_records, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, b.jobs, n_jobs, first,
                       count, out);
    VJB_HIP(hipGetLastError());
    return BOOST_OK;
}

}  // namespace vjb
