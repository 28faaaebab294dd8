// Per-round scan kernel of one job: every feature's best stump under the
// current weights (Section 2.3 step 2 / Section 3.3.2 step 3a, all features
// at once) and the first level of the argmin per workgroup.  Normalisation
// (step 1) happens as each workgroup fills its LDS weight table.
#include "round_core.h"

namespace vjb {

// ---------------------------------------------------------------- scan kernel
// Persistent: every workgroup fills its LDS weight table once, then its waves
// take group-steps of features; each workgroup leaves its best candidate
// (the first level of the argmin).
template <int PREC, bool NARROW, int WG, int UNROLL, int LPF, bool RING>
__global__ __launch_bounds__(WG, (ScanOccupancy<PREC, NARROW, WG, UNROLL, false, RING>::waves_per_eu)) void k_scan(JobDev jd, double2* __restrict__ ferr) {
    using Wt = typename ScanTypes<PREC>::W;
    constexpr int NG = (WG / 64) * (64 / LPF);
    __shared__ ScanLds<Wt, TabCap<PREC, NARROW>::value, NG> lds;
    Wt* tab = lds.tab;
    const int tid = threadIdx.x, wv = tid >> 6;
    WgBest best{DBL_MAX, -1, 0, -1};
    if (!jd.st->stopped) {
        // rotating loads: the first key loads are issued before the table
        // fill, so HBM is busy while the workgroup builds its table
        RingScan<PREC, NARROW, UNROLL, LPF> rs;
        if constexpr (RING)
            rs.prime(jd, 0, jd.F, (int64_t)blockIdx.x * (WG / 64) + wv, (int64_t)gridDim.x * (WG / 64));
        const int par = jd.st->wpar;
        const double S = weight_sum(jd);
        double tp, tn;
        fill_table<PREC>(jd, weights(jd, par), tab, 1.0 / S, WG, lds.sh, tp, tn);
        if (blockIdx.x == 0 && tid == 0) {
            jd.st->sum_w = S; jd.st->t_pos = tp; jd.st->t_neg = tn; jd.st->cur = par;
        }
        const int64_t total_waves = (int64_t)gridDim.x * (WG / 64);
        if constexpr (RING)
            best = rs.run(jd, tab, tp, tn, ferr);
        else
            best = scan_range<PREC, NARROW, UNROLL, LPF>(jd, tab, 0, jd.F, (int64_t)blockIdx.x * (WG / 64) + wv,
                                                         total_waves, tp, tn, ferr);
    }
    const WgBest b = block_best<NG>(lds.wb, best, LPF);
    if (tid == 0) jd.wgb[blockIdx.x] = b;
}

// ---------------------------------------------------------------- launchers
// Launch schedules: workgroup size, units per batch (or register slots of the
// rotating loads), lanes per feature, rotating loads.
struct Schedule { int wg, unroll, lanes; bool ring; };
static const Schedule kSchedules[] = {
    {512, 8, 16, false}, {512, 10, 16, false}, {512, 6, 16, false}, {512, 4, 16, false}, {1024, 8, 16, false},
    {512, 8, 32, false}, {512, 10, 64, false}, {256, 8, 16, false}, {1024, 4, 16, false}, {512, 4, 16, true},
    {1024, 4, 16, true},
};
constexpr int kNumSchedules = (int)(sizeof(kSchedules) / sizeof(kSchedules[0]));

template <int PREC, bool NARROW>
static const void* scan_kernel_ptr(int schedule) {
    switch (schedule) {
    case 1: return (const void*)k_scan<PREC, NARROW, 512, 10, 16, false>;
    case 2: return (const void*)k_scan<PREC, NARROW, 512, 6, 16, false>;
    case 3: return (const void*)k_scan<PREC, NARROW, 512, 4, 16, false>;
    case 4: return (const void*)k_scan<PREC, NARROW, 1024, 8, 16, false>;
    case 5: return (const void*)k_scan<PREC, NARROW, 512, 8, 32, false>;
    case 6: return (const void*)k_scan<PREC, NARROW, 512, 10, 64, false>;
    case 7: return (const void*)k_scan<PREC, NARROW, 256, 8, 16, false>;
    case 8: return (const void*)k_scan<PREC, NARROW, 1024, 4, 16, false>;
    case 9: return (const void*)k_scan<PREC, NARROW, 512, 4, 16, true>;
    case 10: return (const void*)k_scan<PREC, NARROW, 1024, 4, 16, true>;
    default: return (const void*)k_scan<PREC, NARROW, 512, 8, 16, false>;
    }
}

int scan_schedule_count() { return kNumSchedules; }
int scan_schedule_wg(int schedule) {
    return kSchedules[(schedule >= 0 && schedule < kNumSchedules) ? schedule : 0].wg;
}
int scan_schedule_unroll(int schedule) {
    return kSchedules[(schedule >= 0 && schedule < kNumSchedules) ? schedule : 0].unroll;
}
int scan_schedule_lanes(int schedule) {
    return kSchedules[(schedule >= 0 && schedule < kNumSchedules) ? schedule : 0].lanes;
}

const void* scan_kernel(int precision, bool narrow, int schedule) {
    switch (precision) {
    case BOOST_PREC_FP32: return narrow ? scan_kernel_ptr<BOOST_PREC_FP32, true>(schedule) : scan_kernel_ptr<BOOST_PREC_FP32, false>(schedule);
    case BOOST_PREC_FP32_KAHAN: return narrow ? scan_kernel_ptr<BOOST_PREC_FP32_KAHAN, true>(schedule) : scan_kernel_ptr<BOOST_PREC_FP32_KAHAN, false>(schedule);
    case BOOST_PREC_FP64: return narrow ? scan_kernel_ptr<BOOST_PREC_FP64, true>(schedule) : scan_kernel_ptr<BOOST_PREC_FP64, false>(schedule);
    default: return narrow ? scan_kernel_ptr<BOOST_PREC_FP32_WIDE, true>(schedule) : scan_kernel_ptr<BOOST_PREC_FP32_WIDE, false>(schedule);
    }
}

int64_t scan_table_capacity(int precision, bool narrow) {
    if (precision == BOOST_PREC_FP64) return narrow ? 16384 : 20224;
    return narrow ? 16384 : 32768;
}

int scan_plan(ScanPlan& p, int precision, bool narrow, int schedule, int64_t n, int64_t F, int num_cu) {
    p.kernel = scan_kernel(precision, narrow, schedule);
    p.wg = scan_schedule_wg(schedule);
    p.lds = 0;
    if (n + 1 > scan_table_capacity(precision, narrow)) {
        set_error("weight table exceeds the scan kernel's LDS capacity");
        return BOOST_E_INVALID;
    }
    int per_cu = 0;
    VJB_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, p.kernel, p.wg, p.lds));
    if (per_cu < 1) {
        set_error("scan kernel does not fit on a compute unit");
        return BOOST_E_INVALID;
    }
    int64_t grid = (int64_t)per_cu * num_cu;
    const int64_t per_wg = (int64_t)(p.wg / 64) * (64 / scan_schedule_lanes(schedule));   // features per workgroup step
    const int64_t max_grid = (F + per_wg - 1) / per_wg;
    if (grid > max_grid) grid = max_grid;
    if (grid > kMaxScanGrid) grid = kMaxScanGrid;
    p.grid = (int)grid;
    return BOOST_OK;
}

int scan_launch(const ScanPlan& p, const JobDev& jd, double2* ferr, hipStream_t s) {
    void* args[] = {(void*)&jd, (void*)&ferr};
    VJB_HIP(hipLaunchKernel(p.kernel, dim3(p.grid), dim3(p.wg), args, p.lds, s));
    return BOOST_OK;
}

}  // namespace vjb
