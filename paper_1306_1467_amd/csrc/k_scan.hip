// Per-round kernels of one job: the weighted-error scan over every feature
// (Section 2.3 step 2 / Section 3.3.2 step 3a, all features at once) with the
// first level of the argmin, and the finalize kernel that takes the argmin
// over workgroups (Section 3.3.2 step 4a), recovers the threshold, computes
// beta and alpha and applies the weight update and normalisation
// (Section 2.3 steps 1 and 4).
#include <float.h>

#include "launch.h"
#include "scan_core.h"

namespace vjb {

// LDS image of the scan kernel: the weight table at LDS address 0, so the key
// bits of a window are directly its table byte offset; then one record per wave.
template <typename Wt, int CAP, int NW>
struct alignas(16) ScanLds {
    Wt tab[CAP];
    WgBest wb[NW];
};

// Table capacity (entries, including the zero slot at n) per key format.
template <int PREC, bool NARROW>
struct TabCap {
    static constexpr int value = sizeof(typename ScanTypes<PREC>::W) == 4 ? (NARROW ? 16384 : 32768)
                                                                          : (NARROW ? 16384 : 20224);
};

// ---------------------------------------------------------------- scan kernel
// Persistent: every workgroup copies the signed weight table into LDS once,
// then each wave takes features j = wave_id, wave_id + total_waves, ...
template <int PREC, bool NARROW, int WG, int UNROLL>
__global__ __launch_bounds__(WG) void k_scan(JobDev jd, WgBest* __restrict__ out, double2* __restrict__ ferr) {
    using Wt = typename ScanTypes<PREC>::W;
    __shared__ ScanLds<Wt, TabCap<PREC, NARROW>::value, WG / 64> lds;
    Wt* tab = lds.tab;
    WgBest* wb = lds.wb;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (jd.st->stopped) {
        if (tid == 0) out[blockIdx.x] = WgBest{DBL_MAX, -1, 0, 0};
        return;
    }
    const int64_t ntab = jd.g.n + 1;
    const Wt* src = (const Wt*)jd.wtab;
    for (int64_t i = tid; i < ntab; i += WG) tab[i] = src[i];
    __syncthreads();
    const double tp = jd.st->t_pos, tn = jd.st->t_neg;
    const int cnt = jd.g.q + (lane < jd.g.rem ? 1 : 0);
    const int64_t total_waves = (int64_t)gridDim.x * (WG / 64);
    double best = DBL_MAX;
    int64_t bj = -1;
    int bp = 0;
    for (int64_t j = (int64_t)blockIdx.x * (WG / 64) + wv; j < jd.F; j += total_waves) {
        double ep, en;
        scan_feature<PREC, NARROW, UNROLL>(jd.keys + j * jd.g.row_units, lane, cnt, tab, tp, tn, ep, en);
        if (ferr != nullptr && lane == 0) ferr[j] = make_double2(ep, en);
        const double e = fmin(ep, en);
        if (e < best) { best = e; bj = j; bp = ep <= en ? 1 : -1; }
    }
    if (lane == 0) wb[wv] = WgBest{best, bj, bp, 0};
    __syncthreads();
    if (tid == 0) {
        WgBest b = wb[0];
        for (int k = 1; k < WG / 64; ++k) {
            const WgBest c = wb[k];
            if (c.feature >= 0 && (b.feature < 0 || c.eps < b.eps || (c.eps == b.eps && c.feature < b.feature))) b = c;
        }
        out[blockIdx.x] = b;
    }
}

// ---------------------------------------------------------------- finalize
__device__ __forceinline__ bool better(const WgBest& c, const WgBest& b) {
    return c.feature >= 0 && (b.feature < 0 || c.eps < b.eps || (c.eps == b.eps && c.feature < b.feature));
}

// Window index (internal order) at rank r of feature j.
__device__ inline int32_t index_at_rank(const JobDev& jd, int64_t j, int64_t r) {
    const int64_t mu = unit_to_mem(jd.g, r >> 3);
    const uint4 u = jd.keys[j * jd.g.row_units + mu];
    const int e = (int)(r & 7);
    const uint32_t d = (e >> 1) == 0 ? u.x : (e >> 1) == 1 ? u.y : (e >> 1) == 2 ? u.z : u.w;
    uint32_t i0, f0, i1, f1;
    decode_pair(jd.g.narrow, d, i0, f0, i1, f1);
    return (int32_t)((e & 1) ? i1 : i0);
}

// Rescan of the winning feature by one wave, in exactly the arithmetic of
// scan_feature, returning the smallest split k attaining the extreme D.
template <int PREC, bool NARROW>
__device__ int64_t best_split(const JobDev& jd, int64_t j, int pol, int lane) {
    using Wt = typename ScanTypes<PREC>::W;
    using A = typename ScanTypes<PREC>::A;
    const Wt* tab = (const Wt*)jd.wtab;
    LaneAcc<PREC> a;
    const int cnt = jd.g.q + (lane < jd.g.rem ? 1 : 0);
    const int64_t start = lane_start(jd.g, lane);
    const uint4* row = jd.keys + j * jd.g.row_units;
    // same candidate values as LaneAcc::cand (the extreme over a lane is
    // order independent), with the first rank where it is reached
    decltype(a.add(Wt(0))) ext = pol > 0 ? -4 : 4;
    int64_t ext_rank = -1;
    for (int r = 0; r < cnt; ++r) {
        const uint4 u = row[(int64_t)r * 64 + lane];
        const uint32_t dw[4] = {u.x, u.y, u.z, u.w};
        for (int h = 0; h < 4; ++h) {
            const uint32_t d = dw[h];
            const Wt w0 = tab_lo<Wt, NARROW>(tab, d);
            const Wt w1 = tab_hi<Wt, NARROW>(tab, d);
            const auto v0 = a.add(w0);
            if (flag_lo<NARROW>(d) && (pol > 0 ? v0 > ext : v0 < ext)) { ext = v0; ext_rank = 8 * (start + r) + 2 * h; }
            const auto v1 = a.add(w1);
            if (flag_hi<NARROW>(d) && (pol > 0 ? v1 > ext : v1 < ext)) { ext = v1; ext_rank = 8 * (start + r) + 2 * h + 1; }
        }
    }
    const A base = wave_exclusive<A>((A)a.total(), lane);
    A c = ext_rank >= 0 ? base + (A)ext : (pol > 0 ? (A)-8 : (A)8);
    A m = c;
#pragma unroll
    for (int o = 32; o; o >>= 1) m = pol > 0 ? fmax(m, __shfl_xor(m, o)) : fmin(m, __shfl_xor(m, o));
    // k = 0 wins ties with D = 0 (smaller split)
    if (pol > 0 ? !(m > (A)0) : !(m < (A)0)) return 0;
    const unsigned long long hit = __ballot(c == m && ext_rank >= 0);
    const int first = __ffsll(hit) - 1;
    const int64_t rk = __shfl(ext_rank, first);
    return rk + 1;
}

template <int PREC, bool NARROW>
__global__ __launch_bounds__(1024) void k_finalize(JobDev jd, const WgBest* __restrict__ wgb, int n_wg) {
    constexpr int NT = 1024;
    __shared__ double sh[NT / 64];
    __shared__ WgBest red[NT / 64];
    __shared__ int64_t s_k;
    __shared__ int32_t s_theta;
    __shared__ double s_beta;
    __shared__ int32_t s_update;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    JobState* st = jd.st;
    const int32_t t_round = st->round;
    const int32_t slot = st->launches % kRing;
    if (st->stopped) {
        if (tid == 0) {
            boost_stump rec = {};
            rec.feature = -1; rec.round = -1;
            jd.ring[slot] = rec;
            st->launches = st->launches + 1;
        }
        return;
    }
    // 1. argmin over the workgroups' candidates
    WgBest b{DBL_MAX, -1, 0, 0};
    for (int k = tid; k < n_wg; k += NT) {
        const WgBest c = wgb[k];
        if (better(c, b)) b = c;
    }
#pragma unroll
    for (int o = 32; o; o >>= 1) {
        WgBest c;
        c.eps = __shfl_xor(b.eps, o);
        c.feature = __shfl_xor(b.feature, o);
        c.polarity = __shfl_xor(b.polarity, o);
        c.pad = 0;
        if (better(c, b)) b = c;
    }
    if (lane == 0) red[wv] = b;
    __syncthreads();
    b = red[0];
    for (int k = 1; k < NT / 64; ++k)
        if (better(red[k], b)) b = red[k];
    const int64_t j = b.feature;
    const int pol = b.polarity;
    if (j < 0) {   // no finite candidate (cannot happen with validated weights)
        if (tid == 0) {
            boost_stump rec = {};
            rec.feature = -1; rec.round = -1;
            jd.ring[slot] = rec;
            st->launches = st->launches + 1;
        }
        return;
    }
    const uint32_t desc = jd.ftab[j];
    const int wp1 = jd.W + 1;
    const int64_t n = jd.g.n;
    // 2. split rank and 3. threshold (integer, exact under p f < p theta)
    if (wv == 0) {
        const int64_t k = best_split<PREC, NARROW>(jd, j, pol, lane);
        if (lane == 0) {
            int32_t theta;
            if (pol > 0) {
                theta = k < n ? haar_value(jd.ii, jd.ii_stride, wp1, desc, index_at_rank(jd, j, k))
                              : haar_value(jd.ii, jd.ii_stride, wp1, desc, index_at_rank(jd, j, n - 1)) + 1;
            } else {
                theta = k > 0 ? haar_value(jd.ii, jd.ii_stride, wp1, desc, index_at_rank(jd, j, k - 1))
                              : haar_value(jd.ii, jd.ii_stride, wp1, desc, index_at_rank(jd, j, 0)) - 1;
            }
            s_k = k;
            s_theta = theta;
            // 4. beta and alpha (FP64); eps = 0 is clamped to the floor
            const double eps = b.eps;
            const double epsc = eps > jd.eps_floor ? eps : jd.eps_floor;
            const double beta = epsc / (1.0 - epsc);
            s_beta = beta;
            const bool stop = jd.on_perfect == BOOST_ON_PERFECT_STOP && !(eps > jd.eps_floor);
            s_update = stop ? 0 : 1;
            int t, x, y, cw, ch;
            unpack_feature(desc, t, x, y, cw, ch);
            boost_stump rec;
            rec.feature = j; rec.type = t; rec.x = x; rec.y = y; rec.cell_w = cw; rec.cell_h = ch;
            rec.polarity = pol; rec.threshold = theta; rec.split_rank = (int32_t)k; rec.round = t_round;
            rec.pad = 0;
            rec.error_raw = eps; rec.error = epsc; rec.beta = beta; rec.alpha = log(1.0 / beta);
            jd.ring[slot] = rec;
            if (stop) st->stopped = 1;
        }
    }
    __syncthreads();
    if (!s_update) {
        if (tid == 0) { st->round = t_round + 1; st->launches = st->launches + 1; }
        return;
    }
    // 5. update: w_i <- w_i * beta when x_i is classified correctly (e_i = 0)
    const int32_t theta = s_theta;
    const double beta = s_beta;
    const int64_t l = st->n_pos;
    for (int64_t i = tid; i < n; i += NT) {
        const int32_t f = haar_value(jd.ii, jd.ii_stride, wp1, desc, i);
        const int h = (int64_t)pol * f < (int64_t)pol * theta ? 1 : 0;
        const int y = i < l ? 1 : 0;
        if (h == y) jd.w[i] = jd.w[i] * beta;
    }
    __syncthreads();
    // 6. normalisation and the next round's table
    prep_weights<NT>(jd, sh);
    if (tid == 0) { st->round = t_round + 1; st->launches = st->launches + 1; }
}

// ---------------------------------------------------------------- launchers
template <int PREC, bool NARROW>
static const void* scan_kernel_ptr(int schedule) {
    switch (schedule) {
    case 1: return (const void*)k_scan<PREC, NARROW, 1024, 4>;
    case 2: return (const void*)k_scan<PREC, NARROW, 256, 4>;
    case 3: return (const void*)k_scan<PREC, NARROW, 512, 8>;
    case 4: return (const void*)k_scan<PREC, NARROW, 1024, 8>;
    case 5: return (const void*)k_scan<PREC, NARROW, 512, 2>;
    default: return (const void*)k_scan<PREC, NARROW, 512, 4>;
    }
}

int scan_schedule_count() { return 6; }
int scan_schedule_wg(int schedule) {
    static const int wg[6] = {512, 1024, 256, 512, 1024, 512};
    return wg[(schedule >= 0 && schedule < 6) ? schedule : 0];
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
        set_error("scan kernel does not fit on a compute unit (weight table too large)");
        return BOOST_E_INVALID;
    }
    int64_t grid = (int64_t)per_cu * num_cu;
    const int64_t waves_needed = F;  // one feature per wave at least
    const int64_t max_grid = (waves_needed + p.wg / 64 - 1) / (p.wg / 64);
    if (grid > max_grid) grid = max_grid;
    if (grid > kMaxScanGrid) grid = kMaxScanGrid;
    p.grid = (int)grid;
    return BOOST_OK;
}

int scan_launch(const ScanPlan& p, const JobDev& jd, WgBest* out, double2* ferr, hipStream_t s) {
    void* args[] = {(void*)&jd, (void*)&out, (void*)&ferr};
    VJB_HIP(hipLaunchKernel(p.kernel, dim3(p.grid), dim3(p.wg), args, p.lds, s));
    return BOOST_OK;
}

int finalize_launch(const JobDev& jd, const WgBest* wgb, int n_wg, hipStream_t s) {
    const bool narrow = jd.g.narrow != 0;
    const void* k;
    switch (jd.precision) {
    case BOOST_PREC_FP32: k = narrow ? (const void*)k_finalize<BOOST_PREC_FP32, true> : (const void*)k_finalize<BOOST_PREC_FP32, false>; break;
    case BOOST_PREC_FP32_KAHAN: k = narrow ? (const void*)k_finalize<BOOST_PREC_FP32_KAHAN, true> : (const void*)k_finalize<BOOST_PREC_FP32_KAHAN, false>; break;
    case BOOST_PREC_FP64: k = narrow ? (const void*)k_finalize<BOOST_PREC_FP64, true> : (const void*)k_finalize<BOOST_PREC_FP64, false>; break;
    default: k = narrow ? (const void*)k_finalize<BOOST_PREC_FP32_WIDE, true> : (const void*)k_finalize<BOOST_PREC_FP32_WIDE, false>; break;
    }
    void* args[] = {(void*)&jd, (void*)&wgb, (void*)&n_wg};
    VJB_HIP(hipLaunchKernel(k, dim3(1), dim3(1024), args, 0, s));
    return BOOST_OK;
}

}  // namespace vjb
