// Device code of the update workgroup, shared by the single-job and the
// batched update kernels: the second level of the argmin, the split rank,
// the threshold, beta and alpha, and the weight update.
#pragma once

#include "round_core.h"

namespace vjb {

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

// Longest lane segment: ceil(ceil(32767 / 8) / 16) units.
constexpr int kMaxSeg = 257;

template <typename Wt>
struct UpdLds {
    WgBest wb[kUpdWg / 64];
    double sh[kUpdWg / 64];
    Wt val[kMaxSeg * 8];       // table values of the winning lane's keys, rank order
    uint16_t idx[kMaxSeg * 8];   // their window indices
    uint32_t flags[kMaxSeg];   // run-end flags, one byte per unit
    int64_t k;
    int32_t theta;
    int32_t pad;
};

// Inclusive prefix of v across the 64 lanes of a wave.
__device__ __forceinline__ double wave_exclusive_incl(double v, int lane) {
    return group_exclusive<64, double>(v, lane) + v;
}

// Every workgroup: the argmin over the scan's workgroup candidates (Section
// 3.3.2 step 4a), the split rank -- the first run end where the winning
// lane's running sum reaches its extreme, recomputed in exactly the scan's
// arithmetic from that lane's keys and table values -- and the integer
// threshold; then the update of its own 256 windows
//     w_i <- (w_i / S) * beta   if x_i is classified correctly (e_i = 0),
//     w_i <- (w_i / S)          otherwise            (Section 2.3 step 4),
// into the other half of the weight buffer, and its partial sum for the next
// normalisation.  All workgroups reach the same stump; workgroup 0 records it.
// `part` is this workgroup's index within the job; wgb / n_wg the job's
// scan candidates.
template <int PREC>
__device__ __forceinline__ void update_body(const JobDev& jd, const WgBest* __restrict__ wgb, int n_wg, int part) {
    using Wt = typename ScanTypes<PREC>::W;
    __shared__ UpdLds<Wt> lds;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    JobState* st = jd.st;
    // the round's state and this workgroup's own weights, loaded first: none
    // of them depends on the stump
    const int64_t n = jd.g.n;
    const int64_t l = st->n_pos;
    const double S = st->sum_w;
    const double rS = 1.0 / S;
    const int par = st->cur;   // the scan's weights; this kernel writes the other half
    const double* w_in = weights(jd, par);
    double* w_out = weights(jd, par ^ 1);
    const int64_t i = (int64_t)part * kUpdWg + tid;
    const double w_i = i < n ? w_in[i] : 0.0;
    // 1. argmin over the scan workgroups' candidates
    WgBest b{DBL_MAX, -1, 0, -1};
    for (int k = tid; k < n_wg; k += kUpdWg) {
        const WgBest c = wgb[k];
        if (better(c, b)) b = c;
    }
#pragma unroll
    for (int o = 32; o; o >>= 1) {
        WgBest c;
        c.eps = __shfl_xor(b.eps, o);
        c.feature = __shfl_xor(b.feature, o);
        c.polarity = __shfl_xor(b.polarity, o);
        c.lane = __shfl_xor(b.lane, o);
        if (better(c, b)) b = c;
    }
    if (lane == 0) lds.wb[wv] = b;
    __syncthreads();
    b = lds.wb[0];
    for (int k = 1; k < kUpdWg / 64; ++k)
        if (better(lds.wb[k], b)) b = lds.wb[k];
    const bool lead = part == 0 && tid == 0;
    if (b.feature < 0) {   // stopped earlier (or no finite candidate): no round
        if (lead) {
            boost_stump rec = {};
            rec.feature = -1; rec.round = -1;
            jd.ring[st->launches % kRing] = rec;
            st->launches = st->launches + 1;
        }
        return;
    }
    const int64_t j = b.feature;
    const int pol = b.polarity;
    const uint32_t desc = jd.ftab[j];
    const int wp1 = jd.W + 1;
    // this workgroup's windows: values are loaded while the split is found
    const int32_t f = i < n ? haar_value(jd.ii, jd.ii_stride, wp1, desc, i) : 0;
    // 2. split rank: the winning lane's segment (table values, run-end flags)
    // is staged in LDS by the whole workgroup; the lane's prefix at every key
    // is then computed in parallel (unit sums, a block scan of them, then
    // within the unit) in FP64, which is exact for the table's values, and
    // the split is the first run end where that prefix is extreme.  In the
    // exact modes this is the scan's own value bit for bit.  In the rounded
    // modes (FP32, compensated FP32) the scan picked the feature, the
    // polarity and the lane from its rounded sums; within that lane the split
    // is placed where the exact prefix of the same table is extreme, which
    // can differ from the scan's choice only among splits whose errors agree
    // to the scan's rounding.
    const int L = b.lane;
    const int cntL = L >= 0 ? jd.g.q + (L < jd.g.rem ? 1 : 0) : 0;
    for (int u = tid; u < cntL; u += kUpdWg) {
        const uint4 q4 = jd.keys[j * jd.g.row_units + (int64_t)u * jd.g.lanes + L];
        const uint32_t dw[4] = {q4.x, q4.y, q4.z, q4.w};
        uint32_t fb = 0;
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            uint32_t i0, f0, i1, f1;
            decode_pair(jd.g.narrow, dw[h], i0, f0, i1, f1);
            fb |= (f0 << (2 * h)) | (f1 << (2 * h + 1));
            lds.idx[u * 8 + 2 * h] = (uint16_t)i0;
            lds.idx[u * 8 + 2 * h + 1] = (uint16_t)i1;
            lds.val[u * 8 + 2 * h] = i0 < (uint32_t)n ? table_value<PREC>(w_in[i0], rS, i0 < (uint32_t)l) : (Wt)0;
            lds.val[u * 8 + 2 * h + 1] = i1 < (uint32_t)n ? table_value<PREC>(w_in[i1], rS, i1 < (uint32_t)l) : (Wt)0;
        }
        lds.flags[u] = fb;
    }
    __syncthreads();
    int64_t k = 0;
    if (L >= 0) {
        double us[2] = {0.0, 0.0};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int u = tid + h * kUpdWg;
            if (u < cntL)
#pragma unroll
                for (int e = 0; e < 8; ++e) us[h] += (double)lds.val[u * 8 + e];
        }
        // exclusive prefix over units: 2 units per thread in order tid, tid + 256
        const double tsum = us[0];
        double incl = wave_exclusive_incl(tsum, lane);
        if (lane == 63) lds.sh[wv] = incl;
        __syncthreads();
        double wbase = 0.0, all0 = 0.0;
        for (int q = 0; q < kUpdWg / 64; ++q) { if (q < wv) wbase += lds.sh[q]; all0 += lds.sh[q]; }
        double ex0 = wbase + incl - tsum;          // prefix before unit tid
        __syncthreads();
        double incl1 = wave_exclusive_incl(us[1], lane);
        if (lane == 63) lds.sh[wv] = incl1;
        __syncthreads();
        double wbase1 = all0;
        for (int q = 0; q < wv; ++q) wbase1 += lds.sh[q];
        double ex1 = wbase1 + incl1 - us[1];       // prefix before unit tid + 256
        // candidates: extreme value, then the smallest rank
        double best_v = pol > 0 ? -4.0 : 4.0;
        int best_r = 0x7FFFFFFF;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int u = tid + h * kUpdWg;
            if (u < cntL) {
                double acc = h == 0 ? ex0 : ex1;
                const uint32_t fr = lds.flags[u];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    acc += (double)lds.val[u * 8 + e];
                    if ((fr >> e) & 1u) {
                        const bool c = pol > 0 ? acc > best_v : acc < best_v;
                        if (c) { best_v = acc; best_r = u * 8 + e; }
                    }
                }
            }
        }
        // block reduction: extreme value, ties to the smaller rank
#pragma unroll
        for (int o = 32; o; o >>= 1) {
            const double ov = __shfl_xor(best_v, o);
            const int orr = __shfl_xor(best_r, o);
            const bool c = (pol > 0 ? ov > best_v : ov < best_v) || (ov == best_v && orr < best_r);
            if (c) { best_v = ov; best_r = orr; }
        }
        __syncthreads();
        if (lane == 0) { lds.wb[wv].eps = best_v; lds.wb[wv].lane = best_r; }
        __syncthreads();
        if (tid == 0) {
            for (int q = 1; q < kUpdWg / 64; ++q) {
                const double ov = lds.wb[q].eps;
                const int orr = lds.wb[q].lane;
                const bool c = (pol > 0 ? ov > best_v : ov < best_v) || (ov == best_v && orr < best_r);
                if (c) { best_v = ov; best_r = orr; }
            }
            k = 8 * lane_start(jd.g, L) + best_r + 1;
        }
    }
    if (tid == 0) {
        // 3. threshold from the window at the rank just above (p = +1) or at
        // (p = -1) the split; its index is in the staged segment unless the
        // rank is the next lane's first
        const int64_t rk = pol > 0 ? (k < n ? k : n - 1) : (k > 0 ? k - 1 : 0);
        const int64_t pos = L >= 0 ? rk - 8 * lane_start(jd.g, L) : -1;
        const int32_t wi = pos >= 0 && pos < 8 * (int64_t)cntL ? (int32_t)lds.idx[pos] : index_at_rank(jd, j, rk);
        const int32_t v = haar_value(jd.ii, jd.ii_stride, wp1, desc, wi);
        lds.k = k;
        lds.theta = pol > 0 ? (k < n ? v : v + 1) : (k > 0 ? v : v - 1);
    }
    __syncthreads();
    // 4. beta, alpha (FP64); eps = 0 is clamped to the floor
    const double eps = b.eps;
    const double epsc = eps > jd.eps_floor ? eps : jd.eps_floor;
    const double beta = epsc / (1.0 - epsc);
    const bool stop = jd.on_perfect == BOOST_ON_PERFECT_STOP && !(eps > jd.eps_floor);
    const int32_t theta = lds.theta;
    if (lead) {
        int t, x, y, cw, ch;
        unpack_feature(desc, t, x, y, cw, ch);
        boost_stump rec;
        rec.feature = j; rec.type = t; rec.x = x; rec.y = y; rec.cell_w = cw; rec.cell_h = ch;
        rec.polarity = pol; rec.threshold = theta; rec.split_rank = (int32_t)lds.k; rec.round = st->round;
        rec.pad = 0;
        rec.error_raw = eps; rec.error = epsc; rec.beta = beta; rec.alpha = log(1.0 / beta);
        jd.ring[st->launches % kRing] = rec;
        if (stop) st->stopped = 1;
        else st->wpar = par ^ 1;
        st->round = st->round + 1;
        st->launches = st->launches + 1;
    }
    if (stop) return;   // weights unchanged
    // 5. update and partial sum
    double wn = 0.0;
    if (i < n) {
        const int h = (int64_t)pol * f < (int64_t)pol * theta ? 1 : 0;
        const int y = i < l ? 1 : 0;
        wn = w_i * rS;
        if (h == y) wn = wn * beta;
        w_out[i] = wn;
    }
#pragma unroll
    for (int o = 32; o; o >>= 1) wn += __shfl_xor(wn, o);
    if (lane == 0) lds.sh[wv] = wn;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int k = 0; k < kUpdWg / 64; ++k) s += lds.sh[k];
        jd.wpart[part] = s;
    }
}

}  // namespace vjb
