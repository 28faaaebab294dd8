// Device code shared by the single-job and the batched scan kernels: the
// scan of a range of features with a filled LDS table and the workgroup
// reduction of candidates.
#pragma once

#include <float.h>

#include "launch.h"
#include "scan_core.h"

namespace vjb {

// LDS image of the scan kernel: the weight table at LDS address 0, so the key
// bits of a window are directly its table byte offset; then per-group
// records and reduction scratch.
template <typename Wt, int CAP, int NG>
struct alignas(16) ScanLds {
    Wt tab[CAP];
    WgBest wb[NG];
    double sh[8];
};

// Table capacity (entries, including the zero slot at n) per key format.
template <int PREC, bool NARROW>
struct TabCap {
    static constexpr int value = sizeof(typename ScanTypes<PREC>::W) == 4 ? (NARROW ? 16384 : 32768)
                                                                          : (NARROW ? 16384 : 20224);
};

// Waves per SIMD the scan kernels are compiled for: the LDS table admits two
// workgroups per compute unit when it is at most 64 KiB, else one.  Batches
// of more than 4 key units need up to 128 VGPRs per lane (the batch lives in
// registers), so those launches stay at 4 waves per SIMD; the single-job
// kernel with 4-unit batches fits in 64 VGPRs and may run 8 (the batched
// kernel, which also holds the table refill, would spill there, and so would
// the rotating loads, which also hold the fill stream).
template <int PREC, bool NARROW, int WG, int UNROLL, bool BATCHED, bool RING = false>
struct ScanOccupancy {
    static constexpr int wgs = TabCap<PREC, NARROW>::value * (int)sizeof(typename ScanTypes<PREC>::W) <= 65536 ? 2 : 1;
    static constexpr int cap = UNROLL <= 4 && !BATCHED && !RING ? 8 : 4;
    static constexpr int waves_per_eu = wgs * WG / 256 < cap ? wgs * WG / 256 : cap;
};

__device__ __forceinline__ bool better(const WgBest& c, const WgBest& b) {
    return c.feature >= 0 && (b.feature < 0 || c.eps < b.eps || (c.eps == b.eps && c.feature < b.feature));
}

// Rotating-load scan of one wave over features [f0, f1) (the RING
// discipline of scan_range).  The scan stream consumes the UNROLL register
// slots in order; the fill stream runs one batch ahead: (tf, rr) = feature
// step and first unit of the next batch to load, pf / cf = that feature's
// row and this lane's unit count there (0 past f1: the padding unit is read
// instead).  prime() issues the first loads and may run before the LDS table
// is filled; run() needs the table.  Slots past a feature's last owned unit
// are loaded (from the padding unit) but not scanned.
template <int PREC, bool NARROW, int UNROLL, int LPF>
struct RingScan {
    static constexpr int G = 64 / LPF;
    uint4 u[UNROLL];
    int64_t f0, f1, nsteps, t, j, tf;
    int L, grp, cnt, per, nbr, rr, cf;
    const uint4* pf;
    bool any, fill_full, fill_live;

    __device__ __forceinline__ void prime(const JobDev& jd, int64_t f0_, int64_t f1_, int64_t step0,
                                          int64_t nsteps_) {
        f0 = f0_; f1 = f1_; nsteps = nsteps_;
        const int lane = threadIdx.x & 63;
        grp = lane / LPF; L = lane % LPF;
        cnt = jd.g.q + (L < jd.g.rem ? 1 : 0);
        per = jd.g.q + (jd.g.rem > 0 ? 1 : 0);
        nbr = (per + UNROLL - 1) / UNROLL;
        t = step0;
        j = f0 + t * G + grp;
        any = f0 + t * G < f1;
        if (!any) return;
        tf = t;
        rr = 0;
        pf = jd.keys + (j < f1 ? j : 0) * jd.g.row_units + L;
        cf = j < f1 ? cnt : 0;
        fill_full = f0 + tf * G + G - 1 < f1;   // every group of the wave has a feature
        fill_live = true;                        // some group has
#pragma unroll
        for (int k = 0; k < UNROLL; ++k) u[k] = ld_stream(k < cf ? pf + k * LPF : jd.pad);
        advance_fill(jd);
    }

    __device__ __forceinline__ void advance_fill(const JobDev& jd) {
        rr += UNROLL;
        if (rr >= nbr * UNROLL) {
            rr = 0;
            tf += nsteps;
            fill_live = f0 + tf * G < f1;
            fill_full = f0 + tf * G + G - 1 < f1;
            const int64_t jf = f0 + tf * G + grp;
            cf = jf < f1 ? cnt : 0;
            pf = jd.keys + (jf < f1 ? jf : 0) * jd.g.row_units + L;
        }
    }

    // One batch: scan the UNROLL slots in order (in a feature's last batch
    // only its first `last` units, the ones some lane owns), reloading each
    // slot from the fill stream as soon as it is scanned.
    template <bool LAST>
    __device__ __forceinline__ void step(LaneAcc<PREC>& a, const typename ScanTypes<PREC>::W* tab,
                                         const JobDev& jd, int last) {
        if (fill_full && rr + UNROLL <= per - 1) {
            // every lane owns units rr .. rr + UNROLL - 1 (each owns at least per - 1)
            const uint4* base = pf + rr * LPF;
#pragma unroll
            for (int k = 0; k < UNROLL; ++k) {
                if (!LAST || k < last) scan_unit<PREC, NARROW>(a, tab, u[k], (k & 1) != 0);
                u[k] = ld_stream(base + k * LPF);
            }
        } else if (fill_live) {
#pragma unroll
            for (int k = 0; k < UNROLL; ++k) {
                if (!LAST || k < last) scan_unit<PREC, NARROW>(a, tab, u[k], (k & 1) != 0);
                const int r = rr + k;
                u[k] = ld_stream(r < cf ? pf + r * LPF : jd.pad);
            }
        } else {   // nothing left to load: the wave's last batch
#pragma unroll
            for (int k = 0; k < UNROLL; ++k)
                if (!LAST || k < last) scan_unit<PREC, NARROW>(a, tab, u[k], (k & 1) != 0);
        }
        advance_fill(jd);
    }

    __device__ __forceinline__ WgBest run(const JobDev& jd, const typename ScanTypes<PREC>::W* tab, double tp,
                                          double tn, double2* __restrict__ ferr) {
        WgBest best{DBL_MAX, -1, 0, -1};
        if (!any) return best;
        const int last = per - (nbr - 1) * UNROLL;   // units of a feature's last batch that some lane owns
        while (true) {
            LaneAcc<PREC> a;
            for (int b = 0; b + 1 < nbr; ++b) step<false>(a, tab, jd, 0);
            step<true>(a, tab, jd, last);
            const FeatureScan fs = finish_feature<PREC, LPF>(a, threadIdx.x & 63, tp, tn);
            if (j < f1) {
                if (ferr != nullptr && L == 0) ferr[j] = make_double2(fs.e_pos, fs.e_neg);
                const bool pos = fs.e_pos <= fs.e_neg;
                const double e = pos ? fs.e_pos : fs.e_neg;
                if (e < best.eps) best = WgBest{e, j, pos ? 1 : -1, pos ? fs.lane_pos : fs.lane_neg};
            }
            t += nsteps;
            if (f0 + t * G >= f1) break;
            j = f0 + t * G + grp;
        }
        return best;
    }
};

// Scans features [f0, f1) of one job with the LDS table `tab` already filled:
// groups of LPF lanes take one feature each, the g-th group-step of the
// calling wave handles features f0 + (step0 + g * nsteps) * G + group.
// Returns this lane's best candidate (the same in every lane of a group).
//
// Two load disciplines.  Batched (RING = false): a lane loads UNROLL units,
// scans them, then loads the next UNROLL; the next feature's first batch is
// loaded before the current feature's epilogue.  Rotating (RING = true): each
// of the UNROLL register slots is reloaded as soon as its unit is scanned,
// with the unit one batch later -- across feature boundaries too -- so a
// lane keeps UNROLL units in flight all the time at no register cost; lanes
// then scan a whole number of batches per feature (the last one padded).
template <int PREC, bool NARROW, int UNROLL, int LPF, bool RING = false>
__device__ __forceinline__ WgBest scan_range(const JobDev& jd, const typename ScanTypes<PREC>::W* tab, int64_t f0,
                                             int64_t f1, int64_t step0, int64_t nsteps, double tp, double tn,
                                             double2* __restrict__ ferr) {
    constexpr int G = 64 / LPF;
    constexpr int H = UNROLL / 2;
    static_assert(UNROLL % 2 == 0, "batches of an even number of units (the tail batch is half a batch)");
    const int lane = threadIdx.x & 63;
    const int grp = lane / LPF, L = lane % LPF;
    const int cnt = jd.g.q + (L < jd.g.rem ? 1 : 0);
    // Units per lane (the longest lane) = nbf full batches, then a half batch
    // when at most UNROLL / 2 units remain (and at least one full batch came
    // before).  Only the last batch can reach past a lane's own units (into
    // the padding unit).
    const int per = jd.g.q + (jd.g.rem > 0 ? 1 : 0);
    const int rest = per % UNROLL;
    const bool half = rest > 0 && rest <= H && per > UNROLL;
    const int nbf = per / UNROLL + (rest > 0 && !half ? 1 : 0);
    const int nb = nbf + (half ? 1 : 0);
    WgBest best{DBL_MAX, -1, 0, -1};
    // features past f1 read the padding unit (stride 0) and are dropped
    auto row_of = [&](int64_t j, int& stride) -> const uint4* {
        if (j < f1) { stride = LPF; return jd.keys + j * jd.g.row_units + L; }
        stride = 0;
        return jd.pad;
    };
    int64_t t = step0;
    int64_t j = f0 + t * G + grp;
    if (f0 + t * G >= f1) return best;
    if constexpr (RING) {
        RingScan<PREC, NARROW, UNROLL, LPF> rs;
        rs.prime(jd, f0, f1, step0, nsteps);
        return rs.run(jd, tab, tp, tn, ferr);
    }
    uint4 u[UNROLL];
    // batch 0 of the next feature is loaded before the current feature's
    // group epilogue, so loads stay in flight across features
    int stride;
    const uint4* p = row_of(j, stride);
    load_batch<UNROLL>(u, p, stride, 0, nb, stride ? cnt : 0, jd.pad);
    while (true) {
        LaneAcc<PREC> a;
#pragma unroll
        for (int k = 0; k < UNROLL; ++k) scan_unit<PREC, NARROW>(a, tab, u[k], (k & 1) != 0);
        for (int b = 1; b < nbf; ++b) {
            load_batch<UNROLL>(u, p, stride, b, nb, stride ? cnt : 0, jd.pad);
#pragma unroll
            for (int k = 0; k < UNROLL; ++k) scan_unit<PREC, NARROW>(a, tab, u[k], (k & 1) != 0);
        }
        if (half) {
            load_tail<H>(u, p, stride, nbf * UNROLL, stride ? cnt : 0, jd.pad);
#pragma unroll
            for (int k = 0; k < H; ++k) scan_unit<PREC, NARROW>(a, tab, u[k], (k & 1) != 0);
        }
        const int64_t jcur = j;
        t += nsteps;
        const bool more = f0 + t * G < f1;
        if (more) {
            j = f0 + t * G + grp;
            p = row_of(j, stride);
            load_batch<UNROLL>(u, p, stride, 0, nb, stride ? cnt : 0, jd.pad);
        }
        const FeatureScan fs = finish_feature<PREC, LPF>(a, lane, tp, tn);
        if (jcur < f1) {
            if (ferr != nullptr && L == 0) ferr[jcur] = make_double2(fs.e_pos, fs.e_neg);
            const bool pos = fs.e_pos <= fs.e_neg;
            const double e = pos ? fs.e_pos : fs.e_neg;
            if (e < best.eps) best = WgBest{e, jcur, pos ? 1 : -1, pos ? fs.lane_pos : fs.lane_neg};
        }
        if (!more) break;
    }
    return best;
}

// Reduces the groups' candidates of a workgroup (group leaders write theirs
// to lds wb[]) and returns the workgroup's best in thread 0.
template <int NG>
__device__ __forceinline__ WgBest block_best(WgBest* wb, const WgBest& mine, int lpf) {
    const int lane = threadIdx.x & 63;
    if ((lane % lpf) == 0) wb[(threadIdx.x >> 6) * (64 / lpf) + lane / lpf] = mine;
    __syncthreads();
    WgBest b = wb[0];
    if (threadIdx.x == 0)
        for (int k = 1; k < NG; ++k)
            if (better(wb[k], b)) b = wb[k];
    return b;
}

}  // namespace vjb
