// Device building blocks of the per-round weighted-error scan and of the
// weight preparation, shared by the single-job and the batched kernels.
//
// For one feature, the windows in ascending value order with signed weights
// w^_i = +w_i (positive) / -w_i (negative) give the running sum
//   D_k = S+_k - S-_k   over the first k ranks,
// and, at every realisable split k (k = 0 or the end of a run of equal values),
//   e(+1, k) = S-_k + (T+ - S+_k) = T+ - D_k
//   e(-1, k) = S+_k + (T- - S-_k) = T- + D_k
// (Section 2.3: eps = min over f, p, theta of sum_i w_i |h - y_i|, with
// h = 1 iff p f < p theta, Section 2.2).  The best split of a feature is thus
// the largest D_k (p = +1) and the smallest D_k (p = -1) over split points.
//
// A group of LPF lanes (16 by default; a wave holds 64 / LPF groups) scans a
// feature: lane L walks its contiguous segment of ranks, keeping its local
// running sum and the largest / smallest local sum at a run end; an exclusive
// scan of the lane totals across the group then shifts each lane's extremes
// to global D values.  max_k (base + L_k) = base + max_k L_k, so one pass
// over the keys suffices.
#pragma once

#include "common.h"

namespace vjb {

// Masked candidates: at a position that is not the end of a run of equal
// values the candidate becomes a quiet NaN, which v_max / v_min ignore.  The
// mask is added rather than merged: a candidate is v + z with z = +0 (a split
// here: v + 0 = v exactly, -0 aside, which compares equal to +0) or z = the
// all-ones pattern, a quiet NaN (no split: the IEEE sum of a number and a
// quiet NaN is a quiet NaN).  The addition writes a fresh register (pair), so
// the running sum needs no copy.  Both steps are defined behaviour: NaNs are
// honoured in every translation unit (no -ffast-math, no -fno-honor-nans), an
// IEEE addition with a quiet NaN operand returns a quiet NaN, and fmax / fmin
// (LLVM maxnum / minnum, IEEE-754 maxNum / minNum) return the other operand
// when one operand is a quiet NaN.  The sum is an arithmetic result, which
// the compiler knows is not a signalling NaN, so no canonicalisation is
// inserted in front of the max / min.
__device__ __forceinline__ double nan_or_zero(uint32_t m) {
    return __longlong_as_double((long long)((uint64_t)m << 32));
}
__device__ __forceinline__ float nan_or_zero32(uint32_t m) { return __uint_as_float(m); }

// Bit b of d as an all-ones / all-zeros mask.
__device__ __forceinline__ uint32_t bitmask(uint32_t d, int b) {
    return (uint32_t)(((int32_t)(d << (31 - b))) >> 31);
}

// v_max_f64 / v_min_f64 of a value and a candidate that may be a quiet NaN
// (never a signalling one): in the hardware's IEEE mode the result is then
// the other operand (IEEE-754 maxNum / minNum).  Issued directly because
// the compiler, not knowing that an integer-masked value is not a
// signalling NaN, would otherwise first quiet it with an extra max.
__device__ __forceinline__ double max_qnan(double a, double b) {
    double r;
    asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ double min_qnan(double a, double b) {
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

template <int PREC> struct ScanTypes;
template <> struct ScanTypes<BOOST_PREC_FP32>       { using W = float;  using A = float;  };
template <> struct ScanTypes<BOOST_PREC_FP32_KAHAN> { using W = float;  using A = double; };
template <> struct ScanTypes<BOOST_PREC_FP64>       { using W = double; using A = double; };
template <> struct ScanTypes<BOOST_PREC_FP32_WIDE>  { using W = float;  using A = double; };

// Per-lane accumulator.  A = type used across lanes and for the final errors.
// key(w, m): add the next key's table value w to the running sum; the sum is
// a candidate unless m is all ones (no split after this rank).  total(),
// vmax(), vmin(): the lane's local sum and extremes (vmax = -4 / vmin = +4
// when the lane holds no split point: every real prefix lies in [-1, 1]).
template <int PREC> struct LaneAcc;

template <> struct LaneAcc<BOOST_PREC_FP32> {
    float s = 0.f, mx = -4.f, mn = 4.f;
    __device__ __forceinline__ void key(float w, uint32_t m) {
        s += w;
        const float c = s + nan_or_zero32(m);
        mx = fmaxf(mx, c);
        mn = fminf(mn, c);
    }
    __device__ __forceinline__ void unit_end() {}
    __device__ __forceinline__ float total() const { return s; }
    __device__ __forceinline__ float vmax() const { return mx; }
    __device__ __forceinline__ float vmin() const { return mn; }
};

// Compensated FP32 running sum.  The sum is carried as s + c with s biased
// by kKahanBias: s = fl(s + w) tracks kKahanBias + (local prefix), and c
// collects the exact rounding error of every step.  The local prefix of a
// lane lies in [-1, 1] (the table's absolute values sum to 1), so s stays in
// [1, 3] and |w| <= 1 <= |s|: Dekker's Fast2Sum then gives the error of
// s + w exactly as w - ((s + w) - s), three FP32 operations instead of the
// six of a sign-agnostic two-sum.  s + c equals the biased prefix up to the
// rounding of the additions to c, each at most 2^-24 |c|.  Weights below
// half an ulp of s (2^-23) pass into c whole, so c is folded back into s
// after every 16 keys (unit_end: one more exact Fast2Sum, |c| < 1 <= |s|),
// which keeps |c| below about 17 * 2^-23 and each rounding of c below
// 2^-45.  A candidate is s + c evaluated in FP64
// (exact for two floats of these magnitudes); rounding it to FP32 would cost
// 2^-24 of the prefix, more than a 1e-6 relative error once the minimal
// error is below a few percent.
constexpr float kKahanBias = 2.0f;

template <> struct LaneAcc<BOOST_PREC_FP32_KAHAN> {
    float s = kKahanBias, c = 0.f;
    double mx = (double)kKahanBias - 4.0, mn = (double)kKahanBias + 4.0;
    // One unit of eight keys.  s and c step through the eight weights
    // (Fast2Sum for s, the errors added to c in key order).  Only the last
    // key's candidate is formed from s + c; each earlier key's is the next
    // one's minus the next key's weight, in FP64.  The compensated sums
    // after keys k and k + 1 differ by w_{k+1} up to the rounding of one
    // addition to c (at most 2^-24 |c|), and each FP64 subtraction rounds by
    // at most 2^-53 * 4, so every candidate stays within about 1e-12 of the
    // compensated sum at its key.  That is one convert and one FP64
    // operation per key, plus two per unit.  Each candidate is masked by an
    // integer OR of the all-ones pattern into its high word (a quiet NaN,
    // which the maximum and minimum skip) where the key ends no run; the
    // pattern is taken from the key's no-split bit (bit 0 of its dword for
    // the low key, bit 1 or 16 for the high one) where it is used, to keep
    // few registers live.
    template <bool NARROW>
    __device__ __forceinline__ void unit8(const float* w, const uint32_t* d) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const float t = s + w[k];
            const float z = t - s;  // exact: |s| >= |w|
            c += w[k] - z;          // w - z is exact: the rounding error of s + w
            s = t;
        }
        double v = (double)s + (double)c;
#pragma unroll
        for (int k = 7; k >= 0; --k) {
            // the next candidate first: the mask then overwrites v's high word in place
            const double vn = k > 0 ? v - (double)w[k] : 0.0;
            const uint32_t m = bitmask(d[k >> 1], (k & 1) ? (NARROW ? 1 : 16) : 0);
            const double cv = __longlong_as_double(__double_as_longlong(v) | (long long)((uint64_t)m << 32));
            mx = max_qnan(mx, cv);
            mn = min_qnan(mn, cv);
            v = vn;
        }
    }
    __device__ __forceinline__ void unit_end() {
        const float t = s + c;
        const float z = t - s;      // exact: |s| >= 1 > |c|
        c = c - z;
        s = t;
    }
    __device__ __forceinline__ double total() const { return ((double)s - (double)kKahanBias) + (double)c; }
    __device__ __forceinline__ double vmax() const { return mx - (double)kKahanBias; }
    __device__ __forceinline__ double vmin() const { return mn - (double)kKahanBias; }
};

template <> struct LaneAcc<BOOST_PREC_FP64> {
    double s = 0.0, mx = -4.0, mn = 4.0;
    __device__ __forceinline__ void key(double w, uint32_t m) {
        s += w;
        const double c = s + nan_or_zero(m);
        mx = fmax(mx, c);
        mn = fmin(mn, c);
    }
    __device__ __forceinline__ void unit_end() {}
    __device__ __forceinline__ double total() const { return s; }
    __device__ __forceinline__ double vmax() const { return mx; }
    __device__ __forceinline__ double vmin() const { return mn; }
};

template <> struct LaneAcc<BOOST_PREC_FP32_WIDE> {
    double s = 0.0, mx = -4.0, mn = 4.0;
    __device__ __forceinline__ void key(float w, uint32_t m) {
        s += (double)w;
        const double c = s + nan_or_zero(m);
        mx = fmax(mx, c);
        mn = fmin(mn, c);
    }
    __device__ __forceinline__ void unit_end() {}
    __device__ __forceinline__ double total() const { return s; }
    __device__ __forceinline__ double vmax() const { return mx; }
    __device__ __forceinline__ double vmin() const { return mn; }
};

// Weight of the window whose key sits in the low / high half of d.
template <typename Wt, bool NARROW>
__device__ __forceinline__ Wt tab_lo(const Wt* tab, uint32_t d) {
    if constexpr (sizeof(Wt) == 4) {
        const uint32_t off = NARROW ? (d & 0xFFFCu) : ((d << 1) & 0x1FFFCu);
        return *(const Wt*)((const char*)tab + off);
    } else {
        const uint32_t off = NARROW ? ((d << 1) & 0x1FFF8u) : ((d << 2) & 0x3FFF8u);
        return *(const Wt*)((const char*)tab + off);
    }
}
template <typename Wt, bool NARROW>
__device__ __forceinline__ Wt tab_hi(const Wt* tab, uint32_t d) {
    if constexpr (sizeof(Wt) == 4) {
        const uint32_t off = NARROW ? (d >> 16) : ((d >> 15) & 0x1FFFCu);
        return *(const Wt*)((const char*)tab + off);
    } else {
        const uint32_t off = NARROW ? ((d >> 15) & 0x1FFF8u) : ((d >> 14) & 0x3FFF8u);
        return *(const Wt*)((const char*)tab + off);
    }
}
// All ones where the key in the low / high half of d is not the end of a run
// (no split after it), zero where it is.
template <bool NARROW>
__device__ __forceinline__ uint32_t nosplit_lo(uint32_t d) { return bitmask(d, 0); }
template <bool NARROW>
__device__ __forceinline__ uint32_t nosplit_hi(uint32_t d) { return NARROW ? bitmask(d, 1) : bitmask(d, 16); }

template <int PREC, bool NARROW>
__device__ __forceinline__ void scan_dword(LaneAcc<PREC>& a, const typename ScanTypes<PREC>::W* tab, uint32_t d) {
    using Wt = typename ScanTypes<PREC>::W;
    a.key(tab_lo<Wt, NARROW>(tab, d), nosplit_lo<NARROW>(d));
    a.key(tab_hi<Wt, NARROW>(tab, d), nosplit_hi<NARROW>(d));
}

// One unit (8 keys).  The compensated mode folds its correction back into
// the running sum after every odd unit of a lane's segment (unit index r odd):
// every load discipline scans a lane's units in order with batches of an even
// length starting at even r, so the odd-k units of a batch are exactly the
// odd-r units, and the results do not depend on the schedule.
template <int PREC, bool NARROW>
__device__ __forceinline__ void scan_unit(LaneAcc<PREC>& a, const typename ScanTypes<PREC>::W* tab, const uint4& u,
                                          bool odd) {
    if constexpr (PREC == BOOST_PREC_FP32_KAHAN) {
        const uint32_t d[4] = {u.x, u.y, u.z, u.w};
        float w[8];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            w[2 * q] = tab_lo<float, NARROW>(tab, d[q]);
            w[2 * q + 1] = tab_hi<float, NARROW>(tab, d[q]);
        }
        a.template unit8<NARROW>(w, d);
    } else {
        scan_dword<PREC, NARROW>(a, tab, u.x);
        scan_dword<PREC, NARROW>(a, tab, u.y);
        scan_dword<PREC, NARROW>(a, tab, u.z);
        scan_dword<PREC, NARROW>(a, tab, u.w);
    }
    if (odd) a.unit_end();
}

// Streaming 16-byte load of keys (read once per round; not worth caching).
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 ld_stream(const uint4* p) {
    const u32x4_t v = __builtin_nontemporal_load((const u32x4_t*)p);
    return make_uint4(v.x, v.y, v.z, v.w);
}

// ---------------------------------------------------------------- cross-lane (DPP)
// Value of another lane selected by a DPP control (CDNA wave64 encodings:
// 0x111.. row_shr:k, 0x138 wave_shr:1, 0x140 row_mirror, 0x141
// row_half_mirror, 0x142 row_bcast:15, 0x143 row_bcast:31, 0x00-0xFF
// quad_perm); lanes that receive nothing keep `old`.
template <int CTRL, int RM, int BM, bool BC>
__device__ __forceinline__ double dpp(double v, double old) {
    const long long b = __double_as_longlong(v), o = __double_as_longlong(old);
    const int lo = __builtin_amdgcn_update_dpp((int)(uint32_t)o, (int)(uint32_t)b, CTRL, RM, BM, BC);
    const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(b >> 32), CTRL, RM, BM, BC);
    return __longlong_as_double(((long long)hi << 32) | (uint32_t)lo);
}
template <int CTRL, int RM, int BM, bool BC>
__device__ __forceinline__ float dpp(float v, float old) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), CTRL, RM, BM, BC));
}
__device__ __forceinline__ double read_lane(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(uint32_t)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (uint32_t)lo);
}
__device__ __forceinline__ float read_lane(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Exclusive prefix of the lane totals within each group of LPF lanes (16, 32
// or 64), in a fixed order: inclusive scan within rows of 16 (shifts 1, 2, 4,
// 8); for groups of 32 or 64, row 0's total into row 1 and row 2's into row
// 3; for 64, rows 0-1's total into rows 2-3; finally a shift by one lane with
// zero at each group's first lane.
template <int LPF, typename A>
__device__ __forceinline__ A group_exclusive(A tot, int lane) {
    A v = tot;
    v += dpp<0x111, 0xF, 0xF, true>(v, (A)0);
    v += dpp<0x112, 0xF, 0xF, true>(v, (A)0);
    v += dpp<0x114, 0xF, 0xF, true>(v, (A)0);
    v += dpp<0x118, 0xF, 0xF, true>(v, (A)0);
    if constexpr (LPF >= 32) v += dpp<0x142, 0xA, 0xF, false>(v, (A)0);
    if constexpr (LPF == 64) v += dpp<0x143, 0xC, 0xF, false>(v, (A)0);
    const A ex = dpp<0x138, 0xF, 0xF, true>(v, (A)0);   // wave_shr:1
    return (lane & (LPF - 1)) == 0 ? (A)0 : ex;
}

// Maximum (MAX) or minimum over each group of LPF lanes, in every lane of the group.
template <int LPF, bool MAX, typename A>
__device__ __forceinline__ A group_extreme(A v, int lane) {
    auto op = [](A a, A b) { return MAX ? fmax(a, b) : fmin(a, b); };
    v = op(v, dpp<0xB1, 0xF, 0xF, false>(v, v));    // quad_perm [1,0,3,2]
    v = op(v, dpp<0x4E, 0xF, 0xF, false>(v, v));    // quad_perm [2,3,0,1]
    v = op(v, dpp<0x141, 0xF, 0xF, false>(v, v));   // row_half_mirror
    v = op(v, dpp<0x140, 0xF, 0xF, false>(v, v));   // row_mirror: every lane has its row's extreme
    if constexpr (LPF == 16) {
        return v;
    } else if constexpr (LPF == 32) {
        v = op(v, dpp<0x142, 0xA, 0xF, false>(v, v));   // rows 1 and 3 now hold their pair's extreme
        const A lo = read_lane(v, 31), hi = read_lane(v, 63);
        return lane < 32 ? lo : hi;
    } else {
        v = op(v, dpp<0x142, 0xA, 0xF, false>(v, v));
        v = op(v, dpp<0x143, 0xC, 0xF, false>(v, v));
        return read_lane(v, 63);
    }
}

// Result of one feature's scan, identical in every lane of its group.
struct FeatureScan {
    double e_pos, e_neg;     // best error for p = +1 / p = -1
    int lane_pos, lane_neg;  // first lane (within the group) holding the extreme (-1: the empty split k = 0)
};

// Loads batch b (UNROLL units) of one lane's segment; units are `stride`
// apart.  All batches but the last (nb - 1) are full for every lane; in the
// last one, units past the lane's segment come from `pad` (a unit of padding
// keys, cache resident), so the loads need no branches.
template <int UNROLL>
__device__ __forceinline__ void load_batch(uint4* u, const uint4* __restrict__ p, int stride, int b, int nb, int cnt,
                                           const uint4* __restrict__ pad) {
    if (b + 1 < nb) {
#pragma unroll
        for (int k = 0; k < UNROLL; ++k) u[k] = ld_stream(p + stride * (b * UNROLL + k));
    } else {
#pragma unroll
        for (int k = 0; k < UNROLL; ++k) {
            const int r = b * UNROLL + k;
            u[k] = ld_stream(r < cnt ? p + stride * r : pad);
        }
    }
}

// H units from unit `start` on; units at or past cnt read the padding unit.
template <int H>
__device__ __forceinline__ void load_tail(uint4* u, const uint4* __restrict__ p, int stride, int start, int cnt,
                                          const uint4* __restrict__ pad) {
#pragma unroll
    for (int k = 0; k < H; ++k) {
        const int r = start + k;
        u[k] = ld_stream(r < cnt ? p + stride * r : pad);
    }
}

// Group-level end of one feature's scan: lane totals -> exclusive prefix ->
// extremes of the running sum at run ends -> errors for both polarities.
template <int PREC, int LPF>
__device__ __forceinline__ FeatureScan finish_feature(const LaneAcc<PREC>& a, int lane, double t_pos, double t_neg) {
    using A = typename ScanTypes<PREC>::A;
    const A base = group_exclusive<LPF, A>((A)a.total(), lane);
    const A lmx = base + (A)a.vmax();
    const A lmn = base + (A)a.vmin();
    A cmx = group_extreme<LPF, true>(lmx, lane);
    A cmn = group_extreme<LPF, false>(lmn, lane);
    const int sh = (lane / LPF) * LPF;
    const unsigned long long gm = LPF == 64 ? ~0ull : ((1ull << LPF) - 1ull);
    FeatureScan r;
    // k = 0 (nothing below the threshold) is always realisable: D_0 = 0, and
    // it is the smallest split, so it wins ties.
    const unsigned long long bx = (__ballot(lmx == cmx) >> sh) & gm;
    const unsigned long long bn = (__ballot(lmn == cmn) >> sh) & gm;
    r.lane_pos = cmx > (A)0 ? __ffsll(bx) - 1 : -1;
    r.lane_neg = cmn < (A)0 ? __ffsll(bn) - 1 : -1;
    cmx = fmax(cmx, (A)0);
    cmn = fmin(cmn, (A)0);
    r.e_pos = (double)((A)t_pos - cmx);
    r.e_neg = (double)((A)t_neg + cmn);
    return r;
}

// ---------------------------------------------------------------- block sums
// Sum of v(i), i in [0, n), in an order that does not depend on the block
// size (>= 256 threads): thread t < 256 adds v(t), v(t + 256), ... in turn;
// lane 0 of each of the four waves takes a fixed butterfly; the four wave sums
// are added in order.  Every thread returns the same value.  sh: 4 doubles.
template <typename Fn>
__device__ __forceinline__ double fixed_sum256(int64_t n, Fn v, double* sh) {
    double p = 0.0;
    if (threadIdx.x < 256)
        for (int64_t i = threadIdx.x; i < n; i += 256) p += v(i);
#pragma unroll
    for (int o = 32; o; o >>= 1) p += __shfl_xor(p, o);
    __syncthreads();
    if (threadIdx.x < 256 && (threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = p;
    __syncthreads();
    const double s = ((sh[0] + sh[1]) + sh[2]) + sh[3];
    __syncthreads();
    return s;
}

// S = sum of the stored weights from the update workgroups' partial sums, in
// a fixed order (lane k adds partials k and k + 64; a fixed butterfly; lane
// 0's value).  Needs a whole wave; every lane returns the same value.
__device__ __forceinline__ double weight_sum(const JobDev& jd) {
    const int lane = threadIdx.x & 63;
    double p = lane < jd.n_part ? jd.wpart[lane] : 0.0;
    if (lane + 64 < jd.n_part) p += jd.wpart[lane + 64];
#pragma unroll
    for (int o = 32; o; o >>= 1) p += __shfl_xor(p, o);
    return __shfl(p, 0);
}

// Every table value is a multiple of 2^-52 and the table's absolute values
// sum to about 1, so the FP64 sum of any subset of the table, in any order,
// is exact: the class totals, every prefix of the FP64 modes' scans, and the
// update kernel's recomputation of a lane's prefixes.  In the FP32_WIDE and
// FP64 modes the scan's own sums are therefore exact and order-independent.
// One entry of the scan's signed weight table: the normalised weight
// w_i * (1 / S) rounded to the table type and to a multiple of 2^-52 (FP32
// values of magnitude >= 2^-28 already are one; smaller ones move by at most
// 2^-53), negated for negatives.
template <int PREC>
__device__ __forceinline__ typename ScanTypes<PREC>::W table_value(double w, double rS, bool positive) {
    using Wt = typename ScanTypes<PREC>::W;
    constexpr double kGrid = 4503599627370496.0;          // 2^52
    constexpr double kInvGrid = 1.0 / 4503599627370496.0;  // 2^-52
    Wt wn = (Wt)(w * rS);
    if constexpr (sizeof(Wt) == 8) {
        wn = rint(wn * kGrid) * kInvGrid;
    } else {
        if (wn < (Wt)3.7252902984619140625e-9f)           // 2^-28
            wn = (Wt)(rint((double)wn * kGrid) * kInvGrid);
    }
    return positive ? wn : -wn;
}

// Section 2.3 step 1, normalisation, fused into the scan's table fill: the
// signed table, a zero entry at n for padding keys, and the class totals T+ /
// T- of the table (one fixed-order pass: thread t < 256 adds entries t, t +
// 256, ... into T+ or T-, then a fixed butterfly per wave and the four wave
// sums in order).  Every workgroup computes the same values.
template <int PREC>
__device__ __forceinline__ void fill_table(const JobDev& jd, const double* w, typename ScanTypes<PREC>::W* tab,
                                           double rS, int nt, double* sh, double& tp, double& tn) {
    using Wt = typename ScanTypes<PREC>::W;
    const int64_t n = jd.g.n;
    const int64_t l = jd.st->n_pos;
    for (int64_t i = threadIdx.x; i < n; i += nt) tab[i] = table_value<PREC>(w[i], rS, i < l);
    if (threadIdx.x == 0) tab[n] = (Wt)0;
    __syncthreads();
    double p = 0.0, q = 0.0;
    if (threadIdx.x < 256)
        for (int64_t i = threadIdx.x; i < n; i += 256) {
            const double v = (double)tab[i];
            if (i < l) p += v; else q -= v;
        }
#pragma unroll
    for (int o = 32; o; o >>= 1) { p += __shfl_xor(p, o); q += __shfl_xor(q, o); }
    if (threadIdx.x < 256 && (threadIdx.x & 63) == 0) { sh[threadIdx.x >> 6] = p; sh[4 + (threadIdx.x >> 6)] = q; }
    __syncthreads();
    tp = ((sh[0] + sh[1]) + sh[2]) + sh[3];
    tn = ((sh[4] + sh[5]) + sh[6]) + sh[7];
}

// Stored weights w and their partial sums for a fresh weight vector: one
// partial holding the whole (fixed-order) sum, the rest zero.
__device__ __forceinline__ void reset_partials(const JobDev& jd, const double* w, double* sh) {
    const double s = fixed_sum256(jd.g.n, [&](int64_t i) { return w[i]; }, sh);
    for (int k = threadIdx.x; k < jd.n_part; k += blockDim.x) jd.wpart[k] = k == 0 ? s : 0.0;
}

}  // namespace vjb
