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
// A wave scans a feature: lane L walks its contiguous segment of ranks,
// keeping its local running sum and the largest / smallest local sum at a run
// end; an exclusive wave scan of the lane totals then shifts each lane's
// extremes to global D values.  max_k (base + L_k) = base + max_k L_k, so one
// pass over the keys suffices.
#pragma once

#include "common.h"

namespace vjb {

// Masked candidates: a position that is not the end of a run of equal values
// becomes a quiet NaN, which v_max / v_min ignore (IEEE maxNum / minNum: a
// quiet NaN operand yields the other operand).  The scan translation unit is
// built with -fno-honor-nans so that no canonicalisation is inserted around
// these operations; no NaN ever reaches an arithmetic operation.
constexpr uint32_t kQNaNHi = 0x7FF80000u;   // high dword of a double quiet NaN
constexpr uint32_t kQNaN32 = 0x7FC00000u;   // float quiet NaN

__device__ __forceinline__ double with_hi(double v, uint32_t m, uint32_t alt_hi) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t hi = ((uint32_t)(b >> 32) & m) | (alt_hi & ~m);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | (uint32_t)b));
}
__device__ __forceinline__ float with_bits(float v, uint32_t m, uint32_t alt) {
    return __uint_as_float((__float_as_uint(v) & m) | (alt & ~m));
}

// Bit b of d as an all-ones / all-zeros mask.
__device__ __forceinline__ uint32_t bitmask(uint32_t d, int b) {
    return (uint32_t)(((int32_t)(d << (31 - b))) >> 31);
}

template <int PREC> struct ScanTypes;
template <> struct ScanTypes<BOOST_PREC_FP32>       { using W = float;  using A = float;  };
template <> struct ScanTypes<BOOST_PREC_FP32_KAHAN> { using W = float;  using A = double; };
template <> struct ScanTypes<BOOST_PREC_FP64>       { using W = double; using A = double; };
template <> struct ScanTypes<BOOST_PREC_FP32_WIDE>  { using W = float;  using A = double; };

// Per-lane accumulator.  A = type used across lanes and for the final errors.
template <int PREC> struct LaneAcc;

template <> struct LaneAcc<BOOST_PREC_FP32> {
    float s = 0.f, mx = -4.f, mn = 4.f;
    __device__ __forceinline__ float add(float w) { s += w; return s; }
    __device__ __forceinline__ void cand(float v, uint32_t m) {
        const float c = with_bits(v, m, kQNaN32);
        mx = fmaxf(mx, c);
        mn = fminf(mn, c);
    }
    __device__ __forceinline__ float total() const { return s; }
    __device__ __forceinline__ float vmax() const { return mx; }
    __device__ __forceinline__ float vmin() const { return mn; }
};

// Two-sum (Knuth) compensated running sum in FP32: s + c carries the prefix
// with an error of order u^2 per step; candidates are the FP32 value s + c.
template <> struct LaneAcc<BOOST_PREC_FP32_KAHAN> {
    float s = 0.f, c = 0.f, mx = -4.f, mn = 4.f;
    __device__ __forceinline__ float add(float w) {
        const float t = s + w;
        const float bp = t - s;
        const float err = (s - (t - bp)) + (w - bp);
        s = t;
        c += err;
        return s + c;
    }
    __device__ __forceinline__ void cand(float v, uint32_t m) {
        const float c = with_bits(v, m, kQNaN32);
        mx = fmaxf(mx, c);
        mn = fminf(mn, c);
    }
    __device__ __forceinline__ double total() const { return (double)s + (double)c; }
    __device__ __forceinline__ double vmax() const { return (double)mx; }
    __device__ __forceinline__ double vmin() const { return (double)mn; }
};

template <> struct LaneAcc<BOOST_PREC_FP64> {
    double s = 0.0, mx = -4.0, mn = 4.0;
    __device__ __forceinline__ double add(double w) { s += w; return s; }
    __device__ __forceinline__ void cand(double v, uint32_t m) {
        const double c = with_hi(v, m, kQNaNHi);
        mx = fmax(mx, c);
        mn = fmin(mn, c);
    }
    __device__ __forceinline__ double total() const { return s; }
    __device__ __forceinline__ double vmax() const { return mx; }
    __device__ __forceinline__ double vmin() const { return mn; }
};

template <> struct LaneAcc<BOOST_PREC_FP32_WIDE> {
    double s = 0.0, mx = -4.0, mn = 4.0;
    __device__ __forceinline__ double add(float w) { s += (double)w; return s; }
    __device__ __forceinline__ void cand(double v, uint32_t m) {
        const double c = with_hi(v, m, kQNaNHi);
        mx = fmax(mx, c);
        mn = fmin(mn, c);
    }
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
template <bool NARROW>
__device__ __forceinline__ uint32_t flag_lo(uint32_t d) { return bitmask(d, 0); }
template <bool NARROW>
__device__ __forceinline__ uint32_t flag_hi(uint32_t d) { return NARROW ? bitmask(d, 1) : bitmask(d, 16); }

template <int PREC, bool NARROW>
__device__ __forceinline__ void scan_dword(LaneAcc<PREC>& a, const typename ScanTypes<PREC>::W* tab, uint32_t d) {
    using Wt = typename ScanTypes<PREC>::W;
    const Wt w0 = tab_lo<Wt, NARROW>(tab, d);
    const Wt w1 = tab_hi<Wt, NARROW>(tab, d);
    a.cand(a.add(w0), flag_lo<NARROW>(d));
    a.cand(a.add(w1), flag_hi<NARROW>(d));
}

template <int PREC, bool NARROW>
__device__ __forceinline__ void scan_unit(LaneAcc<PREC>& a, const typename ScanTypes<PREC>::W* tab, const uint4& u) {
    scan_dword<PREC, NARROW>(a, tab, u.x);
    scan_dword<PREC, NARROW>(a, tab, u.y);
    scan_dword<PREC, NARROW>(a, tab, u.z);
    scan_dword<PREC, NARROW>(a, tab, u.w);
}

// Streaming 16-byte load of keys (read once per round; not worth caching).
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 ld_stream(const uint4* p) {
    const u32x4_t v = __builtin_nontemporal_load((const u32x4_t*)p);
    return make_uint4(v.x, v.y, v.z, v.w);
}

// Exclusive wave prefix of the lane totals (fixed order: Hillis-Steele).
template <typename A>
__device__ __forceinline__ A wave_exclusive(A tot, int lane) {
    A incl = tot;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const A y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    A ex = __shfl_up(incl, 1);
    return lane == 0 ? (A)0 : ex;
}

// One wave scans one feature's row; returns (e+, e-) in every lane.
// row points at the feature's first unit; cnt = units of this lane.
template <int PREC, bool NARROW, int UNROLL>
__device__ __forceinline__ void scan_feature(const uint4* __restrict__ row, int lane, int cnt,
                                             const typename ScanTypes<PREC>::W* tab, double t_pos,
                                             double t_neg, double& e_pos, double& e_neg) {
    using A = typename ScanTypes<PREC>::A;
    LaneAcc<PREC> a;
    const uint4* p = row + lane;
    int r = 0;
    for (; r + UNROLL <= cnt; r += UNROLL) {
        uint4 u[UNROLL];
#pragma unroll
        for (int k = 0; k < UNROLL; ++k) u[k] = ld_stream(p + 64 * k);
        p += 64 * UNROLL;
#pragma unroll
        for (int k = 0; k < UNROLL; ++k) scan_unit<PREC, NARROW>(a, tab, u[k]);
    }
    for (; r < cnt; ++r) {
        const uint4 u = ld_stream(p);
        p += 64;
        scan_unit<PREC, NARROW>(a, tab, u);
    }
    const A base = wave_exclusive<A>((A)a.total(), lane);
    A cmx = base + (A)a.vmax();
    A cmn = base + (A)a.vmin();
#pragma unroll
    for (int o = 32; o; o >>= 1) {
        cmx = fmax(cmx, __shfl_xor(cmx, o));
        cmn = fmin(cmn, __shfl_xor(cmn, o));
    }
    // k = 0 (nothing below the threshold) is always realisable: D_0 = 0.
    cmx = fmax(cmx, (A)0);
    cmn = fmin(cmn, (A)0);
    e_pos = (double)((A)t_pos - cmx);
    e_neg = (double)((A)t_neg + cmn);
}

// ---------------------------------------------------------------- block reductions
// Deterministic for a fixed block size: per-thread partials in a fixed
// stride pattern, a fixed butterfly per wave, then wave partials in order.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
#pragma unroll
    for (int o = 32; o; o >>= 1) v += __shfl_xor(v, o);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double s = 0.0;
    for (int k = 0; k < NT / 64; ++k) s += sh[k];
    return s;
}

// Weight preparation (Section 2.3 step 1, normalisation): w <- w / sum w, the
// scan's signed table w^ (rounded to the table type) with a zero entry at n
// for padding keys, and the class totals T+ / T- of that table.
// Windows are in internal order, positives (i < l) first.
template <int NT>
__device__ void prep_weights(const JobDev& jd, double* sh) {
    const int64_t n = jd.g.n;
    const int64_t l = jd.st->n_pos;
    double part = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += NT) part += jd.w[i];
    const double sum = block_sum<NT>(part, sh);
    const bool fp64 = jd.precision == BOOST_PREC_FP64;
    double tp = 0.0, tn = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += NT) {
        const double wn = jd.w[i] / sum;
        jd.w[i] = wn;
        if (fp64) {
            ((double*)jd.wtab)[i] = i < l ? wn : -wn;
            if (i < l) tp += wn; else tn += wn;
        } else {
            const float wf = (float)wn;
            ((float*)jd.wtab)[i] = i < l ? wf : -wf;
            if (i < l) tp += (double)wf; else tn += (double)wf;
        }
    }
    if (threadIdx.x == 0) {
        if (fp64) ((double*)jd.wtab)[n] = 0.0; else ((float*)jd.wtab)[n] = 0.f;
    }
    tp = block_sum<NT>(tp, sh);
    tn = block_sum<NT>(tn, sh);
    if (threadIdx.x == 0) {
        jd.st->t_pos = tp;
        jd.st->t_neg = tn;
        jd.st->wsum = sum;
    }
}

}  // namespace vjb
