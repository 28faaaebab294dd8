// Internal definitions shared by the HIP translation units of libvjboost.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

#include "../../include/vjboost.h"

namespace vjb {

// ---------------------------------------------------------------- limits
constexpr int kMaxWindow = 32;          // window side; feature values stay within 18 bits
constexpr int64_t kMaxN = 32767;        // 15-bit window indices in the sorted keys
constexpr int64_t kNarrowMaxN = 16383;  // 14-bit indices (+ dummy index n) in the narrow key format
constexpr int kRing = 4096;             // device stump ring entries
constexpr int kWave = 64;
constexpr int kUpdWg = 256;             // windows per update workgroup

// ---------------------------------------------------------------- feature descriptor
// Packed uint32: type [0,3) | x [3,8) | y [8,13) | (cw-1) [13,18) | (ch-1) [18,23).
__host__ __device__ inline uint32_t pack_feature(int t, int x, int y, int cw, int ch) {
    return (uint32_t)t | ((uint32_t)x << 3) | ((uint32_t)y << 8) | ((uint32_t)(cw - 1) << 13) |
           ((uint32_t)(ch - 1) << 18);
}
__host__ __device__ inline void unpack_feature(uint32_t d, int& t, int& x, int& y, int& cw, int& ch) {
    t = d & 7; x = (d >> 3) & 31; y = (d >> 8) & 31; cw = ((d >> 13) & 31) + 1; ch = ((d >> 18) & 31) + 1;
}

// Haar feature value from the sample-minor integral images.
// g(r, c) = ii[(r * (W+1) + c) * S + i]; S = row stride in samples.
// Each formula is the signed sum of the cells' four-corner rectangle sums,
// collected per corner (Section 2.1 rectangle rule, Section 2.2 shading).
__device__ __forceinline__ int32_t haar_value(const int32_t* __restrict__ ii, int64_t S, int wp1,
                                              uint32_t desc, int64_t i) {
    int t, x, y, cw, ch;
    unpack_feature(desc, t, x, y, cw, ch);
    auto g = [&](int r, int c) -> int32_t { return ii[(int64_t)(r * wp1 + c) * S + i]; };
    switch (t) {
    case BOOST_TYPE_3H: {  // middle - left - right
        auto A = [&](int c) { return g(y + ch, c) - g(y, c); };
        return 2 * A(x + 2 * cw) - 2 * A(x + cw) + A(x) - A(x + 3 * cw);
    }
    case BOOST_TYPE_3V: {  // middle - top - bottom
        auto B = [&](int r) { return g(r, x + cw) - g(r, x); };
        return 2 * B(y + 2 * ch) - 2 * B(y + ch) + B(y) - B(y + 3 * ch);
    }
    case BOOST_TYPE_2H: {  // right - left
        auto A = [&](int c) { return g(y + ch, c) - g(y, c); };
        return A(x + 2 * cw) - 2 * A(x + cw) + A(x);
    }
    case BOOST_TYPE_2V: {  // bottom - top
        auto B = [&](int r) { return g(r, x + cw) - g(r, x); };
        return B(y + 2 * ch) - 2 * B(y + ch) + B(y);
    }
    default: {  // top-right + bottom-left - top-left - bottom-right
        const int x1 = x + cw, x2 = x + 2 * cw, y1 = y + ch, y2 = y + 2 * ch;
        return -g(y, x) + 2 * g(y, x1) - g(y, x2) + 2 * g(y1, x) - 4 * g(y1, x1) + 2 * g(y1, x2) -
               g(y2, x) + 2 * g(y2, x1) - g(y2, x2);
    }
    }
}

// The same value with the type known at compile time: a caller that
// evaluates many windows of one feature dispatches on the type once, so the
// loads of all its windows can be in flight together.
template <int TYPE>
__device__ __forceinline__ int32_t haar_value_t(const int32_t* __restrict__ ii, int64_t S, int wp1, int x, int y,
                                                int cw, int ch, int64_t i) {
    auto g = [&](int r, int c) -> int32_t { return ii[(int64_t)(r * wp1 + c) * S + i]; };
    if constexpr (TYPE == BOOST_TYPE_3H) {
        auto A = [&](int c) { return g(y + ch, c) - g(y, c); };
        return 2 * A(x + 2 * cw) - 2 * A(x + cw) + A(x) - A(x + 3 * cw);
    } else if constexpr (TYPE == BOOST_TYPE_3V) {
        auto B = [&](int r) { return g(r, x + cw) - g(r, x); };
        return 2 * B(y + 2 * ch) - 2 * B(y + ch) + B(y) - B(y + 3 * ch);
    } else if constexpr (TYPE == BOOST_TYPE_2H) {
        auto A = [&](int c) { return g(y + ch, c) - g(y, c); };
        return A(x + 2 * cw) - 2 * A(x + cw) + A(x);
    } else if constexpr (TYPE == BOOST_TYPE_2V) {
        auto B = [&](int r) { return g(r, x + cw) - g(r, x); };
        return B(y + 2 * ch) - 2 * B(y + ch) + B(y);
    } else {
        const int x1 = x + cw, x2 = x + 2 * cw, y1 = y + ch, y2 = y + 2 * ch;
        return -g(y, x) + 2 * g(y, x1) - g(y, x2) + 2 * g(y1, x) - 4 * g(y1, x1) + 2 * g(y1, x2) -
               g(y2, x) + 2 * g(y2, x1) - g(y2, x2);
    }
}

// ---------------------------------------------------------------- sorted-key layout
// Per feature, the n windows in ascending value order are split into 8-key
// units (16 bytes).  The Nc = ceil(n/8) units are dealt to the `lanes` lanes
// (16, 32 or 64) that scan the feature as contiguous segments: lane L owns
// q+1 units if L < rem, else q (q = Nc / lanes, rem = Nc % lanes), starting
// at unit start(L) = L*q + min(L, rem).  In memory, the r-th unit of every
// lane's segment sits together: memory unit r*lanes + L.  The lanes of a
// feature then read lanes*16 contiguous bytes per step while each walks its
// own contiguous run of ranks.
struct KeyGeom {
    int64_t n;        // windows
    int64_t nc;       // units of 8 keys
    int32_t q, rem;   // units per lane (q or q+1)
    int64_t row_units;// units between consecutive features (row stride / 16 B)
    int32_t narrow;   // 1: 14-bit indices (n <= 16383), 0: 15-bit
    int32_t lanes;    // lanes per feature
};

__host__ __device__ inline int64_t lane_start(const KeyGeom& g, int L) {
    return (int64_t)L * g.q + (L < g.rem ? L : g.rem);
}
// rank-order unit u -> memory unit
__host__ __device__ inline int64_t unit_to_mem(const KeyGeom& g, int64_t u) {
    const int64_t big = (int64_t)g.rem * (g.q + 1);
    int64_t L, r;
    if (u < big) { L = u / (g.q + 1); r = u % (g.q + 1); }
    else { const int64_t v = u - big; L = g.rem + v / g.q; r = v % g.q; }
    return r * g.lanes + L;
}
// memory unit -> rank-order unit
__host__ __device__ inline int64_t mem_to_unit(const KeyGeom& g, int64_t mu) {
    const int64_t r = mu / g.lanes;
    const int L = (int)(mu % g.lanes);
    return lane_start(g, L) + r;
}

// Key encodings of one dword holding ranks 2a (low half) and 2a+1 (high half):
//  narrow: low = (i0 << 2) | c0 | (c1 << 1), high = (i1 << 2)
//          -> LDS byte offset of a float table is (dword & 0xFFFC) and (dword >> 16)
//  wide:   low = (i0 << 1) | c0, high = (i1 << 1) | c1
// with c = 1 - f, where f = 1 marks the last rank of a run of equal values (a
// realisable split after it): the stored bit says "no split here", which the
// scan turns into its candidate mask with one bit-field extract.
// encode_pair / decode_pair take and return f.
__host__ __device__ inline uint32_t encode_pair(int narrow, uint32_t i0, uint32_t f0, uint32_t i1, uint32_t f1) {
    const uint32_t c0 = f0 ^ 1u, c1 = f1 ^ 1u;
    if (narrow) return (i0 << 2) | c0 | (c1 << 1) | (i1 << 18);
    return (i0 << 1) | c0 | (((i1 << 1) | c1) << 16);
}
__host__ __device__ inline void decode_pair(int narrow, uint32_t d, uint32_t& i0, uint32_t& f0, uint32_t& i1,
                                            uint32_t& f1) {
    if (narrow) { i0 = (d & 0xFFFF) >> 2; f0 = (d & 1) ^ 1u; f1 = ((d >> 1) & 1) ^ 1u; i1 = d >> 18; }
    else { i0 = (d & 0xFFFF) >> 1; f0 = (d & 1) ^ 1u; i1 = d >> 17; f1 = ((d >> 16) & 1) ^ 1u; }
}

// A dword of two padding keys (window index n: the zero table entry, no run end).
__host__ __device__ inline uint32_t pad_dword(const KeyGeom& g) {
    return encode_pair(g.narrow, (uint32_t)g.n, 0u, (uint32_t)g.n, 0u);
}

// ---------------------------------------------------------------- device state of one job
// Lives in the workspace; written by the kernels, read by the host only on request.
struct JobState {
    double t_pos, t_neg;     // class totals of the last scan's weight table
    double sum_w;            // S: the stored weights divided by S are the normalised weights of the round
    int32_t round;           // rounds completed
    int32_t stopped;         // STOP policy triggered
    int32_t n_pos;           // l
    int32_t label_error;     // a label other than 0/1 was seen
    int32_t weight_error;    // boost_set_weights saw a non-finite / negative / zero-sum input
    int32_t launches;        // scan launches (ring slot of the next record)
    int32_t wpar;            // which half of the weight buffer holds the current weights
    int32_t cur;             // wpar as seen by the last scan (read by the update kernel)
};

// Per-workgroup best stump candidate written by the scan kernel.
struct WgBest {
    double eps;
    int64_t feature;   // -1: none
    int32_t polarity;
    int32_t lane;      // lane holding the extreme running sum (-1: the empty split k = 0)
};

// Everything a kernel needs to know about one job.
struct JobDev {
    const uint4* keys;         // F rows of row_units 16-byte units
    const int32_t* ii;         // [(H+1)(W+1)][ii_stride]
    const uint32_t* ftab;      // [F] packed descriptors
    double* w;                 // [2][n] FP64 weights (internal order), double buffered: half st->wpar is
                               // current; normalised weights = w / sum(wpart)
    double* wpart;             // [n_part] partial sums of w, summed in index order
    WgBest* wgb;               // [scan grid] per-workgroup candidates
    const uint4* pad;          // one unit of padding keys (window index n, no run end)
    JobState* st;
    boost_stump* ring;         // [kRing]
    const int32_t* perm;       // internal -> caller
    const int32_t* inv;        // caller -> internal
    KeyGeom g;
    int64_t F;
    int64_t ii_stride;
    int32_t W, H;
    int32_t precision, on_perfect;
    int32_t n_part;            // update workgroups (256 windows each)
    int32_t unused;
    double eps_floor;
};

__device__ __forceinline__ double* weights(const JobDev& jd, int par) { return jd.w + (int64_t)par * jd.g.n; }

// ---------------------------------------------------------------- host helpers
void set_error(const std::string& msg);
const char* get_error();

#define VJB_HIP(call)                                                          \
    do {                                                                       \
        hipError_t _e = (call);                                                \
        if (_e != hipSuccess) {                                                \
            ::vjb::set_error(std::string(#call) + ": " + hipGetErrorString(_e)); \
            return BOOST_E_DEVICE;                                             \
        }                                                                      \
    } while (0)

// host-side enumeration (closed form and descriptors)
int64_t host_feature_count(const boost_feature_set* fs);
bool valid_feature_set(const boost_feature_set* fs);
bool valid_options(const boost_options* o);
int host_feature_desc(const boost_feature_set* fs, int64_t j, boost_feature* out);
void host_feature_table(const boost_feature_set* fs, uint32_t* out);
// A permutation of 0 .. F - 1: the order the one-time preparation visits
// the features of ftab (integral-image locality; see features.cpp).
void host_sort_order(const uint32_t* ftab, int64_t F, uint32_t* order);

KeyGeom make_geom(int64_t n, int lanes);
int64_t ii_stride_of(int64_t n);

}  // namespace vjb
