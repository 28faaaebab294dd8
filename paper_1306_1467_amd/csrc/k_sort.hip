// One-time preparation of every feature: evaluate the Haar feature on all
// windows (Section 2.2), order the windows by value, and write the per-feature
// keys (window index + end-of-run flag) in the lane-segment layout that the
// per-round scan reads.  Feature values never reach HBM.
//
// One workgroup per feature at a time.  Each thread holds C values in
// registers (window r = k * NT + t in slot k), packed with the window index as
// ((v - vmin) << ib) | r in 32 bits, and the workgroup sorts them with a
// stable least-significant-digit radix sort over the value bits only, 4 bits
// per pass: windows with equal values keep index order, which is the (value,
// index) order.  A pass ranks each item among the items of its wave and slot
// with the same digit (ballots), counts items per (digit, slot, wave) in LDS,
// scans the counts in that order, and scatters through one LDS buffer.
// A feature whose value range does not fit beside the index in 32 bits
// (possible only for n > 16384) is sorted as 64-bit pairs in a per-workgroup
// global scratch buffer (bitonic network) instead.
#include <limits.h>

#include "launch.h"

namespace vjb {

int64_t sort_pow2(int64_t n) {
    int64_t p = 1;
    while (p < n) p <<= 1;
    return p;
}

size_t sort_scratch_bytes(int64_t n) {
    if (n <= kNarrowMaxN) return 0;
    return (size_t)kMaxSortGrid * (size_t)sort_pow2(n) * sizeof(uint64_t);
}

template <int NT, typename T>
__device__ void bitonic_sort(T* s, int64_t npow2) {
    for (int64_t k = 2; k <= npow2; k <<= 1) {
        for (int64_t jj = k >> 1; jj > 0; jj >>= 1) {
            for (int64_t t = threadIdx.x; t < (npow2 >> 1); t += NT) {
                const int64_t i = ((t & ~(jj - 1)) << 1) | (t & (jj - 1));
                const int64_t p = i + jj;
                const T a = s[i], b = s[p];
                const bool up = (i & k) == 0;
                if ((a > b) == up) { s[i] = b; s[p] = a; }
            }
            __syncthreads();
        }
    }
}

// Keys of one feature from its sorted (value, index) words.
template <int NT, typename T>
__device__ void emit_keys(const JobDev& jd, int64_t j, const T* s, int shift, uint64_t imask) {
    const KeyGeom& g = jd.g;
    const int n = (int)g.n;
    const int nc = (int)g.nc;
    const int lsh = __builtin_ctz((unsigned)g.lanes);   // lanes per feature: a power of two
    uint4* row = (uint4*)(jd.keys + j * g.row_units);
    for (int mu = threadIdx.x; mu < nc; mu += NT) {
        // memory unit -> rank-order unit (the key layout's lane segments)
        const int L = mu & (g.lanes - 1);
        const int u = L * g.q + (L < g.rem ? L : g.rem) + (mu >> lsh);
        uint32_t dw[4];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            uint32_t ix[2], fl[2];
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int r = 8 * u + 2 * h + b;
                if (r < n) {
                    const T cur = s[r];
                    ix[b] = (uint32_t)((uint64_t)cur & imask);
                    fl[b] = (r == n - 1) || ((uint64_t)(cur >> shift) != (uint64_t)(s[r + 1] >> shift));
                } else {
                    ix[b] = (uint32_t)n;   // padding key: zero-weight table slot, no split
                    fl[b] = 0;
                }
            }
            dw[h] = encode_pair(g.narrow, ix[0], fl[0], ix[1], fl[1]);
        }
        row[mu] = make_uint4(dw[0], dw[1], dw[2], dw[3]);
    }
}

constexpr int kRadixBits = 4;
constexpr int kDigits = 1 << kRadixBits;

// Exclusive prefix sum, in place, of m 16-bit counters (m <= NT * E); thread t
// owns entries [t * E, t * E + E).  Totals stay below 2^16 (at most n items).
template <int NT, int E>
__device__ __forceinline__ void scan_counts(uint16_t* cnt, int m, uint32_t* wtot) {
    constexpr int NW = NT / 64;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    uint32_t c[E];
    uint32_t sum = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int idx = t * E + e;
        c[e] = idx < m ? cnt[idx] : 0u;
        sum += c[e];
    }
    // inclusive scan of the per-thread sums within the wave
    uint32_t incl = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wtot[wv] = incl;
    __syncthreads();
    uint32_t base = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) base += w < wv ? wtot[w] : 0u;
    uint32_t run = base + incl - sum;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int idx = t * E + e;
        if (idx < m) cnt[idx] = (uint16_t)run;
        run += c[e];
    }
}

template <int NT, int C>
__global__ __launch_bounds__(NT) void k_sort(JobDev jd, int64_t npow2, int ib, uint64_t* __restrict__ scratch) {
    constexpr int NW = NT / 64;
    constexpr int NCNT = kDigits * C * NW;                 // counters in (digit, slot, wave) order
    constexpr int E = (NCNT + NT - 1) / NT;                 // counters per thread in the scan
    extern __shared__ __align__(16) uint32_t buf[];         // NT * C sorted words, then the counters
    __shared__ int32_t rmin[NW], rmax[NW];
    __shared__ uint32_t wtot[NW];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t n = jd.g.n;
    const int wp1 = jd.W + 1;
    const uint32_t imask = (1u << ib) - 1u;
    uint16_t* cnt = (uint16_t*)(buf + NT * C);
    for (int64_t j = blockIdx.x; j < jd.F; j += gridDim.x) {
        const uint32_t desc = jd.ftab[j];
        // values go through the LDS buffer (bounded register use), then the
        // packed words into registers
        int32_t vmin = INT_MAX, vmax = INT_MIN;
        for (int64_t i = tid; i < n; i += NT) {
            const int32_t v = haar_value(jd.ii, jd.ii_stride, wp1, desc, i);
            buf[i] = (uint32_t)v;
            vmin = v < vmin ? v : vmin;
            vmax = v > vmax ? v : vmax;
        }
#pragma unroll
        for (int o = 32; o; o >>= 1) {
            const int32_t a = __shfl_xor(vmin, o), b = __shfl_xor(vmax, o);
            vmin = a < vmin ? a : vmin;
            vmax = b > vmax ? b : vmax;
        }
        if (lane == 0) { rmin[wv] = vmin; rmax[wv] = vmax; }
        __syncthreads();
        vmin = rmin[0]; vmax = rmax[0];
        for (int k = 1; k < NW; ++k) {
            vmin = rmin[k] < vmin ? rmin[k] : vmin;
            vmax = rmax[k] > vmax ? rmax[k] : vmax;
        }
        const uint32_t range = (uint32_t)(vmax - vmin);
        const int rb = range == 0 ? 0 : 32 - __clz(range);
        if (rb + ib <= 32) {
            // packed words; slots past n hold all-ones sentinels, which carry
            // digit 15 in every pass and start after every window, so they
            // stay behind the windows (the passes need no bounds checks)
            for (int i = tid; i < NT * C; i += NT)
                buf[i] = i < n ? (((uint32_t)((int32_t)buf[i] - vmin)) << ib) | (uint32_t)i : 0xFFFFFFFFu;
            __syncthreads();
            uint32_t it[C];
#pragma unroll
            for (int k = 0; k < C; ++k) it[k] = buf[k * NT + tid];
            for (int sh = ib; sh < ib + rb; sh += kRadixBits) {
                for (int e = tid; e < NCNT; e += NT) cnt[e] = 0;
                __syncthreads();
                uint32_t rkp[(C + 3) / 4];   // rank in wave (< 64) of slot k in byte k % 4 of rkp[k / 4]
#pragma unroll
                for (int q = 0; q < (C + 3) / 4; ++q) rkp[q] = 0u;
#pragma unroll
                for (int k = 0; k < C; ++k) {
                    const uint32_t d = (it[k] >> sh) & (kDigits - 1);
                    uint64_t m = ~0ull;
#pragma unroll
                    for (int b = 0; b < kRadixBits; ++b) {
                        const bool bit = (d >> b) & 1u;
                        const uint64_t bb = __ballot(bit);
                        m &= bit ? bb : ~bb;
                    }
                    const uint32_t rk = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                    rkp[k / 4] |= rk << (8 * (k % 4));
                    if (rk == 0) cnt[((int)d * C + k) * NW + wv] = (uint16_t)__popcll(m);
                    // one slot's ballots at a time: interleaving slots would
                    // keep many wave masks live in scalar registers
                    __builtin_amdgcn_sched_barrier(0);
                }
                __syncthreads();
                scan_counts<NT, E>(cnt, NCNT, wtot);
                __syncthreads();
#pragma unroll
                for (int k = 0; k < C; ++k) {
                    const uint32_t d = (it[k] >> sh) & (kDigits - 1);
                    const uint32_t rk = (rkp[k / 4] >> (8 * (k % 4))) & 0xFFu;
                    buf[cnt[((int)d * C + k) * NW + wv] + rk] = it[k];
                }
                __syncthreads();
#pragma unroll
                for (int k = 0; k < C; ++k) it[k] = buf[k * NT + tid];
            }
            __syncthreads();
            emit_keys<NT, uint32_t>(jd, j, buf, ib, imask);
        } else {
            uint64_t* g = scratch + (int64_t)blockIdx.x * npow2;
            for (int64_t i = tid; i < npow2; i += NT)
                g[i] = i < n ? (((uint64_t)(uint32_t)((int32_t)buf[i] - vmin)) << 32) | (uint64_t)i : ~0ull;
            __syncthreads();
            bitonic_sort<NT, uint64_t>(g, npow2);
            emit_keys<NT, uint64_t>(jd, j, g, 32, 0xFFFFFFFFull);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- counting-sort passes
// The kernel used for n <= NT * C with C <= 15 (every n up to 15,360).  Thread
// t owns the C consecutive positions [t C, t C + C) of the current order, so a
// stable pass is a counting sort in (digit, thread, position-in-thread) order:
//   1. each thread counts its items' digits in a 64-bit register of 16 packed
//      4-bit counters (C <= 15, so no field overflows);
//   2. the counts, spread to 16-bit fields, are scanned across the wave's
//      lanes (DPP), the waves' totals across (digit, wave) in digit-major
//      order by one wave, so digit d of thread t starts at
//      base(d, wave) + (the counts of d in the wave's lower lanes);
//   3. each thread writes its 16 start offsets to a private LDS row (indexed
//      by its digits) and scatters its items, in order, to start + (the
//      number of its earlier items with the same digit), that rank taken from
//      a second packed running count.
// Unlike ranking each item among its wave with ballots (several VALU
// operations per key bit), this costs a few operations per item and pass.

// Inclusive / exclusive scan across the 64 lanes of a wave of four 16-bit
// counters packed in a 64-bit word (no carries cross fields: every sum stays
// below 2^16).
template <int CTRL, int RM, int BM, bool BC>
__device__ __forceinline__ uint64_t dpp64(uint64_t v) {
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, CTRL, RM, BM, BC);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), CTRL, RM, BM, BC);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}
__device__ __forceinline__ uint64_t wave_scan_incl_u64(uint64_t v) {
    v += dpp64<0x111, 0xF, 0xF, true>(v);   // row_shr:1
    v += dpp64<0x112, 0xF, 0xF, true>(v);   // row_shr:2
    v += dpp64<0x114, 0xF, 0xF, true>(v);   // row_shr:4
    v += dpp64<0x118, 0xF, 0xF, true>(v);   // row_shr:8
    v += dpp64<0x142, 0xA, 0xF, false>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp64<0x143, 0xC, 0xF, false>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

// Four 4-bit counters (bits 0..15 of x) spread to 16-bit fields.
__device__ __forceinline__ uint64_t spread4(uint32_t x) {
    return (uint64_t)(x & 0xFu) | ((uint64_t)((x >> 4) & 0xFu) << 16) | ((uint64_t)((x >> 8) & 0xFu) << 32) |
           ((uint64_t)((x >> 12) & 0xFu) << 48);
}

template <int NT, int C>
struct SortCntLds {
    uint32_t buf[NT * C];          // the current order (packed words)
    uint16_t tab[16 * NT];         // tab[d * NT + t]: thread t's start offset of digit d
    uint64_t wtot[NT / 64][4];     // per wave: the digit totals, 16-bit fields
    uint16_t base[NT / 64][16];    // per wave: where each digit's run of this wave starts
    int32_t rmin[NT / 64], rmax[NT / 64];
};

template <int NT, int C>
__global__ __launch_bounds__(NT) void k_sort_cnt(JobDev jd, int ib) {
    static_assert(C <= 15 && (C & 1) == 1, "4-bit counters; odd C keeps the chunk reads conflict-free");
    constexpr int NW = NT / 64;
    static_assert(16 * NW <= 256, "one wave scans the (digit, wave) totals, four per lane");
    extern __shared__ __align__(16) unsigned char smem[];
    SortCntLds<NT, C>& L = *reinterpret_cast<SortCntLds<NT, C>*>(smem);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int n = (int)jd.g.n;
    const int wp1 = jd.W + 1;
    // consecutive features run at the same time on the same XCD (workgroups
    // are dealt to the 8 XCDs in turn), so the integral-image columns they
    // share are read from that XCD's L2
    const int G = gridDim.x;
    const int per_xcd = G / 8;
    const int slot = G % 8 == 0 ? (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3) : blockIdx.x;
    for (int64_t j = slot; j < jd.F; j += G) {
        const uint32_t desc = jd.ftab[j];
        // 1. values, all loads of a thread in flight together
        int32_t v[C];
#pragma unroll
        for (int k = 0; k < C; ++k) {
            const int i = k * NT + tid;
            v[k] = i < n ? haar_value(jd.ii, jd.ii_stride, wp1, desc, i) : 0;
        }
        int32_t vmin = INT_MAX, vmax = INT_MIN;
#pragma unroll
        for (int k = 0; k < C; ++k) {
            const int i = k * NT + tid;
            if (i < n) {
                vmin = v[k] < vmin ? v[k] : vmin;
                vmax = v[k] > vmax ? v[k] : vmax;
            }
        }
#pragma unroll
        for (int o = 32; o; o >>= 1) {
            const int32_t a = __shfl_xor(vmin, o), b = __shfl_xor(vmax, o);
            vmin = a < vmin ? a : vmin;
            vmax = b > vmax ? b : vmax;
        }
        if (lane == 0) { L.rmin[wv] = vmin; L.rmax[wv] = vmax; }
        __syncthreads();
        vmin = L.rmin[0]; vmax = L.rmax[0];
#pragma unroll
        for (int w = 1; w < NW; ++w) {
            vmin = L.rmin[w] < vmin ? L.rmin[w] : vmin;
            vmax = L.rmax[w] > vmax ? L.rmax[w] : vmax;
        }
        const uint32_t range = (uint32_t)(vmax - vmin);
        const int rb = range == 0 ? 0 : 32 - __clz(range);   // <= 18 for windows up to 32x32, ib <= 14
        // packed words in index order; positions past n hold all-ones
        // sentinels (digit 15 in every pass, behind every window)
#pragma unroll
        for (int k = 0; k < C; ++k) {
            const int i = k * NT + tid;
            L.buf[i] = i < n ? (((uint32_t)(v[k] - vmin)) << ib) | (uint32_t)i : 0xFFFFFFFFu;
        }
        __syncthreads();
        uint32_t it[C];
#pragma unroll
        for (int k = 0; k < C; ++k) it[k] = L.buf[tid * C + k];
        for (int sh = ib; sh < ib + rb; sh += 4) {
            // 1. counts
            uint64_t cnt = 0;
#pragma unroll
            for (int k = 0; k < C; ++k) cnt += 1ull << (4 * ((it[k] >> sh) & 15u));
            // 2. scan across the wave, then across (digit, wave)
            uint64_t f[4], ex[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                f[q] = spread4((uint32_t)(cnt >> (16 * q)) & 0xFFFFu);
                const uint64_t inc = wave_scan_incl_u64(f[q]);
                ex[q] = inc - f[q];
                if (lane == 63) L.wtot[wv][q] = inc;
            }
            __syncthreads();   // also: every thread has read its chunk of the previous order
            if (wv == 0) {
                // (digit, wave) entries x = d * NW + w in digit-major order, four per lane
                uint32_t e[4], sum = 0;
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const int x = 4 * lane + a;
                    const int d = x / NW, w = x % NW;
                    e[a] = x < 16 * NW ? (uint32_t)((L.wtot[w][d >> 2] >> (16 * (d & 3))) & 0xFFFFu) : 0u;
                    sum += e[a];
                }
                uint32_t incl = sum;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const uint32_t y = __shfl_up(incl, o);
                    if (lane >= o) incl += y;
                }
                uint32_t run = incl - sum;
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const int x = 4 * lane + a;
                    if (x < 16 * NW) L.base[x % NW][x / NW] = (uint16_t)run;
                    run += e[a];
                }
            }
            __syncthreads();
            // 3. this thread's start offsets, then the scatter
#pragma unroll
            for (int d = 0; d < 16; ++d)
                L.tab[d * NT + tid] = (uint16_t)(L.base[wv][d] + (uint32_t)((ex[d >> 2] >> (16 * (d & 3))) & 0xFFFFu));
            uint64_t run = 0;
#pragma unroll
            for (int k = 0; k < C; ++k) {
                const uint32_t d = (it[k] >> sh) & 15u;
                const uint32_t r = (uint32_t)(run >> (4 * d)) & 15u;
                run += 1ull << (4 * d);
                L.buf[L.tab[d * NT + tid] + r] = it[k];
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < C; ++k) it[k] = L.buf[tid * C + k];
        }
        __syncthreads();
        emit_keys<NT, uint32_t>(jd, j, L.buf, ib, (1u << ib) - 1u);
        __syncthreads();
    }
}

template <int NT, int C>
static int sort_cnt_launch(const JobDev& jd, int num_cu, hipStream_t s) {
    const int64_t n = jd.g.n;
    int ib = n <= 1 ? 1 : 32 - __builtin_clz((unsigned)(n - 1));
    const size_t lds = sizeof(SortCntLds<NT, C>);
    const void* k = (const void*)k_sort_cnt<NT, C>;
    VJB_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int per_cu = 0;
    VJB_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, NT, lds));
    if (per_cu < 1) {
        set_error("sort kernel does not fit on a compute unit");
        return BOOST_E_INVALID;
    }
    int64_t grid = (int64_t)per_cu * num_cu;
    if (grid > jd.F) grid = jd.F;
    if (grid > kMaxSortGrid) grid = kMaxSortGrid;
    JobDev a = jd;
    void* args[] = {(void*)&a, (void*)&ib};
    VJB_HIP(hipLaunchKernel(k, dim3((unsigned)grid), dim3(NT), args, lds, s));
    return BOOST_OK;
}

template <int NT, int C>
static int sort_launch_c(const JobDev& jd, uint64_t* scratch, int num_cu, hipStream_t s) {
    const int64_t n = jd.g.n;
    int64_t npow2 = sort_pow2(n);
    int ib = n <= 1 ? 1 : 32 - __builtin_clz((unsigned)(n - 1));
    const size_t lds = (size_t)NT * C * sizeof(uint32_t) + (size_t)kDigits * C * (NT / 64) * sizeof(uint16_t);
    const void* k = (const void*)k_sort<NT, C>;
    VJB_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int per_cu = 0;
    VJB_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, NT, lds));
    if (per_cu < 1) {
        set_error("sort kernel does not fit on a compute unit");
        return BOOST_E_INVALID;
    }
    int64_t grid = (int64_t)per_cu * num_cu;
    if (grid > jd.F) grid = jd.F;
    if (grid > kMaxSortGrid) grid = kMaxSortGrid;
    if (n > kNarrowMaxN && scratch == nullptr) {
        set_error("sort fallback scratch missing");
        return BOOST_E_INVALID;
    }
    JobDev a = jd;
    void* args[] = {(void*)&a, (void*)&npow2, (void*)&ib, (void*)&scratch};
    VJB_HIP(hipLaunchKernel(k, dim3((unsigned)grid), dim3(NT), args, lds, s));
    return BOOST_OK;
}

// Counting-sort passes up to 15,360 windows (C values per thread, the
// smallest odd C of the shape that covers n); ballot-ranked passes beyond.
int sort_launch(const JobDev& jd, uint64_t* scratch, int num_cu, hipStream_t s) {
    const int64_t n = jd.g.n;
    if (n <= 256 * 7) return sort_cnt_launch<256, 7>(jd, num_cu, s);
    if (n <= 512 * 7) return sort_cnt_launch<512, 7>(jd, num_cu, s);
    if (n <= 1024 * 7) return sort_cnt_launch<1024, 7>(jd, num_cu, s);
    if (n <= 1024 * 11) return sort_cnt_launch<1024, 11>(jd, num_cu, s);
    if (n <= 1024 * 15) return sort_cnt_launch<1024, 15>(jd, num_cu, s);
    if (n <= 256) return sort_launch_c<256, 1>(jd, scratch, num_cu, s);
    if (n <= 512) return sort_launch_c<256, 2>(jd, scratch, num_cu, s);
    if (n <= 1024) return sort_launch_c<256, 4>(jd, scratch, num_cu, s);
    if (n <= 2048) return sort_launch_c<256, 8>(jd, scratch, num_cu, s);
    if (n <= 4096) return sort_launch_c<1024, 4>(jd, scratch, num_cu, s);
    if (n <= 8192) return sort_launch_c<1024, 8>(jd, scratch, num_cu, s);
    if (n <= 16384) return sort_launch_c<1024, 16>(jd, scratch, num_cu, s);
    if (n <= 32768) return sort_launch_c<512, 64>(jd, scratch, num_cu, s);
    set_error("too many windows for the sort");
    return BOOST_E_INVALID;
}

}  // namespace vjb
