// One-time preparation of every feature: evaluate the Haar feature on all
// windows (Section 2.2), order the windows by value, and write the per-feature
// keys (window index + end-of-run flag) in the lane-segment layout that the
// per-round scan reads.  Feature values never reach HBM.
//
// k_sort_cnt (every job of up to 31,744 windows): one workgroup per feature
// at a time, in a visiting order that keeps features reading the same
// integral-image corner planes together on one XCD.  Each thread evaluates C
// windows (slot k of thread t is window k * NT + t), the values are packed
// with the window index as ((v - vmin) << ib) | i in 32 bits, and the
// workgroup sorts them with stable least-significant-digit counting passes
// over the value bits only, 4 bits per pass (per-thread packed digit
// counters, DPP wave scans, one scatter through an LDS buffer per pass):
// windows with equal values keep index order, which is the (value, index)
// order.  A feature whose value range does not fit beside a 15-bit index is
// listed for the 64-bit path.
// k_sort (jobs of more than 31,744 windows, and the listed features): ranks
// each item among the items of its wave and slot with the same digit
// (ballots), or, when the words need 64 bits, a bitonic sort in a
// per-workgroup global scratch buffer.
// k_merge (boost_extend): the keys of a job extended by a few windows, from
// the old job's order and the new windows' (see below).
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

// The keys of units mu = threadIdx.x + k NT (k < U) of a feature's row, from
// its sorted 32-bit words in LDS (s 16-byte aligned, at least 8 ceil(n / 8)
// words; a unit's 8 words are read as two 16-byte loads), kept in registers
// so that the caller chooses when the stores issue.  Entries for units past
// the row are left unset.
template <int NT, int U>
__device__ __forceinline__ void unit_keys_w32(const KeyGeom& g, const uint32_t* s, int shift, uint32_t imask,
                                              uint4* out, int mu0 = 0) {
    const int n = (int)g.n;
    const int nc = (int)g.nc;
    const int lsh = __builtin_ctz((unsigned)g.lanes);
#pragma unroll
    for (int k = 0; k < U; ++k) {
        const int mu = mu0 + threadIdx.x + k * NT;
        if (mu >= nc) break;
        const int L = mu & (g.lanes - 1);
        const int u = L * g.q + (L < g.rem ? L : g.rem) + (mu >> lsh);
        const uint4 a = *reinterpret_cast<const uint4*>(s + 8 * u);
        const uint4 b = *reinterpret_cast<const uint4*>(s + 8 * u + 4);
        const int rn = 8 * u + 8;
        const uint32_t w[9] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, s[rn < n ? rn : n - 1]};
        uint32_t dw[4];
        if (rn < n) {   // a unit followed by more windows: no bound checks
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                uint32_t ix[2], fl[2];
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const int q = 2 * h + e;
                    ix[e] = w[q] & imask;
                    fl[e] = (w[q] >> shift) != (w[q + 1] >> shift);
                }
                dw[h] = encode_pair(g.narrow, ix[0], fl[0], ix[1], fl[1]);
            }
        } else {
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                uint32_t ix[2], fl[2];
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const int q = 2 * h + e, r = 8 * u + q;
                    if (r < n) {
                        ix[e] = w[q] & imask;
                        fl[e] = (r == n - 1) || ((w[q] >> shift) != (w[q + 1] >> shift));
                    } else {
                        ix[e] = (uint32_t)n;   // padding key: zero-weight table slot, no split
                        fl[e] = 0;
                    }
                }
                dw[h] = encode_pair(g.narrow, ix[0], fl[0], ix[1], fl[1]);
            }
        }
        out[k] = make_uint4(dw[0], dw[1], dw[2], dw[3]);
    }
}

template <int NT, int U>
__device__ __forceinline__ void store_unit_keys(const JobDev& jd, int64_t j, const uint4* out, int mu0 = 0) {
    uint4* row = (uint4*)(jd.keys + j * jd.g.row_units);
#pragma unroll
    for (int k = 0; k < U; ++k) {
        const int mu = mu0 + threadIdx.x + k * NT;
        if (mu >= (int)jd.g.nc) break;
        row[mu] = out[k];
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
__global__ __launch_bounds__(NT) void k_sort(JobDev jd, int64_t npow2, int ib, uint64_t* __restrict__ scratch,
                                             const uint32_t* __restrict__ list) {
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
    // every feature, or (list != NULL) the list[0] features list[16 + t]
    const int64_t count = list != nullptr ? (int64_t)list[0] : jd.F;
    for (int64_t t = blockIdx.x; t < count; t += gridDim.x) {
        const int64_t j = list != nullptr ? (int64_t)list[16 + t] : t;
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

// Inclusive scan of a 32-bit value across the 64 lanes of a wave (DPP row
// shifts and broadcasts; lanes a shift or broadcast does not reach add 0).
// Also scans two 16-bit counters packed in a word, as long as no field's
// sum reaches 2^16.
template <int CTRL, int RM, bool BC>
__device__ __forceinline__ uint32_t dpp_add(uint32_t v) {
    return v + (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, RM, 0xF, BC);
}
__device__ __forceinline__ uint32_t wave_scan_incl(uint32_t v) {
    v = dpp_add<0x111, 0xF, true>(v);    // row_shr:1
    v = dpp_add<0x112, 0xF, true>(v);    // row_shr:2
    v = dpp_add<0x114, 0xF, true>(v);    // row_shr:4
    v = dpp_add<0x118, 0xF, true>(v);    // row_shr:8
    v = dpp_add<0x142, 0xA, false>(v);   // row_bcast:15 into rows 1 and 3
    v = dpp_add<0x143, 0xC, false>(v);   // row_bcast:31 into rows 2 and 3
    return v;
}
// Eight independent inclusive scans, step by step, so that each DPP read
// has seven other adds between it and the write it depends on.
__device__ __forceinline__ void wave_scan_incl8(const uint32_t* f, uint32_t* v) {
#pragma unroll
    for (int p = 0; p < 8; ++p) v[p] = dpp_add<0x111, 0xF, true>(f[p]);
#pragma unroll
    for (int p = 0; p < 8; ++p) v[p] = dpp_add<0x112, 0xF, true>(v[p]);
#pragma unroll
    for (int p = 0; p < 8; ++p) v[p] = dpp_add<0x114, 0xF, true>(v[p]);
#pragma unroll
    for (int p = 0; p < 8; ++p) v[p] = dpp_add<0x118, 0xF, true>(v[p]);
#pragma unroll
    for (int p = 0; p < 8; ++p) v[p] = dpp_add<0x142, 0xA, false>(v[p]);
#pragma unroll
    for (int p = 0; p < 8; ++p) v[p] = dpp_add<0x143, 0xC, false>(v[p]);
}

// Maximum and minimum of a 32-bit signed value over the 64 lanes of a wave
// (DPP row shifts and broadcasts; a lane a shift or broadcast does not reach
// keeps its own value), returned uniform from the last lane.
template <int CTRL, int RM, bool MAX>
__device__ __forceinline__ int32_t dpp_ext(int32_t v) {
    const int32_t o = __builtin_amdgcn_update_dpp(v, v, CTRL, RM, 0xF, false);
    return MAX ? (o > v ? o : v) : (o < v ? o : v);
}
template <bool MAX>
__device__ __forceinline__ int32_t wave_ext(int32_t v) {
    v = dpp_ext<0x111, 0xF, MAX>(v);   // row_shr:1
    v = dpp_ext<0x112, 0xF, MAX>(v);   // row_shr:2
    v = dpp_ext<0x114, 0xF, MAX>(v);   // row_shr:4
    v = dpp_ext<0x118, 0xF, MAX>(v);   // row_shr:8
    v = dpp_ext<0x142, 0xA, MAX>(v);   // row_bcast:15 into rows 1 and 3
    v = dpp_ext<0x143, 0xC, MAX>(v);   // row_bcast:31 into rows 2 and 3
    return __builtin_amdgcn_readlane(v, 63);
}

// Values of windows k NT + threadIdx.x, k < C (0 past n), the feature type
// fixed at compile time so the loads of all slots issue together.  The
// caller guarantees n >= K0 NT: the first K0 slots need no bound check.
template <int TYPE, int NT, int C, int K0>
__device__ __forceinline__ void eval_windows(const int32_t* __restrict__ ii, int64_t S, int wp1, int x, int y, int cw,
                                             int ch, int n, int32_t* v) {
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const int i = k * NT + threadIdx.x;
        v[k] = (k < K0 || i < n) ? haar_value_t<TYPE>(ii, S, wp1, x, y, cw, ch, i) : 0;
    }
}

// Scratch of the counting-sort passes besides the order buffer.
template <int NT>
struct CntScratch {
    uint16_t tab[16 * NT];         // tab[d * NT + t]: thread t's start offset of digit d
    alignas(16) uint32_t wtot[NT / 64][8];   // per wave: the digit totals, digits 2p, 2p + 1 in word p
    alignas(16) uint16_t base[NT / 64][16];   // per wave: where each digit's run of this wave starts
};

// Stable LSD counting-sort passes (4-bit digits) over bits [sh0, sh1) of
// the NT * C words it[] (thread t holds positions t C .. t C + C - 1 of the
// current order).  Each pass scatters into buf (NT * C words) and reloads;
// on return buf holds the sorted order (untouched when no pass runs; it[] is
// not reloaded after the last pass).  The caller must have finished reading
// buf (a barrier) before the call; when a pass runs, the call ends with buf
// complete (after a barrier).  A thread counts its items' digits in groups
// of at most 15 items (16 4-bit fields per group).
template <int NT, int C>
__device__ __forceinline__ void cnt_sort_passes(uint32_t* it, uint32_t* buf, CntScratch<NT>& cs, int sh0, int sh1) {
    static_assert(C <= 31 && (C & 1) == 1, "at most 31 items a thread; odd C keeps the chunk reads conflict-free");
    constexpr int NG = (C + 14) / 15;   // counter groups
    constexpr int NW = NT / 64;
    static_assert(16 * NW <= 256, "one wave scans the (digit, wave) totals, four per lane");
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int sh = sh0; sh < sh1; sh += 4) {
        // 1. counts: 16 4-bit fields per group of items
        uint64_t cnt[NG];
#pragma unroll
        for (int g = 0; g < NG; ++g) cnt[g] = 0;
#pragma unroll
        for (int k = 0; k < C; ++k) cnt[k / 15] += 1ull << (4 * ((it[k] >> sh) & 15u));
        // 2. scan across the wave (digits 2p, 2p + 1 in word p; the eight
        // scans are independent, so their steps interleave), then across
        // (digit, wave)
        uint32_t ex[8], inc[8];
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            uint32_t f = 0;
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                const uint32_t c2 = (uint32_t)(cnt[g] >> (8 * p));
                f += (c2 & 0xFu) | ((c2 & 0xF0u) << 12);
            }
            ex[p] = f;
        }
        wave_scan_incl8(ex, inc);
#pragma unroll
        for (int p = 0; p < 8; ++p) ex[p] = inc[p] - ex[p];
        if (lane == 63) {
            uint4* wt = reinterpret_cast<uint4*>(&cs.wtot[wv][0]);
            wt[0] = make_uint4(inc[0], inc[1], inc[2], inc[3]);
            wt[1] = make_uint4(inc[4], inc[5], inc[6], inc[7]);
        }
        __syncthreads();   // also: every thread has read its chunk of the previous order
        if (wv == 0) {
            // (digit, wave) entries x = d * NW + w in digit-major order, four per lane
            uint32_t e[4], sum = 0;
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const int x = 4 * lane + a;
                const int d = x / NW, w = x % NW;
                e[a] = x < 16 * NW ? (cs.wtot[w][d >> 1] >> (16 * (d & 1))) & 0xFFFFu : 0u;
                sum += e[a];
            }
            const uint32_t incl = wave_scan_incl(sum);
            uint32_t run = incl - sum;
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const int x = 4 * lane + a;
                if (x < 16 * NW) cs.base[x % NW][x / NW] = (uint16_t)run;
                run += e[a];
            }
        }
        __syncthreads();
        // 3. this thread's start offsets (the wave's bases read at once, as
        // digit pairs), then the scatter
        const uint4 b0 = *reinterpret_cast<const uint4*>(&cs.base[wv][0]);
        const uint4 b1 = *reinterpret_cast<const uint4*>(&cs.base[wv][8]);
        const uint32_t bp[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
        uint64_t run = 0;
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            const uint32_t s2 = bp[p] + ex[p];
            cs.tab[(2 * p) * NT + tid] = (uint16_t)s2;
            cs.tab[(2 * p + 1) * NT + tid] = (uint16_t)(s2 >> 16);
        }
#pragma unroll
        for (int k = 0; k < C; ++k) {
            if (k % 15 == 0) run = 0;   // the rank counts restart with each group ...
            const uint32_t d = (it[k] >> sh) & 15u;
            uint32_t r = (uint32_t)(run >> (4 * d)) & 15u;
#pragma unroll
            for (int g = 0; g < k / 15; ++g) r += (uint32_t)(cnt[g] >> (4 * d)) & 15u;   // ... after the earlier groups
            run += 1ull << (4 * d);
            buf[cs.tab[d * NT + tid] + r] = it[k];
        }
        __syncthreads();
        if (C > 15 || sh + 4 < sh1) {   // (kept for the 31-slot kernel: it spills less so)
#pragma unroll
            for (int k = 0; k < C; ++k) it[k] = buf[tid * C + k];
        }
    }
}

// Values of windows k NT + threadIdx.x (k < C, below n) of a feature of type
// TYPE stored to s[window] in LDS; their minimum and maximum over this
// thread's windows in vmin / vmax.  Partly unrolled: a full unroll of 31
// slots spills registers.
template <int TYPE, int NT, int C>
__device__ __forceinline__ void eval_windows_lds(const int32_t* __restrict__ ii, int64_t S, int wp1, int x, int y,
                                                 int cw, int ch, int n, uint32_t* s, int32_t& vmin,
                                                 int32_t& vmax) {
#pragma unroll 5
    for (int k = 0; k < C; ++k) {
        const int i = k * NT + threadIdx.x;
        if (i < n) {
            const int32_t v = haar_value_t<TYPE>(ii, S, wp1, x, y, cw, ch, i);
            s[i] = (uint32_t)v;
            vmin = v < vmin ? v : vmin;
            vmax = v > vmax ? v : vmax;
        }
    }
}

// Values of feature `desc` on windows k NT + threadIdx.x, k < C: the loads
// are issued here and waited for where the values are first used.
template <int NT, int C, int K0 = 0>
__device__ __forceinline__ void eval_values(const JobDev& jd, uint32_t desc, int n, int32_t* v) {
    const int wp1 = jd.W + 1;
    int t, x, y, cw, ch;
    unpack_feature(desc, t, x, y, cw, ch);
    switch (t) {
    case BOOST_TYPE_3H: eval_windows<BOOST_TYPE_3H, NT, C, K0>(jd.ii, jd.ii_stride, wp1, x, y, cw, ch, n, v); break;
    case BOOST_TYPE_3V: eval_windows<BOOST_TYPE_3V, NT, C, K0>(jd.ii, jd.ii_stride, wp1, x, y, cw, ch, n, v); break;
    case BOOST_TYPE_2H: eval_windows<BOOST_TYPE_2H, NT, C, K0>(jd.ii, jd.ii_stride, wp1, x, y, cw, ch, n, v); break;
    case BOOST_TYPE_2V: eval_windows<BOOST_TYPE_2V, NT, C, K0>(jd.ii, jd.ii_stride, wp1, x, y, cw, ch, n, v); break;
    default: eval_windows<BOOST_TYPE_4, NT, C, K0>(jd.ii, jd.ii_stride, wp1, x, y, cw, ch, n, v); break;
    }
}

// Values of feature `desc` on the first n windows into s[0 .. n) (LDS), and
// their range (every thread gets the same; one barrier).
template <int NT, int C>
__device__ __forceinline__ void eval_to_lds(const JobDev& jd, uint32_t desc, int n, uint32_t* s, int32_t* rmin,
                                            int32_t* rmax, int32_t& vmin, int32_t& vmax) {
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wp1 = jd.W + 1;
    int t, x, y, cw, ch;
    unpack_feature(desc, t, x, y, cw, ch);
    vmin = INT_MAX;
    vmax = INT_MIN;
    switch (t) {
    case BOOST_TYPE_3H: eval_windows_lds<BOOST_TYPE_3H, NT, C>(jd.ii, jd.ii_stride, wp1, x, y, cw, ch, n, s, vmin, vmax); break;
    case BOOST_TYPE_3V: eval_windows_lds<BOOST_TYPE_3V, NT, C>(jd.ii, jd.ii_stride, wp1, x, y, cw, ch, n, s, vmin, vmax); break;
    case BOOST_TYPE_2H: eval_windows_lds<BOOST_TYPE_2H, NT, C>(jd.ii, jd.ii_stride, wp1, x, y, cw, ch, n, s, vmin, vmax); break;
    case BOOST_TYPE_2V: eval_windows_lds<BOOST_TYPE_2V, NT, C>(jd.ii, jd.ii_stride, wp1, x, y, cw, ch, n, s, vmin, vmax); break;
    default: eval_windows_lds<BOOST_TYPE_4, NT, C>(jd.ii, jd.ii_stride, wp1, x, y, cw, ch, n, s, vmin, vmax); break;
    }
    vmin = wave_ext<false>(vmin);
    vmax = wave_ext<true>(vmax);
    if (lane == 0) { rmin[wv] = vmin; rmax[wv] = vmax; }
    __syncthreads();
    vmin = rmin[0];
    vmax = rmax[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) {
        vmin = rmin[w] < vmin ? rmin[w] : vmin;
        vmax = rmax[w] > vmax ? rmax[w] : vmax;
    }
}

// The range of the values over the first n windows (every thread gets the
// same; one barrier).  n >= K0 NT as for eval_windows.
template <int NT, int C, int K0 = 0>
__device__ __forceinline__ void value_range(const int32_t* v, int n, int32_t* rmin, int32_t* rmax, int32_t& vmin,
                                            int32_t& vmax) {
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    vmin = INT_MAX;
    vmax = INT_MIN;
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const int i = k * NT + tid;
        if (k < K0 || i < n) {
            vmin = v[k] < vmin ? v[k] : vmin;
            vmax = v[k] > vmax ? v[k] : vmax;
        }
    }
    vmin = wave_ext<false>(vmin);
    vmax = wave_ext<true>(vmax);
    if (lane == 0) { rmin[wv] = vmin; rmax[wv] = vmax; }
    __syncthreads();
    vmin = rmin[0];
    vmax = rmax[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) {
        vmin = rmin[w] < vmin ? rmin[w] : vmin;
        vmax = rmax[w] > vmax ? rmax[w] : vmax;
    }
}

// The positions of the visiting order (a permutation of the features that
// keeps features reading the same integral-image corner planes adjacent)
// that this workgroup runs: XCD x = blockIdx.x % 8 (workgroups are dealt to
// the 8 XCDs in turn) takes the contiguous share [x F / 8, (x + 1) F / 8),
// its G / 8 workgroups interleaved over it, so the features that run at the
// same time on one XCD are adjacent in the order and share that XCD's L2.
struct FeatureWalk { int64_t p, end, step; };
__device__ __forceinline__ FeatureWalk feature_walk(int64_t F) {
    const int64_t G = gridDim.x;
    if (G % 8 != 0) return FeatureWalk{(int64_t)blockIdx.x, F, G};
    const int64_t x = blockIdx.x & 7;
    return FeatureWalk{x * F / 8 + (int64_t)(blockIdx.x >> 3), (x + 1) * F / 8, G / 8};
}

template <int NT, int C>
struct SortCntLds {
    uint32_t buf[NT * C];          // the current order (packed words)
    CntScratch<NT> cs;
    int32_t rmin[NT / 64], rmax[NT / 64];
};

// One feature per workgroup at a time, in the visiting order sorder.
//
// defer (NULL when every value range fits beside the index, i.e. ib <= 14):
// a feature whose packed words would need more than 32 bits is not sorted
// here; its index goes to defer[16 + c] with c = atomicAdd(defer, 1), for
// the 64-bit path (k_sort over that list).
template <int NT, int C, int K0>
__global__ __launch_bounds__(NT) void k_sort_cnt(JobDev jd, const uint32_t* __restrict__ ftab,
                                                 const uint32_t* __restrict__ sorder, int ib,
                                                 uint32_t* __restrict__ defer) {
    constexpr int U = (C + 7) / 8;   // key units per thread: ceil(n / 8) <= U NT
    extern __shared__ __align__(16) unsigned char smem[];
    SortCntLds<NT, C>& L = *reinterpret_cast<SortCntLds<NT, C>*>(smem);
    const int tid = threadIdx.x;
    const int n = (int)jd.g.n;
    for (FeatureWalk wk = feature_walk(jd.F); wk.p < wk.end; wk.p += wk.step) {
        const int64_t j = sorder[wk.p];
        // values: in registers (up to 15 a thread), else through LDS
        int32_t vmin, vmax;
        int32_t v[C <= 15 ? C : 1];
        constexpr bool kRegs = C <= 15;
        if constexpr (kRegs) {
            eval_values<NT, C, K0>(jd, ftab[j], n, v);
            value_range<NT, C, K0>(v, n, L.rmin, L.rmax, vmin, vmax);
        } else {
            eval_to_lds<NT, C>(jd, ftab[j], n, L.buf, L.rmin, L.rmax, vmin, vmax);
        }
        const uint32_t range = (uint32_t)(vmax - vmin);
        const int rb = range == 0 ? 0 : 32 - __clz(range);   // <= 18 for windows up to 32x32
        if (defer != nullptr && rb + ib > 32) {   // uniform across the workgroup
            if (tid == 0) defer[16 + atomicAdd(defer, 1u)] = (uint32_t)j;
            __syncthreads();   // every thread has read the range before the next feature's
            continue;
        }
        // this thread's chunk (windows tC .. tC + C - 1) as packed words;
        // positions past n are all-ones sentinels (digit 15 in every pass,
        // behind every window)
        uint32_t it[C];
        if constexpr (kRegs) {
#pragma unroll
            for (int k = 0; k < C; ++k) {
                const int i = k * NT + tid;
                L.buf[i] = (k < K0 || i < n) ? (((uint32_t)(v[k] - vmin)) << ib) | (uint32_t)i : 0xFFFFFFFFu;
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < C; ++k) it[k] = L.buf[tid * C + k];
        } else {
#pragma unroll
            for (int k = 0; k < C; ++k) {
                const int i = tid * C + k;
                it[k] = i < n ? ((L.buf[i] - (uint32_t)vmin) << ib) | (uint32_t)i : 0xFFFFFFFFu;
            }
            if (rb == 0) {   // no pass: the words are already in order
#pragma unroll
                for (int k = 0; k < C; ++k) L.buf[tid * C + k] = it[k];
                __syncthreads();
            }
        }
        cnt_sort_passes<NT, C>(it, L.buf, L.cs, ib, ib + rb);
#pragma unroll
        for (int k = 0; k < U; ++k) {
            uint4 kq;
            unit_keys_w32<NT, 1>(jd.g, L.buf, ib, (1u << ib) - 1u, &kq, k * NT);
            store_unit_keys<NT, 1>(jd, j, &kq, k * NT);
        }
        // the next feature overwrites buf: with values in registers only after
        // the barrier of its value range, which every thread reaches after
        // its key reads here; with values through LDS, during its evaluation
        if constexpr (!kRegs) __syncthreads();
    }
}

// ---------------------------------------------------------------- incremental preparation
// Keys of a job extended by m new windows (the union's internal order: the
// old positives, the new positives, the old negatives, the new negatives),
// from the old job's keys: the old windows' order is already known, so only
// the new windows are sorted, and the two ordered lists are merged.
//   1. the union's values of the feature (one per window, as in k_sort_cnt)
//      and its packed words in index order;
//   2. the new windows' words in order (m <= 256), each ranked by counting
//      the new words below it;
//   3. the old windows' words in the old order (decoded from the old keys,
//      each old index moved to its union index; the move keeps their order);
//   4. a merge of the two lists (merge path: each thread finds where its E
//      outputs start by a binary search, then merges E words);
//   5. the keys in the union's layout.
// The words are unique (they carry the window index), so the result is
// exactly the (value, index) order a full sort of the union gives.
struct MergeArgs {
    const uint4* old_keys;   // the old job's keys
    KeyGeom og;              // their geometry
    int32_t l0, lm, n0, m;   // old positives, new positives, old windows, new windows
    int32_t ib;              // index bits of the union
    int32_t rb_off, x_off;   // LDS byte offsets of the new words' buffer and of the shared region
    int32_t nb_off;          // LDS byte offset of the new words in index order (16-byte aligned)
};

// C: window slots a thread holds (n <= 1024 C).  The new windows (m <= 256)
// are put in order by counting: their words are gathered into one array, and
// each new word's rank among them is the number of words below it (one pass
// over the m words, four a read; the counting-sort passes cost more than
// this at such sizes).
template <int C>
__global__ __launch_bounds__(1024) void k_merge(JobDev jd, const uint32_t* __restrict__ ftab,
                                               const uint32_t* __restrict__ sorder, MergeArgs ma) {
    constexpr int NT = 1024;
    constexpr int OU = 2;                                    // old units a thread reads (ceil(n0 / 8) <= 2 NT)
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t* buf = (uint32_t*)smem;                         // NT * C words: index order, then the merged order
    uint32_t* rbuf = (uint32_t*)(smem + ma.rb_off);          // the new windows' words in order
    uint32_t* abuf = (uint32_t*)(smem + ma.x_off);           // the old windows' words in the old order
    __shared__ int32_t rmin[NT / 64], rmax[NT / 64];
    const int tid = threadIdx.x;
    const int n = (int)jd.g.n;           // n0 + m
    const int mn = ma.m - ma.lm;         // new negatives: union indices n - mn .. n - 1
    const int E = (n + NT - 1) / NT;
    const KeyGeom& og = ma.og;
    const int olsh = __builtin_ctz((unsigned)og.lanes);
    auto new_index = [&](int p) { return p < ma.lm ? ma.l0 + p : n - mn + (p - ma.lm); };
    for (FeatureWalk wk = feature_walk(jd.F); wk.p < wk.end; wk.p += wk.step) {
        const int64_t j = sorder[wk.p];
        // the old keys of this feature, issued first so that their loads
        // overlap the evaluation (memory unit mu of the old row holds
        // rank-order unit start(L) + r of lane L = mu % lanes, r = mu / lanes)
        uint4 oq[OU];
#pragma unroll
        for (int k = 0; k < OU; ++k) {
            const int mu = tid + k * NT;
            oq[k] = mu < (int)og.nc ? ma.old_keys[j * og.row_units + mu] : make_uint4(0, 0, 0, 0);
        }
        // 1. the union's values and packed words in index order
        int32_t v[C], vmin, vmax;
        eval_values<NT, C>(jd, ftab[j], n, v);
        value_range<NT, C>(v, n, rmin, rmax, vmin, vmax);
        const uint32_t range = (uint32_t)(vmax - vmin);
        const int rb = range == 0 ? 0 : 32 - __clz(range);
#pragma unroll
        for (int k = 0; k < C; ++k) {
            const int i = k * NT + tid;
            if (i < n) buf[i] = (((uint32_t)(v[k] - vmin)) << ma.ib) | (uint32_t)i;
        }
        __syncthreads();
        // 2. the new windows in order (union indices l0 .. l0 + lm - 1, then n - mn .. n - 1):
        // gathered into nbuf, then each ranked against all of them, four words a read
        (void)rb;
        uint32_t* nbuf = (uint32_t*)(smem + ma.nb_off);
        if (tid < ma.m) nbuf[tid] = buf[new_index(tid)];
        __syncthreads();
        if (tid < ma.m) {
            const uint32_t x = nbuf[tid];
            int r = 0;
            const int m4 = ma.m & ~3;
            for (int q = 0; q < m4; q += 4) {   // words are unique
                const uint4 y = *reinterpret_cast<const uint4*>(nbuf + q);
                r += (y.x < x ? 1 : 0) + (y.y < x ? 1 : 0) + (y.z < x ? 1 : 0) + (y.w < x ? 1 : 0);
            }
            for (int q = m4; q < ma.m; ++q) r += nbuf[q] < x ? 1 : 0;
            rbuf[r] = x;
        }
        // 3. the old windows in the old order
#pragma unroll
        for (int k = 0; k < OU; ++k) {
            const int mu = tid + k * NT;
            if (mu < (int)og.nc) {
                const int L = mu & (og.lanes - 1);
                const int u = L * og.q + (L < og.rem ? L : og.rem) + (mu >> olsh);
                const uint32_t dw[4] = {oq[k].x, oq[k].y, oq[k].z, oq[k].w};
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    uint32_t i0, f0, i1, f1;
                    decode_pair(og.narrow, dw[h], i0, f0, i1, f1);
                    const int r0 = 8 * u + 2 * h;
                    if (r0 < ma.n0) abuf[r0] = buf[(int)i0 < ma.l0 ? i0 : i0 + ma.lm];
                    if (r0 + 1 < ma.n0) abuf[r0 + 1] = buf[(int)i1 < ma.l0 ? i1 : i1 + ma.lm];
                }
            }
        }
        __syncthreads();
        // 4. merge: outputs [p0, p1) of this thread
        {
            const int p0 = tid * E < n ? tid * E : n;
            const int p1 = p0 + E < n ? p0 + E : n;
            int lo = p0 > ma.m ? p0 - ma.m : 0, hi = p0 < ma.n0 ? p0 : ma.n0;
            while (lo < hi) {   // the number a of old words among the first p0 outputs
                const int mid = (lo + hi) >> 1;
                if (abuf[mid] < rbuf[p0 - 1 - mid]) lo = mid + 1; else hi = mid;
            }
            int a = lo, b = p0 - lo;
            uint32_t wa = a < ma.n0 ? abuf[a] : 0xFFFFFFFFu, wb = b < ma.m ? rbuf[b] : 0xFFFFFFFFu;
            uint32_t out[C];
#pragma unroll
            for (int k = 0; k < C; ++k) {
                if (k < E && p0 + k < p1) {
                    const bool ta = wa < wb;
                    out[k] = ta ? wa : wb;
                    if (ta) { ++a; wa = a < ma.n0 ? abuf[a] : 0xFFFFFFFFu; }
                    else { ++b; wb = b < ma.m ? rbuf[b] : 0xFFFFFFFFu; }
                }
            }
            __syncthreads();   // every thread has read its merge inputs (buf is rewritten next)
#pragma unroll
            for (int k = 0; k < C; ++k)
                if (k < E && p0 + k < p1) buf[p0 + k] = out[k];
        }
        __syncthreads();
        // 5.
        uint4 kq[2];
        unit_keys_w32<NT, 2>(jd.g, buf, ma.ib, (1u << ma.ib) - 1u, kq);
        store_unit_keys<NT, 2>(jd, j, kq);
        __syncthreads();
    }
}

int merge_launch(const JobDev& jd, const uint32_t* sorder, const uint4* old_keys, const KeyGeom& og, int l0, int lm, int num_cu,
                 hipStream_t s) {
    const int64_t n = jd.g.n;
    const int n0 = (int)og.n, m = (int)(n - og.n);
    if (n > kMergeMaxN || m < 1 || m > kMergeMaxM || !og.narrow) {
        set_error("merge: at most 256 new windows, a union of at most 15,360, narrow old keys");
        return BOOST_E_INVALID;
    }
    MergeArgs ma;
    ma.old_keys = old_keys;
    ma.og = og;
    ma.l0 = l0; ma.lm = lm; ma.n0 = n0; ma.m = m;
    ma.ib = n <= 1 ? 1 : 32 - __builtin_clz((unsigned)(n - 1));
    const int c = n <= 1024 * 11 ? 11 : 15;
    auto a16 = [](size_t x) { return (x + 15) & ~(size_t)15; };
    ma.rb_off = (int)a16((size_t)1024 * c * 4);
    ma.x_off = (int)a16((size_t)ma.rb_off + (size_t)kMergeMaxM * 4);
    ma.nb_off = (int)a16((size_t)ma.x_off + (size_t)n0 * 4);
    const size_t lds = (size_t)ma.nb_off + (size_t)kMergeMaxM * 4;
    const void* k = c == 11 ? (const void*)k_merge<11> : (const void*)k_merge<15>;
    VJB_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int per_cu = 0;
    VJB_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 1024, lds));
    if (per_cu < 1) {
        set_error("merge kernel does not fit on a compute unit");
        return BOOST_E_INVALID;
    }
    int64_t grid = (int64_t)per_cu * num_cu;
    if (grid > jd.F) grid = jd.F;
    if (grid > kMaxSortGrid) grid = kMaxSortGrid;
    JobDev a = jd;
    const uint32_t* ftab = jd.ftab;
    void* args[] = {(void*)&a, (void*)&ftab, (void*)&sorder, (void*)&ma};
    VJB_HIP(hipLaunchKernel(k, dim3((unsigned)grid), dim3(1024), args, lds, s));
    return BOOST_OK;
}

// K0: slots every thread holds a window in (n >= K0 NT).
template <int NT, int C, int K0>
static int sort_cnt_launch(const JobDev& jd, const uint32_t* sorder, uint32_t* defer, int num_cu, hipStream_t s) {
    const int64_t n = jd.g.n;
    if (n < (int64_t)K0 * NT || n > (int64_t)C * NT) {
        set_error("sort: window count outside the kernel's range");
        return BOOST_E_INVALID;
    }
    int ib = n <= 1 ? 1 : 32 - __builtin_clz((unsigned)(n - 1));
    const size_t lds = sizeof(SortCntLds<NT, C>);
    const void* k = (const void*)k_sort_cnt<NT, C, K0>;
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
    const uint32_t* ftab = jd.ftab;
    void* args[] = {(void*)&a, (void*)&ftab, (void*)&sorder, (void*)&ib, (void*)&defer};
    VJB_HIP(hipLaunchKernel(k, dim3((unsigned)grid), dim3(NT), args, lds, s));
    return BOOST_OK;
}

template <int NT, int C>
static int sort_launch_c(const JobDev& jd, uint64_t* scratch, const uint32_t* list, int num_cu, hipStream_t s) {
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
    void* args[] = {(void*)&a, (void*)&npow2, (void*)&ib, (void*)&scratch, (void*)&list};
    VJB_HIP(hipLaunchKernel(k, dim3((unsigned)grid), dim3(NT), args, lds, s));
    return BOOST_OK;
}

// Counting-sort passes up to 15,360 windows (C values per thread, the
// smallest odd C of the shape that covers n); ballot-ranked passes beyond.
int sort_launch(const JobDev& jd, const uint32_t* sorder, uint64_t* scratch, uint32_t* defer, int num_cu,
                hipStream_t s) {
    const int64_t n = jd.g.n;
    // each tier's K0: the slots the previous tier's bound already fills
    if (n <= 256 * 7) return sort_cnt_launch<256, 7, 0>(jd, sorder, nullptr, num_cu, s);
    if (n <= 512 * 7) return sort_cnt_launch<512, 7, 3>(jd, sorder, nullptr, num_cu, s);
    if (n <= 1024 * 7) return sort_cnt_launch<1024, 7, 3>(jd, sorder, nullptr, num_cu, s);
    if (n <= 1024 * 11) return sort_cnt_launch<1024, 11, 7>(jd, sorder, nullptr, num_cu, s);
    if (n <= 1024 * 15) return sort_cnt_launch<1024, 15, 11>(jd, sorder, nullptr, num_cu, s);
    if (n <= kNarrowMaxN + 1) return sort_cnt_launch<1024, 31, 15>(jd, sorder, nullptr, num_cu, s);   // 14-bit indices
    if (n <= 1024 * 31) {
        // 15-bit indices: features whose values span more than 17 bits go
        // through the 64-bit path, listed by the counting sort
        if (defer == nullptr || scratch == nullptr) {
            set_error("sort: the defer list or the fallback scratch is missing");
            return BOOST_E_INVALID;
        }
        VJB_HIP(hipMemsetAsync(defer, 0, 4, s));
        int rc = sort_cnt_launch<1024, 31, 15>(jd, sorder, defer, num_cu, s);
        if (rc != BOOST_OK) return rc;
        return sort_launch_c<512, 64>(jd, scratch, defer, num_cu, s);
    }
    if (n <= 32768) return sort_launch_c<512, 64>(jd, scratch, nullptr, num_cu, s);
    set_error("too many windows for the sort");
    return BOOST_E_INVALID;
}

}  // namespace vjb
