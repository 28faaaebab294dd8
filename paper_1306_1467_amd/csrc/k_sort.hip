// One-time preparation of every feature: evaluate the Haar feature on all
// windows (Section 2.2), order the windows by value, and write the per-feature
// keys (window index + end-of-run flag) in the lane-segment layout that the
// per-round scan reads.  Feature values never reach HBM: each workgroup holds
// one feature's n values in LDS, packed with their window index as
// ((v - vmin) << ib) | i in 32 bits, and sorts them there (bitonic network).
// A feature whose value range does not fit beside the index in 32 bits
// (possible only for n > 16384) is sorted as 64-bit pairs in a per-workgroup
// global scratch buffer instead.
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
    const int64_t n = g.n;
    uint4* row = (uint4*)(jd.keys + j * g.row_units);
    for (int64_t mu = threadIdx.x; mu < g.nc; mu += NT) {
        const int64_t u = mem_to_unit(g, mu);
        uint32_t dw[4];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            uint32_t ix[2], fl[2];
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int64_t r = 8 * u + 2 * h + b;
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

template <int NT>
__global__ __launch_bounds__(NT) void k_sort(JobDev jd, int64_t npow2, int ib, uint64_t* __restrict__ scratch) {
    extern __shared__ __align__(16) uint32_t s[];
    __shared__ int32_t rmin[NT / 64], rmax[NT / 64];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t n = jd.g.n;
    const int wp1 = jd.W + 1;
    const uint32_t imask = (1u << ib) - 1u;
    for (int64_t j = blockIdx.x; j < jd.F; j += gridDim.x) {
        const uint32_t desc = jd.ftab[j];
        int32_t vmin = INT_MAX, vmax = INT_MIN;
        for (int64_t i = tid; i < n; i += NT) {
            const int32_t v = haar_value(jd.ii, jd.ii_stride, wp1, desc, i);
            s[i] = (uint32_t)v;
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
        for (int k = 1; k < NT / 64; ++k) {
            vmin = rmin[k] < vmin ? rmin[k] : vmin;
            vmax = rmax[k] > vmax ? rmax[k] : vmax;
        }
        const uint32_t range = (uint32_t)(vmax - vmin);
        const int rb = range == 0 ? 0 : 32 - __clz(range);
        if (rb + ib <= 32) {
            for (int64_t i = tid; i < npow2; i += NT)
                s[i] = i < n ? (((uint32_t)((int32_t)s[i] - vmin)) << ib) | (uint32_t)i : 0xFFFFFFFFu;
            __syncthreads();
            bitonic_sort<NT, uint32_t>(s, npow2);
            emit_keys<NT, uint32_t>(jd, j, s, ib, imask);
        } else {
            uint64_t* g = scratch + (int64_t)blockIdx.x * npow2;
            for (int64_t i = tid; i < npow2; i += NT)
                g[i] = i < n ? (((uint64_t)(uint32_t)((int32_t)s[i] - vmin)) << 32) | (uint64_t)i : ~0ull;
            __syncthreads();
            bitonic_sort<NT, uint64_t>(g, npow2);
            emit_keys<NT, uint64_t>(jd, j, g, 32, 0xFFFFFFFFull);
        }
        __syncthreads();
    }
}

int sort_launch(const JobDev& jd, uint64_t* scratch, int num_cu, hipStream_t s) {
    constexpr int NT = 1024;
    const int64_t n = jd.g.n;
    const int64_t npow2 = sort_pow2(n);
    const int ib = n <= 1 ? 1 : 32 - __builtin_clz((unsigned)(n - 1));
    const size_t lds = (size_t)npow2 * sizeof(uint32_t);
    const void* k = (const void*)k_sort<NT>;
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
    int ibv = ib;
    args[2] = (void*)&ibv;
    int64_t np = npow2;
    args[1] = (void*)&np;
    VJB_HIP(hipLaunchKernel(k, dim3((unsigned)grid), dim3(NT), args, lds, s));
    return BOOST_OK;
}

}  // namespace vjb
