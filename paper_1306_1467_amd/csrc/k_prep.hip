// One-time and inspection kernels of one job: ingest (positives-first order),
// integral images (Section 2.1), initial weights (Section 2.3 Table 2), weight
// get/set, feature values (Section 2.2) and decoding of the sorted keys.
#include "launch.h"
#include "scan_core.h"

namespace vjb {

// ---------------------------------------------------------------- ingest
// Stable positives-first order: positive caller index e goes to internal
// index (#positives before e), negative e to l + (#negatives before e).
__global__ __launch_bounds__(1024) void k_ingest(const uint8_t* __restrict__ labels, int64_t n,
                                                 int32_t* __restrict__ perm, int32_t* __restrict__ inv,
                                                 JobState* st) {
    constexpr int NT = 1024;
    __shared__ int32_t wsum[NT / 64];
    __shared__ int32_t s_bad;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (tid == 0) s_bad = 0;
    __syncthreads();
    // pass 1: count positives, validate
    int32_t cnt = 0;
    int bad = 0;
    for (int64_t e = tid; e < n; e += NT) {
        const uint8_t y = labels[e];
        cnt += (y == 1);
        bad |= (y > 1);
    }
    for (int o = 32; o; o >>= 1) cnt += __shfl_xor(cnt, o);
    if (lane == 0) wsum[wv] = cnt;
    if (bad) atomicOr(&s_bad, 1);
    __syncthreads();
    int32_t l = 0;
    for (int k = 0; k < NT / 64; ++k) l += wsum[k];
    __syncthreads();
    // pass 2: ranks within each class, chunk by chunk
    int32_t pos_base = 0, neg_base = 0;
    for (int64_t c0 = 0; c0 < n; c0 += NT) {
        const int64_t e = c0 + tid;
        const bool valid = e < n;
        const bool pos = valid && labels[e] == 1;
        const unsigned long long bp = __ballot(pos);
        const unsigned long long bv = __ballot(valid);
        const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        const int32_t pos_in_wave = __popcll(bp & below);
        const int32_t val_in_wave = __popcll(bv & below);
        if (lane == 0) wsum[wv] = __popcll(bp) | (__popcll(bv) << 16);
        __syncthreads();
        int32_t pos_before = 0, val_before = 0, pos_tot = 0, val_tot = 0;
        for (int k = 0; k < NT / 64; ++k) {
            const int32_t p = wsum[k] & 0xFFFF, v = wsum[k] >> 16;
            if (k < wv) { pos_before += p; val_before += v; }
            pos_tot += p; val_tot += v;
        }
        if (valid) {
            const int32_t pr = pos_before + pos_in_wave;
            const int32_t nr = (val_before + val_in_wave) - pr;
            const int32_t idx = pos ? pos_base + pr : l + neg_base + nr;
            perm[idx] = (int32_t)e;
            inv[e] = idx;
        }
        pos_base += pos_tot;
        neg_base += val_tot - pos_tot;
        __syncthreads();
    }
    if (tid == 0) {
        st->n_pos = l;
        st->label_error = s_bad;
        st->round = 0;
        st->stopped = 0;
        st->weight_error = 0;
        st->launches = 0;
    }
}

int ingest_launch(const JobDev& jd, const uint8_t* d_labels, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_ingest, dim3(1), dim3(1024), 0, s, d_labels, n, (int32_t*)jd.perm, (int32_t*)jd.inv, jd.st);
    VJB_HIP(hipGetLastError());
    return BOOST_OK;
}

// ---------------------------------------------------------------- integral images
// One thread per window; ii[(r*(W+1)+c)*S + i], so a wave's 64 windows write
// 256 contiguous bytes per position.  Sample i is window perm[i] of the
// images (or window i when perm is NULL).
__global__ void k_integral(const uint8_t* __restrict__ images, const int32_t* __restrict__ perm, int64_t n, int W,
                           int H, int32_t* __restrict__ ii, int64_t S) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint8_t* img = images + (perm != nullptr ? (int64_t)perm[i] : i) * W * H;
    const int wp1 = W + 1;
    for (int c = 0; c <= W; ++c) ii[(int64_t)c * S + i] = 0;
    for (int r = 0; r < H; ++r) {
        int32_t row = 0;
        ii[(int64_t)((r + 1) * wp1) * S + i] = 0;
        for (int c = 0; c < W; ++c) {
            row += img[r * W + c];
            const int32_t above = ii[(int64_t)(r * wp1 + c + 1) * S + i];
            ii[(int64_t)((r + 1) * wp1 + c + 1) * S + i] = above + row;
        }
    }
}

int integral_raw_launch(const uint8_t* d_images, const int32_t* perm, int64_t n, int W, int H, int32_t* ii, int64_t S,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_integral, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d_images, perm, n, W, H, ii, S);
    VJB_HIP(hipGetLastError());
    return BOOST_OK;
}

int integral_launch(const JobDev& jd, const uint8_t* d_images, hipStream_t s) {
    return integral_raw_launch(d_images, jd.perm, jd.g.n, jd.W, jd.H, (int32_t*)jd.ii, jd.ii_stride, s);
}

// ---------------------------------------------------------------- extending a job
// Labels of a job extended by m windows, in the union's caller order: the
// old windows' labels from the old positives-first order (caller window e is
// positive iff its internal index is below l0), then the new ones.
__global__ void k_union_labels(const int32_t* __restrict__ old_inv, int64_t n0, int64_t l0,
                               const uint8_t* __restrict__ new_labels, int64_t m, uint8_t* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n0) out[e] = old_inv[e] < l0 ? 1 : 0;
    else if (e < n0 + m) out[e] = new_labels[e - n0];
}

// Integral images of the union: sample i is caller window e = perm[i]; an old
// window's column entries are copied from its old sample, a new window's
// image is integrated.
__global__ void k_extend_ii(const int32_t* __restrict__ perm, int64_t n, int64_t n0,
                            const int32_t* __restrict__ old_inv, const int32_t* __restrict__ old_ii, int64_t old_S,
                            const uint8_t* __restrict__ new_images, int W, int H, int32_t* __restrict__ ii, int64_t S) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t e = perm[i];
    const int wp1 = W + 1;
    const int64_t P = (int64_t)wp1 * (H + 1);
    if (e < n0) {
        const int64_t io = old_inv[e];
        for (int64_t p = 0; p < P; ++p) ii[p * S + i] = old_ii[p * old_S + io];
        return;
    }
    const uint8_t* img = new_images + (e - n0) * W * H;
    for (int c = 0; c <= W; ++c) ii[(int64_t)c * S + i] = 0;
    for (int r = 0; r < H; ++r) {
        int32_t row = 0;
        ii[(int64_t)((r + 1) * wp1) * S + i] = 0;
        for (int c = 0; c < W; ++c) {
            row += img[r * W + c];
            const int32_t above = ii[(int64_t)(r * wp1 + c + 1) * S + i];
            ii[(int64_t)((r + 1) * wp1 + c + 1) * S + i] = above + row;
        }
    }
}

int union_labels_launch(const JobDev& old, int64_t l0, const uint8_t* d_new_labels, int64_t m, uint8_t* d_out,
                        hipStream_t s) {
    const int64_t N = old.g.n + m;
    hipLaunchKernelGGL(k_union_labels, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, old.inv, old.g.n, l0,
                       d_new_labels, m, d_out);
    VJB_HIP(hipGetLastError());
    return BOOST_OK;
}

int extend_ii_launch(const JobDev& jd, const JobDev& old, const uint8_t* d_new_images, hipStream_t s) {
    const int64_t n = jd.g.n;
    hipLaunchKernelGGL(k_extend_ii, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, jd.perm, n, old.g.n, old.inv,
                       old.ii, old.ii_stride, d_new_images, jd.W, jd.H, (int32_t*)jd.ii, jd.ii_stride);
    VJB_HIP(hipGetLastError());
    return BOOST_OK;
}

// ---------------------------------------------------------------- weights
// Table 2 of Section 2.3: 1/(2l) for positives, 1/(2m) for negatives.  The
// stored weights divided by the sum of the partials are the normalised ones
// (step 1); the scan normalises as it fills its table.
__global__ __launch_bounds__(1024) void k_init_weights(JobDev jd) {
    __shared__ double sh[4];
    const int64_t n = jd.g.n, l = jd.st->n_pos, m = n - l;
    const double wp = 1.0 / (2.0 * (double)l), wn = 1.0 / (2.0 * (double)m);
    double* w = weights(jd, jd.st->wpar);
    for (int64_t i = threadIdx.x; i < n; i += 1024) w[i] = i < l ? wp : wn;
    __syncthreads();
    reset_partials(jd, w, sh);
}

int init_weights_launch(const JobDev& jd, hipStream_t s) {
    hipLaunchKernelGGL(k_init_weights, dim3(1), dim3(1024), 0, s, jd);
    VJB_HIP(hipGetLastError());
    return BOOST_OK;
}

// Caller weights -> validate -> internal order.  Rejected input leaves the
// stored weights untouched.
__global__ __launch_bounds__(1024) void k_set_weights(JobDev jd, const double* __restrict__ src, double* __restrict__ tmp) {
    __shared__ double sh[4];
    __shared__ int s_bad;
    const int64_t n = jd.g.n;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    int bad = 0;
    for (int64_t e = threadIdx.x; e < n; e += 1024) {
        const double v = src[e];
        if (!(v >= 0.0) || !(v <= 1.0e308)) bad = 1;
        tmp[jd.inv[e]] = v;
    }
    if (bad) atomicOr(&s_bad, 1);
    __syncthreads();
    const double sum = fixed_sum256(n, [&](int64_t i) { return tmp[i]; }, sh);
    if (s_bad || !(sum > 0.0) || !(sum <= 1.0e308)) {
        if (threadIdx.x == 0) jd.st->weight_error = 1;
        return;
    }
    double* w = weights(jd, jd.st->wpar);
    for (int64_t i = threadIdx.x; i < n; i += 1024) w[i] = tmp[i];
    __syncthreads();
    reset_partials(jd, w, sh);
    if (threadIdx.x == 0) jd.st->weight_error = 0;
}

int set_weights_launch(const JobDev& jd, const double* d_w, double* tmp, hipStream_t s) {
    hipLaunchKernelGGL(k_set_weights, dim3(1), dim3(1024), 0, s, jd, d_w, tmp);
    VJB_HIP(hipGetLastError());
    return BOOST_OK;
}

__global__ void k_get_weights(JobDev jd, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double rS = 1.0 / weight_sum(jd);   // whole wave
    if (i < jd.g.n) out[jd.perm[i]] = weights(jd, jd.st->wpar)[i] * rS;
}

int get_weights_launch(const JobDev& jd, double* d_out, hipStream_t s) {
    const int64_t n = jd.g.n;
    hipLaunchKernelGGL(k_get_weights, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, jd, d_out);
    VJB_HIP(hipGetLastError());
    return BOOST_OK;
}

// ---------------------------------------------------------------- inspection
__global__ void k_feature_values(JobDev jd, int64_t j0, int32_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t jj = blockIdx.y;
    if (i >= jd.g.n) return;
    const uint32_t desc = jd.ftab[j0 + jj];
    out[jj * jd.g.n + jd.perm[i]] = haar_value(jd.ii, jd.ii_stride, jd.W + 1, desc, i);
}

int feature_values_launch(const JobDev& jd, int64_t j0, int64_t nf, int32_t* d_out, hipStream_t s) {
    const int64_t n = jd.g.n;
    for (int64_t c = 0; c < nf; c += 65535) {
        const int64_t m = nf - c < 65535 ? nf - c : 65535;
        hipLaunchKernelGGL(k_feature_values, dim3((unsigned)((n + 255) / 256), (unsigned)m), dim3(256), 0, s, jd,
                           j0 + c, d_out + c * n);
        VJB_HIP(hipGetLastError());
    }
    return BOOST_OK;
}

__global__ void k_integral_out(JobDev jd, int32_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= jd.g.n) return;
    const int64_t P = (int64_t)(jd.W + 1) * (jd.H + 1);
    const int64_t e = jd.perm[i];
    for (int64_t p = 0; p < P; ++p) out[e * P + p] = jd.ii[p * jd.ii_stride + i];
}

int integral_out_launch(const JobDev& jd, int32_t* d_out, hipStream_t s) {
    const int64_t n = jd.g.n;
    hipLaunchKernelGGL(k_integral_out, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, jd, d_out);
    VJB_HIP(hipGetLastError());
    return BOOST_OK;
}

__global__ void k_sorted_out(JobDev jd, int64_t j0, int32_t* __restrict__ order, uint8_t* __restrict__ flags) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t jj = blockIdx.y;
    const int64_t n = jd.g.n;
    if (r >= n) return;
    const int64_t mu = unit_to_mem(jd.g, r >> 3);
    const uint4 u = jd.keys[(j0 + jj) * jd.g.row_units + mu];
    const int e = (int)(r & 7);
    const uint32_t d = (e >> 1) == 0 ? u.x : (e >> 1) == 1 ? u.y : (e >> 1) == 2 ? u.z : u.w;
    uint32_t i0, f0, i1, f1;
    decode_pair(jd.g.narrow, d, i0, f0, i1, f1);
    const uint32_t idx = (e & 1) ? i1 : i0;
    const uint32_t f = (e & 1) ? f1 : f0;
    order[jj * n + r] = idx < (uint32_t)n ? jd.perm[idx] : -1;
    flags[jj * n + r] = (uint8_t)f;
}

int sorted_out_launch(const JobDev& jd, int64_t j0, int64_t nf, int32_t* d_order, uint8_t* d_flags, hipStream_t s) {
    const int64_t n = jd.g.n;
    for (int64_t c = 0; c < nf; c += 65535) {
        const int64_t m = nf - c < 65535 ? nf - c : 65535;
        hipLaunchKernelGGL(k_sorted_out, dim3((unsigned)((n + 255) / 256), (unsigned)m), dim3(256), 0, s, jd, j0 + c,
                           d_order + c * n, d_flags + c * n);
        VJB_HIP(hipGetLastError());
    }
    return BOOST_OK;
}

}  // namespace vjb
