// The strong classifier of Section 2.3 on any set of windows:
//     C(x) = 1  iff  sum_t alpha_t h_t(x) >= 1/2 sum_t alpha_t,
// with h_t(x) = 1 iff p_t f_t(x) < p_t theta_t (Section 2.2), and, when labels
// are known, the training / test error of every prefix classifier C_1 .. C_T
// (the first t stumps) in the same launch.
//
// One thread per window walks the stumps in order, keeping s_t (the alpha of
// the stumps that vote 1) and A_t (all alphas so far) in FP64 and in that
// order; C_t(x) = [s_t >= A_t / 2].  The stump table is uniform across the
// workgroup (scalar loads); the feature values come from sample-minor
// integral images, so a wave's corner reads are coalesced.  Wrong decisions
// are counted per prefix with one wave ballot per stump, per workgroup in LDS,
// then added to the output curve with one atomic per (workgroup, stump).
#include <math.h>

#include <mutex>
#include <string>

#include "launch.h"

namespace vjb {

constexpr int kClsWg = 256;

// LABELS: 0 none, 1 caller's labels (array in caller order), 2 internal
// positives-first order (y = [i < l]).
template <int LABELS>
__global__ __launch_bounds__(kClsWg) void k_classify_any(const int32_t* __restrict__ ii, int64_t S, int wp1, int64_t n,
                                                         const StumpDev* __restrict__ st, int T,
                                                         const int32_t* __restrict__ perm,
                                                         const uint8_t* __restrict__ labels, int64_t l,
                                                         uint8_t* __restrict__ out, double* __restrict__ score,
                                                         int32_t* __restrict__ curve) {
    __shared__ int32_t cnt[kMaxClassifyT];
    const int64_t i = (int64_t)blockIdx.x * kClsWg + threadIdx.x;
    const bool live = i < n;
    const int64_t e = live ? (perm != nullptr ? (int64_t)perm[i] : i) : 0;
    int y = 0;
    if constexpr (LABELS == 1) y = live ? (int)labels[e] : 0;
    if constexpr (LABELS == 2) y = i < l ? 1 : 0;
    if constexpr (LABELS != 0) {
        for (int t = threadIdx.x; t < T; t += kClsWg) cnt[t] = 0;
        __syncthreads();
    }
    double s = 0.0, a = 0.0;
    for (int t = 0; t < T; ++t) {
        const StumpDev sd = st[t];
        const int32_t f = live ? haar_value(ii, S, wp1, sd.desc, i) : 0;
        if ((int64_t)sd.polarity * f < (int64_t)sd.polarity * sd.theta) s += sd.alpha;
        a += sd.alpha;
        if constexpr (LABELS != 0) {
            const int c = s >= 0.5 * a ? 1 : 0;
            const unsigned long long wrong = __ballot(live && c != y);
            if ((threadIdx.x & 63) == 0 && wrong != 0ull) atomicAdd(&cnt[t], (int32_t)__popcll(wrong));
        }
    }
    if (live) {
        if (out != nullptr) out[e] = s >= 0.5 * a ? 1 : 0;
        if (score != nullptr) score[e] = s;
    }
    if constexpr (LABELS != 0) {
        __syncthreads();
        if (curve != nullptr)
            for (int t = threadIdx.x; t < T; t += kClsWg)
                if (cnt[t] != 0) atomicAdd(&curve[t], cnt[t]);
    }
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t m, int32_t v) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < m) p[k] = v;
}

int classify_any_launch(const int32_t* ii, int64_t S, int W, int64_t n, const StumpDev* d_stumps, int T,
                        const int32_t* perm, const uint8_t* labels, int64_t l, uint8_t* d_out, double* d_score,
                        int32_t* d_curve, hipStream_t s) {
    if (d_curve != nullptr && T > 0) {
        hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((T + 255) / 256)), dim3(256), 0, s, d_curve, (int64_t)T, 0);
        VJB_HIP(hipGetLastError());
    }
    const dim3 grid((unsigned)((n + kClsWg - 1) / kClsWg)), block(kClsWg);
    if (labels != nullptr)
        hipLaunchKernelGGL(k_classify_any<1>, grid, block, 0, s, ii, S, W + 1, n, d_stumps, T, perm, labels, l, d_out,
                           d_score, d_curve);
    else if (l >= 0)
        hipLaunchKernelGGL(k_classify_any<2>, grid, block, 0, s, ii, S, W + 1, n, d_stumps, T, perm, labels, l, d_out,
                           d_score, d_curve);
    else
        hipLaunchKernelGGL(k_classify_any<0>, grid, block, 0, s, ii, S, W + 1, n, d_stumps, T, perm, labels, l, d_out,
                           d_score, d_curve);
    VJB_HIP(hipGetLastError());
    return BOOST_OK;
}

// Checks stump records against a window: polarity +-1, finite alpha, a
// known type whose cells fit the window.
static int check_stumps(const boost_stump* stumps, int T, int W, int H) {
    static const int kBw[5] = {3, 1, 2, 1, 2};
    static const int kBh[5] = {1, 3, 1, 2, 2};
    for (int t = 0; t < T; ++t) {
        const boost_stump& r = stumps[t];
        const bool ok = r.type >= 0 && r.type < 5 && r.cell_w >= 1 && r.cell_h >= 1 && r.x >= 0 && r.y >= 0 &&
                        r.x + kBw[r.type < 0 || r.type > 4 ? 0 : r.type] * r.cell_w <= W &&
                        r.y + kBh[r.type < 0 || r.type > 4 ? 0 : r.type] * r.cell_h <= H &&
                        (r.polarity == 1 || r.polarity == -1) && isfinite(r.alpha);
        if (!ok) {
            set_error("invalid stump record " + std::to_string(t) + " for a " + std::to_string(W) + "x" +
                      std::to_string(H) + " window");
            return BOOST_E_INVALID;
        }
    }
    return BOOST_OK;
}

// The device stump table from records already checked on the host.
__global__ void k_pack_stumps(const boost_stump* __restrict__ rec, int T, StumpDev* __restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    const boost_stump r = rec[t];
    StumpDev d;
    d.desc = pack_feature(r.type, r.x, r.y, r.cell_w, r.cell_h);
    d.polarity = r.polarity;
    d.theta = r.threshold;
    d.pad = 0;
    d.alpha = r.alpha;
    out[t] = d;
}

// Device memory of one call: the windows' integral images, the caller's
// records as copied, and the packed stump table.
static size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }
static size_t classify_ii_bytes(int64_t n, int W, int H) {
    return a256((size_t)(W + 1) * (size_t)(H + 1) * (size_t)ii_stride_of(n) * 4);
}
static size_t classify_rec_bytes() { return a256((size_t)kMaxClassifyT * sizeof(boost_stump)); }
static size_t classify_bytes(int64_t n, int W, int H) {
    return classify_ii_bytes(n, W, H) + classify_rec_bytes() + a256((size_t)kMaxClassifyT * sizeof(StumpDev));
}

static int check_classify_args(const uint8_t* d_images, int64_t n, int32_t W, int32_t H, const boost_stump* stumps,
                               int32_t T, const uint8_t* d_labels, int32_t* d_err_curve) {
    if (!d_images || n < 1 || W < 1 || W > kMaxWindow || H < 1 || H > kMaxWindow) {
        set_error("classify: NULL images, n < 1 or a window outside 1..32");
        return BOOST_E_INVALID;
    }
    if (T < 0 || T > kMaxClassifyT || (T > 0 && !stumps)) {
        set_error("classify: 0..4096 stumps required");
        return BOOST_E_INVALID;
    }
    if (d_err_curve && !d_labels) {
        set_error("classify: the error curve needs labels");
        return BOOST_E_INVALID;
    }
    return BOOST_OK;
}

// Integral images of the windows, the stump table, then the classifier, on
// stream s, in device memory `mem` (classify_bytes(n, W, H) bytes) that the
// caller or the library owns.  Allocates nothing.  Synchronises.
static int classify_windows(const uint8_t* d_images, int64_t n, int32_t W, int32_t H, const uint8_t* d_labels,
                            const boost_stump* stumps, int32_t T, uint8_t* d_out, double* d_score,
                            int32_t* d_err_curve, hipStream_t s, char* mem) {
    int rc = check_stumps(stumps, T, W, H);
    if (rc != BOOST_OK) return rc;
    int32_t* ii = (int32_t*)mem;
    boost_stump* rec = (boost_stump*)(mem + classify_ii_bytes(n, W, H));
    StumpDev* tab = (StumpDev*)(mem + classify_ii_bytes(n, W, H) + classify_rec_bytes());
    const int64_t S = ii_stride_of(n);
    if ((rc = integral_raw_launch(d_images, nullptr, n, W, H, ii, S, s)) != BOOST_OK) return rc;
    if (T > 0) {
        VJB_HIP(hipMemcpyAsync(rec, stumps, (size_t)T * sizeof(boost_stump), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_pack_stumps, dim3((unsigned)((T + 255) / 256)), dim3(256), 0, s, rec, T, tab);
        VJB_HIP(hipGetLastError());
    }
    rc = classify_any_launch(ii, S, W, n, tab, T, nullptr, d_labels, -1, d_out, d_score, d_err_curve, s);
    if (rc != BOOST_OK) return rc;
    VJB_HIP(hipStreamSynchronize(s));   // the caller's host records are read by the copy
    return BOOST_OK;
}

// ---------------------------------------------------------------- the allocation-free variant
// Device memory of boost_classify_noalloc: a file-scope array that every GPU
// the library runs on holds from module load until the process ends.  Host
// code never passes `scratch` itself (its host-side name is a stand-in, not a
// device address): the device address of each GPU's copy is looked up once
// per device with that device current, and only that address is used.
constexpr size_t kNoAllocBytes = (size_t)32 << 20;   // 32 MiB
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

static int scratch_ptr(int device, char** out) {
    if (device < 0 || device >= kMaxDevices) { set_error("device index out of range"); return BOOST_E_DEVICE; }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device] == nullptr) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            return BOOST_E_DEVICE;
        }
        g_scratch_ptr[device] = p;
    }
    *out = (char*)g_scratch_ptr[device];
    return BOOST_OK;
}

}  // namespace vjb

using namespace vjb;

extern "C" {

size_t boost_classify_workspace_bytes(int64_t n, int32_t window_w, int32_t window_h) {
    if (n < 1 || window_w < 1 || window_w > kMaxWindow || window_h < 1 || window_h > kMaxWindow) return 0;
    return classify_bytes(n, window_w, window_h);
}

int boost_classify(const uint8_t* d_images, int64_t n, int32_t window_w, int32_t window_h, const uint8_t* d_labels,
                   const boost_stump* stumps, int32_t T, uint8_t* d_out, double* d_score, int32_t* d_err_curve,
                   void* stream, void* d_workspace, size_t workspace_bytes) {
    int rc = check_classify_args(d_images, n, window_w, window_h, stumps, T, d_labels, d_err_curve);
    if (rc != BOOST_OK) return rc;
    if (!d_workspace) { set_error("classify: NULL workspace"); return BOOST_E_INVALID; }
    const size_t need = classify_bytes(n, window_w, window_h);
    if (workspace_bytes < need) {
        set_error("classify: workspace too small: need " + std::to_string(need) + " bytes");
        return BOOST_E_NOMEM;
    }
    return classify_windows(d_images, n, window_w, window_h, d_labels, stumps, T, d_out, d_score, d_err_curve,
                            (hipStream_t)stream, (char*)d_workspace);
}

size_t boost_classify_noalloc_max_windows(int32_t window_w, int32_t window_h) {
    if (window_w < 1 || window_w > kMaxWindow || window_h < 1 || window_h > kMaxWindow) return 0;
    // classify_bytes grows with n in steps of 64 windows (the integral images' stride)
    const size_t fixed = classify_rec_bytes() + a256((size_t)kMaxClassifyT * sizeof(StumpDev));
    const size_t per64 = (size_t)(window_w + 1) * (size_t)(window_h + 1) * 64 * 4;
    if (kNoAllocBytes <= fixed + 256) return 0;
    size_t n = (kNoAllocBytes - fixed - 255) / per64 * 64;
    while (n > 0 && classify_bytes((int64_t)n, window_w, window_h) > kNoAllocBytes) n -= 64;
    return n;
}

int boost_classify_noalloc(const uint8_t* d_images, int64_t n, int32_t window_w, int32_t window_h,
                           const uint8_t* d_labels, const boost_stump* stumps, int32_t T, uint8_t* d_out,
                           double* d_score, int32_t* d_err_curve, void* stream) {
    int rc = check_classify_args(d_images, n, window_w, window_h, stumps, T, d_labels, d_err_curve);
    if (rc != BOOST_OK) return rc;
    const size_t need = classify_bytes(n, window_w, window_h);
    if (need > kNoAllocBytes) {
        set_error("classify_noalloc: " + std::to_string(n) + " windows of " + std::to_string(window_w) + "x" +
                  std::to_string(window_h) + " need " + std::to_string(need) + " bytes of its " +
                  std::to_string(kNoAllocBytes) + "-byte device buffer (at most " +
                  std::to_string(boost_classify_noalloc_max_windows(window_w, window_h)) + " windows per call)");
        return BOOST_E_INVALID;
    }
    int device = 0;
    VJB_HIP(hipGetDevice(&device));
    char* mem = nullptr;
    if ((rc = scratch_ptr(device, &mem)) != BOOST_OK) return rc;
    return classify_windows(d_images, n, window_w, window_h, d_labels, stumps, T, d_out, d_score, d_err_curve,
                            (hipStream_t)stream, mem);
}

}  // extern "C"
