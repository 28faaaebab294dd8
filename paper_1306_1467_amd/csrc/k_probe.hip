// Memory-system ceiling of the per-round scan: a kernel that reads every key
// of the job exactly as the scan does (same grid, workgroup size, lane
// segments, load batches and padding-unit tails, non-temporal 16-byte loads)
// and does no arithmetic on them beyond folding them into one word per
// workgroup.  Its key bytes over its time are the bandwidth the scan could
// reach if its LDS gathers and FP64 sums were free.
#include "launch.h"
#include "scan_core.h"

namespace vjb {

template <int WG, int UNROLL, int LPF>
__global__ __launch_bounds__(WG) void k_probe(JobDev jd, uint32_t* __restrict__ sink) {
    constexpr int G = 64 / LPF;
    __shared__ uint32_t s_acc[WG / 64];
    const int lane = threadIdx.x & 63, grp = lane / LPF, L = lane % LPF, wv = threadIdx.x >> 6;
    const int cnt = jd.g.q + (L < jd.g.rem ? 1 : 0);
    const int per = jd.g.q + (jd.g.rem > 0 ? 1 : 0);
    const int nb = (per + UNROLL - 1) / UNROLL;
    const int64_t nsteps = (int64_t)gridDim.x * (WG / 64);
    uint32_t acc = 0;
    for (int64_t t = (int64_t)blockIdx.x * (WG / 64) + wv; t * G < jd.F; t += nsteps) {
        const int64_t j = t * G + grp;
        const bool ok = j < jd.F;
        const uint4* p = ok ? jd.keys + j * jd.g.row_units + L : jd.pad;
        const int stride = ok ? LPF : 0;
        for (int b = 0; b < nb; ++b) {
            uint4 u[UNROLL];
            load_batch<UNROLL>(u, p, stride, b, nb, ok ? cnt : 0, jd.pad);
#pragma unroll
            for (int k = 0; k < UNROLL; ++k) acc ^= u[k].x ^ u[k].y ^ u[k].z ^ u[k].w;
        }
    }
#pragma unroll
    for (int o = 32; o; o >>= 1) acc ^= __shfl_xor(acc, o);
    if (lane == 0) s_acc[wv] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t a = 0;
        for (int w = 0; w < WG / 64; ++w) a ^= s_acc[w];
        sink[blockIdx.x] = a;
    }
}

static const void* probe_kernel(int wg, int unroll, int lanes) {
    if (lanes == 16) {
        if (wg == 512 && unroll == 8) return (const void*)k_probe<512, 8, 16>;
        if (wg == 512 && unroll == 10) return (const void*)k_probe<512, 10, 16>;
        if (wg == 512 && unroll == 6) return (const void*)k_probe<512, 6, 16>;
        if (wg == 512 && unroll == 4) return (const void*)k_probe<512, 4, 16>;
        if (wg == 1024 && unroll == 8) return (const void*)k_probe<1024, 8, 16>;
        if (wg == 1024 && unroll == 4) return (const void*)k_probe<1024, 4, 16>;
        if (wg == 256 && unroll == 8) return (const void*)k_probe<256, 8, 16>;
    }
    if (lanes == 32 && wg == 512 && unroll == 8) return (const void*)k_probe<512, 8, 32>;
    if (lanes == 64 && wg == 512 && unroll == 10) return (const void*)k_probe<512, 10, 64>;
    return nullptr;
}

int probe_launch(const ScanPlan& p, int schedule, const JobDev& jd, uint32_t* sink, hipStream_t s) {
    const void* k = probe_kernel(scan_schedule_wg(schedule), scan_schedule_unroll(schedule), scan_schedule_lanes(schedule));
    if (!k) { set_error("no stream probe for this schedule"); return BOOST_E_INVALID; }
    void* args[] = {(void*)&jd, (void*)&sink};
    VJB_HIP(hipLaunchKernel(k, dim3((unsigned)p.grid), dim3((unsigned)p.wg), args, 0, s));
    return BOOST_OK;
}

}  // namespace vjb
