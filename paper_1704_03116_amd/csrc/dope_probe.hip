// LDS bandwidth probe: the peak against which the block solver's LDS traffic is put.  Every workgroup fills a
// 16 KiB LDS buffer and then streams 128-bit reads over it (consecutive lanes read consecutive 16-byte words, so
// no bank conflicts), folding the values into registers that feed one guarded store; the rate is the bytes read
// over the launch's event-timed duration with every CU full (eight 256-thread workgroups per CU).
#include "../../include/dope.h"

#include <hip/hip_runtime.h>

namespace {

constexpr int PROBE_NT = 256;
constexpr int PROBE_WORDS = 1024;        // uint4 words: 16 KiB per workgroup
constexpr int PROBE_UNROLL = 16;
constexpr int PROBE_WG_PER_CU = 8;
constexpr int PROBE_CUS = 256;

__global__ __launch_bounds__(PROBE_NT) void k_lds_read(int32_t reps, uint32_t *sink) {
    __shared__ uint4 buf[PROBE_WORDS];
    const int tid = threadIdx.x;
    for (int i = tid; i < PROBE_WORDS; i += PROBE_NT)
        buf[i] = make_uint4(uint32_t(i), uint32_t(i) * 3u, uint32_t(i) * 5u, uint32_t(i) * 7u + blockIdx.x);
    __syncthreads();
    uint32_t a = 0, b = 0, c = 0, d = 0;
    int base = tid;
    for (int r = 0; r < reps; ++r) {
#pragma unroll
        for (int j = 0; j < PROBE_UNROLL; ++j) {
            const uint4 v = buf[(base + j * (PROBE_WORDS / PROBE_UNROLL)) & (PROBE_WORDS - 1)];   // 16 distinct words
            a ^= v.x;
            b += v.y;
            c ^= v.z;
            d += v.w;
        }
        base = (base + 17) & (PROBE_WORDS - 1);   // keeps the addresses changing across repetitions
    }
    const uint32_t h = a ^ (b * 0x9e3779b9u) ^ (c * 0x85ebca6bu) ^ (d * 0xc2b2ae35u);
    if (h == 0x2545f491u) sink[blockIdx.x * PROBE_NT + tid] = h;   // practically never taken: keeps the reads live
}

}  // namespace

extern "C" dope_status dope_measure_lds_bandwidth(void *stream, int32_t reps, double *bytes_per_s) {
    if (!bytes_per_s || reps <= 0) return DOPE_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int grid = PROBE_CUS * PROBE_WG_PER_CU;
    uint32_t *sink = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    dope_status st = DOPE_OK;
    if (hipMalloc(&sink, size_t(grid) * PROBE_NT * sizeof(uint32_t)) != hipSuccess) {
        (void)hipGetLastError();
        return DOPE_ENOMEM;
    }
    double best = 0.0;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        st = DOPE_EDEVICE;
    } else {
        for (int trial = 0; trial < 4 && st == DOPE_OK; ++trial) {
            hipLaunchKernelGGL(k_lds_read, dim3(grid), dim3(PROBE_NT), 0, s, reps, sink);   // trial 0: warm-up
            if (hipEventRecord(e0, s) != hipSuccess) { st = DOPE_EDEVICE; break; }
            hipLaunchKernelGGL(k_lds_read, dim3(grid), dim3(PROBE_NT), 0, s, reps, sink);
            if (hipGetLastError() != hipSuccess || hipEventRecord(e1, s) != hipSuccess ||
                hipEventSynchronize(e1) != hipSuccess) { st = DOPE_EDEVICE; break; }
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess || ms <= 0.f) { st = DOPE_EDEVICE; break; }
            const double bytes = double(grid) * PROBE_NT * double(reps) * PROBE_UNROLL * 16.0;
            const double rate = bytes / (double(ms) * 1e-3);
            if (trial > 0 && rate > best) best = rate;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(sink);
    (void)hipGetLastError();
    if (st == DOPE_OK) *bytes_per_s = best;
    return st;
}
