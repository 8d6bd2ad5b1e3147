// Achievable memory rates of the GPU, the denominators of the scoring
// kernel's memory roofline: a streaming read and random 8-byte gathers into a
// table of a chosen size (a table of the map's level-grid size sits in L2 and
// the Infinity Cache; a large one in HBM).  Measurement only; the search never
// calls this.
#include <algorithm>
#include <vector>

#include "bbs_internal.h"

namespace bbs {
namespace {

constexpr int kProbeThreads = 256;

// 32-bit integer mix (the "lowbias32" constants found by C. Wellons'
// hash-prospector search): spreads consecutive counters over the table.
__device__ inline uint32_t mix32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

__global__ void k_probe_fill(uint2 *t, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        t[i] = make_uint2((uint32_t)i, (uint32_t)(i >> 32) ^ 0x9e3779b9u);
}

// Every 16-byte word of the table read once per pass, grid-stride.
__global__ __launch_bounds__(kProbeThreads) void k_probe_stream(const uint4 *__restrict__ t, int64_t n16, int passes,
                                                                uint32_t *out)
{
    uint32_t acc = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int p = 0; p < passes; ++p)
        for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n16; i += stride) {
            const uint4 v = t[i];
            acc ^= v.x ^ v.y ^ v.z ^ v.w;
        }
    out[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

// `per_thread` independent 8-byte loads per thread at hashed positions of a
// power-of-two table (mask = entries - 1), eight in flight.
__global__ __launch_bounds__(kProbeThreads) void k_probe_gather(const uint2 *__restrict__ t, uint32_t mask,
                                                                int per_thread, uint32_t *out)
{
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t acc = 0;
    for (int i = 0; i < per_thread; i += 8) {
        uint2 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = t[mix32(tid * 0x10001u + (uint32_t)(i + u) * 0x9e3779b1u) & mask];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc ^= v[u].x + v[u].y;
    }
    out[tid] = acc;
}

}  // namespace
}  // namespace bbs

extern "C" bbs_status bbs_bandwidth_probe(int32_t kind, int64_t table_bytes, int64_t loads, double *gbs, double *ms)
{
    using namespace bbs;
    if (kind != 0 && kind != 1) return fail(BBS_ERR_INVALID_ARG, "bbs_bandwidth_probe: kind must be 0 or 1");
    if (table_bytes < 4096 || table_bytes > ((int64_t)1 << 36))
        return fail(BBS_ERR_INVALID_ARG, "bbs_bandwidth_probe: table_bytes must be in [4096, 2^36]");
    if (kind == 1 && (loads < 1 || loads > ((int64_t)1 << 34)))
        return fail(BBS_ERR_INVALID_ARG, "bbs_bandwidth_probe: loads must be in [1, 2^34]");
    if (!gbs || !ms) return fail(BBS_ERR_INVALID_ARG, "bbs_bandwidth_probe: outputs are NULL");
    int dev = 0, cus = 0;
    BBS_HIP(hipGetDevice(&dev));
    BBS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    // the gather table is a power of two of 8-byte entries, at most table_bytes
    int64_t entries = (int64_t)1;
    while (entries * 2 * 8 <= table_bytes) entries *= 2;
    const int64_t bytes = kind == 1 ? entries * 8 : table_bytes / 16 * 16;
    const int grid = std::max(1, cus) * 8;
    const int nthreads = grid * kProbeThreads;
    void *t = nullptr, *o = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bbs_status st = BBS_OK;
    auto cleanup = [&]() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (s) (void)hipStreamDestroy(s);
        if (t) (void)hipFree(t);
        if (o) (void)hipFree(o);
    };
    if ((st = alloc_dev(&t, (size_t)bytes)) || (st = alloc_dev(&o, (size_t)nthreads * 4))) {
        cleanup();
        return st;
    }
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        cleanup();
        return hip_fail(e, "bbs_bandwidth_probe: stream / events");
    }
    k_probe_fill<<<grid, kProbeThreads, 0, s>>>(static_cast<uint2 *>(t), bytes / 8);
    // a streaming pass covers the table at least 4 times; a gather run spreads
    // `loads` over every thread in multiples of 8
    const int passes = (int)std::max<int64_t>(4, std::min<int64_t>(64, ((int64_t)1 << 32) / std::max<int64_t>(bytes, 1)));
    const int per_thread = (int)std::max<int64_t>(8, (loads / nthreads + 7) / 8 * 8);
    auto launch = [&]() {
        if (kind == 0)
            k_probe_stream<<<grid, kProbeThreads, 0, s>>>(static_cast<const uint4 *>(t), bytes / 16, passes,
                                                           static_cast<uint32_t *>(o));
        else
            k_probe_gather<<<grid, kProbeThreads, 0, s>>>(static_cast<const uint2 *>(t), (uint32_t)(entries - 1),
                                                           per_thread, static_cast<uint32_t *>(o));
    };
    launch();   // warm-up (and the table's first touch)
    float best = 0.0f;
    for (int rep = 0; rep < 5 && e == hipSuccess; ++rep) {
        e = hipEventRecord(e0, s);
        launch();
        if (e == hipSuccess) e = hipGetLastError();
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float t_ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t_ms, e0, e1);
        if (e == hipSuccess && (rep == 0 || t_ms < best)) best = t_ms;
    }
    if (e != hipSuccess) {
        cleanup();
        return hip_fail(e, "bbs_bandwidth_probe: run");
    }
    const double useful = kind == 0 ? (double)bytes * passes : (double)nthreads * per_thread * 8.0;
    *ms = best;
    *gbs = best > 0.0f ? useful / (best * 1e-3) / 1e9 : 0.0;
    cleanup();
    return BBS_OK;
}
