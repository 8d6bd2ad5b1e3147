// Scan preprocessing before the search: alignment with the measured gravity
// direction (Sec. III-A; the real experiment of Sec. IV-B aligns each scan
// with the IMU's average acceleration) and the voxel-grid filter that brings
// every scan to about 1,000 points (Sec. IV, parameters).
//
// The filter is exact and order free: coordinates are summed as 64-bit
// integers in units of 2^-24 m (|p| < 1024 m) with atomics into a device hash
// table of the occupied voxels, so the mean of a voxel does not depend on the
// order in which its points arrive.  Voxels are emitted in the order of their
// first point (a scan over "this point opened its voxel" flags).
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>

#include "bbs_internal.h"

namespace bbs {
namespace {

constexpr int kPrepThreads = 256;
constexpr int kScanBlock = 1024;                       // points per block of the flag scan
constexpr unsigned long long kEmptyKey = ~0ull;
constexpr double kFix = 16777216.0;                    // 2^24: sum units of 2^-24 m
constexpr float kCoordLimit = 1024.0f;
constexpr float kMinLeaf = 1.0f / 1024.0f;             // 2^-10 m: voxel indices stay in [-2^20, 2^20)
constexpr int32_t kKeyBias = 1 << 20;
constexpr int kBisectSteps = 24;

struct Rot9 {
    float r[9];
};

// (R_i0 x + R_i1 y) + R_i2 z per output coordinate, float32, no contraction.
__global__ void k_gravity(const float *__restrict__ in, int64_t n, Rot9 R, float *__restrict__ out)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float x = in[3 * i], y = in[3 * i + 1], z = in[3 * i + 2];
        for (int a = 0; a < 3; ++a) {
            const float u = __fmul_rn(R.r[3 * a], x);
            const float v = __fmul_rn(R.r[3 * a + 1], y);
            const float w = __fmul_rn(R.r[3 * a + 2], z);
            out[3 * i + a] = __fadd_rn(__fadd_rn(u, v), w);
        }
    }
}

// Per-axis minimum and maximum (as order-preserving integer images of the
// floats) and a flag for coordinates that are not finite or reach 1024 m.
__device__ inline int32_t ord_of(float f)
{
    const int32_t b = __float_as_int(f);
    return b >= 0 ? b : (int32_t)(b ^ 0x7FFFFFFF);
}

__global__ void k_bounds(const float *__restrict__ p, int64_t n, int32_t *mm, int32_t *bad)
{
    int32_t lo[3] = {INT_MAX, INT_MAX, INT_MAX}, hi[3] = {INT_MIN, INT_MIN, INT_MIN};
    int b = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        for (int a = 0; a < 3; ++a) {
            const float v = p[3 * i + a];
            if (!(fabsf(v) < kCoordLimit)) b = 1;
            const int32_t o = ord_of(v);
            lo[a] = min(lo[a], o);
            hi[a] = max(hi[a], o);
        }
    for (int a = 0; a < 3; ++a) {
        for (int off = 32; off > 0; off >>= 1) {
            lo[a] = min(lo[a], __shfl_xor(lo[a], off));
            hi[a] = max(hi[a], __shfl_xor(hi[a], off));
        }
    }
    b = __ballot(b) != 0ull;
    if ((threadIdx.x & 63) == 0) {
        for (int a = 0; a < 3; ++a) {
            atomicMin(&mm[a], lo[a]);
            atomicMax(&mm[3 + a], hi[a]);
        }
        if (b) atomicOr(bad, 1);
    }
}

__device__ inline uint64_t mix64(uint64_t x)
{
    x ^= x >> 31;
    x *= 0x7fb5d329728ea185ull;
    x ^= x >> 27;
    x *= 0x81dadef4bc2dd44dull;
    x ^= x >> 33;
    return x;
}

// The voxel of a point, packed: 21 bits per axis, index + 2^20.
__device__ inline uint64_t voxel_key(const float *p, int64_t i, float leaf)
{
    uint64_t k = 0;
    for (int a = 0; a < 3; ++a) {
        const int32_t v = (int32_t)floorf(__fdiv_rn(p[3 * i + a], leaf));
        k = (k << 21) | (uint64_t)(uint32_t)(v + kKeyBias);
    }
    return k;
}

// Slot of a voxel key in the table (open addressing, linear probing); *fresh
// is set when this call claimed an empty slot.
__device__ inline uint32_t insert_key(unsigned long long *keys, uint32_t mask, uint64_t key, bool *fresh)
{
    uint32_t h = (uint32_t)mix64(key) & mask;
    for (;;) {
        const unsigned long long old = atomicCAS(&keys[h], kEmptyKey, (unsigned long long)key);
        if (old == kEmptyKey) {
            *fresh = true;
            return h;
        }
        if (old == key) {
            *fresh = false;
            return h;
        }
        h = (h + 1) & mask;
    }
}

__global__ void k_fill_keys(unsigned long long *keys, int32_t *first, int32_t *cnt, long long *sums, int64_t cap)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cap; i += (int64_t)gridDim.x * blockDim.x) {
        keys[i] = kEmptyKey;
        if (first) {
            first[i] = INT_MAX;
            cnt[i] = 0;
            sums[3 * i] = sums[3 * i + 1] = sums[3 * i + 2] = 0;
        }
    }
}

// Occupied voxels only (the leaf search): one count per claimed slot.
__global__ void k_vox_count(const float *__restrict__ p, int64_t n, float leaf, unsigned long long *keys,
                            uint32_t mask, int32_t *count)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        bool fresh;
        insert_key(keys, mask, voxel_key(p, i, leaf), &fresh);
        if (fresh) atomicAdd(count, 1);
    }
}

// Every point into its voxel: first point index, point count and the three
// fixed-point coordinate sums.
__global__ void k_vox_insert(const float *__restrict__ p, int64_t n, float leaf, unsigned long long *keys,
                             uint32_t mask, int32_t *first, int32_t *cnt, long long *sums, int32_t *slot_of)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        bool fresh;
        const uint32_t s = insert_key(keys, mask, voxel_key(p, i, leaf), &fresh);
        slot_of[i] = (int32_t)s;
        atomicMin(&first[s], (int32_t)i);
        atomicAdd(&cnt[s], 1);
        for (int a = 0; a < 3; ++a) {
            const long long f = __double2ll_rn((double)p[3 * i + a] * kFix);
            atomicAdd(reinterpret_cast<unsigned long long *>(&sums[3 * s + a]), (unsigned long long)f);
        }
    }
}

// Block-local inclusive scan of "point i opened its voxel" (one block of
// kScanBlock points), and the block totals.
__global__ __launch_bounds__(kScanBlock) void k_open_scan(const int32_t *slot_of, const int32_t *first, int64_t n,
                                                           int32_t *local, int32_t *btot)
{
    __shared__ int32_t wsum[kScanBlock / 64];
    const int64_t i = blockIdx.x * (int64_t)kScanBlock + threadIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int v = (i < n && first[slot_of[i]] == (int32_t)i) ? 1 : 0;
    // inclusive scan in the wave (shuffles), then over the waves
    for (int off = 1; off < 64; off <<= 1) {
        const int u = __shfl_up(v, off);
        if (lane >= off) v += u;
    }
    if (lane == 63) wsum[wave] = v;
    __syncthreads();
    int add = 0;
    for (int w = 0; w < wave; ++w) add += wsum[w];
    v += add;
    if (i < n) local[i] = v;
    if (threadIdx.x == kScanBlock - 1) btot[blockIdx.x] = v;
}

// Exclusive prefix of the block totals (one workgroup, any number of blocks);
// btot[nb] receives the grand total.
__global__ __launch_bounds__(kScanBlock) void k_block_prefix(int32_t *btot, int64_t nb)
{
    __shared__ int32_t wsum[kScanBlock / 64];
    __shared__ int32_t carry;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < nb; c0 += kScanBlock) {
        const int64_t i = c0 + threadIdx.x;
        const int x = i < nb ? btot[i] : 0;
        int v = x;
        for (int off = 1; off < 64; off <<= 1) {
            const int u = __shfl_up(v, off);
            if (lane >= off) v += u;
        }
        if (lane == 63) wsum[wave] = v;
        __syncthreads();
        int add = carry, tot = carry;
        for (int w = 0; w < kScanBlock / 64; ++w) {
            if (w < wave) add += wsum[w];
            tot += wsum[w];
        }
        if (i < nb) btot[i] = add + v - x;
        __syncthreads();
        if (threadIdx.x == 0) carry = tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) btot[nb] = carry;
}

// The voxel of every opening point goes to its output position: mean =
// double(sum) / count / 2^24, rounded once to float.
__global__ void k_emit(const int32_t *slot_of, const int32_t *first, const int32_t *cnt, const long long *sums,
                       const int32_t *local, const int32_t *bpre, int64_t n, float *out)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t s = slot_of[i];
        if (first[s] != (int32_t)i) continue;
        const int64_t pos = (int64_t)bpre[i / kScanBlock] + local[i] - 1;
        for (int a = 0; a < 3; ++a)
            out[3 * pos + a] = (float)(((double)sums[3 * s + a] / (double)cnt[s]) / kFix);
    }
}

// The rotation of the gravity reading (a = g / |g| to +z), entries in double
// as in the closed form, rounded once to float.
Rot9 gravity_rotation(const float g[3])
{
    const double gx = g[0], gy = g[1], gz = g[2];
    const double norm = std::sqrt((gx * gx + gy * gy) + gz * gz);
    const double ax = gx / norm, ay = gy / norm, az = gz / norm;
    double R[9];
    if (1.0 + az < 1e-9) {
        const double h[9] = {1.0, 0.0, 0.0, 0.0, -1.0, 0.0, 0.0, 0.0, -1.0};
        std::copy(h, h + 9, R);
    } else {
        const double k = 1.0 / (1.0 + az);
        R[0] = 1.0 - k * (ax * ax);
        R[1] = -(k * (ax * ay));
        R[2] = -ax;
        R[3] = -(k * (ax * ay));
        R[4] = 1.0 - k * (ay * ay);
        R[5] = -ay;
        R[6] = ax;
        R[7] = ay;
        R[8] = az;
    }
    Rot9 r;
    for (int i = 0; i < 9; ++i) r.r[i] = (float)R[i];
    return r;
}

int grid_of(int64_t n)
{
    return (int)std::max<int64_t>(1, std::min<int64_t>((n + kPrepThreads - 1) / kPrepThreads, 4096));
}

// Device scratch of one call, freed on every return path.
struct Scratch {
    void *p[16] = {};
    int k = 0;
    ~Scratch()
    {
        for (int i = 0; i < k; ++i)
            if (p[i]) (void)hipFree(p[i]);
    }
    template <class T>
    bbs_status get(T **out, size_t count)
    {
        void *q = nullptr;
        const bbs_status st = alloc_dev(&q, std::max<size_t>(count, 1) * sizeof(T));
        if (st) return st;
        p[k++] = q;
        *out = static_cast<T *>(q);
        return BBS_OK;
    }
};

}  // namespace
}  // namespace bbs

extern "C" bbs_status bbs_preprocess_scan(const float *xyz, int64_t n, int32_t on_device,
                                          const bbs_preprocess_options *opt, float *out_xyz, int64_t out_cap,
                                          int64_t *out_n, float *leaf_used, void *stream)
{
    using namespace bbs;
    if (!opt || !out_n) return fail(BBS_ERR_INVALID_ARG, "bbs_preprocess_scan: opt and out_n must not be NULL");
    if (n < 0 || n >= ((int64_t)1 << 31))
        return fail(BBS_ERR_INVALID_ARG, "bbs_preprocess_scan: n must be in [0, 2^31)");
    if (n > 0 && (!xyz || !out_xyz))
        return fail(BBS_ERR_INVALID_ARG, "bbs_preprocess_scan: xyz and out_xyz must not be NULL");
    if (out_cap < 0) return fail(BBS_ERR_INVALID_ARG, "bbs_preprocess_scan: out_cap must not be negative");
    const bool align = opt->gravity[0] != 0.0f || opt->gravity[1] != 0.0f || opt->gravity[2] != 0.0f;
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(opt->gravity[a]))
            return fail(BBS_ERR_INVALID_ARG, "bbs_preprocess_scan: gravity must be finite");
    if (opt->target_points < 0) return fail(BBS_ERR_INVALID_ARG, "bbs_preprocess_scan: target_points must be >= 0");
    if (opt->target_points == 0 && opt->leaf != 0.0f && !(opt->leaf >= kMinLeaf && std::isfinite(opt->leaf)))
        return fail(BBS_ERR_INVALID_ARG, "bbs_preprocess_scan: leaf must be 0 or in [2^-10, inf) m");
    const bool filter = opt->target_points > 0 || opt->leaf != 0.0f;
    if (leaf_used) *leaf_used = 0.0f;
    *out_n = 0;
    if (n == 0) return BBS_OK;
    if (!filter && out_cap < n) {
        *out_n = n;
        return fail(BBS_ERR_INVALID_ARG, "bbs_preprocess_scan: out_cap is below the number of output points");
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    Scratch S;
    bbs_status st;
    const float *src = xyz;
    float *staged = nullptr, *aligned = nullptr, *dout = nullptr;
    if (!on_device) {
        if ((st = S.get(&staged, (size_t)(3 * n)))) return st;
        BBS_HIP(hipMemcpyAsync(staged, xyz, (size_t)(3 * n) * sizeof(float), hipMemcpyHostToDevice, s));
        src = staged;
    }
    if (align) {
        const Rot9 R = gravity_rotation(opt->gravity);
        if (!filter && on_device) aligned = out_xyz;
        else if ((st = S.get(&aligned, (size_t)(3 * n)))) return st;
        k_gravity<<<grid_of(n), kPrepThreads, 0, s>>>(src, n, R, aligned);
        BBS_HIP(hipGetLastError());
        src = aligned;
    }
    int64_t m = n;
    if (!filter) {
        if (on_device) {
            if (!align) BBS_HIP(hipMemcpyAsync(out_xyz, src, (size_t)(3 * n) * sizeof(float),
                                               hipMemcpyDeviceToDevice, s));
        } else {
            BBS_HIP(hipMemcpyAsync(out_xyz, src, (size_t)(3 * n) * sizeof(float), hipMemcpyDeviceToHost, s));
        }
        BBS_HIP(hipStreamSynchronize(s));
        *out_n = n;
        return BBS_OK;
    }
    // bounds: |p| < 1024 m, and the extent for the leaf search
    int32_t *mm = nullptr, *bad = nullptr, *count = nullptr;
    if ((st = S.get(&mm, 8)) || (st = S.get(&count, 1))) return st;
    bad = mm + 6;
    {
        const int32_t init[8] = {INT_MAX, INT_MAX, INT_MAX, INT_MIN, INT_MIN, INT_MIN, 0, 0};
        BBS_HIP(hipMemcpyAsync(mm, init, sizeof(init), hipMemcpyHostToDevice, s));
        k_bounds<<<grid_of(n), kPrepThreads, 0, s>>>(src, n, mm, bad);
        BBS_HIP(hipGetLastError());
    }
    int32_t hm[8];
    BBS_HIP(hipMemcpyAsync(hm, mm, sizeof(hm), hipMemcpyDeviceToHost, s));
    BBS_HIP(hipStreamSynchronize(s));
    if (hm[6]) return fail(BBS_ERR_INVALID_ARG, "bbs_preprocess_scan: coordinates must be finite and below 1024 m");
    // the hash table: a power of two of at least 2 n slots
    int64_t cap = 1024;
    while (cap < 2 * n) cap *= 2;
    unsigned long long *keys = nullptr;
    int32_t *first = nullptr, *cnt = nullptr, *slot_of = nullptr, *local = nullptr, *btot = nullptr;
    long long *sums = nullptr;
    const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
    if ((st = S.get(&keys, (size_t)cap)) || (st = S.get(&first, (size_t)cap)) || (st = S.get(&cnt, (size_t)cap)) ||
        (st = S.get(&sums, (size_t)(3 * cap))) || (st = S.get(&slot_of, (size_t)n)) ||
        (st = S.get(&local, (size_t)n)) || (st = S.get(&btot, (size_t)(nb + 1))))
        return st;
    const uint32_t mask = (uint32_t)(cap - 1);
    float leaf = opt->leaf;
    if (opt->target_points > 0) {
        // 24 bisection steps in float on [2^-10, max(2 extent, 1)]
        auto as_float = [](int32_t o) {
            const int32_t b = o >= 0 ? o : (int32_t)(o ^ 0x7FFFFFFF);
            float f;
            std::memcpy(&f, &b, 4);
            return f;
        };
        float ext = 0.0f;
        for (int a = 0; a < 3; ++a) ext = std::max(ext, as_float(hm[3 + a]) - as_float(hm[a]));
        float lo = kMinLeaf, hi = std::max(2.0f * ext, 1.0f);
        for (int step = 0; step < kBisectSteps; ++step) {
            const float mid = (lo + hi) * 0.5f;
            k_fill_keys<<<grid_of(cap), kPrepThreads, 0, s>>>(keys, nullptr, nullptr, nullptr, cap);
            BBS_HIP(hipMemsetAsync(count, 0, sizeof(int32_t), s));
            k_vox_count<<<grid_of(n), kPrepThreads, 0, s>>>(src, n, mid, keys, mask, count);
            BBS_HIP(hipGetLastError());
            int32_t c = 0;
            BBS_HIP(hipMemcpyAsync(&c, count, sizeof(c), hipMemcpyDeviceToHost, s));
            BBS_HIP(hipStreamSynchronize(s));
            if ((int64_t)c > opt->target_points) lo = mid;
            else hi = mid;
        }
        leaf = hi;
    }
    if (leaf_used) *leaf_used = leaf;
    k_fill_keys<<<grid_of(cap), kPrepThreads, 0, s>>>(keys, first, cnt, sums, cap);
    k_vox_insert<<<grid_of(n), kPrepThreads, 0, s>>>(src, n, leaf, keys, mask, first, cnt, sums, slot_of);
    k_open_scan<<<(unsigned)nb, kScanBlock, 0, s>>>(slot_of, first, n, local, btot);
    k_block_prefix<<<1, kScanBlock, 0, s>>>(btot, nb);
    BBS_HIP(hipGetLastError());
    int32_t total = 0;
    BBS_HIP(hipMemcpyAsync(&total, btot + nb, sizeof(total), hipMemcpyDeviceToHost, s));
    BBS_HIP(hipStreamSynchronize(s));
    m = total;
    *out_n = m;
    if (m > out_cap) return fail(BBS_ERR_INVALID_ARG, "bbs_preprocess_scan: out_cap is below the number of output points");
    if (on_device) dout = out_xyz;
    else if ((st = S.get(&dout, (size_t)(3 * m)))) return st;
    k_emit<<<grid_of(n), kPrepThreads, 0, s>>>(slot_of, first, cnt, sums, local, btot, n, dout);
    BBS_HIP(hipGetLastError());
    if (!on_device)
        BBS_HIP(hipMemcpyAsync(out_xyz, dout, (size_t)(3 * m) * sizeof(float), hipMemcpyDeviceToHost, s));
    BBS_HIP(hipStreamSynchronize(s));
    return BBS_OK;
}
