// Multi-resolution voxel map on the device (Sec. III-C).
//
// Level l holds D_l: the voxels floor(floor(m / r) / 2^l) of the map points m
// and, for dilated levels, every v - j with j in {0,1}^3 (the set V_add of
// Sec. III-C).  Build steps, all on the device:
//   1. voxelize: level-0 voxel of every point (float32 division, floor);
//   2. dedupe: a set of distinct level-0 voxels (open addressing, CAS);
//   3. per level: shift, dilate and OR each voxel into every brick that
//      covers it (a scratch table sized from the voxel count, grown and
//      rebuilt if it would pass half load);
//   4. compact: re-insert the bricks into a table at load <= 1/2 and record
//      the level's brick bounding box and voxel count.
#include <algorithm>
#include <climits>
#include <cmath>
#include <vector>

#include "bbs_internal.h"

namespace bbs {
namespace {

constexpr int kThreads = 256;
constexpr unsigned long long kEmpty64 = 0xFFFFFFFFFFFFFFFFull;
constexpr int32_t kPackBias = 1 << 20;
constexpr int64_t kDenseRatio = 4;              // dense grid only if its bricks <= 4 x the hash capacity
constexpr int64_t kDenseMax = (int64_t)1 << 28; // and at most 2^28 entries (2 GiB, byte offsets < 2^31)
constexpr int64_t kDenseAxis = 4096;            // and at most 4096 bricks along x and y
constexpr int64_t kDenseZY = (int64_t)1 << 24;  // and z voxels x y bricks <= 2^24 (24-bit index products)
constexpr int32_t kMaxMargin = 8;               // box margin of a grown level table

inline int grid_for(int64_t n, int threads = kThreads, int cap = 8192)
{
    int64_t g = (n + threads - 1) / threads;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

inline uint64_t next_pow2(uint64_t v)
{
    uint64_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

__device__ inline unsigned long long pack_voxel(int32_t x, int32_t y, int32_t z)
{
    return ((unsigned long long)(uint32_t)(x + kPackBias) << 42) |
           ((unsigned long long)(uint32_t)(y + kPackBias) << 21) | (unsigned long long)(uint32_t)(z + kPackBias);
}

__device__ inline void unpack_voxel(unsigned long long k, int32_t &x, int32_t &y, int32_t &z)
{
    x = (int32_t)((k >> 42) & 0x1FFFFF) - kPackBias;
    y = (int32_t)((k >> 21) & 0x1FFFFF) - kPackBias;
    z = (int32_t)(k & 0x1FFFFF) - kPackBias;
}

// 64-bit avalanche of a packed key (the SplitMix64 finaliser).
__device__ inline unsigned long long mix64(unsigned long long x)
{
    x ^= x >> 30;
    x *= 0xbf58476d1ce4e5b9ull;
    x ^= x >> 27;
    x *= 0x94d049bb133111ebull;
    x ^= x >> 31;
    return x;
}

__global__ void k_fill_slots(Slot *s, uint64_t n)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        s[i].head = make_uint4(kEmptyLo, kEmptyHi, 0u, 0u);
        s[i].bits = make_uint4(0u, 0u, 0u, 0u);
    }
}

__global__ void k_fill_u64(unsigned long long *p, uint64_t n, unsigned long long v)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Level-0 voxel of each point: floor(m / r) in float32.  err |= 1 on a
// non-finite coordinate or a voxel outside (-2^20 + 2, 2^20 - 2).
__global__ void k_voxelize(const float *xyz, int64_t n, float r, float inv_r, int r_pow2, unsigned long long *keys,
                           int *err)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int32_t v[3];
        bool ok = true;
        for (int a = 0; a < 3; ++a) {
            float c = xyz[3 * i + a];
            if (!isfinite(c)) ok = false;
            float q = r_pow2 ? c * inv_r : c / r;
            float f = floorf(q);
            if (!(f >= -(float)kVoxelLimit + 2.0f && f < (float)kVoxelLimit - 2.0f)) ok = false;
            v[a] = ok ? (int32_t)f : 0;
        }
        if (!ok) atomicOr(err, 1);
        keys[i] = pack_voxel(v[0], v[1], v[2]);
    }
}

// Distinct level-0 voxels.  err |= 2 if the set runs full.
__global__ void k_dedupe(const unsigned long long *keys, int64_t n, unsigned long long *set, uint64_t cap_mask,
                         unsigned long long *uniq, unsigned long long *n_uniq, int *err)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        unsigned long long key = keys[i];
        uint64_t h = mix64(key) & cap_mask;
        bool done = false;
        for (uint64_t probe = 0; probe <= cap_mask; ++probe) {
            unsigned long long old = atomicCAS(&set[h], kEmpty64, key);
            if (old == kEmpty64) {
                unsigned long long pos = atomicAdd(n_uniq, 1ull);
                uniq[pos] = key;
                done = true;
                break;
            }
            if (old == key) {
                done = true;
                break;
            }
            h = (h + 1) & cap_mask;
        }
        if (!done) atomicOr(err, 2);
    }
}

// Find the slot of brick (bx, by, bz), inserting it if absent.  Returns
// UINT32_MAX if the table has no room left.
__device__ inline uint32_t find_or_insert(Slot *table, uint32_t cap_mask, int32_t bx, int32_t by, int32_t bz,
                                          unsigned long long *n_bricks)
{
    unsigned long long key = brick_key(bx, by, bz);
    uint32_t h = brick_hash(bx, by, bz) & cap_mask;
    for (uint32_t probe = 0; probe <= cap_mask; ++probe) {
        unsigned long long *kp = reinterpret_cast<unsigned long long *>(&table[h].head);
        unsigned long long old = atomicCAS(kp, kEmpty64, key);
        if (old == kEmpty64) {
            atomicAdd(n_bricks, 1ull);
            return h;
        }
        if (old == key) return h;
        h = (h + 1) & cap_mask;
    }
    return 0xFFFFFFFFu;
}

// OR every voxel of D_level into each brick that covers it.  `occ` holds the
// distinct occupied voxels of the level (Occ_level); each marks v - j for
// every j in [jlo, jhi]^3: j in {0} undilated, {0,1}^3 with the dilation of
// Sec. III-C, [-M, 1 + M]^3 for the table grown by the box margin M.  A voxel
// v lies in brick floor(v / 4) and, on each axis where v is a multiple of 4,
// also in the brick below (as its fifth layer).
__global__ void k_insert_bricks(const unsigned long long *occ, int64_t n_occ, int jlo, int jhi, Slot *table,
                                uint32_t cap_mask, unsigned long long *n_bricks, int *err)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_occ; i += (int64_t)gridDim.x * blockDim.x) {
        int32_t w[3];
        unpack_voxel(occ[i], w[0], w[1], w[2]);
        for (int jx = jlo; jx <= jhi; ++jx)
            for (int jy = jlo; jy <= jhi; ++jy)
                for (int jz = jlo; jz <= jhi; ++jz) {
                    int32_t v[3] = {w[0] - jx, w[1] - jy, w[2] - jz};
                    int32_t b0[3];
                    int nb[3];
                    for (int a = 0; a < 3; ++a) {
                        b0[a] = v[a] >> 2;
                        nb[a] = ((v[a] & 3) == 0) ? 2 : 1;
                    }
                    for (int ex = 0; ex < nb[0]; ++ex)
                        for (int ey = 0; ey < nb[1]; ++ey)
                            for (int ez = 0; ez < nb[2]; ++ez) {
                                int32_t bx = b0[0] - ex, by = b0[1] - ey, bz = b0[2] - ez;
                                int dx = v[0] - 4 * bx, dy = v[1] - 4 * by, dz = v[2] - 4 * bz;
                                int bit = (dz * 5 + dy) * 5 + dx;
                                uint32_t s = find_or_insert(table, cap_mask, bx, by, bz, n_bricks);
                                if (s == 0xFFFFFFFFu) {
                                    atomicOr(err, 4);
                                    continue;
                                }
                                uint32_t *words = reinterpret_cast<uint32_t *>(&table[s].bits);
                                atomicOr(&words[bit >> 5], 1u << (bit & 31));
                            }
                }
    }
}

// Occupied voxels one level up: floor(v / 2) of every voxel (its parent).
__global__ void k_parent_keys(const unsigned long long *occ, int64_t n, unsigned long long *out)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int32_t x, y, z;
        unpack_voxel(occ[i], x, y, z);
        out[i] = pack_voxel(x >> 1, y >> 1, z >> 1);
    }
}

__device__ inline int popc4(uint4 a, uint4 m)
{
    return __popc(a.x & m.x) + __popc(a.y & m.y) + __popc(a.z & m.z) + __popc(a.w & m.w);
}

// Move the bricks of a scratch table into the final one; reduce the brick
// bounding box and count each voxel once (in its home brick, dx, dy, dz <= 3).
__global__ void k_compact(const Slot *src, uint64_t src_n, uint2 *dkeys, uint4 *dbits, uint32_t dst_mask, uint4 home,
                          int *bbox, unsigned long long *n_voxels, int *err)
{
    __shared__ int sb[6][kThreads];
    __shared__ unsigned long long sv[kThreads];
    int mn[3] = {INT_MAX, INT_MAX, INT_MAX}, mx[3] = {INT_MIN, INT_MIN, INT_MIN};
    unsigned long long cnt = 0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < src_n; i += (uint64_t)gridDim.x * blockDim.x) {
        uint4 hd = src[i].head;
        if (hd.x == kEmptyLo && hd.y == kEmptyHi) continue;
        unsigned long long key = ((unsigned long long)hd.y << 32) | hd.x;
        int32_t b[3] = {(int32_t)((key >> 38) & 0x7FFFF) - kBrickBias, (int32_t)((key >> 19) & 0x7FFFF) - kBrickBias,
                        (int32_t)(key & 0x7FFFF) - kBrickBias};
        uint32_t h = brick_hash(b[0], b[1], b[2]) & dst_mask;
        bool placed = false;
        for (uint32_t probe = 0; probe <= dst_mask; ++probe) {
            unsigned long long *kp = reinterpret_cast<unsigned long long *>(&dkeys[h]);
            if (atomicCAS(kp, kEmpty64, key) == kEmpty64) {
                dbits[h] = src[i].bits;
                placed = true;
                break;
            }
            h = (h + 1) & dst_mask;
        }
        if (!placed) atomicOr(err, 8);
        for (int a = 0; a < 3; ++a) {
            mn[a] = min(mn[a], b[a]);
            mx[a] = max(mx[a], b[a]);
        }
        cnt += (unsigned long long)popc4(src[i].bits, home);
    }
    for (int a = 0; a < 3; ++a) {
        sb[a][threadIdx.x] = mn[a];
        sb[3 + a][threadIdx.x] = mx[a];
    }
    sv[threadIdx.x] = cnt;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            for (int a = 0; a < 3; ++a) {
                sb[a][threadIdx.x] = min(sb[a][threadIdx.x], sb[a][threadIdx.x + s]);
                sb[3 + a][threadIdx.x] = max(sb[3 + a][threadIdx.x], sb[3 + a][threadIdx.x + s]);
            }
            sv[threadIdx.x] += sv[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int a = 0; a < 3; ++a) {
            atomicMin(&bbox[a], sb[a][0]);
            atomicMax(&bbox[3 + a], sb[3 + a][0]);
        }
        atomicAdd(n_voxels, sv[0]);
    }
}

// Copy every brick of a finished level into its dense column grid (zeroed
// before): column c of a brick is its z-slabs c and c + 1, bits 25 c to
// 25 c + 49 of the 125-bit mask.
__global__ void k_fill_dense(const uint2 *keys, const uint4 *bits, uint64_t cap, uint2 *dense, int32_t bx0, int32_t by0,
                             int32_t bz0, int32_t nx, int32_t ny)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < cap; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint2 kk = keys[i];
        if (kk.x == kEmptyLo && kk.y == kEmptyHi) continue;
        const unsigned long long key = ((unsigned long long)kk.y << 32) | kk.x;
        const int32_t bx = (int32_t)((key >> 38) & 0x7FFFF) - kBrickBias;
        const int32_t by = (int32_t)((key >> 19) & 0x7FFFF) - kBrickBias;
        const int32_t bz = (int32_t)(key & 0x7FFFF) - kBrickBias;
        const uint4 b = bits[i];
        const unsigned __int128 m = ((unsigned __int128)b.w << 96) | ((unsigned __int128)b.z << 64) |
                                    ((unsigned __int128)b.y << 32) | (unsigned __int128)b.x;
        for (int c = 0; c < 4; ++c) {
            const unsigned long long col = (unsigned long long)(m >> (25 * c)) & ((1ull << 50) - 1ull);
            const uint32_t z = 4u * (uint32_t)(bz - bz0) + (uint32_t)c;
            dense[dense_index((uint32_t)(bx - bx0), (uint32_t)(by - by0), z, nx, ny)] =
                make_uint2((uint32_t)col, (uint32_t)(col >> 32));
        }
    }
}

__global__ void k_fill_level(uint2 *keys, uint4 *bits, uint64_t n)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        keys[i] = make_uint2(kEmptyLo, kEmptyHi);
        bits[i] = make_uint4(0u, 0u, 0u, 0u);
    }
}

__global__ void k_dump(LevelView lv, uint64_t n, uint4 home, int32_t *out, uint64_t cap, unsigned long long *count)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        uint2 kk = lv.keys[i];
        if (kk.x == kEmptyLo && kk.y == kEmptyHi) continue;
        unsigned long long key = ((unsigned long long)kk.y << 32) | kk.x;
        int32_t b[3] = {(int32_t)((key >> 38) & 0x7FFFF) - kBrickBias, (int32_t)((key >> 19) & 0x7FFFF) - kBrickBias,
                        (int32_t)(key & 0x7FFFF) - kBrickBias};
        uint4 bb = lv.bits[i];
        uint32_t w[4] = {bb.x, bb.y, bb.z, bb.w};
        for (int dz = 0; dz < 4; ++dz)
            for (int dy = 0; dy < 4; ++dy)
                for (int dx = 0; dx < 4; ++dx) {
                    int bit = (dz * 5 + dy) * 5 + dx;
                    if (!((w[bit >> 5] >> (bit & 31)) & 1u)) continue;
                    unsigned long long pos = atomicAdd(count, 1ull);
                    if (pos < cap) {
                        out[3 * pos + 0] = 4 * b[0] + dx;
                        out[3 * pos + 1] = 4 * b[1] + dy;
                        out[3 * pos + 2] = 4 * b[2] + dz;
                    }
                }
    }
}

__device__ inline bool lookup_bits(const LevelView &lv, int32_t bx, int32_t by, int32_t bz, uint4 &bits)
{
    if (bx < lv.bmin[0] || bx > lv.bmax[0] || by < lv.bmin[1] || by > lv.bmax[1] || bz < lv.bmin[2] ||
        bz > lv.bmax[2])
        return false;
    uint32_t klo = brick_key_lo(bx, by, bz), khi = brick_key_hi(bx, by, bz);
    uint32_t h = brick_hash(bx, by, bz) & lv.cap_mask;
    for (;;) {
        uint2 kk = lv.keys[h];
        if (kk.x == klo && kk.y == khi) {
            bits = lv.bits[h];
            return true;
        }
        if (kk.x == kEmptyLo && kk.y == kEmptyHi) return false;
        h = (h + 1) & lv.cap_mask;
    }
}

// Membership of voxels, read through every brick that covers each voxel; err
// |= 16 if two covering bricks disagree.
__global__ void k_contains(LevelView lv, const int32_t *xyz, int64_t n, uint8_t *out, int *err)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int32_t v[3] = {xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]};
        int32_t b0[3];
        int nb[3];
        for (int a = 0; a < 3; ++a) {
            b0[a] = v[a] >> 2;
            nb[a] = ((v[a] & 3) == 0) ? 2 : 1;
        }
        int home = -1;
        bool mismatch = false;
        for (int ex = 0; ex < nb[0]; ++ex)
            for (int ey = 0; ey < nb[1]; ++ey)
                for (int ez = 0; ez < nb[2]; ++ez) {
                    int32_t bx = b0[0] - ex, by = b0[1] - ey, bz = b0[2] - ez;
                    int bit = ((v[2] - 4 * bz) * 5 + (v[1] - 4 * by)) * 5 + (v[0] - 4 * bx);
                    uint4 bits;
                    int hit = 0;
                    if (lookup_bits(lv, bx, by, bz, bits)) {
                        uint32_t w[4] = {bits.x, bits.y, bits.z, bits.w};
                        hit = (w[bit >> 5] >> (bit & 31)) & 1u;
                    }
                    if (home < 0) home = hit;
                    else if (hit != home) mismatch = true;
                }
        out[i] = (uint8_t)home;
        if (mismatch) atomicOr(err, 16);
    }
}

uint4 home_mask()
{
    uint32_t w[4] = {0, 0, 0, 0};
    for (int dz = 0; dz < 4; ++dz)
        for (int dy = 0; dy < 4; ++dy)
            for (int dx = 0; dx < 4; ++dx) {
                int bit = (dz * 5 + dy) * 5 + dx;
                w[bit >> 5] |= 1u << (bit & 31);
            }
    return make_uint4(w[0], w[1], w[2], w[3]);
}

bool is_pow2_float(float r)
{
    int e = 0;
    float m = std::frexp(r, &e);
    return m == 0.5f;
}

struct DevBuf {
    void *p = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { reset(); }
    void reset()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
    }
    template <class T>
    T *as() const { return static_cast<T *>(p); }
};

struct StreamGuard {
    hipStream_t s = nullptr;
    bool own = false;
    ~StreamGuard()
    {
        if (own && s) (void)hipStreamDestroy(s);
    }
};

}  // namespace

bbs_status alloc_dev(void **p, size_t bytes)
{
    hipError_t e = hipMalloc(p, bytes ? bytes : 16);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(BBS_ERR_OOM, std::string("device allocation of ") + std::to_string(bytes) + " bytes failed");
    }
    return BBS_OK;
}

}  // namespace bbs

using namespace bbs;

bbs::MapView bbs_map::view() const
{
    MapView v;
    for (int l = 0; l < kMaxLevels; ++l) {
        LevelView &lv = v.lv[l];
        lv.keys = l <= levels ? keys[l] : nullptr;
        lv.bits = l <= levels ? bits[l] : nullptr;
        lv.dense = l <= levels ? dense[l] : nullptr;
        lv.nx = l <= levels ? nx[l] : 0;
        lv.ny = l <= levels ? ny[l] : 0;
        lv.cap_mask = l <= levels ? (uint32_t)(cap[l] - 1) : 0u;
        for (int a = 0; a < 3; ++a) {
            lv.bmin[a] = l <= levels ? bmin[l][a] : 1;
            lv.bmax[a] = l <= levels ? bmax[l][a] : 0;
        }
    }
    return v;
}

// The levels of the exact rotational bound: level 0 as built, every level
// l >= 1 with a margin from the grown tables.
bbs::MapView bbs_map::view_exact() const
{
    MapView v = view();
    if (!grown) return v;
    const MapView gv = grown->view();
    for (int l = 1; l <= levels; ++l)
        if (margin[l] > 0) v.lv[l] = gv.lv[l];
    return v;
}

extern "C" void bbs_free_map(bbs_map *map)
{
    if (!map) return;
    for (int l = 0; l < kMaxLevels; ++l) {
        if (map->keys[l]) (void)hipFree(map->keys[l]);
        if (map->bits[l]) (void)hipFree(map->bits[l]);
        if (map->dense[l]) (void)hipFree(map->dense[l]);
    }
    bbs_free_map(map->grown);
    delete map;
}

namespace bbs {
namespace {

// Scratch of one map build (device counters and the level's bounding box).
struct BuildScratch {
    DevBuf dcount, derr, dbbox, dvox;
};

// The brick table (and, where it pays, the dense column grid) of level l of
// m from the level's occupied voxels occ, each marking v - j for j in
// [jlo, jhi]^3.
bbs_status build_level(bbs_map *m, int l, const unsigned long long *occ, int64_t n_occ, int jlo, int jhi,
                       hipStream_t s, BuildScratch &B)
{
    const uint4 home = home_mask();
    int err = 0;
    const int span = jhi - jlo + 1;
    uint64_t tmp_cap = next_pow2(std::max<uint64_t>(1024, 4 * (uint64_t)n_occ * std::max(1, span * span * span / 8)));
    for (;;) {
        DevBuf tmp;
        if (alloc_dev(&tmp.p, tmp_cap * sizeof(Slot))) return BBS_ERR_OOM;
        BBS_HIP(hipMemsetAsync(B.dcount.p, 0, 64, s));
        BBS_HIP(hipMemsetAsync(B.derr.p, 0, 64, s));
        k_fill_slots<<<grid_for((int64_t)tmp_cap), kThreads, 0, s>>>(tmp.as<Slot>(), tmp_cap);
        k_insert_bricks<<<grid_for(n_occ), kThreads, 0, s>>>(occ, n_occ, jlo, jhi, tmp.as<Slot>(),
                                                              (uint32_t)(tmp_cap - 1),
                                                              B.dcount.as<unsigned long long>(), B.derr.as<int>());
        BBS_HIP(hipGetLastError());
        unsigned long long nb = 0;
        BBS_HIP(hipMemcpyAsync(&nb, B.dcount.p, 8, hipMemcpyDeviceToHost, s));
        BBS_HIP(hipMemcpyAsync(&err, B.derr.p, 4, hipMemcpyDeviceToHost, s));
        BBS_HIP(hipStreamSynchronize(s));
        if (err || nb * 2 > tmp_cap) {   // too full: grow and rebuild this level
            if (tmp_cap >= ((uint64_t)1 << 31))
                return fail(BBS_ERR_OOM, "bbs_build_map: brick table would exceed 2^31 slots");
            tmp_cap *= 4;
            continue;
        }
        uint64_t cap = next_pow2(std::max<uint64_t>(16, 2 * nb));
        void *dk = nullptr, *db = nullptr;
        if (alloc_dev(&dk, cap * sizeof(uint2)) || alloc_dev(&db, cap * sizeof(uint4))) {
            if (dk) (void)hipFree(dk);
            return BBS_ERR_OOM;
        }
        m->keys[l] = static_cast<uint2 *>(dk);
        m->bits[l] = static_cast<uint4 *>(db);
        m->cap[l] = cap;
        m->bricks[l] = (int64_t)nb;
        int bbox_init[6] = {INT_MAX, INT_MAX, INT_MAX, INT_MIN, INT_MIN, INT_MIN};
        BBS_HIP(hipMemcpyAsync(B.dbbox.p, bbox_init, sizeof(bbox_init), hipMemcpyHostToDevice, s));
        BBS_HIP(hipMemsetAsync(B.dvox.p, 0, 8, s));
        k_fill_level<<<grid_for((int64_t)cap), kThreads, 0, s>>>(m->keys[l], m->bits[l], cap);
        k_compact<<<grid_for((int64_t)tmp_cap, kThreads, 2048), kThreads, 0, s>>>(
            tmp.as<Slot>(), tmp_cap, m->keys[l], m->bits[l], (uint32_t)(cap - 1), home, B.dbbox.as<int>(),
            B.dvox.as<unsigned long long>(), B.derr.as<int>());
        BBS_HIP(hipGetLastError());
        int bbox[6];
        unsigned long long nv = 0;
        BBS_HIP(hipMemcpyAsync(bbox, B.dbbox.p, sizeof(bbox), hipMemcpyDeviceToHost, s));
        BBS_HIP(hipMemcpyAsync(&nv, B.dvox.p, 8, hipMemcpyDeviceToHost, s));
        BBS_HIP(hipMemcpyAsync(&err, B.derr.p, 4, hipMemcpyDeviceToHost, s));
        BBS_HIP(hipStreamSynchronize(s));
        if (err) return fail(BBS_ERR_INTERNAL, "bbs_build_map: brick compaction failed");
        for (int a = 0; a < 3; ++a) {
            m->bmin[l][a] = bbox[a];
            m->bmax[l][a] = bbox[3 + a];
        }
        m->voxels[l] = (int64_t)nv;
        // dense column grid when the bounding box holds at most kDenseRatio x
        // the hash capacity in bricks and the index products stay within 24
        // bits; one extra layer of empty entries past the box maximum on
        // every axis is where the scoring clamps points outside the box
        const int64_t n3[3] = {(int64_t)bbox[3] - bbox[0] + 2, (int64_t)bbox[4] - bbox[1] + 2,
                               4 * ((int64_t)bbox[5] - bbox[2] + 1) + 1};
        const int64_t dn = n3[0] * n3[1] * n3[2];
        const int64_t box_bricks = n3[0] * n3[1] * ((int64_t)bbox[5] - bbox[2] + 2);
        const bool axes_ok = n3[0] <= kDenseAxis && n3[1] <= kDenseAxis && n3[2] * n3[1] <= kDenseZY;
        if (axes_ok && box_bricks <= kDenseRatio * (int64_t)cap && dn <= kDenseMax) {
            void *dd = nullptr;
            if (alloc_dev(&dd, (size_t)dn * sizeof(uint2))) return BBS_ERR_OOM;
            m->dense[l] = static_cast<uint2 *>(dd);
            m->dense_n[l] = dn;
            m->nx[l] = (int32_t)n3[0];
            m->ny[l] = (int32_t)n3[1];
            BBS_HIP(hipMemsetAsync(dd, 0, (size_t)dn * sizeof(uint2), s));
            k_fill_dense<<<grid_for((int64_t)cap), kThreads, 0, s>>>(m->keys[l], m->bits[l], cap, m->dense[l],
                                                                     bbox[0], bbox[1], bbox[2], m->nx[l], m->ny[l]);
            BBS_HIP(hipGetLastError());
            BBS_HIP(hipStreamSynchronize(s));
        }
        return BBS_OK;
    }
}

}  // namespace
}  // namespace bbs

extern "C" bbs_status bbs_build_map_margins(const float *xyz, int64_t n, int32_t xyz_on_device, float min_res,
                                            int32_t levels, int32_t dilate_leaf, const int32_t *margins, void *stream,
                                            bbs_map **out)
{
    if (!out) return fail(BBS_ERR_INVALID_ARG, "bbs_build_map: out is NULL");
    *out = nullptr;
    if (!xyz) return fail(BBS_ERR_INVALID_ARG, "bbs_build_map: xyz is NULL");
    if (n < 1) return fail(BBS_ERR_INVALID_ARG, "bbs_build_map: n must be >= 1");
    if (n > ((int64_t)1 << 31)) return fail(BBS_ERR_INVALID_ARG, "bbs_build_map: n must be <= 2^31");
    if (!(min_res > 0.0f) || !std::isfinite(min_res))
        return fail(BBS_ERR_INVALID_ARG, "bbs_build_map: min_res must be finite and > 0");
    if (levels < 0 || levels >= kMaxLevels) return fail(BBS_ERR_INVALID_ARG, "bbs_build_map: levels must be in [0, 15]");
    bool any_margin = false;
    if (margins)
        for (int l = 1; l <= levels; ++l) {
            if (margins[l] < 0 || margins[l] > kMaxMargin)
                return fail(BBS_ERR_INVALID_ARG, "bbs_build_map_margins: margins must be in [0, 8]");
            any_margin = any_margin || margins[l] > 0;
        }

    StreamGuard sg;
    sg.s = static_cast<hipStream_t>(stream);
    if (!sg.s) {
        BBS_HIP(hipStreamCreateWithFlags(&sg.s, hipStreamNonBlocking));
        sg.own = true;
    }
    hipStream_t s = sg.s;

    DevBuf dxyz, dkeys, dset, duniq;
    BuildScratch B;
    DevBuf &dcount = B.dcount, &derr = B.derr, &dbbox = B.dbbox, &dvox = B.dvox;
    const float *pts = xyz;
    if (!xyz_on_device) {
        if (alloc_dev(&dxyz.p, (size_t)n * 3 * sizeof(float))) return BBS_ERR_OOM;
        BBS_HIP(hipMemcpyAsync(dxyz.p, xyz, (size_t)n * 3 * sizeof(float), hipMemcpyHostToDevice, s));
        pts = dxyz.as<float>();
    }
    uint64_t set_cap = next_pow2((uint64_t)n * 2);
    if (alloc_dev(&dkeys.p, (size_t)n * 8) || alloc_dev(&dset.p, set_cap * 8) || alloc_dev(&duniq.p, (size_t)n * 8) ||
        alloc_dev(&dcount.p, 64) || alloc_dev(&derr.p, 64) || alloc_dev(&dbbox.p, 64) || alloc_dev(&dvox.p, 64))
        return BBS_ERR_OOM;
    BBS_HIP(hipMemsetAsync(dcount.p, 0, 64, s));
    BBS_HIP(hipMemsetAsync(derr.p, 0, 64, s));
    bool pow2 = is_pow2_float(min_res);
    float inv_r = 1.0f / min_res;
    k_voxelize<<<grid_for(n), kThreads, 0, s>>>(pts, n, min_res, inv_r, pow2 ? 1 : 0, dkeys.as<unsigned long long>(),
                                                 derr.as<int>());
    k_fill_u64<<<grid_for((int64_t)set_cap), kThreads, 0, s>>>(dset.as<unsigned long long>(), set_cap, kEmpty64);
    k_dedupe<<<grid_for(n), kThreads, 0, s>>>(dkeys.as<unsigned long long>(), n, dset.as<unsigned long long>(),
                                               set_cap - 1, duniq.as<unsigned long long>(),
                                               dcount.as<unsigned long long>(), derr.as<int>());
    BBS_HIP(hipGetLastError());
    unsigned long long n_uniq = 0;
    int err = 0;
    BBS_HIP(hipMemcpyAsync(&n_uniq, dcount.p, 8, hipMemcpyDeviceToHost, s));
    BBS_HIP(hipMemcpyAsync(&err, derr.p, 4, hipMemcpyDeviceToHost, s));
    BBS_HIP(hipStreamSynchronize(s));
    if (err & 1)
        return fail(BBS_ERR_INVALID_ARG,
                    "bbs_build_map: a map point is not finite or its voxel is outside [-2^20 + 2, 2^20 - 2)");
    if (err) return fail(BBS_ERR_INTERNAL, "bbs_build_map: voxel set overflow");
    dxyz.reset();

    bbs_map *m = new bbs_map();
    m->levels = levels;
    m->r = min_res;
    m->dilate_leaf = dilate_leaf ? 1 : 0;
    (void)hipGetDevice(&m->device);
    if (any_margin) {
        m->grown = new bbs_map();
        m->grown->levels = levels;
        m->grown->r = min_res;
        m->grown->dilate_leaf = m->dilate_leaf;
        m->grown->device = m->device;
        for (int l = 1; l <= levels; ++l) m->margin[l] = margins[l];
    }

    // Occ_0 is in duniq; Occ_{l+1} = distinct parents of Occ_l (floor division
    // nests), so every level inserts only its own distinct voxels
    DevBuf docc2;
    if (alloc_dev(&docc2.p, (size_t)n_uniq * 8)) {
        bbs_free_map(m);
        return BBS_ERR_OOM;
    }
    unsigned long long *occ = duniq.as<unsigned long long>(), *occ_next = docc2.as<unsigned long long>();
    int64_t n_occ = (int64_t)n_uniq;
    for (int l = 0; l <= levels; ++l) {
        if (l > 0) {
            // occ_next = distinct parents of occ
            k_parent_keys<<<grid_for(n_occ), kThreads, 0, s>>>(occ, n_occ, dkeys.as<unsigned long long>());
            const uint64_t pcap = next_pow2((uint64_t)n_occ * 2);
            k_fill_u64<<<grid_for((int64_t)pcap), kThreads, 0, s>>>(dset.as<unsigned long long>(), pcap, kEmpty64);
            BBS_HIP(hipMemsetAsync(dcount.p, 0, 64, s));
            k_dedupe<<<grid_for(n_occ), kThreads, 0, s>>>(dkeys.as<unsigned long long>(), n_occ,
                                                           dset.as<unsigned long long>(), pcap - 1, occ_next,
                                                           dcount.as<unsigned long long>(), derr.as<int>());
            BBS_HIP(hipGetLastError());
            unsigned long long n_next = 0;
            BBS_HIP(hipMemcpyAsync(&n_next, dcount.p, 8, hipMemcpyDeviceToHost, s));
            BBS_HIP(hipMemcpyAsync(&err, derr.p, 4, hipMemcpyDeviceToHost, s));
            BBS_HIP(hipStreamSynchronize(s));
            if (err) {
                bbs_free_map(m);
                return fail(BBS_ERR_INTERNAL, "bbs_build_map: voxel set overflow");
            }
            std::swap(occ, occ_next);
            n_occ = (int64_t)n_next;
        }
        const int jhi = (l > 0 || dilate_leaf) ? 1 : 0;
        bbs_status st = build_level(m, l, occ, n_occ, 0, jhi, s, B);
        if (st == BBS_OK && l > 0 && m->margin[l] > 0)
            st = build_level(m->grown, l, occ, n_occ, -m->margin[l], 1 + m->margin[l], s, B);
        if (st) {
            bbs_free_map(m);
            return st;
        }
    }
    *out = m;
    return BBS_OK;
}

extern "C" bbs_status bbs_build_map(const float *xyz, int64_t n, int32_t xyz_on_device, float min_res, int32_t levels,
                                    int32_t dilate_leaf, void *stream, bbs_map **out)
{
    return bbs_build_map_margins(xyz, n, xyz_on_device, min_res, levels, dilate_leaf, nullptr, stream, out);
}

extern "C" bbs_status bbs_map_layout(const bbs_map *map, int32_t level, int32_t *dense, int64_t *dense_entries)
{
    if (!map) return fail(BBS_ERR_INVALID_ARG, "bbs_map_layout: map is NULL");
    if (level < 0 || level > map->levels) return fail(BBS_ERR_INVALID_ARG, "bbs_map_layout: level out of range");
    if (dense) *dense = map->dense[level] ? 1 : 0;
    if (dense_entries) *dense_entries = map->dense_n[level];
    return BBS_OK;
}

extern "C" bbs_status bbs_map_info(const bbs_map *map, int32_t *levels, float *min_res, int64_t *voxels,
                                   int64_t *slots, int64_t *bricks)
{
    if (!map) return fail(BBS_ERR_INVALID_ARG, "bbs_map_info: map is NULL");
    if (levels) *levels = map->levels;
    if (min_res) *min_res = map->r;
    for (int l = 0; l < kMaxLevels; ++l) {
        bool on = l <= map->levels;
        if (voxels) voxels[l] = on ? map->voxels[l] : 0;
        if (slots) slots[l] = on ? (int64_t)map->cap[l] : 0;
        if (bricks) bricks[l] = on ? map->bricks[l] : 0;
    }
    return BBS_OK;
}

extern "C" bbs_status bbs_map_dump_level(const bbs_map *map, int32_t level, int32_t *out_xyz, int64_t cap,
                                         int64_t *count)
{
    if (!map) return fail(BBS_ERR_INVALID_ARG, "bbs_map_dump_level: map is NULL");
    if (level < 0 || level > map->levels) return fail(BBS_ERR_INVALID_ARG, "bbs_map_dump_level: level out of range");
    if (cap < 0 || (cap > 0 && !out_xyz)) return fail(BBS_ERR_INVALID_ARG, "bbs_map_dump_level: bad output buffer");
    hipStream_t s = nullptr;
    BBS_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    StreamGuard sg;
    sg.s = s;
    sg.own = true;
    DevBuf dout, dcnt;
    if (alloc_dev(&dout.p, (size_t)std::max<int64_t>(cap, 1) * 12) || alloc_dev(&dcnt.p, 8)) return BBS_ERR_OOM;
    BBS_HIP(hipMemsetAsync(dcnt.p, 0, 8, s));
    MapView v = map->view();
    k_dump<<<grid_for((int64_t)map->cap[level]), kThreads, 0, s>>>(v.lv[level], map->cap[level], home_mask(),
                                                                    dout.as<int32_t>(), (uint64_t)cap,
                                                                    dcnt.as<unsigned long long>());
    BBS_HIP(hipGetLastError());
    unsigned long long c = 0;
    BBS_HIP(hipMemcpyAsync(&c, dcnt.p, 8, hipMemcpyDeviceToHost, s));
    BBS_HIP(hipStreamSynchronize(s));
    int64_t w = std::min<int64_t>((int64_t)c, cap);
    if (w > 0) BBS_HIP(hipMemcpy(out_xyz, dout.p, (size_t)w * 12, hipMemcpyDeviceToHost));
    if (count) *count = (int64_t)c;
    return BBS_OK;
}

extern "C" bbs_status bbs_map_contains(const bbs_map *map, int32_t level, const int32_t *xyz, int64_t n, uint8_t *out)
{
    if (!map) return fail(BBS_ERR_INVALID_ARG, "bbs_map_contains: map is NULL");
    if (level < 0 || level > map->levels) return fail(BBS_ERR_INVALID_ARG, "bbs_map_contains: level out of range");
    if (n < 0 || (n > 0 && (!xyz || !out))) return fail(BBS_ERR_INVALID_ARG, "bbs_map_contains: bad buffers");
    if (n == 0) return BBS_OK;
    for (int64_t i = 0; i < 3 * n; ++i)
        if (xyz[i] <= -kVoxelLimit || xyz[i] >= kVoxelLimit)
            return fail(BBS_ERR_INVALID_ARG, "bbs_map_contains: voxel coordinate outside (-2^20, 2^20)");
    hipStream_t s = nullptr;
    BBS_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    StreamGuard sg;
    sg.s = s;
    sg.own = true;
    DevBuf din, dout, derr;
    if (alloc_dev(&din.p, (size_t)n * 12) || alloc_dev(&dout.p, (size_t)n) || alloc_dev(&derr.p, 4)) return BBS_ERR_OOM;
    BBS_HIP(hipMemcpyAsync(din.p, xyz, (size_t)n * 12, hipMemcpyHostToDevice, s));
    BBS_HIP(hipMemsetAsync(derr.p, 0, 4, s));
    MapView v = map->view();
    k_contains<<<grid_for(n), kThreads, 0, s>>>(v.lv[level], din.as<int32_t>(), n, dout.as<uint8_t>(), derr.as<int>());
    BBS_HIP(hipGetLastError());
    int err = 0;
    BBS_HIP(hipMemcpyAsync(out, dout.p, (size_t)n, hipMemcpyDeviceToHost, s));
    BBS_HIP(hipMemcpyAsync(&err, derr.p, 4, hipMemcpyDeviceToHost, s));
    BBS_HIP(hipStreamSynchronize(s));
    if (err) return fail(BBS_ERR_INTERNAL, "bbs_map_contains: overlapping bricks disagree");
    return BBS_OK;
}
