// Internal declarations of libbbs (not part of the C ABI).
//
// Voxel map layout.  Level l of the map is the dilated voxel set D_l of
// Sec. III-C, stored as an open-addressing hash table (linear probing, as in
// the paper) whose entries are bricks: brick B covers voxels 4B .. 4B+4 on
// each axis (5 x 5 x 5 voxels, overlapping its +x/+y/+z neighbours by one
// voxel) and holds their occupancy as a 125-bit mask.  Membership of a voxel
// is therefore unchanged, but every 2 x 2 x 2 block w + {0,1}^3 with
// B = floor(w / 4) lies inside one brick, so the eight translational siblings
// of a node (which share a rotation, Sec. III-D) are answered by one probe.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "bbs.h"

namespace bbs {

constexpr int kMaxLevels = BBS_MAX_LEVELS;
constexpr int32_t kVoxelLimit = 1 << 20;   // |voxel coordinate| < 2^20
constexpr int32_t kBrickBias = 1 << 18;    // brick coordinates are in [-2^18, 2^18)
constexpr uint32_t kEmptyLo = 0xFFFFFFFFu; // empty slot: key = all ones
constexpr uint32_t kEmptyHi = 0xFFFFFFFFu;
constexpr int32_t kTransLimit = 1 << 14;   // |translation cell index| bound (int16 node fields)

// Build-time hash slot: 32 bytes.  head = (key lo, key hi, unused, unused),
// bits = occupancy of the brick's 5^3 voxels, bit (dz * 5 + dy) * 5 + dx.
struct alignas(32) Slot {
    uint4 head;
    uint4 bits;
};

// A level of the finished map: keys and occupancy masks in separate arrays
// (structure of arrays), so the key array that every probe walks stays
// small and cache resident; a mask is read only when its key matches.
//
// Where the level's brick bounding box is small enough (at most a few times
// the hash capacity, at most 4096 bricks along x and y), the masks are also
// laid out as a dense row-major grid of columns over that box (x fastest),
// which the scoring kernel reads instead: one 8-byte load per lookup, no key
// compare and no probe chain.  A column is a brick's x-y extent at a single
// voxel z: entry (x brick, y brick, z voxel) holds the brick's bits of the
// z-slabs z and z + 1 (50 bits, bit 25 dz + 5 dy + dx), so the eight
// translational siblings of any voxel sit in one 32-bit window of one
// entry.  Absent bricks hold zero columns.  The grid has one more layer of
// (empty) entries past the box maximum on each axis: a lookup clamps each
// coordinate into it, so every point outside the box lands on an empty entry
// without a bounds branch.
struct LevelView {
    const uint2 *keys;   // (key lo, key hi); empty = all ones
    const uint4 *bits;   // occupancy of the brick in the same slot
    const uint2 *dense;  // dense column grid over the bounding box, or NULL
    uint32_t cap_mask;   // capacity - 1 (power of two)
    int32_t bmin[3];     // brick-coordinate bounding box of the level
    int32_t bmax[3];
    int32_t nx, ny;      // dense grid: bricks along x and y (border layer included)
};

// Index of the column at brick (rx, ry) and voxel rz (relative to the
// bounding box minimum) in the dense grid.
__host__ __device__ inline uint32_t dense_index(uint32_t rx, uint32_t ry, uint32_t rz, int32_t nx, int32_t ny)
{
    return (rz * (uint32_t)ny + ry) * (uint32_t)nx + rx;
}

struct MapView {
    LevelView lv[kMaxLevels];
};

__host__ __device__ inline uint32_t brick_key_lo(int32_t bx, int32_t by, int32_t bz)
{
    uint64_t k = ((uint64_t)(uint32_t)(bx + kBrickBias) << 38) | ((uint64_t)(uint32_t)(by + kBrickBias) << 19) |
                 (uint64_t)(uint32_t)(bz + kBrickBias);
    return (uint32_t)k;
}
__host__ __device__ inline uint32_t brick_key_hi(int32_t bx, int32_t by, int32_t bz)
{
    uint64_t k = ((uint64_t)(uint32_t)(bx + kBrickBias) << 38) | ((uint64_t)(uint32_t)(by + kBrickBias) << 19) |
                 (uint64_t)(uint32_t)(bz + kBrickBias);
    return (uint32_t)(k >> 32);
}
__host__ __device__ inline uint64_t brick_key(int32_t bx, int32_t by, int32_t bz)
{
    return ((uint64_t)(uint32_t)(bx + kBrickBias) << 38) | ((uint64_t)(uint32_t)(by + kBrickBias) << 19) |
           (uint64_t)(uint32_t)(bz + kBrickBias);
}

// Spatial hash of a brick coordinate: the three-prime XOR hash of Teschner et
// al. followed by a 32-bit avalanche (the finaliser of MurmurHash3, fmix32)
// so that power-of-two tables see mixed low bits.
__host__ __device__ inline uint32_t brick_hash(int32_t bx, int32_t by, int32_t bz)
{
    uint32_t h = ((uint32_t)bx * 73856093u) ^ ((uint32_t)by * 19349663u) ^ ((uint32_t)bz * 83492791u);
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

// Node of the search tree (Sec. III-D), 16 bytes:
//   x = cx | cy << 16, y = cz | i_roll << 16, z = i_pitch | i_yaw << 16, w = level
// Group of translational siblings sharing one rotation, 16 bytes:
//   x = bx | by << 16, y = bz | i_roll << 16, z = i_pitch | i_yaw << 16,
//   w = level | mask << 8; member j = 4 jx + 2 jy + jz (set in mask) is the
//   node (bx + jx, by + jy, bz + jz) at that level and rotation.
__host__ __device__ inline int32_t lo16s(uint32_t v) { return (int32_t)(int16_t)(v & 0xFFFFu); }
__host__ __device__ inline int32_t hi16s(uint32_t v) { return (int32_t)(int16_t)(v >> 16); }
__host__ __device__ inline int32_t hi16u(uint32_t v) { return (int32_t)(v >> 16); }
__host__ __device__ inline int32_t lo16u(uint32_t v) { return (int32_t)(v & 0xFFFFu); }
__host__ __device__ inline uint32_t pack16(int32_t lo, int32_t hi)
{
    return ((uint32_t)lo & 0xFFFFu) | ((uint32_t)hi << 16);
}

// Search grid (Sec. III-B Eq. (2), Sec. III-D), built on the host in double.
struct Grid {
    int32_t levels;
    int32_t translation_only;
    float r;
    double dmax;
    double delta[kMaxLevels];
    int32_t n[3][kMaxLevels];
    double dprime[3][kMaxLevels];
    int32_t a[3][kMaxLevels];
    double wmin[3], wmax[3];
    int32_t lo[3], hi[3];
};

// Small per-search constants passed by value to kernels.
struct SearchConst {
    int32_t levels;
    int32_t K;                     // scan size
    int32_t n[3][kMaxLevels];      // angular cells per axis and level
    int32_t a[3][kMaxLevels];      // divisions from level l to l - 1
    int32_t tlo[3][kMaxLevels];    // valid translation cells per axis and level: [tlo, thi]
    int32_t thi[3][kMaxLevels];
    int32_t trig_off[3][kMaxLevels]; // offset of (axis, level) in the cos/sin table
    int32_t q_count;               // number of queue buckets
    int32_t max_children;          // most children of one node on this grid
    int32_t threshold;             // initial best score (clamped to [0, K + 1])
    int64_t batch;                 // b
    float r;
    float inv_r;
    int32_t r_pow2;                // r is a power of two: p / r == p * (1 / r) exactly
    int32_t score_items;           // scoring work items to aim for (groups x point splits)
    int32_t dedup_levels;          // bit l: runs of level-l groups are scored through the scan's
                                   // histogram of level-l voxels (packed keys fit, counts fit 16 bits)
    int32_t depth_first;           // queue order: 0 score desc then level asc (Alg. 2); 1 level asc
                                   // then score desc (the depth-first order of Alg. 1)
    int32_t n_scores;              // K - threshold + 1: scores a queued node can have
};

// Error reporting (thread-local message).
void set_error(const std::string &msg);
bbs_status fail(bbs_status st, const std::string &msg);
bbs_status hip_fail(hipError_t e, const char *what);
bbs_status alloc_dev(void **p, size_t bytes);

#define BBS_HIP(call)                                        \
    do {                                                     \
        hipError_t e__ = (call);                             \
        if (e__ != hipSuccess) return hip_fail(e__, #call);  \
    } while (0)

}  // namespace bbs

// Host-side map object (the opaque bbs_map of the C ABI).
struct bbs_map {
    int32_t levels;
    float r;
    int32_t dilate_leaf;
    int32_t device;
    uint2 *keys[bbs::kMaxLevels];
    uint4 *bits[bbs::kMaxLevels];
    uint2 *dense[bbs::kMaxLevels];        // dense column grid of the level, or NULL (hash only)
    int64_t dense_n[bbs::kMaxLevels];     // its entries
    int32_t nx[bbs::kMaxLevels], ny[bbs::kMaxLevels];
    uint64_t cap[bbs::kMaxLevels];
    int64_t bricks[bbs::kMaxLevels];
    int64_t voxels[bbs::kMaxLevels];
    int32_t bmin[bbs::kMaxLevels][3];
    int32_t bmax[bbs::kMaxLevels][3];
    // exact rotational bound: level l >= 1 grown by the box margin margin[l]
    // (0: no grown table), held in the same layout by `grown` (levels >= 1)
    int32_t margin[bbs::kMaxLevels];
    bbs_map *grown;
    bbs::MapView view() const;
    bbs::MapView view_exact() const;
};
