// Batched best-first branch and bound on the device (Sec. III-D, III-E).
//
// One search iteration ("flush" of Alg. 2) is two kernels on one stream:
//   k_score   the node score of Eq. (12) for every pending node;
//             the last workgroup to finish a tile of 32 groups also sorts
//             that tile's kept children by queue bucket (stable ranks);
//   k_serial  one workgroup: finishes the stable counting sort of the batch
//             into the bucket queue (one bucket per (score, level), FIFO
//             inside a bucket), then pops the queue in (score desc, level
//             asc, FIFO) order, accepts leaves and branches accepted inner
//             nodes until more than b children are pending (or the queue is
//             exhausted), writing them as rotation groups.
// A bucket's FIFO is a chain of 1024-node chunks taken from one pool, so the
// gather reads a bucket 1024 nodes at a time.  The initial set (every
// top-level cell) goes through the same kernels.  Nothing but a done flag
// crosses to the host per iteration.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "bbs_internal.h"

namespace bbs {
namespace {

constexpr int kScoreThreads = 256;
// Resident scoring workgroups per CU: five (93 vector registers a lane).  The
// grid is sized from this, not from the occupancy query alone, which counts
// fewer registers than the hardware allots here (it reported seven workgroups
// where six ran for an earlier version of the kernel); workgroups launched
// beyond the resident number only start once the first ones finish.
constexpr int kScoreWgPerCu = 5;
constexpr int kUnroll = 4;                       // scan points in flight per thread in the scoring loop
constexpr int kScanPad = 1024 * kUnroll;          // scan padding: the largest scoring round (1024 threads)
constexpr int kTileGroups = 32;                  // push tile: 32 groups = 256 node slots
constexpr int kTileSlots = kTileGroups * 8;
constexpr int kSerialThreads = 1024;
constexpr int kChunk = 1024;                     // nodes per queue chunk (= serial block size)
constexpr int kItersPerSync = 8;
constexpr int64_t kDefaultQueueNodes = (int64_t)64 << 20;

struct Bucket {
    int32_t head_chunk, head_off, tail_chunk, tail_fill;   // empty: head_chunk = tail_chunk = -1
};

struct State {
    int32_t best;
    int32_t have_match;
    int32_t match[6];
    int32_t done;
    int32_t error;            // 1: node pool overflow
    int32_t top_q;            // no bucket below this index holds nodes
    int32_t n_groups;         // pending groups of the current batch
    int32_t batch;            // 1: the pending batch is to be scored and pushed
    int32_t q_min, q_max;     // bucket range of the kept children of the batch
    int32_t chunk_top, chunk_cap;
    int32_t pad0;
    int64_t pend_nodes;
    int64_t kept;             // children of the batch with score >= best
    int64_t pushed;           // nodes pushed since the start
    int64_t nodes_expanded, nodes_scored, flushes, leaves_accepted;
    int64_t groups_scored;
    int64_t dive_scored;      // children scored by the seed beam
    int32_t seeded, seed_score;
    int64_t t_push, t_gather; // device real-time ticks (100 MHz) spent in the serial push and gather
    int64_t t_push_prefix, t_push_alloc;   // of t_push: bucket prefix over tiles, chunk allocation
    // the pending batch as scoring items (written by the gather): runs of
    // groups that share a level and rotation (`rgroups`), cut into n_items
    // item descriptors (`items`): histogram items, pairs of groups, or point
    // slices (n_slices per group) of groups scored point by point
    int32_t runs;             // 1: the fields below describe the batch; 0: groups in index order, all direct
    int32_t n_items;
    int32_t n_slices;
    int32_t pad2;
    int64_t dedup_groups;     // groups scored through a histogram, since the start
    int64_t dedup_items;      // histogram items, since the start
    int32_t hist_off;         // bit l: a level-l scan histogram overflowed; later level-l runs go point by point
    int32_t hist_fallbacks;   // histogram items that overflowed and were scored point by point
    int64_t level_groups[kMaxLevels];   // groups scored per level (children batches, since the start)
};

// ---- learned prior: seed beam (not in the paper)
constexpr int kMaxBeam = 64;
constexpr int kBeamThreads = 1024;
constexpr int kBeamSlots = 2048;                 // children (8 slots per group) one beam step may score

struct BeamNode {
    uint4 node;               // packed node (translation, angle indices, level)
    int32_t score, pad;
    double key;               // prior key
};

struct BeamBuf {
    int32_t count, pad[3];
    BeamNode nodes[kMaxBeam];
};

// What the prior key needs of the search grid: the leaf yaw grid, the yaw
// divisions per level, the leaf translation grid and the search box.
struct PriorConst {
    double wmin_yaw, dprime_yaw0;     // leaf yaw cell i has angle wmin + dprime (i + 1/2)
    double r;                         // leaf translation cell i sits at r i
    double tmin[2], tmax[2];          // x and y search intervals
    int32_t n_yaw0;
    int32_t lo[2], hi[2];             // leaf translation cells in the search range
    int32_t a_yaw[kMaxLevels];        // yaw divisions from level l to l - 1
};

// Yaw bin of an angle: 64 bins over [0, 2 pi) after reduction mod 2 pi.
__host__ __device__ inline int prior_yaw_bin(double th)
{
    const double two_pi = 2.0 * 3.14159265358979323846;
    const double tm = th - two_pi * floor(th / two_pi);
    int yb = (int)floor(tm / (two_pi / 64));
    return yb < 0 ? 0 : (yb > 63 ? 63 : yb);
}

// Cell (of 32) of leaf translation index i along x (ax = 0) or y (ax = 1).
__host__ __device__ inline int prior_xy_cell(const PriorConst &P, int ax, int32_t i)
{
    const double x = P.r * (double)i;
    const double lo = P.tmin[ax], hi = P.tmax[ax];
    const int c = hi > lo ? (int)floor(32 * (x - lo) / (hi - lo)) : 0;
    return c < 0 ? 0 : (c > 31 ? 31 : c);
}

// Prior key of a level-l node: the best yaw-bin logit over the leaf yaws
// below it plus the best cell logit over the leaf translations below it.
// The leaf yaw cells below yaw cell c are [c P, (c+1) P - 1] (P: product of
// the yaw divisions of levels 1..l, clipped to the leaf cell count); the
// leaf translation cells below t are [t 2^l, (t+1) 2^l - 1] (clipped to the
// search range).
__host__ __device__ inline double prior_key(const PriorConst &P, const float *prior, int level, int32_t tx, int32_t ty,
                                            int32_t yaw)
{
    int64_t span = 1;
    for (int m = 1; m <= level; ++m) span *= P.a_yaw[m];
    const int64_t y0 = (int64_t)yaw * span;
    int64_t y1 = ((int64_t)yaw + 1) * span - 1;
    if (y1 > P.n_yaw0 - 1) y1 = P.n_yaw0 - 1;
    double ky = -__builtin_huge_val();
    for (int64_t i = y0; i <= y1; ++i) {
        const double v = prior[prior_yaw_bin(P.wmin_yaw + P.dprime_yaw0 * ((double)i + 0.5))];
        if (v > ky) ky = v;
    }
    uint32_t cells[2] = {0u, 0u};
    const int32_t t[2] = {tx, ty};
    for (int ax = 0; ax < 2; ++ax) {
        int64_t i0 = (int64_t)t[ax] * ((int64_t)1 << level), i1 = ((int64_t)t[ax] + 1) * ((int64_t)1 << level) - 1;
        if (i0 < P.lo[ax]) i0 = P.lo[ax];
        if (i1 > P.hi[ax]) i1 = P.hi[ax];
        for (int64_t i = i0; i <= i1; ++i) cells[ax] |= 1u << prior_xy_cell(P, ax, (int32_t)i);
    }
    double kxy = -__builtin_huge_val();
    for (int cx = 0; cx < 32; ++cx) {
        if (!((cells[0] >> cx) & 1u)) continue;
        for (int cy = 0; cy < 32; ++cy) {
            if (!((cells[1] >> cy) & 1u)) continue;
            const double v = prior[64 + cx * 32 + cy];
            if (v > kxy) kxy = v;
        }
    }
    return ky + kxy;
}

inline int grid_for(int64_t n, int threads, int cap)
{
    int64_t g = (n + threads - 1) / threads;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

// ------------------------------------------------------------------ block helpers

// Inclusive scans over the 64 lanes of a wave with DPP lane moves (row
// shifts by 1, 2, 4, 8 inside each row of 16 lanes, then the row-15 and
// row-31 broadcasts to the later rows): six VALU steps, no LDS round trips.
// A lane whose source lies outside its row, or a row left out by the row
// mask, takes the identity.
__device__ inline int wave_scan_add(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);   // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);   // row_bcast:15 to rows 1, 3
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);   // row_bcast:31 to rows 2, 3
    return v;
}

__device__ inline int wave_scan_min(int v)
{
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x111, 0xf, 0xf, false));
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x112, 0xf, 0xf, false));
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x114, 0xf, 0xf, false));
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x118, 0xf, 0xf, false));
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x142, 0xa, 0xf, false));
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x143, 0xc, 0xf, false));
    return v;
}

// Sum over the wave, the same in every lane (all 64 lanes active).
__device__ inline int wave_sum(int v)
{
    return __builtin_amdgcn_readlane(wave_scan_add(v), 63);
}

template <int N>
__device__ inline int block_min_int(int v, int *sm)
{
    v = __builtin_amdgcn_readlane(wave_scan_min(v), 63);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sm[wave] = v;
    __syncthreads();
    int r = sm[0];
    for (int w = 1; w < N / 64; ++w) r = min(r, sm[w]);
    return r;
}

// Inclusive prefix sum over the block; *total receives the block sum.
template <int N>
__device__ inline int block_scan_incl(int v, int *sm, int *total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = wave_scan_add(v);
    __syncthreads();
    if (lane == 63) sm[wave] = v;
    __syncthreads();
    int add = 0, tot = 0;
    for (int w = 0; w < N / 64; ++w) {
        if (w < wave) add += sm[w];
        tot += sm[w];
    }
    *total = tot;
    return v + add;
}

__device__ inline bool leaf_less(const int32_t *a, const int32_t *b)
{
    for (int i = 0; i < 6; ++i)
        if (a[i] != b[i]) return a[i] < b[i];
    return false;
}

__device__ inline void node_unpack(uint4 nd, int32_t t[3], int32_t ang[3], int32_t &level)
{
    t[0] = lo16s(nd.x);
    t[1] = hi16s(nd.x);
    t[2] = lo16s(nd.y);
    ang[0] = hi16u(nd.y);
    ang[1] = lo16u(nd.z);
    ang[2] = hi16u(nd.z);
    level = (int32_t)(nd.w & 0xFF);
}

// ------------------------------------------------------------------ scan set-up

// Scan to structure-of-arrays, and the largest squared range in double
// (evaluated as (x*x + y*y) + z*z).  The square root is taken on the host.
__global__ void k_scan_soa(const float *xyz, int32_t K, float *X, float *Y, float *Z, unsigned long long *max_sq)
{
    __shared__ double sm[256];
    double m = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < K; i += gridDim.x * blockDim.x) {
        float x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
        X[i] = x;
        Y[i] = y;
        Z[i] = z;
        double dx = x, dy = y, dz = z;
        double d = dx * dx + dy * dy + dz * dz;
        if (!(d <= 1.0e300)) d = INFINITY;   // a non-finite coordinate propagates as +inf
        m = fmax(m, d);
    }
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(max_sq, (unsigned long long)__double_as_longlong(sm[0]));
}

// Spatial order of the scan: a counting sort of the points on a 15-bit Morton
// key (32 cells per axis over [-d_max, d_max]).  Neighbouring lanes of the
// scoring kernel then probe neighbouring bricks.  The scores are sums over
// points, so the permutation (and the order inside a cell) changes nothing.
constexpr int kMortonBits = 5;
constexpr int kMortonBins = 1 << (3 * kMortonBits);

__device__ inline uint32_t morton_key(float x, float y, float z, float lo, float inv_cell)
{
    const int cells = 1 << kMortonBits;
    int c[3] = {(int)floorf((x - lo) * inv_cell), (int)floorf((y - lo) * inv_cell), (int)floorf((z - lo) * inv_cell)};
    uint32_t key = 0;
    for (int b = 0; b < kMortonBits; ++b)
        for (int a = 0; a < 3; ++a) {
            int v = min(max(c[a], 0), cells - 1);
            key |= (uint32_t)((v >> b) & 1) << (3 * b + a);
        }
    return key;
}

__global__ void k_morton_hist(const float *X, const float *Y, const float *Z, int32_t K, float lo, float inv_cell,
                              uint32_t *keys, int32_t *hist)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < K; i += gridDim.x * blockDim.x) {
        uint32_t k = morton_key(X[i], Y[i], Z[i], lo, inv_cell);
        keys[i] = k;
        atomicAdd(&hist[k], 1);
    }
}

__global__ __launch_bounds__(1024) void k_morton_offsets(int32_t *hist)
{
    __shared__ int sm[16];
    const int per = kMortonBins / 1024;
    int loc[kMortonBins / 1024];
    int sum = 0;
    for (int u = 0; u < per; ++u) {
        loc[u] = hist[threadIdx.x * per + u];
        sum += loc[u];
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int v = sum;
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(v, o);
        if (lane >= o) v += t;
    }
    if (lane == 63) sm[wave] = v;
    __syncthreads();
    int add = 0;
    for (int w = 0; w < wave; ++w) add += sm[w];
    int run = v + add - sum;
    for (int u = 0; u < per; ++u) {
        hist[threadIdx.x * per + u] = run;
        run += loc[u];
    }
}

__global__ void k_morton_scatter(const float *X, const float *Y, const float *Z, const uint32_t *keys, int32_t K,
                                 int32_t *offsets, float *Xs, float *Ys, float *Zs)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < K; i += gridDim.x * blockDim.x) {
        int pos = atomicAdd(&offsets[keys[i]], 1);
        Xs[pos] = X[i];
        Ys[pos] = Y[i];
        Zs[pos] = Z[i];
    }
}

// Scan padding past the K points up to the next multiple of the largest
// scoring round: a point whose every rotation leaves the map's boxes (one
// coordinate at least 2^22 cells from the origin), so it never counts.
__global__ void k_scan_pad(float *Xs, float *Ys, float *Zs, int32_t K, int32_t kpad, float v)
{
    for (int i = K + blockIdx.x * blockDim.x + threadIdx.x; i < kpad; i += gridDim.x * blockDim.x) {
        Xs[i] = v;
        Ys[i] = v;
        Zs[i] = v;
    }
}

__global__ void k_fill_buckets(Bucket *b, int32_t n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        b[i] = Bucket{-1, 0, -1, 0};
}

// Rotation of node angles (i_roll, i_pitch, i_yaw) at a level, from the
// cos/sin table: R = Rz(yaw) Ry(pitch) Rx(roll), entries formed in double with
// the products evaluated left to right and rounded once to float.
__device__ inline void rotation(const double2 *trig, const SearchConst &C, int level, int ia, int ib, int ig,
                                float R[9])
{
    double2 A = trig[C.trig_off[0][level] + ia];
    double2 B = trig[C.trig_off[1][level] + ib];
    double2 G = trig[C.trig_off[2][level] + ig];
    double ca = A.x, sa = A.y, cb = B.x, sb = B.y, cg = G.x, sg = G.y;
    R[0] = (float)(cg * cb);
    R[1] = (float)(cg * sb * sa - sg * ca);
    R[2] = (float)(cg * sb * ca + sg * sa);
    R[3] = (float)(sg * cb);
    R[4] = (float)(sg * sb * sa + cg * ca);
    R[5] = (float)(sg * sb * ca - cg * sa);
    R[6] = (float)(-sb);
    R[7] = (float)(cb * sa);
    R[8] = (float)(cb * ca);
}

// ------------------------------------------------------------------ scoring (Eq. (12), Sec. III-C)

// Scores the eight translational siblings of each group against D_level.
// For scan point s and the group's rotation R, the level-l voxel of node
// (bx + jx, by + jy, bz + jz) is w + j with w = floor(floor(R s / r) / 2^l) +
// (bx, by, bz) (float32 transform, fixed evaluation order, no contraction).
// The brick floor(w / 4) holds all eight candidate voxels, so one probe per
// point answers the whole group.  A level with a dense mask grid is read with
// one load per point; otherwise the brick is looked up in the hash table.
// Each thread keeps kUnroll points (and their probe chains) in flight.  A group's points are split over several
// workgroups when the batch has few groups; partial counts are added with
// integer atomics into scores zeroed by the producer of the batch.
// Batch header fields written by another workgroup of the same launch are
// read with device-scope loads (no stale first-level cache line).
__device__ inline int32_t ld_agent(const int32_t *p)
{
    return __hip_atomic_load(const_cast<int32_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// a * b + c for a, b < 2^24 (the full-rate 24-bit multiply-add)
__device__ inline uint32_t mad24(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t d;
    asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    return d;
}

// Queue bucket of a (score, level): buckets are popped in index order, so
// the best-first order (Alg. 2; ties: lower level first) is score-major and
// the depth-first order (Alg. 1: deeper level first, then higher score) is
// level-major.  Scores below the threshold are never queued.
__device__ inline int bucket_of(int score, int level, const SearchConst &C)
{
    return C.depth_first ? level * C.n_scores + (C.K - score) : (C.K - score) * (C.levels + 1) + level;
}

__device__ inline int bucket_score(int q, const SearchConst &C)
{
    return C.depth_first ? C.K - q % C.n_scores : C.K - q / (C.levels + 1);
}

__device__ inline int bucket_level(int q, const SearchConst &C)
{
    return C.depth_first ? q / C.n_scores : q % (C.levels + 1);
}

// The tile pass's LDS table of buckets: a key per entry and, per entry, the
// count of each of the four slot waves (a byte each).
constexpr int kRankBits = 9;
constexpr int kRankSlots = 1 << kRankBits;      // twice the slots of a tile
static_assert(kTileSlots / 64 == 4 && kRankSlots >= 2 * kTileSlots, "rank table layout");
struct RankTab {
    int key[kRankSlots];
    uint32_t cnt[kRankSlots];
};

// One tile of 32 groups (256 node slots) of a scored batch: the queue bucket
// of every kept child (score >= best), its rank among the tile's earlier
// children of the same bucket, and the tile's count per bucket.  The kept
// children are listed compactly in slot order (bucket, rank, packed node)
// with their number, since most children of a batch are pruned.  Run by a
// whole workgroup of NT >= 256 threads; thread s < 256 handles slot s.
template <int NT>
__device__ void tile_pass(int t, const uint4 *groups, int32_t *scores, State *st, const SearchConst &C,
                          int n_groups, int best, int32_t *kq, int32_t *krank, uint4 *knode, int32_t *kcnt, int32_t *hist,
                          uint32_t *qmask, RankTab &rt, int *sm)
{
    const int s = threadIdx.x;
    const bool slot = s < kTileSlots;
    const int g = t * kTileGroups + s / 8, j = s & 7;
    int q = -1;
    uint4 child = make_uint4(0u, 0u, 0u, 0u);
    if (slot && g < n_groups) {
        const uint4 G = groups[g];
        const uint32_t mask = (G.w >> 8) & 0xFF;
        if ((mask >> j) & 1u) {
            // read with an atomic at the adds' coherence point (see the scoring
            // hand-off); the zero is opaque so the add is not turned into a load
            int zero;
            asm volatile("v_mov_b32 %0, 0" : "=v"(zero));
            const int sc = __hip_atomic_fetch_add(&scores[8 * (int64_t)g + j], zero, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
            if (sc >= best) {
                q = bucket_of(sc, (int)(G.w & 0xFF), C);
                const int jx = (j >> 2) & 1, jy = (j >> 1) & 1, jz = j & 1;
                child = make_uint4(pack16(lo16s(G.x) + jx, hi16s(G.x) + jy), pack16(lo16s(G.y) + jz, hi16u(G.y)),
                                   G.z, G.w & 0xFFu);
            }
        }
    }
    // The slot's rank among the tile's earlier slots of its bucket, and the
    // bucket's count in the tile, without a pass over all 256 slots.  Within
    // a wave, the lanes of one bucket are found with ballots (a round per
    // distinct bucket of the wave, none for a wave without kept children).
    // The wave's first lane of a bucket enters the bucket into an LDS table
    // (open addressing, twice as many entries as slots) and writes the
    // wave's count there, a byte per wave; a slot then adds the counts of the
    // earlier waves.  The barrier that publishes the table also publishes
    // each wave's bucket range and kept count.
    for (int i = threadIdx.x; i < kRankSlots; i += NT) {
        rt.key[i] = -1;
        rt.cnt[i] = 0u;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int wrank = 0, hslot = 0;
    if (wave < kTileSlots / 64) {
        uint64_t todo = __ballot(q >= 0);
        int lead = 0, wcnt = 0;
        while (todo) {
            const int l = __builtin_ctzll(todo);
            const int q0 = __builtin_amdgcn_readlane(q, l);
            const uint64_t m = __ballot(q == q0);
            if (q == q0) {
                // set bits of m below this lane
                wrank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                wcnt = __popcll(m);
                lead = l;
            }
            todo &= ~m;
        }
        if (q >= 0 && wrank == 0) {
            uint32_t h = ((uint32_t)q * 2654435761u) >> (32 - kRankBits);
            for (;;) {
                const int old = atomicCAS(&rt.key[h], -1, q);
                if (old == -1 || old == q) break;
                h = (h + 1) & (kRankSlots - 1);
            }
            reinterpret_cast<uint8_t *>(rt.cnt)[4 * h + wave] = (uint8_t)wcnt;
            hslot = (int)h;
        }
        hslot = __builtin_amdgcn_ds_bpermute(lead << 2, hslot);
    }
    const int wmin = __builtin_amdgcn_readlane(wave_scan_min(q >= 0 ? q : INT_MAX), 63);
    const int wmaxn = __builtin_amdgcn_readlane(wave_scan_min(q >= 0 ? -q : INT_MAX), 63);
    const int wscan = wave_scan_add(q >= 0 ? 1 : 0);
    if (lane == 63) {
        sm[3 * wave] = wmin;
        sm[3 * wave + 1] = wmaxn;
        sm[3 * wave + 2] = wscan;
    }
    __syncthreads();
    int rank = 0, cnt = 0;
    if (q >= 0) {
        const uint32_t c4 = rt.cnt[hslot];
#pragma unroll
        for (int w = 0; w < kTileSlots / 64; ++w) {
            const int c = (int)((c4 >> (8 * w)) & 0xFFu);
            cnt += c;
            rank += w < wave ? c : 0;
        }
        rank += wrank;
    }
    int qmn = INT_MAX, qmxn = INT_MAX, before = 0, tot = 0;
    for (int w = 0; w < NT / 64; ++w) {
        qmn = min(qmn, sm[3 * w]);
        qmxn = min(qmxn, sm[3 * w + 1]);
        const int c = sm[3 * w + 2];
        before += w < wave ? c : 0;
        tot += c;
    }
    const int qmx = -qmxn;
    const int kin = wscan + before;
    if (q >= 0) {
        const int64_t k = (int64_t)t * kTileSlots + kin - 1;
        kq[k] = q;
        krank[k] = rank;
        knode[k] = child;
    }
    if (q >= 0 && rank == 0) {
        hist[(int64_t)t * C.q_count + q] = cnt;
        atomicOr(&qmask[q >> 5], 1u << (q & 31));
    }
    if (threadIdx.x == 0) kcnt[t] = tot;
    if (threadIdx.x == 0 && tot > 0) {
        atomicMin(&st->q_min, qmn);
        atomicMax(&st->q_max, qmx);
        atomicAdd((unsigned long long *)&st->kept, (unsigned long long)tot);
    }
}

// Histogram of the scan's level-l voxels under one rotation (LDS open
// addressing on the packed voxel, linear probing), then the same table
// compacted in place to its D distinct voxels with their point counts.
constexpr int kHistSlots = 2048;
constexpr int kHistMax = 1536;                   // distinct voxels beyond this: the item scores point by point
constexpr uint32_t kHistEmpty = 0xFFFFFFFFu;
constexpr int kHistBias = 512;                   // packed voxel: 10 bits per axis, v + 512
constexpr int kItemGroups = 64;                  // groups of one run per histogram item

// Item descriptor (int4): x = first entry of rgroups, y = groups, z = kind,
// w = point slice (kind 2).
constexpr int kItemHist = 0;                     // one run's groups through the scan histogram
constexpr int kItemPair = 1;                     // one or two groups, point by point
constexpr int kItemSlice = 2;                    // a point slice of one group

struct HistSmem {
    uint32_t key[kHistSlots];
    uint32_t cnt[kHistSlots / 2];                // two 16-bit counts per word (slot s: half s & 1)
    uint32_t ckey[kHistMax];                     // the distinct voxels, compacted
    uint16_t ccnt[kHistMax];                     // and their point counts
    int n_distinct;
    int full;                                    // more than kHistMax distinct voxels (or a long probe)
    int n_compact;
    int n_tiles;
    int tiles[kItemGroups];                      // tiles this item completed
};

template <int NT>
struct ScoreSmem {
    int red[NT / 64][16];
    RankTab rt;
    int sm[3 * (NT / 64)];
    int s_last;
    int s_next;
};

// The same, with the histogram of the scoring through runs.
template <int NT>
struct ScoreSmemRuns : ScoreSmem<NT> {
    HistSmem h;
};

struct ScoreArgs {
    const uint4 *groups;
    int32_t n_groups_fixed;    // used when st is NULL
    const float *X, *Y, *Z;
    const double2 *trig;
    int32_t *scores;
    int32_t *tile_done;        // NULL: no tile pass
    int32_t *kq, *krank, *hist;  // kept children per tile: bucket, rank; tile x bucket counts
    uint4 *knode;              // kept children per tile: packed node
    int32_t *kcnt;             // kept children per tile: number
    uint32_t *qmask;           // bit q: some tile of the batch holds a child of bucket q
    int32_t *ticket;           // NULL: items round-robin; else [0] next item ticket, [1] workgroups
                               // done (both 0 between launches)
    const int32_t *rgroups;    // the batch's groups by run (with st->runs)
    const int4 *items;         // item descriptors (with st->runs)
    int32_t *gslices;          // per group: point slices done (0 between launches)
};

// A rotated coordinate in level-0 cells, as p / r: RM 0 divides (correctly
// rounded), RM 1 multiplies by 1 / r (exact for a power-of-two r), RM 2 is
// r = 1 (p itself).
template <int RM>
__device__ inline float scale_to_cells(float p, const SearchConst &C)
{
    if (RM == 2) return p;
    if (RM == 1) return p * C.inv_r;
    return p / C.r;
}

// Constants of one group for the dense-grid loop (uniform over the workgroup).
struct DenseGroup {
    float R[9];
    const uint2 *dense;
    uint32_t nx, ny;
    uint32_t lim[3];          // border layer index per axis
    int32_t off[3];           // (group base - 4 box minimum) 2^l per axis
    uint32_t level;
};

// Dense-grid scoring of the points [k_begin, k_end) against NG groups at once:
// each thread keeps KU points in flight and tests every loaded point against
// every group, so the scan is read once for all of them.
//
// Branch-free: every scan and grid load of a round is issued before any
// result is used.  Per axis, w = floor(R s / r) + (group base - 4 box
// minimum) 2^l is the level-0 coordinate of the level-l voxel relative to the
// box (adding a multiple of 2^l commutes with the floor of the shift):
// w >> (l + 2) is the x or y brick and w >> l the z voxel, clamped into the
// grid's empty border layer when outside the box (a negative w is a large
// unsigned value), and bits l, l+1 of w the x or y voxel inside the brick,
// which picks the 32-bit window of the column.  The eight counts of a group
// are bit-sliced into two 64-bit words, members 0..3 of the window bits 0, 5,
// 25, 30 and members 4..7 of bits 1, 6, 26, 31, in fields of at least 5 bits,
// folded every kFold rounds.
template <int RM, int NT, int NG, int KU>
__device__ inline void dense_loop(const float *__restrict__ X, const float *__restrict__ Y,
                                  const float *__restrict__ Z, int k_begin, int k_end, const SearchConst &C,
                                  const DenseGroup (&dg)[NG], int (&cnt)[NG][8])
{
    constexpr int kStepL = NT * KU;
    constexpr int kFold = 31 / KU;
    constexpr uint32_t kSliceA = 0x42000021u;          // window bits 0, 5, 25, 30
    constexpr uint32_t kSliceB = kSliceA << 1;         // window bits 1, 6, 26, 31
    uint64_t acc_a[NG], acc_b[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) acc_a[g] = acc_b[g] = 0;
    int rounds = 0;
    auto fold = [&]() {
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            cnt[g][0] += (int)(acc_a[g] & 31u);
            cnt[g][2] += (int)((acc_a[g] >> 5) & 0xFFFFFu);
            cnt[g][1] += (int)((acc_a[g] >> 25) & 31u);
            cnt[g][3] += (int)(acc_a[g] >> 30);
            cnt[g][4] += (int)((acc_b[g] >> 1) & 31u);
            cnt[g][6] += (int)((acc_b[g] >> 6) & 0xFFFFFu);
            cnt[g][5] += (int)((acc_b[g] >> 26) & 31u);
            cnt[g][7] += (int)(acc_b[g] >> 31);
            acc_a[g] = acc_b[g] = 0;
        }
    };
    for (int kb = k_begin + (int)threadIdx.x; kb < k_end; kb += kStepL) {
        // 32-bit byte offsets (K <= 2^24), one per round; the KU points sit
        // at fixed distances from it
        const uint32_t koff = (uint32_t)kb * 4u;
        float sx[KU], sy[KU], sz[KU];
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            sx[u] = *reinterpret_cast<const float *>(reinterpret_cast<const char *>(X) + koff + u * NT * 4);
            sy[u] = *reinterpret_cast<const float *>(reinterpret_cast<const char *>(Y) + koff + u * NT * 4);
            sz[u] = *reinterpret_cast<const float *>(reinterpret_cast<const char *>(Z) + koff + u * NT * 4);
        }
        uint32_t idx[NG][KU], i0[NG][KU];
#pragma unroll
        for (int g = 0; g < NG; ++g)
#pragma unroll
            for (int u = 0; u < KU; ++u) {
                uint32_t rb[3], f[2];
#pragma unroll
                for (int row = 0; row < 3; ++row) {
                    float t0 = dg[g].R[3 * row + 0] * sx[u];
                    float t1 = dg[g].R[3 * row + 1] * sy[u];
                    float t2 = dg[g].R[3 * row + 2] * sz[u];
                    float p = (t0 + t1) + t2;
                    float q = scale_to_cells<RM>(p, C);
                    // floor and convert in one instruction (equal to floorf then
                    // conversion for the finite, in-range q here; denormals kept)
                    int32_t fl;
                    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(fl) : "v"(q));
                    const int32_t w = fl + dg[g].off[row];
                    const uint32_t shr = row < 2 ? dg[g].level + 2u : dg[g].level;
                    rb[row] = min((uint32_t)(w >> shr), dg[g].lim[row]);
                    if (row < 2) f[row] = __builtin_amdgcn_ubfe((uint32_t)w, dg[g].level, 2u);
                }
                // z voxels x y bricks <= 2^24, x bricks <= 4096: 24-bit products are exact
                idx[g][u] = mad24(mad24(rb[2], dg[g].ny, rb[1]), dg[g].nx, rb[0]);
                i0[g][u] = f[1] * 5u + f[0];   // 0 .. 18
            }
        uint2 bits[NG][KU];
#pragma unroll
        for (int g = 0; g < NG; ++g)
#pragma unroll
            for (int u = 0; u < KU; ++u)     // grid entries <= 2^28: byte offset < 2^31
                bits[g][u] =
                    *reinterpret_cast<const uint2 *>(reinterpret_cast<const char *>(dg[g].dense) + idx[g][u] * 8u);
#pragma unroll
        for (int g = 0; g < NG; ++g)
#pragma unroll
            for (int u = 0; u < KU; ++u) {
                const uint32_t win = __builtin_amdgcn_alignbit(bits[g][u].y, bits[g][u].x, i0[g][u]);
                // member j = 4 jx + 2 jy + jz sits at window bit 25 jz + 5 jy + jx
                acc_a[g] += (uint64_t)(win & kSliceA);
                acc_b[g] += (uint64_t)(win & kSliceB);
            }
        if (++rounds == kFold) {
            fold();
            rounds = 0;
        }
    }
    fold();
}

// Hash-table scoring of the points [k_begin, k_end) against one group (a
// level without a dense grid): the brick key is probed with linear probing,
// kUnroll points per thread in flight.
template <int RM, int NT>
__device__ inline void hash_loop(const float *__restrict__ X, const float *__restrict__ Y,
                                 const float *__restrict__ Z, int k_begin, int k_end, const SearchConst &C,
                                 const LevelView &lv, const float (&R)[9], int bx, int by, int bz, int level,
                                 int (&cnt)[8])
{
    const uint2 *__restrict__ keys = lv.keys;
    const uint4 *__restrict__ bitsv = lv.bits;
    const uint32_t cap_mask = lv.cap_mask;
    const uint32_t ex = (uint32_t)(lv.bmax[0] - lv.bmin[0]);
    const uint32_t ey = (uint32_t)(lv.bmax[1] - lv.bmin[1]);
    const uint32_t ez = (uint32_t)(lv.bmax[2] - lv.bmin[2]);
    for (int kb = k_begin + (int)threadIdx.x; kb < k_end; kb += NT * kUnroll) {
        uint32_t h[kUnroll], klo[kUnroll], khi[kUnroll];
        int i0[kUnroll];
        int state[kUnroll];   // 0: miss, 1: probing, 2: found
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int k = kb + u * NT;
            state[u] = 0;
            h[u] = 0;
            klo[u] = khi[u] = 0;
            i0[u] = 0;
            if (k < k_end) {
                const float sx = X[k], sy = Y[k], sz = Z[k];
                int32_t w[3];
#pragma unroll
                for (int row = 0; row < 3; ++row) {
                    float t0 = R[3 * row + 0] * sx;
                    float t1 = R[3 * row + 1] * sy;
                    float t2 = R[3 * row + 2] * sz;
                    float p = (t0 + t1) + t2;
                    float q = scale_to_cells<RM>(p, C);
                    w[row] = ((int32_t)floorf(q) >> level);
                }
                const int32_t wx = w[0] + bx, wy = w[1] + by, wz = w[2] + bz;
                const int32_t Bx = wx >> 2, By = wy >> 2, Bz = wz >> 2;
                const uint32_t rx = (uint32_t)(Bx - lv.bmin[0]), ry = (uint32_t)(By - lv.bmin[1]),
                               rz = (uint32_t)(Bz - lv.bmin[2]);
                if (rx <= ex && ry <= ey && rz <= ez) {
                    i0[u] = ((wz & 3) * 5 + (wy & 3)) * 5 + (wx & 3);   // 0 .. 93
                    state[u] = 1;
                    klo[u] = brick_key_lo(Bx, By, Bz);
                    khi[u] = brick_key_hi(Bx, By, Bz);
                    h[u] = brick_hash(Bx, By, Bz) & cap_mask;
                }
            }
        }
        for (;;) {
            bool again = false;
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                if (state[u] == 1) {
                    const uint2 kk = keys[h[u]];
                    if (kk.x == klo[u] && kk.y == khi[u]) state[u] = 2;
                    else if (kk.x == kEmptyLo && kk.y == kEmptyHi) state[u] = 0;
                    else {
                        h[u] = (h[u] + 1) & cap_mask;
                        again = true;
                    }
                }
            }
            if (!again) break;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            if (state[u] == 2) {
                const uint4 bits = bitsv[h[u]];
                const int word = i0[u] >> 5;
                const uint32_t lo = word == 0 ? bits.x : (word == 1 ? bits.y : bits.z);
                const uint32_t hi = word == 0 ? bits.y : (word == 1 ? bits.z : bits.w);
                const uint32_t win = __builtin_amdgcn_alignbit(hi, lo, (uint32_t)(i0[u] & 31));
                // member j = 4 jx + 2 jy + jz sits at window bit 25 jz + 5 jy + jx
                cnt[0] += (win >> 0) & 1u;
                cnt[1] += (win >> 25) & 1u;
                cnt[2] += (win >> 5) & 1u;
                cnt[3] += (win >> 30) & 1u;
                cnt[4] += (win >> 1) & 1u;
                cnt[5] += (win >> 26) & 1u;
                cnt[6] += (win >> 6) & 1u;
                cnt[7] += (win >> 31) & 1u;
            }
        }
    }
}

// The eight member counts of a looked-up window, each weighted by c (the
// points of one histogram voxel): member j = 4 jx + 2 jy + jz sits at window
// bit 25 jz + 5 jy + jx.
__device__ inline void add_window(uint32_t win, uint32_t c, uint32_t (&acc)[8])
{
    acc[0] = mad24(__builtin_amdgcn_ubfe(win, 0u, 1u), c, acc[0]);
    acc[1] = mad24(__builtin_amdgcn_ubfe(win, 25u, 1u), c, acc[1]);
    acc[2] = mad24(__builtin_amdgcn_ubfe(win, 5u, 1u), c, acc[2]);
    acc[3] = mad24(__builtin_amdgcn_ubfe(win, 30u, 1u), c, acc[3]);
    acc[4] = mad24(__builtin_amdgcn_ubfe(win, 1u, 1u), c, acc[4]);
    acc[5] = mad24(__builtin_amdgcn_ubfe(win, 26u, 1u), c, acc[5]);
    acc[6] = mad24(__builtin_amdgcn_ubfe(win, 6u, 1u), c, acc[6]);
    acc[7] = mad24(__builtin_amdgcn_ubfe(win, 31u, 1u), c, acc[7]);
}

// 32-bit window of the eight siblings of voxel (x, y, z) (level-l voxel
// coordinates of the group base plus the point's voxel) in a level held only
// as a hash table: 0 when the brick is absent.
__device__ inline uint32_t hash_window(const LevelView &lv, int32_t wx, int32_t wy, int32_t wz)
{
    const int32_t Bx = wx >> 2, By = wy >> 2, Bz = wz >> 2;
    if ((uint32_t)(Bx - lv.bmin[0]) > (uint32_t)(lv.bmax[0] - lv.bmin[0]) ||
        (uint32_t)(By - lv.bmin[1]) > (uint32_t)(lv.bmax[1] - lv.bmin[1]) ||
        (uint32_t)(Bz - lv.bmin[2]) > (uint32_t)(lv.bmax[2] - lv.bmin[2]))
        return 0u;
    const uint32_t klo = brick_key_lo(Bx, By, Bz), khi = brick_key_hi(Bx, By, Bz);
    uint32_t h = brick_hash(Bx, By, Bz) & lv.cap_mask;
    for (;;) {
        const uint2 kk = lv.keys[h];
        if (kk.x == klo && kk.y == khi) break;
        if (kk.x == kEmptyLo && kk.y == kEmptyHi) return 0u;
        h = (h + 1) & lv.cap_mask;
    }
    const uint4 bits = lv.bits[h];
    const int i0 = ((wz & 3) * 5 + (wy & 3)) * 5 + (wx & 3);
    const int word = i0 >> 5;
    const uint32_t lo = word == 0 ? bits.x : (word == 1 ? bits.y : bits.z);
    const uint32_t hi = word == 0 ? bits.y : (word == 1 ? bits.z : bits.w);
    return __builtin_amdgcn_alignbit(hi, lo, (uint32_t)(i0 & 31));
}

// A histogram item: up to kItemGroups groups of one run (one level l, one
// rotation R).  Every scan point's level-l voxel v = floor(floor(R s / r) /
// 2^l) goes into an LDS histogram; a group with base b then scores, for each
// member j, the sum over distinct voxels v of count(v) [v + b + j in D_l]
// (Eq. (12) with the points of one voxel taken together: the voxel of a
// point, and hence every lookup, depends on the point only through v).
// Returns false, having scored nothing, if the scan has more than kHistMax
// distinct voxels at this level and rotation.
template <int RM, int NT>
__device__ bool hist_item(State *st, const int4 desc, const ScoreArgs &A, const MapView &map, const SearchConst &C,
                          ScoreSmemRuns<NT> &sh, int32_t *__restrict__ scores)
{
    HistSmem &H = sh.h;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int first = desc.x, m = desc.y;
    const uint4 Gv = A.groups[A.rgroups[first]];
    const uint32_t gy = __builtin_amdgcn_readfirstlane(Gv.y), gz = __builtin_amdgcn_readfirstlane(Gv.z);
    const int level = (int)(__builtin_amdgcn_readfirstlane(Gv.w) & 0xFF);
    float R[9];
    rotation(A.trig, C, level, hi16u(gy), lo16u(gz), hi16u(gz), R);
    for (int i = tid; i < kHistSlots; i += NT) H.key[i] = kHistEmpty;
    for (int i = tid; i < kHistSlots / 2; i += NT) H.cnt[i] = 0u;
    if (tid == 0) {
        H.n_distinct = 0;
        H.full = 0;
        H.n_compact = 0;
    }
    __syncthreads();
    // 1. histogram of the points' level-l voxels
    const float *__restrict__ X = A.X;
    const float *__restrict__ Y = A.Y;
    const float *__restrict__ Z = A.Z;
    const int K = C.K;
    volatile int *full = &H.full;
    // wave-uniform trip count (the lane shuffle and ballot below need every
    // lane); points past K get the empty key
    for (int kb = tid; __builtin_amdgcn_readfirstlane(kb) < K && !__builtin_amdgcn_readfirstlane(*full);
         kb += NT * 4) {
        uint32_t key[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = kb + u * NT;
            key[u] = kHistEmpty;
            if (k < K) {
                const float sx = X[k], sy = Y[k], sz = Z[k];
                uint32_t packed = 0;
#pragma unroll
                for (int row = 0; row < 3; ++row) {
                    float t0 = R[3 * row + 0] * sx;
                    float t1 = R[3 * row + 1] * sy;
                    float t2 = R[3 * row + 2] * sz;
                    float p = (t0 + t1) + t2;
                    float q = scale_to_cells<RM>(p, C);
                    int32_t fl;
                    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(fl) : "v"(q));
                    packed |= (uint32_t)((fl >> level) + kHistBias) << (10 * row);
                }
                key[u] = packed;
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            // the lanes of a wave hold consecutive scan points, which the
            // spatial sort keeps close together: a run of lanes with the same
            // voxel is inserted once, by its first lane, with the run's length
            const uint32_t prev = __shfl_up(key[u], 1);
            const bool head = lane == 0 || key[u] != prev;
            const uint64_t heads = __ballot(head);
            const uint64_t after = lane == 63 ? 0ull : heads >> (lane + 1);
            const uint32_t run = after ? (uint32_t)__ffsll((long long)after) : (uint32_t)(64 - lane);
            if (!head || key[u] == kHistEmpty) continue;
            uint32_t h = (key[u] * 0x9E3779B1u) >> 21;
            bool placed = false;
            for (int probe = 0; probe < 32; ++probe) {
                const uint32_t old = atomicCAS(&H.key[h], kHistEmpty, key[u]);
                if (old == kHistEmpty) {
                    if (atomicAdd(&H.n_distinct, 1) >= kHistMax) *full = 1;
                    placed = true;
                    break;
                }
                if (old == key[u]) {
                    placed = true;
                    break;
                }
                h = (h + 1) & (kHistSlots - 1);
            }
            if (!placed) *full = 1;
            else atomicAdd(&H.cnt[h >> 1], run << ((h & 1) << 4));
        }
    }
    __syncthreads();
    if (H.full) {
        // too many distinct voxels at this level: later runs of the level go point by point
        if (tid == 0) {
            atomicOr(&st->hist_off, 1 << level);
            atomicAdd(&st->hist_fallbacks, 1);
        }
        return false;
    }
    // 2. compact: each wave appends its non-empty slots (order is free: the
    // scores are sums over the voxels)
    for (int sl = tid; sl < kHistSlots; sl += NT) {
        const uint32_t k = H.key[sl];
        const bool live = k != kHistEmpty;
        const uint64_t bal = __ballot(live);
        int base = 0;
        if (lane == 0 && bal) base = atomicAdd(&H.n_compact, (int)__popcll(bal));
        base = __builtin_amdgcn_readfirstlane(base);
        if (live) {
            const int p = base + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
            H.ckey[p] = k;
            H.ccnt[p] = (uint16_t)((H.cnt[sl >> 1] >> ((sl & 1) << 4)) & 0xFFFFu);
        }
    }
    __syncthreads();
    const int D = H.n_compact;
    // 3. every group of the item against the D voxels, one group per wave at a time
    const LevelView &lv = map.lv[level];
    const bool dense = lv.dense != nullptr;
    const uint32_t nx = (uint32_t)lv.nx, ny = (uint32_t)lv.ny;
    const uint32_t lim0 = (uint32_t)(lv.bmax[0] - lv.bmin[0]) + 1u, lim1 = (uint32_t)(lv.bmax[1] - lv.bmin[1]) + 1u;
    const uint32_t lim2 = 4u * ((uint32_t)(lv.bmax[2] - lv.bmin[2]) + 1u);
    for (int gi = wave; gi < m; gi += NT / 64) {
        const int g = __builtin_amdgcn_readfirstlane(A.rgroups[first + gi]);
        const uint4 G = A.groups[g];
        const int32_t bx = lo16s(__builtin_amdgcn_readfirstlane(G.x)), by = hi16s(__builtin_amdgcn_readfirstlane(G.x));
        const int32_t bz = lo16s(__builtin_amdgcn_readfirstlane(G.y));
        uint32_t acc[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
        if (dense) {
            // level-l voxel relative to 4 x the box minimum, with the key's bias taken off
            const int32_t ox = bx - 4 * lv.bmin[0] - kHistBias, oy = by - 4 * lv.bmin[1] - kHistBias;
            const int32_t oz = bz - 4 * lv.bmin[2] - kHistBias;
            for (int d = lane; d < D; d += 64) {
                const uint32_t key = H.ckey[d];
                const uint32_t c = H.ccnt[d];
                const int32_t ux = (int32_t)(key & 1023u) + ox;
                const int32_t uy = (int32_t)((key >> 10) & 1023u) + oy;
                const int32_t uz = (int32_t)(key >> 20) + oz;
                const uint32_t rx = min((uint32_t)(ux >> 2), lim0), ry = min((uint32_t)(uy >> 2), lim1);
                const uint32_t rz = min((uint32_t)uz, lim2);
                const uint2 col = lv.dense[mad24(mad24(rz, ny, ry), nx, rx)];
                const uint32_t i0 = ((uint32_t)uy & 3u) * 5u + ((uint32_t)ux & 3u);
                add_window(__builtin_amdgcn_alignbit(col.y, col.x, i0), c, acc);
            }
        } else {
            for (int d = lane; d < D; d += 64) {
                const uint32_t key = H.ckey[d];
                const uint32_t c = H.ccnt[d];
                const int32_t wx = (int32_t)(key & 1023u) - kHistBias + bx;
                const int32_t wy = (int32_t)((key >> 10) & 1023u) - kHistBias + by;
                const int32_t wz = (int32_t)(key >> 20) - kHistBias + bz;
                add_window(hash_window(lv, wx, wy, wz), c, acc);
            }
        }
        int sum[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) sum[j] = wave_sum((int)acc[j]);
        // hand-off to the tile pass: returning atomics (see score_items)
        if (lane < 8) {
            int v = sum[0];
#pragma unroll
            for (int j = 1; j < 8; ++j) v = lane == j ? sum[j] : v;
            const int old = __hip_atomic_exchange(&scores[8 * (int64_t)g + lane], v, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
            asm volatile("" ::"v"(old));
        }
    }
    return true;
}

// Point-by-point scoring of the points [k_begin, k_end) of one or two groups
// (dense grid or hash table per group); cnt receives their member counts.
template <int RM, int NT>
__device__ void direct_groups(const ScoreArgs &A, const MapView &map, const SearchConst &C, const int gs[2], int ng,
                              int k_begin, int k_end, int (&cnt)[2][8])
{
    const float *__restrict__ X = A.X;
    const float *__restrict__ Y = A.Y;
    const float *__restrict__ Z = A.Z;
    // the groups are the same for every lane of the item: scalar registers
    DenseGroup dg[2];
    int lvl[2], base[2][3];
    bool dense[2];
    float R[2][9];
#pragma unroll
    for (int gi = 0; gi < 2; ++gi) {
        const uint4 Gv = A.groups[gs[gi]];
        const uint4 G = make_uint4(__builtin_amdgcn_readfirstlane(Gv.x), __builtin_amdgcn_readfirstlane(Gv.y),
                                   __builtin_amdgcn_readfirstlane(Gv.z), __builtin_amdgcn_readfirstlane(Gv.w));
        const int level = (int)(G.w & 0xFF);
        lvl[gi] = level;
        base[gi][0] = lo16s(G.x);
        base[gi][1] = hi16s(G.x);
        base[gi][2] = lo16s(G.y);
        rotation(A.trig, C, level, hi16u(G.y), lo16u(G.z), hi16u(G.z), R[gi]);
        const LevelView &lv = map.lv[level];
        dense[gi] = lv.dense != nullptr;
#pragma unroll
        for (int e = 0; e < 9; ++e) dg[gi].R[e] = R[gi][e];
        dg[gi].dense = lv.dense;
        dg[gi].nx = (uint32_t)lv.nx;
        dg[gi].ny = (uint32_t)lv.ny;
        dg[gi].lim[0] = (uint32_t)(lv.bmax[0] - lv.bmin[0]) + 1u;
        dg[gi].lim[1] = (uint32_t)(lv.bmax[1] - lv.bmin[1]) + 1u;
        dg[gi].lim[2] = 4u * ((uint32_t)(lv.bmax[2] - lv.bmin[2]) + 1u);
        const int32_t scale = 1 << level;
#pragma unroll
        for (int a = 0; a < 3; ++a) dg[gi].off[a] = (base[gi][a] - 4 * lv.bmin[a]) * scale;
        dg[gi].level = (uint32_t)level;
    }
#pragma unroll
    for (int gi = 0; gi < 2; ++gi)
#pragma unroll
        for (int j = 0; j < 8; ++j) cnt[gi][j] = 0;
    if (ng == 2 && dense[0] && dense[1]) {
        dense_loop<RM, NT, 2, kUnroll / 2>(X, Y, Z, k_begin, k_end, C, dg, cnt);
    } else {
#pragma unroll
        for (int gi = 0; gi < 2; ++gi) {
            if (gi >= ng) break;
            if (dense[gi]) {
                const DenseGroup one[1] = {dg[gi]};
                int c1[1][8] = {{0, 0, 0, 0, 0, 0, 0, 0}};
                dense_loop<RM, NT, 1, kUnroll>(X, Y, Z, k_begin, k_end, C, one, c1);
#pragma unroll
                for (int j = 0; j < 8; ++j) cnt[gi][j] = c1[0][j];
            } else {
                hash_loop<RM, NT>(X, Y, Z, k_begin, k_end, C, map.lv[lvl[gi]], R[gi], base[gi][0], base[gi][1],
                                  base[gi][2], lvl[gi], cnt[gi]);
            }
        }
    }
}

// Scoring of a batch the gather cut into runs and item descriptors (with
// the histogram option; see score_items for the point-by-point scheme).
template <int RM, int NT>
__device__ void score_items_runs(State *st, const ScoreArgs &A, const MapView &map, const SearchConst &C,
                                 ScoreSmemRuns<NT> &sh)
{
    int32_t *__restrict__ scores = A.scores;
    int32_t *tile_done = A.tile_done;
    auto &red = sh.red;
    // the batch header in one round trip (independent loads, issued together)
    int n_groups = A.n_groups_fixed, best = 0, hr = 0, hs = 0, hi = 0;
    if (st) {
        const int pending = ld_agent(&st->batch), ng = ld_agent(&st->n_groups);
        best = ld_agent(&st->best);
        hr = ld_agent(&st->runs);
        hs = ld_agent(&st->n_slices);
        hi = ld_agent(&st->n_items);
        n_groups = pending ? ng : 0;
    }
    if (n_groups <= 0) return;
    // Work items.  A batch the gather wrote comes as item descriptors over
    // its runs (groups sharing a level and rotation): histogram items, or
    // groups scored point by point.  Point by point, groups are scored two to
    // an item, so that a workgroup reads every scan point once for both and
    // pays the per-item latency (groups, rotations, count reduction, atomics)
    // once per pair; groups too few to fill the grid are split score_items /
    // groups ways into point slices.  Items go round-robin over the
    // workgroups (the grid is as large as the device holds at once), or, with
    // a ticket counter, to whichever workgroup asks next.
    const bool runs = st && hr;
    const int K = C.K;
    constexpr int kStep = NT * kUnroll;                 // points of one round of the workgroup
    const int max_s = (K + kStep - 1) / kStep;
    const int P = (int)gridDim.x;
    // without runs (initial set, seed beam, node lists): groups in index
    // order, paired, or split into point slices when they are too few
    const int s_min = min(max_s, max(1, (C.score_items + n_groups - 1) / n_groups));
    const bool legacy_pairs = s_min == 1;
    const int S = runs ? max(1, hs) : (legacy_pairs ? 1 : s_min);
    const int64_t n_items = runs ? (int64_t)hi : (legacy_pairs ? (n_groups + 1) / 2 : (int64_t)n_groups * S);
    int32_t *ticket = A.ticket;
    int64_t item = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    while (item < n_items) {
        // the next item's ticket, drawn now so that its latency is hidden
        // behind the item (one atomic counter for the whole grid: used by
        // the persistent loop, whose grid is one workgroup per CU)
        int nxt = 0;
        if (ticket && threadIdx.x == 0) nxt = atomicAdd(&ticket[0], 1);
        // the item: x = first entry, y = groups, z = kind, w = slice
        int4 desc;
        if (runs) {
            const int4 dv = A.items[item];
            desc = make_int4(__builtin_amdgcn_readfirstlane(dv.x), __builtin_amdgcn_readfirstlane(dv.y),
                             __builtin_amdgcn_readfirstlane(dv.z), __builtin_amdgcn_readfirstlane(dv.w));
        } else if (legacy_pairs) {
            desc = make_int4(2 * (int)item, 2 * (int)item + 1 < n_groups ? 2 : 1, kItemPair, 0);
        } else {
            desc = make_int4((int)(item / S), 1, kItemSlice, (int)(item % S));
        }
        auto group_at = [&](int e) { return runs ? A.rgroups[e] : e; };
        const bool sliced = desc.z == kItemSlice;
        bool done = false;
        if (desc.z == kItemHist) done = hist_item<RM, NT>(st, desc, A, map, C, sh, scores);
        int gs[2] = {0, 0}, ng = 0;
        if (!done) {
            // point by point: a pair, a slice, or (rarely) a histogram item
            // whose scan had too many distinct voxels, one group at a time
            const int n_pass = desc.z == kItemHist ? desc.y : 1;
            for (int pass = 0; pass < n_pass; ++pass) {
                int k_begin = 0, k_end = K;
                if (desc.z == kItemHist) {
                    gs[0] = gs[1] = group_at(desc.x + pass);
                    ng = 1;
                } else if (desc.z == kItemPair) {
                    ng = desc.y;
                    gs[0] = group_at(desc.x);
                    gs[1] = group_at(desc.x + ng - 1);
                } else {
                    gs[0] = gs[1] = group_at(desc.x);
                    ng = 1;
                    // slices are whole rounds, so only the last one is ragged; its tail
                    // runs over the scan padding (points that fall outside every box)
                    const int chunk = ((K + S - 1) / S + kStep - 1) / kStep * kStep;
                    k_begin = min(K, desc.w * chunk);
                    k_end = min(K, k_begin + chunk);
                }
                gs[0] = __builtin_amdgcn_readfirstlane(gs[0]);
                gs[1] = __builtin_amdgcn_readfirstlane(gs[1]);
                int cnt[2][8];
                direct_groups<RM, NT>(A, map, C, gs, ng, k_begin, k_end, cnt);
#pragma unroll
                for (int gi = 0; gi < 2; ++gi) {
                    if (gi < ng) {
#pragma unroll
                        for (int j = 0; j < 8; ++j) {
                            const int v = wave_sum(cnt[gi][j]);
                            if (lane == 0) red[wave][8 * gi + j] = v;
                        }
                    }
                }
                __syncthreads();
                // Hand-off to the tile pass without a device-scope fence (which on this
                // GPU writes back and invalidates the XCD's L2): the scores are written
                // with returning atomics, which have been performed once the barrier's
                // wait for outstanding memory operations is over; only then is the
                // tile counter bumped, and the tile pass reads the scores with atomics
                // too, at the same coherence point.  Whole groups store their counts;
                // the slices of a group add theirs to scores zeroed by the batch's producer.
                if (threadIdx.x < 8 * ng) {
                    int sum = 0;
                    for (int wv = 0; wv < NT / 64; ++wv) sum += red[wv][threadIdx.x];
                    const int g = threadIdx.x >= 8 ? gs[1] : gs[0];
                    int32_t *dst = &scores[8 * (int64_t)g + (threadIdx.x & 7)];
                    const int old = !sliced ? __hip_atomic_exchange(dst, sum, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                            : __hip_atomic_fetch_add(dst, sum, __ATOMIC_RELAXED,
                                                                     __HIP_MEMORY_SCOPE_AGENT);
                    asm volatile("" ::"v"(old));          // keep the returning form of the atomic
                }
                __syncthreads();
            }
        }
        __syncthreads();
        if (tile_done) {
            // every group this item completed counts towards its tile (32
            // consecutive groups); the item that completes a tile sorts it into
            // queue buckets
            if (threadIdx.x == 0) sh.h.n_tiles = 0;
            __syncthreads();
            const int n_done = desc.y;
            if ((int)threadIdx.x < n_done) {
                int g = desc.z == kItemHist ? group_at(desc.x + (int)threadIdx.x) : (threadIdx.x == 0 ? gs[0] : gs[1]);
                bool whole = true;
                if (sliced) whole = atomicAdd(&A.gslices[g], 1) == S - 1;
                if (whole) {
                    if (sliced) __hip_atomic_store(&A.gslices[g], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const int t = g / kTileGroups;
                    const int in_tile = min(n_groups, (t + 1) * kTileGroups) - t * kTileGroups;
                    if (atomicAdd(&tile_done[t], 1) == in_tile - 1) sh.h.tiles[atomicAdd(&sh.h.n_tiles, 1)] = t;
                }
            }
            __syncthreads();
            const int n_t = sh.h.n_tiles;
            for (int i = 0; i < n_t; ++i) {
                const int t = sh.h.tiles[i];
                tile_pass<NT>(t, A.groups, scores, st, C, n_groups, best, A.kq, A.krank, A.knode, A.kcnt, A.hist, A.qmask,
                              sh.rt, sh.sm);
                if (threadIdx.x == 0) __hip_atomic_store(&tile_done[t], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __syncthreads();
            }
        }
        if (ticket) {
            if (threadIdx.x == 0) sh.s_next = nxt;
            __syncthreads();
            item = (int64_t)P + sh.s_next;
        } else {
            item += P;
        }
    }
    // Every workgroup has drawn its last ticket: the last one to get here
    // rewinds the counters for the next launch.
    if (ticket && threadIdx.x == 0 && atomicAdd(&ticket[1], 1) == P - 1) {
        __hip_atomic_store(&ticket[0], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ticket[1], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <int RM, int NT>
__device__ void score_items(State *st, const ScoreArgs &A, const MapView &map, const SearchConst &C,
                            ScoreSmem<NT> &sh)
{
    const uint4 *__restrict__ groups = A.groups;
    const float *__restrict__ X = A.X;
    const float *__restrict__ Y = A.Y;
    const float *__restrict__ Z = A.Z;
    const double2 *__restrict__ trig = A.trig;
    int32_t *__restrict__ scores = A.scores;
    int32_t *tile_done = A.tile_done;
    auto &red = sh.red;
    // the batch header in one round trip (independent loads, issued together)
    int n_groups = A.n_groups_fixed, best = 0;
    if (st) {
        const int pending = ld_agent(&st->batch), ng = ld_agent(&st->n_groups);
        best = ld_agent(&st->best);
        n_groups = pending ? ng : 0;
    }
    if (n_groups <= 0) return;
    const int K = C.K;
    constexpr int kStep = NT * kUnroll;                 // points of one round of the workgroup
    const int max_s = (K + kStep - 1) / kStep;
    // Work items.  A large batch is scored two groups to an item, so that a
    // workgroup reads every scan point once for both and pays the per-item
    // latency (group, rotations, count reduction, atomics) once per pair; a
    // batch too small to fill the grid is split score_items / n_groups ways
    // into point slices of single groups.  The grid is as large as the device
    // holds at once; items go round-robin over the workgroups, or, with a
    // ticket counter, to whichever workgroup asks next.
    const int P = (int)gridDim.x;
    const int s_min = min(max_s, max(1, (C.score_items + n_groups - 1) / n_groups));
    const bool pairs = s_min == 1;
    const int S = pairs ? 1 : s_min;
    const int64_t n_items = pairs ? (n_groups + 1) / 2 : (int64_t)n_groups * S;
    int32_t *ticket = A.ticket;
    int64_t item = blockIdx.x;
    while (item < n_items) {
        // the next item's ticket, drawn now so that its latency is hidden
        // behind the item (one atomic counter for the whole grid: used by
        // the persistent loop, whose grid is one workgroup per CU)
        int nxt = 0;
        if (ticket && threadIdx.x == 0) nxt = atomicAdd(&ticket[0], 1);
        int gs[2], ng, k_begin, k_end;
        if (pairs) {
            gs[0] = 2 * (int)item;
            ng = gs[0] + 1 < n_groups ? 2 : 1;
            gs[1] = gs[0] + ng - 1;
            k_begin = 0;
            k_end = K;
        } else {
            gs[0] = gs[1] = (int)(item / S);
            ng = 1;
            const int sp = (int)(item % S);
            // slices are whole rounds, so only the last one is ragged; its tail
            // runs over the scan padding (points that fall outside every box)
            const int chunk = ((K + S - 1) / S + kStep - 1) / kStep * kStep;
            k_begin = min(K, sp * chunk);
            k_end = min(K, k_begin + chunk);
        }
        // the groups are the same for every lane of the item: scalar registers
        DenseGroup dg[2];
        int lvl[2], base[2][3];
        bool dense[2];
        float R[2][9];
#pragma unroll
        for (int gi = 0; gi < 2; ++gi) {
            const uint4 Gv = groups[gs[gi]];
            const uint4 G = make_uint4(__builtin_amdgcn_readfirstlane(Gv.x), __builtin_amdgcn_readfirstlane(Gv.y),
                                       __builtin_amdgcn_readfirstlane(Gv.z), __builtin_amdgcn_readfirstlane(Gv.w));
            const int level = (int)(G.w & 0xFF);
            lvl[gi] = level;
            base[gi][0] = lo16s(G.x);
            base[gi][1] = hi16s(G.x);
            base[gi][2] = lo16s(G.y);
            rotation(trig, C, level, hi16u(G.y), lo16u(G.z), hi16u(G.z), R[gi]);
            const LevelView &lv = map.lv[level];
            dense[gi] = lv.dense != nullptr;
#pragma unroll
            for (int e = 0; e < 9; ++e) dg[gi].R[e] = R[gi][e];
            dg[gi].dense = lv.dense;
            dg[gi].nx = (uint32_t)lv.nx;
            dg[gi].ny = (uint32_t)lv.ny;
            dg[gi].lim[0] = (uint32_t)(lv.bmax[0] - lv.bmin[0]) + 1u;
            dg[gi].lim[1] = (uint32_t)(lv.bmax[1] - lv.bmin[1]) + 1u;
            dg[gi].lim[2] = 4u * ((uint32_t)(lv.bmax[2] - lv.bmin[2]) + 1u);
            const int32_t scale = 1 << level;
#pragma unroll
            for (int a = 0; a < 3; ++a) dg[gi].off[a] = (base[gi][a] - 4 * lv.bmin[a]) * scale;
            dg[gi].level = (uint32_t)level;
        }
        int cnt[2][8];
#pragma unroll
        for (int gi = 0; gi < 2; ++gi)
#pragma unroll
            for (int j = 0; j < 8; ++j) cnt[gi][j] = 0;
        if (ng == 2 && dense[0] && dense[1]) {
            dense_loop<RM, NT, 2, kUnroll / 2>(X, Y, Z, k_begin, k_end, C, dg, cnt);
        } else {
#pragma unroll
            for (int gi = 0; gi < 2; ++gi) {
                if (gi >= ng) break;
                if (dense[gi]) {
                    const DenseGroup one[1] = {dg[gi]};
                    int c1[1][8] = {{0, 0, 0, 0, 0, 0, 0, 0}};
                    dense_loop<RM, NT, 1, kUnroll>(X, Y, Z, k_begin, k_end, C, one, c1);
#pragma unroll
                    for (int j = 0; j < 8; ++j) cnt[gi][j] = c1[0][j];
                } else {
                    hash_loop<RM, NT>(X, Y, Z, k_begin, k_end, C, map.lv[lvl[gi]], R[gi], base[gi][0], base[gi][1],
                                      base[gi][2], lvl[gi], cnt[gi]);
                }
            }
        }
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
        for (int gi = 0; gi < 2; ++gi) {
            if (gi < ng) {
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int v = wave_sum(cnt[gi][j]);
                    if (lane == 0) red[wave][8 * gi + j] = v;
                }
            }
        }
        __syncthreads();
        // Hand-off to the tile pass without a device-scope fence (which on this
        // GPU writes back and invalidates the XCD's L2): the scores are added
        // with returning atomics, which have been performed once the barrier's
        // wait for outstanding memory operations is over; only then is the
        // tile counter bumped, and the tile pass reads the scores with atomics
        // too, at the same coherence point.
        // (a pair holds its groups whole, so it stores their counts; the
        // slices of a group add theirs to scores zeroed by the batch's producer)
        if (threadIdx.x < 8 * ng) {
            int sum = 0;
            for (int wv = 0; wv < NT / 64; ++wv) sum += red[wv][threadIdx.x];
            const int g = threadIdx.x >= 8 ? gs[1] : gs[0];
            int32_t *dst = &scores[8 * (int64_t)g + (threadIdx.x & 7)];
            const int old = pairs ? __hip_atomic_exchange(dst, sum, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                  : __hip_atomic_fetch_add(dst, sum, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            asm volatile("" ::"v"(old));          // keep the returning form of the atomic
        }
        __syncthreads();
        if (tile_done) {
            // the last workgroup to finish a tile sorts it into queue buckets
            // (a pair never straddles two tiles: tiles hold an even number of groups)
            const int t = gs[0] / kTileGroups;
            if (threadIdx.x == 0) {
                const int t0 = t * kTileGroups, te = min(n_groups, t0 + kTileGroups);
                const int in_tile = pairs ? (te - t0 + 1) / 2 : (te - t0) * S;
                const int prev = atomicAdd(&tile_done[t], 1);
                sh.s_last = (prev == in_tile - 1);
            }
            __syncthreads();
            if (sh.s_last) {
                tile_pass<NT>(t, groups, scores, st, C, n_groups, best, A.kq, A.krank, A.knode, A.kcnt, A.hist, A.qmask,
                              sh.rt, sh.sm);
                if (threadIdx.x == 0) __hip_atomic_store(&tile_done[t], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        if (ticket) {
            if (threadIdx.x == 0) sh.s_next = nxt;
            __syncthreads();
            item = (int64_t)P + sh.s_next;
        } else {
            item += P;
        }
    }
    // Every workgroup has drawn its last ticket: the last one to get here
    // rewinds the counters for the next launch.
    if (ticket && threadIdx.x == 0 && atomicAdd(&ticket[1], 1) == P - 1) {
        __hip_atomic_store(&ticket[0], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ticket[1], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <int RM>
__global__ __launch_bounds__(kScoreThreads) void k_score(State *st, ScoreArgs A, MapView map, SearchConst C)
{
    __shared__ ScoreSmem<kScoreThreads> sh;
    score_items<RM, kScoreThreads>(st, A, map, C, sh);
}

// The run-scheduled scoring, at most 96 vector registers a lane (five
// resident workgroups per CU; the histogram path alone would take it to 116).
template <int RM>
__global__ __launch_bounds__(kScoreThreads) __attribute__((amdgpu_waves_per_eu(kScoreWgPerCu))) void k_score_runs(
    State *st, ScoreArgs A, MapView map, SearchConst C)
{
    __shared__ ScoreSmemRuns<kScoreThreads> sh;
    score_items_runs<RM, kScoreThreads>(st, A, map, C, sh);
}

// ------------------------------------------------------------------ initial set

// Top-level cells as the valid children of virtual cells one level above:
// virtual cell (lexicographic) outer, top-level rotation (lexicographic), then
// the eight translation children as one group.
__global__ void k_enum_initial(uint4 *groups, int32_t *scores, int64_t g0, int32_t count, SearchConst C,
                               int32_t px0, int32_t py0, int32_t pz0, int32_t npy, int32_t npz, State *st)
{
    const int L = C.levels;
    const int na = C.n[0][L], nb = C.n[1][L], ng = C.n[2][L];
    const int64_t nrot = (int64_t)na * nb * ng;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
        int64_t q = g0 + i;
        int64_t rot = q % nrot;
        int64_t par = q / nrot;
        int ig = (int)(rot % ng);
        int ib = (int)((rot / ng) % nb);
        int ia = (int)(rot / ((int64_t)ng * nb));
        int pz = (int)(par % npz) + pz0;
        int py = (int)((par / npz) % npy) + py0;
        int px = (int)(par / ((int64_t)npz * npy)) + px0;
        uint32_t mask = 0;
        for (int jx = 0; jx < 2; ++jx)
            for (int jy = 0; jy < 2; ++jy)
                for (int jz = 0; jz < 2; ++jz) {
                    int t[3] = {2 * px + jx, 2 * py + jy, 2 * pz + jz};
                    bool ok = true;
                    for (int a = 0; a < 3; ++a) ok = ok && t[a] >= C.tlo[a][L] && t[a] <= C.thi[a][L];
                    if (ok) mask |= 1u << (4 * jx + 2 * jy + jz);
                }
        groups[i] = make_uint4(pack16(2 * px, 2 * py), pack16(2 * pz, ia), pack16(ib, ig), (uint32_t)L | (mask << 8));
        for (int j = 0; j < 8; ++j) scores[8 * (int64_t)i + j] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->n_groups = count;
        st->runs = 0;
        st->batch = 1;
        st->q_min = INT_MAX;
        st->q_max = -1;
        st->kept = 0;
    }
}

// ------------------------------------------------------------------ push (stable counting sort)

// Where bucket q's children of this batch go: first the free slots of its
// tail chunk, then fresh chunks from the pool (allocated in bucket order).
__device__ inline void bucket_space(const Bucket &b, int cnt, int &T, int &f, int &space, int &nch)
{
    T = b.head_chunk >= 0 ? b.tail_chunk : -1;
    f = T >= 0 ? b.tail_fill : kChunk;
    space = kChunk - f;
    const int need = max(0, cnt - space);
    nch = (need + kChunk - 1) / kChunk;
}

struct PushBufs {
    int32_t *kq, *krank, *hist, *totals, *pT, *pf, *pc0, *chunk_next;
    int32_t *hbase;            // tile x bucket: first rank of the tile's children in the bucket
    uint4 *knode;
    int32_t *kcnt;
    uint4 *arena;
    uint32_t *qmask;           // occupied buckets of the batch (set by the tile passes, cleared here)
    int32_t *qlist;            // the occupied buckets in order
};

// Second half of the stable counting sort, run by the serial workgroup after
// the scoring kernel's tile passes: per bucket the prefix of the tile counts
// (tile order = batch order), chunk allocation and chain link, then every
// kept child is written to its slot and the histogram is cleared.
template <int NT>
__device__ void push_finish(State *st, const SearchConst &C, Bucket *bk, const uint4 *groups, const PushBufs &B,
                            int *sm, int *blk)
{
    const int tid = threadIdx.x;
    const int q_min = st->q_min, q_max = st->q_max;
    const int64_t kept = st->kept;
    const int n_tiles = (st->n_groups + kTileGroups - 1) / kTileGroups;
    if (q_max < q_min || kept == 0) return;
    const uint64_t tp0 = __builtin_amdgcn_s_memrealtime();
    // the occupied buckets in order (bitmap words of [q_min, q_max], read and cleared)
    const int w0 = q_min >> 5, nw = (q_max >> 5) - w0 + 1;
    int n_occ = 0;
    for (int c = 0; c < nw; c += NT) {
        const int wi = c + tid;
        uint32_t m = 0;
        if (wi < nw) {
            m = B.qmask[w0 + wi];
            if (m) B.qmask[w0 + wi] = 0u;
        }
        const int pc = __popc(m);
        int tot;
        const int incl = block_scan_incl<NT>(pc, sm, &tot);
        int pos = n_occ + incl - pc;
        while (m) {
            const int bit = __ffs(m) - 1;
            m &= m - 1u;
            B.qlist[pos++] = (w0 + wi) * 32 + bit;
        }
        n_occ += tot;
    }
    __syncthreads();
    // per-bucket prefix over tiles (tile-major histogram, in blocks of 16 tiles)
    const int n_blk = (n_tiles + 15) / 16;
    if (n_occ * n_blk <= NT) {
        // one (bucket, block) pair per thread, consecutive threads on
        // consecutive occupied buckets of one block (neighbouring entries of a
        // histogram row): every load in one round, block sums scanned per
        // bucket in LDS, the counts rewritten from registers
        const int pidx = tid, j = pidx / n_occ, i = pidx - j * n_occ;
        const bool act = pidx < n_occ * n_blk;
        const int q = act ? B.qlist[i] : 0;
        int v[16], sum = 0;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int t = j * 16 + u;
            v[u] = (act && t < n_tiles) ? B.hist[(int64_t)t * C.q_count + q] : 0;
            sum += v[u];
        }
        if (act) blk[pidx] = sum;
        __syncthreads();
        if (tid < n_occ) {
            int acc = 0;
            for (int jj = 0; jj < n_blk; ++jj) {
                const int x = blk[jj * n_occ + tid];
                blk[jj * n_occ + tid] = acc;
                acc += x;
            }
            B.totals[tid] = acc;
        }
        __syncthreads();
        if (act) {
            int acc = blk[pidx];
#pragma unroll
            for (int u = 0; u < 16; ++u)
                if (v[u]) {
                    const int64_t h = (int64_t)(j * 16 + u) * C.q_count + q;
                    B.hbase[h] = acc;
                    B.hist[h] = 0;
                    acc += v[u];
                }
        }
    } else {
        for (int i = tid; i < n_occ; i += NT) {
            const int q = B.qlist[i];
            int acc = 0;
            for (int t0 = 0; t0 < n_tiles; t0 += 16) {
                int v[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) v[u] = (t0 + u < n_tiles) ? B.hist[(int64_t)(t0 + u) * C.q_count + q] : 0;
#pragma unroll
                for (int u = 0; u < 16; ++u)
                    if (v[u]) {
                        const int64_t h = (int64_t)(t0 + u) * C.q_count + q;
                        B.hbase[h] = acc;
                        B.hist[h] = 0;
                        acc += v[u];
                    }
            }
            B.totals[i] = acc;
        }
    }
    __syncthreads();
    const uint64_t tp1 = __builtin_amdgcn_s_memrealtime();
    // chunks needed, then allocation in bucket order
    int64_t total_new = 0;
    for (int c = 0; c < n_occ; c += NT) {
        const int i = c + tid;
        int nch = 0;
        if (i < n_occ) {
            int T, f, space;
            bucket_space(bk[B.qlist[i]], B.totals[i], T, f, space, nch);
        }
        int tot;
        (void)block_scan_incl<NT>(nch, sm, &tot);
        total_new += tot;
    }
    const int chunk_top = st->chunk_top;
    if ((int64_t)chunk_top + total_new > (int64_t)st->chunk_cap) {
        __syncthreads();
        if (tid == 0) {
            st->error = 1;
            st->done = 1;
        }
        return;
    }
    int64_t run = 0;
    for (int c = 0; c < n_occ; c += NT) {
        const int i = c + tid;
        const int q = i < n_occ ? B.qlist[i] : 0;
        const int cnt = i < n_occ ? B.totals[i] : 0;
        int T = -1, f = kChunk, space = 0, nch = 0;
        Bucket b = Bucket{-1, 0, -1, 0};
        if (cnt > 0) {
            b = bk[q];
            bucket_space(b, cnt, T, f, space, nch);
        }
        int tot;
        const int incl = block_scan_incl<NT>(nch, sm, &tot);
        if (cnt > 0) {
            const int qi = q - q_min;
            const int c0 = chunk_top + (int)run + incl - nch;
            B.pT[qi] = T;
            B.pf[qi] = f;
            B.pc0[qi] = c0;
            if (nch > 0) {
                if (T >= 0) B.chunk_next[T] = c0;
                else {
                    b.head_chunk = c0;
                    b.head_off = 0;
                }
                for (int m = 0; m + 1 < nch; ++m) B.chunk_next[c0 + m] = c0 + m + 1;
                B.chunk_next[c0 + nch - 1] = -1;
                b.tail_chunk = c0 + nch - 1;
                b.tail_fill = (cnt - space) - kChunk * (nch - 1);
            } else {
                b.tail_fill = f + cnt;
            }
            bk[q] = b;
        }
        run += tot;
    }
    __syncthreads();
    if (tid == 0) {
        st->t_push_prefix += (int64_t)(tp1 - tp0);
        st->t_push_alloc += (int64_t)(__builtin_amdgcn_s_memrealtime() - tp1);
    }
    // scatter: the child of rank r in its bucket fills the tail chunk first.
    // Kept children only, from the tiles' compact lists, NT tiles at a time.
    for (int c0t = 0; c0t < n_tiles; c0t += NT) {
        const int nt_c = min(NT, n_tiles - c0t);
        const int kc = tid < nt_c ? B.kcnt[c0t + tid] : 0;
        int E;
        const int kincl = block_scan_incl<NT>(kc, sm, &E);
        if (tid < nt_c) blk[tid] = kincl;
        __syncthreads();
        for (int e = tid; e < E; e += NT) {
            int lo = 0, hi = nt_c - 1;                // the tile holding kept child e
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (blk[mid] > e) hi = mid;
                else lo = mid + 1;
            }
            const int t = c0t + lo;
            const int64_t k = (int64_t)t * kTileSlots + e - (lo > 0 ? blk[lo - 1] : 0);
            const int q = B.kq[k];
            const int r = B.hbase[(int64_t)t * C.q_count + q] + B.krank[k];
            const uint4 node = B.knode[k];
            const int Tc = B.pT[q - q_min], fc = B.pf[q - q_min];
            const int space = Tc >= 0 ? kChunk - fc : 0;
            int64_t pos;
            if (r < space) pos = (int64_t)Tc * kChunk + fc + r;
            else {
                const int r2 = r - space;
                pos = (int64_t)(B.pc0[q - q_min] + r2 / kChunk) * kChunk + (r2 % kChunk);
            }
            B.arena[pos] = node;
        }
        __syncthreads();
    }
    if (tid == 0) {
        st->chunk_top = chunk_top + (int)total_new;
        st->pushed += kept;
        st->top_q = min(st->top_q, q_min);
    }
}

// ------------------------------------------------------------------ gather + branch

// Per-level grid tables (the members of SearchConst of the same names); the
// gather keeps a copy in LDS, since each lane indexes them by its own node's
// level.
struct LevelTables {
    int32_t n[3][kMaxLevels];
    int32_t a[3][kMaxLevels];
    int32_t tlo[3][kMaxLevels];
    int32_t thi[3][kMaxLevels];
};

template <class Tab>
__device__ inline void child_counts(const Tab &C, const int32_t t[3], const int32_t ang[3], int level,
                                    int rc[3], uint32_t &tmask, int &n_nodes, int &n_groups)
{
    const int cl = level - 1;
    for (int a = 0; a < 3; ++a) {
        int lo = C.a[a][level] * ang[a];
        int c = C.n[a][cl] - lo;
        rc[a] = max(0, min(C.a[a][level], c));
    }
    tmask = 0;
    int nt = 0;
    for (int jx = 0; jx < 2; ++jx)
        for (int jy = 0; jy < 2; ++jy)
            for (int jz = 0; jz < 2; ++jz) {
                int c[3] = {2 * t[0] + jx, 2 * t[1] + jy, 2 * t[2] + jz};
                bool ok = true;
                for (int a = 0; a < 3; ++a) ok = ok && c[a] >= C.tlo[a][cl] && c[a] <= C.thi[a][cl];
                if (ok) {
                    tmask |= 1u << (4 * jx + 2 * jy + jz);
                    ++nt;
                }
            }
    n_groups = nt ? rc[0] * rc[1] * rc[2] : 0;
    n_nodes = n_groups * nt;
}

// Pops the queue until more than b children are pending (Alg. 2).  Between
// two flushes nothing is pushed, so pops come in (score desc, level asc,
// FIFO) order straight off the buckets: a leaf bucket is accepted whole (its
// lexicographically smallest leaf competes for the match), inner nodes are
// consumed in order until the pending count passes b.  Buckets below the
// running best are never touched (their nodes would be pruned).
//
// The non-empty buckets of the live range are listed first (one pass of NT
// buckets at a time).  Inner nodes are then consumed in windows of up to NT
// nodes that may span several buckets: a window is a run of consecutive
// listed inner buckets, each contributing the rest of its head chunk, and it
// extends past a bucket only if that bucket ends in this chunk (otherwise its
// next chunk comes first).  Writes the pending children as groups and zeroes
// their score slots.
// Runs of the pending batch: groups that share a level and rotation, found
// with an LDS hash on (level, angle indices).  Each hash slot owns a region
// of kRunCap entries of rgroups; slot kRunSlots is the overflow run (groups
// of a full table or a full region, scored point by point), whose region
// follows the others and holds a whole batch.
constexpr int kRunSlots = 2048;
constexpr int kRunCap = 256;
constexpr unsigned long long kRunEmpty = ~0ull;

// The run hash of the gather (only in the run-scheduled variant).
template <bool RUNS>
struct RunSmem {
    unsigned long long rkey[kRunSlots];   // level | roll << 8 | pitch << 24 | yaw << 40
    int rcnt[kRunSlots + 1];              // groups of the run
    int roff[kRunSlots + 1];              // first entry of the run in rgroups
    int lvl_groups[kMaxLevels];           // groups of the batch per level (runs of the hash table)
};
template <>
struct RunSmem<false> {
};

template <int NT, bool RUNS>
struct GatherSmem {
    int sm[NT / 64];
    int smatch[NT][6];
    int lq[NT];               // listed buckets (bucket index), in queue order
    Bucket lb[NT];            // their current head / tail
    int pre[NT];              // window: inclusive prefix of segment lengths
    LevelTables lt;           // the grid tables, indexed per lane by level
    int s_last[2];
    int s_end;
    int s_cut;
    RunSmem<RUNS> run;
};

// Where the gather leaves the batch's runs for the scoring kernel.
struct RunBufs {
    int32_t *rgroups;         // group indices by run: kRunSlots x kRunCap, then the overflow run
    int4 *items;              // item descriptors (first entry, groups, kind, slice)
};

// Slot of a run key in the LDS hash (kRunSlots when the table is full).
__device__ inline int run_slot(unsigned long long *rkey, unsigned long long key)
{
    uint32_t h = (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> 53);
    for (int p = 0; p < kRunSlots; ++p) {
        const unsigned long long old = atomicCAS(&rkey[h], kRunEmpty, key);
        if (old == kRunEmpty || old == key) return (int)h;
        h = (h + 1) & (kRunSlots - 1);
    }
    return kRunSlots;
}

__device__ inline int seg_len(const Bucket &b)
{
    return (b.head_chunk == b.tail_chunk ? b.tail_fill : kChunk) - b.head_off;
}

template <int NT, bool RUNS>
__device__ void gather(State *st, Bucket *bk, const int32_t *chunk_next, const uint4 *arena, const SearchConst &C,
                       uint4 *groups, int32_t *scores, const RunBufs &RB, GatherSmem<NT, RUNS> &sh)
{
    static_assert(NT >= kChunk, "a window must be able to hold a whole chunk segment");
    const int tid = threadIdx.x;
    const int Lp1 = C.levels + 1;
    int best = st->best;
    int have = st->have_match;
    int32_t match[6];
    for (int i = 0; i < 6; ++i) match[i] = st->match[i];
    int q = st->top_q;                 // no bucket below q holds nodes
    int64_t pend = 0;
    int ngrp = 0;
    int64_t expanded = 0, leaves = 0;
    bool cut = false;
    for (int i = tid; i < 3 * kMaxLevels; i += NT) {
        const int ax = i / kMaxLevels, l = i % kMaxLevels;
        sh.lt.n[ax][l] = C.n[ax][l];
        sh.lt.a[ax][l] = C.a[ax][l];
        sh.lt.tlo[ax][l] = C.tlo[ax][l];
        sh.lt.thi[ax][l] = C.thi[ax][l];
    }
    constexpr bool runs = RUNS;
    int hist_levels = 0;
    if constexpr (RUNS) {
        hist_levels = C.dedup_levels & ~ld_agent(&st->hist_off);
        for (int i = tid; i < kRunSlots; i += NT) sh.run.rkey[i] = kRunEmpty;
        for (int i = tid; i <= kRunSlots; i += NT) sh.run.rcnt[i] = 0;
        if (tid < kMaxLevels) sh.run.lvl_groups[tid] = 0;
    }
    __syncthreads();
    // buckets past qlim hold only scores below best (best-first); in the
    // depth-first order those lie inside every level's range and are skipped
    auto last_live = [&](int b) { return C.depth_first ? C.q_count - 1 : min((C.K - b) * Lp1 + C.levels, C.q_count - 1); };
    while (!cut && best <= C.K) {
        int qlim = last_live(best);
        if (q > qlim) break;
        // list the non-empty buckets among the next NT
        const int scan_end = min(q + NT - 1, qlim);
        {
            const int qq = q + tid;
            Bucket b = Bucket{-1, 0, -1, 0};
            if (qq <= scan_end) b = bk[qq];
            const int ne = b.head_chunk >= 0 ? 1 : 0;
            int n_list;
            const int pos = block_scan_incl<NT>(ne, sh.sm, &n_list) - ne;
            if (ne) {
                sh.lq[pos] = qq;
                sh.lb[pos] = b;
            }
            __syncthreads();
            int e = 0;
            while (e < n_list && !cut) {
                const int qe = sh.lq[e];
                if (qe > qlim) break;
                if (bucket_score(qe, C) < best) {   // depth-first only: below best, never popped
                    ++e;
                    continue;
                }
                if (bucket_level(qe, C) == 0) {
                    // a leaf bucket: accept all of it
                    const int score = bucket_score(qe, C);
                    const Bucket lbk = sh.lb[e];
                    int c = lbk.head_chunk, off = lbk.head_off;
                    int32_t mine[6] = {INT_MAX, INT_MAX, INT_MAX, INT_MAX, INT_MAX, INT_MAX};
                    while (c >= 0) {
                        const int end = c == lbk.tail_chunk ? lbk.tail_fill : kChunk;
                        for (int i = off + tid; i < end; i += NT) {
                            int32_t t[3], ang[3], lv;
                            node_unpack(arena[(int64_t)c * kChunk + i], t, ang, lv);
                            const int32_t cand[6] = {t[0], t[1], t[2], ang[0], ang[1], ang[2]};
                            if (leaf_less(cand, mine))
                                for (int k = 0; k < 6; ++k) mine[k] = cand[k];
                        }
                        leaves += end - off;
                        c = c == lbk.tail_chunk ? -1 : chunk_next[c];
                        off = 0;
                    }
                    __syncthreads();
                    for (int k = 0; k < 6; ++k) sh.smatch[tid][k] = mine[k];
                    __syncthreads();
                    for (int h = NT / 2; h > 0; h >>= 1) {
                        if (tid < h && leaf_less(sh.smatch[tid + h], sh.smatch[tid]))
                            for (int k = 0; k < 6; ++k) sh.smatch[tid][k] = sh.smatch[tid + h][k];
                        __syncthreads();
                    }
                    if (!have || score > best || leaf_less(sh.smatch[0], match))
                        for (int k = 0; k < 6; ++k) match[k] = sh.smatch[0][k];
                    __syncthreads();
                    have = 1;
                    best = score;
                    qlim = last_live(best);
                    if (tid == 0) bk[qe] = Bucket{-1, 0, -1, 0};
                    ++e;
                    continue;
                }
                // window of inner buckets e .. e + n_win - 1
                {
                    const int i = e + tid;
                    int seg = 0;
                    bool ok = false;
                    if (i < n_list) {
                        const int qi = sh.lq[i];
                        ok = qi <= qlim && bucket_level(qi, C) != 0 && bucket_score(qi, C) >= best;
                        seg = ok ? seg_len(sh.lb[i]) : 0;
                    }
                    int tot;
                    const int incl = block_scan_incl<NT>(seg, sh.sm, &tot);
                    // an entry may follow the previous one only if that one ends in its head chunk
                    bool prev_last = true;
                    if (tid > 0 && i < n_list) prev_last = sh.lb[i - 1].head_chunk == sh.lb[i - 1].tail_chunk;
                    const bool in_win = i < n_list && ok && incl <= NT && (tid == 0 || prev_last);
                    const int first_out = block_min_int<NT>(in_win ? INT_MAX : tid, sh.sm);
                    const int n_win = first_out == INT_MAX ? min(NT, n_list - e) : first_out;
                    if (tid < n_win) sh.pre[tid] = incl;
                    if (tid == 0) sh.s_end = n_win;
                    __syncthreads();
                }
                const int n_win = sh.s_end;
                const int W = sh.pre[n_win - 1];
                // node t of the window: entry j with pre[j-1] <= t < pre[j]
                int32_t t3[3] = {0, 0, 0}, ang[3] = {0, 0, 0}, lv = 0;
                int rc[3] = {0, 0, 0}, nn = 0, ng = 0;
                uint32_t tmask = 0;
                int level = 0;
                const bool valid = tid < W;
                if (valid) {
                    int lo = 0, hi = n_win - 1;
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (sh.pre[mid] > tid) hi = mid;
                        else lo = mid + 1;
                    }
                    const int j = lo;
                    const int base = j > 0 ? sh.pre[j - 1] : 0;
                    const Bucket bj = sh.lb[e + j];
                    level = bucket_level(sh.lq[e + j], C);
                    node_unpack(arena[(int64_t)bj.head_chunk * kChunk + bj.head_off + (tid - base)], t3, ang, lv);
                    child_counts(sh.lt, t3, ang, level, rc, tmask, nn, ng);
                }
                int incl_n, incl_g;
                if (C.max_children <= 64) {
                    // one scan of (children, groups) packed as nn | ng << 17: a
                    // window holds at most NT * 64 = 2^16 children, NT * 8 groups
                    int tot_p;
                    const int incl_p = block_scan_incl<NT>(nn | (ng << 17), sh.sm, &tot_p);
                    incl_n = incl_p & 0x1FFFF;
                    incl_g = incl_p >> 17;
                } else {
                    int tot_n, tot_g;
                    incl_n = block_scan_incl<NT>(nn, sh.sm, &tot_n);
                    incl_g = block_scan_incl<NT>(ng, sh.sm, &tot_g);
                }
                // pend <= b here, and the running count passes b at exactly one
                // node of the window, if any
                if (tid == 0) sh.s_cut = INT_MAX;
                __syncthreads();
                if (valid && pend + incl_n > C.batch && pend + incl_n - nn <= C.batch) sh.s_cut = tid;
                __syncthreads();
                const int cutidx = sh.s_cut;
                const int consumed = cutidx != INT_MAX ? cutidx + 1 : W;
                if (tid < consumed && ng > 0) {
                    int gi = ngrp + incl_g - ng;
                    for (int ja = 0; ja < rc[0]; ++ja)
                        for (int jb = 0; jb < rc[1]; ++jb)
                            for (int jg = 0; jg < rc[2]; ++jg) {
                                const int ra = sh.lt.a[0][level] * ang[0] + ja;
                                const int rb = sh.lt.a[1][level] * ang[1] + jb;
                                const int rg = sh.lt.a[2][level] * ang[2] + jg;
                                if constexpr (RUNS) {
                                    const unsigned long long key =
                                        (unsigned long long)(level - 1) | ((unsigned long long)ra << 8) |
                                        ((unsigned long long)rb << 24) | ((unsigned long long)rg << 40);
                                    int slot = run_slot(sh.run.rkey, key);
                                    int rank = slot < kRunSlots ? atomicAdd(&sh.run.rcnt[slot], 1) : kRunCap;
                                    if (rank >= kRunCap) {
                                        slot = kRunSlots;
                                        rank = atomicAdd(&sh.run.rcnt[kRunSlots], 1);
                                    }
                                    RB.rgroups[(int64_t)slot * kRunCap + rank] = gi;
                                }
                                groups[gi++] = make_uint4(pack16(2 * t3[0], 2 * t3[1]), pack16(2 * t3[2], ra),
                                                          pack16(rb, rg), (uint32_t)(level - 1) | (tmask << 8));
                            }
                }
                if (tid == consumed - 1) {
                    sh.s_last[0] = incl_n;
                    sh.s_last[1] = incl_g;
                }
                __syncthreads();
                pend += sh.s_last[0];
                ngrp += sh.s_last[1];
                expanded += consumed;
                // advance the window's buckets (one thread per entry)
                int next_e = e + n_win;
                if (tid < n_win) {
                    const int base = tid > 0 ? sh.pre[tid - 1] : 0;
                    const int seg = sh.pre[tid] - base;
                    const int used = min(max(consumed - base, 0), seg);
                    Bucket b = sh.lb[e + tid];
                    if (used == seg) {
                        if (b.head_chunk == b.tail_chunk) b = Bucket{-1, 0, -1, 0};
                        else {
                            b.head_chunk = chunk_next[b.head_chunk];
                            b.head_off = 0;
                        }
                    } else {
                        b.head_off += used;
                    }
                    if (used > 0) {
                        bk[sh.lq[e + tid]] = b;
                        sh.lb[e + tid] = b;
                    }
                }
                __syncthreads();
                if (cutidx != INT_MAX) {
                    cut = true;
                    break;
                }
                // the last window bucket may continue in its next chunk
                const Bucket lastb = sh.lb[e + n_win - 1];
                if (lastb.head_chunk >= 0) next_e = e + n_win - 1;
                e = next_e;
            }
            // after a cut the window's first bucket (at or before the cut) is
            // the lowest that may still hold nodes; otherwise every listed
            // bucket up to scan_end is empty or lies below the running best
            q = cut ? sh.lq[e] : scan_end + 1;
            __syncthreads();
        }
    }
    __syncthreads();
    // The batch as scoring items.  Runs of a level whose scan histogram fits
    // (C.dedup_levels, less the levels whose histogram overflowed) become
    // histogram items of at most kItemGroups groups; the other groups are
    // scored point by point, in pairs within a run, or, when fewer than
    // score_items of them are pending, in point slices.
    int n_items = 0, n_hist_items = 0, n_hist_groups = 0, n_slices = 1;
    if constexpr (RUNS) {
        constexpr int kPer = (kRunSlots + NT) / NT;    // slots per thread, the overflow slot included
        int cnt_s[kPer];
        bool hist_s[kPer];
        int xcnt = 0, hcnt = 0, hitems = 0;
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int sl = tid * kPer + i;
            int c = 0;
            bool h = false;
            if (sl < kRunSlots) {
                c = min(sh.run.rcnt[sl], kRunCap);
                if (c > 0) h = (hist_levels >> (int)(sh.run.rkey[sl] & 0xFF)) & 1;
            } else if (sl == kRunSlots) {
                c = sh.run.rcnt[sl];
            }
            cnt_s[i] = c;
            hist_s[i] = h;
            if (h) {
                hcnt += c;
                hitems += (c + kItemGroups - 1) / kItemGroups;
            } else {
                xcnt += c;
            }
            if (c > 0 && sl < kRunSlots) atomicAdd(&sh.run.lvl_groups[(int)(sh.run.rkey[sl] & 0xFF)], c);
        }
        int x_tot;
        (void)block_scan_incl<NT>(xcnt, sh.sm, &x_tot);
        const int max_s = (C.K + kScoreThreads * kUnroll - 1) / (kScoreThreads * kUnroll);
        if (x_tot > 0 && x_tot < C.score_items) n_slices = max(1, min(max_s, (C.score_items + x_tot - 1) / x_tot));
        // items of this thread's slots, then their offsets
        int mine = hitems;
#pragma unroll
        for (int i = 0; i < kPer; ++i)
            if (!hist_s[i]) mine += n_slices > 1 ? cnt_s[i] * n_slices : (cnt_s[i] + 1) / 2;
        int i_tot, h_tot;
        int at = block_scan_incl<NT>(mine, sh.sm, &i_tot) - mine;
        (void)block_scan_incl<NT>(hcnt, sh.sm, &h_tot);
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int sl = tid * kPer + i;
            const int c = cnt_s[i];
            const int first = sl * kRunCap;
            if (hist_s[i]) {
                for (int q = 0; q < c; q += kItemGroups)
                    RB.items[at++] = make_int4(first + q, min(kItemGroups, c - q), kItemHist, 0);
            } else if (n_slices > 1) {
                for (int q = 0; q < c; ++q)
                    for (int j = 0; j < n_slices; ++j) RB.items[at++] = make_int4(first + q, 1, kItemSlice, j);
            } else {
                for (int q = 0; q < c; q += 2) RB.items[at++] = make_int4(first + q, min(2, c - q), kItemPair, 0);
            }
        }
        n_items = i_tot;
        n_hist_groups = h_tot;
        int hi_tot;
        (void)block_scan_incl<NT>(hitems, sh.sm, &hi_tot);
        n_hist_items = hi_tot;
    }
    // sliced groups add their counts to zeroed scores (so does the legacy
    // scheme when fewer than score_items groups are pending)
    if (runs ? n_slices > 1 : ngrp < C.score_items)
        for (int i = tid; i < 8 * ngrp; i += NT) scores[i] = 0;
    if constexpr (RUNS) {
        if (tid < kMaxLevels) st->level_groups[tid] += sh.run.lvl_groups[tid];
    }
    if (tid == 0) {
        st->runs = runs ? 1 : 0;
        st->n_items = n_items;
        st->n_slices = n_slices;
        st->dedup_items += n_hist_items;
        st->dedup_groups += n_hist_groups;
        st->best = best;
        st->have_match = have;
        for (int i = 0; i < 6; ++i) st->match[i] = match[i];
        st->top_q = q;
        st->nodes_expanded += expanded;
        st->leaves_accepted += leaves;
        st->n_groups = ngrp;
        st->pend_nodes = pend;
        st->q_min = INT_MAX;
        st->q_max = -1;
        st->kept = 0;
        if (pend > 0) {
            st->batch = 1;
            st->flushes += 1;
            st->nodes_scored += pend;
            st->groups_scored += ngrp;
        } else {
            st->batch = 0;
            st->done = 1;
        }
    }
}

// The serial part of an iteration, one workgroup: push the scored batch,
// then (unless this is an initial-set chunk with more to come) gather the
// next one.
// LDS copies of the push's per-bucket lists (occupied buckets, their totals,
// tail chunk, fill and first new chunk), which only the serial workgroup
// writes and reads: used when the queue has at most kPushLds buckets (and
// the gather keeps no run hash), otherwise the global workspace arrays.
constexpr int kPushLds = 4096;
template <bool ON>
struct PushSmem {
    int qlist[kPushLds];
    int totals[kPushLds];
    int pT[kPushLds];
    int pf[kPushLds];
    int pc0[kPushLds];
};
template <>
struct PushSmem<false> {
};

template <int NT, bool RUNS>
struct SerialSmem {
    int sm[NT / 64];
    GatherSmem<NT, RUNS> g;
    PushSmem<!RUNS> p;
};

template <int NT, bool RUNS>
__device__ void serial_body(State *st, const SearchConst &C, Bucket *bk, uint4 *groups, int32_t *scores,
                            const PushBufs &B, const RunBufs &RB, int do_gather, SerialSmem<NT, RUNS> &sh)
{
    if (ld_agent(&st->done)) return;
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    PushBufs Bp = B;
    if constexpr (!RUNS) {
        if (C.q_count <= kPushLds) {
            Bp.qlist = sh.p.qlist;
            Bp.totals = sh.p.totals;
            Bp.pT = sh.p.pT;
            Bp.pf = sh.p.pf;
            Bp.pc0 = sh.p.pc0;
        }
    }
    if (ld_agent(&st->batch)) push_finish<NT>(st, C, bk, groups, Bp, sh.sm, sh.g.pre);
    __syncthreads();
    const uint64_t t1 = __builtin_amdgcn_s_memrealtime();
    if (threadIdx.x == 0) st->t_push += (int64_t)(t1 - t0);
    if (ld_agent(&st->done)) return;
    if (threadIdx.x == 0) st->batch = 0;
    __syncthreads();
    if (do_gather) {
        gather<NT, RUNS>(st, bk, B.chunk_next, B.arena, C, groups, scores, RB, sh.g);
        __syncthreads();
        if (threadIdx.x == 0) st->t_gather += (int64_t)(__builtin_amdgcn_s_memrealtime() - t1);
    }
}

template <bool RUNS>
__global__ __launch_bounds__(kSerialThreads) void k_serial(State *st, SearchConst C, Bucket *bk, uint4 *groups,
                                                           int32_t *scores, PushBufs B, RunBufs RB, int do_gather)
{
    __shared__ SerialSmem<kSerialThreads, RUNS> sh;
    serial_body<kSerialThreads, RUNS>(st, C, bk, groups, scores, B, RB, do_gather, sh);
}

// ------------------------------------------------------------------ persistent search loop

constexpr int kPersistThreads = 1024;   // as wide as k_serial: the serial phase runs in workgroup 0
constexpr unsigned kSpinLimit = 1u << 23;
static_assert(kPersistThreads * kUnroll <= kScanPad, "scan padding must cover a whole scoring round");

// Grid-wide barrier for a cooperative launch: arrive on bar[0], wait for the
// generation in bar[1] to move.  The wait is bounded: on timeout the error
// flag gets bit 4 and every workgroup leaves the loop.  Device-scope fences
// on both sides publish the workgroups' writes to each other.
__device__ bool grid_sync(unsigned *bar, int32_t *err, int *s_ok)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned gen = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int ok = 1;
        if (atomicAdd(&bar[0], 1u) == gridDim.x - 1) {
            __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __threadfence();
            atomicAdd(&bar[1], 1u);
        } else {
            unsigned spins = 0;
            while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                __builtin_amdgcn_s_sleep(10);
                if (++spins > kSpinLimit) {
                    atomicOr(err, 4);
                    ok = 0;
                    break;
                }
            }
        }
        __threadfence();
        *s_ok = ok && !(ld_agent(err) & 4);
    }
    __syncthreads();
    return *s_ok != 0;
}

// The whole search loop in one cooperative launch: every workgroup scores
// the pending batch, then workgroup 0 pushes it and gathers the next one.
template <int RM>
__global__ __launch_bounds__(kPersistThreads) void k_persistent(State *st, ScoreArgs A, MapView map, SearchConst C,
                                                                Bucket *bk, uint4 *groups, int32_t *scores,
                                                                PushBufs B, RunBufs RB, unsigned *bar,
                                                                int32_t max_iters)
{
    __shared__ ScoreSmem<kPersistThreads> ssh;
    __shared__ SerialSmem<kPersistThreads, false> sh;
    __shared__ int s_ok;
    for (int it = 0; it < max_iters; ++it) {
        if (ld_agent(&st->done)) break;
        score_items<RM, kPersistThreads>(st, A, map, C, ssh);
        if (!grid_sync(bar, &st->error, &s_ok)) break;
        if (blockIdx.x == 0) serial_body<kPersistThreads, false>(st, C, bk, groups, scores, B, RB, 1, sh);
        if (!grid_sync(bar, &st->error, &s_ok)) break;
    }
}

// ------------------------------------------------------------------ learned prior: batches and seed beam

// A batch already written to `groups` (initial nodes in prior order): zero
// its scores and reset the push bookkeeping.
__global__ void k_begin_batch(State *st, int32_t *scores, int32_t n_groups)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < 8 * n_groups; i += gridDim.x * blockDim.x) scores[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->n_groups = n_groups;
        st->runs = 0;
        st->batch = 1;
        st->q_min = INT_MAX;
        st->q_max = -1;
        st->kept = 0;
    }
}

// Seed beam step 1: the children of every beam node as groups, beam order
// then branching order (one wave; the beam holds at most 64 nodes).  `ds` is
// the batch header the scoring kernel reads.
__global__ __launch_bounds__(64) void k_beam_expand(BeamBuf *bb, SearchConst C, uint4 *groups, int32_t *scores,
                                                    State *st, State *ds)
{
    __shared__ int s_ng[kMaxBeam];
    const int tid = threadIdx.x;
    const int n = bb->count;
    int32_t t[3] = {0, 0, 0}, ang[3] = {0, 0, 0}, level = 0;
    int rc[3] = {0, 0, 0}, nn = 0, ng = 0;
    uint32_t tmask = 0;
    if (tid < n) {
        node_unpack(bb->nodes[tid].node, t, ang, level);
        if (level > 0) child_counts(C, t, ang, level, rc, tmask, nn, ng);
    }
    s_ng[tid] = ng;
    __syncthreads();
    int g = 0, total = 0;
    for (int i = 0; i < n; ++i) {
        if (i < tid) g += s_ng[i];
        total += s_ng[i];
    }
    if (ng > 0) {
        for (int ja = 0; ja < rc[0]; ++ja)
            for (int jb = 0; jb < rc[1]; ++jb)
                for (int jg = 0; jg < rc[2]; ++jg) {
                    const int ra = C.a[0][level] * ang[0] + ja;
                    const int rb = C.a[1][level] * ang[1] + jb;
                    const int rg = C.a[2][level] * ang[2] + jg;
                    for (int j = 0; j < 8; ++j) scores[8 * g + j] = 0;
                    groups[g++] = make_uint4(pack16(2 * t[0], 2 * t[1]), pack16(2 * t[2], ra), pack16(rb, rg),
                                             (uint32_t)(level - 1) | (tmask << 8));
                }
    }
    if (tid == 0) {
        st->nodes_expanded += n;
        ds->n_groups = total;
        ds->batch = total > 0 ? 1 : 0;
    }
}

// Seed beam step 2: among the scored children at or above the threshold,
// the `W` first in (score desc, prior key desc, position asc) order become
// the next beam; position is the child's slot (group, member), i.e. beam
// order then branching order.
__global__ __launch_bounds__(kBeamThreads) void k_beam_pick(BeamBuf *bb, int W, const uint4 *groups,
                                                            const int32_t *scores, const State *ds, State *st,
                                                            PriorConst P, const float *prior, int32_t threshold)
{
    __shared__ int s_score[kBeamSlots];
    __shared__ double s_key[kBeamSlots];
    __shared__ int s_children, s_valid;
    const int tid = threadIdx.x;
    const int n_slots = 8 * min(ds->n_groups, kBeamSlots / 8);
    if (tid == 0) {
        s_children = 0;
        s_valid = 0;
    }
    __syncthreads();
    int children = 0, valid = 0;
    for (int sl = tid; sl < n_slots; sl += kBeamThreads) {
        const uint4 G = groups[sl >> 3];
        const int j = sl & 7;
        int sc = -1;
        double key = 0.0;
        if (((G.w >> 8) >> j) & 1u) {
            ++children;
            const int v = scores[sl];
            if (v >= threshold) {
                sc = v;
                ++valid;
                key = prior_key(P, prior, (int)(G.w & 0xFF), lo16s(G.x) + ((j >> 2) & 1), hi16s(G.x) + ((j >> 1) & 1),
                                (int32_t)hi16u(G.z));
            }
        }
        s_score[sl] = sc;
        s_key[sl] = key;
    }
    atomicAdd(&s_children, children);
    atomicAdd(&s_valid, valid);
    __syncthreads();
    for (int sl = tid; sl < n_slots; sl += kBeamThreads) {
        const int sc = s_score[sl];
        if (sc < 0) continue;
        const double key = s_key[sl];
        int rank = 0;
        for (int u = 0; u < n_slots; ++u) {
            const int su = s_score[u];
            rank += su > sc || (su == sc && (s_key[u] > key || (s_key[u] == key && u < sl)));
        }
        if (rank < W) {
            const uint4 G = groups[sl >> 3];
            const int j = sl & 7;
            const int jx = (j >> 2) & 1, jy = (j >> 1) & 1, jz = j & 1;
            BeamNode b;
            b.node = make_uint4(pack16(lo16s(G.x) + jx, hi16s(G.x) + jy), pack16(lo16s(G.y) + jz, hi16u(G.y)), G.z,
                                G.w & 0xFFu);
            b.score = sc;
            b.pad = 0;
            b.key = key;
            bb->nodes[rank] = b;
        }
    }
    __syncthreads();
    if (tid == 0) {
        bb->count = min(W, s_valid);
        st->dive_scored += s_children;
    }
}

// The best beam leaf (highest score, then lexicographically smallest) seeds
// the incumbent if it reaches the running best.
__global__ void k_beam_seed(const BeamBuf *bb, State *st)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int have = 0, best = -1;
    int32_t leaf[6] = {0, 0, 0, 0, 0, 0};
    for (int i = 0; i < bb->count; ++i) {
        int32_t t[3], ang[3], level;
        node_unpack(bb->nodes[i].node, t, ang, level);
        if (level != 0) continue;
        const int32_t cand[6] = {t[0], t[1], t[2], ang[0], ang[1], ang[2]};
        const int sc = bb->nodes[i].score;
        if (!have || sc > best || (sc == best && leaf_less(cand, leaf))) {
            for (int k = 0; k < 6; ++k) leaf[k] = cand[k];
            best = sc;
            have = 1;
        }
    }
    if (!have || best < st->best) return;
    if (!st->have_match || best > st->best || leaf_less(leaf, st->match))
        for (int k = 0; k < 6; ++k) st->match[k] = leaf[k];
    st->have_match = 1;
    st->best = best;
    st->seeded = 1;
    st->seed_score = best;
}

// ------------------------------------------------------------------ host side

bool is_pow2_float(float r)
{
    int e = 0;
    float m = std::frexp(r, &e);
    return m == 0.5f;
}


}  // namespace
}  // namespace bbs

using namespace bbs;

struct bbs_workspace {
    int32_t device = 0;
    hipStream_t own_stream = nullptr;
    int64_t queue_nodes = 0;
    uint4 *arena = nullptr;
    int64_t arena_n = 0;
    int32_t *chunk_next = nullptr;
    int64_t chunk_next_n = 0;
    Bucket *buckets = nullptr;
    int64_t buckets_n = 0;
    int32_t *hist = nullptr;
    int64_t hist_n = 0;
    uint32_t *qmask = nullptr;
    int64_t qmask_n = 0;
    int32_t *qlist = nullptr;
    int64_t qlist_n = 0;
    int32_t *totals = nullptr;
    int64_t totals_n = 0;
    int32_t *pT = nullptr, *pf = nullptr, *pc0 = nullptr;
    int64_t pT_n = 0, pf_n = 0, pc0_n = 0;
    uint4 *groups = nullptr;
    int64_t groups_n = 0;
    int32_t *scores = nullptr;
    int64_t scores_n = 0;
    int32_t *hbase = nullptr;
    int64_t hbase_n = 0;
    uint4 *knode = nullptr;
    int64_t knode_n = 0;
    int32_t *kcnt = nullptr;
    int64_t kcnt_n = 0;
    int32_t *kq = nullptr;
    int64_t kq_n = 0;
    int32_t *krank = nullptr;
    int64_t krank_n = 0;
    int32_t *tile_done = nullptr;
    int64_t tile_done_n = 0;
    int32_t *ticket = nullptr;   // scoring item tickets (2 counters, zero between launches)
    int64_t ticket_n = 0;
    int32_t *rgroups = nullptr;  // runs of the pending batch and their items (see RunBufs)
    int64_t rgroups_n = 0;
    int4 *items = nullptr;
    int64_t items_n = 0;
    int32_t *gslices = nullptr;  // point slices done per group (zero between launches)
    int64_t gslices_n = 0;
    int32_t score_grid[3] = {0, 0, 0};   // resident k_score workgroups, per division mode
    float *scan = nullptr;
    int64_t scan_n = 0;
    float *scan_aos = nullptr;
    int64_t scan_aos_n = 0;
    float *scan_tmp = nullptr;
    int64_t scan_tmp_n = 0;
    uint32_t *mkeys = nullptr;
    int64_t mkeys_n = 0;
    int32_t *mhist = nullptr;
    int64_t mhist_n = 0;
    double2 *trig = nullptr;
    int64_t trig_n = 0;
    State *state = nullptr;
    int64_t state_n = 0;
    unsigned long long *maxsq = nullptr;
    int64_t maxsq_n = 0;
    BeamBuf *beam = nullptr;
    int64_t beam_n = 0;
    float *prior = nullptr;
    int64_t prior_n = 0;
    unsigned *bar = nullptr;
    int64_t bar_n = 0;
    State *dstate = nullptr;
    int64_t dstate_n = 0;
    State *host_state = nullptr;   // pinned
    State *host_state2 = nullptr;  // pinned: the second of the two in-flight search-loop checks
    hipEvent_t sync_ev[2] = {nullptr, nullptr};
    std::vector<hipEvent_t> ev;
    bool hist_dirty = true;
    // no-allocation mode (bbs_localize_noalloc): every buffer is carved from
    // one fixed device region for the duration of a call; nothing is
    // allocated or freed
    bool fixed = false;
    char *fixed_base = nullptr;
    size_t fixed_used = 0, fixed_cap = 0;
};

namespace bbs {
namespace {

// Grows a workspace buffer to at least `need` elements (contents are not
// kept).  In no-allocation mode the buffer is instead carved, 256-byte
// aligned, from the workspace's fixed region; running out of it is an
// argument error, since the caller chose the region's size.
template <class T>
bbs_status ensure(bbs_workspace *w, T *&p, int64_t &cap, int64_t need)
{
    if (p && cap >= need) return BBS_OK;
    const int64_t n = std::max<int64_t>(need, 1);
    if (w->fixed) {
        const size_t off = (w->fixed_used + 255) & ~(size_t)255;
        const size_t bytes = (size_t)n * sizeof(T);
        if (p || off > w->fixed_cap || bytes > w->fixed_cap - off)
            return fail(BBS_ERR_INVALID_ARG, "bbs_localize_noalloc: the search needs more device memory than the "
                                             "static scratch region holds (BBS_NOALLOC_SCRATCH_BYTES)");
        p = reinterpret_cast<T *>(w->fixed_base + off);
        cap = n;
        w->fixed_used = off + bytes;
        return BBS_OK;
    }
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
    void *q = nullptr;
    if (alloc_dev(&q, (size_t)n * sizeof(T))) return BBS_ERR_OOM;
    p = static_cast<T *>(q);
    cap = n;
    return BBS_OK;
}

// Status of a failed ensure(): the message is already set.
inline bbs_status ws_fail(const bbs_workspace *w) { return w->fixed ? BBS_ERR_INVALID_ARG : BBS_ERR_OOM; }

// Zeroes `bytes` (a multiple of 4) with a fill kernel rather than a memset
// node, so that the same code may be captured into a graph.
__global__ void k_zero_u32(uint32_t *p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

hipError_t zero_async(void *p, size_t bytes, hipStream_t s)
{
    const int64_t n = (int64_t)(bytes / 4);
    if (n <= 0) return hipSuccess;
    k_zero_u32<<<grid_for(n, 256, 2048), 256, 0, s>>>(static_cast<uint32_t *>(p), n);
    return hipGetLastError();
}

void free_ws(bbs_workspace *w)
{
    void *ptrs[] = {w->arena,   w->chunk_next, w->buckets, w->hist,     w->totals,  w->pT,    w->pf,
                    w->pc0,     w->groups,     w->scores,  w->kq,       w->krank,   w->hbase, w->knode,
                    w->kcnt,    w->tile_done,  w->ticket,  w->scan,     w->scan_aos, w->scan_tmp, w->mkeys,
                    w->mhist,   w->trig,       w->state,   w->maxsq,    w->beam,    w->prior, w->dstate,
                    w->bar,     w->qmask,      w->qlist,   w->rgroups,  w->items,   w->gslices};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (w->host_state) (void)hipHostFree(w->host_state);
    if (w->host_state2) (void)hipHostFree(w->host_state2);
    for (hipEvent_t e : w->sync_ev)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : w->ev) (void)hipEventDestroy(e);
    if (w->own_stream) (void)hipStreamDestroy(w->own_stream);
    delete w;
}

// Angular and translational grid (Sec. III-B Eq. (2); Sec. III-D).
bbs_status make_grid(const bbs_map *m, double dmax, const bbs_search_range *range, int translation_only, Grid &g)
{
    std::memset(&g, 0, sizeof(g));
    g.levels = m->levels;
    g.translation_only = translation_only ? 1 : 0;
    g.r = m->r;
    g.dmax = dmax;
    for (int l = 0; l <= g.levels; ++l) {
        double rl = std::ldexp((double)g.r, l);
        double c = 1.0 - (rl * rl) / (2.0 * dmax * dmax);
        if (c < -1.0) c = -1.0;
        if (c > 1.0) c = 1.0;
        g.delta[l] = std::acos(c);
    }
    for (int ax = 0; ax < 3; ++ax) {
        g.wmin[ax] = range->min[3 + ax];
        g.wmax[ax] = range->max[3 + ax];
        double W = g.wmax[ax] - g.wmin[ax];
        for (int l = 0; l <= g.levels; ++l) {
            int src = g.translation_only ? 0 : l;
            int32_t n = 1;
            if (W != 0.0) {
                double q = std::ceil(W / g.delta[src]);
                if (!(q >= 1.0)) q = 1.0;
                if (q > 65535.0)
                    return fail(BBS_ERR_INVALID_ARG, "bbs_localize: more than 65535 angular cells on an axis");
                n = (int32_t)q;
            }
            g.n[ax][l] = n;
            g.dprime[ax][l] = W / n;
        }
        g.a[ax][0] = 1;
        for (int l = 1; l <= g.levels; ++l) g.a[ax][l] = (g.n[ax][l - 1] + g.n[ax][l] - 1) / g.n[ax][l];
    }
    for (int ax = 0; ax < 3; ++ax) {
        double lo = std::ceil((double)range->min[ax] / (double)g.r);
        double hi = std::floor((double)range->max[ax] / (double)g.r);
        if (lo > hi) return fail(BBS_ERR_INVALID_ARG, "bbs_localize: a translation range holds no leaf cell");
        if (lo < -(double)kTransLimit || hi > (double)kTransLimit)
            return fail(BBS_ERR_INVALID_ARG, "bbs_localize: translation range exceeds 2^14 cells from the origin");
        g.lo[ax] = (int32_t)lo;
        g.hi[ax] = (int32_t)hi;
    }
    if (!(dmax / g.r + 4.0 < (double)(1 << 18)))
        return fail(BBS_ERR_INVALID_ARG, "bbs_localize: scan range / min_res must stay below 2^18");
    return BBS_OK;
}

// Nested angular cells (option nested_angles; not the default reading).
// Eq. (13) sets each level's cells independently and Eq. (14) takes the
// children a c + j with a = ceil(n_{l-1} / n_l) (Eq. (15)); a child cell lies
// inside its parent only when n_{l-1} = a n_l, and otherwise children drift
// from their parent's angle (a = 3 where n_{l-1} is just above 2 n_l puts
// the children of cell c at about 1.5 times its angle).  Here the grid is
// built top down: n_lmax as in Eq. (13), then a_l = ceil((W / n_l) /
// delta(r_{l-1})) and n_{l-1} = a_l n_l, so every cell splits into a_l equal
// children, each at most delta(r_{l-1}) wide.  Translation-only grids and
// axes with W = 0 are unchanged.
bbs_status nest_grid(Grid &g)
{
    if (g.translation_only) return BBS_OK;
    for (int ax = 0; ax < 3; ++ax) {
        const double W = g.wmax[ax] - g.wmin[ax];
        if (W == 0.0) continue;
        for (int l = g.levels; l >= 1; --l) {
            const double a = std::max(1.0, std::ceil((W / g.n[ax][l]) / g.delta[l - 1]));
            if (a * g.n[ax][l] > 65535.0)
                return fail(BBS_ERR_INVALID_ARG, "bbs_localize: nested angular grid with more than 65535 cells");
            g.n[ax][l - 1] = (int32_t)(a * g.n[ax][l]);
        }
        for (int l = 0; l <= g.levels; ++l) g.dprime[ax][l] = W / g.n[ax][l];
        g.a[ax][0] = 1;
        for (int l = 1; l <= g.levels; ++l) g.a[ax][l] = g.n[ax][l - 1] / g.n[ax][l];
    }
    return BBS_OK;
}

double cell_angle(const Grid &g, int ax, int c, int l)
{
    return g.wmin[ax] + g.dprime[ax][l] * ((double)c + 0.5);
}

// Box margins of the exact rotational bound (not in the paper, whose bound is
// not strictly exact under rotation, Sec. III-D).  A level-l node is scored at
// the centre rotation of its cell; the leaves below it lie within dev_ax of
// that centre per axis (their cells are [c P, (c + 1) P - 1], P the product of
// the divisions of levels 1..l), so a scan point moves by at most d_max times
// the sum of the three deviations (Rz Ry Rx changes by at most the sum of its
// angle changes in operator norm), i.e. its level-0 voxel by at most
// D = ceil((move + 1e-5 d_max + 1e-6) / r) cells (the slack covers the float
// transform) and its level-l voxel by at most e_l = ceil(D / 2^l).  Scoring
// level l against D_l grown by [-e_l, e_l]^3 then bounds every leaf below
// the node.  e_0 = 0, and every e_l = 0 on a translation-only grid.
void rotation_margins(const Grid &g, int32_t e[kMaxLevels])
{
    for (int l = 0; l < kMaxLevels; ++l) e[l] = 0;
    if (g.translation_only) return;
    for (int l = 1; l <= g.levels; ++l) {
        double sum_dev = 0.0;
        for (int ax = 0; ax < 3; ++ax) {
            int64_t P = 1;
            for (int j = 1; j <= l; ++j) P *= g.a[ax][j];
            const int64_t last = g.n[ax][0] - 1;
            double dev = 0.0;
            for (int c = 0; c < g.n[ax][l] && (int64_t)c * P <= last; ++c) {
                const int64_t i0 = (int64_t)c * P, i1 = std::min<int64_t>((int64_t)(c + 1) * P - 1, last);
                const double mid = cell_angle(g, ax, c, l);
                dev = std::max(dev, std::fabs(cell_angle(g, ax, (int)i0, 0) - mid));
                dev = std::max(dev, std::fabs(cell_angle(g, ax, (int)i1, 0) - mid));
            }
            sum_dev += dev;
        }
        const double cells = std::ceil((g.dmax * sum_dev + 1e-5 * g.dmax + 1e-6) / (double)g.r);
        e[l] = (int32_t)std::ceil(cells / std::ldexp(1.0, l));
    }
}

// The map's grown tables cover every level's margin of this grid.
bbs_status check_margins(const bbs_map *m, const Grid &g, const char *who)
{
    int32_t e[kMaxLevels];
    rotation_margins(g, e);
    for (int l = 1; l <= g.levels; ++l)
        if (e[l] > 0 && (!m->grown || m->margin[l] < e[l]))
            return fail(BBS_ERR_INVALID_ARG, std::string(who) + ": the exact rotational bound needs a margin of " +
                                                 std::to_string(e[l]) + " at level " + std::to_string(l) +
                                                 " and the map has " + std::to_string(m->margin[l]) +
                                                 " (see bbs_rotation_margins / bbs_build_map_margins)");
    return BBS_OK;
}

struct Setup {
    Grid g;
    SearchConst C;
    hipStream_t s;
    bool pow2;
    bool exact = false;       // exact rotational bound: levels >= 1 scored against the grown tables
    int rmode;                // scoring's division by r: 0 divide, 1 multiply by 1 / r, 2 r = 1
    int64_t kpad;             // scan arrays' stride: K rounded up to whole scoring rounds
    int32_t score_grid;       // k_score workgroups: as many as the device holds at once
};


// Upload the scan, derive d_max, the grid and the cos/sin tables.
bbs_status setup_search(const bbs_map *m, bbs_workspace *ws, const float *scan, int64_t k, int on_device,
                        const bbs_search_range *range, int translation_only, int32_t threshold, int64_t batch,
                        hipStream_t s, Setup &S, bool nested = false)
{
    if (k < 1 || k > (1 << 24)) return fail(BBS_ERR_INVALID_ARG, "bbs_localize: k must be in [1, 2^24]");
    if (!scan) return fail(BBS_ERR_INVALID_ARG, "bbs_localize: scan is NULL");
    if (!range) return fail(BBS_ERR_INVALID_ARG, "bbs_localize: range is NULL");
    for (int i = 0; i < 6; ++i)
        if (!std::isfinite(range->min[i]) || !std::isfinite(range->max[i]) || range->min[i] > range->max[i])
            return fail(BBS_ERR_INVALID_ARG, "bbs_localize: search range must be finite with min <= max");
    if (batch < 1 || batch > (1 << 24)) return fail(BBS_ERR_INVALID_ARG, "bbs_localize: batch_size must be in [1, 2^24]");
    S.s = s;
    if (!ws->ticket) {
        if (ensure(ws, ws->ticket, ws->ticket_n, 2)) return ws_fail(ws);
        BBS_HIP(zero_async(ws->ticket, 2 * sizeof(int32_t), s));
    }
    const int64_t kp = (k + kScanPad - 1) / kScanPad * kScanPad;
    S.kpad = kp;
    if (ensure(ws, ws->scan, ws->scan_n, 3 * kp) || ensure(ws, ws->scan_tmp, ws->scan_tmp_n, 3 * k) ||
        ensure(ws, ws->mkeys, ws->mkeys_n, k) || ensure(ws, ws->mhist, ws->mhist_n, kMortonBins) ||
        ensure(ws, ws->maxsq, ws->maxsq_n, 1))
        return ws_fail(ws);
    const float *aos = scan;
    if (!on_device) {
        if (ensure(ws, ws->scan_aos, ws->scan_aos_n, 3 * k)) return ws_fail(ws);
        BBS_HIP(hipMemcpyAsync(ws->scan_aos, scan, (size_t)k * 12, hipMemcpyHostToDevice, s));
        aos = ws->scan_aos;
    }
    BBS_HIP(zero_async(ws->maxsq, 8, s));
    k_scan_soa<<<grid_for(k, 256, 1024), 256, 0, s>>>(aos, (int32_t)k, ws->scan_tmp, ws->scan_tmp + k,
                                                       ws->scan_tmp + 2 * k, ws->maxsq);
    BBS_HIP(hipGetLastError());
    unsigned long long bits = 0;
    BBS_HIP(hipMemcpyAsync(&bits, ws->maxsq, 8, hipMemcpyDeviceToHost, s));
    BBS_HIP(hipStreamSynchronize(s));
    double maxsq;
    std::memcpy(&maxsq, &bits, 8);
    if (!std::isfinite(maxsq)) return fail(BBS_ERR_INVALID_ARG, "bbs_localize: scan has a non-finite coordinate");
    double dmax = std::sqrt(maxsq);
    bbs_status st = make_grid(m, dmax, range, translation_only, S.g);
    if (st) return st;
    if (nested && (st = nest_grid(S.g))) return st;
    {
        const float lo = -(float)dmax - 1.0f;
        const float inv_cell = (float)(1 << kMortonBits) / (2.0f * ((float)dmax + 1.0f));
        BBS_HIP(zero_async(ws->mhist, kMortonBins * sizeof(int32_t), s));
        const float *tx = ws->scan_tmp, *ty = ws->scan_tmp + k, *tz = ws->scan_tmp + 2 * k;
        k_morton_hist<<<grid_for(k, 256, 1024), 256, 0, s>>>(tx, ty, tz, (int32_t)k, lo, inv_cell, ws->mkeys,
                                                              ws->mhist);
        k_morton_offsets<<<1, 1024, 0, s>>>(ws->mhist);
        k_morton_scatter<<<grid_for(k, 256, 1024), 256, 0, s>>>(tx, ty, tz, ws->mkeys, (int32_t)k, ws->mhist, ws->scan,
                                                                 ws->scan + kp, ws->scan + 2 * kp);
        if (kp > k)
            k_scan_pad<<<grid_for(kp - k, 256, 64), 256, 0, s>>>(ws->scan, ws->scan + kp, ws->scan + 2 * kp, (int32_t)k,
                                                                 (int32_t)kp, std::ldexp(m->r, 22));
        BBS_HIP(hipGetLastError());
    }
    const Grid &g = S.g;
    SearchConst &C = S.C;
    std::memset(&C, 0, sizeof(C));
    C.levels = g.levels;
    C.K = (int32_t)k;
    std::vector<double2> trig;
    for (int ax = 0; ax < 3; ++ax)
        for (int l = 0; l <= g.levels; ++l) {
            C.n[ax][l] = g.n[ax][l];
            C.a[ax][l] = g.a[ax][l];
            C.tlo[ax][l] = g.lo[ax] >> l;
            C.thi[ax][l] = g.hi[ax] >> l;
            C.trig_off[ax][l] = (int32_t)trig.size();
            for (int c = 0; c < g.n[ax][l]; ++c) {
                double th = cell_angle(g, ax, c, l);
                trig.push_back(make_double2(std::cos(th), std::sin(th)));
            }
        }
    int32_t T = std::max<int32_t>(threshold, 0);
    if (T > C.K + 1) T = C.K + 1;
    C.threshold = T;
    C.q_count = (C.K - T + 1) * (C.levels + 1);
    if (C.q_count < 0) C.q_count = 0;
    C.n_scores = std::max<int32_t>(C.K - T + 1, 1);
    C.batch = batch;
    C.r = g.r;
    S.pow2 = is_pow2_float(g.r);
    S.rmode = g.r == 1.0f ? 2 : (S.pow2 ? 1 : 0);
    int32_t &sg = ws->score_grid[S.rmode];
    if (sg == 0) {
        int dev = 0, cus = 0, per_cu = 0;
        BBS_HIP(hipGetDevice(&dev));
        BBS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        const void *fn = S.rmode == 2   ? reinterpret_cast<const void *>(&k_score<2>)
                         : S.rmode == 1 ? reinterpret_cast<const void *>(&k_score<1>)
                                        : reinterpret_cast<const void *>(&k_score<0>);
        BBS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kScoreThreads, 0));
        sg = std::max(1, cus * std::max(1, std::min(per_cu, kScoreWgPerCu)));
    }
    S.score_grid = sg;
    C.inv_r = 1.0f / g.r;
    C.r_pow2 = S.pow2 ? 1 : 0;
    C.score_items = 2048;
    if (ensure(ws, ws->trig, ws->trig_n, (int64_t)trig.size())) return ws_fail(ws);
    BBS_HIP(hipMemcpyAsync(ws->trig, trig.data(), trig.size() * sizeof(double2), hipMemcpyHostToDevice, s));
    return BBS_OK;
}

ScoreArgs score_args(const Setup &S, bbs_workspace *ws, int32_t n_fixed, bool tile_pass)
{
    ScoreArgs A;
    A.groups = ws->groups;
    A.n_groups_fixed = n_fixed;
    A.X = ws->scan;
    A.Y = ws->scan + S.kpad;
    A.Z = ws->scan + 2 * S.kpad;
    A.trig = ws->trig;
    A.scores = ws->scores;
    A.tile_done = tile_pass ? ws->tile_done : nullptr;
    A.kq = ws->kq;
    A.krank = ws->krank;
    A.knode = ws->knode;
    A.kcnt = ws->kcnt;
    A.hist = ws->hist;
    A.qmask = ws->qmask;
    A.ticket = nullptr;
    A.rgroups = ws->rgroups;
    A.items = ws->items;
    A.gslices = ws->gslices;
    return A;
}

void launch_score(const Setup &S, const bbs_map *m, bbs_workspace *ws, State *st, int32_t n_fixed, int grid,
                  bool tile_pass)
{
    const ScoreArgs A = score_args(S, ws, n_fixed, tile_pass);
    const MapView v = S.exact ? m->view_exact() : m->view();
    if (S.C.dedup_levels) {
        if (S.rmode == 2) k_score_runs<2><<<grid, kScoreThreads, 0, S.s>>>(st, A, v, S.C);
        else if (S.rmode == 1) k_score_runs<1><<<grid, kScoreThreads, 0, S.s>>>(st, A, v, S.C);
        else k_score_runs<0><<<grid, kScoreThreads, 0, S.s>>>(st, A, v, S.C);
    } else {
        if (S.rmode == 2) k_score<2><<<grid, kScoreThreads, 0, S.s>>>(st, A, v, S.C);
        else if (S.rmode == 1) k_score<1><<<grid, kScoreThreads, 0, S.s>>>(st, A, v, S.C);
        else k_score<0><<<grid, kScoreThreads, 0, S.s>>>(st, A, v, S.C);
    }
}

int64_t max_children(const Grid &g)
{
    int64_t mc = 8;
    for (int l = 1; l <= g.levels; ++l) mc = std::max<int64_t>(mc, 8LL * g.a[0][l] * g.a[1][l] * g.a[2][l]);
    return mc;
}

PriorConst prior_const(const Grid &g, const bbs_search_range *range)
{
    PriorConst P;
    std::memset(&P, 0, sizeof(P));
    P.wmin_yaw = g.wmin[2];
    P.dprime_yaw0 = g.dprime[2][0];
    P.r = (double)g.r;
    for (int ax = 0; ax < 2; ++ax) {
        P.tmin[ax] = (double)range->min[ax];
        P.tmax[ax] = (double)range->max[ax];
        P.lo[ax] = g.lo[ax];
        P.hi[ax] = g.hi[ax];
    }
    P.n_yaw0 = g.n[2][0];
    for (int l = 0; l <= g.levels; ++l) P.a_yaw[l] = g.a[2][l];
    return P;
}

// Initial nodes (enumeration order as in k_enum_initial) sorted by
// descending prior key, ties in enumeration order, as one-node groups, with
// their keys.
struct KeyedGroup {
    double key;
    uint4 grp;
};

std::vector<KeyedGroup> prior_order(const Grid &g, const PriorConst &P, const float *prior)
{
    const int L = g.levels;
    std::vector<KeyedGroup> items;
    const int32_t P0[3] = {g.lo[0] >> (L + 1), g.lo[1] >> (L + 1), g.lo[2] >> (L + 1)};
    const int32_t P1[3] = {g.hi[0] >> (L + 1), g.hi[1] >> (L + 1), g.hi[2] >> (L + 1)};
    for (int32_t px = P0[0]; px <= P1[0]; ++px)
        for (int32_t py = P0[1]; py <= P1[1]; ++py)
            for (int32_t pz = P0[2]; pz <= P1[2]; ++pz)
                for (int32_t ia = 0; ia < g.n[0][L]; ++ia)
                    for (int32_t ib = 0; ib < g.n[1][L]; ++ib)
                        for (int32_t ig = 0; ig < g.n[2][L]; ++ig)
                            for (int j = 0; j < 8; ++j) {
                                const int jx = (j >> 2) & 1, jy = (j >> 1) & 1, jz = j & 1;
                                const int32_t t[3] = {2 * px + jx, 2 * py + jy, 2 * pz + jz};
                                bool ok = true;
                                for (int a = 0; a < 3; ++a) ok = ok && t[a] >= (g.lo[a] >> L) && t[a] <= (g.hi[a] >> L);
                                if (!ok) continue;
                                const double key = prior_key(P, prior, L, t[0], t[1], ig);
                                const uint4 grp = make_uint4(pack16(2 * px, 2 * py), pack16(2 * pz, ia), pack16(ib, ig),
                                                             (uint32_t)L | ((1u << j) << 8));
                                items.push_back(KeyedGroup{key, grp});
                            }
    std::stable_sort(items.begin(), items.end(),
                     [](const KeyedGroup &a, const KeyedGroup &b) { return a.key > b.key; });
    return items;
}

}  // namespace
}  // namespace bbs

extern "C" void bbs_default_options(bbs_options *opt)
{
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->batch_size = 10000;
}

extern "C" bbs_status bbs_workspace_create(int64_t max_queue_nodes, bbs_workspace **out)
{
    if (!out) return fail(BBS_ERR_INVALID_ARG, "bbs_workspace_create: out is NULL");
    *out = nullptr;
    if (max_queue_nodes < 0 || max_queue_nodes > ((int64_t)1 << 31) - 1)
        return fail(BBS_ERR_INVALID_ARG, "bbs_workspace_create: max_queue_nodes must be in [0, 2^31)");
    bbs_workspace *w = new bbs_workspace();
    (void)hipGetDevice(&w->device);
    w->queue_nodes = max_queue_nodes ? max_queue_nodes : kDefaultQueueNodes;
    hipError_t e = hipHostMalloc((void **)&w->host_state, sizeof(State), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&w->host_state2, sizeof(State), hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        free_ws(w);
        return fail(BBS_ERR_OOM, "bbs_workspace_create: pinned host allocation failed");
    }
    e = hipStreamCreateWithFlags(&w->own_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        free_ws(w);
        return hip_fail(e, "hipStreamCreateWithFlags");
    }
    for (hipEvent_t &ev : w->sync_ev) {
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            free_ws(w);
            return hip_fail(e, "hipEventCreateWithFlags");
        }
    }
    *out = w;
    return BBS_OK;
}

extern "C" void bbs_workspace_free(bbs_workspace *ws)
{
    if (ws) free_ws(ws);
}

namespace {

struct WsGuard {
    bbs_workspace *w = nullptr;
    ~WsGuard()
    {
        if (w) free_ws(w);
    }
};

double ms_since(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

namespace {

// The search of bbs_localize on a prepared workspace (growing buffers, or a
// fixed region in no-allocation mode, which also checks the end of the
// search synchronously instead of through events and pinned memory).
bbs_status localize_impl(const bbs_map *map, bbs_workspace *ws, const float *scan_xyz, int64_t k,
                         int32_t scan_on_device, const bbs_search_range *range, int32_t score_threshold,
                         const bbs_options &o, bbs_result *out)
{
    const auto t_start = std::chrono::steady_clock::now();
    hipStream_t s = o.stream ? static_cast<hipStream_t>(o.stream) : ws->own_stream;
    Setup S;
    if (o.nested_angles != 0 && o.nested_angles != 1)
        return fail(BBS_ERR_INVALID_ARG, "bbs_localize: nested_angles must be 0 or 1");
    bbs_status st = setup_search(map, ws, scan_xyz, k, scan_on_device, range, o.translation_only, score_threshold,
                                 o.batch_size, s, S, o.nested_angles != 0);
    if (st) return st;
    if (o.score_items < 0 || o.score_items > (1 << 20))
        return fail(BBS_ERR_INVALID_ARG, "bbs_localize: score_items must be in [0, 2^20]");
    if (o.score_items > 0) S.C.score_items = o.score_items;
    if (o.strategy != 0 && o.strategy != 1)
        return fail(BBS_ERR_INVALID_ARG, "bbs_localize: strategy must be 0 (best first) or 1 (depth first)");
    S.C.depth_first = o.strategy;
    if (o.rot_exact != 0 && o.rot_exact != 1) return fail(BBS_ERR_INVALID_ARG, "bbs_localize: rot_exact must be 0 or 1");
    if (o.rot_exact) {
        if ((st = check_margins(map, S.g, "bbs_localize"))) return st;
        S.exact = true;
    }
    const Grid &g = S.g;
    const SearchConst &C = S.C;
    const int L = g.levels;

    // virtual cells one level above the top (initial-set enumeration)
    int32_t P0[3], PN[3];
    for (int a = 0; a < 3; ++a) {
        P0[a] = g.lo[a] >> (L + 1);
        PN[a] = (g.hi[a] >> (L + 1)) - P0[a] + 1;
    }
    const int64_t n_rot_top = (int64_t)g.n[0][L] * g.n[1][L] * g.n[2][L];
    const int64_t n_init_groups = (int64_t)PN[0] * PN[1] * PN[2] * n_rot_top;
    int64_t init_nodes = 0;
    {
        int64_t cnt[3];
        for (int a = 0; a < 3; ++a) cnt[a] = (int64_t)(g.hi[a] >> L) - (g.lo[a] >> L) + 1;
        init_nodes = cnt[0] * cnt[1] * cnt[2] * n_rot_top;
    }
    const int64_t mc = max_children(g);
    S.C.max_children = (int32_t)std::min<int64_t>(mc, INT32_MAX);
    const int64_t cap_groups = std::max<int64_t>(o.batch_size + mc, 4096);
    const int64_t n_tiles = (cap_groups + kTileGroups - 1) / kTileGroups;
    // levels whose runs are scored through the scan's voxel histogram: from
    // hist_min_level up (off by default; -1: from level 0), where the packed
    // voxel fits (|v| < 512), the 16-bit counts cannot overflow and the run
    // ranks fit 20 bits
    {
        const int lo_l = o.hist_min_level > 0 ? o.hist_min_level : (o.hist_min_level < 0 ? 0 : 99);
        S.C.dedup_levels = 0;
        if (k <= 65535 && cap_groups < (1 << 20))
            for (int l = lo_l; l <= L; ++l)
                if ((g.dmax / (double)g.r + 2.0) / (double)(1 << l) < 500.0) S.C.dedup_levels |= 1 << l;
    }
    const int64_t qn = std::max<int32_t>(C.q_count, 1);
    if (ensure(ws, ws->groups, ws->groups_n, cap_groups) || ensure(ws, ws->scores, ws->scores_n, 8 * cap_groups) ||
        ensure(ws, ws->kq, ws->kq_n, n_tiles * kTileSlots) || ensure(ws, ws->knode, ws->knode_n, n_tiles * kTileSlots) ||
        ensure(ws, ws->kcnt, ws->kcnt_n, n_tiles) || ensure(ws, ws->hbase, ws->hbase_n, n_tiles * qn) ||
        ensure(ws, ws->krank, ws->krank_n, n_tiles * kTileSlots) || ensure(ws, ws->totals, ws->totals_n, qn) ||
        ensure(ws, ws->pT, ws->pT_n, qn) || ensure(ws, ws->pf, ws->pf_n, qn) || ensure(ws, ws->pc0, ws->pc0_n, qn) ||
        ensure(ws, ws->buckets, ws->buckets_n, qn) || ensure(ws, ws->state, ws->state_n, 1) ||
        ensure(ws, ws->rgroups, ws->rgroups_n, (int64_t)kRunSlots * kRunCap + cap_groups) ||
        ensure(ws, ws->items, ws->items_n, 2 * cap_groups + S.C.score_items + 4 * (kRunSlots + 1)))
        return ws_fail(ws);
    if (!ws->gslices || ws->gslices_n < cap_groups) {
        if (ensure(ws, ws->gslices, ws->gslices_n, cap_groups)) return ws_fail(ws);
        ws->hist_dirty = true;
    }
    if (!ws->tile_done || ws->tile_done_n < n_tiles) {
        if (ensure(ws, ws->tile_done, ws->tile_done_n, n_tiles)) return ws_fail(ws);
        ws->hist_dirty = true;
    }
    if (!ws->hist || ws->hist_n < n_tiles * qn) {
        if (ensure(ws, ws->hist, ws->hist_n, n_tiles * qn)) return ws_fail(ws);
        ws->hist_dirty = true;
    }
    if (!ws->qmask || ws->qmask_n < qn / 32 + 1) {
        if (ensure(ws, ws->qmask, ws->qmask_n, qn / 32 + 1) || ensure(ws, ws->qlist, ws->qlist_n, qn)) return ws_fail(ws);
        ws->hist_dirty = true;
    }
    // the node queue: the workspace's capacity, or in no-allocation mode
    // whatever the fixed region has left once the small buffers that a
    // prior or the persistent loop may need have been carved too
    int64_t chunk_cap = std::max<int64_t>(ws->queue_nodes / kChunk, 16);
    if (ws->fixed) {
        if (ensure(ws, ws->beam, ws->beam_n, 1) || ensure(ws, ws->dstate, ws->dstate_n, 1) ||
            ensure(ws, ws->prior, ws->prior_n, 1088) || ensure(ws, ws->bar, ws->bar_n, 2))
            return ws_fail(ws);
        const size_t used = ((ws->fixed_used + 255) & ~(size_t)255) + 512;
        const size_t left = ws->fixed_cap > used ? ws->fixed_cap - used : 0;
        chunk_cap = std::min<int64_t>((int64_t)(left / ((size_t)kChunk * sizeof(uint4) + sizeof(int32_t))),
                                      ws->queue_nodes / kChunk);
        if (chunk_cap < 16)
            return fail(BBS_ERR_INVALID_ARG, "bbs_localize_noalloc: the static scratch region leaves no room for "
                                             "the node queue at this scan size and batch size");
        ws->hist_dirty = true;   // the region keeps whatever the last call left in it
    }
    if (ensure(ws, ws->arena, ws->arena_n, chunk_cap * kChunk) ||
        ensure(ws, ws->chunk_next, ws->chunk_next_n, chunk_cap))
        return ws_fail(ws);
    if (ws->hist_dirty) {
        BBS_HIP(zero_async(ws->qmask, (size_t)ws->qmask_n * 4, s));
        BBS_HIP(zero_async(ws->hist, (size_t)ws->hist_n * 4, s));
        BBS_HIP(zero_async(ws->tile_done, (size_t)ws->tile_done_n * 4, s));
        BBS_HIP(zero_async(ws->gslices, (size_t)ws->gslices_n * 4, s));
        BBS_HIP(zero_async(ws->ticket, 2 * sizeof(int32_t), s));
        ws->hist_dirty = false;
    }
    k_fill_buckets<<<grid_for(qn, 256, 4096), 256, 0, s>>>(ws->buckets, (int32_t)qn);

    State h;
    std::memset(&h, 0, sizeof(h));
    h.best = C.threshold;
    h.top_q = 0;
    h.chunk_cap = (int32_t)std::min<int64_t>(chunk_cap, INT_MAX);
    h.q_min = INT_MAX;
    h.q_max = -1;
    BBS_HIP(hipMemcpyAsync(ws->state, &h, sizeof(State), hipMemcpyHostToDevice, s));

    const bool prof = o.profile > 0;
    const int64_t prof_every = prof ? o.profile : 1;   // time every prof_every-th scoring launch
    int64_t score_li = 0;                                // scoring launches issued so far
    int64_t ev_used = 0;
    auto record = [&](int64_t i) -> hipError_t {
        while ((int64_t)ws->ev.size() <= i) {
            hipEvent_t e;
            hipError_t err = hipEventCreate(&e);
            if (err != hipSuccess) return err;
            ws->ev.push_back(e);
        }
        return hipEventRecord(ws->ev[i], s);
    };
    const int score_grid = S.score_grid;
    PushBufs B;
    B.kq = ws->kq;
    B.krank = ws->krank;
    B.hist = ws->hist;
    B.qmask = ws->qmask;
    B.qlist = ws->qlist;
    B.totals = ws->totals;
    B.pT = ws->pT;
    B.pf = ws->pf;
    B.pc0 = ws->pc0;
    B.chunk_next = ws->chunk_next;
    B.arena = ws->arena;
    B.hbase = ws->hbase;
    B.knode = ws->knode;
    B.kcnt = ws->kcnt;
    RunBufs RB;
    RB.rgroups = ws->rgroups;
    RB.items = ws->items;
    auto serial = [&](int do_gather) {
        if (C.dedup_levels)
            k_serial<true><<<1, kSerialThreads, 0, s>>>(ws->state, C, ws->buckets, ws->groups, ws->scores, B, RB,
                                                         do_gather);
        else
            k_serial<false><<<1, kSerialThreads, 0, s>>>(ws->state, C, ws->buckets, ws->groups, ws->scores, B, RB,
                                                          do_gather);
    };
    const double t_setup = ms_since(t_start);

    // prior (learned proposal): usable only if every logit is finite
    bool use_prior = o.prior != nullptr;
    for (int i = 0; use_prior && i < 1088; ++i) use_prior = std::isfinite(o.prior[i]);
    // beam width: at most 64, at most kBeamSlots children per step, and never
    // more children than the group buffer holds
    const int beam_w = use_prior ? (int)std::max<int64_t>(0, std::min<int64_t>({(int64_t)o.seed_beam, kMaxBeam,
                                                                                kBeamSlots / mc,
                                                                                cap_groups / std::max<int64_t>(1, mc / 8)}))
                                 : 0;
    const PriorConst PC = prior_const(g, range);
    std::vector<KeyedGroup> ordered;
    std::vector<uint4> ordered_groups;
    if (use_prior) {
        ordered = prior_order(g, PC, o.prior);
        ordered_groups.resize(ordered.size());
        for (size_t i = 0; i < ordered.size(); ++i) ordered_groups[i] = ordered[i].grp;
    }
    struct BeamCand {
        int32_t score;
        double key;
        int64_t pos;
    };
    std::vector<BeamCand> cands;      // initial nodes reaching the threshold (pos: place in the prior order)

    // initial set, in chunks of the group buffer; the last chunk's serial
    // kernel also gathers the first batch of the search (unless the beam comes first)
    int64_t init_chunks = 0;
    const int64_t n_groups_init = use_prior ? (int64_t)ordered.size() : n_init_groups;
    for (int64_t g0 = 0; g0 < n_groups_init; g0 += cap_groups) {
        const int32_t cnt = (int32_t)std::min<int64_t>(cap_groups, n_groups_init - g0);
        const bool last = g0 + cnt >= n_groups_init;
        if (use_prior) {
            BBS_HIP(hipMemcpyAsync(ws->groups, ordered_groups.data() + g0, (size_t)cnt * sizeof(uint4),
                                   hipMemcpyHostToDevice, s));
            k_begin_batch<<<grid_for(8 * (int64_t)cnt, 256, 1024), 256, 0, s>>>(ws->state, ws->scores, cnt);
        } else {
            k_enum_initial<<<grid_for(cnt, 256, 4096), 256, 0, s>>>(ws->groups, ws->scores, g0, cnt, C, P0[0], P0[1],
                                                                     P0[2], PN[1], PN[2], ws->state);
        }
        const bool timed = prof && score_li++ % prof_every == 0;
        if (timed) BBS_HIP(record(ev_used++));
        launch_score(S, map, ws, ws->state, 0, score_grid, true);
        if (timed) BBS_HIP(record(ev_used++));
        if (beam_w > 0) {
            std::vector<int32_t> sc((size_t)cnt * 8);
            BBS_HIP(hipMemcpyAsync(sc.data(), ws->scores, sc.size() * 4, hipMemcpyDeviceToHost, s));
            BBS_HIP(hipStreamSynchronize(s));
            for (int32_t i = 0; i < cnt; ++i) {
                const uint4 G = ordered_groups[(size_t)(g0 + i)];
                const int j = __builtin_ctz((G.w >> 8) & 0xFF);
                const int32_t v = sc[(size_t)i * 8 + j];
                if (v >= C.threshold) cands.push_back(BeamCand{v, ordered[(size_t)(g0 + i)].key, g0 + i});
            }
        }
        serial(last && cands.empty() ? 1 : 0);
        ++init_chunks;
    }
    int beam_used = 0;
    if (!cands.empty()) {
        // initial beam: the beam_w best by (score desc, key desc, position asc)
        const size_t W = std::min(cands.size(), (size_t)beam_w);
        std::partial_sort(cands.begin(), cands.begin() + W, cands.end(), [](const BeamCand &a, const BeamCand &b) {
            if (a.score != b.score) return a.score > b.score;
            if (a.key != b.key) return a.key > b.key;
            return a.pos < b.pos;
        });
        BeamBuf hb;
        std::memset(&hb, 0, sizeof(hb));
        hb.count = (int32_t)W;
        for (size_t i = 0; i < W; ++i) {
            const uint4 G = ordered_groups[(size_t)cands[i].pos];
            const int j = __builtin_ctz((G.w >> 8) & 0xFF);
            const int jx = (j >> 2) & 1, jy = (j >> 1) & 1, jz = j & 1;
            hb.nodes[i].node = make_uint4(pack16(lo16s(G.x) + jx, hi16s(G.x) + jy), pack16(lo16s(G.y) + jz, hi16u(G.y)),
                                          G.z, G.w & 0xFFu);
            hb.nodes[i].score = cands[i].score;
            hb.nodes[i].key = cands[i].key;
        }
        if (ensure(ws, ws->beam, ws->beam_n, 1) || ensure(ws, ws->dstate, ws->dstate_n, 1) ||
            ensure(ws, ws->prior, ws->prior_n, 1088))
            return ws_fail(ws);
        BBS_HIP(hipMemcpyAsync(ws->beam, &hb, sizeof(hb), hipMemcpyHostToDevice, s));
        BBS_HIP(hipMemcpyAsync(ws->prior, o.prior, 1088 * sizeof(float), hipMemcpyHostToDevice, s));
        BBS_HIP(zero_async(ws->dstate, sizeof(State), s));
        for (int step = 0; step < L; ++step) {
            k_beam_expand<<<1, 64, 0, s>>>(ws->beam, C, ws->groups, ws->scores, ws->state, ws->dstate);
            launch_score(S, map, ws, ws->dstate, 0, score_grid, false);
            k_beam_pick<<<1, kBeamThreads, 0, s>>>(ws->beam, beam_w, ws->groups, ws->scores, ws->dstate, ws->state, PC,
                                                   ws->prior, C.threshold);
        }
        k_beam_seed<<<1, 64, 0, s>>>(ws->beam, ws->state);
        serial(1);
        beam_used = beam_w;
        // the host copies above read pageable memory; finish them before hb goes away
        BBS_HIP(hipStreamSynchronize(s));
    }
    BBS_HIP(hipGetLastError());
    BBS_HIP(hipMemcpyAsync(ws->host_state, ws->state, sizeof(State), hipMemcpyDeviceToHost, s));
    BBS_HIP(hipStreamSynchronize(s));
    const int64_t initial_kept = ws->host_state->pushed;
    const bool init_done = ws->host_state->done != 0;
    const double t_init = ms_since(t_start);
    if (ws->host_state->error) {
        ws->hist_dirty = true;
        return fail(BBS_ERR_QUEUE_OVERFLOW, "bbs_localize: node queue capacity exceeded by the initial set");
    }

    // persistent search loop: one cooperative launch runs every iteration
    bool persistent_used = false;
    if (o.persistent && !init_done) {
        if (ensure(ws, ws->bar, ws->bar_n, 2)) return ws_fail(ws);
        BBS_HIP(zero_async(ws->bar, 2 * sizeof(unsigned), s));
        int dev = 0, cus = 0, per_cu = 0;
        BBS_HIP(hipGetDevice(&dev));
        BBS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        const void *fn = S.rmode == 2   ? reinterpret_cast<const void *>(&k_persistent<2>)
                         : S.rmode == 1 ? reinterpret_cast<const void *>(&k_persistent<1>)
                                        : reinterpret_cast<const void *>(&k_persistent<0>);
        hipError_t oe = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kPersistThreads, 0);
        if (oe == hipSuccess && per_cu > 0) {
            ScoreArgs A = score_args(S, ws, 0, true);
            A.ticket = ws->ticket;            // items to whichever workgroup asks next
            MapView v = S.exact ? map->view_exact() : map->view();
            SearchConst Cv = C;
            State *stp = ws->state;
            Bucket *bkp = ws->buckets;
            uint4 *gp = ws->groups;
            int32_t *sp = ws->scores;
            unsigned *barp = ws->bar;
            int32_t max_it = 1 << 24;
            void *args[] = {&stp, &A, &v, &Cv, &bkp, &gp, &sp, &B, &RB, &barp, &max_it};
            const int grid = cus * std::min(per_cu, 4);
            oe = hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kPersistThreads), args, 0, s);
            if (oe == hipSuccess) persistent_used = true;
        }
        if (!persistent_used) (void)hipGetLastError();
        else {
            BBS_HIP(hipMemcpyAsync(ws->host_state, ws->state, sizeof(State), hipMemcpyDeviceToHost, s));
            BBS_HIP(hipStreamSynchronize(s));
            if (ws->host_state->error & 4) {
                ws->hist_dirty = true;
                return fail(BBS_ERR_INTERNAL, "bbs_localize: persistent kernel barrier timed out");
            }
        }
    }

    // graph path: the kItersPerSync iterations are captured once and replayed
    bool graph_used = false;
    if (o.graph && !prof && !persistent_used && !init_done) {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        hipError_t ge = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        if (ge == hipSuccess) {
            for (int it = 0; it < kItersPerSync; ++it) {
                launch_score(S, map, ws, ws->state, 0, score_grid, true);
                serial(1);
            }
            ge = hipStreamEndCapture(s, &graph);
        }
        if (ge == hipSuccess) ge = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (ge == hipSuccess) {
            graph_used = true;
            for (int64_t rounds = 0;; ++rounds) {
                if (rounds * kItersPerSync >= ((int64_t)1 << 26)) {
                    ge = hipErrorUnknown;
                    break;
                }
                ge = hipGraphLaunch(exec, s);
                if (ge == hipSuccess) ge = hipMemcpyAsync(ws->host_state, ws->state, sizeof(State), hipMemcpyDeviceToHost, s);
                if (ge == hipSuccess) ge = hipStreamSynchronize(s);
                if (ge != hipSuccess || ws->host_state->done || ws->host_state->error) break;
            }
        }
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (ge != hipSuccess) {
            if (graph_used) {
                ws->hist_dirty = true;
                return hip_fail(ge, "bbs_localize: graph replay");
            }
            (void)hipGetLastError();   // capture not available on this stream: plain launches
        }
    }

    // search loop; every iteration before the last pops at least one node, so
    // the cap only guards against a broken queue.  Groups of kItersPerSync
    // iterations go out two at a time: the next group is queued before the
    // host reads the state after the previous one, so the device never waits
    // for that check.  Iterations queued after the search is done return at
    // once, and the state after the last group is the final one.
    const int64_t max_iters = (int64_t)1 << 26;
    if (!persistent_used && !graph_used && !init_done && ws->fixed) {
        // no events and no pinned memory: every two groups of iterations end
        // with a synchronous read of the state
        for (int64_t iters = 0;; iters += 2 * kItersPerSync) {
            if (iters >= max_iters) {
                BBS_HIP(hipStreamSynchronize(s));
                return fail(BBS_ERR_INTERNAL, "bbs_localize: search did not terminate");
            }
            for (int it = 0; it < 2 * kItersPerSync; ++it) {
                launch_score(S, map, ws, ws->state, 0, score_grid, true);
                serial(1);
            }
            BBS_HIP(hipGetLastError());
            BBS_HIP(hipMemcpyAsync(ws->host_state, ws->state, sizeof(State), hipMemcpyDeviceToHost, s));
            BBS_HIP(hipStreamSynchronize(s));
            if (ws->host_state->done || ws->host_state->error) break;
        }
    } else if (!persistent_used && !graph_used && !init_done) {
        State *slot[2] = {ws->host_state, ws->host_state2};
        auto issue = [&](int k) -> bbs_status {
            for (int it = 0; it < kItersPerSync; ++it) {
                const bool timed = prof && score_li++ % prof_every == 0;
                if (timed) BBS_HIP(record(ev_used++));
                launch_score(S, map, ws, ws->state, 0, score_grid, true);
                if (timed) BBS_HIP(record(ev_used++));
                serial(1);
            }
            BBS_HIP(hipGetLastError());
            BBS_HIP(hipMemcpyAsync(slot[k], ws->state, sizeof(State), hipMemcpyDeviceToHost, s));
            BBS_HIP(hipEventRecord(ws->sync_ev[k], s));
            return BBS_OK;
        };
        bbs_status ist = issue(0);
        if (ist) return ist;
        int64_t iters = kItersPerSync;
        for (int cur = 0;; cur = 1 - cur) {
            if (iters >= max_iters) {
                BBS_HIP(hipStreamSynchronize(s));
                ws->hist_dirty = true;
                return fail(BBS_ERR_INTERNAL, "bbs_localize: search did not terminate");
            }
            ist = issue(1 - cur);
            if (ist) return ist;
            iters += kItersPerSync;
            BBS_HIP(hipEventSynchronize(ws->sync_ev[cur]));
            if (slot[cur]->done || slot[cur]->error) {
                BBS_HIP(hipEventSynchronize(ws->sync_ev[1 - cur]));
                if (slot[1 - cur] != ws->host_state) *ws->host_state = *slot[1 - cur];
                break;
            }
        }
    }
    const State &fs = *ws->host_state;
    if (fs.error) {
        ws->hist_dirty = true;
        return fail(BBS_ERR_QUEUE_OVERFLOW, fs.error == 1 ? "bbs_localize: node queue capacity exceeded"
                                                          : "bbs_localize: run table capacity exceeded");
    }
    const double t_loop = ms_since(t_start);

    out->found = fs.have_match ? 1 : 0;
    out->score = fs.have_match ? fs.best : 0;
    if (fs.have_match) {
        for (int i = 0; i < 6; ++i) out->leaf[i] = fs.match[i];
        for (int a = 0; a < 3; ++a) {
            out->pose[a] = (float)((double)g.r * fs.match[a]);
            out->pose[3 + a] = (float)cell_angle(g, a, fs.match[3 + a], 0);
        }
    }
    out->nodes_expanded = fs.nodes_expanded;
    out->nodes_scored = init_nodes + fs.nodes_scored + fs.dive_scored;
    out->prior_used = use_prior ? 1 : 0;
    out->seed_beam_used = beam_used;
    out->persistent_used = persistent_used ? 1 : 0;
    out->seeded = fs.seeded;
    out->serial_ms[0] = (double)fs.t_push * 1e-5;
    out->serial_ms[1] = (double)fs.t_gather * 1e-5;
    out->serial_ms[2] = (double)fs.t_push_prefix * 1e-5;
    out->serial_ms[3] = (double)fs.t_push_alloc * 1e-5;
    out->seed_score = fs.seeded ? fs.seed_score : 0;
    for (int l = 0; l < kMaxLevels; ++l) out->level_groups[l] = fs.level_groups[l];
    out->hist_groups = fs.dedup_groups;
    out->hist_items = fs.dedup_items;
    out->hist_fallbacks = fs.hist_fallbacks;
    out->hist_off = fs.hist_off;
    out->flushes = fs.flushes;
    out->leaves_accepted = fs.leaves_accepted;
    out->initial_size = init_nodes;
    out->initial_kept = initial_kept;
    out->score_pairs = out->nodes_scored * k;
    out->score_groups = n_init_groups + fs.groups_scored;
    if (prof) {
        // every iteration before the one that found the queue exhausted scored a batch
        // (event pair i brackets launch i * prof_every; the total is the mean
        // of the timed launches times the number of launches)
        int64_t launches = init_chunks + (persistent_used ? 0 : fs.flushes);
        double total = 0.0;
        int64_t timed = 0;
        for (int64_t i = 0; i * prof_every < launches && 2 * i + 1 < ev_used; ++i) {
            float ms = 0.0f;
            BBS_HIP(hipEventElapsedTime(&ms, ws->ev[2 * i], ws->ev[2 * i + 1]));
            total += ms;
            ++timed;
        }
        out->score_kernel_ms = timed > 0 ? total / (double)timed * (double)launches : 0.0;
        out->score_launches = launches;
    }
    out->phase_ms[0] = t_setup;
    out->phase_ms[1] = t_init - t_setup;
    out->phase_ms[2] = t_loop - t_init;
    out->phase_ms[3] = ms_since(t_start);
    return BBS_OK;
}

// Static scratch of bbs_localize_noalloc: one copy per GPU, held until the
// process ends.  Host code never passes `scratch` itself to a kernel (on the
// host it is only a stand-in for the symbol); it uses the device address
// that hipGetSymbolAddress returns for the current device.
constexpr size_t kNoAllocBytes = (size_t)BBS_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch, looked up once per device.
bbs_status scratch_for_current_device(void **out)
{
    int dev = 0;
    BBS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(BBS_ERR_DEVICE, "bbs_localize_noalloc: device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return BBS_OK;
}

}  // namespace

extern "C" bbs_status bbs_localize(const bbs_map *map, bbs_workspace *ws, const float *scan_xyz, int64_t k,
                                   int32_t scan_on_device, const bbs_search_range *range, int32_t score_threshold,
                                   const bbs_options *opt, bbs_result *out)
{
    if (!out) return fail(BBS_ERR_INVALID_ARG, "bbs_localize: out is NULL");
    std::memset(out, 0, sizeof(*out));
    if (!map) return fail(BBS_ERR_INVALID_ARG, "bbs_localize: map is NULL");
    bbs_options o;
    bbs_default_options(&o);
    if (opt) o = *opt;
    WsGuard tmp;
    if (!ws) {
        bbs_status st = bbs_workspace_create(0, &tmp.w);
        if (st) return st;
        ws = tmp.w;
    }
    return localize_impl(map, ws, scan_xyz, k, scan_on_device, range, score_threshold, o, out);
}

extern "C" bbs_status bbs_localize_noalloc(const bbs_map *map, const float *scan_xyz, int64_t k,
                                           int32_t scan_on_device, const bbs_search_range *range,
                                           int32_t score_threshold, const bbs_options *opt, bbs_result *out)
{
    if (!out) return fail(BBS_ERR_INVALID_ARG, "bbs_localize_noalloc: out is NULL");
    std::memset(out, 0, sizeof(*out));
    if (!map) return fail(BBS_ERR_INVALID_ARG, "bbs_localize_noalloc: map is NULL");
    bbs_options o;
    bbs_default_options(&o);
    if (opt) o = *opt;
    if (o.profile != 0 || o.graph != 0)
        return fail(BBS_ERR_INVALID_ARG, "bbs_localize_noalloc: profile and graph need allocations; set both to 0");
    void *base = nullptr;
    bbs_status st = scratch_for_current_device(&base);
    if (st) return st;
    // a workspace that lives for this call only: its buffers are carved from
    // the scratch, its host state is ordinary memory, it owns no stream
    bbs_workspace w;
    State host[2];
    w.fixed = true;
    w.fixed_base = static_cast<char *>(base);
    w.fixed_cap = kNoAllocBytes;
    w.queue_nodes = kDefaultQueueNodes;
    w.host_state = &host[0];
    w.host_state2 = &host[1];
    (void)hipGetDevice(&w.device);
    return localize_impl(map, &w, scan_xyz, k, scan_on_device, range, score_threshold, o, out);
}

extern "C" bbs_status bbs_rotation_margins(float min_res, int32_t levels, double d_max, const bbs_search_range *range,
                                           int32_t nested_angles, int32_t *margins)
{
    if (!range || !margins) return fail(BBS_ERR_INVALID_ARG, "bbs_rotation_margins: NULL argument");
    if (!(min_res > 0.0f) || !std::isfinite(min_res) || levels < 0 || levels >= kMaxLevels)
        return fail(BBS_ERR_INVALID_ARG, "bbs_rotation_margins: min_res must be > 0 and levels in [0, 15]");
    if (!(d_max > 0.0) || !std::isfinite(d_max)) return fail(BBS_ERR_INVALID_ARG, "bbs_rotation_margins: d_max must be > 0");
    for (int i = 0; i < 6; ++i)
        if (!std::isfinite(range->min[i]) || !std::isfinite(range->max[i]) || range->min[i] > range->max[i])
            return fail(BBS_ERR_INVALID_ARG, "bbs_rotation_margins: bad search range");
    bbs_map shape{};              // the grid needs only the level count and r
    shape.levels = levels;
    shape.r = min_res;
    Grid g;
    bbs_status st = make_grid(&shape, d_max, range, 0, g);
    if (st) return st;
    if (nested_angles && (st = nest_grid(g))) return st;
    int32_t e[kMaxLevels];
    rotation_margins(g, e);
    for (int l = 0; l <= levels; ++l) margins[l] = e[l];
    return BBS_OK;
}

extern "C" bbs_status bbs_score_nodes(const bbs_map *map, const float *scan_xyz, int64_t k,
                                      const bbs_search_range *range, int32_t mode, const int32_t *nodes,
                                      int64_t n, int32_t *scores)
{
    if (!map) return fail(BBS_ERR_INVALID_ARG, "bbs_score_nodes: map is NULL");
    if (n < 0 || (n > 0 && (!nodes || !scores))) return fail(BBS_ERR_INVALID_ARG, "bbs_score_nodes: bad node buffers");
    if (n > (1 << 24)) return fail(BBS_ERR_INVALID_ARG, "bbs_score_nodes: n must be <= 2^24");
    WsGuard tmp;
    bbs_status st = bbs_workspace_create(1 << 16, &tmp.w);
    if (st) return st;
    bbs_workspace *ws = tmp.w;
    hipStream_t s = ws->own_stream;
    Setup S;
    if (mode & ~7) return fail(BBS_ERR_INVALID_ARG, "bbs_score_nodes: mode must be in [0, 7]");
    st = setup_search(map, ws, scan_xyz, k, 0, range, mode & 1, 0, 1, s, S, (mode & 4) != 0);
    if (st) return st;
    if (mode & 2) {
        if ((st = check_margins(map, S.g, "bbs_score_nodes"))) return st;
        S.exact = true;
    }
    if (n == 0) return BBS_OK;
    std::vector<uint4> groups((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        const int32_t *c = nodes + 7 * i;
        int level = c[0];
        if (level < 0 || level > map->levels) return fail(BBS_ERR_INVALID_ARG, "bbs_score_nodes: node level out of range");
        for (int a = 0; a < 3; ++a) {
            if (c[1 + a] < -kTransLimit || c[1 + a] > kTransLimit)
                return fail(BBS_ERR_INVALID_ARG, "bbs_score_nodes: translation index out of range");
            if (c[4 + a] < 0 || c[4 + a] >= S.g.n[a][level])
                return fail(BBS_ERR_INVALID_ARG, "bbs_score_nodes: angle index outside the level's grid");
        }
        int j[3], b[3];
        for (int a = 0; a < 3; ++a) {
            j[a] = c[1 + a] & 1;
            b[a] = c[1 + a] - j[a];
        }
        uint32_t mask = 1u << (4 * j[0] + 2 * j[1] + j[2]);
        groups[i] = make_uint4(pack16(b[0], b[1]), pack16(b[2], c[4]), pack16(c[5], c[6]), (uint32_t)level | (mask << 8));
    }
    if (ensure(ws, ws->groups, ws->groups_n, n) || ensure(ws, ws->scores, ws->scores_n, 8 * n)) return ws_fail(ws);
    BBS_HIP(hipMemcpyAsync(ws->groups, groups.data(), (size_t)n * sizeof(uint4), hipMemcpyHostToDevice, s));
    BBS_HIP(zero_async(ws->scores, (size_t)n * 8 * sizeof(int32_t), s));
    launch_score(S, map, ws, nullptr, (int32_t)n, S.score_grid, false);
    BBS_HIP(hipGetLastError());
    std::vector<int32_t> all((size_t)n * 8);
    BBS_HIP(hipMemcpyAsync(all.data(), ws->scores, all.size() * 4, hipMemcpyDeviceToHost, s));
    BBS_HIP(hipStreamSynchronize(s));
    for (int64_t i = 0; i < n; ++i) {
        const int32_t *c = nodes + 7 * i;
        scores[i] = all[(size_t)i * 8 + 4 * (c[1] & 1) + 2 * (c[2] & 1) + (c[3] & 1)];
    }
    return BBS_OK;
}
