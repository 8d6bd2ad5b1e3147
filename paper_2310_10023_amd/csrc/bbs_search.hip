// Batched best-first branch and bound on the device (Sec. III-D, III-E).
//
// One search iteration ("flush" of Alg. 2) is six kernels on one stream:
//   gather   1 workgroup: pops the queue in (score desc, level asc, FIFO)
//            order, accepts leaves, and branches accepted inner nodes until
//            more than b children are pending (or the queue is exhausted);
//            writes the pending children as rotation groups;
//   score    the node score of Eq. (eq:3Dupperbound) for every pending node;
//   push1..3 stable counting sort of the scored children into the bucket
//            queue (one bucket per (score, level), FIFO inside a bucket).
// The initial set (every top-level cell) is pushed through the same score and
// push kernels.  Nothing but a done flag crosses to the host per iteration.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <vector>

#include "bbs_internal.h"

namespace bbs {
namespace {

constexpr int kScoreThreads = 256;
constexpr int kTileGroups = 32;                  // push tile: 32 groups = 256 node slots
constexpr int kTileSlots = kTileGroups * 8;
constexpr int kGatherThreads = 256;
constexpr int kLinkThreads = 1024;
constexpr int kItersPerSync = 8;
constexpr int64_t kDefaultQueueNodes = (int64_t)64 << 20;

struct Bucket {
    int32_t head_run, head_off, tail_run, pad;
};

struct Run {
    int32_t start, count, next, pad;
};

struct State {
    int32_t best;
    int32_t have_match;
    int32_t match[6];
    int32_t done;
    int32_t error;            // 1: node queue overflow, 2: run table overflow
    int32_t top_q;            // no bucket below this index holds nodes
    int32_t n_groups;         // pending groups of the current batch
    int32_t batch;            // 1: the pending batch is to be scored and pushed
    int32_t q_min, q_max;     // bucket range of the kept children of the batch
    int32_t runs_top, runs_cap;
    int32_t pad0;
    int64_t pend_nodes;
    int64_t kept;             // children of the batch with score >= best
    int64_t pushed;           // nodes pushed since the start
    int64_t nodes_expanded, nodes_scored, flushes, leaves_accepted;
    int64_t arena_top, arena_cap, flush_base;
};

inline int grid_for(int64_t n, int threads, int cap)
{
    int64_t g = (n + threads - 1) / threads;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

// ------------------------------------------------------------------ block helpers

template <int N>
__device__ inline int block_min_int(int v, int *sm)
{
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
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
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(v, o);
        if (lane >= o) v += t;
    }
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

// ------------------------------------------------------------------ scoring (Eq. eq:3Dupperbound)

// Scores the eight translational siblings of each group against D_level.
// For scan point s and the group's rotation R, the level-l voxel of node
// (bx + jx, by + jy, bz + jz) is w + j with w = floor(floor(R s / r) / 2^l) +
// (bx, by, bz) (float32 transform, fixed evaluation order, no contraction).
// The brick floor(w / 4) holds all eight candidate voxels, so one probe per
// point answers the whole group.
template <bool POW2>
__global__ __launch_bounds__(kScoreThreads) void k_score(const uint4 *__restrict__ groups, const State *st,
                                                          int32_t n_groups_fixed, const float *__restrict__ X,
                                                          const float *__restrict__ Y, const float *__restrict__ Z,
                                                          MapView map, const double2 *__restrict__ trig, SearchConst C,
                                                          int32_t *__restrict__ scores)
{
    __shared__ int red[kScoreThreads / 64][8];
    const int n_groups = st ? (st->batch ? st->n_groups : 0) : n_groups_fixed;
    const int K = C.K;
    for (int g = blockIdx.x; g < n_groups; g += gridDim.x) {
        const uint4 G = groups[g];
        const int level = (int)(G.w & 0xFF);
        const int bx = lo16s(G.x), by = hi16s(G.x), bz = lo16s(G.y);
        float R[9];
        rotation(trig, C, level, hi16u(G.y), lo16u(G.z), hi16u(G.z), R);
        const LevelView lv = map.lv[level];
        const Slot *__restrict__ slots = lv.slots;
        const uint32_t cap_mask = lv.cap_mask;
        const uint32_t ex = (uint32_t)(lv.bmax[0] - lv.bmin[0]);
        const uint32_t ey = (uint32_t)(lv.bmax[1] - lv.bmin[1]);
        const uint32_t ez = (uint32_t)(lv.bmax[2] - lv.bmin[2]);
        int c0 = 0, c1 = 0, c2 = 0, c3 = 0, c4 = 0, c5 = 0, c6 = 0, c7 = 0;
        for (int k = threadIdx.x; k < K; k += kScoreThreads) {
            const float sx = X[k], sy = Y[k], sz = Z[k];
            float p[3];
#pragma unroll
            for (int row = 0; row < 3; ++row) {
                float t0 = R[3 * row + 0] * sx;
                float t1 = R[3 * row + 1] * sy;
                float t2 = R[3 * row + 2] * sz;
                p[row] = (t0 + t1) + t2;
            }
            int32_t w[3];
#pragma unroll
            for (int row = 0; row < 3; ++row) {
                float q = POW2 ? p[row] * C.inv_r : p[row] / C.r;
                w[row] = ((int32_t)floorf(q) >> level);
            }
            const int32_t wx = w[0] + bx, wy = w[1] + by, wz = w[2] + bz;
            const int32_t Bx = wx >> 2, By = wy >> 2, Bz = wz >> 2;
            if ((uint32_t)(Bx - lv.bmin[0]) > ex || (uint32_t)(By - lv.bmin[1]) > ey ||
                (uint32_t)(Bz - lv.bmin[2]) > ez)
                continue;
            const uint32_t klo = brick_key_lo(Bx, By, Bz), khi = brick_key_hi(Bx, By, Bz);
            uint32_t h = brick_hash(Bx, By, Bz) & cap_mask;
            uint4 bits = make_uint4(0u, 0u, 0u, 0u);
            for (;;) {
                const uint4 hd = slots[h].head;
                const uint4 bb = slots[h].bits;
                if (hd.x == klo && hd.y == khi) {
                    bits = bb;
                    break;
                }
                if (hd.x == kEmptyLo && hd.y == kEmptyHi) break;
                h = (h + 1) & cap_mask;
            }
            const int i0 = ((wz & 3) * 5 + (wy & 3)) * 5 + (wx & 3);   // 0 .. 93
            const int word = i0 >> 5;
            const uint32_t lo = word == 0 ? bits.x : (word == 1 ? bits.y : bits.z);
            const uint32_t hi = word == 0 ? bits.y : (word == 1 ? bits.z : bits.w);
            const uint32_t win = __builtin_amdgcn_alignbit(hi, lo, (uint32_t)(i0 & 31));
            // member j = 4 jx + 2 jy + jz sits at window bit 25 jz + 5 jy + jx
            c0 += (win >> 0) & 1u;
            c1 += (win >> 25) & 1u;
            c2 += (win >> 5) & 1u;
            c3 += (win >> 30) & 1u;
            c4 += (win >> 1) & 1u;
            c5 += (win >> 26) & 1u;
            c6 += (win >> 6) & 1u;
            c7 += (win >> 31) & 1u;
        }
        int c[8] = {c0, c1, c2, c3, c4, c5, c6, c7};
#pragma unroll
        for (int j = 0; j < 8; ++j)
            for (int o = 32; o > 0; o >>= 1) c[j] += __shfl_xor(c[j], o);
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        if (lane == 0)
            for (int j = 0; j < 8; ++j) red[wave][j] = c[j];
        __syncthreads();
        if (threadIdx.x < 8) {
            int s = 0;
            for (int wv = 0; wv < kScoreThreads / 64; ++wv) s += red[wv][threadIdx.x];
            scores[8 * (int64_t)g + threadIdx.x] = s;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ initial set

// Top-level cells as the valid children of virtual cells one level above:
// virtual cell (lexicographic) outer, top-level rotation (lexicographic), then
// the eight translation children as one group.
__global__ void k_enum_initial(uint4 *groups, int64_t g0, int32_t count, SearchConst C, int32_t px0, int32_t py0,
                               int32_t pz0, int32_t npy, int32_t npz, State *st)
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
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->n_groups = count;
        st->batch = 1;
        st->q_min = INT_MAX;
        st->q_max = -1;
        st->kept = 0;
    }
}

// ------------------------------------------------------------------ push (stable counting sort)

__device__ inline int bucket_of(int score, int level, const SearchConst &C)
{
    return (C.K - score) * (C.levels + 1) + level;
}

// Per tile of 256 node slots: bucket of every kept child, its rank among the
// tile's earlier children of the same bucket, and the tile's count per bucket.
__global__ __launch_bounds__(kTileSlots) void k_push_tiles(const uint4 *groups, const int32_t *scores, State *st,
                                                           SearchConst C, int32_t *q_arr, int32_t *rank_arr,
                                                           int32_t *hist)
{
    __shared__ int sq[kTileSlots];
    __shared__ int sm[kTileSlots / 64];
    if (!st->batch) return;
    const int n_groups = st->n_groups;
    const int best = st->best;
    const int n_tiles = (n_groups + kTileGroups - 1) / kTileGroups;
    for (int t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const int s = threadIdx.x;
        const int g = t * kTileGroups + s / 8, j = s & 7;
        int q = -1;
        if (g < n_groups) {
            uint4 G = groups[g];
            uint32_t mask = (G.w >> 8) & 0xFF;
            if ((mask >> j) & 1u) {
                int sc = scores[8 * (int64_t)g + j];
                if (sc >= best) q = bucket_of(sc, (int)(G.w & 0xFF), C);
            }
        }
        __syncthreads();
        sq[s] = q;
        __syncthreads();
        int rank = 0, cnt = 0;
        if (q >= 0) {
            for (int i = 0; i < kTileSlots; ++i) {
                int e = (sq[i] == q);
                cnt += e;
                rank += e & (i < s);
            }
        }
        q_arr[(int64_t)t * kTileSlots + s] = q;
        rank_arr[(int64_t)t * kTileSlots + s] = rank;
        if (q >= 0 && rank == 0) hist[(int64_t)t * C.q_count + q] = cnt;
        int qmn = block_min_int<kTileSlots>(q >= 0 ? q : INT_MAX, sm);
        int qmx = -block_min_int<kTileSlots>(q >= 0 ? -q : INT_MAX, sm);
        int tot;
        (void)block_scan_incl<kTileSlots>(q >= 0 ? 1 : 0, sm, &tot);
        if (threadIdx.x == 0 && tot > 0) {
            atomicMin(&st->q_min, qmn);
            atomicMax(&st->q_max, qmx);
            atomicAdd((unsigned long long *)&st->kept, (unsigned long long)tot);
        }
    }
}

// Per bucket of the batch: exclusive prefix of the tile counts (in tile order)
// and the bucket's total.
__global__ void k_push_scan(State *st, SearchConst C, int32_t *hist, int32_t *totals)
{
    if (!st->batch) return;
    const int q_min = st->q_min, q_max = st->q_max;
    if (q_max < q_min) return;
    const int n_tiles = (st->n_groups + kTileGroups - 1) / kTileGroups;
    for (int q = q_min + blockIdx.x * blockDim.x + threadIdx.x; q <= q_max; q += gridDim.x * blockDim.x) {
        int acc = 0;
        for (int t = 0; t < n_tiles; ++t) {
            int64_t idx = (int64_t)t * C.q_count + q;
            int v = hist[idx];
            if (v) {
                hist[idx] = acc;
                acc += v;
            }
        }
        totals[q - q_min] = acc;
    }
}

// One workgroup: place each non-empty bucket's run in the node arena (in
// bucket order) and append it to that bucket's FIFO of runs.
__global__ __launch_bounds__(kLinkThreads) void k_push_link(State *st, SearchConst C, const int32_t *totals,
                                                            int32_t *segoff, Bucket *bk, Run *runs)
{
    __shared__ int sm[kLinkThreads / 64];
    if (!st->batch) return;
    const int q_min = st->q_min, q_max = st->q_max;
    const int64_t kept = st->kept;
    const int64_t base = st->arena_top;
    if (q_max < q_min || kept == 0) {
        if (threadIdx.x == 0) st->flush_base = base;
        return;
    }
    if (base + kept > st->arena_cap) {
        if (threadIdx.x == 0) {
            st->error = 1;
            st->done = 1;
            st->batch = 0;
        }
        return;
    }
    const int nq = q_max - q_min + 1;
    // count runs first so that an overflow leaves the queue untouched
    int n_runs = 0;
    for (int c = 0; c < nq; c += kLinkThreads) {
        int i = c + threadIdx.x;
        int ne = (i < nq && totals[i] > 0) ? 1 : 0;
        int tot;
        (void)block_scan_incl<kLinkThreads>(ne, sm, &tot);
        n_runs += tot;
    }
    const int runs_top = st->runs_top;
    if ((int64_t)runs_top + n_runs > (int64_t)st->runs_cap) {
        __syncthreads();
        if (threadIdx.x == 0) {
            st->error = 2;
            st->done = 1;
            st->batch = 0;
        }
        return;
    }
    int64_t node_off = 0;
    int run_off = 0;
    for (int c = 0; c < nq; c += kLinkThreads) {
        int i = c + threadIdx.x;
        int tot_n = (i < nq) ? totals[i] : 0;
        int ne = tot_n > 0 ? 1 : 0;
        int sum_n, sum_r;
        int incl_n = block_scan_incl<kLinkThreads>(tot_n, sm, &sum_n);
        int incl_r = block_scan_incl<kLinkThreads>(ne, sm, &sum_r);
        if (ne) {
            int q = q_min + i;
            int64_t off = node_off + incl_n - tot_n;
            int r = runs_top + run_off + incl_r - 1;
            segoff[i] = (int32_t)off;
            runs[r] = Run{(int32_t)(base + off), tot_n, -1, 0};
            int tail = bk[q].tail_run;
            if (tail >= 0) runs[tail].next = r;
            else {
                bk[q].head_run = r;
                bk[q].head_off = 0;
            }
            bk[q].tail_run = r;
        }
        node_off += sum_n;
        run_off += sum_r;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        st->flush_base = base;
        st->arena_top = base + kept;
        st->runs_top = runs_top + n_runs;
        st->pushed += kept;
        st->top_q = min(st->top_q, q_min);
    }
}

// Write every kept child to arena[flush_base + bucket offset + earlier tiles'
// count + rank in tile], then clear the tile's histogram entries.
__global__ __launch_bounds__(kTileSlots) void k_push_scatter(const uint4 *groups, State *st, SearchConst C,
                                                             const int32_t *q_arr, const int32_t *rank_arr,
                                                             const int32_t *segoff, int32_t *hist, uint4 *arena)
{
    if (!st->batch) return;
    const int n_groups = st->n_groups;
    const int n_tiles = (n_groups + kTileGroups - 1) / kTileGroups;
    const int q_min = st->q_min;
    const int64_t base = st->flush_base;
    for (int t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const int s = threadIdx.x;
        const int q = q_arr[(int64_t)t * kTileSlots + s];
        const int rank = rank_arr[(int64_t)t * kTileSlots + s];
        if (q >= 0) {
            const int g = t * kTileGroups + s / 8, j = s & 7;
            const uint4 G = groups[g];
            const int64_t hidx = (int64_t)t * C.q_count + q;
            const int64_t pos = base + segoff[q - q_min] + hist[hidx] + rank;
            const int jx = (j >> 2) & 1, jy = (j >> 1) & 1, jz = j & 1;
            const int x = lo16s(G.x) + jx, y = hi16s(G.x) + jy, z = lo16s(G.y) + jz;
            arena[pos] = make_uint4(pack16(x, y), pack16(z, hi16u(G.y)), G.z, G.w & 0xFFu);
        }
        __syncthreads();
        if (q >= 0 && rank == 0) hist[(int64_t)t * C.q_count + q] = 0;
        __syncthreads();
    }
}

// ------------------------------------------------------------------ gather + branch

__device__ inline void child_counts(const SearchConst &C, const int32_t t[3], const int32_t ang[3], int level,
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
// lexicographically smallest leaf competes for the match), an inner bucket
// is consumed node by node until the pending count passes b.  Buckets below
// the running best are never touched (their nodes would be pruned).
__global__ __launch_bounds__(kGatherThreads) void k_gather(State *st, Bucket *bk, const Run *runs,
                                                           const uint4 *arena, SearchConst C, uint4 *groups)
{
    __shared__ int sm[kGatherThreads / 64];
    __shared__ int smatch[kGatherThreads][6];
    if (st->done) return;
    const int tid = threadIdx.x;
    const int Lp1 = C.levels + 1;
    int best = st->best;
    int have = st->have_match;
    int32_t match[6];
    for (int i = 0; i < 6; ++i) match[i] = st->match[i];
    int q = st->top_q;
    int64_t pend = 0;
    int ngrp = 0;
    int64_t expanded = 0, leaves = 0;
    bool cut = false;
    for (;;) {
        if (best > C.K) break;
        const int qlim = min((C.K - best) * Lp1 + C.levels, C.q_count - 1);
        int found = INT_MAX;
        for (int b0 = q; b0 <= qlim; b0 += kGatherThreads) {
            int qq = b0 + tid;
            int cand = (qq <= qlim && bk[qq].head_run >= 0) ? qq : INT_MAX;
            found = block_min_int<kGatherThreads>(cand, sm);
            if (found != INT_MAX) break;
        }
        if (found == INT_MAX) break;
        q = found;
        const int level = q % Lp1;
        const int score = C.K - q / Lp1;
        const Bucket b = bk[q];
        if (level == 0) {
            int32_t mine[6] = {INT_MAX, INT_MAX, INT_MAX, INT_MAX, INT_MAX, INT_MAX};
            int run = b.head_run, off = b.head_off;
            while (run >= 0) {
                const Run R = runs[run];
                const int cnt = R.count - off;
                for (int i = tid; i < cnt; i += kGatherThreads) {
                    int32_t t[3], ang[3], lv;
                    node_unpack(arena[R.start + off + i], t, ang, lv);
                    int32_t cand[6] = {t[0], t[1], t[2], ang[0], ang[1], ang[2]};
                    if (leaf_less(cand, mine))
                        for (int k = 0; k < 6; ++k) mine[k] = cand[k];
                }
                leaves += cnt;
                off = 0;
                run = R.next;
            }
            __syncthreads();
            for (int k = 0; k < 6; ++k) smatch[tid][k] = mine[k];
            __syncthreads();
            for (int s = kGatherThreads / 2; s > 0; s >>= 1) {
                if (tid < s && leaf_less(smatch[tid + s], smatch[tid]))
                    for (int k = 0; k < 6; ++k) smatch[tid][k] = smatch[tid + s][k];
                __syncthreads();
            }
            if (!have || score > best || leaf_less(smatch[0], match))
                for (int k = 0; k < 6; ++k) match[k] = smatch[0][k];
            __syncthreads();
            have = 1;
            best = score;
            if (tid == 0) {
                bk[q].head_run = -1;
                bk[q].tail_run = -1;
            }
            ++q;
            continue;
        }
        int run = b.head_run, off = b.head_off;
        while (run >= 0 && !cut) {
            const Run R = runs[run];
            const int avail = R.count - off;
            int base = 0;
            for (; base < avail && !cut; base += kGatherThreads) {
                const int i = base + tid;
                const bool valid = i < avail;
                int32_t t[3] = {0, 0, 0}, ang[3] = {0, 0, 0}, lv = level;
                int rc[3] = {0, 0, 0}, nn = 0, ng = 0;
                uint32_t tmask = 0;
                if (valid) {
                    node_unpack(arena[R.start + off + i], t, ang, lv);
                    child_counts(C, t, ang, level, rc, tmask, nn, ng);
                }
                int tot_n, tot_g;
                const int incl_n = block_scan_incl<kGatherThreads>(nn, sm, &tot_n);
                const int incl_g = block_scan_incl<kGatherThreads>(ng, sm, &tot_g);
                const int over = (valid && pend + incl_n > C.batch) ? tid : INT_MAX;
                const int cutidx = block_min_int<kGatherThreads>(over, sm);
                const int consumed = cutidx != INT_MAX ? cutidx + 1 : min(kGatherThreads, avail - base);
                if (tid < consumed && ng > 0) {
                    int gi = ngrp + incl_g - ng;
                    for (int ja = 0; ja < rc[0]; ++ja)
                        for (int jb = 0; jb < rc[1]; ++jb)
                            for (int jg = 0; jg < rc[2]; ++jg) {
                                int ra = C.a[0][level] * ang[0] + ja;
                                int rb = C.a[1][level] * ang[1] + jb;
                                int rg = C.a[2][level] * ang[2] + jg;
                                groups[gi++] = make_uint4(pack16(2 * t[0], 2 * t[1]), pack16(2 * t[2], ra),
                                                          pack16(rb, rg), (uint32_t)(level - 1) | (tmask << 8));
                            }
                }
                // totals up to and including the last consumed node
                __syncthreads();
                __shared__ int s_last_n, s_last_g;
                if (tid == consumed - 1) {
                    s_last_n = incl_n;
                    s_last_g = incl_g;
                }
                __syncthreads();
                pend += s_last_n;
                ngrp += s_last_g;
                expanded += consumed;
                if (cutidx != INT_MAX) {
                    cut = true;
                    off += base + consumed;
                }
            }
            if (!cut) {
                off = 0;
                run = R.next;
            } else if (off == R.count) {
                off = 0;
                run = R.next;
            }
        }
        if (tid == 0) {
            if (run < 0) {
                bk[q].head_run = -1;
                bk[q].tail_run = -1;
            } else {
                bk[q].head_run = run;
                bk[q].head_off = off;
            }
        }
        if (cut) break;
        ++q;
    }
    __syncthreads();
    if (tid == 0) {
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
        } else {
            st->batch = 0;
            st->done = 1;
        }
    }
}

// ------------------------------------------------------------------ host side

bool is_pow2_float(float r)
{
    int e = 0;
    float m = std::frexp(r, &e);
    return m == 0.5f;
}

template <class T>
bbs_status ensure(T *&p, int64_t &cap, int64_t need)
{
    if (p && cap >= need) return BBS_OK;
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
    int64_t n = std::max<int64_t>(need, 1);
    void *q = nullptr;
    if (alloc_dev(&q, (size_t)n * sizeof(T))) return BBS_ERR_OOM;
    p = static_cast<T *>(q);
    cap = n;
    return BBS_OK;
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
    Run *runs = nullptr;
    int64_t runs_n = 0;
    Bucket *buckets = nullptr;
    int64_t buckets_n = 0;
    int32_t *hist = nullptr;
    int64_t hist_n = 0;
    int32_t *totals = nullptr;
    int64_t totals_n = 0;
    int32_t *segoff = nullptr;
    int64_t segoff_n = 0;
    uint4 *groups = nullptr;
    int64_t groups_n = 0;
    int32_t *scores = nullptr;
    int64_t scores_n = 0;
    int32_t *q_arr = nullptr;
    int64_t q_arr_n = 0;
    int32_t *rank_arr = nullptr;
    int64_t rank_arr_n = 0;
    float *scan = nullptr;
    int64_t scan_n = 0;
    float *scan_aos = nullptr;
    int64_t scan_aos_n = 0;
    double2 *trig = nullptr;
    int64_t trig_n = 0;
    State *state = nullptr;
    int64_t state_n = 0;
    unsigned long long *maxsq = nullptr;
    int64_t maxsq_n = 0;
    State *host_state = nullptr;   // pinned
    std::vector<hipEvent_t> ev;
    bool hist_dirty = true;
};

namespace bbs {
namespace {

void free_ws(bbs_workspace *w)
{
    void *ptrs[] = {w->arena, w->runs, w->buckets, w->hist, w->totals, w->segoff, w->groups, w->scores,
                    w->q_arr, w->rank_arr, w->scan, w->scan_aos, w->trig, w->state, w->maxsq};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (w->host_state) (void)hipHostFree(w->host_state);
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

double cell_angle(const Grid &g, int ax, int c, int l)
{
    return g.wmin[ax] + g.dprime[ax][l] * ((double)c + 0.5);
}

struct Setup {
    Grid g;
    SearchConst C;
    hipStream_t s;
    bool pow2;
};

// Upload the scan, derive d_max, the grid and the cos/sin tables.
bbs_status setup_search(const bbs_map *m, bbs_workspace *ws, const float *scan, int64_t k, int on_device,
                        const bbs_search_range *range, int translation_only, int32_t threshold, int64_t batch,
                        hipStream_t s, Setup &S)
{
    if (k < 1 || k > (1 << 24)) return fail(BBS_ERR_INVALID_ARG, "bbs_localize: k must be in [1, 2^24]");
    if (!scan) return fail(BBS_ERR_INVALID_ARG, "bbs_localize: scan is NULL");
    if (!range) return fail(BBS_ERR_INVALID_ARG, "bbs_localize: range is NULL");
    for (int i = 0; i < 6; ++i)
        if (!std::isfinite(range->min[i]) || !std::isfinite(range->max[i]) || range->min[i] > range->max[i])
            return fail(BBS_ERR_INVALID_ARG, "bbs_localize: search range must be finite with min <= max");
    if (batch < 1 || batch > (1 << 24)) return fail(BBS_ERR_INVALID_ARG, "bbs_localize: batch_size must be in [1, 2^24]");
    S.s = s;
    if (ensure(ws->scan, ws->scan_n, 3 * k) || ensure(ws->maxsq, ws->maxsq_n, 1)) return BBS_ERR_OOM;
    const float *aos = scan;
    if (!on_device) {
        if (ensure(ws->scan_aos, ws->scan_aos_n, 3 * k)) return BBS_ERR_OOM;
        BBS_HIP(hipMemcpyAsync(ws->scan_aos, scan, (size_t)k * 12, hipMemcpyHostToDevice, s));
        aos = ws->scan_aos;
    }
    BBS_HIP(hipMemsetAsync(ws->maxsq, 0, 8, s));
    k_scan_soa<<<grid_for(k, 256, 1024), 256, 0, s>>>(aos, (int32_t)k, ws->scan, ws->scan + k, ws->scan + 2 * k,
                                                       ws->maxsq);
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
    C.batch = batch;
    C.r = g.r;
    S.pow2 = is_pow2_float(g.r);
    C.inv_r = 1.0f / g.r;
    C.r_pow2 = S.pow2 ? 1 : 0;
    if (ensure(ws->trig, ws->trig_n, (int64_t)trig.size())) return BBS_ERR_OOM;
    BBS_HIP(hipMemcpyAsync(ws->trig, trig.data(), trig.size() * sizeof(double2), hipMemcpyHostToDevice, s));
    return BBS_OK;
}

void launch_score(const Setup &S, const bbs_map *m, bbs_workspace *ws, const State *st, int32_t n_fixed, int grid)
{
    const float *X = ws->scan, *Y = ws->scan + S.C.K, *Z = ws->scan + 2 * (int64_t)S.C.K;
    MapView v = m->view();
    if (S.pow2)
        k_score<true><<<grid, kScoreThreads, 0, S.s>>>(ws->groups, st, n_fixed, X, Y, Z, v, ws->trig, S.C, ws->scores);
    else
        k_score<false><<<grid, kScoreThreads, 0, S.s>>>(ws->groups, st, n_fixed, X, Y, Z, v, ws->trig, S.C, ws->scores);
}

int64_t max_children(const Grid &g)
{
    int64_t mc = 8;
    for (int l = 1; l <= g.levels; ++l) mc = std::max<int64_t>(mc, 8LL * g.a[0][l] * g.a[1][l] * g.a[2][l]);
    return mc;
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
    const auto t_start = std::chrono::steady_clock::now();
    hipStream_t s = o.stream ? static_cast<hipStream_t>(o.stream) : ws->own_stream;
    Setup S;
    bbs_status st = setup_search(map, ws, scan_xyz, k, scan_on_device, range, o.translation_only, score_threshold,
                                 o.batch_size, s, S);
    if (st) return st;
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
    const int64_t cap_groups = std::max<int64_t>(o.batch_size + mc, 4096);
    const int64_t n_tiles = (cap_groups + kTileGroups - 1) / kTileGroups;
    const int64_t qn = std::max<int32_t>(C.q_count, 1);
    const int64_t runs_cap = std::max<int64_t>(ws->queue_nodes / 4, 1 << 16);
    if (ensure(ws->groups, ws->groups_n, cap_groups) || ensure(ws->scores, ws->scores_n, 8 * cap_groups) ||
        ensure(ws->q_arr, ws->q_arr_n, n_tiles * kTileSlots) ||
        ensure(ws->rank_arr, ws->rank_arr_n, n_tiles * kTileSlots) || ensure(ws->totals, ws->totals_n, qn) ||
        ensure(ws->segoff, ws->segoff_n, qn) || ensure(ws->buckets, ws->buckets_n, qn) ||
        ensure(ws->arena, ws->arena_n, ws->queue_nodes) || ensure(ws->runs, ws->runs_n, runs_cap) ||
        ensure(ws->state, ws->state_n, 1))
        return BBS_ERR_OOM;
    if (!ws->hist || ws->hist_n < n_tiles * qn) {
        if (ensure(ws->hist, ws->hist_n, n_tiles * qn)) return BBS_ERR_OOM;
        ws->hist_dirty = true;
    }
    if (ws->hist_dirty) {
        BBS_HIP(hipMemsetAsync(ws->hist, 0, (size_t)ws->hist_n * 4, s));
        ws->hist_dirty = false;
    }
    k_fill_buckets<<<grid_for(qn, 256, 4096), 256, 0, s>>>(ws->buckets, (int32_t)qn);

    State h;
    std::memset(&h, 0, sizeof(h));
    h.best = C.threshold;
    h.top_q = 0;
    h.runs_cap = (int32_t)std::min<int64_t>(runs_cap, INT_MAX);
    h.arena_cap = ws->queue_nodes;
    h.q_min = INT_MAX;
    h.q_max = -1;
    BBS_HIP(hipMemcpyAsync(ws->state, &h, sizeof(State), hipMemcpyHostToDevice, s));

    const bool prof = o.profile != 0;
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
    const int score_grid = 4096;
    const int tile_grid = (int)std::min<int64_t>(n_tiles, 2048);
    const int scan_grid = 64;
    auto push = [&]() {
        k_push_tiles<<<tile_grid, kTileSlots, 0, s>>>(ws->groups, ws->scores, ws->state, C, ws->q_arr, ws->rank_arr,
                                                       ws->hist);
        k_push_scan<<<scan_grid, 256, 0, s>>>(ws->state, C, ws->hist, ws->totals);
        k_push_link<<<1, kLinkThreads, 0, s>>>(ws->state, C, ws->totals, ws->segoff, ws->buckets, ws->runs);
        k_push_scatter<<<tile_grid, kTileSlots, 0, s>>>(ws->groups, ws->state, C, ws->q_arr, ws->rank_arr, ws->segoff,
                                                         ws->hist, ws->arena);
    };
    const double t_setup = ms_since(t_start);

    // initial set, in chunks of the group buffer
    int64_t init_chunks = 0;
    for (int64_t g0 = 0; g0 < n_init_groups; g0 += cap_groups) {
        int32_t cnt = (int32_t)std::min<int64_t>(cap_groups, n_init_groups - g0);
        k_enum_initial<<<grid_for(cnt, 256, 4096), 256, 0, s>>>(ws->groups, g0, cnt, C, P0[0], P0[1], P0[2], PN[1],
                                                                 PN[2], ws->state);
        if (prof) BBS_HIP(record(ev_used++));
        launch_score(S, map, ws, ws->state, 0, score_grid);
        if (prof) BBS_HIP(record(ev_used++));
        push();
        ++init_chunks;
    }
    BBS_HIP(hipGetLastError());
    BBS_HIP(hipMemcpyAsync(ws->host_state, ws->state, sizeof(State), hipMemcpyDeviceToHost, s));
    BBS_HIP(hipStreamSynchronize(s));
    const int64_t initial_kept = ws->host_state->pushed;
    const double t_init = ms_since(t_start);
    if (ws->host_state->error) {
        ws->hist_dirty = true;
        return fail(BBS_ERR_QUEUE_OVERFLOW, "bbs_localize: node queue capacity exceeded by the initial set");
    }

    // search loop; every iteration before the last pops at least one node, so
    // the cap only guards against a broken queue
    const int64_t max_iters = (int64_t)1 << 26;
    int64_t iters = 0;
    for (;;) {
        if (iters >= max_iters) {
            ws->hist_dirty = true;
            return fail(BBS_ERR_INTERNAL, "bbs_localize: search did not terminate");
        }
        iters += kItersPerSync;
        for (int it = 0; it < kItersPerSync; ++it) {
            k_gather<<<1, kGatherThreads, 0, s>>>(ws->state, ws->buckets, ws->runs, ws->arena, C, ws->groups);
            if (prof) BBS_HIP(record(ev_used++));
            launch_score(S, map, ws, ws->state, 0, score_grid);
            if (prof) BBS_HIP(record(ev_used++));
            push();
        }
        BBS_HIP(hipGetLastError());
        BBS_HIP(hipMemcpyAsync(ws->host_state, ws->state, sizeof(State), hipMemcpyDeviceToHost, s));
        BBS_HIP(hipStreamSynchronize(s));
        if (ws->host_state->done || ws->host_state->error) break;
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
    out->nodes_scored = init_nodes + fs.nodes_scored;
    out->flushes = fs.flushes;
    out->leaves_accepted = fs.leaves_accepted;
    out->initial_size = init_nodes;
    out->initial_kept = initial_kept;
    out->score_pairs = out->nodes_scored * k;
    if (prof) {
        // every iteration before the one that found the queue exhausted scored a batch
        int64_t launches = init_chunks + fs.flushes;
        double total = 0.0;
        for (int64_t i = 0; i < launches && 2 * i + 1 < ev_used; ++i) {
            float ms = 0.0f;
            BBS_HIP(hipEventElapsedTime(&ms, ws->ev[2 * i], ws->ev[2 * i + 1]));
            total += ms;
        }
        out->score_kernel_ms = total;
        out->score_launches = launches;
    }
    out->phase_ms[0] = t_setup;
    out->phase_ms[1] = t_init - t_setup;
    out->phase_ms[2] = t_loop - t_init;
    out->phase_ms[3] = ms_since(t_start);
    return BBS_OK;
}

extern "C" bbs_status bbs_score_nodes(const bbs_map *map, const float *scan_xyz, int64_t k,
                                      const bbs_search_range *range, int32_t translation_only, const int32_t *nodes,
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
    st = setup_search(map, ws, scan_xyz, k, 0, range, translation_only, 0, 1, s, S);
    if (st) return st;
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
    if (ensure(ws->groups, ws->groups_n, n) || ensure(ws->scores, ws->scores_n, 8 * n)) return BBS_ERR_OOM;
    BBS_HIP(hipMemcpyAsync(ws->groups, groups.data(), (size_t)n * sizeof(uint4), hipMemcpyHostToDevice, s));
    launch_score(S, map, ws, nullptr, (int32_t)n, (int)std::min<int64_t>(n, 8192));
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
