// Pose refinement after the search: GICP (Segal et al.) with voxel statistics
// as its distributions.  The paper accepts a BBS pose when it is close enough
// for local registration with GICP to finish (Sec. IV, the success criterion;
// Sec. IV-B uses GICP for the ground truth too) and gives no GICP arithmetic;
// the readings are stated in include/bbs.h beside bbs_gicp_refine.
//
// Device work: voxel statistics of the target (once) and of the scan (per
// call), both through a hash table of voxel keys with double atomics; per
// Gauss-Newton step one kernel pairs every scan point with the nearest voxel
// mean of the 27 voxels around it and accumulates J^T Omega J, J^T Omega r
// and the cost into per-workgroup partials.  The host sums the partials in a
// fixed order, solves the 6 x 6 system and updates the pose.
#include <algorithm>
#include <climits>
#include <cmath>
#include <vector>

#include "bbs_internal.h"

namespace bbs {
namespace {

constexpr int kGThreads = 256;
constexpr unsigned long long kGEmpty = ~0ull;
constexpr int32_t kGBias = 1 << 20;
constexpr double kRegEps = 1e-3;
constexpr int kPartials = 29;        // 21 entries of H (upper triangle), 6 of g, cost, pairs

int ggrid(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + kGThreads - 1) / kGThreads, 8192)); }

// Voxel statistics: a hash of voxel keys (21 bits per axis, index + 2^20), a
// dense index per key, and per index the point count, the sums of p and of
// p p^T (upper triangle), then the mean and the regularized covariance.
struct VoxelStats {
    unsigned long long *keys = nullptr;   // table of cap slots
    int32_t *index = nullptr;             // slot -> dense index
    uint32_t cap = 0;
    int32_t n = 0;                         // distinct voxels
    int32_t *count = nullptr;
    double *sum = nullptr;                // 9 per voxel: x, y, z, xx, xy, xz, yy, yz, zz
    double *dist = nullptr;               // 9 per voxel: mean (3), covariance upper triangle (6); valid if count >= min
    void release()
    {
        for (void *p : {(void *)keys, (void *)index, (void *)count, (void *)sum, (void *)dist})
            if (p) (void)hipFree(p);
        keys = nullptr;
        index = nullptr;
        count = nullptr;
        sum = nullptr;
        dist = nullptr;
    }
};

__device__ inline bool voxel_of(double x, double y, double z, double voxel, unsigned long long &key)
{
    const double v[3] = {floor(x / voxel), floor(y / voxel), floor(z / voxel)};
    key = 0;
    for (int a = 0; a < 3; ++a) {
        if (!(v[a] >= -(double)kGBias && v[a] < (double)kGBias)) return false;
        key = (key << 21) | (unsigned long long)(uint32_t)((int32_t)v[a] + kGBias);
    }
    return true;
}

__device__ inline uint32_t gmix(unsigned long long x)
{
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ull;
    x ^= x >> 33;
    return (uint32_t)x;
}

__device__ inline uint32_t g_insert(unsigned long long *keys, uint32_t mask, unsigned long long key)
{
    uint32_t h = gmix(key) & mask;
    for (;;) {
        const unsigned long long old = atomicCAS(&keys[h], kGEmpty, key);
        if (old == kGEmpty || old == key) return h;
        h = (h + 1) & mask;
    }
}

__device__ inline int32_t g_find(const unsigned long long *keys, const int32_t *index, uint32_t mask,
                                 unsigned long long key)
{
    uint32_t h = gmix(key) & mask;
    for (;;) {
        const unsigned long long k = keys[h];
        if (k == key) return index[h];
        if (k == kGEmpty) return -1;
        h = (h + 1) & mask;
    }
}

__global__ void k_g_fill(unsigned long long *keys, uint32_t cap)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cap; i += gridDim.x * blockDim.x) keys[i] = kGEmpty;
}

// Keys of every point (err |= 1 if a voxel index leaves [-2^20, 2^20) or a
// coordinate is not finite).
__global__ void k_g_insert(const float *p, int64_t n, double voxel, unsigned long long *keys, uint32_t mask,
                           int *err)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        unsigned long long key;
        if (!voxel_of(p[3 * i], p[3 * i + 1], p[3 * i + 2], voxel, key)) {
            atomicOr(err, 1);
            continue;
        }
        g_insert(keys, mask, key);
    }
}

__global__ void k_g_number(const unsigned long long *keys, uint32_t cap, int32_t *index, int32_t *counter)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cap; i += gridDim.x * blockDim.x)
        index[i] = keys[i] != kGEmpty ? atomicAdd(counter, 1) : -1;
}

__global__ void k_g_zero(int32_t *count, double *sum, int32_t m)
{
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
        count[i] = 0;
        for (int j = 0; j < 9; ++j) sum[9 * i + j] = 0.0;
    }
}

// Sums per voxel; voxel_of_point[i] receives the point's voxel index.
__global__ void k_g_accumulate(const float *p, int64_t n, double voxel, const unsigned long long *keys,
                               const int32_t *index, uint32_t mask, int32_t *count, double *sum, int32_t *vox)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double x = p[3 * i], y = p[3 * i + 1], z = p[3 * i + 2];
        unsigned long long key;
        int32_t v = -1;
        if (voxel_of(x, y, z, voxel, key)) v = g_find(keys, index, mask, key);
        if (vox) vox[i] = v;
        if (v < 0) continue;
        atomicAdd(&count[v], 1);
        const double t[9] = {x, y, z, x * x, x * y, x * z, y * y, y * z, z * z};
        for (int j = 0; j < 9; ++j) atomicAdd(&sum[9 * v + j], t[j]);
    }
}

// Eigenvectors of a symmetric 3 x 3 matrix by cyclic Jacobi rotations (ten
// sweeps; the off-diagonal part is then at rounding level).
__device__ void jacobi3(double A[3][3], double V[3][3])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) V[i][j] = i == j ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 10; ++sweep)
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                const double apq = A[p][q];
                if (fabs(apq) < 1e-300) continue;
                const double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
                const double tt = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double c = 1.0 / sqrt(tt * tt + 1.0), s = tt * c;
                for (int k = 0; k < 3; ++k) {       // A <- A J
                    const double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - s * akq;
                    A[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < 3; ++k) {       // A <- J^T A
                    const double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - s * aqk;
                    A[q][k] = s * apk + c * aqk;
                }
                for (int k = 0; k < 3; ++k) {       // V <- V J
                    const double vkp = V[k][p], vkq = V[k][q];
                    V[k][p] = c * vkp - s * vkq;
                    V[k][q] = s * vkp + c * vkq;
                }
            }
}

// Mean and plane-to-plane covariance U diag(eps, 1, 1) U^T (eigenvalues
// ascending) of every voxel with at least min_points points.
__global__ void k_g_finalize(const int32_t *count, const double *sum, int32_t m, int32_t min_points, double *dist)
{
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
        const int32_t c = count[i];
        if (c < min_points) {
            dist[9 * i] = NAN;
            continue;
        }
        const double *s = sum + 9 * i;
        const double nn = (double)c;
        const double mu[3] = {s[0] / nn, s[1] / nn, s[2] / nn};
        double A[3][3];
        A[0][0] = s[3] / nn - mu[0] * mu[0];
        A[0][1] = A[1][0] = s[4] / nn - mu[0] * mu[1];
        A[0][2] = A[2][0] = s[5] / nn - mu[0] * mu[2];
        A[1][1] = s[6] / nn - mu[1] * mu[1];
        A[1][2] = A[2][1] = s[7] / nn - mu[1] * mu[2];
        A[2][2] = s[8] / nn - mu[2] * mu[2];
        double V[3][3];
        jacobi3(A, V);
        int o[3] = {0, 1, 2};                       // eigenvalues ascending
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2 - a; ++b)
                if (A[o[b]][o[b]] > A[o[b + 1]][o[b + 1]]) {
                    const int t = o[b];
                    o[b] = o[b + 1];
                    o[b + 1] = t;
                }
        const double lam[3] = {kRegEps, 1.0, 1.0};
        double C[3][3] = {};
        for (int e = 0; e < 3; ++e)
            for (int r = 0; r < 3; ++r)
                for (int q = 0; q < 3; ++q) C[r][q] += lam[e] * V[r][o[e]] * V[q][o[e]];
        double *d = dist + 9 * i;
        d[0] = mu[0];
        d[1] = mu[1];
        d[2] = mu[2];
        d[3] = C[0][0];
        d[4] = C[0][1];
        d[5] = C[0][2];
        d[6] = C[1][1];
        d[7] = C[1][2];
        d[8] = C[2][2];
    }
}

struct Pose {
    double R[9];
    double t[3];
};

// One Gauss-Newton linearization: per scan point with a covariance, the
// nearest voxel mean among the 27 voxels around q = R p + t (lexicographic
// offsets, first of equal distances, closer than one edge), then J^T Omega J,
// J^T Omega r and r^T Omega r into per-workgroup partials.
__global__ __launch_bounds__(kGThreads) void k_g_linearize(const float *p, int64_t n, const int32_t *svox,
                                                            const double *sdist, const unsigned long long *tkeys,
                                                            const int32_t *tindex, uint32_t tmask,
                                                            const double *tdist, double voxel, Pose P,
                                                            double *partials)
{
    __shared__ double red[kGThreads / 64][kPartials];
    double acc[kPartials];
    for (int j = 0; j < kPartials; ++j) acc[j] = 0.0;
    const double *R = P.R;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t sv = svox[i];
        if (sv < 0 || isnan(sdist[9 * sv])) continue;
        const double px = p[3 * i], py = p[3 * i + 1], pz = p[3 * i + 2];
        double q[3];
        for (int a = 0; a < 3; ++a) q[a] = ((R[3 * a] * px + R[3 * a + 1] * py) + R[3 * a + 2] * pz) + P.t[a];
        const double b[3] = {floor(q[0] / voxel), floor(q[1] / voxel), floor(q[2] / voxel)};
        int32_t best = -1;
        double best_d = voxel * voxel;
        for (int dx = -1; dx <= 1; ++dx)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dz = -1; dz <= 1; ++dz) {
                    const double c[3] = {b[0] + dx, b[1] + dy, b[2] + dz};
                    bool ok = true;
                    unsigned long long key = 0;
                    for (int a = 0; a < 3; ++a) {
                        ok = ok && c[a] >= -(double)kGBias && c[a] < (double)kGBias;
                        key = (key << 21) | (unsigned long long)(uint32_t)((int32_t)c[a] + kGBias);
                    }
                    if (!ok) continue;
                    const int32_t v = g_find(tkeys, tindex, tmask, key);
                    if (v < 0 || isnan(tdist[9 * v])) continue;
                    const double ex = tdist[9 * v] - q[0], ey = tdist[9 * v + 1] - q[1], ez = tdist[9 * v + 2] - q[2];
                    const double d2 = (ex * ex + ey * ey) + ez * ez;
                    if (d2 < best_d) {
                        best_d = d2;
                        best = v;
                    }
                }
        if (best < 0) continue;
        const double *td = tdist + 9 * best;
        const double *sd = sdist + 9 * sv;
        const double r[3] = {td[0] - q[0], td[1] - q[1], td[2] - q[2]};
        const double Cs[3][3] = {{sd[3], sd[4], sd[5]}, {sd[4], sd[6], sd[7]}, {sd[5], sd[7], sd[8]}};
        double RC[3][3], M[3][3];
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c)
                RC[a][c] = R[3 * a] * Cs[0][c] + R[3 * a + 1] * Cs[1][c] + R[3 * a + 2] * Cs[2][c];
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c)
                M[a][c] = RC[a][0] * R[3 * c] + RC[a][1] * R[3 * c + 1] + RC[a][2] * R[3 * c + 2];
        M[0][0] += td[3];
        M[0][1] += td[4];
        M[0][2] += td[5];
        M[1][0] += td[4];
        M[1][1] += td[6];
        M[1][2] += td[7];
        M[2][0] += td[5];
        M[2][1] += td[7];
        M[2][2] += td[8];
        // Omega = M^-1 by cofactors
        const double c00 = M[1][1] * M[2][2] - M[1][2] * M[2][1];
        const double c01 = M[1][2] * M[2][0] - M[1][0] * M[2][2];
        const double c02 = M[1][0] * M[2][1] - M[1][1] * M[2][0];
        const double det = M[0][0] * c00 + M[0][1] * c01 + M[0][2] * c02;
        const double id = 1.0 / det;
        double O[3][3];
        O[0][0] = c00 * id;
        O[1][0] = c01 * id;
        O[2][0] = c02 * id;
        O[0][1] = (M[0][2] * M[2][1] - M[0][1] * M[2][2]) * id;
        O[1][1] = (M[0][0] * M[2][2] - M[0][2] * M[2][0]) * id;
        O[2][1] = (M[0][1] * M[2][0] - M[0][0] * M[2][1]) * id;
        O[0][2] = (M[0][1] * M[1][2] - M[0][2] * M[1][1]) * id;
        O[1][2] = (M[0][2] * M[1][0] - M[0][0] * M[1][2]) * id;
        O[2][2] = (M[0][0] * M[1][1] - M[0][1] * M[1][0]) * id;
        // J = [ [q]_x , -I ]
        double J[3][6] = {{0.0, -q[2], q[1], -1.0, 0.0, 0.0},
                          {q[2], 0.0, -q[0], 0.0, -1.0, 0.0},
                          {-q[1], q[0], 0.0, 0.0, 0.0, -1.0}};
        double JO[6][3];
        for (int a = 0; a < 6; ++a)
            for (int c = 0; c < 3; ++c) JO[a][c] = J[0][a] * O[0][c] + J[1][a] * O[1][c] + J[2][a] * O[2][c];
        int k = 0;
        for (int a = 0; a < 6; ++a)
            for (int c = a; c < 6; ++c) acc[k++] += JO[a][0] * J[0][c] + JO[a][1] * J[1][c] + JO[a][2] * J[2][c];
        for (int a = 0; a < 6; ++a) acc[21 + a] += JO[a][0] * r[0] + JO[a][1] * r[1] + JO[a][2] * r[2];
        double Or[3];
        for (int a = 0; a < 3; ++a) Or[a] = O[a][0] * r[0] + O[a][1] * r[1] + O[a][2] * r[2];
        acc[27] += r[0] * Or[0] + r[1] * Or[1] + r[2] * Or[2];
        acc[28] += 1.0;
    }
    // workgroup sum: waves by shuffles, then the four wave sums in order
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int j = 0; j < kPartials; ++j) {
        double v = acc[j];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
        if (lane == 0) red[wave][j] = v;
    }
    __syncthreads();
    if (threadIdx.x < kPartials) {
        double v = 0.0;
        for (int w = 0; w < kGThreads / 64; ++w) v += red[w][threadIdx.x];
        partials[(int64_t)blockIdx.x * kPartials + threadIdx.x] = v;
    }
}

// Voxel statistics of n device points at the given edge.
bbs_status build_stats(const float *p, int64_t n, double voxel, int32_t min_points, hipStream_t s, VoxelStats &V,
                       int32_t *point_voxel)
{
    uint64_t cap = 1024;
    while (cap < 2 * (uint64_t)n) cap *= 2;
    if (cap > ((uint64_t)1 << 31)) return fail(BBS_ERR_INVALID_ARG, "GICP: too many points");
    V.cap = (uint32_t)cap;
    int32_t *cnt = nullptr;
    bbs_status st;
    if ((st = alloc_dev((void **)&V.keys, cap * 8)) || (st = alloc_dev((void **)&V.index, cap * 4)) ||
        (st = alloc_dev((void **)&cnt, 8)))
        return st;
    BBS_HIP(hipMemsetAsync(cnt, 0, 8, s));
    k_g_fill<<<ggrid((int64_t)cap), kGThreads, 0, s>>>(V.keys, V.cap);
    k_g_insert<<<ggrid(n), kGThreads, 0, s>>>(p, n, voxel, V.keys, V.cap - 1, cnt + 1);
    k_g_number<<<ggrid((int64_t)cap), kGThreads, 0, s>>>(V.keys, V.cap, V.index, cnt);
    BBS_HIP(hipGetLastError());
    int32_t h[2];
    BBS_HIP(hipMemcpyAsync(h, cnt, 8, hipMemcpyDeviceToHost, s));
    BBS_HIP(hipStreamSynchronize(s));
    (void)hipFree(cnt);
    if (h[1]) return fail(BBS_ERR_INVALID_ARG, "GICP: a point is not finite or its voxel index leaves +-2^20");
    V.n = h[0];
    if ((st = alloc_dev((void **)&V.count, (size_t)std::max(V.n, 1) * 4)) ||
        (st = alloc_dev((void **)&V.sum, (size_t)std::max(V.n, 1) * 72)) ||
        (st = alloc_dev((void **)&V.dist, (size_t)std::max(V.n, 1) * 72)))
        return st;
    k_g_zero<<<ggrid(V.n), kGThreads, 0, s>>>(V.count, V.sum, V.n);
    k_g_accumulate<<<ggrid(n), kGThreads, 0, s>>>(p, n, voxel, V.keys, V.index, V.cap - 1, V.count, V.sum,
                                                   point_voxel);
    k_g_finalize<<<ggrid(V.n), kGThreads, 0, s>>>(V.count, V.sum, V.n, min_points, V.dist);
    BBS_HIP(hipGetLastError());
    return BBS_OK;
}

void so3_exp(const double w[3], double E[9])
{
    const double th = std::sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    if (th < 1e-12) {
        const double e[9] = {1.0, -w[2], w[1], w[2], 1.0, -w[0], -w[1], w[0], 1.0};
        std::copy(e, e + 9, E);
        return;
    }
    const double k[3] = {w[0] / th, w[1] / th, w[2] / th};
    const double K[9] = {0.0, -k[2], k[1], k[2], 0.0, -k[0], -k[1], k[0], 0.0};
    const double s = std::sin(th), c = 1.0 - std::cos(th);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double kk = 0.0;
            for (int m = 0; m < 3; ++m) kk += K[3 * i + m] * K[3 * m + j];
            E[3 * i + j] = (i == j ? 1.0 : 0.0) + s * K[3 * i + j] + c * kk;
        }
}

// Solve H x = b (6 x 6) by Gaussian elimination with partial pivoting.
bool solve6(double H[36], double b[6], double x[6])
{
    int piv[6] = {0, 1, 2, 3, 4, 5};
    for (int c = 0; c < 6; ++c) {
        int m = c;
        for (int r = c + 1; r < 6; ++r)
            if (std::fabs(H[6 * r + c]) > std::fabs(H[6 * m + c])) m = r;
        if (!(std::fabs(H[6 * m + c]) > 0.0)) return false;
        if (m != c) {
            for (int j = 0; j < 6; ++j) std::swap(H[6 * m + j], H[6 * c + j]);
            std::swap(b[m], b[c]);
            std::swap(piv[m], piv[c]);
        }
        for (int r = c + 1; r < 6; ++r) {
            const double f = H[6 * r + c] / H[6 * c + c];
            for (int j = c; j < 6; ++j) H[6 * r + j] -= f * H[6 * c + j];
            b[r] -= f * b[c];
        }
    }
    for (int r = 5; r >= 0; --r) {
        double v = b[r];
        for (int j = r + 1; j < 6; ++j) v -= H[6 * r + j] * x[j];
        x[r] = v / H[6 * r + r];
    }
    return true;
}

}  // namespace
}  // namespace bbs

struct bbs_gicp_target {
    bbs::VoxelStats V;
    double voxel = 1.0;
    int32_t device = 0;
};

extern "C" bbs_status bbs_gicp_target_create(const float *xyz, int64_t n, int32_t on_device, double voxel,
                                             int32_t min_points, void *stream, bbs_gicp_target **out)
{
    using namespace bbs;
    if (!out) return fail(BBS_ERR_INVALID_ARG, "bbs_gicp_target_create: out is NULL");
    *out = nullptr;
    if (!xyz || n < 1 || n >= ((int64_t)1 << 30))
        return fail(BBS_ERR_INVALID_ARG, "bbs_gicp_target_create: need 1 <= n < 2^30 points");
    if (!(voxel > 0.0) || !std::isfinite(voxel)) return fail(BBS_ERR_INVALID_ARG, "bbs_gicp_target_create: voxel must be > 0");
    if (min_points < 4) return fail(BBS_ERR_INVALID_ARG, "bbs_gicp_target_create: min_points must be >= 4");
    hipStream_t s = static_cast<hipStream_t>(stream);
    float *staged = nullptr;
    const float *p = xyz;
    bbs_status st;
    if (!on_device) {
        if ((st = alloc_dev((void **)&staged, (size_t)n * 12))) return st;
        BBS_HIP(hipMemcpyAsync(staged, xyz, (size_t)n * 12, hipMemcpyHostToDevice, s));
        p = staged;
    }
    bbs_gicp_target *t = new bbs_gicp_target();
    t->voxel = voxel;
    (void)hipGetDevice(&t->device);
    st = build_stats(p, n, voxel, min_points, s, t->V, nullptr);
    if (st == BBS_OK) {
        const hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = hip_fail(e, "bbs_gicp_target_create");
    }
    if (staged) (void)hipFree(staged);
    if (st) {
        t->V.release();
        delete t;
        return st;
    }
    *out = t;
    return BBS_OK;
}

extern "C" void bbs_gicp_target_free(bbs_gicp_target *t)
{
    if (!t) return;
    t->V.release();
    delete t;
}

namespace bbs {
namespace {

// A scan prepared for refinement: device points and per-point voxel index
// into the scan's own statistics.
struct ScanPrep {
    float *pts = nullptr;
    bool own = false;
    int32_t *vox = nullptr;
    double *partials = nullptr;
    VoxelStats V;
    ~ScanPrep()
    {
        if (own && pts) (void)hipFree(pts);
        if (vox) (void)hipFree(vox);
        if (partials) (void)hipFree(partials);
        V.release();
    }
};

bbs_status prep_scan(const bbs_gicp_target *t, const float *scan, int64_t k, int32_t on_device, int32_t min_points,
                     hipStream_t s, ScanPrep &S)
{
    if (!t) return fail(BBS_ERR_INVALID_ARG, "GICP: target is NULL");
    if (!scan || k < 1 || k >= ((int64_t)1 << 30)) return fail(BBS_ERR_INVALID_ARG, "GICP: need 1 <= k < 2^30 scan points");
    if (min_points < 4) return fail(BBS_ERR_INVALID_ARG, "GICP: min_points must be >= 4");
    bbs_status st;
    if (on_device) S.pts = const_cast<float *>(scan);
    else {
        if ((st = alloc_dev((void **)&S.pts, (size_t)k * 12))) return st;
        S.own = true;
        BBS_HIP(hipMemcpyAsync(S.pts, scan, (size_t)k * 12, hipMemcpyHostToDevice, s));
    }
    if ((st = alloc_dev((void **)&S.vox, (size_t)k * 4)) ||
        (st = alloc_dev((void **)&S.partials, (size_t)ggrid(k) * kPartials * 8)))
        return st;
    return build_stats(S.pts, k, t->voxel, min_points, s, S.V, S.vox);
}

bbs_status linearize_at(const bbs_gicp_target *t, const ScanPrep &S, int64_t k, const Pose &P, hipStream_t s,
                        double H[36], double g[6], double *cost, int64_t *pairs)
{
    const int grid = ggrid(k);
    k_g_linearize<<<grid, kGThreads, 0, s>>>(S.pts, k, S.vox, S.V.dist, t->V.keys, t->V.index, t->V.cap - 1,
                                             t->V.dist, t->voxel, P, S.partials);
    BBS_HIP(hipGetLastError());
    std::vector<double> part((size_t)grid * kPartials);
    BBS_HIP(hipMemcpyAsync(part.data(), S.partials, part.size() * 8, hipMemcpyDeviceToHost, s));
    BBS_HIP(hipStreamSynchronize(s));
    double acc[kPartials] = {};
    for (int b = 0; b < grid; ++b)
        for (int j = 0; j < kPartials; ++j) acc[j] += part[(size_t)b * kPartials + j];
    int m = 0;
    for (int a = 0; a < 6; ++a)
        for (int c = a; c < 6; ++c) {
            H[6 * a + c] = acc[m];
            H[6 * c + a] = acc[m];
            ++m;
        }
    for (int a = 0; a < 6; ++a) g[a] = acc[21 + a];
    *cost = acc[27];
    *pairs = (int64_t)acc[28];
    return BBS_OK;
}

}  // namespace
}  // namespace bbs

extern "C" bbs_status bbs_gicp_linearize(const bbs_gicp_target *target, const float *scan, int64_t k,
                                         int32_t on_device, const double R[9], const double t[3], int32_t min_points,
                                         void *stream, double H[36], double g[6], double *cost, int64_t *pairs)
{
    using namespace bbs;
    if (!R || !t || !H || !g || !cost || !pairs) return fail(BBS_ERR_INVALID_ARG, "bbs_gicp_linearize: NULL argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    ScanPrep S;
    bbs_status st = prep_scan(target, scan, k, on_device, min_points, s, S);
    if (st) return st;
    Pose P;
    std::copy(R, R + 9, P.R);
    std::copy(t, t + 3, P.t);
    return linearize_at(target, S, k, P, s, H, g, cost, pairs);
}

extern "C" void bbs_gicp_default_options(bbs_gicp_options *o)
{
    if (!o) return;
    o->max_iterations = 20;
    o->min_points = 5;
    o->eps_rot = 1e-6;
    o->eps_trans = 1e-5;
}

extern "C" bbs_status bbs_gicp_refine(const bbs_gicp_target *target, const float *scan, int64_t k, int32_t on_device,
                                      const double R0[9], const double t0[3], const bbs_gicp_options *opt,
                                      void *stream, bbs_gicp_result *out)
{
    using namespace bbs;
    if (!R0 || !t0 || !opt || !out) return fail(BBS_ERR_INVALID_ARG, "bbs_gicp_refine: NULL argument");
    if (opt->max_iterations < 0 || opt->max_iterations > 1000)
        return fail(BBS_ERR_INVALID_ARG, "bbs_gicp_refine: max_iterations must be in [0, 1000]");
    hipStream_t s = static_cast<hipStream_t>(stream);
    ScanPrep S;
    bbs_status st = prep_scan(target, scan, k, on_device, opt->min_points, s, S);
    if (st) return st;
    Pose P;
    std::copy(R0, R0 + 9, P.R);
    std::copy(t0, t0 + 3, P.t);
    double H[36], g[6], cost = 0.0;
    int64_t pairs = 0;
    int it = 0;
    bool converged = false;
    while (it < opt->max_iterations) {
        if ((st = linearize_at(target, S, k, P, s, H, g, &cost, &pairs))) return st;
        if (pairs < 6) break;
        double b[6], dx[6];
        for (int a = 0; a < 6; ++a) b[a] = -g[a];
        if (!solve6(H, b, dx)) break;
        double E[9];
        so3_exp(dx, E);
        Pose Q;
        for (int i = 0; i < 3; ++i) {
            for (int j = 0; j < 3; ++j)
                Q.R[3 * i + j] = E[3 * i] * P.R[j] + E[3 * i + 1] * P.R[3 + j] + E[3 * i + 2] * P.R[6 + j];
            Q.t[i] = E[3 * i] * P.t[0] + E[3 * i + 1] * P.t[1] + E[3 * i + 2] * P.t[2] + dx[3 + i];
        }
        P = Q;
        ++it;
        const double nw = std::sqrt(dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2]);
        const double nt = std::sqrt(dx[3] * dx[3] + dx[4] * dx[4] + dx[5] * dx[5]);
        if (nw < opt->eps_rot && nt < opt->eps_trans) {
            converged = true;
            break;
        }
    }
    if ((st = linearize_at(target, S, k, P, s, H, g, &cost, &pairs))) return st;
    std::copy(P.R, P.R + 9, out->R);
    std::copy(P.t, P.t + 3, out->t);
    out->cost = cost;
    out->pairs = pairs;
    out->iterations = it;
    out->converged = converged ? 1 : 0;
    return BBS_OK;
}
