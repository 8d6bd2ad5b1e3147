// Learned proposal network: BF16 MFMA training and inference kernels.
//
// A small encoder of the scan's bird's-eye polar occupancy (64 range x 64
// azimuth bins) gives a prior over 64 yaw bins and 32 x 32 translation cells.
// The search uses it only to order ties among the initial nodes and to seed
// the incumbent (bbs_localize options), never to change a node score.
//
// Layers: four 3x3 stride-2 convolutions (1->16->32->64->64 channels, zero
// padding along range, circular along azimuth, ReLU), FC 1024->256 (ReLU),
// FC 256->1088 (64 yaw + 1024 xy logits).  Weights and activations are bf16;
// every product runs on v_mfma_f32_16x16x16bf16_1k with float accumulation.
// Each layer is one GEMM whose operands are gathered on the fly: im2col for
// the forward pass and the weight gradient, its transpose for the input
// gradient.  Master weights and AdamW moments are float.
//
// Parameter order (flat, row-major): c1w [16,3,3,1] c1b, c2w [32,3,3,16] c2b,
// c3w [64,3,3,32] c3b, c4w [64,3,3,64] c4b, f1w [256,1024] f1b,
// f2w [1088,256] f2b.  Activations are [B, H, W, C].
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "bbs_internal.h"

namespace bbs {
namespace net {

constexpr int kBins = 64;
constexpr int kYaw = 64;
constexpr int kXY = 1024;
constexpr int kOut = kYaw + kXY;
constexpr int kCh[5] = {1, 16, 32, 64, 64};
constexpr int kF0 = 1024, kF1 = 256;

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__host__ __device__ inline uint16_t f2bf(float f)
{
    union {
        float f;
        uint32_t u;
    } c;
    c.f = f;
    uint32_t u = c.u + 0x7FFFu + ((c.u >> 16) & 1u);   // round to nearest, ties to even
    return (uint16_t)(u >> 16);
}

__host__ __device__ inline float bf2f(uint16_t h)
{
    union {
        uint32_t u;
        float f;
    } c;
    c.u = (uint32_t)h << 16;
    return c.f;
}

// ------------------------------------------------------------------ operand gathers (bf16 bits)

struct MatRM {          // M[r][c] = p[r * ld + c]
    const uint16_t *p;
    int ld;
    __device__ uint16_t operator()(int r, int c) const { return p[(int64_t)r * ld + c]; }
};

struct MatT {           // M[r][c] = p[c * ld + r]
    const uint16_t *p;
    int ld;
    __device__ uint16_t operator()(int r, int c) const { return p[(int64_t)c * ld + r]; }
};

// im2col of x [B, H, W, C]: row (b, oy, ox) of the stride-2 output, column
// (ky, kx, ci); padded row 2 oy + ky (zero outside), padded column 2 ox + kx
// (circular).
struct Im2col {
    const uint16_t *x;
    int H, W, C;
    __device__ uint16_t operator()(int m, int k) const
    {
        const int OW = W / 2, OH = H / 2;
        const int ci = k % C, kk = k / C, kx = kk % 3, ky = kk / 3;
        const int ox = m % OW, t = m / OW, oy = t % OH, b = t / OH;
        const int iy = 2 * oy + ky - 1;
        if (iy < 0 || iy >= H) return 0;
        const int ix = (2 * ox + kx - 1 + W) % W;
        return x[(((int64_t)b * H + iy) * W + ix) * C + ci];
    }
};

// Input-gradient operand: row (b, iy, ix) of the layer input, column
// (ky, kx, co); the output pixel that read this input through tap (ky, kx),
// if any (stride 2 and even W: at most one).
struct Dgrad {
    const uint16_t *dy;   // [B, OH, OW, Cout]
    int H, W, Cout;
    __device__ uint16_t operator()(int m, int k) const
    {
        const int OW = W / 2, OH = H / 2;
        const int co = k % Cout, kk = k / Cout, kx = kk % 3, ky = kk / 3;
        const int ix = m % W, t = m / W, iy = t % H, b = t / H;
        const int pr = iy + 1 - ky;
        if (pr < 0 || (pr & 1) || pr / 2 >= OH) return 0;
        const int oy = pr / 2;
        int ox = -1;
        int pc = ix + 1 - kx;
        if (pc >= 0 && !(pc & 1) && pc / 2 < OW) ox = pc / 2;
        else if (ix == W - 1 && kx == 0) ox = 0;     // left pad column holds x[W - 1]
        if (ox < 0) return 0;
        return dy[(((int64_t)b * OH + oy) * OW + ox) * Cout + co];
    }
};

// Weights as the input-gradient's B operand: row (ky, kx, co), column ci.
struct WDgrad {
    const uint16_t *w;    // [Cout, 3, 3, Cin]
    int Cin, Cout;
    __device__ uint16_t operator()(int k, int n) const
    {
        const int co = k % Cout, kk = k / Cout;
        return w[((int64_t)co * 9 + kk) * Cin + n];
    }
};

// ------------------------------------------------------------------ epilogues

struct EpiBiasRelu {    // bf16(relu(acc + bias))
    uint16_t *out;
    const float *bias;
    int ld;
    __device__ void operator()(int m, int n, float v) const
    {
        v += bias[n];
        out[(int64_t)m * ld + n] = f2bf(v > 0.0f ? v : 0.0f);
    }
};

struct EpiBiasF32 {     // logits
    float *out;
    const float *bias;
    int ld;
    __device__ void operator()(int m, int n, float v) const { out[(int64_t)m * ld + n] = v + bias[n]; }
};

struct EpiMaskBf16 {    // bf16(acc) where the forward activation is positive, else 0
    uint16_t *out;
    const uint16_t *act;
    int ld;
    __device__ void operator()(int m, int n, float v) const
    {
        const int64_t i = (int64_t)m * ld + n;
        out[i] = (act == nullptr || bf2f(act[i]) > 0.0f) ? f2bf(v) : (uint16_t)0;
    }
};

struct EpiSplitF32 {    // split-K partial of split blockIdx.z into out[split][M][N]
    float *out;
    int M, N;
    __device__ void operator()(int m, int n, float v) const { out[((int64_t)blockIdx.z * M + m) * N + n] = v; }
};

struct EpiAtomicF32 {   // accumulate into float (split K)
    float *out;
    int ld;
    __device__ void operator()(int m, int n, float v) const { atomicAdd(&out[(int64_t)m * ld + n], v); }
};

// ------------------------------------------------------------------ GEMM on MFMA

// C[M x N] = A[M x K] B[K x N].  A workgroup of 4 waves covers a 16 x 64
// block (one 16 x 16 tile per wave); blockIdx.z splits K.  Lane l feeds
// A[l % 16][4 (l / 16) + i] and B[4 (l / 16) + i][l % 16] (i < 4) and
// receives C[4 (l / 16) + i][l % 16].
template <class AOp, class BOp, class Epi>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, int kchunk, AOp A, BOp B, Epi E)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m0 = blockIdx.x * 16, n0 = (blockIdx.y * 4 + wave) * 16;
    const int kb = blockIdx.z * kchunk, ke = min(K, kb + kchunk);
    const int r = lane & 15, q = lane >> 4;
    v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
    if (n0 < N) {
        for (int k0 = kb; k0 < ke; k0 += 16) {
            v4s a, b;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int k = k0 + 4 * q + i;
                const bool kin = k < ke;
                a[i] = (short)((kin && m0 + r < M) ? A(m0 + r, k) : 0);
                b[i] = (short)((kin && n0 + r < N) ? B(k, n0 + r) : 0);
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m = m0 + 4 * q + i, n = n0 + r;
            if (m < M && n < N) E(m, n, acc[i]);
        }
    }
}

template <class AOp, class BOp, class Epi>
void gemm(hipStream_t s, int M, int N, int K, AOp A, BOp B, Epi E, int splits = 1)
{
    const int kchunk = ((K + splits - 1) / splits + 15) / 16 * 16;
    dim3 grid((M + 15) / 16, (N + 63) / 64, (K + kchunk - 1) / kchunk);
    k_gemm<<<grid, 256, 0, s>>>(M, N, K, kchunk, A, B, E);
}

// The partials of a split-K product summed in split order (deterministic),
// then the layer's epilogue.
template <class Epi>
__global__ void k_splitk_finish(const float *part, int splits, int M, int N, Epi E)
{
    const int64_t mn = (int64_t)M * N;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < mn; i += (int64_t)gridDim.x * blockDim.x) {
        float v = 0.0f;
        for (int sp = 0; sp < splits; ++sp) v += part[sp * mn + i];
        E((int)(i / N), (int)(i % N), v);
    }
}

// A forward product: when its output covers few workgroups (small batches,
// the inference path), K is split into up to 16 parts whose partials go to a
// scratch buffer, so that more workgroups share the reduction; a second
// kernel adds them in order and applies the epilogue.
template <class AOp, class BOp, class Epi>
void gemm_fwd(hipStream_t s, int M, int N, int K, AOp A, BOp B, Epi E, float *scratch, int64_t scratch_floats)
{
    const int tiles = ((M + 15) / 16) * ((N + 63) / 64);
    int splits = 1;
    if (tiles < 64 && K >= 128)
        splits = (int)std::max<int64_t>(1, std::min<int64_t>({16, K / 64, 128 / tiles,
                                                              scratch_floats / ((int64_t)M * N)}));
    if (splits <= 1) {
        gemm(s, M, N, K, A, B, E);
        return;
    }
    const int kchunk = ((K + splits - 1) / splits + 15) / 16 * 16;
    const int used = (K + kchunk - 1) / kchunk;            // splits that hold work
    dim3 grid((M + 15) / 16, (N + 63) / 64, used);
    k_gemm<<<grid, 256, 0, s>>>(M, N, K, kchunk, A, B, EpiSplitF32{scratch, M, N});
    const int64_t mn = (int64_t)M * N;
    k_splitk_finish<<<(int)std::min<int64_t>((mn + 255) / 256, 1024), 256, 0, s>>>(scratch, used, M, N, E);
}

// ------------------------------------------------------------------ small kernels

__global__ void k_input(const uint8_t *img, int64_t n, const uint16_t *table, uint16_t *x0)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x0[i] = table[img[i]];
}

// Softmax cross-entropy of both heads: loss += mean CE, dlogits = (softmax -
// onehot) / B as bf16.  One workgroup per sample.
__global__ __launch_bounds__(256) void k_loss(const float *logits, const int32_t *yaw, const int32_t *xy, int B,
                                             uint16_t *dlogits, float *loss)
{
    __shared__ float red[256];
    const int b = blockIdx.x;
    const float *z = logits + (int64_t)b * kOut;
    for (int head = 0; head < 2; ++head) {
        const int off = head ? kYaw : 0, n = head ? kXY : kYaw;
        const int label = head ? xy[b] : yaw[b];
        float mx = -INFINITY;
        for (int i = threadIdx.x; i < n; i += 256) mx = fmaxf(mx, z[off + i]);
        red[threadIdx.x] = mx;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
            __syncthreads();
        }
        mx = red[0];
        __syncthreads();
        float se = 0.0f;
        for (int i = threadIdx.x; i < n; i += 256) se += expf(z[off + i] - mx);
        red[threadIdx.x] = se;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
            __syncthreads();
        }
        const float lse = mx + logf(red[0]);
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += 256) {
            float p = expf(z[off + i] - lse);
            if (i == label) p -= 1.0f;
            dlogits[(int64_t)b * kOut + off + i] = f2bf(p / (float)B);
        }
        if (threadIdx.x == 0) atomicAdd(loss, (lse - z[off + label]) / (float)B);
    }
}

// Column sums of a bf16 [M x N] matrix into float (bias gradients).
__global__ void k_colsum(const uint16_t *dy, int M, int N, float *out)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int rows = (M + gridDim.y - 1) / gridDim.y;
    const int r0 = blockIdx.y * rows, r1 = min(M, r0 + rows);
    float s = 0.0f;
    for (int m = r0; m < r1; ++m) s += bf2f(dy[(int64_t)m * N + n]);
    atomicAdd(&out[n], s);
}

// The same for N dividing 256 (the convolutions' channel counts): thread t
// sums column t % N over rows t / N, t / N + 256 / N, ... of its block's
// rows, so that consecutive threads read consecutive elements; the block's
// partial sums meet in LDS and each column takes one atomic add per block.
__global__ __launch_bounds__(256) void k_colsum_narrow(const uint16_t *dy, int64_t M, int N, float *out)
{
    __shared__ float red[256];
    const int col = threadIdx.x % N, rstep = 256 / N;
    float acc = 0.0f;
    for (int64_t m = (int64_t)blockIdx.x * rstep + threadIdx.x / N; m < M; m += (int64_t)gridDim.x * rstep)
        acc += bf2f(dy[m * N + col]);
    red[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < N) {
        float t = 0.0f;
        for (int r = 0; r < rstep; ++r) t += red[r * N + threadIdx.x];
        atomicAdd(&out[threadIdx.x], t);
    }
}

__global__ void k_adamw(float *p, float *m, float *v, const float *g, uint16_t *pb, int64_t n, float lr, float b1,
                        float b2, float eps, float wd, float c1, float c2, const uint8_t *decay)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        float pi = p[i];
        if (decay[i]) pi -= lr * wd * pi;
        pi -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        p[i] = pi;
        pb[i] = f2bf(pi);
    }
}

__global__ void k_to_bf16(const float *p, uint16_t *pb, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        pb[i] = f2bf(p[i]);
}

// Bird's-eye polar counts: range bin floor(64 |(x, y)| / d_max) (clamped to
// 63), azimuth bin floor(64 atan2(y, x) / 2 pi) mod 64, min(255, count).
__global__ void k_bev_count(const float *xyz, int64_t k, float dmax, int32_t *cnt)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < k; i += (int64_t)gridDim.x * blockDim.x) {
        const float x = xyz[3 * i], y = xyz[3 * i + 1];
        const float rho = sqrtf(x * x + y * y);
        int rb = (int)(kBins * rho / dmax);
        rb = min(max(rb, 0), kBins - 1);
        int ab = (int)floorf(kBins * atan2f(y, x) / 6.283185307179586f);
        ab = ((ab % kBins) + kBins) % kBins;
        atomicAdd(&cnt[rb * kBins + ab], 1);
    }
}

__global__ void k_bev_pack(const int32_t *cnt, uint8_t *img)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kBins * kBins) img[i] = (uint8_t)min(cnt[i], 255);
}

// The largest squared range of the scan in double ((x*x + y*y) + z*z), as
// the bits of a non-negative double, by atomic maximum; a non-finite
// coordinate gives +inf.
__global__ void k_bev_maxsq(const float *xyz, int64_t k, unsigned long long *max_sq)
{
    __shared__ double sm[256];
    double m = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < k; i += (int64_t)gridDim.x * blockDim.x) {
        const double x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
        double d = x * x + y * y + z * z;
        if (!(d <= 1.0e300)) d = INFINITY;
        m = fmax(m, d);
    }
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(max_sq, (unsigned long long)__double_as_longlong(sm[0]));
}

// The BEV counts with d_max read from the device (float of the double square
// root, as the host path computes it); an empty or non-finite scan leaves
// the counts at zero and sets *bad.
__global__ void k_bev_count_dev(const float *xyz, int64_t k, const unsigned long long *max_sq, int32_t *cnt,
                                int32_t *bad)
{
    const double mx = __longlong_as_double((long long)*max_sq);
    const float dmax = (float)sqrt(mx);
    if (!(dmax > 0.0f) || !isfinite(dmax)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *bad = 1;
        return;
    }
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < k; i += (int64_t)gridDim.x * blockDim.x) {
        const float x = xyz[3 * i], y = xyz[3 * i + 1];
        const float rho = sqrtf(x * x + y * y);
        int rb = (int)(kBins * rho / dmax);
        rb = min(max(rb, 0), kBins - 1);
        int ab = (int)floorf(kBins * atan2f(y, x) / 6.283185307179586f);
        ab = ((ab % kBins) + kBins) % kBins;
        atomicAdd(&cnt[rb * kBins + ab], 1);
    }
}

struct Shapes {
    int64_t off[12], size[12], total;
    Shapes()
    {
        int64_t sz[12];
        for (int i = 0; i < 4; ++i) {
            sz[2 * i] = (int64_t)kCh[i + 1] * 9 * kCh[i];
            sz[2 * i + 1] = kCh[i + 1];
        }
        sz[8] = (int64_t)kF1 * kF0;
        sz[9] = kF1;
        sz[10] = (int64_t)kOut * kF1;
        sz[11] = kOut;
        total = 0;
        for (int i = 0; i < 12; ++i) {
            off[i] = total;
            size[i] = sz[i];
            total += sz[i];
        }
    }
};

}  // namespace net
}  // namespace bbs

using namespace bbs;
using namespace bbs::net;

struct bbs_net {
    int32_t max_batch = 0;
    hipStream_t own = nullptr;
    Shapes sh;
    float *p = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
    uint16_t *pb = nullptr;
    uint8_t *decay = nullptr;
    uint16_t *table = nullptr;
    uint16_t *x0 = nullptr, *a[5] = {nullptr, nullptr, nullptr, nullptr, nullptr}, *h1 = nullptr;
    float *logits = nullptr;
    uint16_t *dlog = nullptr, *dh1 = nullptr, *dh0 = nullptr, *da[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    float *loss = nullptr;
    int64_t step = 0;
    // on-device prior of one scan (bbs_net_prior): scan staging (grows),
    // squared range, BEV counts, failure flag
    float *scan = nullptr;
    int64_t scan_cap = 0;
    unsigned long long *maxsq = nullptr;
    int32_t *bev_cnt = nullptr;
    int32_t *bev_bad = nullptr;
    float *splitk = nullptr;              // split-K partials of small forward products
    std::vector<void *> owned;
};

constexpr int64_t kSplitKFloats = 1 << 20;

namespace {

bbs_status net_alloc(bbs_net *n, void **p, size_t bytes)
{
    bbs_status st = alloc_dev(p, bytes);
    if (st == BBS_OK) n->owned.push_back(*p);
    return st;
}

int act_hw(int layer) { return kBins >> layer; }   // spatial size of activation a[layer] (a[0] = input)

// Forward pass for `batch` images already converted into n->x0.
void forward(bbs_net *n, int batch, hipStream_t s)
{
    const Shapes &S = n->sh;
    const uint16_t *x = n->x0;
    for (int i = 0; i < 4; ++i) {
        const int H = act_hw(i), C = kCh[i], OH = H / 2, Co = kCh[i + 1];
        const uint16_t *w = n->pb + S.off[2 * i];
        gemm_fwd(s, batch * OH * OH, Co, 9 * C, Im2col{x, H, H, C}, MatT{w, 9 * C},
                 EpiBiasRelu{n->a[i + 1], n->p + S.off[2 * i + 1], Co}, n->splitk, kSplitKFloats);
        x = n->a[i + 1];
    }
    gemm_fwd(s, batch, kF1, kF0, MatRM{n->a[4], kF0}, MatT{n->pb + S.off[8], kF0},
             EpiBiasRelu{n->h1, n->p + S.off[9], kF1}, n->splitk, kSplitKFloats);
    gemm_fwd(s, batch, kOut, kF1, MatRM{n->h1, kF1}, MatT{n->pb + S.off[10], kF1},
             EpiBiasF32{n->logits, n->p + S.off[11], kOut}, n->splitk, kSplitKFloats);
}

// Backward pass from n->dlog into n->g (zeroed here).
bbs_status backward(bbs_net *n, int batch, hipStream_t s)
{
    const Shapes &S = n->sh;
    BBS_HIP(hipMemsetAsync(n->g, 0, (size_t)S.total * sizeof(float), s));
    const int B = batch;
    // fc2
    gemm(s, kOut, kF1, B, MatT{n->dlog, kOut}, MatRM{n->h1, kF1}, EpiAtomicF32{n->g + S.off[10], kF1}, 4);
    k_colsum<<<dim3((kOut + 255) / 256, 8), 256, 0, s>>>(n->dlog, B, kOut, n->g + S.off[11]);
    gemm(s, B, kF1, kOut, MatRM{n->dlog, kOut}, MatRM{n->pb + S.off[10], kF1}, EpiMaskBf16{n->dh1, n->h1, kF1});
    // fc1
    gemm(s, kF1, kF0, B, MatT{n->dh1, kF1}, MatRM{n->a[4], kF0}, EpiAtomicF32{n->g + S.off[8], kF0}, 4);
    k_colsum<<<dim3((kF1 + 255) / 256, 8), 256, 0, s>>>(n->dh1, B, kF1, n->g + S.off[9]);
    gemm(s, B, kF0, kF1, MatRM{n->dh1, kF1}, MatRM{n->pb + S.off[8], kF0}, EpiMaskBf16{n->da[4], n->a[4], kF0});
    // convolutions, last to first; da[i] is the gradient of a[i]
    for (int i = 3; i >= 0; --i) {
        const int H = act_hw(i), C = kCh[i], OH = H / 2, Co = kCh[i + 1];
        const uint16_t *dy = n->da[i + 1];
        const int Mo = B * OH * OH;
        // the weight gradient reduces over all Mo output pixels into a small
        // Co x 9C block: split K so that there are enough workgroups to fill
        // the device (256 output rows a workgroup)
        const int splits = std::max(1, std::min(1024, Mo / 256));
        gemm(s, Co, 9 * C, Mo, MatT{dy, Co}, Im2col{i == 0 ? n->x0 : n->a[i], H, H, C},
             EpiAtomicF32{n->g + S.off[2 * i], 9 * C}, splits);
        static_assert(256 % kCh[1] == 0 && 256 % kCh[2] == 0 && 256 % kCh[3] == 0 && 256 % kCh[4] == 0,
                      "conv channel counts divide the block");
        k_colsum_narrow<<<std::max(1, std::min(512, Mo / (256 / Co) / 16)), 256, 0, s>>>(dy, Mo, Co,
                                                                                      n->g + S.off[2 * i + 1]);
        if (i > 0)
            gemm(s, B * H * H, C, 9 * Co, Dgrad{dy, H, H, Co}, WDgrad{n->pb + S.off[2 * i], C, Co},
                 EpiMaskBf16{n->da[i], n->a[i], C});
    }
    BBS_HIP(hipGetLastError());
    return BBS_OK;
}

bbs_status load_images(bbs_net *n, const uint8_t *images, int32_t on_device, int batch, hipStream_t s)
{
    const int64_t cnt = (int64_t)batch * kBins * kBins;
    const uint8_t *src = images;
    if (!on_device) {
        // stage through the first bytes of the last activation-gradient buffer (large enough: B*64*64*2 bytes)
        BBS_HIP(hipMemcpyAsync(n->da[1], images, (size_t)cnt, hipMemcpyHostToDevice, s));
        src = reinterpret_cast<const uint8_t *>(n->da[1]);
    }
    k_input<<<(int)std::min<int64_t>((cnt + 255) / 256, 4096), 256, 0, s>>>(src, cnt, n->table, n->x0);
    BBS_HIP(hipGetLastError());
    return BBS_OK;
}

}  // namespace

extern "C" int64_t bbs_net_param_count(void) { return Shapes().total; }

extern "C" bbs_status bbs_net_create(int32_t max_batch, bbs_net **out)
{
    if (!out) return fail(BBS_ERR_INVALID_ARG, "bbs_net_create: out is NULL");
    *out = nullptr;
    if (max_batch < 1 || max_batch > 65536) return fail(BBS_ERR_INVALID_ARG, "bbs_net_create: max_batch in [1, 65536]");
    bbs_net *n = new bbs_net();
    n->max_batch = max_batch;
    const int64_t P = n->sh.total, B = max_batch;
    bool bad = net_alloc(n, (void **)&n->p, P * 4) || net_alloc(n, (void **)&n->m, P * 4) ||
               net_alloc(n, (void **)&n->v, P * 4) || net_alloc(n, (void **)&n->g, P * 4) ||
               net_alloc(n, (void **)&n->pb, P * 2) || net_alloc(n, (void **)&n->decay, P) ||
               net_alloc(n, (void **)&n->table, 256 * 2) || net_alloc(n, (void **)&n->x0, B * 64 * 64 * 2) ||
               net_alloc(n, (void **)&n->h1, B * kF1 * 2) || net_alloc(n, (void **)&n->logits, B * kOut * 4) ||
               net_alloc(n, (void **)&n->dlog, B * kOut * 2) || net_alloc(n, (void **)&n->dh1, B * kF1 * 2) ||
               net_alloc(n, (void **)&n->loss, 64) || net_alloc(n, (void **)&n->maxsq, 64) ||
               net_alloc(n, (void **)&n->bev_cnt, kBins * kBins * 4) || net_alloc(n, (void **)&n->bev_bad, 64) ||
               net_alloc(n, (void **)&n->splitk, kSplitKFloats * 4);
    for (int i = 1; i <= 4 && !bad; ++i) {
        const int64_t e = B * act_hw(i) * act_hw(i) * kCh[i];
        bad = net_alloc(n, (void **)&n->a[i], e * 2) || net_alloc(n, (void **)&n->da[i], std::max<int64_t>(e, B * 4096) * 2);
    }
    if (bad) {
        bbs_net_free(n);
        return BBS_ERR_OOM;
    }
    hipError_t e = hipStreamCreateWithFlags(&n->own, hipStreamNonBlocking);
    if (e != hipSuccess) {
        bbs_net_free(n);
        return hip_fail(e, "hipStreamCreateWithFlags");
    }
    std::vector<uint16_t> table(256);
    for (int c = 0; c < 256; ++c) table[c] = f2bf((float)(std::log2(1.0 + c) / 8.0));
    std::vector<uint8_t> decay((size_t)P, 0);
    for (int i = 0; i < 12; i += 2)
        std::fill(decay.begin() + n->sh.off[i], decay.begin() + n->sh.off[i] + n->sh.size[i], 1);
    e = hipMemcpy(n->table, table.data(), 512, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(n->decay, decay.data(), (size_t)P, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(n->m, 0, (size_t)P * 4);
    if (e == hipSuccess) e = hipMemset(n->v, 0, (size_t)P * 4);
    if (e == hipSuccess) e = hipMemset(n->p, 0, (size_t)P * 4);
    if (e == hipSuccess) e = hipMemset(n->pb, 0, (size_t)P * 2);
    if (e != hipSuccess) {
        bbs_net_free(n);
        return hip_fail(e, "bbs_net_create");
    }
    *out = n;
    return BBS_OK;
}

extern "C" void bbs_net_free(bbs_net *n)
{
    if (!n) return;
    for (void *p : n->owned) (void)hipFree(p);
    if (n->own) (void)hipStreamDestroy(n->own);
    delete n;
}

extern "C" bbs_status bbs_net_set_params(bbs_net *n, const float *params, int64_t count)
{
    if (!n || !params) return fail(BBS_ERR_INVALID_ARG, "bbs_net_set_params: NULL argument");
    if (count != n->sh.total) return fail(BBS_ERR_INVALID_ARG, "bbs_net_set_params: wrong parameter count");
    BBS_HIP(hipMemcpyAsync(n->p, params, (size_t)count * 4, hipMemcpyHostToDevice, n->own));
    BBS_HIP(hipMemsetAsync(n->m, 0, (size_t)count * 4, n->own));
    BBS_HIP(hipMemsetAsync(n->v, 0, (size_t)count * 4, n->own));
    k_to_bf16<<<1024, 256, 0, n->own>>>(n->p, n->pb, count);
    BBS_HIP(hipGetLastError());
    BBS_HIP(hipStreamSynchronize(n->own));
    n->step = 0;
    return BBS_OK;
}

extern "C" bbs_status bbs_net_get_params(const bbs_net *n, float *params, int64_t count)
{
    if (!n || !params) return fail(BBS_ERR_INVALID_ARG, "bbs_net_get_params: NULL argument");
    if (count != n->sh.total) return fail(BBS_ERR_INVALID_ARG, "bbs_net_get_params: wrong parameter count");
    BBS_HIP(hipMemcpy(params, n->p, (size_t)count * 4, hipMemcpyDeviceToHost));
    return BBS_OK;
}

extern "C" bbs_status bbs_net_forward(bbs_net *n, const uint8_t *images, int32_t images_on_device, int32_t batch,
                                      float *logits)
{
    if (!n || !images || !logits) return fail(BBS_ERR_INVALID_ARG, "bbs_net_forward: NULL argument");
    if (batch < 1 || batch > n->max_batch) return fail(BBS_ERR_INVALID_ARG, "bbs_net_forward: batch out of range");
    hipStream_t s = n->own;
    bbs_status st = load_images(n, images, images_on_device, batch, s);
    if (st) return st;
    forward(n, batch, s);
    BBS_HIP(hipGetLastError());
    BBS_HIP(hipMemcpyAsync(logits, n->logits, (size_t)batch * kOut * 4, hipMemcpyDeviceToHost, s));
    BBS_HIP(hipStreamSynchronize(s));
    return BBS_OK;
}

// The prior of one scan: its BEV image and the forward pass, on the device
// (d_max included), with only the 1088 logits copied back.
extern "C" bbs_status bbs_net_prior(bbs_net *n, const float *scan_xyz, int64_t k, int32_t scan_on_device,
                                    float *logits)
{
    if (!n || !scan_xyz || !logits || k < 1) return fail(BBS_ERR_INVALID_ARG, "bbs_net_prior: bad arguments");
    hipStream_t s = n->own;
    const float *dev = scan_xyz;
    if (!scan_on_device) {
        if (n->scan_cap < k) {
            void *q = nullptr;
            if (alloc_dev(&q, (size_t)k * 12)) return BBS_ERR_OOM;
            if (n->scan) {
                n->owned.erase(std::find(n->owned.begin(), n->owned.end(), (void *)n->scan));
                (void)hipFree(n->scan);
            }
            n->owned.push_back(q);
            n->scan = static_cast<float *>(q);
            n->scan_cap = k;
        }
        BBS_HIP(hipMemcpyAsync(n->scan, scan_xyz, (size_t)k * 12, hipMemcpyHostToDevice, s));
        dev = n->scan;
    }
    BBS_HIP(hipMemsetAsync(n->maxsq, 0, 8, s));
    BBS_HIP(hipMemsetAsync(n->bev_cnt, 0, kBins * kBins * 4, s));
    BBS_HIP(hipMemsetAsync(n->bev_bad, 0, 4, s));
    const int grid = (int)std::min<int64_t>((k + 255) / 256, 1024);
    k_bev_maxsq<<<grid, 256, 0, s>>>(dev, k, n->maxsq);
    k_bev_count_dev<<<grid, 256, 0, s>>>(dev, k, n->maxsq, n->bev_cnt, n->bev_bad);
    uint8_t *img = reinterpret_cast<uint8_t *>(n->da[1]);   // as load_images stages host images
    k_bev_pack<<<kBins * kBins / 256, 256, 0, s>>>(n->bev_cnt, img);
    BBS_HIP(hipGetLastError());
    bbs_status st = load_images(n, img, 1, 1, s);
    if (st) return st;
    forward(n, 1, s);
    BBS_HIP(hipGetLastError());
    int32_t bad = 0;
    BBS_HIP(hipMemcpyAsync(logits, n->logits, kOut * 4, hipMemcpyDeviceToHost, s));
    BBS_HIP(hipMemcpyAsync(&bad, n->bev_bad, 4, hipMemcpyDeviceToHost, s));
    BBS_HIP(hipStreamSynchronize(s));
    if (bad) return fail(BBS_ERR_INVALID_ARG, "bbs_net_prior: scan range must be finite and > 0");
    return BBS_OK;
}

// One optimisation step (or, with lr < 0, only the gradients: copied to
// grads_out when it is not NULL).
extern "C" bbs_status bbs_net_train_step(bbs_net *n, const uint8_t *images, int32_t images_on_device,
                                         const int32_t *yaw, const int32_t *xy, int32_t batch, float lr,
                                         float weight_decay, float *loss_out, float *grads_out)
{
    if (!n || !images || !yaw || !xy) return fail(BBS_ERR_INVALID_ARG, "bbs_net_train_step: NULL argument");
    if (batch < 1 || batch > n->max_batch) return fail(BBS_ERR_INVALID_ARG, "bbs_net_train_step: batch out of range");
    for (int i = 0; i < batch; ++i)
        if (yaw[i] < 0 || yaw[i] >= kYaw || xy[i] < 0 || xy[i] >= kXY)
            return fail(BBS_ERR_INVALID_ARG, "bbs_net_train_step: label out of range");
    hipStream_t s = n->own;
    bbs_status st = load_images(n, images, images_on_device, batch, s);
    if (st) return st;
    forward(n, batch, s);
    int32_t *lab = reinterpret_cast<int32_t *>(n->dh1);   // labels staged in a buffer not yet in use
    // dh1 holds B * 256 bf16 = 512 B bytes >= 8 B bytes for the two label arrays
    BBS_HIP(hipMemcpyAsync(lab, yaw, (size_t)batch * 4, hipMemcpyHostToDevice, s));
    BBS_HIP(hipMemcpyAsync(lab + batch, xy, (size_t)batch * 4, hipMemcpyHostToDevice, s));
    BBS_HIP(hipMemsetAsync(n->loss, 0, 4, s));
    k_loss<<<batch, 256, 0, s>>>(n->logits, lab, lab + batch, batch, n->dlog, n->loss);
    st = backward(n, batch, s);
    if (st) return st;
    if (lr >= 0.0f) {
        n->step += 1;
        const float b1 = 0.9f, b2 = 0.999f;
        const float c1 = 1.0f - std::pow(b1, (float)n->step), c2 = 1.0f - std::pow(b2, (float)n->step);
        k_adamw<<<1024, 256, 0, s>>>(n->p, n->m, n->v, n->g, n->pb, n->sh.total, lr, b1, b2, 1e-8f, weight_decay, c1,
                                     c2, n->decay);
    }
    BBS_HIP(hipGetLastError());
    float loss = 0.0f;
    BBS_HIP(hipMemcpyAsync(&loss, n->loss, 4, hipMemcpyDeviceToHost, s));
    if (grads_out) BBS_HIP(hipMemcpyAsync(grads_out, n->g, (size_t)n->sh.total * 4, hipMemcpyDeviceToHost, s));
    BBS_HIP(hipStreamSynchronize(s));
    if (loss_out) *loss_out = loss;
    return BBS_OK;
}

extern "C" bbs_status bbs_bev_image(const float *scan_xyz, int64_t k, int32_t scan_on_device, uint8_t *image)
{
    if (!scan_xyz || !image || k < 1) return fail(BBS_ERR_INVALID_ARG, "bbs_bev_image: bad arguments");
    std::vector<float> host;
    const float *hp = scan_xyz;
    hipStream_t s = nullptr;
    BBS_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    void *d = nullptr, *cnt = nullptr, *img = nullptr;
    auto cleanup = [&]() {
        if (d) (void)hipFree(d);
        if (cnt) (void)hipFree(cnt);
        if (img) (void)hipFree(img);
        (void)hipStreamDestroy(s);
    };
    if (alloc_dev(&cnt, kBins * kBins * 4) || alloc_dev(&img, kBins * kBins)) {
        cleanup();
        return BBS_ERR_OOM;
    }
    const float *dev = scan_xyz;
    if (scan_on_device) {
        host.resize((size_t)k * 3);
        hipError_t e = hipMemcpy(host.data(), scan_xyz, (size_t)k * 12, hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
            cleanup();
            return hip_fail(e, "bbs_bev_image");
        }
        hp = host.data();
    } else {
        if (alloc_dev(&d, (size_t)k * 12)) {
            cleanup();
            return BBS_ERR_OOM;
        }
        hipError_t e = hipMemcpyAsync(d, scan_xyz, (size_t)k * 12, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) {
            cleanup();
            return hip_fail(e, "bbs_bev_image");
        }
        dev = static_cast<const float *>(d);
    }
    double mx = 0.0;
    for (int64_t i = 0; i < k; ++i) {
        double x = hp[3 * i], y = hp[3 * i + 1], z = hp[3 * i + 2];
        mx = std::max(mx, x * x + y * y + z * z);
    }
    const float dmax = (float)std::sqrt(mx);
    if (!(dmax > 0.0f) || !std::isfinite(dmax)) {
        cleanup();
        return fail(BBS_ERR_INVALID_ARG, "bbs_bev_image: scan range must be finite and > 0");
    }
    hipError_t e = hipMemsetAsync(cnt, 0, kBins * kBins * 4, s);
    if (e == hipSuccess) {
        k_bev_count<<<(int)std::min<int64_t>((k + 255) / 256, 1024), 256, 0, s>>>(dev, k, dmax,
                                                                                   static_cast<int32_t *>(cnt));
        k_bev_pack<<<kBins * kBins / 256, 256, 0, s>>>(static_cast<int32_t *>(cnt), static_cast<uint8_t *>(img));
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(image, img, kBins * kBins, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    cleanup();
    if (e != hipSuccess) return hip_fail(e, "bbs_bev_image");
    return BBS_OK;
}
