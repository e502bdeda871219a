// Learned low-rank factor for the Section 3.2 preconditioner P = U U^T + lambda I.
//
// Network (one row per input point, inputs x / l):
//     a1 = x W1 + b1,  h1 = gelu(a1),  a2 = h1 W2 + b2,  h2 = gelu(a2),
//     U  = h2 W3 + b3,  gelu(a) = a (1 + erf(a / sqrt 2)) / 2.
// Weights are kept as FP32 master copies (trained by Adam) and as BF16 copies
// packed in MFMA operand order for the forward pass.
//
// Forward (inference and training): one fused kernel; each wave carries 16
// rows through all three layers on 16x16x32 BF16 MFMA with FP32
// accumulation.  The hidden activations pass between layers through a
// per-wave LDS tile (FP32 MFMA results -> BF16 -> A-operand layout).
//
// Training loss on probe pairs (Z, K Z): L = |U (U^T Z) - K Z|_F^2 / |K Z|_F^2,
// gradient dL/dU = 2 (R M^T + Z (R^T U)) / |K Z|^2 with M = U^T Z,
// R = U M - K Z, then the chain rule through the layers.  Backward products
// run on an FP32 tiled GEMM (exact FP32 operands, split reductions summed in
// a fixed order).

#include "pkm_internal.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace pkm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int HID = 128;   // hidden width (fixed)

struct MlpLayout {
    int64_t W1, b1, W2, b2, W3, b3, total;
};

static MlpLayout layout(int d_in, int hidden, int rank) {
    MlpLayout L;
    L.W1 = 0;
    L.b1 = L.W1 + int64_t(d_in) * hidden;
    L.W2 = L.b1 + hidden;
    L.b2 = L.W2 + int64_t(hidden) * hidden;
    L.W3 = L.b2 + hidden;
    L.b3 = L.W3 + int64_t(hidden) * rank;
    L.total = L.b3 + rank;
    return L;
}

// packed BF16 weights: W (K x N, FP32 row-major) -> [kb][ct][lane][8]
//   element (kb, ct, lane, q) = W[32 kb + 8 (lane / 16) + q][16 ct + lane % 16]
__global__ void k_pack_w(const float* __restrict__ W, int K, int N, int KB, int CT,
                         __bf16* __restrict__ out) {
    int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    int64_t tot = int64_t(KB) * CT * 64 * 8;
    if (e >= tot) return;
    int q = int(e & 7);
    int lane = int((e >> 3) & 63);
    int64_t rest = e >> 9;
    int ct = int(rest % CT);
    int kb = int(rest / CT);
    int k = 32 * kb + 8 * (lane >> 4) + q;
    int c = 16 * ct + (lane & 15);
    out[e] = (__bf16)((k < K && c < N) ? W[int64_t(k) * N + c] : 0.0f);
}

__device__ inline float gelu_f(float a) { return 0.5f * a * (1.0f + erff(a * 0.70710678118654752f)); }
__device__ inline float gelu_grad_f(float a) {
    return 0.5f * (1.0f + erff(a * 0.70710678118654752f)) +
           a * 0.39894228040143268f * __expf(-0.5f * a * a);
}

// Fused forward.  Work-group: 4 waves x 16 rows.  RT = rank / 16.
// Writes a1, a2 (FP32, n x 128) when train != 0, U32 (FP32, n x rank) when
// non-null and U64 (FP64, n x rank) when non-null.
template <int RT>
__global__ __launch_bounds__(256) void k_mlp_fwd(const double* __restrict__ xs, int d_in,
                                                 int64_t n, const bf16x8* __restrict__ w1p,
                                                 const bf16x8* __restrict__ w2p,
                                                 const bf16x8* __restrict__ w3p,
                                                 const float* __restrict__ p32, int64_t ob1,
                                                 int64_t ob2, int64_t ob3,
                                                 float* __restrict__ a1, float* __restrict__ a2,
                                                 float* __restrict__ U32, double* __restrict__ U64) {
    __shared__ __bf16 hb[4][16][HID + 8];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = lane >> 4, cc = lane & 15;
    const int64_t row0 = (int64_t(blockIdx.x) * 4 + w) * 16;
    // layer 1: A = x rows (BF16), K = d_in padded to 32
    bf16x8 ax;
    {
        const int64_t row = row0 + cc;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int k = 8 * g + q;
            ax[q] = (__bf16)((row < n && k < d_in) ? float(xs[row * d_in + k]) : 0.0f);
        }
    }
    f32x4 acc[8];
#pragma unroll
    for (int ct = 0; ct < 8; ++ct)
        acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ax, w1p[ct * 64 + lane], f32x4{0, 0, 0, 0}, 0, 0, 0);
    // bias, store pre-activation, gelu, BF16 to LDS (rows 4 g + r, col 16 ct + cc)
#pragma unroll
    for (int ct = 0; ct < 8; ++ct) {
        const float bb = p32[ob1 + 16 * ct + cc];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float a = acc[ct][r] + bb;
            const int64_t row = row0 + 4 * g + r;
            if (a1 && row < n) a1[row * HID + 16 * ct + cc] = a;
            hb[w][4 * g + r][16 * ct + cc] = (__bf16)gelu_f(a);
        }
    }
    __syncthreads();
    // layer 2
#pragma unroll
    for (int ct = 0; ct < 8; ++ct) acc[ct] = f32x4{0, 0, 0, 0};
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
        bf16x8 ah;
#pragma unroll
        for (int q = 0; q < 8; ++q) ah[q] = hb[w][cc][32 * kb + 8 * g + q];
#pragma unroll
        for (int ct = 0; ct < 8; ++ct)
            acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, w2p[(kb * 8 + ct) * 64 + lane], acc[ct], 0, 0, 0);
    }
    __syncthreads();
#pragma unroll
    for (int ct = 0; ct < 8; ++ct) {
        const float bb = p32[ob2 + 16 * ct + cc];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float a = acc[ct][r] + bb;
            const int64_t row = row0 + 4 * g + r;
            if (a2 && row < n) a2[row * HID + 16 * ct + cc] = a;
            hb[w][4 * g + r][16 * ct + cc] = (__bf16)gelu_f(a);
        }
    }
    __syncthreads();
    // layer 3
    f32x4 au[RT];
#pragma unroll
    for (int ct = 0; ct < RT; ++ct) au[ct] = f32x4{0, 0, 0, 0};
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
        bf16x8 ah;
#pragma unroll
        for (int q = 0; q < 8; ++q) ah[q] = hb[w][cc][32 * kb + 8 * g + q];
#pragma unroll
        for (int ct = 0; ct < RT; ++ct)
            au[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, w3p[(kb * RT + ct) * 64 + lane], au[ct], 0, 0, 0);
    }
    const int rank = 16 * RT;
#pragma unroll
    for (int ct = 0; ct < RT; ++ct) {
        const float bb = p32[ob3 + 16 * ct + cc];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t row = row0 + 4 * g + r;
            if (row < n) {
                const float u = au[ct][r] + bb;
                if (U32) U32[row * rank + 16 * ct + cc] = u;
                if (U64) U64[row * rank + 16 * ct + cc] = double(u);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// FP32 GEMM for the backward pass: C = alpha op(A) op(B) + beta C, row-major.
// ---------------------------------------------------------------------------
constexpr int ST = 64, SK = 16;

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_sgemm(int64_t M, int64_t N, int64_t K, float alpha,
                                               const float* __restrict__ A, int64_t lda,
                                               const float* __restrict__ B, int64_t ldb,
                                               float beta, float* __restrict__ C, int64_t ldc,
                                               int64_t kchunk, float* __restrict__ part) {
    __shared__ float sa[SK][ST + 1];
    __shared__ float sb[SK][ST + 1];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int64_t i0 = int64_t(blockIdx.y) * ST, j0 = int64_t(blockIdx.x) * ST;
    const int64_t kbeg = int64_t(blockIdx.z) * kchunk;
    const int64_t kend = min(K, kbeg + kchunk);
    float acc[4][4] = {};
    for (int64_t k0 = kbeg; k0 < kend; k0 += SK) {
        for (int e = threadIdx.x; e < SK * ST; e += 256) {
            int kk, ii;
            if (TA) { ii = e % ST; kk = e / ST; } else { kk = e % SK; ii = e / SK; }
            int64_t gi = i0 + ii, gk = k0 + kk;
            sa[kk][ii] = (gi < M && gk < kend) ? (TA ? A[gk * lda + gi] : A[gi * lda + gk]) : 0.f;
        }
        for (int e = threadIdx.x; e < SK * ST; e += 256) {
            int kk, jj;
            if (TB) { kk = e % SK; jj = e / SK; } else { jj = e % ST; kk = e / ST; }
            int64_t gj = j0 + jj, gk = k0 + kk;
            sb[kk][jj] = (gj < N && gk < kend) ? (TB ? B[gj * ldb + gk] : B[gk * ldb + gj]) : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < SK; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                a[q] = sa[kk][ty + 16 * q];
                b[q] = sb[kk][tx + 16 * q];
            }
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[p][q] = fmaf(a[p], b[q], acc[p][q]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        int64_t gi = i0 + ty + 16 * p;
        if (gi >= M) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int64_t gj = j0 + tx + 16 * q;
            if (gj >= N) continue;
            if (part) part[int64_t(blockIdx.z) * M * N + gi * N + gj] = acc[p][q];
            else C[gi * ldc + gj] = alpha * acc[p][q] + (beta != 0.f ? beta * C[gi * ldc + gj] : 0.f);
        }
    }
}

__global__ void k_sgemm_reduce(int64_t M, int64_t N, int nsplit, const float* __restrict__ part,
                               float alpha, float beta, float* __restrict__ C, int64_t ldc) {
    int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= M * N) return;
    int64_t i = e / N, j = e - i * N;
    float s = 0.f;
    for (int z = 0; z < nsplit; ++z) s += part[z * M * N + e];
    C[i * ldc + j] = alpha * s + (beta != 0.f ? beta * C[i * ldc + j] : 0.f);
}

static void sgemm(pkm_ctx* ctx, pkm_mlp* net, bool ta, bool tb, int64_t M, int64_t N, int64_t K,
                  float alpha, const float* A, int64_t lda, const float* B, int64_t ldb, float beta,
                  float* C, int64_t ldc) {
    hipStream_t s = ctx->stream;
    if (M <= 0 || N <= 0) return;
    PKM_REQUIRE(cdiv(M, ST) <= 65535, "sgemm: M too large");
    int64_t tiles = cdiv(M, ST) * cdiv(N, ST);
    int nsplit = 1;
    while (tiles * nsplit < 1024 && K / (nsplit * 2) >= 512 && nsplit < 512) nsplit *= 2;
    int64_t kchunk = round_up(cdiv(K, nsplit), SK);
    nsplit = int(cdiv(K, kchunk));
    float* part = nullptr;
    if (nsplit > 1) {
        net->split.ensure(sizeof(float) * M * N * nsplit);
        part = net->split.as<float>();
    }
    dim3 grid((unsigned)cdiv(N, ST), (unsigned)cdiv(M, ST), (unsigned)nsplit);
    if (!ta && !tb) k_sgemm<false, false><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, part);
    else if (ta && !tb) k_sgemm<true, false><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, part);
    else if (!ta && tb) k_sgemm<false, true><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, part);
    else k_sgemm<true, true><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, part);
    PKM_CHECK_LAUNCH();
    if (nsplit > 1) {
        k_sgemm_reduce<<<cdiv(M * N, 256), 256, 0, s>>>(M, N, nsplit, part, alpha, beta, C, ldc);
        PKM_CHECK_LAUNCH();
    }
}

// ---- elementwise helpers ----
__global__ void k_f64_to_f32(int64_t tot, const double* __restrict__ a, float* __restrict__ b) {
    int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e < tot) b[e] = float(a[e]);
}
__global__ void k_gelu(int64_t tot, const float* __restrict__ a, float* __restrict__ h) {
    int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e < tot) h[e] = gelu_f(a[e]);
}
__global__ void k_mul_gelu_grad(int64_t tot, const float* __restrict__ a, float* __restrict__ d) {
    int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e < tot) d[e] *= gelu_grad_f(a[e]);
}
__global__ void k_fill(int64_t tot, float v, float* __restrict__ a) {
    int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e < tot) a[e] = v;
}
// per-block partial sums (FP64) of a[e] * b[e]
__global__ void k_sdot_part(int64_t tot, const float* __restrict__ a, const float* __restrict__ b,
                            double* __restrict__ part) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int64_t e = blockIdx.x * int64_t(256) + threadIdx.x; e < tot; e += int64_t(gridDim.x) * 256)
        acc += double(a[e]) * double(b[e]);
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}
__global__ void k_adam(int64_t tot, float* __restrict__ w, const float* __restrict__ g,
                       float* __restrict__ m, float* __restrict__ v, float lr, float b1, float b2,
                       float c1, float c2, float eps) {
    int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= tot) return;
    const float gg = g[e];
    const float mm = b1 * m[e] + (1.f - b1) * gg;
    const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
    m[e] = mm;
    v[e] = vv;
    w[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

static double sdot(pkm_ctx* ctx, pkm_mlp* net, int64_t tot, const float* a, const float* b) {
    const int nb = 256;
    net->scal.ensure(sizeof(double) * nb);
    k_sdot_part<<<nb, 256, 0, ctx->stream>>>(tot, a, b, net->scal.as<double>());
    PKM_CHECK_LAUNCH();
    std::vector<double> h(nb);
    PKM_HIP(hipMemcpyAsync(h.data(), net->scal.p, sizeof(double) * nb, hipMemcpyDeviceToHost, ctx->stream));
    PKM_HIP(hipStreamSynchronize(ctx->stream));
    double s = 0.0;
    for (double v : h) s += v;
    return s;
}

static void repack(pkm_ctx* ctx, pkm_mlp* net) {
    const MlpLayout L = layout(net->d_in, net->hidden, net->rank);
    const int RT = net->rank / 16;
    __bf16* wp = net->wpack.as<__bf16>();
    const float* p = net->p32.as<float>();
    hipStream_t s = ctx->stream;
    const int64_t n1 = int64_t(1) * 8 * 512, n2 = int64_t(4) * 8 * 512, n3 = int64_t(4) * RT * 512;
    k_pack_w<<<cdiv(n1, 256), 256, 0, s>>>(p + L.W1, net->d_in, HID, 1, 8, wp);
    k_pack_w<<<cdiv(n2, 256), 256, 0, s>>>(p + L.W2, HID, HID, 4, 8, wp + n1);
    k_pack_w<<<cdiv(n3, 256), 256, 0, s>>>(p + L.W3, HID, net->rank, 4, RT, wp + n1 + n2);
    PKM_CHECK_LAUNCH();
}

void mlp_create(pkm_ctx* ctx, int d_in, int hidden, int rank, const float* params_host, pkm_mlp* net) {
    PKM_REQUIRE(hidden == HID, "hidden width must be 128");
    PKM_REQUIRE(d_in >= 1 && d_in <= 32, "d_in must be in [1, 32]");
    PKM_REQUIRE(rank >= 16 && rank <= 128 && rank % 16 == 0, "rank must be a multiple of 16 in [16, 128]");
    net->device = ctx->device;
    net->d_in = d_in;
    net->hidden = hidden;
    net->rank = rank;
    const MlpLayout L = layout(d_in, hidden, rank);
    net->nparams = L.total;
    const size_t bytes = sizeof(float) * L.total;
    net->p32.ensure(bytes);
    net->m32.ensure(bytes);
    net->v32.ensure(bytes);
    net->g32.ensure(bytes);
    net->wpack.ensure(sizeof(__bf16) * int64_t(512) * (8 + 32 + 4 * (rank / 16)));
    PKM_HIP(hipMemcpyAsync(net->p32.p, params_host, bytes, hipMemcpyHostToDevice, ctx->stream));
    PKM_HIP(hipMemsetAsync(net->m32.p, 0, bytes, ctx->stream));
    PKM_HIP(hipMemsetAsync(net->v32.p, 0, bytes, ctx->stream));
    repack(ctx, net);
    PKM_HIP(hipStreamSynchronize(ctx->stream));
}

static void forward(pkm_ctx* ctx, pkm_mlp* net, int64_t n, const double* xs, bool train,
                    double* U64) {
    const MlpLayout L = layout(net->d_in, net->hidden, net->rank);
    float* a1 = nullptr;
    float* a2 = nullptr;
    float* U32 = nullptr;
    if (train) {
        net->act[0].ensure(sizeof(float) * n * HID);
        net->act[1].ensure(sizeof(float) * n * HID);
        net->act[2].ensure(sizeof(float) * n * net->rank);
        a1 = net->act[0].as<float>();
        a2 = net->act[1].as<float>();
        U32 = net->act[2].as<float>();
    }
    const bf16x8* wp = net->wpack.as<bf16x8>();
    const bf16x8* w1p = wp;
    const bf16x8* w2p = wp + 8 * 64;
    const bf16x8* w3p = wp + 40 * 64;
    const unsigned grid = unsigned(cdiv(n, 64));
    const float* p = net->p32.as<float>();
    hipStream_t s = ctx->stream;
    switch (net->rank / 16) {
#define PKM_MLP_CASE(RT)                                                                       \
    case RT:                                                                                   \
        k_mlp_fwd<RT><<<grid, 256, 0, s>>>(xs, net->d_in, n, w1p, w2p, w3p, p, L.b1, L.b2, L.b3, \
                                            a1, a2, U32, U64);                                 \
        break;
        PKM_MLP_CASE(1) PKM_MLP_CASE(2) PKM_MLP_CASE(3) PKM_MLP_CASE(4)
        PKM_MLP_CASE(5) PKM_MLP_CASE(6) PKM_MLP_CASE(7) PKM_MLP_CASE(8)
#undef PKM_MLP_CASE
        default: fail(PKM_ERR_UNSUPPORTED, "rank");
    }
    PKM_CHECK_LAUNCH();
}

void mlp_forward(pkm_ctx* ctx, pkm_mlp* net, int64_t n, const double* xs, double* U) {
    forward(ctx, net, n, xs, false, U);
}

// Loss and gradient (into net->g32); returns L.
double mlp_loss_grad(pkm_ctx* ctx, pkm_mlp* net, int64_t n, const double* xs, int nz,
                     const double* Z, const double* KZ) {
    hipStream_t s = ctx->stream;
    const int r = net->rank, d = net->d_in;
    const MlpLayout L = layout(d, HID, r);
    forward(ctx, net, n, xs, true, nullptr);
    float* a1 = net->act[0].as<float>();
    float* a2 = net->act[1].as<float>();
    float* U = net->act[2].as<float>();
    // FP32 copies of Z, K Z and the inputs
    net->act[3].ensure(sizeof(float) * n * nz);
    net->act[4].ensure(sizeof(float) * n * nz);
    net->act[5].ensure(sizeof(float) * n * std::max(d, 1));
    float* Z32 = net->act[3].as<float>();
    float* KZ32 = net->act[4].as<float>();
    float* X32 = net->act[5].as<float>();
    k_f64_to_f32<<<cdiv(n * nz, 256), 256, 0, s>>>(n * nz, Z, Z32);
    k_f64_to_f32<<<cdiv(n * nz, 256), 256, 0, s>>>(n * nz, KZ, KZ32);
    k_f64_to_f32<<<cdiv(n * d, 256), 256, 0, s>>>(n * d, xs, X32);
    PKM_CHECK_LAUNCH();
    // small buffers: M (r x nz), S (nz x r)
    net->act[6].ensure(sizeof(float) * (int64_t(r) * nz * 2));
    float* M = net->act[6].as<float>();
    float* S = M + int64_t(r) * nz;
    // work: R (n x nz), dU (n x r), dh (n x 128), h (n x 128)
    net->act[7].ensure(sizeof(float) * n * (int64_t(nz) + r + 2 * HID));
    float* R = net->act[7].as<float>();
    float* dU = R + n * nz;
    float* dh = dU + n * r;
    float* h = dh + n * HID;
    // M = U^T Z; R = U M - K Z
    sgemm(ctx, net, true, false, r, nz, n, 1.f, U, r, Z32, nz, 0.f, M, nz);
    PKM_HIP(hipMemcpyAsync(R, KZ32, sizeof(float) * n * nz, hipMemcpyDeviceToDevice, s));
    sgemm(ctx, net, false, false, n, nz, r, 1.f, U, r, M, nz, -1.f, R, nz);
    const double c = sdot(ctx, net, n * nz, KZ32, KZ32);
    const double rr = sdot(ctx, net, n * nz, R, R);
    PKM_REQUIRE(c > 0.0, "K Z is zero");
    const double loss = rr / c;
    // S = R^T U; dU = (2/c) (R M^T + Z S)
    sgemm(ctx, net, true, false, nz, r, n, 1.f, R, nz, U, r, 0.f, S, r);
    const float sc = float(2.0 / c);
    sgemm(ctx, net, false, true, n, r, nz, sc, R, nz, M, nz, 0.f, dU, r);
    sgemm(ctx, net, false, false, n, r, nz, sc, Z32, nz, S, r, 1.f, dU, r);
    // layer 3: dW3 = h2^T dU, db3 = 1^T dU, dh2 = dU W3^T
    net->ones.ensure(sizeof(float) * n);
    float* ones = net->ones.as<float>();
    k_fill<<<cdiv(n, 256), 256, 0, s>>>(n, 1.f, ones);
    float* g = net->g32.as<float>();
    const float* P = net->p32.as<float>();
    k_gelu<<<cdiv(n * HID, 256), 256, 0, s>>>(n * HID, a2, h);
    PKM_CHECK_LAUNCH();
    sgemm(ctx, net, true, false, HID, r, n, 1.f, h, HID, dU, r, 0.f, g + L.W3, r);
    sgemm(ctx, net, true, false, 1, r, n, 1.f, ones, 1, dU, r, 0.f, g + L.b3, r);
    sgemm(ctx, net, false, true, n, HID, r, 1.f, dU, r, P + L.W3, r, 0.f, dh, HID);
    k_mul_gelu_grad<<<cdiv(n * HID, 256), 256, 0, s>>>(n * HID, a2, dh);   // dh = da2
    PKM_CHECK_LAUNCH();
    // layer 2: dW2 = h1^T da2, db2, dh1 = da2 W2^T (reuses dU's space as needed)
    k_gelu<<<cdiv(n * HID, 256), 256, 0, s>>>(n * HID, a1, h);
    PKM_CHECK_LAUNCH();
    sgemm(ctx, net, true, false, HID, HID, n, 1.f, h, HID, dh, HID, 0.f, g + L.W2, HID);
    sgemm(ctx, net, true, false, 1, HID, n, 1.f, ones, 1, dh, HID, 0.f, g + L.b2, HID);
    // dh1 into h (h1 no longer needed)
    sgemm(ctx, net, false, true, n, HID, HID, 1.f, dh, HID, P + L.W2, HID, 0.f, h, HID);
    k_mul_gelu_grad<<<cdiv(n * HID, 256), 256, 0, s>>>(n * HID, a1, h);   // h = da1
    PKM_CHECK_LAUNCH();
    // layer 1: dW1 = x^T da1, db1
    sgemm(ctx, net, true, false, d, HID, n, 1.f, X32, d, h, HID, 0.f, g + L.W1, HID);
    sgemm(ctx, net, true, false, 1, HID, n, 1.f, ones, 1, h, HID, 0.f, g + L.b1, HID);
    PKM_HIP(hipStreamSynchronize(s));
    return loss;
}

double mlp_train_step(pkm_ctx* ctx, pkm_mlp* net, int64_t n, const double* xs, int nz,
                      const double* Z, const double* KZ, double lr) {
    const double loss = mlp_loss_grad(ctx, net, n, xs, nz, Z, KZ);
    net->t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, float(net->t));
    const float c2 = 1.f - std::pow(b2, float(net->t));
    k_adam<<<cdiv(net->nparams, 256), 256, 0, ctx->stream>>>(
        net->nparams, net->p32.as<float>(), net->g32.as<float>(), net->m32.as<float>(),
        net->v32.as<float>(), float(lr), b1, b2, c1, c2, 1e-8f);
    PKM_CHECK_LAUNCH();
    repack(ctx, net);
    PKM_HIP(hipStreamSynchronize(ctx->stream));
    return loss;
}

// Checkpoint state: master weights, Adam first and second moments (each
// nparams FP32 in params layout, one after the other) and the Adam step count.
void mlp_state_get(pkm_ctx* ctx, const pkm_mlp* net, float* state, int64_t* t) {
    const size_t bytes = sizeof(float) * net->nparams;
    const pkm::DevBuf* parts[3] = {&net->p32, &net->m32, &net->v32};
    for (int i = 0; i < 3; ++i)
        PKM_HIP(hipMemcpyAsync(state + i * net->nparams, parts[i]->p, bytes,
                               hipMemcpyDeviceToHost, ctx->stream));
    PKM_HIP(hipStreamSynchronize(ctx->stream));
    *t = net->t;
}

void mlp_state_set(pkm_ctx* ctx, pkm_mlp* net, const float* state, int64_t t) {
    const size_t bytes = sizeof(float) * net->nparams;
    pkm::DevBuf* parts[3] = {&net->p32, &net->m32, &net->v32};
    for (int i = 0; i < 3; ++i)
        PKM_HIP(hipMemcpyAsync(parts[i]->p, state + i * net->nparams, bytes,
                               hipMemcpyHostToDevice, ctx->stream));
    net->t = t;
    repack(ctx, net);
    PKM_HIP(hipStreamSynchronize(ctx->stream));
}

int64_t mlp_nparams(const pkm_mlp* net) { return net->nparams; }
float* mlp_grad_ptr(pkm_mlp* net) { return net->g32.as<float>(); }
const float* mlp_param_ptr(const pkm_mlp* net) { return net->p32.as<float>(); }
int mlp_d_in(const pkm_mlp* net) { return net->d_in; }

void mlp_release(pkm_mlp* net) {
    for (pkm::DevBuf* b : {&net->p32, &net->m32, &net->v32, &net->g32, &net->wpack, &net->ones,
                           &net->scal, &net->split})
        b->release();
    for (auto& b : net->act) b.release();
}

}  // namespace pkm
