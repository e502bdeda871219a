// FP64 dense routines for preconditioner setup and apply: general matrix
// product (tiled through LDS, split over the reduction dimension when the
// output is small), blocked right-looking Cholesky, and the triangular solve
// B <- B L^{-T}.  All row-major.

#include "pkm_internal.h"

#include <algorithm>

namespace pkm {

constexpr int GT = 64;   // output tile edge
constexpr int GK = 16;   // reduction step

// C_part[z] = alpha op(A) op(B) over k-range z (or C = alpha op(A) op(B) + beta C
// when nsplit == 1).  256 threads, each 4x4 outputs.
template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_dgemm(int64_t M, int64_t N, int64_t K, double alpha,
                                               const double* __restrict__ A, int64_t lda,
                                               const double* __restrict__ B, int64_t ldb,
                                               double beta, double* __restrict__ C, int64_t ldc,
                                               int64_t kchunk, double* __restrict__ part) {
    __shared__ double sa[GK][GT + 1];
    __shared__ double sb[GK][GT + 1];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int64_t i0 = int64_t(blockIdx.y) * GT, j0 = int64_t(blockIdx.x) * GT;
    const int64_t kbeg = int64_t(blockIdx.z) * kchunk;
    const int64_t kend = min(K, kbeg + kchunk);
    double acc[4][4] = {};
    for (int64_t k0 = kbeg; k0 < kend; k0 += GK) {
        for (int e = threadIdx.x; e < GK * GT; e += 256) {
            int kk, ii;
            if (TA) { ii = e % GT; kk = e / GT; } else { kk = e % GK; ii = e / GK; }
            int64_t gi = i0 + ii, gk = k0 + kk;
            double v = 0.0;
            if (gi < M && gk < kend) v = TA ? A[gk * lda + gi] : A[gi * lda + gk];
            sa[kk][ii] = v;
        }
        for (int e = threadIdx.x; e < GK * GT; e += 256) {
            int kk, jj;
            if (TB) { kk = e % GK; jj = e / GK; } else { jj = e % GT; kk = e / GT; }
            int64_t gj = j0 + jj, gk = k0 + kk;
            double v = 0.0;
            if (gj < N && gk < kend) v = TB ? B[gj * ldb + gk] : B[gk * ldb + gj];
            sb[kk][jj] = v;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GK; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                a[q] = sa[kk][ty + 16 * q];
                b[q] = sb[kk][tx + 16 * q];
            }
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[p][q] = fma(a[p], b[q], acc[p][q]);
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
            if (part) {
                part[int64_t(blockIdx.z) * M * N + gi * N + gj] = acc[p][q];
            } else {
                double c = alpha * acc[p][q];
                if (beta != 0.0) c += beta * C[gi * ldc + gj];
                C[gi * ldc + gj] = c;
            }
        }
    }
}

__global__ void k_dgemm_reduce(int64_t M, int64_t N, int nsplit, const double* __restrict__ part,
                               double alpha, double beta, double* __restrict__ C, int64_t ldc) {
    int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= M * N) return;
    int64_t i = e / N, j = e - i * N;
    double s = 0.0;
    for (int z = 0; z < nsplit; ++z) s += part[z * M * N + e];
    double c = alpha * s;
    if (beta != 0.0) c += beta * C[i * ldc + j];
    C[i * ldc + j] = c;
}

void dgemm(pkm_ctx* ctx, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
           const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
           int64_t ldc) {
    hipStream_t s = ctx->stream;
    if (M <= 0 || N <= 0) return;
    if (K <= 0) {
        // C = beta C
        int64_t tot = M * N;
        k_dgemm_reduce<<<cdiv(tot, 256), 256, 0, s>>>(M, N, 0, nullptr, 0.0, beta, C, ldc);
        PKM_CHECK_LAUNCH();
        return;
    }
    int64_t tiles = cdiv(M, GT) * cdiv(N, GT);
    int nsplit = 1;
    // small outputs with a long reduction: split the reduction dimension
    while (tiles * nsplit < 512 && K / (nsplit * 2) >= 256 && nsplit < 256) nsplit *= 2;
    int64_t kchunk = round_up(cdiv(K, nsplit), GK);
    nsplit = int(cdiv(K, kchunk));
    double* part = nullptr;
    if (nsplit > 1) {
        ctx->ws_split.ensure(sizeof(double) * M * N * nsplit);
        part = ctx->ws_split.as<double>();
    }
    dim3 grid(unsigned(cdiv(N, GT)), unsigned(cdiv(M, GT)), unsigned(nsplit));
    PKM_REQUIRE(cdiv(M, GT) <= 65535, "dgemm: M too large for one launch");
    if (!ta && !tb) k_dgemm<false, false><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, part);
    else if (ta && !tb) k_dgemm<true, false><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, part);
    else if (!ta && tb) k_dgemm<false, true><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, part);
    else k_dgemm<true, true><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, part);
    PKM_CHECK_LAUNCH();
    if (nsplit > 1) {
        k_dgemm_reduce<<<cdiv(M * N, 256), 256, 0, s>>>(M, N, nsplit, part, alpha, beta, C, ldc);
        PKM_CHECK_LAUNCH();
    }
}

void dgemm_large(pkm_ctx* ctx, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
                 const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                 double* C, int64_t ldc) {
    // row-chunk very tall outputs to respect the grid limit
    const int64_t maxM = int64_t(65535) * GT;
    for (int64_t r0 = 0; r0 < M; r0 += maxM) {
        int64_t mm = std::min(maxM, M - r0);
        const double* Ar = ta ? A + r0 : A + r0 * lda;
        dgemm(ctx, ta, tb, mm, N, K, alpha, Ar, lda, B, ldb, beta, C + r0 * ldc, ldc);
    }
}

// ---------------------------------------------------------------------------
// Cholesky
// ---------------------------------------------------------------------------
constexpr int NB = 64;

// Factor the nb x nb diagonal block in place (lower) and write its inverse
// to W (nb x NB, row-major).  A non-positive pivot records its global index
// + 1 in *info (first failure wins) and is replaced by 1 to keep going.
__global__ __launch_bounds__(256) void k_potrf_diag(double* __restrict__ A, int64_t lda, int nb,
                                                    int64_t gofs, double* __restrict__ W,
                                                    int* __restrict__ info) {
    __shared__ double a[NB][NB + 1];
    __shared__ double w[NB][NB + 1];
    for (int e = threadIdx.x; e < NB * NB; e += 256) {
        int i = e / NB, j = e % NB;
        a[i][j] = (i < nb && j < nb) ? A[int64_t(i) * lda + j] : (i == j ? 1.0 : 0.0);
    }
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
        if (threadIdx.x == 0) {
            double v = a[j][j];
            if (!(v > 0.0) || !isfinite(v)) {
                atomicCAS(info, 0, int(gofs + j + 1));
                v = 1.0;
            }
            a[j][j] = sqrt(v);
        }
        __syncthreads();
        const double piv = a[j][j];
        for (int i = j + 1 + threadIdx.x; i < nb; i += 256) a[i][j] /= piv;
        __syncthreads();
        for (int e = threadIdx.x; e < (nb - j - 1) * (nb - j - 1); e += 256) {
            int i = j + 1 + e / (nb - j - 1), c = j + 1 + e % (nb - j - 1);
            if (c <= i) a[i][c] -= a[i][j] * a[c][j];
        }
        __syncthreads();
    }
    // inverse of the lower factor, one column per thread
    if (threadIdx.x < NB) {
        const int c = threadIdx.x;
        for (int i = 0; i < NB; ++i) {
            double v;
            if (i < c) v = 0.0;
            else {
                double sacc = (i == c) ? 1.0 : 0.0;
                for (int p = c; p < i; ++p) sacc -= a[i][p] * w[p][c];
                v = sacc / a[i][i];
            }
            w[i][c] = v;
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < NB * NB; e += 256) {
        int i = e / NB, j = e % NB;
        if (i < nb && j < nb) A[int64_t(i) * lda + j] = (j <= i) ? a[i][j] : 0.0;
        W[int64_t(i) * NB + j] = (i < nb && j < nb) ? w[i][j] : 0.0;
    }
}

__global__ void k_copy2d(int64_t rows, int64_t cols, const double* __restrict__ src, int64_t lds,
                         double* __restrict__ dst, int64_t ldd) {
    int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= rows * cols) return;
    int64_t i = e / cols, j = e - i * cols;
    dst[i * ldd + j] = src[i * lds + j];
}

__global__ void k_zero_upper(int64_t m, double* __restrict__ A, int64_t lda) {
    int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= m * m) return;
    int64_t i = e / m, j = e - i * m;
    if (j > i) A[i * lda + j] = 0.0;
}

void dpotrf_lower(pkm_ctx* ctx, int64_t m, double* A, int64_t lda, double* winv, int* dev_info) {
    hipStream_t s = ctx->stream;
    PKM_HIP(hipMemsetAsync(dev_info, 0, sizeof(int), s));
    for (int64_t k0 = 0; k0 < m; k0 += NB) {
        int nb = int(std::min<int64_t>(NB, m - k0));
        double* Akk = A + k0 * lda + k0;
        double* Wk = winv + k0 * NB;
        k_potrf_diag<<<1, 256, 0, s>>>(Akk, lda, nb, k0, Wk, dev_info);
        PKM_CHECK_LAUNCH();
        int64_t rest = m - k0 - nb;
        if (rest <= 0) break;
        // panel <- panel L_kk^{-T}
        ctx->ws_tmp.ensure(sizeof(double) * rest * NB);
        double* T = ctx->ws_tmp.as<double>();
        double* Pn = A + (k0 + nb) * lda + k0;
        k_copy2d<<<cdiv(rest * nb, 256), 256, 0, s>>>(rest, nb, Pn, lda, T, nb);
        PKM_CHECK_LAUNCH();
        dgemm(ctx, false, true, rest, nb, nb, 1.0, T, nb, Wk, NB, 0.0, Pn, lda);
        // trailing <- trailing - panel panel^T
        double* Tr = A + (k0 + nb) * lda + (k0 + nb);
        dgemm(ctx, false, true, rest, rest, nb, -1.0, Pn, lda, Pn, lda, 1.0, Tr, lda);
    }
    k_zero_upper<<<cdiv(m * m, 256), 256, 0, s>>>(m, A, lda);
    PKM_CHECK_LAUNCH();
}

// B (n x m) <- B L^{-T}; winv holds the inverses of L's 64x64 diagonal blocks.
void dtrsm_right_lt(pkm_ctx* ctx, int64_t n, int64_t m, const double* L, int64_t ldl,
                    const double* winv, double* B, int64_t ldb) {
    hipStream_t s = ctx->stream;
    for (int64_t k0 = 0; k0 < m; k0 += NB) {
        int nb = int(std::min<int64_t>(NB, m - k0));
        double* Bk = B + k0;
        if (k0 > 0)   // Bk -= B[:, :k0] L[k0:k0+nb, :k0]^T
            dgemm_large(ctx, false, true, n, nb, k0, -1.0, B, ldb, L + k0 * ldl, ldl, 1.0, Bk, ldb);
        ctx->ws_tmp.ensure(sizeof(double) * n * NB);
        double* T = ctx->ws_tmp.as<double>();
        k_copy2d<<<cdiv(n * nb, 256), 256, 0, s>>>(n, nb, Bk, ldb, T, nb);
        PKM_CHECK_LAUNCH();
        dgemm_large(ctx, false, true, n, nb, nb, 1.0, T, nb, winv + k0 * NB, NB, 0.0, Bk, ldb);
    }
}

}  // namespace pkm
