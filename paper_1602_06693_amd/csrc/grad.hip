// Gradient pass: Eq. (2) with the trace replaced by the Rademacher-probe
// estimate of Section 2.1, in log-parameter space.
//
// With column pairs (u_0, v_0) = (alpha, alpha), weight w_0 = 1/2, and
// (u_c, v_c) = (s_c, z_c), weight w_c = -1/(2N), every component is one
// bilinear form over all pairs (i, j):
//     G_ij = sum_c w_c u_c[i] v_c[j]
//     g_sigma2 = sum_ij K_ij G_ij
//     g_l_r    = sum_ij K_ij G_ij (xt_ir - xt_jr)^2,     xt = x / l
//     g_lambda = lambda sum_i G_ii
// One O(n^2) sweep regenerates K_ij from direct FP64 differences (never
// stored) and accumulates the d + 1 sums per row; blocks write partials that
// the host adds in a fixed order.

#include "pkm_internal.h"

#include <cmath>

namespace pkm {

template <int DP, int NC>
__global__ __launch_bounds__(256) void k_grad64(const double* __restrict__ xs, int d,
                                                const double* __restrict__ AS,
                                                const double* __restrict__ YZ, int ldc, int c0,
                                                int ncols, double w0, double wc, int64_t n,
                                                double sigma2, int64_t j_per_split,
                                                double* __restrict__ part) {
    constexpr int JT = 64;
    __shared__ double sx[JT][DP];
    __shared__ double sv[JT][NC];
    __shared__ double red[256];
    const int64_t i = blockIdx.x * int64_t(256) + threadIdx.x;
    const int64_t j0 = blockIdx.y * j_per_split;
    const int64_t j1 = min(n, j0 + j_per_split);
    double xi[DP], wu[NC];
#pragma unroll
    for (int r = 0; r < DP; ++r) xi[r] = (i < n && r < d) ? xs[i * d + r] : 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        int cc = c0 + c;
        double w = cc == 0 ? w0 : wc;
        wu[c] = (i < n && cc < ncols) ? w * AS[i * ldc + cc] : 0.0;
    }
    double acc[DP + 1];
#pragma unroll
    for (int r = 0; r <= DP; ++r) acc[r] = 0.0;
    const double ls2 = log(sigma2);
    for (int64_t jb = j0; jb < j1; jb += JT) {
        __syncthreads();
        for (int e = threadIdx.x; e < JT * DP; e += 256) {
            int jj = e / DP, r = e % DP;
            int64_t j = jb + jj;
            sx[jj][r] = (j < j1 && r < d) ? xs[j * d + r] : 0.0;
        }
        for (int e = threadIdx.x; e < JT * NC; e += 256) {
            int jj = e / NC, c = e % NC;
            int64_t j = jb + jj;
            sv[jj][c] = (j < j1 && c0 + c < ncols) ? YZ[j * ldc + c0 + c] : 0.0;
        }
        __syncthreads();
        const int jn = int(min<int64_t>(JT, j1 - jb));
        for (int jj = 0; jj < jn; ++jj) {
            double dd[DP];
            double s = 0.0;
#pragma unroll
            for (int r = 0; r < DP; ++r) {
                dd[r] = xi[r] - sx[jj][r];
                s = fma(dd[r], dd[r], s);
            }
            double g = 0.0;
#pragma unroll
            for (int c = 0; c < NC; ++c) g = fma(wu[c], sv[jj][c], g);
            const double t = exp(fma(-0.5, s, ls2)) * g;
            acc[0] += t;
#pragma unroll
            for (int r = 0; r < DP; ++r) acc[1 + r] = fma(t * dd[r], dd[r], acc[1 + r]);
        }
    }
    // block reduction of the d + 1 sums
    const int64_t blk = int64_t(blockIdx.y) * gridDim.x + blockIdx.x;
    for (int q = 0; q <= d; ++q) {
        double v = 0.0;
#pragma unroll
        for (int r = 0; r <= DP; ++r)
            if (r == q) v = acc[r];
        __syncthreads();
        red[threadIdx.x] = v;
        __syncthreads();
        for (int sft = 128; sft > 0; sft >>= 1) {
            if (threadIdx.x < sft) red[threadIdx.x] += red[threadIdx.x + sft];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[blk * (d + 1) + q] = red[0];
    }
}

// lambda-term: sum_i sum_c w_c u_c[i] v_c[i], per-block partials
__global__ void k_grad_lambda(const double* __restrict__ AS, const double* __restrict__ YZ,
                              int ldc, int ncols, double w0, double wc, int64_t n,
                              double* __restrict__ part) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int64_t i = blockIdx.x * int64_t(256) + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
        for (int c = 0; c < ncols; ++c) acc += (c == 0 ? w0 : wc) * AS[i * ldc + c] * YZ[i * ldc + c];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int sft = 128; sft > 0; sft >>= 1) {
        if (threadIdx.x < sft) red[threadIdx.x] += red[threadIdx.x + sft];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

template <int DP>
static void launch_grad_d(int nc, dim3 grid, hipStream_t s, const double* xs, int d,
                          const double* AS, const double* YZ, int ldc, int c0, int ncols,
                          double w0, double wc, int64_t n, double sigma2, int64_t jps,
                          double* part) {
#define PKM_G_CASE(NC)                                                                        \
    case NC:                                                                                  \
        k_grad64<DP, NC><<<grid, 256, 0, s>>>(xs, d, AS, YZ, ldc, c0, ncols, w0, wc, n, sigma2, \
                                               jps, part);                                    \
        break;
    switch (nc) {
        PKM_G_CASE(1) PKM_G_CASE(5) PKM_G_CASE(9) PKM_G_CASE(17) PKM_G_CASE(33)
        default: fail(PKM_ERR_UNSUPPORTED, "gradient pass: bad column chunk");
    }
#undef PKM_G_CASE
}

void grad_pass(pkm_ctx* ctx, const pkm_problem* prob, int N, const double* AS,
               const double* YZ, double* grad) {
    prepare(ctx, prob, true, false);
    hipStream_t s = ctx->stream;
    const int64_t n = prob->n;
    const int d = prob->d;
    const int ncols = 1 + N;
    const double w0 = 0.5, wc = N > 0 ? -0.5 / double(N) : 0.0;
    int64_t nrb = cdiv(n, 256);
    int jsplit = 1;
    while (jsplit < 64 && nrb * jsplit < 1024 && n / (jsplit * 2) >= 256) jsplit <<= 1;
    int64_t jps = round_up(cdiv(n, jsplit), 64);
    jsplit = int(cdiv(n, jps));
    dim3 grid((unsigned)(nrb), (unsigned)(jsplit));
    const int64_t nblk = nrb * jsplit;
    const int nlam = 256;
    std::vector<double> acc(d + 2, 0.0);
    ctx->grad.ensure(sizeof(double) * (nblk * (d + 1) + nlam));
    double* part = ctx->grad.as<double>();
    std::vector<double> hp(nblk * (d + 1));
    const double* xs = ctx->P().xs64.as<double>();
    for (int c0 = 0; c0 < ncols;) {
        int rem = ncols - c0;
        int nc = rem > 17 ? 33 : rem > 9 ? 17 : rem > 5 ? 9 : rem > 1 ? 5 : 1;
        if (d <= 4) launch_grad_d<4>(nc, grid, s, xs, d, AS, YZ, ncols, c0, ncols, w0, wc, n, prob->sigma2, jps, part);
        else if (d <= 8) launch_grad_d<8>(nc, grid, s, xs, d, AS, YZ, ncols, c0, ncols, w0, wc, n, prob->sigma2, jps, part);
        else if (d <= 16) launch_grad_d<16>(nc, grid, s, xs, d, AS, YZ, ncols, c0, ncols, w0, wc, n, prob->sigma2, jps, part);
        else if (d <= 32) launch_grad_d<32>(nc, grid, s, xs, d, AS, YZ, ncols, c0, ncols, w0, wc, n, prob->sigma2, jps, part);
        else fail(PKM_ERR_UNSUPPORTED, "gradient pass: d <= 32");
        PKM_CHECK_LAUNCH();
        PKM_HIP(hipMemcpyAsync(hp.data(), part, sizeof(double) * hp.size(), hipMemcpyDeviceToHost, s));
        PKM_HIP(hipStreamSynchronize(s));
        for (int64_t b = 0; b < nblk; ++b)
            for (int q = 0; q <= d; ++q) acc[q] += hp[b * (d + 1) + q];
        c0 += nc;
    }
    double* plam = part + nblk * (d + 1);
    k_grad_lambda<<<nlam, 256, 0, s>>>(AS, YZ, ncols, ncols, w0, wc, n, plam);
    PKM_CHECK_LAUNCH();
    std::vector<double> hl(nlam);
    PKM_HIP(hipMemcpyAsync(hl.data(), plam, sizeof(double) * nlam, hipMemcpyDeviceToHost, s));
    PKM_HIP(hipStreamSynchronize(s));
    double lamsum = 0.0;
    for (double v : hl) lamsum += v;
    for (int q = 0; q <= d; ++q) grad[q] = acc[q];
    grad[d + 1] = prob->lambda * lamsum;
}

}  // namespace pkm
