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

// ---------------------------------------------------------------------------
// Gradient pass on FP64 matrix cores.  With T = K o G (G_ij = sum_c w_c
// u_c[i] v_c[j]) and centred scaled inputs x~ = (x - mean) / l,
//     g_sigma2 = sum_i (T 1)_i,
//     g_l_r    = sum_ij T_ij (x~_ir - x~_jr)^2
//              = sum_i [x~_ir^2 (T 1)_i - 2 x~_ir (T x~_r)_i + (T x~_r^2)_i],
// so one sweep forms, per row i, R_i = T_i: [x~, x~^2] (2d columns) and the
// row sum (T 1)_i; every term is row-local (no column sums across
// work-groups).  Per 16-row j-tile and i-tile of a wave:
//   S^T = B_J A_I^T          S4 MFMAs (the product's augmented operands)
//   G^T = W_J U_I^T          CQ MFMAs over the 1 + N columns, 4 at a time
//   T = 2^S o G              exp2_tab on the vector ALUs, in the MFMA
//                            result layout: lane l holds (i = l % 16,
//                            j = 4 r + l / 16), r = 0..3 -- the A operands
//   R_I += T_IJ [x~_J, x~_J^2]   CT MFMA column tiles of 16
// and the row sum on the vector ALUs.  Each j-split writes its R and row
// sums as a partial plane; k_grad_combine forms the d + 1 per-row terms.
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <int S4, int CQ, int CT, int U>
__global__ __launch_bounds__(256) void k_grad_f64x(
    const double* __restrict__ jside, const double* __restrict__ iside,
    const double* __restrict__ AS, const double* __restrict__ YZ, int ldc, int c0, int ncols,
    double w0, double wc, const double* __restrict__ X, int d,
    const double* __restrict__ inv_l, const double* __restrict__ mean, int64_t n,
    int64_t ntiles, int64_t tiles_per_split, double* __restrict__ part, int ldp,
    int64_t split_stride) {
    __shared__ double tab[64];
    if (threadIdx.x < 64) tab[threadIdx.x] = exp2(double(threadIdx.x) / 64.0);
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = lane >> 4, cc = lane & 15;
    const int64_t itile0 = (int64_t(blockIdx.x) * 4 + w) * U;
    const int64_t t0 = int64_t(blockIdx.y) * tiles_per_split;
    const int64_t t1 = min(ntiles, t0 + tiles_per_split);
    double ai[U][S4], ui[U][CQ];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int q = 0; q < S4; ++q) ai[u][q] = iside[((itile0 + u) * 64 + lane) * S4 + q];
        // B operand of the weight MFMAs: lane l holds U[i = 16 tile + l % 16][c = 4 q + l / 16]
        const int64_t i = (itile0 + u) * 16 + cc;
#pragma unroll
        for (int q = 0; q < CQ; ++q) {
            const int c = c0 + 4 * q + g;
            ui[u][q] = (i < n && c < ncols) ? (c == 0 ? w0 : wc) * AS[i * ldc + c] : 0.0;
        }
    }
    f64x4 acc[U][CT];
    double rs[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        rs[u] = 0.0;
#pragma unroll
        for (int q = 0; q < CT; ++q) acc[u][q] = f64x4{0.0, 0.0, 0.0, 0.0};
    }
    for (int64_t t = t0; t < t1; ++t) {
        double bj[S4], wj[CQ], xb[CT][4];
#pragma unroll
        for (int q = 0; q < S4; ++q) bj[q] = jside[(t * 64 + lane) * S4 + q];
        {   // A operand of the weight MFMAs: W[j = 16 t + l % 16][c = 4 q + l / 16]
            const int64_t j = t * 16 + cc;
#pragma unroll
            for (int q = 0; q < CQ; ++q) {
                const int c = c0 + 4 * q + g;
                wj[q] = (j < n && c < ncols) ? YZ[j * ldc + c] : 0.0;
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {   // B operands: [x~, x~^2][j = 16 t + 4 r + l / 16][col]
            const int64_t j = t * 16 + 4 * r + g;
#pragma unroll
            for (int q = 0; q < CT; ++q) {
                const int col = 16 * q + cc;
                const int rr = col < d ? col : col - d;
                double v = 0.0;
                if (j < n && col < 2 * d) {
                    const double xt = (X[j * d + rr] - mean[rr]) * inv_l[rr];
                    v = col < d ? xt : xt * xt;
                }
                xb[q][r] = v;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            f64x4 st = {0.0, 0.0, 0.0, 0.0}, gt = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int q = 0; q < S4; ++q)
                st = __builtin_amdgcn_mfma_f64_16x16x4f64(bj[q], ai[u][q], st, 0, 0, 0);
#pragma unroll
            for (int q = 0; q < CQ; ++q)
                gt = __builtin_amdgcn_mfma_f64_16x16x4f64(wj[q], ui[u][q], gt, 0, 0, 0);
            double tv[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                tv[r] = exp2_tab(st[r], tab) * gt[r];
                rs[u] += tv[r];
            }
#pragma unroll
            for (int q = 0; q < CT; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    acc[u][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(tv[r], xb[q][r], acc[u][q], 0, 0, 0);
        }
    }
    double* po = part + blockIdx.y * split_stride;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        // row sums: lane l holds row l % 16's sum over the j with j % 4 = l / 16
        double v = rs[u];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        const int64_t i = (itile0 + u) * 16 + cc;
        if (g == 0 && i < n) po[i * ldp] = v;
        // FP64 16x16x4 results: lane l holds rows l / 16 + 4 r, column l % 16
#pragma unroll
        for (int q = 0; q < CT; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t ir = (itile0 + u) * 16 + g + 4 * r;
                const int col = 16 * q + cc;
                if (ir < n && col < 2 * d) po[ir * ldp + 1 + col] = acc[u][q][r];
            }
    }
}

// Per row i: the split planes summed, then (T 1)_i and, for each r,
// x~_ir^2 (T 1)_i - 2 x~_ir (T x~_r)_i + (T x~_r^2)_i; per-block sums of the
// d + 1 terms (fixed order), added on the host in block order.
__global__ __launch_bounds__(256) void k_grad_combine(const double* __restrict__ part, int nsplit,
                                                      int64_t split_stride, int ldp,
                                                      const double* __restrict__ X, int d,
                                                      const double* __restrict__ inv_l,
                                                      const double* __restrict__ mean, int64_t n,
                                                      double* __restrict__ out) {
    __shared__ double red[256];
    const int64_t i = blockIdx.x * int64_t(256) + threadIdx.x;
    double rsum = 0.0;
    if (i < n)
        for (int s = 0; s < nsplit; ++s) rsum += part[s * split_stride + i * ldp];
    for (int q = 0; q <= d; ++q) {
        double v = 0.0;
        if (i < n) {
            if (q == 0) {
                v = rsum;
            } else {
                const int r = q - 1;
                double t1 = 0.0, t2 = 0.0;
                for (int s = 0; s < nsplit; ++s) {
                    t1 += part[s * split_stride + i * ldp + 1 + r];
                    t2 += part[s * split_stride + i * ldp + 1 + d + r];
                }
                const double xt = (X[i * d + r] - mean[r]) * inv_l[r];
                v = fma(xt * xt, rsum, fma(-2.0 * xt, t1, t2));
            }
        }
        __syncthreads();
        red[threadIdx.x] = v;
        __syncthreads();
        for (int sft = 128; sft > 0; sft >>= 1) {
            if (threadIdx.x < sft) red[threadIdx.x] += red[threadIdx.x + sft];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[blockIdx.x * int64_t(d + 1) + q] = red[0];
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

// i-tiles per wave of the matrix-core gradient: four while the operands fit
// two waves per SIMD, else two
constexpr int grad_tiles(int s4, int cq) { return (s4 <= 6 && cq <= 5) ? 4 : 2; }

template <int S4, int CT>
static void launch_gradx_cq(int CQ, dim3 grid, hipStream_t s, const double* js,
                            const double* is, const double* AS, const double* YZ, int ldc,
                            int c0, int ncols, double w0, double wc, const double* X, int d,
                            const double* inv_l, const double* mean, int64_t n, int64_t ntiles,
                            int64_t tps, double* part, int ldp, int64_t sstride) {
#define PKM_GX_CASE(cq)                                                                        \
    case cq:                                                                                   \
        k_grad_f64x<S4, cq, CT, grad_tiles(S4, cq)><<<grid, 256, 0, s>>>(                      \
            js, is, AS, YZ, ldc, c0, ncols, w0, wc, X, d, inv_l, mean, n, ntiles, tps, part,   \
            ldp, sstride);                                                                     \
        return;
    switch (CQ) {
        PKM_GX_CASE(1) PKM_GX_CASE(3) PKM_GX_CASE(5) PKM_GX_CASE(9)
        default: fail(PKM_ERR_UNSUPPORTED, "gradient pass: bad column chunk");
    }
#undef PKM_GX_CASE
}

static void launch_gradx(int S4, int CT, int CQ, dim3 grid, hipStream_t s, const double* js,
                         const double* is, const double* AS, const double* YZ, int ldc, int c0,
                         int ncols, double w0, double wc, const double* X, int d,
                         const double* inv_l, const double* mean, int64_t n, int64_t ntiles,
                         int64_t tps, double* part, int ldp, int64_t sstride) {
#define PKM_GX(s4, ct)                                                                         \
    if (S4 == s4 && CT == ct) {                                                                \
        launch_gradx_cq<s4, ct>(CQ, grid, s, js, is, AS, YZ, ldc, c0, ncols, w0, wc, X, d,     \
                                inv_l, mean, n, ntiles, tps, part, ldp, sstride);              \
        return;                                                                                \
    }
    // (augmented slices, column tiles of [x~, x~^2]) for d = 1 .. 32
    PKM_GX(1, 1) PKM_GX(2, 1) PKM_GX(3, 1) PKM_GX(3, 2) PKM_GX(4, 2) PKM_GX(5, 2)
    PKM_GX(5, 3) PKM_GX(6, 3) PKM_GX(7, 3) PKM_GX(7, 4) PKM_GX(8, 4) PKM_GX(9, 4)
#undef PKM_GX
    fail(PKM_ERR_UNSUPPORTED, "gradient pass: unsupported dimension");
}

// Matrix-core gradient pass: column chunks of up to 36 (the weight MFMAs'
// contraction), each one sweep plus the per-row combination; the chunks'
// per-block sums and the lambda term are added on the host in fixed order.
static void grad_pass_mfma(pkm_ctx* ctx, const pkm_problem* prob, int N, const double* AS,
                           const double* YZ, double* grad) {
    Prepared& P = ctx->P();
    hipStream_t s = ctx->stream;
    const int64_t n = prob->n;
    const int d = prob->d;
    const int ncols = 1 + N;
    const double w0 = 0.5, wc = N > 0 ? -0.5 / double(N) : 0.0;
    const int S4 = P.d4 / 4, CT = (d + 7) / 8;
    const int ldp = 2 * d + 1;
    const int64_t ntiles = P.n_pad / 16;
    const double* inv_l = ctx->scal.as<double>();
    const double* mean = inv_l + 64;
    const int64_t ncomb = cdiv(n, 256);
    const int nlam = 256;
    std::vector<double> acc(d + 1, 0.0);
    for (int c0 = 0; c0 < ncols;) {
        const int rem = ncols - c0;
        const int CQ = rem <= 4 ? 1 : rem <= 12 ? 3 : rem <= 20 ? 5 : 9;
        const int U = grad_tiles(S4, CQ);
        const int64_t nrb = cdiv(n, 64 * U);
        int jsplit = 1;
        while (jsplit < 64 && nrb * jsplit < 2048 && n / (jsplit * 2) >= 256) jsplit <<= 1;
        const int64_t jps = round_up(cdiv(n, jsplit), 64);
        jsplit = int(cdiv(n, jps));
        const int64_t sstride = n * ldp;
        ctx->grad.ensure(sizeof(double) * (jsplit * sstride + ncomb * (d + 1) + nlam));
        double* part = ctx->grad.as<double>();
        double* comb = part + jsplit * sstride;
        launch_gradx(S4, CT, CQ, dim3((unsigned)nrb, (unsigned)jsplit), s, P.jside64.as<double>(),
                     P.iside64.as<double>(), AS, YZ, ncols, c0, ncols, w0, wc, prob->X, d, inv_l,
                     mean, n, ntiles, jps / 16, part, ldp, sstride);
        PKM_CHECK_LAUNCH();
        k_grad_combine<<<(unsigned)ncomb, 256, 0, s>>>(part, jsplit, sstride, ldp, prob->X, d,
                                                        inv_l, mean, n, comb);
        PKM_CHECK_LAUNCH();
        std::vector<double> hc(ncomb * (d + 1));
        PKM_HIP(hipMemcpyAsync(hc.data(), comb, sizeof(double) * hc.size(), hipMemcpyDeviceToHost, s));
        PKM_HIP(hipStreamSynchronize(s));
        for (int64_t b = 0; b < ncomb; ++b)
            for (int q = 0; q <= d; ++q) acc[q] += hc[b * (d + 1) + q];
        c0 += 4 * CQ;
    }
    double* plam = ctx->grad.as<double>();   // the sweeps' partials are no longer needed
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

void grad_pass(pkm_ctx* ctx, const pkm_problem* prob, int N, const double* AS,
               const double* YZ, double* grad) {
    prepare(ctx, prob, true, false);
    if (ctx->P().d4 <= kAug64MaxD4 && prob->d <= 32) {
        grad_pass_mfma(ctx, prob, N, AS, YZ, grad);
        return;
    }
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
