// Input preparation (once per theta) and FP64 kernel blocks for setup.
//
// The ARD-RBF kernel of Eq. (1) depends on the inputs only through the
// scaled differences (x_ir - x_jr) / l_r, so every product works on scaled
// rows.  Two forms are prepared:
//
//  * FP64 rows xs_i = x_i / l (direct differences, used by the setup
//    kernels and the FP64 product for large d).
//  * FP32 operands of one augmented contraction whose value is the base-2
//    exponent of the kernel entry.  With xh_i = (x_i - mean) / l * c,
//    c = sqrt(log2(e) / 2), and
//        a_i = [2 xh_i, log2 sigma2 - |xh_i|^2, 1, 0 ...]
//        b_j = [  xh_j,                     1, -|xh_j|^2, 0 ...]
//    a_i . b_j = log2 sigma2 - |xh_i - xh_j|^2, hence
//        k(x_i, x_j) = 2^(a_i . b_j).
//    Centring (the kernel is translation invariant) keeps |xh|^2 small,
//    which bounds the cancellation error of the expansion.  Padded j rows
//    get a huge negative exponent so their entries vanish.
//
// The same operands are prepared in FP32 and in FP64 (the FP64 product's
// contraction has an absolute exponent error of a few units of 2^-53 times
// |xh|^2).  Both are stored in the lane order of the 16x16x4 MFMA (the FP32
// and FP64 forms share it): element (tile t, lane l, group s) =
// row 16 t + l % 16, slot 4 s + l / 16.

#include "pkm_internal.h"

#include <cmath>
#include <cstring>

namespace pkm {

void validate_problem(const pkm_problem* p) {
    PKM_REQUIRE(p != nullptr, "problem is NULL");
    PKM_REQUIRE(p->n >= 1, "n must be >= 1");
    PKM_REQUIRE(p->n <= (int64_t(1) << 31) - 4096, "n too large");
    PKM_REQUIRE(p->d >= 1 && p->d <= 64, "d must be in [1, 64]");
    PKM_REQUIRE(p->reserved == 0, "reserved field must be 0");
    PKM_REQUIRE(p->X != nullptr, "X is NULL");
    PKM_REQUIRE(p->lengthscales != nullptr, "lengthscales is NULL");
    PKM_REQUIRE(std::isfinite(p->sigma2) && p->sigma2 > 0, "sigma2 must be > 0");
    PKM_REQUIRE(std::isfinite(p->lambda) && p->lambda > 0, "lambda must be > 0");
    for (int r = 0; r < p->d; ++r)
        PKM_REQUIRE(std::isfinite(p->lengthscales[r]) && p->lengthscales[r] > 0,
                    "every lengthscale must be > 0");
    PKM_REQUIRE((reinterpret_cast<uintptr_t>(p->X) & 7) == 0, "X must be 8-byte aligned");
}

// Column means of X (n x d), one block per dimension, fixed summation order.
__global__ void k_colmean(const double* __restrict__ X, int64_t n, int d,
                          double* __restrict__ mean) {
    __shared__ double sh[256];
    int r = blockIdx.x;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) acc += X[i * d + r];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) mean[r] = sh[0] / double(n);
}

struct ScaleArgs {
    double inv_l[64];
    double mean[64];
};

// FP64 scaled rows; padded rows are zero.
__global__ void k_scale64(const double* __restrict__ X, int64_t n, int64_t n_pad, int d,
                          const double* __restrict__ inv_l, double* __restrict__ xs) {
    int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= n_pad * d) return;
    int64_t i = e / d;
    int r = int(e - i * d);
    xs[e] = i < n ? X[i * d + r] * inv_l[r] : 0.0;
}

// Augmented operands in MFMA lane order (see file header), FP32 or FP64.
template <class T>
__global__ void k_aug(const double* __restrict__ X, int64_t n, int64_t n_pad, int d,
                      int d4, const double* __restrict__ inv_l,
                      const double* __restrict__ mean, double log2s2,
                      T* __restrict__ jside, T* __restrict__ iside) {
    int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i >= n_pad) return;
    const double c = sqrt(0.5 * 1.4426950408889634);  // sqrt(log2(e) / 2)
    int64_t t = i >> 4;
    int row = int(i & 15);
    int groups = d4 >> 2;
    auto put = [&](T* base, int slot, double v) {
        int s = slot >> 2, kk = slot & 3;
        int lane = row + 16 * kk;
        base[(t * 64 + lane) * groups + s] = T(v);
    };
    if (i < n) {
        double nrm = 0.0;
        for (int r = 0; r < d; ++r) {
            // the stored (rounded) coordinate enters the norm, so the
            // expansion is exact for the stored values up to its own rounding
            T xh = T((X[i * d + r] - mean[r]) * inv_l[r] * c);
            nrm += double(xh) * double(xh);
            put(iside, r, 2.0 * double(xh));
            put(jside, r, double(xh));
        }
        put(iside, d, log2s2 - nrm);
        put(iside, d + 1, 1.0);
        put(jside, d, 1.0);
        put(jside, d + 1, -nrm);
    } else {
        for (int r = 0; r < d; ++r) {
            put(iside, r, 0.0);
            put(jside, r, 0.0);
        }
        put(iside, d, log2s2);
        put(iside, d + 1, 1.0);
        put(jside, d, 1.0);
        put(jside, d + 1, -1.0e30);
    }
    for (int sl = d + 2; sl < d4; ++sl) {
        put(iside, sl, 0.0);
        put(jside, sl, 0.0);
    }
}

void prepare(pkm_ctx* ctx, const pkm_problem* prob, bool need64, bool need32) {
    // Inputs are prepared afresh on every entry point (O(n d) work): the
    // caller may have changed X in place since the last call.
    Prepared& P = ctx->P();
    std::vector<double> ls(prob->lengthscales, prob->lengthscales + prob->d);
    P.valid64 = P.valid32 = P.validb = P.validi8 = false;
    P.X = prob->X;
    P.n = prob->n;
    P.d = prob->d;
    P.sigma2 = prob->sigma2;
    P.lambda = prob->lambda;
    P.ls = ls;
    P.n_pad = round_up(prob->n, 256);

    const int d = P.d;
    const int64_t n = P.n, n_pad = P.n_pad;
    hipStream_t s = ctx->stream;
    // small constant arrays: 1/l and the column means
    ctx->scal.ensure(4096);
    double* inv_l = ctx->scal.as<double>();
    double* mean = inv_l + 64;
    double hbuf[64];
    for (int r = 0; r < d; ++r) hbuf[r] = 1.0 / ls[r];
    PKM_HIP(hipMemcpyAsync(inv_l, hbuf, sizeof(double) * d, hipMemcpyHostToDevice, s));
    k_colmean<<<d, 256, 0, s>>>(prob->X, n, d, mean);
    PKM_CHECK_LAUNCH();
    P.d4 = int(round_up(d + 2, 4));
    if (need64 && !P.valid64) {
        P.xs64.ensure(sizeof(double) * n_pad * d);
        int64_t tot = n_pad * d;
        k_scale64<<<cdiv(tot, 256), 256, 0, s>>>(prob->X, n, n_pad, d, inv_l,
                                                  P.xs64.as<double>());
        PKM_CHECK_LAUNCH();
        if (P.d4 <= kAug64MaxD4) {
            P.jside64.ensure(sizeof(double) * n_pad * P.d4);
            P.iside64.ensure(sizeof(double) * n_pad * P.d4);
            k_aug<double><<<cdiv(n_pad, 256), 256, 0, s>>>(prob->X, n, n_pad, d, P.d4, inv_l, mean,
                                                           std::log2(P.sigma2),
                                                           P.jside64.as<double>(),
                                                           P.iside64.as<double>());
            PKM_CHECK_LAUNCH();
        }
        P.valid64 = true;
    }
    if (need32 && !P.valid32) {
        P.jside.ensure(sizeof(float) * n_pad * P.d4);
        P.iside.ensure(sizeof(float) * n_pad * P.d4);
        k_aug<float><<<cdiv(n_pad, 256), 256, 0, s>>>(prob->X, n, n_pad, d, P.d4, inv_l, mean,
                                                      std::log2(P.sigma2), P.jside.as<float>(),
                                                      P.iside.as<float>());
        PKM_CHECK_LAUNCH();
        P.valid32 = true;
    }
    // inv_l / mean live in ctx->scal; keep them ordered before later reuse
    PKM_HIP(hipStreamSynchronize(s));
}

// FP64 augmented operands of a cross product K(Xa, Xb): b_j from Xb (written
// to jside, nb rounded up to 256 rows), a_i from Xa (to iside, na rounded up
// to 256); both centred by Xb's column mean (the kernel is translation
// invariant, one shared centre keeps a_i . b_j = log2 sigma2 - |xh_i - xh_j|^2).
// scratch holds the unused side of each call (max of the two padded sizes).
void prepare_cross64(pkm_ctx* ctx, const pkm_problem* prob, const double* Xa, int64_t na,
                     const double* Xb, int64_t nb, double* jside, double* iside,
                     double* scratch) {
    hipStream_t s = ctx->stream;
    const int d = prob->d;
    const int d4 = int(round_up(d + 2, 4));
    ctx->scal.ensure(4096);
    double* inv_l = ctx->scal.as<double>();
    double* mean = inv_l + 64;
    double hbuf[64];
    for (int r = 0; r < d; ++r) hbuf[r] = 1.0 / prob->lengthscales[r];
    PKM_HIP(hipMemcpyAsync(inv_l, hbuf, sizeof(double) * d, hipMemcpyHostToDevice, s));
    k_colmean<<<d, 256, 0, s>>>(Xb, nb, d, mean);
    PKM_CHECK_LAUNCH();
    const double l2s = std::log2(prob->sigma2);
    const int64_t nbp = round_up(nb, 256), nap = round_up(na, 256);
    k_aug<double><<<cdiv(nbp, 256), 256, 0, s>>>(Xb, nb, nbp, d, d4, inv_l, mean, l2s, jside,
                                                  scratch);
    PKM_CHECK_LAUNCH();
    k_aug<double><<<cdiv(nap, 256), 256, 0, s>>>(Xa, na, nap, d, d4, inv_l, mean, l2s, scratch,
                                                  iside);
    PKM_CHECK_LAUNCH();
    PKM_HIP(hipStreamSynchronize(s));   // hbuf is host stack memory
}

// Out[i][j] = sigma2 exp(-1/2 |xa_ia(i) - xb_ib(j)|^2) with optional row
// gathers ia / ib (NULL: identity).  One thread per output entry.
__global__ void k_rbf_cross64(const double* __restrict__ xa, const int32_t* __restrict__ ia,
                              int64_t p, const double* __restrict__ xb,
                              const int32_t* __restrict__ ib, int64_t q, int d,
                              double sigma2, double* __restrict__ out, int64_t ldo) {
    int64_t j = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    int64_t i = blockIdx.y;
    if (j >= q || i >= p) return;
    const double* a = xa + (ia ? int64_t(ia[i]) : i) * d;
    const double* b = xb + (ib ? int64_t(ib[j]) : j) * d;
    double s = 0.0;
    for (int r = 0; r < d; ++r) {
        double t = a[r] - b[r];
        s = fma(t, t, s);
    }
    out[i * ldo + j] = sigma2 * exp(-0.5 * s);
}

void rbf_cross64(hipStream_t s, const double* xa, const int32_t* ia, int64_t p,
                 const double* xb, const int32_t* ib, int64_t q, int d, double sigma2,
                 double* out, int64_t ldo) {
    if (p == 0 || q == 0) return;
    PKM_REQUIRE(p <= 2147483647, "rbf_cross64: too many rows");
    int64_t rows_left = p;
    int64_t row0 = 0;
    while (rows_left > 0) {
        int64_t rows = std::min<int64_t>(rows_left, 65535);
        dim3 grid(unsigned(cdiv(q, 256)), unsigned(rows));
        k_rbf_cross64<<<grid, 256, 0, s>>>(xa + (ia ? 0 : row0 * d), ia ? ia + row0 : nullptr,
                                            rows, xb, ib, q, d, sigma2, out + row0 * ldo, ldo);
        PKM_CHECK_LAUNCH();
        row0 += rows;
        rows_left -= rows;
    }
}

}  // namespace pkm
