// Low-rank preconditioners through the matrix inversion lemma (Sections 3.1,
// 3.1.1, 3.2), set up and applied on the GPU in FP64.
//
// Every kind is represented in one form,
//     P = D + Phi Phi^T,      P^-1 = D^-1 - Psi Psi^T,
//     C = I + Phi^T D^-1 Phi = L_C L_C^T,   Psi = D^-1 Phi L_C^-T,
// which is the matrix inversion lemma with the core factorised once:
//   Nystrom  Phi = K_XU L_U^-T (L_U L_U^T = K_UU + jitter I), D = lambda I;
//            then Phi Phi^T = K_XU K_UU^-1 K_UX.
//   FITC     same Phi, D = max(diag(K - Phi Phi^T), 0) + lambda.
//   LOWRANK  Phi given by the caller, D = lambda I.
// Scaling Phi by D^-1/2 before forming C keeps the core well conditioned:
// C's eigenvalues are 1 + (those of Phi^T D^-1 Phi) >= 1.
//
// Apply: Z = D^-1 R - Psi (Psi^T R), two products that each read Psi once.

#include "pkm_internal.h"

#include <cmath>

namespace pkm {

__global__ void k_add_diag(int64_t m, double* __restrict__ A, int64_t lda, double v) {
    int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i < m) A[i * lda + i] += v;
}

__global__ void k_identity_plus(int64_t m, double* __restrict__ A) {
    int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= m * m) return;
    int64_t i = e / m, j = e - i * m;
    if (i == j) A[e] += 1.0;
}

// FITC diagonal: D_i = max(sigma2 - |Phi_i|^2, 0) + lambda; Nystrom: lambda.
__global__ void k_diag_d(const double* __restrict__ phi, int64_t n, int m, int fitc,
                         double sigma2, double lambda, double* __restrict__ D) {
    int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i >= n) return;
    double v = lambda;
    if (fitc) {
        double s = 0.0;
        const double* row = phi + i * m;
        for (int c = 0; c < m; ++c) s = fma(row[c], row[c], s);
        v = fmax(sigma2 - s, 0.0) + lambda;
    }
    D[i] = v;
}

// rows of A (n x m) scaled by f(D_i): mode 0: D^-1/2, mode 1: D^-1/2 again.
__global__ void k_row_scale_rsqrt(int64_t n, int m, const double* __restrict__ D,
                                  double* __restrict__ A) {
    int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= n * int64_t(m)) return;
    int64_t i = e / m;
    A[e] *= 1.0 / sqrt(D[i]);
}

__global__ void k_recip(int64_t n, const double* __restrict__ D, double* __restrict__ out) {
    int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i < n) out[i] = 1.0 / D[i];
}

// Z = dinv o R (row scaling), n x k
__global__ void k_diag_apply(int64_t n, int k, const double* __restrict__ dinv,
                             const double* __restrict__ R, double* __restrict__ Z) {
    int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= n * int64_t(k)) return;
    Z[e] = dinv[e / k] * R[e];
}

__global__ void k_check_idx(const int32_t* __restrict__ idx, int m, int64_t n, int* __restrict__ bad) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m && (idx[i] < 0 || idx[i] >= n)) atomicOr(bad, 1);
}

static void read_info(pkm_ctx* ctx, const int* dinfo, int* out) {
    PKM_HIP(hipMemcpyAsync(out, dinfo, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    PKM_HIP(hipStreamSynchronize(ctx->stream));
}

void precond_setup(pkm_ctx* ctx, const pkm_problem* prob, int kind, int m, const int32_t* idx,
                   const double* Phi, double jitter, pkm_precond* pc) {
    const int64_t n = prob->n;
    hipStream_t s = ctx->stream;
    prepare(ctx, prob, true, false);
    pc->kind = kind;
    pc->n = n;
    pc->m = m;
    pc->device = ctx->device;
    pc->psi.ensure(sizeof(double) * n * m);
    pc->dinv.ensure(sizeof(double) * n);
    double* psi = pc->psi.as<double>();

    // scratch: m x m core, m x 64 block inverses, n diagonal, info word
    ctx->ws_setup[0].ensure(sizeof(double) * int64_t(m) * m);
    ctx->ws_setup[1].ensure(sizeof(double) * int64_t(round_up(m, 64)) * 64);
    ctx->ws_setup[2].ensure(sizeof(double) * n);
    ctx->ws_setup[3].ensure(256);
    double* core = ctx->ws_setup[0].as<double>();
    double* winv = ctx->ws_setup[1].as<double>();
    double* D = ctx->ws_setup[2].as<double>();
    int* dinfo = ctx->ws_setup[3].as<int>();
    int hinfo = 0;

    if (kind == PKM_PC_NYSTROM || kind == PKM_PC_FITC) {
        PKM_HIP(hipMemsetAsync(dinfo, 0, sizeof(int), s));
        k_check_idx<<<cdiv(m, 256), 256, 0, s>>>(idx, m, n, dinfo);
        PKM_CHECK_LAUNCH();
        read_info(ctx, dinfo, &hinfo);
        PKM_REQUIRE(hinfo == 0, "inducing index out of range");
        const double* xs = ctx->prep.xs64.as<double>();
        const int d = prob->d;
        // K_UU + jitter I, then L_U
        rbf_cross64(s, xs, idx, m, xs, idx, m, d, prob->sigma2, core, m);
        if (jitter > 0.0) {
            k_add_diag<<<cdiv(m, 256), 256, 0, s>>>(m, core, m, jitter);
            PKM_CHECK_LAUNCH();
        }
        dpotrf_lower(ctx, m, core, m, winv, dinfo);
        read_info(ctx, dinfo, &hinfo);
        if (hinfo != 0)
            fail(PKM_ERR_BREAKDOWN, "K_UU + jitter I is not positive definite (pivot " +
                                        std::to_string(hinfo - 1) +
                                        "); duplicate inducing points need jitter > 0");
        // Phi = K_XU L_U^-T
        rbf_cross64(s, xs, nullptr, n, xs, idx, m, d, prob->sigma2, psi, m);
        dtrsm_right_lt(ctx, n, m, core, m, winv, psi, m);
        k_diag_d<<<cdiv(n, 256), 256, 0, s>>>(psi, n, m, kind == PKM_PC_FITC, prob->sigma2,
                                              prob->lambda, D);
        PKM_CHECK_LAUNCH();
    } else {
        PKM_HIP(hipMemcpyAsync(psi, Phi, sizeof(double) * n * m, hipMemcpyDeviceToDevice, s));
        k_diag_d<<<cdiv(n, 256), 256, 0, s>>>(psi, n, m, 0, prob->sigma2, prob->lambda, D);
        PKM_CHECK_LAUNCH();
    }
    // Phi~ = D^-1/2 Phi;  C = I + Phi~^T Phi~;  L_C;  Psi = D^-1/2 Phi~ L_C^-T
    k_row_scale_rsqrt<<<cdiv(n * m, 256), 256, 0, s>>>(n, m, D, psi);
    PKM_CHECK_LAUNCH();
    dgemm(ctx, true, false, m, m, n, 1.0, psi, m, psi, m, 0.0, core, m);
    k_identity_plus<<<cdiv(int64_t(m) * m, 256), 256, 0, s>>>(m, core);
    PKM_CHECK_LAUNCH();
    dpotrf_lower(ctx, m, core, m, winv, dinfo);
    read_info(ctx, dinfo, &hinfo);
    if (hinfo != 0)
        fail(PKM_ERR_BREAKDOWN, "Woodbury core I + Phi^T D^-1 Phi is not positive definite "
                                "(non-finite factor?)");
    dtrsm_right_lt(ctx, n, m, core, m, winv, psi, m);
    k_row_scale_rsqrt<<<cdiv(n * m, 256), 256, 0, s>>>(n, m, D, psi);
    PKM_CHECK_LAUNCH();
    k_recip<<<cdiv(n, 256), 256, 0, s>>>(n, D, pc->dinv.as<double>());
    PKM_CHECK_LAUNCH();
    PKM_HIP(hipStreamSynchronize(s));
}

void precond_apply(pkm_ctx* ctx, const pkm_precond* pc, int k, const double* R, double* Z) {
    hipStream_t s = ctx->stream;
    const int64_t n = pc->n;
    const int m = pc->m;
    // T = Psi^T R  (m x k)
    ctx->red2.ensure(sizeof(double) * int64_t(m) * k);
    double* T = ctx->red2.as<double>();
    dgemm(ctx, true, false, m, k, n, 1.0, pc->psi.as<double>(), m, R, k, 0.0, T, k);
    // Z = D^-1 R - Psi T
    k_diag_apply<<<cdiv(n * k, 256), 256, 0, s>>>(n, k, pc->dinv.as<double>(), R, Z);
    PKM_CHECK_LAUNCH();
    dgemm_large(ctx, false, false, n, k, m, -1.0, pc->psi.as<double>(), m, T, k, 1.0, Z, k);
}

}  // namespace pkm
