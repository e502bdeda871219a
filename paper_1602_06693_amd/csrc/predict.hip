// Prediction at test inputs (the GP predictive equations the paper's Section
// 2.1 refers to for test data): mean m_* = K(X_*, X) K_y^-1 y and latent
// variance v_* = k(x_*, x_*) - k_*^T K_y^-1 k_*, one solve per test point
// (the test points' cross-kernel columns are the right-hand sides of one
// block solve).

#include "pkm_internal.h"

#include <algorithm>

namespace pkm {


// I (k x k) on the device
__global__ void k_eye(int64_t k, double* __restrict__ I) {
    const int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= k * k) return;
    I[e] = (e / k == e % k) ? 1.0 : 0.0;
}

// var[c] = sigma2 - sum_i B[i][c] A[i][c]; one work-group per column
__global__ __launch_bounds__(256) void k_pred_var(const double* __restrict__ B,
                                                  const double* __restrict__ A, int64_t n, int k,
                                                  double sigma2, double* __restrict__ var) {
    __shared__ double sh[256];
    const int c = blockIdx.x;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) acc = fma(B[i * k + c], A[i * k + c], acc);
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) var[c] = sigma2 - sh[0];
}

int predict(pkm_ctx* ctx, const pkm_problem* prob, const pkm_precond* pc, const double* y,
            int64_t ns, const double* Xs, const pkm_solve_opts* o, double* mean, double* var,
            pkm_solve_info* info_mean, pkm_solve_info* info_var) {
    hipStream_t s = ctx->stream;
    const int64_t n = prob->n;
    // alpha = K_y^-1 y, then m_* = K(X_*, X) alpha
    ctx->cross[3].ensure(sizeof(double) * std::max<int64_t>(n, 1));
    double* alpha = ctx->cross[3].as<double>();
    int rc = solve(ctx, prob, pc, 1, y, alpha, o, info_mean);
    if (rc < 0) return rc;
    cross_k64(ctx, prob, Xs, ns, prob->X, n, 1, alpha, mean);
    if (!var) return rc;
    // B = K(X, X_*) (n x ns) = K(X, X_*) I;  A = K_y^-1 B;  v = sigma2 - diag(B^T A)
    ctx->pred[0].ensure(sizeof(double) * ns * ns);
    ctx->pred[1].ensure(sizeof(double) * n * ns);
    ctx->pred[2].ensure(sizeof(double) * n * ns);
    double* I = ctx->pred[0].as<double>();
    double* B = ctx->pred[1].as<double>();
    double* A = ctx->pred[2].as<double>();
    k_eye<<<cdiv(ns * ns, 256), 256, 0, s>>>(ns, I);
    PKM_CHECK_LAUNCH();
    cross_k64(ctx, prob, prob->X, n, Xs, ns, int(ns), I, B);
    const int rc2 = solve(ctx, prob, pc, int(ns), B, A, o, info_var);
    if (rc2 < 0) return rc2;
    k_pred_var<<<(unsigned)ns, 256, 0, s>>>(B, A, n, int(ns), prob->sigma2, var);
    PKM_CHECK_LAUNCH();
    PKM_HIP(hipStreamSynchronize(s));
    return std::max(rc, rc2);
}

}  // namespace pkm
