// Laplace approximation for GP classification with a probit likelihood
// (Section 2.2 and the supplementary derivations), every linear system a PCG
// solve with B = I + W^1/2 K W^1/2 and every K product matrix-free.
//
//   Newton step:   b = W f + dlog p,  c = W^1/2 K b,  B z = c,
//                  a = b - W^1/2 z,   f <- K a
//   log q = -1/2 log|B| - 1/2 f^T a + sum log Phi(y f)  (Psi = the last two)
//   gradient (theta = log sigma2, log l_r), probes r_c:
//     -1/(2N) sum_c (W^1/2 B^-1 r_c)^T dK (W^1/2 r_c) + 1/2 a^T dK a
//     -1/2 (W^1/2 B^-1 W^-1/2 u)^T dK (dlog p),
//     u_j = (1/N) sum_c r_cj [K (r_c - W^1/2 B^-1 W^1/2 K r_c)]_j (dW/df_j),
//     dW/df = -d^3 log p / df^3 (W is the negative Hessian)
//   prediction: m = k_*^T dlog p(f_hat), s^2 = k_** - (W^1/2 k_*)^T B^-1
//     (W^1/2 k_*), p(y_* = 1) = Phi(m / sqrt(1 + s^2)).
// B's preconditioner: the low-rank factor Phi of a Nystrom-type
// preconditioner of K, scaled to W^1/2 Phi, through the matrix inversion
// lemma with D = I (the supplement's low-rank preconditioning for B).

#include "pkm_internal.h"

#include <chrono>
#include <cmath>
#include <vector>

namespace pkm {

void precond_setup(pkm_ctx* ctx, const pkm_problem* prob, int kind, int m, const int32_t* idx,
                   const double* Phi, double jitter, pkm_precond* pc, int aux);
void grad_pass(pkm_ctx* ctx, const pkm_problem* prob, int N, const double* AS,
               const double* YZ, double* grad);

// log Phi(z) and r(z) = N(z) / Phi(z), stable in both tails
__device__ inline void probit_parts(double z, double& logphi, double& r) {
    const double e = erfcx(-z * 0.7071067811865476);   // Phi(z) = e exp(-z^2/2) / 2
    r = 0.7978845608028654 / e;                         // 2 / (sqrt(2 pi) e)
    logphi = z < 0.0 ? log(0.5 * e) - 0.5 * z * z : log1p(-0.5 * erfc(z * 0.7071067811865476));
}

// per point: d1 = dlog p/df, W, sw = W^1/2, d3 = d^3 log p/df^3, logp
__global__ void k_probit(int64_t n, const double* __restrict__ y, const double* __restrict__ f,
                         double* __restrict__ d1, double* __restrict__ W,
                         double* __restrict__ sw, double* __restrict__ d3,
                         double* __restrict__ logp) {
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i >= n) return;
    const double yi = y[i], z = yi * f[i];
    double lp, r;
    probit_parts(z, lp, r);
    const double w = r * (z + r);
    d1[i] = yi * r;
    W[i] = w;
    sw[i] = sqrt(w);
    if (d3) d3[i] = yi * r * (z * z + 3.0 * z * r + 2.0 * r * r - 1.0);
    if (logp) logp[i] = lp;
}

// b = W o f + d1
__global__ void k_newton_b(int64_t n, const double* __restrict__ W, const double* __restrict__ f,
                           const double* __restrict__ d1, double* __restrict__ b) {
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i < n) b[i] = fma(W[i], f[i], d1[i]);
}

// out = w o V row-wise (n x k; out may be V)
__global__ void k_scale_rows_n(int64_t n, int k, const double* __restrict__ w, const double* V,
                               double* out) {
    const int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e < n * k) out[e] = w[e / k] * V[e];
}

// out = R - w o Z row-wise (n x k; out may be Z)
__global__ void k_sub_scaled(int64_t n, int k, const double* __restrict__ R,
                             const double* __restrict__ w, const double* Z, double* out) {
    const int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e < n * k) out[e] = R[e] - w[e / k] * Z[e];
}

// I (k x k)
__global__ void k_eye_n(int64_t k, double* __restrict__ I) {
    const int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e < k * k) I[e] = (e / k == e % k) ? 1.0 : 0.0;
}

// a = b - sw o z
__global__ void k_newton_a(int64_t n, const double* __restrict__ b, const double* __restrict__ sw,
                           const double* __restrict__ z, double* __restrict__ a) {
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i < n) a[i] = b[i] - sw[i] * z[i];
}

// block partial sums of u o v (v NULL: of u)
__global__ __launch_bounds__(256) void k_dot_blocks(int64_t n, const double* __restrict__ u,
                                                    const double* __restrict__ v,
                                                    double* __restrict__ part) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
        acc += v ? u[i] * v[i] : u[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// rows of Phi (n x m) scaled by sw
__global__ void k_rows_scale(int64_t n, int m, const double* __restrict__ sw,
                             const double* __restrict__ phi, double* __restrict__ out) {
    const int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e < n * m) out[e] = sw[e / m] * phi[e];
}

// u_j = (1/N) sum_c R_jc P_jc (-d3_j) / sw_j  (the right-hand side W^-1/2 u)
__global__ void k_implicit_u(int64_t n, int N, const double* __restrict__ R,
                             const double* __restrict__ P, const double* __restrict__ d3,
                             const double* __restrict__ sw, double* __restrict__ out) {
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int c = 0; c < N; ++c) s = fma(R[i * N + c], P[i * N + c], s);
    out[i] = (s / N) * (-d3[i]) / sw[i];
}

// Assemble the grad_pass blocks: AS = [a, S1 * (N+1)/N, s3 * (N+1)],
// YZ = [a, V1, d1]  (n x (N + 2)); S1 = sw o Z1, V1 = sw o R, s3 = sw o z3.
__global__ void k_laplace_blocks(int64_t n, int N, const double* __restrict__ a,
                                 const double* __restrict__ sw, const double* __restrict__ Z1,
                                 const double* __restrict__ R, const double* __restrict__ z3,
                                 const double* __restrict__ d1, double* __restrict__ AS,
                                 double* __restrict__ YZ) {
    const int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    const int w = N + 2;
    if (e >= n * w) return;
    const int64_t i = e / w;
    const int c = int(e - i * w);
    const double np1 = double(N + 1);
    if (c == 0) {
        AS[e] = a[i];
        YZ[e] = a[i];
    } else if (c <= N) {
        AS[e] = sw[i] * Z1[i * N + c - 1] * (np1 / N);
        YZ[e] = sw[i] * R[i * N + c - 1];
    } else {
        AS[e] = sw[i] * z3[i] * np1;
        YZ[e] = d1[i];
    }
}

// mean, variance and class probability from m, C = W^1/2 K(X, X_*) and
// Z = B^-1 C (n x ns)
__global__ __launch_bounds__(256) void k_laplace_pred(int64_t n, int ns, double sigma2,
                                                      const double* __restrict__ C,
                                                      const double* __restrict__ Z,
                                                      const double* __restrict__ m,
                                                      double* __restrict__ var,
                                                      double* __restrict__ prob) {
    __shared__ double sh[256];
    const int c = blockIdx.x;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) acc = fma(C[i * ns + c], Z[i * ns + c], acc);
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double v = sigma2 - sh[0];
        var[c] = v;
        prob[c] = 0.5 * erfc(-m[c] / sqrt(1.0 + v) * 0.7071067811865476);
    }
}

static double reduce(pkm_ctx* ctx, int64_t n, const double* u, const double* v) {
    constexpr int NB = 256;
    ctx->lap[7].ensure(sizeof(double) * NB);
    double* part = ctx->lap[7].as<double>();
    k_dot_blocks<<<NB, 256, 0, ctx->stream>>>(n, u, v, part);
    PKM_CHECK_LAUNCH();
    std::vector<double> h(NB);
    PKM_HIP(hipMemcpyAsync(h.data(), part, sizeof(double) * NB, hipMemcpyDeviceToHost, ctx->stream));
    PKM_HIP(hipStreamSynchronize(ctx->stream));
    double s = 0.0;
    for (double x : h) s += x;
    return s;
}

// B's preconditioner from a factor-form preconditioner of K (kept factor
// Phi): P_B = I + (W^1/2 Phi)(W^1/2 Phi)^T.  NULL if base is NULL.
struct PcHolder {
    pkm_precond* p = nullptr;
    ~PcHolder() { reset(); }
    void reset() {
        if (p) {
            p->psi.release();
            p->dinv.release();
            p->dblk.release();
            p->phi.release();
            delete p;
            p = nullptr;
        }
    }
};

static void b_precond(pkm_ctx* ctx, const pkm_problem* prob, const pkm_precond* base,
                      const double* sw, PcHolder& out) {
    out.reset();
    if (!base) return;
    PKM_REQUIRE(base->phi.p != nullptr, "preconditioner has no low-rank factor");
    const int64_t n = prob->n;
    const int m = base->m;
    ctx->lap[6].ensure(sizeof(double) * n * m);
    double* sphi = ctx->lap[6].as<double>();
    k_rows_scale<<<cdiv(n * m, 256), 256, 0, ctx->stream>>>(n, m, sw, base->phi.as<double>(), sphi);
    PKM_CHECK_LAUNCH();
    pkm_problem unit = *prob;
    unit.lambda = 1.0;
    out.p = new pkm_precond();
    precond_setup(ctx, &unit, PKM_PC_LOWRANK, m, nullptr, sphi, 0.0, out.p, 0);
}

int laplace_mode(pkm_ctx* ctx, const pkm_problem* prob, const pkm_precond* base, const double* y,
                 const pkm_solve_opts* o, int max_newton, double tol, double* f, double* a,
                 pkm_laplace_info* info) {
    hipStream_t s = ctx->stream;
    const int64_t n = prob->n;
    const unsigned gn = unsigned(cdiv(n, 256));
    auto t0 = std::chrono::steady_clock::now();
    for (int q = 0; q < 6; ++q) ctx->lap[q].ensure(sizeof(double) * n);
    double* d1 = ctx->lap[0].as<double>();
    double* W = ctx->lap[1].as<double>();
    double* sw = ctx->lap[2].as<double>();
    double* lp = ctx->lap[3].as<double>();
    double* b = ctx->lap[4].as<double>();
    double* t = ctx->lap[5].as<double>();
    ctx->lap[8].ensure(sizeof(double) * n);
    double* z = ctx->lap[8].as<double>();
    prepare(ctx, prob, true, o->prec != PKM_FP64);
    PKM_HIP(hipMemsetAsync(f, 0, sizeof(double) * n, s));
    PcHolder pcb;
    double psi_old = -INFINITY, psi = 0.0;
    int64_t steps = 0;
    int it = 0, rc = PKM_OK;
    for (it = 1; it <= max_newton; ++it) {
        k_probit<<<gn, 256, 0, s>>>(n, y, f, d1, W, sw, nullptr, lp);
        PKM_CHECK_LAUNCH();
        k_newton_b<<<gn, 256, 0, s>>>(n, W, f, d1, b);                   // b = W f + d1
        PKM_CHECK_LAUNCH();
        mvm_shift(ctx, PKM_FP64, 1, b, t, 0.0);                          // K b
        k_scale_rows_n<<<gn, 256, 0, s>>>(n, 1, sw, t, t);               // c = W^1/2 K b
        PKM_CHECK_LAUNCH();
        b_precond(ctx, prob, base, sw, pcb);
        pkm_solve_info si{};
        const int r = solve(ctx, prob, pcb.p, 1, t, z, o, &si, sw);      // B z = c
        steps += si.total_iters;
        if (r < 0) return r;
        if (r > rc) rc = r;
        k_newton_a<<<gn, 256, 0, s>>>(n, b, sw, z, a);                   // a = b - W^1/2 z
        PKM_CHECK_LAUNCH();
        mvm_shift(ctx, PKM_FP64, 1, a, f, 0.0);                          // f = K a
        k_probit<<<gn, 256, 0, s>>>(n, y, f, d1, W, sw, nullptr, lp);
        PKM_CHECK_LAUNCH();
        psi = reduce(ctx, n, lp, nullptr) - 0.5 * reduce(ctx, n, a, f);
        if (!std::isfinite(psi)) fail(PKM_ERR_BREAKDOWN, "Laplace: non-finite objective");
        if (std::fabs(psi - psi_old) <= tol * std::fmax(1.0, std::fabs(psi))) break;
        psi_old = psi;
    }
    if (it > max_newton) {
        it = max_newton;
        if (rc == PKM_OK) rc = PKM_NOT_CONVERGED;
        ctx->err = "Laplace: Newton iterations reached max_newton";
    }
    if (info) {
        info->newton_iters = it;
        info->pcg_steps = steps;
        info->psi = psi;
        info->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return rc;
}

int laplace_grad(pkm_ctx* ctx, const pkm_problem* prob, const pkm_precond* base, const double* y,
                 const double* f, int N, const double* R, const pkm_solve_opts* o, double* grad,
                 int64_t* pcg_steps) {
    hipStream_t s = ctx->stream;
    const int64_t n = prob->n;
    const unsigned gn = unsigned(cdiv(n, 256));
    const unsigned gnN = unsigned(cdiv(n * N, 256));
    for (int q = 0; q < 6; ++q) ctx->lap[q].ensure(sizeof(double) * n);
    double* d1 = ctx->lap[0].as<double>();
    double* W = ctx->lap[1].as<double>();
    double* sw = ctx->lap[2].as<double>();
    double* d3 = ctx->lap[3].as<double>();
    double* u = ctx->lap[4].as<double>();
    double* z3 = ctx->lap[5].as<double>();
    ctx->lap[9].ensure(sizeof(double) * n * N);
    ctx->lap[10].ensure(sizeof(double) * n * N);
    ctx->lap[11].ensure(sizeof(double) * n * N);
    double* Z1 = ctx->lap[9].as<double>();
    double* T = ctx->lap[10].as<double>();
    double* Z2 = ctx->lap[11].as<double>();
    prepare(ctx, prob, true, o->prec != PKM_FP64);
    k_probit<<<gn, 256, 0, s>>>(n, y, f, d1, W, sw, d3, nullptr);
    PKM_CHECK_LAUNCH();
    PcHolder pcb;
    b_precond(ctx, prob, base, sw, pcb);
    int64_t steps = 0;
    int rc = PKM_OK;
    auto bsolve = [&](int k, const double* rhs, double* out) {
        pkm_solve_info si{};
        const int r = solve(ctx, prob, pcb.p, k, rhs, out, o, &si, sw);
        steps += si.total_iters;
        if (r < 0) fail(r, ctx->err);
        rc = std::max(rc, r);
    };
    // explicit trace term: Z1 = B^-1 R
    bsolve(N, R, Z1);
    // implicit term: T = W^1/2 K R, Z2 = B^-1 T, T = K (R - W^1/2 Z2)
    mvm_shift(ctx, PKM_FP64, N, R, T, 0.0);
    k_scale_rows_n<<<gnN, 256, 0, s>>>(n, N, sw, T, T);
    PKM_CHECK_LAUNCH();
    bsolve(N, T, Z2);
    k_sub_scaled<<<gnN, 256, 0, s>>>(n, N, R, sw, Z2, Z2);   // Z2 <- R - W^1/2 Z2
    PKM_CHECK_LAUNCH();
    mvm_shift(ctx, PKM_FP64, N, Z2, T, 0.0);                  // (K^-1 + W)^-1 r_c
    k_implicit_u<<<gn, 256, 0, s>>>(n, N, R, T, d3, sw, u);   // W^-1/2 u
    PKM_CHECK_LAUNCH();
    bsolve(1, u, z3);
    // bilinear forms through the gradient pass: [a, S1 (N+1)/N, s3 (N+1)] vs [a, V1, d1]
    ctx->lap[12].ensure(sizeof(double) * n * (N + 2));
    ctx->lap[13].ensure(sizeof(double) * n * (N + 2));
    double* AS = ctx->lap[12].as<double>();
    double* YZ = ctx->lap[13].as<double>();
    k_laplace_blocks<<<cdiv(n * (N + 2), 256), 256, 0, s>>>(n, N, d1, sw, Z1, R, z3, d1, AS, YZ);
    PKM_CHECK_LAUNCH();
    std::vector<double> g(prob->d + 2);
    grad_pass(ctx, prob, N + 1, AS, YZ, g.data());
    for (int i = 0; i <= prob->d; ++i) grad[i] = g[i];
    if (pcg_steps) *pcg_steps = steps;
    return rc;
}

int laplace_predict(pkm_ctx* ctx, const pkm_problem* prob, const pkm_precond* base,
                    const double* y, const double* f, int64_t ns, const double* Xs,
                    const pkm_solve_opts* o, double* mean, double* var, double* prob_out) {
    hipStream_t s = ctx->stream;
    const int64_t n = prob->n;
    const unsigned gn = unsigned(cdiv(n, 256));
    for (int q = 0; q < 3; ++q) ctx->lap[q].ensure(sizeof(double) * n);
    double* d1 = ctx->lap[0].as<double>();
    double* W = ctx->lap[1].as<double>();
    double* sw = ctx->lap[2].as<double>();
    prepare(ctx, prob, true, o->prec != PKM_FP64);
    k_probit<<<gn, 256, 0, s>>>(n, y, f, d1, W, sw, nullptr, nullptr);
    PKM_CHECK_LAUNCH();
    cross_k64(ctx, prob, Xs, ns, prob->X, n, 1, d1, mean);    // m = K(X_*, X) dlog p
    // C = W^1/2 K(X, X_*),  Z = B^-1 C
    ctx->pred[0].ensure(sizeof(double) * ns * ns);
    ctx->pred[1].ensure(sizeof(double) * n * ns);
    ctx->pred[2].ensure(sizeof(double) * n * ns);
    double* I = ctx->pred[0].as<double>();
    double* C = ctx->pred[1].as<double>();
    double* Z = ctx->pred[2].as<double>();
    k_eye_n<<<cdiv(ns * ns, 256), 256, 0, s>>>(ns, I);
    PKM_CHECK_LAUNCH();
    cross_k64(ctx, prob, prob->X, n, Xs, ns, int(ns), I, C);
    k_scale_rows_n<<<unsigned(cdiv(n * ns, 256)), 256, 0, s>>>(n, int(ns), sw, C, C);
    PKM_CHECK_LAUNCH();
    PcHolder pcb;
    b_precond(ctx, prob, base, sw, pcb);
    pkm_solve_info si{};
    const int rc = solve(ctx, prob, pcb.p, int(ns), C, Z, o, &si, sw);
    if (rc < 0) return rc;
    k_laplace_pred<<<unsigned(ns), 256, 0, s>>>(n, int(ns), prob->sigma2, C, Z, mean, var,
                                                prob_out);
    PKM_CHECK_LAUNCH();
    PKM_HIP(hipStreamSynchronize(s));
    return rc;
}

}  // namespace pkm
