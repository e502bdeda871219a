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
//   SKETCH   Phi = K S L^-T (L L^T = S^T K S + jitter), D = lambda I.
//   PITC     Nystrom's Phi, D block diagonal (see the PITC kernels below).
//   HYBRID   SKETCH with S = [columns of I at idx, caller's U].
//   SPECTRAL Phi = random Fourier features (Section 3.2), D = lambda I.
// Scaling Phi by D^-1/2 before forming C keeps the core well conditioned:
// C's eigenvalues are 1 + (those of Phi^T D^-1 Phi) >= 1.
//
// Apply: Z = D^-1 R - Psi (Psi^T R), two products that each read Psi once.

#include "pkm_internal.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace pkm {

// A_ii *= f (relative jitter: invariant to rescaling a sketch column)
__global__ void k_scale_diag(int64_t m, double* __restrict__ A, int64_t lda, double f) {
    int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i < m) A[i * lda + i] *= f;
}

__global__ void k_add_diag(int64_t m, double* __restrict__ A, int64_t lda, double v) {
    int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i < m) A[i * lda + i] += v;
}

// Y -= lambda V (n x m)
__global__ void k_axpy_neg(int64_t tot, double lambda, const double* __restrict__ V,
                           double* __restrict__ Y) {
    int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e < tot) Y[e] -= lambda * V[e];
}

// A <- (A + A^T) / 2 for an m x m matrix
__global__ void k_symmetrize(int64_t m, double* __restrict__ A) {
    int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= m * m) return;
    int64_t i = e / m, j = e - i * m;
    if (j < i) {
        double v = 0.5 * (A[e] + A[j * m + i]);
        A[e] = v;
        A[j * m + i] = v;
    }
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

// ---------------------------------------------------------------------------
// PITC (Section 3.1.1): D = blockdiag(K_BB - Phi_B Phi_B^T) + lambda I over
// consecutive row blocks of size b (last block ragged).  With block Cholesky
// D_B = L_B L_B^T the unified form holds with L_D^-1 in place of D^-1/2:
//     Phi~ = L_D^-1 Phi,  C = I + Phi~^T Phi~ = L_C L_C^T,
//     Psi = L_D^-T Phi~ L_C^-T,   P^-1 = D^-1 - Psi Psi^T.
// Blocks are stored row-major per row: element (i, lj) at i * b + lj is
// block(i)'s entry (i mod b, lj); columns past a ragged block's size are 0.
// ---------------------------------------------------------------------------
__global__ void k_pitc_blocks(const double* __restrict__ xs, int64_t n, int d, double sigma2,
                              double lambda, const double* __restrict__ phi, int m, int b,
                              double* __restrict__ Dblk) {
    const int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= n * b) return;
    const int64_t i = e / b;
    const int lj = int(e - i * b);
    const int64_t j = (i / b) * b + lj;
    if (j >= n) {
        Dblk[e] = 0.0;
        return;
    }
    double sq = 0.0;
    for (int r = 0; r < d; ++r) {
        const double t = xs[i * d + r] - xs[j * d + r];
        sq = fma(t, t, sq);
    }
    double q = 0.0;
    const double* pi = phi + i * m;
    const double* pj = phi + j * m;
    for (int c = 0; c < m; ++c) q = fma(pi[c], pj[c], q);
    Dblk[e] = sigma2 * exp(-0.5 * sq) - q + (i == j ? lambda : 0.0);
}

// One work-group per block: Cholesky D_B = L L^T in LDS, then L^-1 (written
// to Linv) and D_B^-1 = L^-T L^-1 (written over Dblk).  b <= 64.  info gets
// 1 + (first failing block) if a pivot is not positive.
constexpr int kPitcMaxBlock = 64;
__global__ __launch_bounds__(256) void k_pitc_factor(int64_t n, int b, double* __restrict__ Dblk,
                                                     double* __restrict__ Linv,
                                                     int* __restrict__ info) {
    __shared__ double A[kPitcMaxBlock][kPitcMaxBlock + 1];
    __shared__ double Li[kPitcMaxBlock][kPitcMaxBlock + 1];
    __shared__ int bad;
    const int64_t r0 = int64_t(blockIdx.x) * b;
    const int bs = int(min(int64_t(b), n - r0));
    const int tid = threadIdx.x;
    if (tid == 0) bad = 0;
    for (int e = tid; e < bs * bs; e += blockDim.x) {
        const int li = e / bs, lj = e - li * bs;
        A[li][lj] = Dblk[(r0 + li) * b + lj];
        Li[li][lj] = 0.0;
    }
    __syncthreads();
    // right-looking Cholesky, lower triangle
    for (int j = 0; j < bs; ++j) {
        const double piv = A[j][j];
        if (!(piv > 0.0)) {
            if (tid == 0) bad = 1;
            break;   // uniform: every thread reads the same A[j][j]
        }
        const double lj = sqrt(piv);
        __syncthreads();
        for (int i = j + tid; i < bs; i += blockDim.x) A[i][j] = (i == j) ? lj : A[i][j] / lj;
        __syncthreads();
        const int rem = bs - j - 1;
        for (int e = tid; e < rem * rem; e += blockDim.x) {
            const int i = j + 1 + e / rem, c = j + 1 + e % rem;
            if (c <= i) A[i][c] -= A[i][j] * A[c][j];
        }
        __syncthreads();
    }
    __syncthreads();
    if (bad) {
        if (tid == 0) atomicCAS(info, 0, int(blockIdx.x) + 1);
        return;
    }
    // L^-1 column by column (forward substitution), one thread per column
    for (int c = tid; c < bs; c += blockDim.x) {
        for (int i = c; i < bs; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int t = c; t < i; ++t) s -= A[i][t] * Li[t][c];
            Li[i][c] = s / A[i][i];
        }
    }
    __syncthreads();
    for (int e = tid; e < b * b; e += blockDim.x) {
        const int li = e / b, lj = e - li * b;
        if (li >= bs) continue;
        double inv = 0.0, dinvv = 0.0;
        if (lj < bs) {
            inv = Li[li][lj];
            const int t0 = li > lj ? li : lj;
            for (int t = t0; t < bs; ++t) dinvv = fma(Li[t][li], Li[t][lj], dinvv);
        }
        Linv[(r0 + li) * b + lj] = inv;
        Dblk[(r0 + li) * b + lj] = dinvv;
    }
}

// out = blockdiag(L^-1) in (trans = 0) or blockdiag(L^-T) in (trans = 1),
// in / out n x m row-major, distinct.
__global__ void k_pitc_tri_mul(int64_t n, int b, const double* __restrict__ Linv, int trans,
                               const double* __restrict__ in, int m, double* __restrict__ out) {
    const int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= n * m) return;
    const int64_t i = e / m;
    const int c = int(e - i * m);
    const int64_t r0 = (i / b) * b;
    const int li = int(i - r0);
    const int bs = int(min(int64_t(b), n - r0));
    double s = 0.0;
    if (!trans) {
        for (int t = 0; t <= li; ++t) s = fma(Linv[i * b + t], in[(r0 + t) * m + c], s);
    } else {
        for (int t = li; t < bs; ++t) s = fma(Linv[(r0 + t) * b + li], in[(r0 + t) * m + c], s);
    }
    out[e] = s;
}

// Z = blockdiag(D^-1) R (R, Z n x k row-major, distinct)
__global__ void k_pitc_dinv(int64_t n, int b, const double* __restrict__ Dinv,
                            const double* __restrict__ R, int k, double* __restrict__ Z) {
    const int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= n * k) return;
    const int64_t i = e / k;
    const int c = int(e - i * k);
    const int64_t r0 = (i / b) * b;
    const int bs = int(min(int64_t(b), n - r0));
    double s = 0.0;
    for (int t = 0; t < bs; ++t) s = fma(Dinv[i * b + t], R[(r0 + t) * k + c], s);
    Z[e] = s;
}

// 1 / D_ii from the (not yet inverted) blocks, for pkm_precond_diag
__global__ void k_pitc_diag_recip(int64_t n, int b, const double* __restrict__ Dblk,
                                  double* __restrict__ dinv) {
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i >= n) return;
    dinv[i] = 1.0 / Dblk[i * b + (i % b)];
}

// dst[:, col0 : col0 + cols] (leading dimension ldd) = src (rows x cols, dense)
__global__ void k_put_cols(int64_t rows, int cols, const double* __restrict__ src,
                           double* __restrict__ dst, int64_t ldd, int col0) {
    const int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= rows * cols) return;
    const int64_t i = e / cols;
    const int c = int(e - i * cols);
    dst[i * ldd + col0 + c] = src[e];
}

// Random Fourier features (Section 3.2, spectral approximation): omega_r =
// W_r / l (W standard normal, m x d), Phi (n x 2m) row i = sqrt(sigma2 / m)
// [cos(omega_1^T x_i) .. cos(omega_m^T x_i), sin(omega_1^T x_i) .. ].
__global__ void k_spectral_features(const double* __restrict__ X, int64_t n, int d,
                                    const double* __restrict__ inv_l,
                                    const double* __restrict__ W, int m, double scale,
                                    double* __restrict__ Phi) {
    const int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= n * m) return;
    const int64_t i = e / m;
    const int r = int(e - i * m);
    double a = 0.0;
    for (int t = 0; t < d; ++t) a = fma(X[i * d + t], W[int64_t(r) * d + t] * inv_l[t], a);
    double sn, cs;
    sincos(a, &sn, &cs);
    Phi[i * 2 * m + r] = scale * cs;
    Phi[i * 2 * m + m + r] = scale * sn;
}

// out[t, :] = W[idx[t], :] for t < m (W and out with row length w)
__global__ void k_gather_rows(const double* __restrict__ W, const int32_t* __restrict__ idx,
                              int m, int w, double* __restrict__ out) {
    const int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= int64_t(m) * w) return;
    const int64_t t = e / w;
    const int c = int(e - t * w);
    out[e] = W[int64_t(idx[t]) * w + c];
}

static void read_info(pkm_ctx* ctx, const int* dinfo, int* out) {
    PKM_HIP(hipMemcpyAsync(out, dinfo, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    PKM_HIP(hipStreamSynchronize(ctx->stream));
}

// The low-rank factor Phi of P = D + Phi Phi^T (pc->psi holds it at this
// point) is kept for pkm_precond_sub_lowrank.
static void keep_factor(pkm_ctx* ctx, pkm_precond* pc) {
    pc->phi.ensure(sizeof(double) * pc->n * pc->m);
    PKM_HIP(hipMemcpyAsync(pc->phi.p, pc->psi.p, sizeof(double) * pc->n * pc->m,
                           hipMemcpyDeviceToDevice, ctx->stream));
}

// Hybrid sketch S = [columns of I at idx (m_idx), U (n x r)]: the factor
// W L^-T with W = K S (K_XU and K U in FP64) and
// L L^T = S^T W + jitter * diag(S^T W) (rows idx of W, then U^T W).
// Written to out (n x (m_idx + r)); core / winv: (m_idx + r)^2 scratch.
static void hybrid_factor(pkm_ctx* ctx, const pkm_problem* prob, int m_idx, int r,
                          const int32_t* idx, const double* U, double jitter, double* out,
                          double* core, double* winv, int* dinfo) {
    const int64_t n = prob->n;
    const int w = m_idx + r;
    hipStream_t s = ctx->stream;
    const double* xs = ctx->P().xs64.as<double>();
    rbf_cross64(s, xs, nullptr, n, xs, idx, m_idx, prob->d, prob->sigma2, out, w);
    ctx->ws_pitc[1].ensure(sizeof(double) * n * r);
    double* KU = ctx->ws_pitc[1].as<double>();
    mvm_shift(ctx, PKM_FP64, r, U, KU, 0.0);
    k_put_cols<<<cdiv(n * r, 256), 256, 0, s>>>(n, r, KU, out, w, m_idx);
    PKM_CHECK_LAUNCH();
    k_gather_rows<<<cdiv(int64_t(m_idx) * w, 256), 256, 0, s>>>(out, idx, m_idx, w, core);
    PKM_CHECK_LAUNCH();
    dgemm(ctx, true, false, r, w, n, 1.0, U, r, out, w, 0.0, core + int64_t(m_idx) * w, w);
    k_symmetrize<<<cdiv(int64_t(w) * w, 256), 256, 0, s>>>(w, core);
    PKM_CHECK_LAUNCH();
    k_scale_diag<<<cdiv(w, 256), 256, 0, s>>>(w, core, w, 1.0 + jitter);
    PKM_CHECK_LAUNCH();
    dpotrf_lower(ctx, w, core, w, winv, dinfo);
    int hinfo = 0;
    read_info(ctx, dinfo, &hinfo);
    if (hinfo != 0)
        fail(PKM_ERR_BREAKDOWN, "hybrid: S^T K S + jitter I is not positive definite "
                                "(dependent sketch columns need jitter > 0)");
    dtrsm_right_lt(ctx, n, w, core, w, winv, out, w);
}

// PITC from Nystrom's Phi (already in pc->psi): block factors, Phi~, core,
// Psi.  Scratch: Linv (n x b), Phi~ (n x m).
static void setup_pitc(pkm_ctx* ctx, const pkm_problem* prob, int m, int b, pkm_precond* pc) {
    const int64_t n = prob->n;
    hipStream_t s = ctx->stream;
    double* psi = pc->psi.as<double>();
    pc->block = b;
    pc->dblk.ensure(sizeof(double) * n * b);
    double* Dblk = pc->dblk.as<double>();
    ctx->ws_pitc[0].ensure(sizeof(double) * n * b);
    ctx->ws_pitc[1].ensure(sizeof(double) * n * m);
    double* Linv = ctx->ws_pitc[0].as<double>();
    double* ptil = ctx->ws_pitc[1].as<double>();
    double* core = ctx->ws_setup[0].as<double>();
    double* winv = ctx->ws_setup[1].as<double>();
    int* dinfo = ctx->ws_setup[3].as<int>();
    int hinfo = 0;
    const double* xs = ctx->P().xs64.as<double>();
    k_pitc_blocks<<<cdiv(n * b, 256), 256, 0, s>>>(xs, n, prob->d, prob->sigma2, prob->lambda,
                                                   psi, m, b, Dblk);
    PKM_CHECK_LAUNCH();
    k_pitc_diag_recip<<<cdiv(n, 256), 256, 0, s>>>(n, b, Dblk, pc->dinv.as<double>());   // 1 / D_ii
    PKM_CHECK_LAUNCH();
    PKM_HIP(hipMemsetAsync(dinfo, 0, sizeof(int), s));
    k_pitc_factor<<<(unsigned)cdiv(n, b), 256, 0, s>>>(n, b, Dblk, Linv, dinfo);
    PKM_CHECK_LAUNCH();
    read_info(ctx, dinfo, &hinfo);
    if (hinfo != 0)
        fail(PKM_ERR_BREAKDOWN, "PITC: diagonal block " + std::to_string(hinfo - 1) +
                                    " of K - Q + lambda I is not positive definite");
    // Phi~ = L_D^-1 Phi;  C = I + Phi~^T Phi~;  Phi~ L_C^-T;  Psi = L_D^-T (.)
    k_pitc_tri_mul<<<cdiv(n * m, 256), 256, 0, s>>>(n, b, Linv, 0, psi, m, ptil);
    PKM_CHECK_LAUNCH();
    dgemm(ctx, true, false, m, m, n, 1.0, ptil, m, ptil, m, 0.0, core, m);
    k_identity_plus<<<cdiv(int64_t(m) * m, 256), 256, 0, s>>>(m, core);
    PKM_CHECK_LAUNCH();
    dpotrf_lower(ctx, m, core, m, winv, dinfo);
    read_info(ctx, dinfo, &hinfo);
    if (hinfo != 0)
        fail(PKM_ERR_BREAKDOWN, "Woodbury core I + Phi^T D^-1 Phi is not positive definite "
                                "(non-finite factor?)");
    dtrsm_right_lt(ctx, n, m, core, m, winv, ptil, m);
    k_pitc_tri_mul<<<cdiv(n * m, 256), 256, 0, s>>>(n, b, Linv, 1, ptil, m, psi);
    PKM_CHECK_LAUNCH();
    PKM_HIP(hipStreamSynchronize(s));
}

// aux: block size (PITC) or number of learned columns r (HYBRID: the sketch
// is [columns of I at idx (m of them), Phi (n x r)], m + r columns in all).
void precond_setup(pkm_ctx* ctx, const pkm_problem* prob, int kind, int m_in, const int32_t* idx,
                   const double* Phi, double jitter, pkm_precond* pc, int aux) {
    const int64_t n = prob->n;
    hipStream_t s = ctx->stream;
    prepare(ctx, prob, true, kind == PKM_PC_SKETCH);
    const int m = kind == PKM_PC_HYBRID ? m_in + aux : kind == PKM_PC_SPECTRAL ? 2 * m_in : m_in;
    const int block = aux;
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

    if (kind == PKM_PC_NYSTROM || kind == PKM_PC_FITC || kind == PKM_PC_PITC ||
        kind == PKM_PC_HYBRID) {
        PKM_HIP(hipMemsetAsync(dinfo, 0, sizeof(int), s));
        k_check_idx<<<cdiv(m_in, 256), 256, 0, s>>>(idx, m_in, n, dinfo);
        PKM_CHECK_LAUNCH();
        read_info(ctx, dinfo, &hinfo);
        PKM_REQUIRE(hinfo == 0, "inducing index out of range");
        const double* xs = ctx->P().xs64.as<double>();
        const int d = prob->d;
        if (kind == PKM_PC_HYBRID) {
            hybrid_factor(ctx, prob, m_in, aux, idx, Phi, jitter, psi, core, winv, dinfo);
            k_diag_d<<<cdiv(n, 256), 256, 0, s>>>(psi, n, m, 0, prob->sigma2, prob->lambda, D);
            PKM_CHECK_LAUNCH();
        } else {
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
        if (kind == PKM_PC_PITC) {
            keep_factor(ctx, pc);
            setup_pitc(ctx, prob, m, block, pc);
            return;
        }
        k_diag_d<<<cdiv(n, 256), 256, 0, s>>>(psi, n, m, kind == PKM_PC_FITC, prob->sigma2,
                                              prob->lambda, D);
        PKM_CHECK_LAUNCH();
        }
    } else if (kind == PKM_PC_SKETCH) {
        // K S with the FP32 product (K S = (K + lambda I) S - lambda S)
        mvm(ctx, PKM_FP32, m, Phi, psi);
        k_axpy_neg<<<cdiv(n * m, 256), 256, 0, s>>>(n * m, prob->lambda, Phi, psi);
        PKM_CHECK_LAUNCH();
        // C = S^T K S (+ jitter * its diagonal), L = chol(C), factor = K S L^-T
        dgemm(ctx, true, false, m, m, n, 1.0, Phi, m, psi, m, 0.0, core, m);
        k_symmetrize<<<cdiv(int64_t(m) * m, 256), 256, 0, s>>>(m, core);
        PKM_CHECK_LAUNCH();
        k_scale_diag<<<cdiv(m, 256), 256, 0, s>>>(m, core, m, 1.0 + jitter);
        PKM_CHECK_LAUNCH();
        dpotrf_lower(ctx, m, core, m, winv, dinfo);
        read_info(ctx, dinfo, &hinfo);
        if (hinfo != 0)
            fail(PKM_ERR_BREAKDOWN, "sketch: S^T K S + jitter I is not positive definite "
                                    "(dependent sketch columns need jitter > 0)");
        dtrsm_right_lt(ctx, n, m, core, m, winv, psi, m);
        k_diag_d<<<cdiv(n, 256), 256, 0, s>>>(psi, n, m, 0, prob->sigma2, prob->lambda, D);
        PKM_CHECK_LAUNCH();
    } else if (kind == PKM_PC_SPECTRAL) {
        // Phi holds the m x d standard normal draws; m (here) = 2 m_in features
        const double* inv_l = ctx->scal.as<double>();   // written by prepare()
        k_spectral_features<<<cdiv(n * m_in, 256), 256, 0, s>>>(
            prob->X, n, prob->d, inv_l, Phi, m_in, std::sqrt(prob->sigma2 / m_in), psi);
        PKM_CHECK_LAUNCH();
        k_diag_d<<<cdiv(n, 256), 256, 0, s>>>(psi, n, m, 0, prob->sigma2, prob->lambda, D);
        PKM_CHECK_LAUNCH();
    } else {
        PKM_HIP(hipMemcpyAsync(psi, Phi, sizeof(double) * n * m, hipMemcpyDeviceToDevice, s));
        k_diag_d<<<cdiv(n, 256), 256, 0, s>>>(psi, n, m, 0, prob->sigma2, prob->lambda, D);
        PKM_CHECK_LAUNCH();
    }
    keep_factor(ctx, pc);
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

// ---------------------------------------------------------------------------
// Apply: Z = D^-1 R - Psi (Psi^T R).  Both phases stream Psi from HBM once.
// ---------------------------------------------------------------------------
constexpr int AT = 64;   // Psi columns per work-group (phase 1), rows (phase 2)

typedef double f64x4 __attribute__((ext_vector_type(4)));

// Psi is read as FP64 or as its FP32 rounding (pkm_precond_psi_f32); either
// way every entry is widened to FP64 on load and the sums are FP64 MFMA.
template <typename T> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };

// Phase 1: part[chunk][j][c] = sum_{i in chunk} Psi[i][j] R[i][c] on 16x16x4
// FP64 MFMA.  Wave w owns the 16 Psi columns j0 .. j0 + 15; lane l feeds
// A[j0 + l % 16][i] = Psi[i][j0 + l % 16] and B[i][c] = R[i][c0 + 16 kt + l % 16]
// for rows i = ib + 4 (l / 16) + q, so each load instruction reads four rows
// of 16 consecutive doubles (whole 128-byte lines of Psi).  Whole 16-row
// blocks load without guards -- a lane past the last column or past column
// kc reads a clamped in-bounds address, which only feeds output entries that
// are never stored -- and the next block's loads are issued before this
// block's MFMAs, so a wave keeps a block of HBM reads in flight behind its
// matrix-core work; the ragged last block of a chunk loads under guards.
// PAIR (JT = 2, m even): lane cc of the wave's two tiles takes the adjacent
// Psi columns j0 + 2 cc and j0 + 2 cc + 1, one 16-byte load for both tiles;
// output row rho of tile t is then column j0 + 2 rho + t.
template <int KT, int JT, bool PAIR, typename PT>
__global__ __launch_bounds__(256) void k_psit_r(const PT* __restrict__ psi, int m,
                                                const double* __restrict__ R, int k, int c0,
                                                int kc, int64_t n, int64_t rows_per_chunk,
                                                double* __restrict__ part) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = lane >> 4, cc = lane & 15;
    const int j0 = (blockIdx.x * 4 + w) * 16 * JT;   // JT 16-column tiles of Psi per wave
    if (j0 >= m) return;
    const int64_t i0 = int64_t(blockIdx.y) * rows_per_chunk;
    const int64_t i1 = min(n, i0 + rows_per_chunk);
    int jc[JT];
#pragma unroll
    for (int t = 0; t < JT; ++t)
        jc[t] = PAIR ? min(j0 + 2 * cc, m - 2) + t : min(j0 + 16 * t + cc, m - 1);
    int col[KT];
    bool cv[KT];
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) {
        cv[kt] = 16 * kt + cc < kc;
        col[kt] = c0 + min(16 * kt + cc, kc - 1);
    }
    f64x4 acc[JT][KT];
#pragma unroll
    for (int t = 0; t < JT; ++t)
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) acc[t][kt] = f64x4{0.0, 0.0, 0.0, 0.0};
    const int64_t ifull = i0 + ((i1 - i0) & ~int64_t(15));
    double a[JT][4], b[4][KT];
    auto load = [&](int64_t ib, double (&la)[JT][4], double (&lb)[4][KT]) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t i = ib + 4 * g + q;
            if (PAIR) {
                using P2 = typename Vec2<PT>::type;
                const P2 x = *reinterpret_cast<const P2*>(psi + i * m + jc[0]);
                la[0][q] = double(x.x);
                la[1][q] = double(x.y);
            } else {
#pragma unroll
                for (int t = 0; t < JT; ++t) la[t][q] = double(psi[i * m + jc[t]]);
            }
#pragma unroll
            for (int kt = 0; kt < KT; ++kt) lb[q][kt] = R[i * k + col[kt]];
        }
    };
    auto step = [&](const double (&la)[JT][4], const double (&lb)[4][KT]) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int kt = 0; kt < KT; ++kt)
#pragma unroll
                for (int t = 0; t < JT; ++t)
                    acc[t][kt] = __builtin_amdgcn_mfma_f64_16x16x4f64(la[t][q], lb[q][kt], acc[t][kt],
                                                                      0, 0, 0);
    };
    // two register buffers in turn: a block's loads are issued one block
    // ahead of its MFMAs and never copied (a copy would wait for them)
    // (unconditional loads -- past the end they re-read the last block -- so
    // that every wait counts exactly the loads it needs)
    double a2[JT][4], b2[4][KT];
    if (i0 < ifull) {
        const int64_t last = ifull - 16;
        load(i0, a, b);
        for (int64_t ib = i0; ib < ifull; ib += 32) {
            load(min(ib + 16, last), a2, b2);
            step(a, b);
            if (ib + 16 >= ifull) break;
            load(min(ib + 32, last), a, b);
            step(a2, b2);
        }
    }
    if (ifull < i1) {   // ragged last block: rows past i1 contribute zero
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t i = ifull + 4 * g + q;
            const bool iv = i < i1;
#pragma unroll
            for (int t = 0; t < JT; ++t) a[t][q] = iv ? double(psi[i * m + jc[t]]) : 0.0;
#pragma unroll
            for (int kt = 0; kt < KT; ++kt) b[q][kt] = iv ? R[i * k + col[kt]] : 0.0;
        }
        step(a, b);
    }
    // FP64 16x16x4 results: lane l holds rows l / 16 + 4 r (here: Psi columns)
#pragma unroll
    for (int t = 0; t < JT; ++t)
#pragma unroll
        for (int kt = 0; kt < KT; ++kt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = PAIR ? j0 + 2 * (g + 4 * r) + t : j0 + 16 * t + g + 4 * r;
                if (j < m && cv[kt])
                    part[(int64_t(blockIdx.y) * m + j) * k + c0 + 16 * kt + cc] = acc[t][kt][r];
            }
}

// T[j][c] = sum over chunks of part, written zero-padded as an m_pad x ldt
// block (m_pad = m rounded up to 16, ldt = 16 KT) for the phase-2 MFMA.
// 64 outputs per work-group; its four waves each sum a quarter of the chunks
// (fixed order), then one wave adds the four partial sums.
__global__ __launch_bounds__(256) void k_sum_chunks(const double* __restrict__ part, int nchunk,
                                                    int m, int k, int c0, int kc, int m_pad,
                                                    int ldt, double* __restrict__ T) {
    __shared__ double sh[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t e = blockIdx.x * int64_t(64) + lane;
    const bool ev = e < int64_t(m_pad) * ldt;
    const int j = ev ? int(e / ldt) : 0, c = ev ? int(e % ldt) : 0;
    double s = 0.0;
    if (ev && j < m && c < kc && c0 + c < k)
        for (int q = w; q < nchunk; q += 4) s += part[(int64_t(q) * m + j) * k + c0 + c];
    sh[w][lane] = s;
    __syncthreads();
    // stored column-tile-interleaved: (j, 16 kt + rr) at (16 j + rr) ldt/16 + kt,
    // so a phase-2 lane finds its KT values of one row next to each other
    if (w == 0 && ev)
        T[(int64_t(j) * 16 + c % 16) * (ldt / 16) + c / 16] =
            (sh[0][lane] + sh[1][lane]) + (sh[2][lane] + sh[3][lane]);
}

// Phase 2: Z = D^-1 R - Psi T for columns [c0, c0 + 16 KT).  Each wave owns
// U 16-row tiles, so every T value it reads (T is zero-padded to
// m_pad x 16 KT, read without guards) feeds U MFMAs (U = 2 halves the T
// traffic from L2 once T has two or more column tiles); lane l reads
// Psi[row + l % 16][m0 + 4 (l / 16) + q], q = 0..3 (32 contiguous bytes; four
// lanes cover a 128-byte line of a row) for each tile, and the reduction
// index q pairs with the matching rows of T.  Whole 16-column blocks load
// without guards (a row past n reads row 0 and is never stored) and one
// block ahead of their MFMAs; a ragged last block loads under guards.
template <int KT, int U, bool VEC, typename PT>
__global__ __launch_bounds__(256) void k_apply_z(const PT* __restrict__ psi, int m,
                                                 const double* __restrict__ T, int ldt,
                                                 const double* __restrict__ dinv,
                                                 const double* __restrict__ R, int k, int c0,
                                                 int64_t n, double* __restrict__ Z) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = lane >> 4, rr = lane & 15;
    const int64_t row0 = (int64_t(blockIdx.x) * 4 + w) * 16 * U;
    if (row0 >= n) return;
    const PT* prow[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t row = row0 + 16 * u + rr;
        prow[u] = psi + (row < n ? row : 0) * m;
    }
    f64x4 acc[U][KT];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) acc[u][kt] = f64x4{0.0, 0.0, 0.0, 0.0};
    const int mfull = m & ~15;
    double a[U][4], t[4][KT];
    auto load_t = [&](int m0, double (&lt)[4][KT]) {   // T column-tile-interleaved
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double* tp = T + (int64_t(m0 + 4 * g + q) * 16 + rr) * KT;
            if (KT == 2) {   // T starts 16-byte aligned
                const double2 x = *reinterpret_cast<const double2*>(tp);
                lt[q][0] = x.x;
                lt[q][KT - 1] = x.y;
            } else {
#pragma unroll
                for (int kt = 0; kt < KT; ++kt) lt[q][kt] = tp[kt];
            }
        }
    };
    auto load = [&](int m0, double (&la)[U][4], double (&lt)[4][KT]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (VEC && sizeof(PT) == 8) {   // the lane's four entries: two 16-byte loads
                const double2* p2 = reinterpret_cast<const double2*>(prow[u] + m0 + 4 * g);
                const double2 x0 = p2[0], x1 = p2[1];
                la[u][0] = x0.x;
                la[u][1] = x0.y;
                la[u][2] = x1.x;
                la[u][3] = x1.y;
            } else if (VEC) {               // FP32: one 16-byte load
                const float4 x = *reinterpret_cast<const float4*>(prow[u] + m0 + 4 * g);
                la[u][0] = double(x.x);
                la[u][1] = double(x.y);
                la[u][2] = double(x.z);
                la[u][3] = double(x.w);
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) la[u][q] = double(prow[u][m0 + 4 * g + q]);
            }
        }
        load_t(m0, lt);
    };
    auto step = [&](const double (&la)[U][4], const double (&lt)[4][KT]) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int kt = 0; kt < KT; ++kt)
#pragma unroll
                for (int u = 0; u < U; ++u)
                    acc[u][kt] = __builtin_amdgcn_mfma_f64_16x16x4f64(la[u][q], lt[q][kt],
                                                                      acc[u][kt], 0, 0, 0);
    };
    // two register buffers in turn (see k_psit_r)
    double a2[U][4], t2[4][KT];
    if (mfull > 0) {
        const int last = mfull - 16;
        load(0, a, t);
        for (int m0 = 0; m0 < mfull; m0 += 32) {
            load(min(m0 + 16, last), a2, t2);
            step(a, t);
            if (m0 + 16 >= mfull) break;
            load(min(m0 + 32, last), a, t);
            step(a2, t2);
        }
    }
    if (mfull < m) {   // ragged last block: columns past m contribute zero
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int mm = mfull + 4 * g + q;
                a[u][q] = mm < m ? double(prow[u][mm]) : 0.0;
            }
        load_t(mfull, t);
        step(a, t);
    }
    // FP64 16x16x4 results: lane l holds rows l / 16 + 4 r of column l % 16
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int kt = 0; kt < KT; ++kt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = row0 + 16 * u + g + 4 * r;
                const int c = c0 + 16 * kt + rr;
                if (i < n && c < k)
                    Z[i * k + c] = (dinv ? dinv[i] * R[i * k + c] : Z[i * k + c]) - acc[u][kt][r];
            }
}

constexpr int kPsitJT = 2;   // Psi column tiles per wave in phase 1

template <int KC>
static void apply_chunk(pkm_ctx* ctx, const pkm_precond* pc, int k, int c0, const double* R,
                        double* Z) {
    hipStream_t s = ctx->stream;
    const int64_t n = pc->n;
    const int m = pc->m;
    const int mt = int(cdiv(m, AT));
    const int kc = std::min(KC, k - c0);
    constexpr int KT = (KC + 15) / 16;
    const int ldt = 16 * KT;
    const int m_pad = int(round_up(m, 16));
    // row chunks: ~1024 work-groups in phase 1, each at least 256 rows
    int64_t nchunk = std::max<int64_t>(1, std::min<int64_t>(cdiv(n, 256), 1024 / mt));
    int64_t rpc = round_up(cdiv(n, nchunk), 16);
    nchunk = cdiv(n, rpc);
    ctx->red2.ensure(sizeof(double) * (round_up(nchunk * int64_t(m) * k, 2) + int64_t(m_pad) * ldt));
    double* part = ctx->red2.as<double>();
    double* T = part + round_up(nchunk * int64_t(m) * k, 2);   // 16-byte aligned
    // phase 1: each wave takes kPsitJT 16-column tiles of Psi, so the R rows
    // it loads serve kPsitJT MFMA tiles
    const dim3 grid1((unsigned)cdiv(m, AT * kPsitJT), (unsigned)nchunk);
    const bool p32 = pc->psi32_on;
    const float* psi32 = pc->psi32.as<float>();
    const double* psi64 = pc->psi.as<double>();
    // m even: a lane's two adjacent Psi columns are one aligned 16- (8-) byte load
    if (kPsitJT == 2 && m % 2 == 0) {
        if (p32)
            k_psit_r<KT, kPsitJT, true><<<grid1, 256, 0, s>>>(psi32, m, R, k, c0, kc, n, rpc, part);
        else
            k_psit_r<KT, kPsitJT, true><<<grid1, 256, 0, s>>>(psi64, m, R, k, c0, kc, n, rpc, part);
    } else {
        if (p32)
            k_psit_r<KT, kPsitJT, false><<<grid1, 256, 0, s>>>(psi32, m, R, k, c0, kc, n, rpc, part);
        else
            k_psit_r<KT, kPsitJT, false><<<grid1, 256, 0, s>>>(psi64, m, R, k, c0, kc, n, rpc, part);
    }
    PKM_CHECK_LAUNCH();
    k_sum_chunks<<<cdiv(int64_t(m_pad) * ldt, 64), 256, 0, s>>>(part, int(nchunk), m, k, c0, kc,
                                                                m_pad, ldt, T);
    PKM_CHECK_LAUNCH();
    // PITC: Z already holds blockdiag(D^-1) R; the kernel subtracts Psi T
    const double* dv = pc->kind == PKM_PC_PITC ? nullptr : pc->dinv.as<double>();
    constexpr int U = KT >= 2 ? 2 : 1;
    // Psi rows are 16-byte aligned when m is even (FP64) or a multiple of 4
    // (FP32): vector loads in phase 2
    const unsigned grid2 = (unsigned)cdiv(n, 64 * U);
    if (p32) {
        if (m % 4 == 0)
            k_apply_z<KT, U, true><<<grid2, 256, 0, s>>>(psi32, m, T, ldt, dv, R, k, c0, n, Z);
        else
            k_apply_z<KT, U, false><<<grid2, 256, 0, s>>>(psi32, m, T, ldt, dv, R, k, c0, n, Z);
    } else {
        if (m % 2 == 0)
            k_apply_z<KT, U, true><<<grid2, 256, 0, s>>>(psi64, m, T, ldt, dv, R, k, c0, n, Z);
        else
            k_apply_z<KT, U, false><<<grid2, 256, 0, s>>>(psi64, m, T, ldt, dv, R, k, c0, n, Z);
    }
    PKM_CHECK_LAUNCH();
}

__global__ void k_round_f32(int64_t tot, const double* __restrict__ src, float* __restrict__ dst) {
    const int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e < tot) dst[e] = float(src[e]);   // round to nearest even
}

// Apply from the FP32 rounding of Psi (on) or from Psi itself (off).
void precond_psi_f32(pkm_ctx* ctx, pkm_precond* pc, bool on) {
    if (!on) {
        pc->psi32_on = false;
        pc->psi32.release();
        return;
    }
    const int64_t tot = pc->n * int64_t(pc->m);
    pc->psi32.ensure(sizeof(float) * tot);
    k_round_f32<<<cdiv(tot, 256), 256, 0, ctx->stream>>>(tot, pc->psi.as<double>(),
                                                         pc->psi32.as<float>());
    PKM_CHECK_LAUNCH();
    PKM_HIP(hipStreamSynchronize(ctx->stream));
    pc->psi32_on = true;
}

// Y <- Y - Phi Phi^T V (V, Y n x k; Phi the kept low-rank factor)
void precond_sub_lowrank(pkm_ctx* ctx, const pkm_precond* pc, int k, const double* V, double* Y) {
    const int64_t n = pc->n;
    const int m = pc->m;
    ctx->ws_pitc[0].ensure(sizeof(double) * int64_t(m) * k);
    double* T = ctx->ws_pitc[0].as<double>();
    const double* phi = pc->phi.as<double>();
    dgemm(ctx, true, false, m, k, n, 1.0, phi, m, V, k, 0.0, T, k);
    dgemm_large(ctx, false, false, n, k, m, -1.0, phi, m, T, k, 1.0, Y, k);
}

void precond_apply(pkm_ctx* ctx, const pkm_precond* pc, int k, const double* R, double* Z) {
    if (pc->kind == PKM_PC_PITC) {
        k_pitc_dinv<<<cdiv(pc->n * k, 256), 256, 0, ctx->stream>>>(pc->n, pc->block,
                                                                   pc->dblk.as<double>(), R, k, Z);
        PKM_CHECK_LAUNCH();
    }
    for (int c0 = 0; c0 < k;) {
        int rem = k - c0;
        if (rem > 17) { apply_chunk<33>(ctx, pc, k, c0, R, Z); c0 += 33; }
        else if (rem > 9) { apply_chunk<17>(ctx, pc, k, c0, R, Z); c0 += 17; }
        else if (rem > 4) { apply_chunk<9>(ctx, pc, k, c0, R, Z); c0 += 9; }
        else if (rem > 1) { apply_chunk<4>(ctx, pc, k, c0, R, Z); c0 += 4; }
        else { apply_chunk<1>(ctx, pc, k, c0, R, Z); c0 += 1; }
    }
}

}  // namespace pkm
