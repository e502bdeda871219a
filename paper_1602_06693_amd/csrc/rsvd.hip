// Randomised truncated SVD preconditioner (Section 3.2, partial SVD by
// random sampling) and the host symmetric eigensolver it needs.
//
//   Y = K Omega;  q times: Q = orth(Y), Y = K Q;  Q = orth(Y);
//   B = Q^T (K Q) = V diag(w) V^T;  Phi = Q V_r diag(w_r)^1/2 (r largest w,
//   negatives clipped to 0);  P = Phi Phi^T + lambda I (the factor form).
//
// The products with K run on the library's kernel products (the arithmetic
// the caller picks); orth is shifted Cholesky QR followed by two plain
// Cholesky QR passes in FP64 on the device; the l x l eigenproblem is solved
// on the host (Householder tridiagonalisation, then implicit symmetric QR
// steps with Wilkinson shifts, eigenvectors accumulated).

#include "pkm_internal.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <limits>
#include <memory>
#include <numeric>
#include <thread>
#include <vector>

namespace pkm {

void precond_setup(pkm_ctx* ctx, const pkm_problem* prob, int kind, int m, const int32_t* idx,
                   const double* Phi, double jitter, pkm_precond* pc, int aux);

// ---------------------------------------------------------------------------
// Host symmetric eigensolver: A (n x n, row-major, symmetric) -> eigenvalues
// w (descending) and eigenvectors as the columns of Z (row-major n x n).
// ---------------------------------------------------------------------------

// Householder reduction: A = Q T Q^T with T tridiagonal (diagonal d, first
// off-diagonal e, e[i] coupling i and i + 1).  Only the lower triangle of A
// is read and updated (A is overwritten); Qt = Q^T is formed afterwards by
// applying the reflectors to the identity in reverse order, each touching
// only its trailing block.
static void tridiagonalize(int n, std::vector<double>& Avec, std::vector<double>& d,
                           std::vector<double>& e, std::vector<double>& Qt) {
    double* __restrict__ A = Avec.data();
    d.assign(n, 0.0);
    e.assign(std::max(n - 1, 0), 0.0);
    std::vector<double> V(size_t(n) * n, 0.0);   // reflector k in row k, entries k + 1 .. n - 1
    std::vector<char> has(n, 0);
    std::vector<double> pbuf(n), wbuf(n);
    double* __restrict__ p = pbuf.data();
    double* __restrict__ w = wbuf.data();
    for (int k = 0; k + 2 < n; ++k) {
        d[k] = A[size_t(k) * n + k];
        const double x0 = A[size_t(k + 1) * n + k];
        double tail = 0.0;
        for (int i = k + 2; i < n; ++i) tail += A[size_t(i) * n + k] * A[size_t(i) * n + k];
        if (tail == 0.0) {   // column k is already tridiagonal
            e[k] = x0;
            continue;
        }
        const double alpha = -std::copysign(std::sqrt(x0 * x0 + tail), x0);
        double* __restrict__ v = &V[size_t(k) * n];
        // v = (x - alpha e_1) / |x - alpha e_1| on rows k + 1 .. n - 1
        v[k + 1] = x0 - alpha;
        for (int i = k + 2; i < n; ++i) v[i] = A[size_t(i) * n + k];
        const double sc = 1.0 / std::sqrt(v[k + 1] * v[k + 1] + tail);
        for (int i = k + 1; i < n; ++i) v[i] *= sc;
        has[k] = 1;
        e[k] = alpha;
        // p = A v over the trailing block, one pass over its lower triangle
        for (int i = k + 1; i < n; ++i) p[i] = 0.0;
        for (int i = k + 1; i < n; ++i) {
            const double* __restrict__ ai = &A[size_t(i) * n];
            const double vi = v[i];
            double s[4] = {0.0, 0.0, 0.0, 0.0};   // four partial sums: independent chains
            int j = k + 1;
            for (; j + 3 < i; j += 4)
                for (int u = 0; u < 4; ++u) {
                    s[u] += ai[j + u] * v[j + u];
                    p[j + u] += ai[j + u] * vi;
                }
            for (; j < i; ++j) {
                s[0] += ai[j] * v[j];
                p[j] += ai[j] * vi;
            }
            p[i] += ((s[0] + s[1]) + (s[2] + s[3])) + ai[i] * vi;
        }
        // trailing block <- H A H = A - v w^T - w v^T, w = 2 A v - 2 (v^T A v) v
        double vav = 0.0;
        for (int i = k + 1; i < n; ++i) vav += v[i] * p[i];
        for (int i = k + 1; i < n; ++i) w[i] = 2.0 * (p[i] - vav * v[i]);
        for (int i = k + 1; i < n; ++i) {
            double* __restrict__ ai = &A[size_t(i) * n];
            const double vi = v[i], wi = w[i];
            for (int j = k + 1; j <= i; ++j) ai[j] -= vi * w[j] + wi * v[j];
        }
    }
    for (int k = std::max(n - 2, 0); k < n; ++k) d[k] = A[size_t(k) * n + k];
    if (n >= 2) e[n - 2] = A[size_t(n - 1) * n + (n - 2)];
    // Qt = H_{n-3} ... H_0: right-multiply the identity by H_k for k
    // descending; H_k changes rows k + 1 .. n - 1 on columns k + 1 .. n - 1
    Qt.assign(size_t(n) * n, 0.0);
    for (int i = 0; i < n; ++i) Qt[size_t(i) * n + i] = 1.0;
    for (int k = n - 3; k >= 0; --k) {
        if (!has[k]) continue;
        const double* __restrict__ v = &V[size_t(k) * n];
        for (int i = k + 1; i < n; ++i) {
            double* __restrict__ qi = &Qt[size_t(i) * n];
            double s[4] = {0.0, 0.0, 0.0, 0.0};
            int j = k + 1;
            for (; j + 3 < n; j += 4)
                for (int u = 0; u < 4; ++u) s[u] += qi[j + u] * v[j + u];
            for (; j < n; ++j) s[0] += qi[j] * v[j];
            const double t = 2.0 * ((s[0] + s[1]) + (s[2] + s[3]));
            for (int j = k + 1; j < n; ++j) qi[j] -= t * v[j];
        }
    }
}

struct Rotation {
    int k;
    double c, s;
};

// Applies the rotations in order to Qt (n x n, row-major): rotation (k, c, s)
// replaces rows k, k + 1 by (c q_k + s q_k1, -s q_k + c q_k1).  Every column
// of Qt is rotated on its own, so blocks of 64 columns are handed to host
// threads (PKM_EIG_THREADS of them if set, else up to 16), each running the
// whole sequence over its block (which stays in cache); the rows are padded
// to 64-byte multiples so that no two threads write one cache line.
static void apply_rotations(int n, const std::vector<Rotation>& rots, std::vector<double>& Qt) {
    if (rots.empty()) return;
    constexpr int kCols = 64;
    const int ld = (n + 7) / 8 * 8;
    std::unique_ptr<double, void (*)(void*)> buf(
        static_cast<double*>(std::aligned_alloc(64, sizeof(double) * size_t(ld) * n)), std::free);
    PKM_REQUIRE(buf != nullptr, "host eigensolver: out of memory");
    double* P = buf.get();
    for (int i = 0; i < n; ++i)
        std::copy(&Qt[size_t(i) * n], &Qt[size_t(i) * n] + n, P + size_t(i) * ld);
    const int nblocks = (n + kCols - 1) / kCols;
    std::atomic<int> next{0};
    auto work = [&]() {
        for (int b; (b = next.fetch_add(1)) < nblocks;) {
            const int c0 = b * kCols, c1 = std::min(n, c0 + kCols);
            for (const Rotation& R : rots) {
                double* __restrict__ q0 = P + size_t(R.k) * ld;
                double* __restrict__ q1 = q0 + ld;
                const double c = R.c, s = R.s;
                for (int j = c0; j < c1; ++j) {
                    const double a = q0[j], b2 = q1[j];
                    q0[j] = c * a + s * b2;
                    q1[j] = -s * a + c * b2;
                }
            }
        }
    };
    int want = std::min(16, int(std::max(1u, std::thread::hardware_concurrency())));
    if (const char* env = std::getenv("PKM_EIG_THREADS")) want = std::max(1, std::atoi(env));
    const int nt = std::min({want, nblocks,
                             int(std::max<size_t>(1, rots.size() * size_t(n) / (size_t(1) << 22)))});
    std::vector<std::thread> pool;
    try {
        for (int t = 1; t < nt; ++t) pool.emplace_back(work);
    } catch (...) {   // fewer threads: the started ones and this one share the blocks
    }
    work();
    for (auto& th : pool) th.join();
    for (int i = 0; i < n; ++i)
        std::copy(P + size_t(i) * ld, P + size_t(i) * ld + n, &Qt[size_t(i) * n]);
}

// Implicit symmetric QR steps with Wilkinson shifts on the unreduced
// trailing block until every off-diagonal has deflated; each rotation R on
// (k, k + 1) (R [x; z] = [r; 0]) updates T <- R T R^T and Q <- Q R^T.  Q is
// held transposed (Qt, row c = column c of Q); the rotations are recorded
// while T is reduced and applied to Qt afterwards, in order.
static void tridiagonal_qr(int n, std::vector<double>& d, std::vector<double>& e,
                           std::vector<double>& Qt) {
    std::vector<Rotation> rots;
    rots.reserve(size_t(n) * n + 16);
    const double eps = std::numeric_limits<double>::epsilon();
    int hi = n - 1;
    int64_t steps = 0;
    while (hi > 0) {
        for (int i = 0; i < hi; ++i)
            if (std::fabs(e[i]) <= eps * (std::fabs(d[i]) + std::fabs(d[i + 1])) ||
                std::fabs(e[i]) < std::numeric_limits<double>::min())
                e[i] = 0.0;
        while (hi > 0 && e[hi - 1] == 0.0) --hi;
        if (hi == 0) break;
        int lo = hi - 1;
        while (lo > 0 && e[lo - 1] != 0.0) --lo;
        PKM_REQUIRE(++steps <= int64_t(60) * n + 60, "symmetric eigensolver did not converge");
        const double a = d[hi - 1], b = e[hi - 1], c = d[hi];
        const double delta = 0.5 * (a - c);
        const double den = delta + std::copysign(std::hypot(delta, b), delta == 0.0 ? 1.0 : delta);
        const double mu = den != 0.0 ? c - b * b / den : c - std::fabs(b);
        double x = d[lo] - mu, z = e[lo];
        for (int k = lo; k < hi; ++k) {
            const double r = std::hypot(x, z);
            const double cs = r == 0.0 ? 1.0 : x / r, sn = r == 0.0 ? 0.0 : z / r;
            if (k > lo) e[k - 1] = r;
            const double dk = d[k], dk1 = d[k + 1], ek = e[k];
            d[k] = cs * cs * dk + 2.0 * cs * sn * ek + sn * sn * dk1;
            d[k + 1] = sn * sn * dk - 2.0 * cs * sn * ek + cs * cs * dk1;
            e[k] = cs * sn * (dk1 - dk) + (cs * cs - sn * sn) * ek;
            if (k + 1 < hi) {   // the rotation pushes e[k + 1] into a bulge at (k, k + 2)
                const double f = e[k + 1];
                x = e[k];
                z = sn * f;
                e[k + 1] = cs * f;
            }
            rots.push_back(Rotation{k, cs, sn});
        }
    }
    apply_rotations(n, rots, Qt);
}

void sym_eig_host(int n, const double* A, double* w, double* Z) {
    std::vector<double> M(A, A + size_t(n) * n), d, e, Qt;
    for (int i = 0; i < n; ++i)   // symmetrise against rounding in the caller's matrix
        for (int j = 0; j < i; ++j) M[size_t(i) * n + j] = M[size_t(j) * n + i] =
            0.5 * (M[size_t(i) * n + j] + M[size_t(j) * n + i]);
    tridiagonalize(n, M, d, e, Qt);
    tridiagonal_qr(n, d, e, Qt);
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return d[x] > d[y]; });
    for (int c = 0; c < n; ++c) {
        w[c] = d[order[c]];
        for (int r = 0; r < n; ++r) Z[size_t(r) * n + c] = Qt[size_t(order[c]) * n + r];
    }
}

// ---------------------------------------------------------------------------
// Device orthonormalisation of Y (n x l, row-major) in place.
// ---------------------------------------------------------------------------

__global__ void k_add_diag_r(int64_t m, double* __restrict__ A, int64_t lda, double v) {
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i < m) A[i * lda + i] += v;
}

// One Cholesky QR pass: G = Y^T Y (+ shift I), G = L L^T, Y <- Y L^-T.
// Returns false (Y untouched) when G is not positive definite.
static bool cholqr_pass(pkm_ctx* ctx, int64_t n, int l, double* Y, double shift) {
    hipStream_t s = ctx->stream;
    ctx->ws_setup[0].ensure(sizeof(double) * int64_t(l) * l);
    ctx->ws_setup[1].ensure(sizeof(double) * int64_t(round_up(l, 64)) * 64);
    ctx->ws_setup[3].ensure(256);
    double* G = ctx->ws_setup[0].as<double>();
    double* winv = ctx->ws_setup[1].as<double>();
    int* dinfo = ctx->ws_setup[3].as<int>();
    dgemm(ctx, true, false, l, l, n, 1.0, Y, l, Y, l, 0.0, G, l);
    if (shift > 0.0) {
        k_add_diag_r<<<cdiv(l, 256), 256, 0, s>>>(l, G, l, shift);
        PKM_CHECK_LAUNCH();
    }
    dpotrf_lower(ctx, l, G, l, winv, dinfo);
    int hinfo = 0;
    PKM_HIP(hipMemcpyAsync(&hinfo, dinfo, sizeof(int), hipMemcpyDeviceToHost, s));
    PKM_HIP(hipStreamSynchronize(s));
    if (hinfo != 0) return false;
    dtrsm_right_lt(ctx, n, l, G, l, winv, Y, l);
    return true;
}

// Shifted Cholesky QR, then two plain passes (CholeskyQR3 with a shift in
// the first pass: the shift keeps the first factorisation defined for an
// ill-conditioned or rank-deficient Y, the plain passes restore
// orthonormality).  A later pass that finds G singular (a rank-deficient
// sketch) is shifted by l u: the sketch's null directions then stay of
// negligible norm, contributing nothing to Q B Q^T.
static void orthonormalize(pkm_ctx* ctx, int64_t n, int l, double* Y) {
    hipStream_t s = ctx->stream;
    ctx->ws_setup[0].ensure(sizeof(double) * int64_t(l) * l);
    double* G = ctx->ws_setup[0].as<double>();
    dgemm(ctx, true, false, l, l, n, 1.0, Y, l, Y, l, 0.0, G, l);
    std::vector<double> hg(size_t(l) * l);
    PKM_HIP(hipMemcpyAsync(hg.data(), G, sizeof(double) * hg.size(), hipMemcpyDeviceToHost, s));
    PKM_HIP(hipStreamSynchronize(s));
    double trace = 0.0;
    for (int i = 0; i < l; ++i) trace += hg[size_t(i) * l + i];
    PKM_REQUIRE(std::isfinite(trace), "randomised SVD: non-finite sketch");
    if (trace == 0.0) fail(PKM_ERR_BREAKDOWN, "randomised SVD: the sketch K Omega is zero");
    const double u = std::numeric_limits<double>::epsilon() / 2;
    const double shift = 11.0 * (double(n) * l + double(l) * (l + 1)) * u * trace;
    if (!cholqr_pass(ctx, n, l, Y, shift))
        fail(PKM_ERR_BREAKDOWN, "randomised SVD: shifted Cholesky QR failed");
    for (int pass = 0; pass < 2; ++pass)
        if (!cholqr_pass(ctx, n, l, Y, 0.0) && !cholqr_pass(ctx, n, l, Y, l * u))
            fail(PKM_ERR_BREAKDOWN, "randomised SVD: Cholesky QR failed");
}

// ---------------------------------------------------------------------------
// Setup
// ---------------------------------------------------------------------------

void precond_setup_rsvd(pkm_ctx* ctx, const pkm_problem* prob, int r, int l, const double* Omega,
                        int q, int prec, pkm_precond* pc) {
    const int64_t n = prob->n;
    hipStream_t s = ctx->stream;
    prepare(ctx, prob, true, prec != PKM_FP64);
    ctx->ws_pitc[0].ensure(sizeof(double) * n * l);
    ctx->ws_pitc[1].ensure(sizeof(double) * n * l);
    double* Y = ctx->ws_pitc[0].as<double>();
    double* W = ctx->ws_pitc[1].as<double>();
    mvm_shift(ctx, prec, l, Omega, Y, 0.0);          // Y = K Omega
    for (int it = 0; it < q; ++it) {
        orthonormalize(ctx, n, l, Y);
        mvm_shift(ctx, prec, l, Y, W, 0.0);          // W = K Q
        PKM_HIP(hipMemcpyAsync(Y, W, sizeof(double) * n * l, hipMemcpyDeviceToDevice, s));
    }
    orthonormalize(ctx, n, l, Y);                    // Q
    mvm_shift(ctx, prec, l, Y, W, 0.0);              // K Q
    ctx->ws_setup[0].ensure(sizeof(double) * int64_t(l) * l);
    double* B = ctx->ws_setup[0].as<double>();
    dgemm(ctx, true, false, l, l, n, 1.0, Y, l, W, l, 0.0, B, l);   // Q^T K Q
    std::vector<double> hb(size_t(l) * l), w(l), V(size_t(l) * l);
    PKM_HIP(hipMemcpyAsync(hb.data(), B, sizeof(double) * hb.size(), hipMemcpyDeviceToHost, s));
    PKM_HIP(hipStreamSynchronize(s));
    for (double v : hb) PKM_REQUIRE(std::isfinite(v), "randomised SVD: non-finite Q^T K Q");
    sym_eig_host(l, hb.data(), w.data(), V.data());
    // C = V_r diag(w_r)^1/2 (l x r), Phi = Q C (n x r)
    std::vector<double> hc(size_t(l) * r);
    for (int i = 0; i < l; ++i)
        for (int c = 0; c < r; ++c) hc[size_t(i) * r + c] = V[size_t(i) * l + c] * std::sqrt(std::max(w[c], 0.0));
    PKM_HIP(hipMemcpyAsync(B, hc.data(), sizeof(double) * hc.size(), hipMemcpyHostToDevice, s));
    dgemm_large(ctx, false, false, n, r, l, 1.0, Y, l, B, r, 0.0, W, r);
    PKM_HIP(hipStreamSynchronize(s));   // hc is pageable host memory
    precond_setup(ctx, prob, PKM_PC_LOWRANK, r, nullptr, W, 0.0, pc, 0);
}

}  // namespace pkm
