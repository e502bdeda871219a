// Internal declarations shared by the translation units of libpkm.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/pkm.h"

namespace pkm {

// Internal failures travel as exceptions and become status codes at the ABI.
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(int code, const std::string& msg) { throw Error(code, msg); }

#define PKM_HIP(expr)                                                              \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess)                                                      \
            ::pkm::fail(e_ == hipErrorOutOfMemory ? PKM_ERR_OOM : PKM_ERR_HIP,     \
                        std::string(#expr) + ": " + hipGetErrorString(e_));        \
    } while (0)

#define PKM_CHECK_LAUNCH() PKM_HIP(hipGetLastError())

#define PKM_REQUIRE(cond, msg)                                                     \
    do {                                                                           \
        if (!(cond)) ::pkm::fail(PKM_ERR_INVALID, msg);                            \
    } while (0)

__host__ __device__ inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }
__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Watches the largest FP64 true relative residual of a problem's live columns
// across residual replacements.  Refinement with a reduced-precision product
// converges only while the product's perturbation of K stays small against
// lambda; past that the true residual hovers around a floor (or grows).
// "Stalled": the largest true residual has not fallen below 0.7 of its best
// value at the current arithmetic for three replacements in a row and,
// unless it grew at the latest one, for at least kStallSteps PCG steps (the
// step floor keeps a short replacement period from reading the early pace
// of PCG as a stall; a growing residual needs no such patience).
constexpr int64_t kStallSteps = 150;
// True / recursive residual ratio up to which the recursion counts as
// faithful (adaptive replacement period below).
constexpr double kStallGap = 2.0;
// With the FP64-class int8-digit product and a faithful recursion, steps
// without a 0.7 improvement of the largest true residual before that counts
// as a stall (slow, non-monotone residuals of long solves are PCG's pace).
constexpr int64_t kI8PatienceSteps = 10 * kStallSteps;

// 2^S in FP64, table-driven (Tang's method, ACM TOMS 1989): S = N / 64 + r
// with N = rint(64 S) and |r| <= 1/128, so 2^S = 2^(N >> 6) * 2^((N & 63) / 64)
// * 2^r.  2^(j / 64) comes from a 64-entry table; 2^r = e^(r ln 2) is its
// Taylor polynomial of degree 6 (truncation below 3e-20 relative on
// |r| <= 1/128).  S below -1100 gives 0 (2^-1100 underflows); NaN stays NaN.
__device__ inline double exp2_tab(double S, const double* __restrict__ tab) {
    constexpr double L = 0.6931471805599453;   // ln 2
    constexpr double c1 = L, c2 = c1 * L / 2, c3 = c2 * L / 3, c4 = c3 * L / 4,
                     c5 = c4 * L / 5, c6 = c5 * L / 6;
    S = S < -1100.0 ? -1100.0 : S;
    const double y = rint(S * 64.0);
    const double r = fma(y, -1.0 / 64.0, S);   // exact
    const int N = int(y);
    double p = fma(c6, r, c5);
    p = fma(p, r, c4);
    p = fma(p, r, c3);
    p = fma(p, r, c2);
    p = fma(p, r, c1);
    p = fma(p, r, 1.0);
    return ldexp(tab[N & 63] * p, N >> 6);
}

struct StallMonitor {
    double best = 1e300, last = 1e300;
    int since = 0;
    int64_t step_best = 0;
    bool stalled(double max_true, int64_t step) {
        if (!(max_true > 0.0)) return false;   // nothing live
        const bool grew = !(max_true < last);
        last = max_true;
        if (max_true < 0.7 * best) {
            best = max_true;
            since = 0;
            step_best = step;
        } else {
            ++since;
        }
        return since >= 3 && (grew || step - step_best >= kStallSteps);
    }
    void reset() { best = last = 1e300; since = 0; step_best = 0; }
};

// Adaptive replacement period (a negative reliable_every): starts at
// base = -reliable_every and doubles (up to 8 base) after a replacement that
// finds the recursion faithful (largest true / recursive residual at most
// kStallGap) and the largest true residual below 0.7 of its value at the
// previous replacement -- progress that no stall test could fault -- and
// returns to base after any other, so that a slow or stalling solve keeps
// the base cadence of its stall test.
struct ReplacementPeriod {
    int base = 0, cur = 0;
    bool adaptive = false;
    double last = 1e300;
    explicit ReplacementPeriod(int every)
        : base(every < 0 ? -every : every), cur(every < 0 ? -every : every),
          adaptive(every < 0) {}
    void update(double max_gap, double max_true) {
        if (!adaptive) return;
        const bool fast = max_true < 0.7 * last;
        last = max_true;
        if (max_gap <= kStallGap && fast) cur = cur * 2 > 8 * base ? 8 * base : cur * 2;
        else cur = base;
    }
};

// Refinement mode: an inner PCG solve with the fast product ends once its
// recursive residual is this factor below the last FP64 true residual.
constexpr double kRefineEta = 1e-3;

// Largest augmented length (d + 2 rounded up to 4) of the FP64 MFMA product;
// larger d takes the FP64 vector-ALU product on direct differences.
constexpr int kAug64MaxD4 = 36;

// 16-bit products: columns per pass (seven 16-column tiles; wider blocks go
// in passes of this many), and the column-maxima slots of the FP16 scales.
// Measured at 65,536 points (FP16x3): one pass of seven tiles 2.23 ms at
// k = 100 against 2.84 ms as two passes; eight or nine tiles per pass ran
// slower than splitting (k = 144: 6.8 ms in one pass at four i-tiles per
// wave, 4.1 ms at two, 3.4 ms as two passes).
constexpr int kBf16MaxCols = 112;
constexpr int kColmaxSlots = 256;

// Grow-only device buffer.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    void ensure(size_t want) {
        if (want <= bytes) return;
        if (p) {
            // work queued earlier may still read the old allocation
            PKM_HIP(hipDeviceSynchronize());
            PKM_HIP(hipFree(p));
        }
        p = nullptr;
        bytes = 0;
        PKM_HIP(hipMalloc(&p, want));
        bytes = want;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

// Accumulated timing of kernel-product launches, per arithmetic.
struct MvmStats {
    int64_t launches = 0;
    double ms = 0.0, pairs = 0.0, flops = 0.0;
};

// A timed launch whose events are not read yet (timing never blocks the
// host per launch: the elapsed times are collected in batches).
struct PendingTime {
    hipEvent_t e0, e1;
    int prec;
    double pairs, flops;
};

// Prepared inputs of one problem (input preparation, done once per theta).
struct Prepared {
    int64_t n = 0, n_pad = 0;
    int d = 0;
    // FP64: X scaled by 1/l_r (direct differences need no centring)
    DevBuf xs64;            // n_pad x d
    // FP64 MFMA operands of the augmented contraction (same form and lane
    // order as the FP32 ones, d4 slots)
    DevBuf jside64, iside64;
    // FP32 MFMA operands of the augmented distance contraction.
    int d4 = 0;             // augmented length d + 2 rounded up to 4
    DevBuf jside;           // j-side operand tiles, MFMA lane order
    DevBuf iside;           // i-side operand rows, n_pad x d4
    // BF16 split operands of the same contraction (mvm_bf16.hip)
    int s6 = 0;             // 16x16x32 MFMAs per tile: ceil((6 d + 6) / 32)
    DevBuf jsb, isb;
    bool validb = false;
    // FP64 operands of the int8-digit product (mvm_i8.hip): the cross term
    // 2 xh_i . xh_j on FP64 MFMA (dq = d rounded up to 4 slots, 16x16x4 lane
    // order) and the row norms |xh_i|^2 (plain and, negated, in lane order)
    int dq = 0;
    DevBuf xi8, xj8, ni8, njl8;
    bool validi8 = false;
    double sigma2 = 1.0, lambda = 0.0;
    std::vector<double> ls;
    const double* X = nullptr;
    bool valid64 = false, valid32 = false;
};

}  // namespace pkm

struct pkm_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    bool timing = false;
    pkm::MvmStats stats[6];
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::vector<hipEvent_t> ev_pool;            // reusable timing events
    std::vector<pkm::PendingTime> pending;      // timed launches not yet read
    hipEvent_t poll_ev[2] = {nullptr, nullptr};   // lag-one status polls of the solvers
    pkm::Prepared prep;                 // the context's own prepared inputs
    pkm::Prepared* active = &prep;      // inputs the kernels use (batched solves switch it)
    pkm::Prepared& P() { return *active; }
    // scratch (grow-only), by purpose
    pkm::DevBuf vbf, v32, y32, v64pad, y64pad, red, red2, scal, state, pcg[8], grad;
    pkm::DevBuf ws_split, ws_tmp, ws_setup[4];
    pkm::DevBuf ws_pitc[2];             // PITC setup: block inverses, L_D^-1 Phi
    pkm::DevBuf cross[4];               // cross-product operands and prediction scratch
    pkm::DevBuf pred[3];                // predictive variance: I, K(X, X_*), solutions
    pkm::DevBuf lap[14];                // Laplace approximation vectors and blocks
    pkm::DevBuf batch[18];              // batched-solve workspace
    void* pinned = nullptr;   // pinned host staging area (PKM_PINNED_BYTES)
    void* pinned_dev = nullptr;   // the same memory as kernels address it
    pkm::DevBuf i8v, i8part;  // int8-digit products: packed V digits, FP64 split partials
    pkm::DevBuf i8cm;         // int8-digit products: column maxima and exponents
    pkm::DevBuf colmax;       // FP16x3 products: column maxima (128 slots)
    bool colmax_clean = false;   // colmax holds zeros (reset by k_finish32)
    const double* colmax_src = nullptr;   // colmax already holds this V's maxima
    int colmax_k = 0;                     // (the PCG direction update fills it)
};

struct pkm_precond {
    int kind = 0;
    int64_t n = 0;
    int m = 0;
    int device = 0;
    pkm::DevBuf psi;    // n x m FP64: P^-1 = D^-1 - psi psi^T
    pkm::DevBuf psi32;  // n x m FP32 rounding of psi, read by the apply when psi32_on
    bool psi32_on = false;
    pkm::DevBuf dinv;   // n FP64: 1 / diag(D)
    int block = 0;      // PITC: block size b; dblk holds blockdiag(D^-1), n x b
    pkm::DevBuf dblk;
    pkm::DevBuf phi;    // n x m FP64: the low-rank factor of P = D + phi phi^T
};

// Learned factor network (mlp.hip).
struct pkm_mlp {
    int device = 0;
    int d_in = 0, hidden = 0, rank = 0;
    int64_t nparams = 0;
    int64_t t = 0;                 // Adam step count
    pkm::DevBuf p32, m32, v32;     // master weights and Adam moments (FP32)
    pkm::DevBuf g32;               // gradient (FP32)
    pkm::DevBuf wpack;             // BF16 packed W1, W2, W3
    pkm::DevBuf act[8];            // activations and work buffers
    pkm::DevBuf ones, scal, split;
};

namespace pkm {

// ---- input preparation (prep.hip) ----
void prepare(pkm_ctx* ctx, const pkm_problem* prob, bool need64, bool need32);
void validate_problem(const pkm_problem* prob);

// ---- kernel products (mvm.hip) ----
// Y64 = (K + lambda I) V64 for row-major n x k FP64 blocks (device).
// prec: PKM_FP64 .. PKM_BF16X3.  Uses ctx->prep (must be prepared).
void mvm(pkm_ctx* ctx, int prec, int k, const double* V, double* Y);
// Y64 = (K + shift I) V64.
void mvm_shift(pkm_ctx* ctx, int prec, int k, const double* V, double* Y, double shift);
// K V only (no lambda term) in FP64, writing into Y (n x k FP64).
void mvm_k64(pkm_ctx* ctx, int k, const double* V, int ldv, double* Y, int ldy);
// FP32 product pipeline: pack V (n x k FP64, row-major) into MFMA tiles,
// run the fused kernel, return FP32 partials pointer and layout.
struct F32Out {
    const float* y;   // jsplit x n_pad x kp FP32 partial sums of K V
    int jsplit;
    int64_t stride;   // elements between consecutive split planes
    int kp;           // row stride in floats
    unsigned long long* zero_after = nullptr;   // 128 slots the finishing kernel clears
};
// Product timing (pkm_timing_enable): timing_start records a start event on
// the context stream and returns it; timing_stop records the end event and
// queues the launch; timing_flush waits for the last queued event and adds
// every queued launch to ctx->stats (also done when 256 are queued).
hipEvent_t timing_start(pkm_ctx* ctx);
void timing_stop(pkm_ctx* ctx, hipEvent_t e0, int prec, double pairs, double flops);
void timing_flush(pkm_ctx* ctx);
F32Out mvm_k32(pkm_ctx* ctx, int k, const double* V, int ldv);
// BF16 products (prec PKM_BF16X1 / PKM_BF16X3), same partial-sum layout.
F32Out mvm_kbf16(pkm_ctx* ctx, int prec, int k, const double* V, int ldv);
void prepare_bf16(pkm_ctx* ctx);
// FP64-class product on int8 matrix cores (prec PKM_I8X): Y = (K + shift I) V
// for row-major n x k FP64 blocks (leading dimensions ldv, ldy).
void mvm_i8(pkm_ctx* ctx, int k, const double* V, int ldv, double* Y, int ldy, double shift);
// Allocation-free PKM_I8X product (noalloc.hip): scratch in a static device
// array whose per-device address noalloc_init looks up (device current).
void noalloc_init(int device);
size_t noalloc_capacity();
void mvm_i8_noalloc(pkm_ctx* ctx, const pkm_problem* prob, int k, const double* V, double* Y,
                    double shift);

// ---- PCG (pcg.hip): K_y X = B, or B_laplace X = B when wscale (W^1/2) is given
int solve(pkm_ctx* ctx, const pkm_problem* prob, const pkm_precond* pc, int k, const double* B,
          double* X, const pkm_solve_opts* o, pkm_solve_info* info,
          const double* wscale = nullptr);

// ---- cross products (prediction) ----
void prepare_cross64(pkm_ctx* ctx, const pkm_problem* prob, const double* Xa, int64_t na,
                     const double* Xb, int64_t nb, double* jside, double* iside,
                     double* scratch);
// Y (na x k) = K(Xa, Xb) V, V nb x k; FP64 MFMA product, d + 2 <= 36.
void cross_k64(pkm_ctx* ctx, const pkm_problem* prob, const double* Xa, int64_t na,
               const double* Xb, int64_t nb, int k, const double* V, double* Y);

// ---- setup BLAS (blas64.hip) ----
// C[M x N] = alpha * op(A) op(B) + beta * C, FP64, row-major with leading
// dimensions.  op = transpose when the flag is set.  M < 65535 * 64.
void dgemm(pkm_ctx* ctx, bool ta, bool tb, int64_t M, int64_t N, int64_t K,
           double alpha, const double* A, int64_t lda, const double* B,
           int64_t ldb, double beta, double* C, int64_t ldc);
// Same, any M (row-chunked).
void dgemm_large(pkm_ctx* ctx, bool ta, bool tb, int64_t M, int64_t N, int64_t K,
                 double alpha, const double* A, int64_t lda, const double* B,
                 int64_t ldb, double beta, double* C, int64_t ldc);
// In-place lower Cholesky of an m x m FP64 matrix (row-major, lda); the
// upper triangle is zeroed.  winv (m x 64) receives the inverses of the
// 64 x 64 diagonal blocks.  *dev_info (device) = first failing pivot + 1.
void dpotrf_lower(pkm_ctx* ctx, int64_t m, double* A, int64_t lda, double* winv,
                  int* dev_info);
// B (n x m) <- B L^{-T}, L m x m lower (row-major), winv from dpotrf_lower.
void dtrsm_right_lt(pkm_ctx* ctx, int64_t n, int64_t m, const double* L,
                    int64_t ldl, const double* winv, double* B, int64_t ldb);

// ---- kernel blocks for setup (prep.hip) ----
// Out[p x q] = sigma2 exp(-1/2 |xa_i - xb_j|^2) for scaled FP64 rows.
void rbf_cross64(hipStream_t s, const double* xa, const int32_t* ia, int64_t p,
                 const double* xb, const int32_t* ib, int64_t q, int d,
                 double sigma2, double* out, int64_t ldo);

// ---- preconditioner apply (precond.hip) ----
void precond_apply(pkm_ctx* ctx, const pkm_precond* pc, int k, const double* R,
                   double* Z);

}  // namespace pkm
