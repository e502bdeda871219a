// C ABI of libpkm: argument validation, context and object lifetime, and the
// translation of internal failures into status codes.  No exception crosses
// this boundary.

#include "pkm_internal.h"

#include <cmath>
#include <cstring>
#include <new>

namespace pkm {
void precond_setup(pkm_ctx* ctx, const pkm_problem* prob, int kind, int m, const int32_t* idx,
                   const double* Phi, double jitter, pkm_precond* pc, int aux);
void precond_sub_lowrank(pkm_ctx* ctx, const pkm_precond* pc, int k, const double* V, double* Y);
void precond_psi_f32(pkm_ctx* ctx, pkm_precond* pc, bool on);
void precond_setup_rsvd(pkm_ctx* ctx, const pkm_problem* prob, int r, int l, const double* Omega,
                        int q, int prec, pkm_precond* pc);
void sym_eig_host(int n, const double* A, double* w, double* Z);
void rademacher(pkm_ctx* ctx, int64_t n, int ncols, uint64_t seed, double* Z, int64_t ldz);
int laplace_mode(pkm_ctx* ctx, const pkm_problem* prob, const pkm_precond* base, const double* y,
                 const pkm_solve_opts* o, int max_newton, double tol, double* f, double* a,
                 pkm_laplace_info* info);
int laplace_grad(pkm_ctx* ctx, const pkm_problem* prob, const pkm_precond* base, const double* y,
                 const double* f, int N, const double* R, const pkm_solve_opts* o, double* grad,
                 int64_t* pcg_steps);
int laplace_predict(pkm_ctx* ctx, const pkm_problem* prob, const pkm_precond* base,
                    const double* y, const double* f, int64_t ns, const double* Xs,
                    const pkm_solve_opts* o, double* mean, double* var, double* prob_out);
int predict(pkm_ctx* ctx, const pkm_problem* prob, const pkm_precond* pc, const double* y,
            int64_t ns, const double* Xs, const pkm_solve_opts* o, double* mean, double* var,
            pkm_solve_info* info_mean, pkm_solve_info* info_var);
int solve_batched(pkm_ctx* ctx, int P, const pkm_problem* probs, const pkm_precond* const* pcs,
                  int k, const double* const* B, double* const* X, const pkm_solve_opts* o,
                  pkm_solve_info* infos);
void grad_pass(pkm_ctx* ctx, const pkm_problem* prob, int N, const double* AS,
               const double* YZ, double* grad);
void tune_cache_load(const char* path, int* accepted, int* rejected);
void mlp_create(pkm_ctx* ctx, int d_in, int hidden, int rank, const float* params_host,
                pkm_mlp* net);
void mlp_forward(pkm_ctx* ctx, pkm_mlp* net, int64_t n, const double* xs, double* U);
double mlp_loss_grad(pkm_ctx* ctx, pkm_mlp* net, int64_t n, const double* xs, int nz,
                     const double* Z, const double* KZ);
double mlp_train_step(pkm_ctx* ctx, pkm_mlp* net, int64_t n, const double* xs, int nz,
                      const double* Z, const double* KZ, double lr);
void mlp_release(pkm_mlp* net);
int64_t mlp_nparams(const pkm_mlp* net);
float* mlp_grad_ptr(pkm_mlp* net);
const float* mlp_param_ptr(const pkm_mlp* net);
int mlp_d_in(const pkm_mlp* net);
void mlp_state_get(pkm_ctx* ctx, const pkm_mlp* net, float* state, int64_t* t);
void mlp_state_set(pkm_ctx* ctx, pkm_mlp* net, const float* state, int64_t t);
}  // namespace pkm

using namespace pkm;

static thread_local std::string g_last_error = "no error";
static constexpr size_t PKM_PINNED_BYTES = 1 << 18;   // 3 batched status slots at P = 4096

template <class F>
static int guarded(pkm_ctx* ctx, F&& f) {
    try {
        if (ctx) PKM_HIP(hipSetDevice(ctx->device));
        int rc = f();
        if (rc != PKM_OK && ctx) g_last_error = ctx->err;
        return rc;
    } catch (const pkm::Error& e) {
        g_last_error = e.what();
        if (ctx) ctx->err = e.what();
        return e.code;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        if (ctx) ctx->err = g_last_error;
        return PKM_ERR_OOM;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        if (ctx) ctx->err = e.what();
        return PKM_ERR_HIP;
    } catch (...) {
        g_last_error = "unknown failure";
        if (ctx) ctx->err = g_last_error;
        return PKM_ERR_HIP;
    }
}

static void fill_opts(const pkm_solve_opts* in, pkm_solve_opts* o);

static void check_prec(int prec, int d) {
    PKM_REQUIRE(prec >= PKM_FP64 && prec <= PKM_I8X, "unknown precision");
    PKM_REQUIRE(prec != PKM_FP32 || d <= 34, "FP32 product supports d <= 34");
    PKM_REQUIRE(prec < PKM_BF16X1 || prec > PKM_F16X3 || d <= 36,
                "16-bit products support d <= 36");
    PKM_REQUIRE(prec != PKM_I8X || d <= 32, "int8-digit product supports d <= 32");
}

static void require_dev(const void* p, const char* what) {
    PKM_REQUIRE(p != nullptr, std::string(what) + " is NULL");
    PKM_REQUIRE((reinterpret_cast<uintptr_t>(p) & 7) == 0, std::string(what) + " must be 8-byte aligned");
}

extern "C" {

const char* pkm_version(void) { return "pkm 0.1 gfx950"; }

const char* pkm_last_error(const pkm_ctx* ctx) {
    if (ctx) return ctx->err.c_str();
    return g_last_error.c_str();
}

int pkm_create(pkm_ctx** out, int device, void* stream) {
    if (!out) {
        g_last_error = "out is NULL";
        return PKM_ERR_INVALID;
    }
    *out = nullptr;
    pkm_ctx* ctx = nullptr;
    int rc = guarded(nullptr, [&] {
        int count = 0;
        PKM_HIP(hipGetDeviceCount(&count));
        PKM_REQUIRE(device >= 0 && device < count, "device index out of range");
        PKM_HIP(hipSetDevice(device));
        noalloc_init(device);   // per-device address of the allocation-free scratch
        ctx = new pkm_ctx();
        ctx->device = device;
        ctx->stream = static_cast<hipStream_t>(stream);
        PKM_HIP(hipEventCreate(&ctx->ev0));
        PKM_HIP(hipEventCreate(&ctx->ev1));
        for (auto& e : ctx->poll_ev) PKM_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        PKM_HIP(hipHostMalloc(&ctx->pinned, PKM_PINNED_BYTES, hipHostMallocDefault));
        PKM_HIP(hipHostGetDevicePointer(&ctx->pinned_dev, ctx->pinned, 0));
        return PKM_OK;
    });
    if (rc != PKM_OK) {
        if (ctx) pkm_destroy(ctx);
        return rc;
    }
    *out = ctx;
    return PKM_OK;
}

int pkm_destroy(pkm_ctx* ctx) {
    if (!ctx) return PKM_OK;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    else (void)hipDeviceSynchronize();
    ctx->prep.xs64.release();
    ctx->prep.jside64.release();
    ctx->prep.iside64.release();
    ctx->prep.jside.release();
    ctx->prep.iside.release();
    ctx->prep.jsb.release();
    ctx->prep.isb.release();
    for (DevBuf* b : {&ctx->vbf, &ctx->v32, &ctx->y32, &ctx->v64pad, &ctx->y64pad, &ctx->red, &ctx->red2,
                      &ctx->scal, &ctx->state, &ctx->grad, &ctx->ws_split, &ctx->ws_tmp,
                      &ctx->colmax})
        b->release();
    for (auto& b : ctx->pcg) b.release();
    for (auto& b : ctx->ws_setup) b.release();
    for (auto& b : ctx->ws_pitc) b.release();
    for (auto& b : ctx->cross) b.release();
    for (auto& b : ctx->pred) b.release();
    for (auto& b : ctx->lap) b.release();
    for (auto& b : ctx->batch) b.release();
    for (auto& q : ctx->pending) {
        (void)hipEventDestroy(q.e0);
        (void)hipEventDestroy(q.e1);
    }
    for (auto& e : ctx->ev_pool) (void)hipEventDestroy(e);
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    for (auto& e : ctx->poll_ev)
        if (e) (void)hipEventDestroy(e);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    delete ctx;
    return PKM_OK;
}

int pkm_kernel_mvm(pkm_ctx* ctx, const pkm_problem* prob, int32_t k, int32_t prec,
                   const double* V, double* Y) {
    if (!ctx) return PKM_ERR_INVALID;
    return guarded(ctx, [&] {
        validate_problem(prob);
        PKM_REQUIRE(k >= 1 && k <= 4096, "k must be in [1, 4096]");
        check_prec(prec, prob->d);
        require_dev(V, "V");
        require_dev(Y, "Y");
        PKM_REQUIRE(V != Y, "Y may not alias V");
        prepare(ctx, prob, prec == PKM_FP64, prec != PKM_FP64 && prec != PKM_I8X);
        mvm(ctx, prec, k, V, Y);
        return PKM_OK;
    });
}

int pkm_kernel_mvm_noalloc(pkm_ctx* ctx, const pkm_problem* prob, int32_t k, int32_t prec,
                           const double* V, double* Y) {
    if (!ctx) return PKM_ERR_INVALID;
    return guarded(ctx, [&] {
        validate_problem(prob);
        PKM_REQUIRE(k >= 1 && k <= 4096, "k must be in [1, 4096]");
        if (prec != PKM_I8X)
            fail(PKM_ERR_UNSUPPORTED, "pkm_kernel_mvm_noalloc supports PKM_I8X only");
        check_prec(prec, prob->d);
        require_dev(V, "V");
        require_dev(Y, "Y");
        PKM_REQUIRE(V != Y, "Y may not alias V");
        mvm_i8_noalloc(ctx, prob, k, V, Y, prob->lambda);
        return PKM_OK;
    });
}

int pkm_kernel_mvm_shift(pkm_ctx* ctx, const pkm_problem* prob, int32_t k, int32_t prec,
                         double shift, const double* V, double* Y) {
    if (!ctx) return PKM_ERR_INVALID;
    return guarded(ctx, [&] {
        validate_problem(prob);
        PKM_REQUIRE(k >= 1 && k <= 4096, "k must be in [1, 4096]");
        PKM_REQUIRE(std::isfinite(shift) && shift >= 0.0, "shift must be >= 0");
        check_prec(prec, prob->d);
        require_dev(V, "V");
        require_dev(Y, "Y");
        PKM_REQUIRE(V != Y, "Y may not alias V");
        prepare(ctx, prob, prec == PKM_FP64, prec != PKM_FP64 && prec != PKM_I8X);
        mvm_shift(ctx, prec, k, V, Y, shift);
        return PKM_OK;
    });
}

int pkm_precond_setup(pkm_ctx* ctx, const pkm_problem* prob, int32_t kind, int32_t m,
                      const int32_t* idx, const double* Phi, double jitter, pkm_precond** out) {
    if (!ctx) return PKM_ERR_INVALID;
    if (out) *out = nullptr;
    pkm_precond* pc = nullptr;
    int rc = guarded(ctx, [&] {
        PKM_REQUIRE(out != nullptr, "out is NULL");
        validate_problem(prob);
        PKM_REQUIRE(kind >= PKM_PC_NYSTROM && kind <= PKM_PC_SKETCH,
                    "unknown preconditioner kind");
        PKM_REQUIRE(kind != PKM_PC_SKETCH || prob->d <= 34, "sketch preconditioner needs d <= 34");
        PKM_REQUIRE(m >= 1 && m <= 4096 && m <= prob->n, "m must be in [1, min(n, 4096)]");
        PKM_REQUIRE(std::isfinite(jitter) && jitter >= 0.0, "jitter must be >= 0");
        if (kind == PKM_PC_LOWRANK || kind == PKM_PC_SKETCH) require_dev(Phi, "Phi");
        else {
            PKM_REQUIRE(idx != nullptr, "idx is NULL");
            PKM_REQUIRE((reinterpret_cast<uintptr_t>(idx) & 3) == 0, "idx must be 4-byte aligned");
        }
        pc = new pkm_precond();
        precond_setup(ctx, prob, kind, m, idx, Phi, jitter, pc, 0);
        return PKM_OK;
    });
    if (rc != PKM_OK) {
        if (pc) pkm_precond_destroy(pc);
        return rc;
    }
    *out = pc;
    return PKM_OK;
}

int pkm_precond_setup_pitc(pkm_ctx* ctx, const pkm_problem* prob, int32_t m, const int32_t* idx,
                           int32_t block, double jitter, pkm_precond** out) {
    if (!ctx) return PKM_ERR_INVALID;
    if (out) *out = nullptr;
    pkm_precond* pc = nullptr;
    int rc = guarded(ctx, [&] {
        PKM_REQUIRE(out != nullptr, "out is NULL");
        validate_problem(prob);
        PKM_REQUIRE(m >= 1 && m <= 4096 && m <= prob->n, "m must be in [1, min(n, 4096)]");
        PKM_REQUIRE(block >= 1 && block <= 64, "block must be in [1, 64]");
        PKM_REQUIRE(std::isfinite(jitter) && jitter >= 0.0, "jitter must be >= 0");
        PKM_REQUIRE(idx != nullptr, "idx is NULL");
        PKM_REQUIRE((reinterpret_cast<uintptr_t>(idx) & 3) == 0, "idx must be 4-byte aligned");
        pc = new pkm_precond();
        precond_setup(ctx, prob, PKM_PC_PITC, m, idx, nullptr, jitter, pc, block);
        return PKM_OK;
    });
    if (rc != PKM_OK) {
        if (pc) pkm_precond_destroy(pc);
        return rc;
    }
    *out = pc;
    return PKM_OK;
}

int pkm_precond_setup_hybrid(pkm_ctx* ctx, const pkm_problem* prob, int32_t m,
                             const int32_t* idx, int32_t r, const double* U, double jitter,
                             pkm_precond** out) {
    if (!ctx) return PKM_ERR_INVALID;
    if (out) *out = nullptr;
    pkm_precond* pc = nullptr;
    int rc = guarded(ctx, [&] {
        PKM_REQUIRE(out != nullptr, "out is NULL");
        validate_problem(prob);
        PKM_REQUIRE(prob->d <= 34, "hybrid preconditioner needs d <= 34");
        PKM_REQUIRE(m >= 1 && r >= 1 && int64_t(m) + r <= 4096 && int64_t(m) + r <= prob->n,
                    "m, r >= 1 and m + r <= min(n, 4096)");
        PKM_REQUIRE(std::isfinite(jitter) && jitter >= 0.0, "jitter must be >= 0");
        PKM_REQUIRE(idx != nullptr, "idx is NULL");
        PKM_REQUIRE((reinterpret_cast<uintptr_t>(idx) & 3) == 0, "idx must be 4-byte aligned");
        require_dev(U, "U");
        pc = new pkm_precond();
        precond_setup(ctx, prob, PKM_PC_HYBRID, m, idx, U, jitter, pc, r);
        return PKM_OK;
    });
    if (rc != PKM_OK) {
        if (pc) pkm_precond_destroy(pc);
        return rc;
    }
    *out = pc;
    return PKM_OK;
}

int pkm_precond_setup_spectral(pkm_ctx* ctx, const pkm_problem* prob, int32_t m,
                               const double* W, pkm_precond** out) {
    if (!ctx) return PKM_ERR_INVALID;
    if (out) *out = nullptr;
    pkm_precond* pc = nullptr;
    int rc = guarded(ctx, [&] {
        PKM_REQUIRE(out != nullptr, "out is NULL");
        validate_problem(prob);
        PKM_REQUIRE(m >= 1 && m <= 2048, "m must be in [1, 2048] (2 m features)");
        require_dev(W, "W");
        pc = new pkm_precond();
        precond_setup(ctx, prob, PKM_PC_SPECTRAL, m, nullptr, W, 0.0, pc, 0);
        return PKM_OK;
    });
    if (rc != PKM_OK) {
        if (pc) pkm_precond_destroy(pc);
        return rc;
    }
    *out = pc;
    return PKM_OK;
}

int pkm_precond_setup_rsvd(pkm_ctx* ctx, const pkm_problem* prob, int32_t r, int32_t l,
                           const double* Omega, int32_t q, int32_t prec, pkm_precond** out) {
    if (!ctx) return PKM_ERR_INVALID;
    if (out) *out = nullptr;
    pkm_precond* pc = nullptr;
    int rc = guarded(ctx, [&] {
        PKM_REQUIRE(out != nullptr, "out is NULL");
        validate_problem(prob);
        PKM_REQUIRE(l >= 1 && l <= 1024 && l <= prob->n, "l must be in [1, min(n, 1024)]");
        PKM_REQUIRE(r >= 1 && r <= l, "r must be in [1, l]");
        PKM_REQUIRE(q >= 0 && q <= 8, "q must be in [0, 8]");
        check_prec(prec, prob->d);
        require_dev(Omega, "Omega");
        pc = new pkm_precond();
        precond_setup_rsvd(ctx, prob, r, l, Omega, q, prec, pc);
        return PKM_OK;
    });
    if (rc != PKM_OK) {
        if (pc) pkm_precond_destroy(pc);
        return rc;
    }
    *out = pc;
    return PKM_OK;
}

int pkm_rademacher(pkm_ctx* ctx, int64_t n, int32_t ncols, uint64_t seed, double* Z,
                   int64_t ldz) {
    if (!ctx) return PKM_ERR_INVALID;
    return guarded(ctx, [&] {
        PKM_REQUIRE(n >= 1 && n <= (int64_t(1) << 32), "n must be in [1, 2^32]");
        PKM_REQUIRE(ncols >= 1 && ncols <= 4096, "ncols must be in [1, 4096]");
        PKM_REQUIRE(ldz >= ncols, "ldz must be >= ncols");
        require_dev(Z, "Z");
        rademacher(ctx, n, ncols, seed, Z, ldz);
        return PKM_OK;
    });
}

int pkm_sym_eig(int32_t n, const double* A, double* w, double* Z) {
    if (n < 1 || n > 4096 || !A || !w || !Z) return PKM_ERR_INVALID;
    for (int64_t i = 0; i < int64_t(n) * n; ++i)
        if (!std::isfinite(A[i])) return PKM_ERR_INVALID;
    try {
        sym_eig_host(n, A, w, Z);
    } catch (...) {
        return PKM_ERR_BREAKDOWN;
    }
    return PKM_OK;
}

int pkm_cross_mvm(pkm_ctx* ctx, const pkm_problem* prob, int64_t n_star, const double* X_star,
                  int32_t k, const double* V, double* Y) {
    if (!ctx) return PKM_ERR_INVALID;
    return guarded(ctx, [&] {
        validate_problem(prob);
        PKM_REQUIRE(prob->d <= 34, "cross product needs d <= 34");
        PKM_REQUIRE(n_star >= 1 && n_star <= (int64_t(1) << 31) - 4096, "bad n_star");
        PKM_REQUIRE(k >= 1 && k <= 4096, "k must be in [1, 4096]");
        require_dev(X_star, "X_star");
        require_dev(V, "V");
        require_dev(Y, "Y");
        PKM_REQUIRE((reinterpret_cast<uintptr_t>(X_star) & 7) == 0, "X_star must be 8-byte aligned");
        cross_k64(ctx, prob, X_star, n_star, prob->X, prob->n, k, V, Y);
        return PKM_OK;
    });
}

int pkm_predict(pkm_ctx* ctx, const pkm_problem* prob, const pkm_precond* pc, const double* y,
                int64_t n_star, const double* X_star, const pkm_solve_opts* opts, double* mean,
                double* var, pkm_solve_info* info_mean, pkm_solve_info* info_var) {
    if (!ctx) return PKM_ERR_INVALID;
    return guarded(ctx, [&] {
        validate_problem(prob);
        PKM_REQUIRE(prob->d <= 34, "prediction needs d <= 34");
        PKM_REQUIRE(n_star >= 1 && (var == nullptr || n_star <= 256),
                    "n_star must be >= 1 (and <= 256 when variances are requested)");
        require_dev(y, "y");
        require_dev(X_star, "X_star");
        require_dev(mean, "mean");
        if (pc) {
            PKM_REQUIRE(pc->n == prob->n, "preconditioner built for another n");
            PKM_REQUIRE(pc->device == ctx->device, "preconditioner on another device");
        }
        pkm_solve_opts o;
        fill_opts(opts, &o);
        check_prec(o.prec, prob->d);
        if (var) require_dev(var, "var");
        return predict(ctx, prob, pc, y, n_star, X_star, &o, mean, var, info_mean, info_var);
    });
}

static void check_laplace_args(pkm_ctx* ctx, const pkm_problem* prob, const pkm_precond* pc,
                               const double* y) {
    validate_problem(prob);
    PKM_REQUIRE(prob->d <= 34, "Laplace approximation needs d <= 34");
    require_dev(y, "y");
    if (pc) {
        PKM_REQUIRE(pc->n == prob->n, "preconditioner built for another n");
        PKM_REQUIRE(pc->device == ctx->device, "preconditioner on another device");
        PKM_REQUIRE(pc->phi.p != nullptr, "preconditioner has no low-rank factor");
    }
}

int pkm_laplace_mode(pkm_ctx* ctx, const pkm_problem* prob, const pkm_precond* pc,
                     const double* y, const pkm_solve_opts* opts, int32_t max_newton,
                     double tol, double* f, double* a, pkm_laplace_info* info) {
    if (!ctx) return PKM_ERR_INVALID;
    return guarded(ctx, [&] {
        check_laplace_args(ctx, prob, pc, y);
        PKM_REQUIRE(max_newton >= 1 && std::isfinite(tol) && tol > 0.0, "bad Newton controls");
        require_dev(f, "f");
        require_dev(a, "a");
        pkm_solve_opts o;
        fill_opts(opts, &o);
        check_prec(o.prec, prob->d);
        return laplace_mode(ctx, prob, pc, y, &o, max_newton, tol, f, a, info);
    });
}

int pkm_laplace_grad(pkm_ctx* ctx, const pkm_problem* prob, const pkm_precond* pc,
                     const double* y, const double* f, int32_t N, const double* R,
                     const pkm_solve_opts* opts, double* grad, int64_t* pcg_steps) {
    if (!ctx) return PKM_ERR_INVALID;
    return guarded(ctx, [&] {
        check_laplace_args(ctx, prob, pc, y);
        PKM_REQUIRE(N >= 1 && N <= 255, "N must be in [1, 255]");
        require_dev(f, "f");
        require_dev(R, "R");
        PKM_REQUIRE(grad != nullptr, "grad is NULL");
        pkm_solve_opts o;
        fill_opts(opts, &o);
        check_prec(o.prec, prob->d);
        return laplace_grad(ctx, prob, pc, y, f, N, R, &o, grad, pcg_steps);
    });
}

int pkm_laplace_predict(pkm_ctx* ctx, const pkm_problem* prob, const pkm_precond* pc,
                        const double* y, const double* f, int64_t n_star,
                        const double* X_star, const pkm_solve_opts* opts, double* mean,
                        double* var, double* p) {
    if (!ctx) return PKM_ERR_INVALID;
    return guarded(ctx, [&] {
        check_laplace_args(ctx, prob, pc, y);
        PKM_REQUIRE(n_star >= 1 && n_star <= 256, "n_star must be in [1, 256]");
        require_dev(f, "f");
        require_dev(X_star, "X_star");
        require_dev(mean, "mean");
        require_dev(var, "var");
        require_dev(p, "p");
        pkm_solve_opts o;
        fill_opts(opts, &o);
        check_prec(o.prec, prob->d);
        return laplace_predict(ctx, prob, pc, y, f, n_star, X_star, &o, mean, var, p);
    });
}

int pkm_precond_sub_lowrank(pkm_ctx* ctx, const pkm_precond* pc, int32_t k, const double* V,
                            double* Y) {
    if (!ctx) return PKM_ERR_INVALID;
    return guarded(ctx, [&] {
        PKM_REQUIRE(pc != nullptr, "preconditioner is NULL");
        PKM_REQUIRE(pc->device == ctx->device, "preconditioner belongs to another device");
        PKM_REQUIRE(k >= 1 && k <= 4096, "k must be in [1, 4096]");
        require_dev(V, "V");
        require_dev(Y, "Y");
        PKM_REQUIRE(V != Y, "Y may not alias V");
        precond_sub_lowrank(ctx, pc, k, V, Y);
        return PKM_OK;
    });
}

int pkm_precond_apply(pkm_ctx* ctx, const pkm_precond* pc, int32_t k, const double* R,
                      double* Z) {
    if (!ctx) return PKM_ERR_INVALID;
    return guarded(ctx, [&] {
        PKM_REQUIRE(pc != nullptr, "preconditioner is NULL");
        PKM_REQUIRE(pc->device == ctx->device, "preconditioner belongs to another device");
        PKM_REQUIRE(k >= 1 && k <= 4096, "k must be in [1, 4096]");
        require_dev(R, "R");
        require_dev(Z, "Z");
        PKM_REQUIRE(R != Z, "Z may not alias R");
        precond_apply(ctx, pc, k, R, Z);
        return PKM_OK;
    });
}

int pkm_precond_diag(pkm_ctx* ctx, const pkm_precond* pc, double* D_host) {
    if (!ctx) return PKM_ERR_INVALID;
    return guarded(ctx, [&] {
        PKM_REQUIRE(pc != nullptr && D_host != nullptr, "NULL argument");
        std::vector<double> dinv(pc->n);
        PKM_HIP(hipMemcpyAsync(dinv.data(), pc->dinv.p, sizeof(double) * pc->n,
                               hipMemcpyDeviceToHost, ctx->stream));
        PKM_HIP(hipStreamSynchronize(ctx->stream));
        for (int64_t i = 0; i < pc->n; ++i) D_host[i] = 1.0 / dinv[i];
        return PKM_OK;
    });
}

int pkm_precond_psi_f32(pkm_ctx* ctx, pkm_precond* pc, int32_t on) {
    if (!ctx) return PKM_ERR_INVALID;
    return guarded(ctx, [&] {
        PKM_REQUIRE(pc != nullptr, "NULL argument");
        PKM_REQUIRE(pc->device == ctx->device, "preconditioner on another device");
        PKM_REQUIRE(on == 0 || on == 1, "on must be 0 or 1");
        precond_psi_f32(ctx, pc, on == 1);
        return PKM_OK;
    });
}

int pkm_precond_destroy(pkm_precond* pc) {
    if (!pc) return PKM_OK;
    (void)hipSetDevice(pc->device);
    (void)hipDeviceSynchronize();
    pc->psi.release();
    pc->psi32.release();
    pc->dinv.release();
    pc->dblk.release();
    pc->phi.release();
    delete pc;
    return PKM_OK;
}

static void fill_opts(const pkm_solve_opts* in, pkm_solve_opts* o) {
    *o = in ? *in : pkm_solve_opts{};
    if (o->tol == 0.0) o->tol = 1e-6;
    if (o->max_iter == 0) o->max_iter = 100000;
    if (o->reliable_every == 0) o->reliable_every = 25;
    if (o->check_every == 0) o->check_every = 1;
    if (!in) o->prec = PKM_FP32;
    PKM_REQUIRE(std::isfinite(o->tol) && o->tol > 0.0, "tol must be > 0");
    PKM_REQUIRE(o->max_iter >= 1, "max_iter must be >= 1");
    PKM_REQUIRE(o->prec >= PKM_FP64 && o->prec <= PKM_I8X, "unknown precision");
    PKM_REQUIRE(o->reliable_every != 0 && o->check_every >= 1,
                "periods must be >= 1 (a negative replacement period adapts)");
    PKM_REQUIRE(o->reliable_every >= -(1 << 24) && o->reliable_every <= (1 << 24),
                "replacement period must be at most 2^24 steps");
}

int pkm_solve(pkm_ctx* ctx, const pkm_problem* prob, const pkm_precond* pc, int32_t k,
              const double* B, double* X, const pkm_solve_opts* opts, pkm_solve_info* info) {
    if (!ctx) return PKM_ERR_INVALID;
    return guarded(ctx, [&] {
        validate_problem(prob);
        pkm_solve_opts o;
        fill_opts(opts, &o);
        PKM_REQUIRE(k >= 1 && k <= 256, "k must be in [1, 256]");
        check_prec(o.prec, prob->d);
        require_dev(B, "B");
        require_dev(X, "X");
        PKM_REQUIRE(B != X, "X may not alias B");
        if (pc) {
            PKM_REQUIRE(pc->n == prob->n, "preconditioner was built for another n");
            PKM_REQUIRE(pc->device == ctx->device, "preconditioner belongs to another device");
        }
        return solve(ctx, prob, pc, k, B, X, &o, info);
    });
}

int pkm_solve_batched(pkm_ctx* ctx, int32_t P, const pkm_problem* probs,
                      const pkm_precond* const* pcs, int32_t k, const double* const* B,
                      double* const* X, const pkm_solve_opts* opts, pkm_solve_info* infos) {
    if (!ctx) return PKM_ERR_INVALID;
    return guarded(ctx, [&] {
        PKM_REQUIRE(P >= 1 && P <= 4096, "P must be in [1, 4096]");
        PKM_REQUIRE(probs != nullptr && B != nullptr && X != nullptr, "NULL argument");
        pkm_solve_opts o;
        fill_opts(opts, &o);
        PKM_REQUIRE(o.prec == PKM_FP32 || o.prec == PKM_FP64 || o.prec == PKM_F16X3,
                    "batched solve supports FP32, F16X3 or FP64 products");
        PKM_REQUIRE(k >= 1 && k <= 33, "batched solve supports 1 <= k <= 33");
        for (int b = 0; b < P; ++b) {
            validate_problem(&probs[b]);
            check_prec(o.prec, probs[b].d);
            require_dev(B[b], "B[b]");
            require_dev(X[b], "X[b]");
            PKM_REQUIRE(B[b] != X[b], "X[b] may not alias B[b]");
            if (pcs && pcs[b]) {
                PKM_REQUIRE(pcs[b]->n == probs[b].n, "preconditioner built for another n");
                PKM_REQUIRE(pcs[b]->device == ctx->device, "preconditioner on another device");
                if (pcs[b]->kind == PKM_PC_PITC)
                    fail(PKM_ERR_UNSUPPORTED, "batched solve: PITC preconditioners are not supported");
            }
        }
        return solve_batched(ctx, P, probs, pcs, k, B, X, &o, infos);
    });
}

int pkm_tune_cache_load(const char* path, int32_t* accepted, int32_t* rejected) {
    return guarded(nullptr, [&] {
        PKM_REQUIRE(path != nullptr, "path is NULL");
        int a = 0, r = 0;
        tune_cache_load(path, &a, &r);
        if (accepted) *accepted = a;
        if (rejected) *rejected = r;
        return PKM_OK;
    });
}

int pkm_grad_pass(pkm_ctx* ctx, const pkm_problem* prob, int32_t N, const double* AS,
                  const double* YZ, double* grad_host) {
    if (!ctx) return PKM_ERR_INVALID;
    return guarded(ctx, [&] {
        validate_problem(prob);
        PKM_REQUIRE(prob->d <= 32, "gradient pass supports d <= 32");
        PKM_REQUIRE(N >= 0 && N <= 4095, "N must be in [0, 4095]");
        require_dev(AS, "AS");
        require_dev(YZ, "YZ");
        PKM_REQUIRE(grad_host != nullptr, "grad is NULL");
        grad_pass(ctx, prob, N, AS, YZ, grad_host);
        return PKM_OK;
    });
}

int pkm_lml_grad(pkm_ctx* ctx, const pkm_problem* prob, const pkm_precond* pc, const double* y,
                 int32_t N, const double* Z, const pkm_solve_opts* opts, double* grad_host,
                 double* sol, pkm_solve_info* info) {
    if (!ctx) return PKM_ERR_INVALID;
    return guarded(ctx, [&] {
        validate_problem(prob);
        PKM_REQUIRE(prob->d <= 32, "gradient pass supports d <= 32");
        PKM_REQUIRE(N >= 1 && N <= 255, "N must be in [1, 255]");
        require_dev(y, "y");
        require_dev(Z, "Z");
        PKM_REQUIRE(grad_host != nullptr, "grad is NULL");
        pkm_solve_opts o;
        fill_opts(opts, &o);
        check_prec(o.prec, prob->d);
        if (pc) {
            PKM_REQUIRE(pc->n == prob->n, "preconditioner was built for another n");
            PKM_REQUIRE(pc->device == ctx->device, "preconditioner belongs to another device");
        }
        // a warm start comes from the caller's sol (x0 of all 1 + N columns)
        PKM_REQUIRE(!o.use_x0 || sol != nullptr, "use_x0 needs sol to hold x0");
        if (sol) require_dev(sol, "sol");
        const int64_t n = prob->n;
        const int k = 1 + N;
        // [y, Z] and [alpha, Z] blocks (row-major n x k), solutions in S
        ctx->pcg[5].ensure(sizeof(double) * n * k);
        ctx->pcg[6].ensure(sizeof(double) * n * k);
        ctx->pcg[7].ensure(sizeof(double) * n * k);
        double* Bk = ctx->pcg[5].as<double>();
        double* S = ctx->pcg[6].as<double>();
        double* AZ = ctx->pcg[7].as<double>();
        hipStream_t s = ctx->stream;
        if (o.use_x0)
            PKM_HIP(hipMemcpyAsync(S, sol, sizeof(double) * n * k, hipMemcpyDeviceToDevice, s));
        PKM_HIP(hipMemcpy2DAsync(Bk, sizeof(double) * k, y, sizeof(double), sizeof(double), n,
                                 hipMemcpyDeviceToDevice, s));
        PKM_HIP(hipMemcpy2DAsync(Bk + 1, sizeof(double) * k, Z, sizeof(double) * N,
                                 sizeof(double) * N, n, hipMemcpyDeviceToDevice, s));
        int rc = solve(ctx, prob, pc, k, Bk, S, &o, info);
        if (rc < 0) return rc;
        PKM_HIP(hipMemcpyAsync(AZ, Bk, sizeof(double) * n * k, hipMemcpyDeviceToDevice, s));
        PKM_HIP(hipMemcpy2DAsync(AZ, sizeof(double) * k, S, sizeof(double) * k, sizeof(double), n,
                                 hipMemcpyDeviceToDevice, s));
        grad_pass(ctx, prob, N, S, AZ, grad_host);
        if (sol)
            PKM_HIP(hipMemcpyAsync(sol, S, sizeof(double) * n * k, hipMemcpyDeviceToDevice, s));
        PKM_HIP(hipStreamSynchronize(s));
        return rc;
    });
}

int pkm_mlp_create(pkm_ctx* ctx, int32_t d_in, int32_t hidden, int32_t rank,
                   const float* params, pkm_mlp** out) {
    if (!ctx) return PKM_ERR_INVALID;
    if (out) *out = nullptr;
    pkm_mlp* net = nullptr;
    int rc = guarded(ctx, [&] {
        PKM_REQUIRE(out != nullptr && params != nullptr, "NULL argument");
        net = new pkm_mlp();
        mlp_create(ctx, d_in, hidden, rank, params, net);
        return PKM_OK;
    });
    if (rc != PKM_OK) {
        if (net) pkm_mlp_destroy(net);
        return rc;
    }
    *out = net;
    return PKM_OK;
}

int pkm_mlp_destroy(pkm_mlp* net) {
    if (!net) return PKM_OK;
    (void)hipDeviceSynchronize();
    mlp_release(net);
    delete net;
    return PKM_OK;
}

int pkm_mlp_params(pkm_ctx* ctx, const pkm_mlp* net, float* params) {
    if (!ctx) return PKM_ERR_INVALID;
    return guarded(ctx, [&] {
        PKM_REQUIRE(net != nullptr && params != nullptr, "NULL argument");
        PKM_HIP(hipMemcpyAsync(params, mlp_param_ptr(net), sizeof(float) * mlp_nparams(net),
                               hipMemcpyDeviceToHost, ctx->stream));
        PKM_HIP(hipStreamSynchronize(ctx->stream));
        return PKM_OK;
    });
}

int pkm_mlp_nparams(const pkm_mlp* net, int64_t* nparams) {
    if (!net || !nparams) return PKM_ERR_INVALID;
    *nparams = mlp_nparams(net);
    return PKM_OK;
}

int pkm_mlp_state_get(pkm_ctx* ctx, const pkm_mlp* net, float* state, int64_t* t) {
    if (!ctx) return PKM_ERR_INVALID;
    return guarded(ctx, [&] {
        PKM_REQUIRE(net != nullptr && state != nullptr && t != nullptr, "NULL argument");
        PKM_REQUIRE(net->device == ctx->device, "network on another device");
        mlp_state_get(ctx, net, state, t);
        return PKM_OK;
    });
}

int pkm_mlp_state_set(pkm_ctx* ctx, pkm_mlp* net, const float* state, int64_t t) {
    if (!ctx) return PKM_ERR_INVALID;
    return guarded(ctx, [&] {
        PKM_REQUIRE(net != nullptr && state != nullptr, "NULL argument");
        PKM_REQUIRE(net->device == ctx->device, "network on another device");
        PKM_REQUIRE(t >= 0, "Adam step count must be >= 0");
        for (int64_t i = 0; i < 3 * mlp_nparams(net); ++i)
            PKM_REQUIRE(std::isfinite(state[i]), "state holds a non-finite value");
        mlp_state_set(ctx, net, state, t);
        return PKM_OK;
    });
}

static void mlp_check(pkm_ctx* ctx, const pkm_mlp* net, const pkm_problem* prob) {
    PKM_REQUIRE(net != nullptr, "network is NULL");
    validate_problem(prob);
    PKM_REQUIRE(prob->d == mlp_d_in(net), "problem dimension differs from the network input width");
    prepare(ctx, prob, true, false);
}

int pkm_mlp_forward(pkm_ctx* ctx, pkm_mlp* net, const pkm_problem* prob, double* U) {
    if (!ctx) return PKM_ERR_INVALID;
    return guarded(ctx, [&] {
        require_dev(U, "U");
        mlp_check(ctx, net, prob);
        mlp_forward(ctx, net, prob->n, ctx->P().xs64.as<double>(), U);
        return PKM_OK;
    });
}

int pkm_mlp_loss_grad(pkm_ctx* ctx, pkm_mlp* net, const pkm_problem* prob, int32_t nz,
                      const double* Z, const double* KZ, double* loss, float* grads) {
    if (!ctx) return PKM_ERR_INVALID;
    return guarded(ctx, [&] {
        PKM_REQUIRE(nz >= 1 && nz <= 4096, "nz must be in [1, 4096]");
        require_dev(Z, "Z");
        require_dev(KZ, "KZ");
        PKM_REQUIRE(loss != nullptr, "loss is NULL");
        mlp_check(ctx, net, prob);
        *loss = mlp_loss_grad(ctx, net, prob->n, ctx->P().xs64.as<double>(), nz, Z, KZ);
        if (grads) {
            PKM_HIP(hipMemcpyAsync(grads, mlp_grad_ptr(net), sizeof(float) * mlp_nparams(net),
                                   hipMemcpyDeviceToHost, ctx->stream));
            PKM_HIP(hipStreamSynchronize(ctx->stream));
        }
        return PKM_OK;
    });
}

int pkm_mlp_train_step(pkm_ctx* ctx, pkm_mlp* net, const pkm_problem* prob, int32_t nz,
                       const double* Z, const double* KZ, double lr, double* loss) {
    if (!ctx) return PKM_ERR_INVALID;
    return guarded(ctx, [&] {
        PKM_REQUIRE(nz >= 1 && nz <= 4096, "nz must be in [1, 4096]");
        PKM_REQUIRE(std::isfinite(lr) && lr > 0.0, "lr must be > 0");
        require_dev(Z, "Z");
        require_dev(KZ, "KZ");
        mlp_check(ctx, net, prob);
        double L = mlp_train_step(ctx, net, prob->n, ctx->P().xs64.as<double>(), nz, Z, KZ, lr);
        if (loss) *loss = L;
        return PKM_OK;
    });
}

int pkm_adagrad_step(int32_t p, double* theta, const double* g, double* G, double eta,
                     double eps) {
    if (p < 1 || !theta || !g || !G || !(eta > 0.0) || !(eps >= 0.0)) {
        g_last_error = "pkm_adagrad_step: invalid argument";
        return PKM_ERR_INVALID;
    }
    for (int i = 0; i < p; ++i)
        if (!std::isfinite(g[i])) {
            g_last_error = "pkm_adagrad_step: non-finite gradient";
            return PKM_ERR_INVALID;
        }
    for (int i = 0; i < p; ++i) {
        G[i] += g[i] * g[i];
        theta[i] += eta * g[i] / (std::sqrt(G[i]) + eps);
    }
    return PKM_OK;
}

int pkm_timing_enable(pkm_ctx* ctx, int32_t on) {
    if (!ctx) return PKM_ERR_INVALID;
    return guarded(ctx, [&] {
        if (!on) timing_flush(ctx);
        ctx->timing = on != 0;
        return PKM_OK;
    });
}

int pkm_mvm_stats(pkm_ctx* ctx, int32_t prec, int64_t* launches, double* ms, double* pairs,
                  double* flops) {
    if (!ctx || prec < PKM_FP64 || prec > PKM_I8X) return PKM_ERR_INVALID;
    const int rc = guarded(ctx, [&] {
        timing_flush(ctx);
        return PKM_OK;
    });
    if (rc != PKM_OK) return rc;
    const MvmStats& s = ctx->stats[prec];
    if (launches) *launches = s.launches;
    if (ms) *ms = s.ms;
    if (pairs) *pairs = s.pairs;
    if (flops) *flops = s.flops;
    return PKM_OK;
}

int pkm_mvm_stats_reset(pkm_ctx* ctx) {
    if (!ctx) return PKM_ERR_INVALID;
    const int rc = guarded(ctx, [&] {
        timing_flush(ctx);
        return PKM_OK;
    });
    for (auto& s : ctx->stats) s = MvmStats{};
    return rc;
}

}  // extern "C"

namespace pkm {

hipEvent_t timing_start(pkm_ctx* ctx) {
    hipEvent_t e;
    if (!ctx->ev_pool.empty()) {
        e = ctx->ev_pool.back();
        ctx->ev_pool.pop_back();
    } else {
        PKM_HIP(hipEventCreate(&e));
    }
    PKM_HIP(hipEventRecord(e, ctx->stream));
    return e;
}

void timing_stop(pkm_ctx* ctx, hipEvent_t e0, int prec, double pairs, double flops) {
    hipEvent_t e1;
    if (!ctx->ev_pool.empty()) {
        e1 = ctx->ev_pool.back();
        ctx->ev_pool.pop_back();
    } else {
        PKM_HIP(hipEventCreate(&e1));
    }
    PKM_HIP(hipEventRecord(e1, ctx->stream));
    ctx->pending.push_back(PendingTime{e0, e1, prec, pairs, flops});
    if (ctx->pending.size() >= 256) timing_flush(ctx);
}

void timing_flush(pkm_ctx* ctx) {
    if (ctx->pending.empty()) return;
    PKM_HIP(hipEventSynchronize(ctx->pending.back().e1));
    for (const PendingTime& q : ctx->pending) {
        float ms = 0.f;
        PKM_HIP(hipEventElapsedTime(&ms, q.e0, q.e1));
        MvmStats& st = ctx->stats[q.prec];
        st.launches += 1;
        st.ms += ms;
        st.pairs += q.pairs;
        st.flops += q.flops;
        ctx->ev_pool.push_back(q.e0);
        ctx->ev_pool.push_back(q.e1);
    }
    ctx->pending.clear();
}

}  // namespace pkm
