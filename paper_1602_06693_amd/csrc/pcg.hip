// Preconditioned CG on a block of right-hand sides (Algorithm 1, textbook
// reading: alpha = r^T z / p^T K_y p, r <- r - alpha K_y p,
// beta = r'^T z' / r^T z, p <- z + beta p), every column an independent
// recurrence sharing one kernel product per step.
//
// All vectors (x, r, z, p, K_y p) are FP64, row-major n x k, resident on the
// device; per-column scalars live in a device array of ColState and are
// computed by single-work-group kernels, so the host only polls a two-word
// flag every few steps.  Dot products reduce in a fixed order (block
// partials, then one pass), so results are deterministic.
//
// A column whose recursive residual meets the tolerance is parked (it stops
// taking steps) until the next FP64 true-residual check, which runs as soon
// as every live column is parked.  A parked column whose true residual
// b - K_y x (x is always FP64) meets the tolerance is accepted; otherwise r
// is replaced by that true residual and the column resumes.  With FP32
// kernel products the recursive residual drifts from the true one, so the
// same replacement also runs every reliable_every steps.
//
// When the product's error is large against lambda, keeping p across a
// replacement stops helping: the search directions belong to the perturbed
// operator and the recursion stalls.  A column in refinement mode (eta > 0)
// therefore restarts (p = z) at every replacement and parks as soon as its
// recursive residual has dropped by the factor eta below the true residual
// of the last replacement: an outer iterative refinement in FP64 around
// short inner PCG solves with the fast product.

#include "pkm_internal.h"

#include <chrono>
#include <cmath>
#include <cstdlib>

namespace pkm {

struct ColState {
    double rz, alpha, beta, bnorm, rec, tru, rr;
    int32_t active, status;   // active: not yet accepted / failed
    int32_t parked;           // recursive residual met tol, awaiting check
    int32_t restart;          // next direction update takes beta = 0
    int64_t iters;
    double gap;               // true / recursive residual at the last replacement
    double ref;               // true relative residual at the last replacement
    double eta;               // refinement mode: inner solve target eta * ref (0: off)
};

struct Flags {
    int32_t live;      // active columns
    int32_t pending;   // active columns that are not parked
    int32_t broke;     // columns that broke down
    int32_t pad;
    double max_tru;    // largest FP64 true relative residual of active columns
    double max_gap;    // largest true / recursive residual ratio at the replacement
};

__device__ inline bool stepping(const ColState& s) { return s.active && !s.parked; }

constexpr int NRED = 256;   // blocks of a dot-product reduction

// Per-block partial sums of u o v over columns (k <= 256).  Thread t always
// sees column t % k because the thread stride is a multiple of k.
__global__ __launch_bounds__(256) void k_dot_part(const double* __restrict__ u,
                                                  const double* __restrict__ v, int64_t n,
                                                  int k, double* __restrict__ part) {
    __shared__ double sh[256];
    const int per = 256 / k;
    const int T = per * k;
    const int64_t tot = n * k;
    const int64_t chunk = round_up(cdiv(tot, NRED), k);
    const int64_t beg = blockIdx.x * chunk, end = min(tot, beg + chunk);
    double acc = 0.0;
    if (threadIdx.x < T) {
        // unrolled so that several iterations' loads are in flight at once;
        // the additions keep their order
#pragma unroll 4
        for (int64_t e = beg + threadIdx.x; e < end; e += T) acc = fma(u[e], v[e], acc);
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < k) {
        double s = 0.0;
        for (int q = 0; q < per; ++q) s += sh[threadIdx.x + q * k];
        part[blockIdx.x * k + threadIdx.x] = s;
    }
}

__device__ inline double sum_parts(const double* part, int k, int c) {
    double s = 0.0;
    for (int b = 0; b < NRED; ++b) s += part[b * k + c];
    return s;
}

// Column sums of the NRED x k partials by a whole 256-thread work-group:
// threads c, c + k, ... add every per-th partial of column c, then the per
// slices are added in a fixed order into out[c] (deterministic).  Every
// thread of the group must call it.
__device__ inline void sum_parts_wg(const double* __restrict__ part, int k, double* out) {
    __shared__ double sh[256];
    const int per = 256 / k;
    double acc = 0.0;
    if (int(threadIdx.x) < per * k)
        for (int b = threadIdx.x / k; b < NRED; b += per) acc += part[b * k + threadIdx.x % k];
    sh[threadIdx.x] = acc;
    __syncthreads();
    if (int(threadIdx.x) < k) {
        double s = 0.0;
        for (int q = 0; q < per; ++q) s += sh[threadIdx.x + q * k];
        out[threadIdx.x] = s;
    }
    __syncthreads();
}

// initial state: bnorm, rz = r^T z
__global__ void k_init_state(const double* __restrict__ pbb, const double* __restrict__ prz,
                             int k, ColState* __restrict__ st) {
    int c = threadIdx.x;
    if (c >= k) return;
    double bb = sum_parts(pbb, k, c);
    ColState s{};
    s.bnorm = sqrt(bb);
    s.rz = sum_parts(prz, k, c);
    s.active = bb > 0.0 ? 1 : 0;
    s.parked = 0;
    s.status = PKM_COL_CONVERGED;
    s.iters = 0;
    s.rec = bb > 0.0 ? 1.0 : 0.0;
    s.tru = s.rec;
    s.ref = s.rec;
    s.eta = 0.0;
    if (!isfinite(bb) || !isfinite(s.rz)) {   // NaN or Inf in b or x0
        s.active = 0;
        s.status = PKM_COL_BREAKDOWN;
    } else if (s.active && !(s.rz > 0.0)) {   // P not positive definite
        s.active = 0;
        s.status = PKM_COL_BREAKDOWN;
    }
    st[c] = s;
}

__global__ __launch_bounds__(256) void k_alpha(const double* __restrict__ ppap, int k,
                                               ColState* __restrict__ st) {
    __shared__ double sums[256];
    sum_parts_wg(ppap, k, sums);
    int c = threadIdx.x;
    if (c >= k) return;
    ColState s = st[c];
    if (stepping(s)) {
        double pap = sums[c];
        if (!(pap > 0.0) || !isfinite(pap)) {
            s.active = 0;
            s.status = PKM_COL_BREAKDOWN;
            s.alpha = 0.0;
        } else {
            s.alpha = s.rz / pap;
            s.iters += 1;
        }
    } else {
        s.alpha = 0.0;
    }
    st[c] = s;
}

// x += alpha p; r -= alpha Ap, and the partial sums of r o r over the updated
// r in the same pass: the grid, the element order and the additions are
// those of k_dot_part, so the partials equal k_dot_part(r, r) bit for bit
// (thread t keeps column t % k, whose alpha it reads once)
__global__ __launch_bounds__(256) void k_update_xr_rr(int64_t n, int k,
                                                      const ColState* __restrict__ st,
                                                      const double* __restrict__ p,
                                                      const double* __restrict__ Ap,
                                                      double* __restrict__ x,
                                                      double* __restrict__ r,
                                                      double* __restrict__ part) {
    __shared__ double sh[256];
    const int per = 256 / k;
    const int T = per * k;
    const int64_t tot = n * k;
    const int64_t chunk = round_up(cdiv(tot, NRED), k);
    const int64_t beg = blockIdx.x * chunk, end = min(tot, beg + chunk);
    double acc = 0.0;
    if (threadIdx.x < T) {
        const double a = st[threadIdx.x % k].alpha;
        if (a != 0.0) {
#pragma unroll 4
            for (int64_t e = beg + threadIdx.x; e < end; e += T) {
                x[e] = fma(a, p[e], x[e]);
                const double re = fma(-a, Ap[e], r[e]);
                r[e] = re;
                acc = fma(re, re, acc);
            }
        } else {
#pragma unroll 4
            for (int64_t e = beg + threadIdx.x; e < end; e += T) acc = fma(r[e], r[e], acc);
        }
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < k) {
        double s = 0.0;
        for (int q = 0; q < per; ++q) s += sh[threadIdx.x + q * k];
        part[blockIdx.x * k + threadIdx.x] = s;
    }
}

// recursive residual norms and flags; with `mirror` (pinned host memory as
// the device addresses it) the flags also go straight to the host
__global__ __launch_bounds__(256) void k_rr(const double* __restrict__ prr, int k, double tol,
                                            ColState* __restrict__ st, Flags* __restrict__ fl,
                                            Flags* __restrict__ mirror) {
    __shared__ int live, pending, broke;
    __shared__ double sums[256];
    if (threadIdx.x == 0) live = pending = broke = 0;
    sum_parts_wg(prr, k, sums);
    int c = threadIdx.x;
    if (c < k) {
        ColState s = st[c];
        double rr = sums[c];
        s.rr = rr;
        s.rec = s.bnorm > 0.0 ? sqrt(rr) / s.bnorm : 0.0;
        if (s.active && !isfinite(rr)) {
            s.active = 0;
            s.status = PKM_COL_BREAKDOWN;
        }
        if (stepping(s) && s.rec <= fmax(tol, s.eta * s.ref)) s.parked = 1;
        if (s.active) {
            atomicAdd(&live, 1);
            if (!s.parked) atomicAdd(&pending, 1);
        }
        if (s.status == PKM_COL_BREAKDOWN) atomicAdd(&broke, 1);
        st[c] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        fl->live = live;
        fl->pending = pending;
        fl->broke = broke;
        if (mirror) {
            mirror->live = live;
            mirror->pending = pending;
            mirror->broke = broke;
            mirror->max_tru = fl->max_tru;
            mirror->max_gap = fl->max_gap;
        }
    }
}

// r = b - Ax (true residual) for live columns
__global__ void k_true_res(int64_t n, int k, const ColState* __restrict__ st,
                           const double* __restrict__ b, const double* __restrict__ Ax,
                           double* __restrict__ r) {
    int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= n * k) return;
    int c = int(e % k);
    if (st[c].active) r[e] = b[e] - Ax[e];
}

// true residual norms (k_dot_part over the new r), acceptance
__global__ void k_true_final(const double* __restrict__ prr, int k, double tol,
                             ColState* __restrict__ st, Flags* __restrict__ fl) {
    __shared__ int live, broke;
    if (threadIdx.x == 0) live = broke = 0;
    __syncthreads();
    int c = threadIdx.x;
    if (c < k) {
        ColState s = st[c];
        if (s.active) {
            double rr = sum_parts(prr, k, c);
            s.rr = rr;
            const double rec_before = s.rec;
            s.tru = s.bnorm > 0.0 ? sqrt(rr) / s.bnorm : 0.0;
            s.gap = s.tru / fmax(rec_before, 1e-300);
            s.rec = s.tru;
            if (!isfinite(rr)) {
                s.active = 0;
                s.status = PKM_COL_BREAKDOWN;
            } else if (s.tru <= tol) {
                s.active = 0;
                s.status = PKM_COL_CONVERGED;
            } else {
                s.ref = s.tru;
                if (s.eta > 0.0) s.restart = 1;
            }
            s.parked = 0;
        }
        if (s.active) atomicAdd(&live, 1);
        if (s.status == PKM_COL_BREAKDOWN) atomicAdd(&broke, 1);
        st[c] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        fl->live = live;
        fl->pending = live;
        fl->broke = broke;
        double mx = 0.0, mg = 0.0;
        for (int q = 0; q < k; ++q)
            if (st[q].active) {
                mx = fmax(mx, st[q].tru);
                mg = fmax(mg, st[q].gap);
            }
        fl->max_tru = mx;
        fl->max_gap = mg;
    }
}

// columns that broke down resume (their residual is replaced next)
__global__ void k_reactivate(int k, ColState* __restrict__ st) {
    int c = threadIdx.x;
    if (c < k && st[c].status == PKM_COL_BREAKDOWN) {
        st[c].active = 1;
        st[c].status = PKM_COL_CONVERGED;
        st[c].parked = 0;
    }
}

// every active column restarts its directions at the next update (p = z)
// and takes refinement parameter eta (0: plain residual replacement)
__global__ void k_set_restart(int k, ColState* __restrict__ st, double eta) {
    int c = threadIdx.x;
    if (c < k && st[c].active) {
        st[c].restart = 1;
        st[c].eta = eta;
        st[c].ref = st[c].tru;
    }
}

// true residual of every column, for the report (no state change)
__global__ void k_report_true(const double* __restrict__ prr, int k, ColState* __restrict__ st) {
    int c = threadIdx.x;
    if (c >= k) return;
    double rr = sum_parts(prr, k, c);
    st[c].tru = st[c].bnorm > 0.0 ? sqrt(rr) / st[c].bnorm : 0.0;
}

__global__ __launch_bounds__(256) void k_beta(const double* __restrict__ prz, int k,
                                              ColState* __restrict__ st) {
    __shared__ double sums[256];
    sum_parts_wg(prz, k, sums);
    int c = threadIdx.x;
    if (c >= k) return;
    ColState s = st[c];
    if (stepping(s)) {
        double rz = sums[c];
        if (rz < 0.0 || !isfinite(rz)) {
            s.active = 0;
            s.status = PKM_COL_BREAKDOWN;
            s.beta = 0.0;
        } else {
            s.beta = (s.rz > 0.0 && !s.restart) ? rz / s.rz : 0.0;
            s.rz = rz;
            s.restart = 0;
        }
    } else {
        s.beta = 0.0;
    }
    st[c] = s;
}

// p = z + beta p (live columns)
__global__ void k_update_p(int64_t n, int k, const ColState* __restrict__ st,
                           const double* __restrict__ z, double* __restrict__ p) {
    int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= n * k) return;
    int c = int(e % k);
    if (stepping(st[c])) p[e] = fma(st[c].beta, p[e], z[e]);
}

// p = z + beta p (live columns) and, for FP16x3 products, the largest |p|
// of every column (updated or not) max-reduced into colmax (zeroed slots).
// Thread t takes column t % k of rows t / k, t / k + L, ... (L = 256 / k),
// so a pass reads consecutive addresses.
__global__ __launch_bounds__(256) void k_update_p_cm(int64_t n, int k,
                                                     const ColState* __restrict__ st,
                                                     const double* __restrict__ z,
                                                     double* __restrict__ p,
                                                     unsigned long long* __restrict__ colmax) {
    __shared__ unsigned long long sm[kColmaxSlots];
    const int t = threadIdx.x;
    if (t < k) sm[t] = 0ull;
    __syncthreads();
    const int L = 256 / k;
    if (t < L * k) {
        const int col = t % k;
        const bool stp = stepping(st[col]);
        const double beta = st[col].beta;
        double m = 0.0;
#pragma unroll 4
        for (int64_t row = int64_t(blockIdx.x) * L + t / k; row < n; row += int64_t(gridDim.x) * L) {
            const int64_t e = row * k + col;
            double v = p[e];
            if (stp) {
                v = fma(beta, v, z[e]);
                p[e] = v;
            }
            m = fmax(m, fabs(v));
        }
        atomicMax(&sm[col], (unsigned long long)__double_as_longlong(m));
    }
    __syncthreads();
    if (t < k) atomicMax(&colmax[t], sm[t]);
}

__global__ void k_mark_maxiter(int k, ColState* __restrict__ st) {
    int c = threadIdx.x;
    if (c < k && st[c].active) {
        st[c].active = 0;
        st[c].status = PKM_COL_MAX_ITER;
    }
}

__global__ void k_sub(int64_t tot, const double* __restrict__ a, const double* __restrict__ b,
                      double* __restrict__ out) {
    int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e < tot) out[e] = a[e] - b[e];
}

// out = w o V (rows scaled by w), n x k
__global__ void k_scale_rows(int64_t n, int k, const double* __restrict__ w,
                             const double* __restrict__ V, double* __restrict__ out) {
    int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= n * k) return;
    out[e] = w[e / k] * V[e];
}

// Y = w o Y + shift V
__global__ void k_scale_rows_add(int64_t n, int k, const double* __restrict__ w,
                                 const double* __restrict__ V, double shift,
                                 double* __restrict__ Y) {
    int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= n * k) return;
    Y[e] = fma(w[e / k], Y[e], shift * V[e]);
}

static void dot_part(pkm_ctx* ctx, const double* u, const double* v, int64_t n, int k,
                     double* part) {
    k_dot_part<<<NRED, 256, 0, ctx->stream>>>(u, v, n, k, part);
    PKM_CHECK_LAUNCH();
}

// The system matrix is K_y = K + lambda I, or, when wscale is given (device
// n), the Laplace matrix B = I + diag(w) K diag(w) (w = W^1/2).
int solve(pkm_ctx* ctx, const pkm_problem* prob, const pkm_precond* pc, int k, const double* B,
          double* X, const pkm_solve_opts* o, pkm_solve_info* info, const double* wscale) {
    const int64_t n = prob->n;
    hipStream_t s = ctx->stream;
    const int prec = o->prec;
    prepare(ctx, prob, true, prec != PKM_FP64 && prec != PKM_I8X);
    auto t_start = std::chrono::steady_clock::now();

    const size_t vec = sizeof(double) * n * k;
    for (int i = 0; i < 5; ++i) ctx->pcg[i].ensure(vec);
    double* r = ctx->pcg[0].as<double>();
    double* z = ctx->pcg[1].as<double>();
    double* p = ctx->pcg[2].as<double>();
    double* Ap = ctx->pcg[3].as<double>();
    double* tmp = ctx->pcg[4].as<double>();
    ctx->red.ensure(sizeof(double) * NRED * k * 2);
    double* partA = ctx->red.as<double>();
    double* partB = partA + NRED * k;
    ctx->state.ensure(sizeof(ColState) * k + sizeof(Flags) + 64);
    ColState* st = ctx->state.as<ColState>();
    Flags* fl = reinterpret_cast<Flags*>(st + k);
    Flags* hfl = static_cast<Flags*>(ctx->pinned);
    const int64_t tot = n * k;
    const unsigned gb = unsigned(cdiv(tot, 256));
    if (wscale) ctx->pcg[5].ensure(vec);
    // Y = A V for the system matrix A (see above), product arithmetic `pr`
    auto apply_A = [&](int pr, const double* V, double* Y) {
        if (!wscale) {
            mvm(ctx, pr, k, V, Y);
            return;
        }
        double* sv = ctx->pcg[5].as<double>();
        k_scale_rows<<<gb, 256, 0, s>>>(n, k, wscale, V, sv);
        PKM_CHECK_LAUNCH();
        mvm_shift(ctx, pr, k, sv, Y, 0.0);
        k_scale_rows_add<<<gb, 256, 0, s>>>(n, k, wscale, V, 1.0, Y);
        PKM_CHECK_LAUNCH();
    };

    auto precond = [&](const double* R, double* Zo) {
        if (pc) precond_apply(ctx, pc, k, R, Zo);
        else PKM_HIP(hipMemcpyAsync(Zo, R, vec, hipMemcpyDeviceToDevice, s));
    };
    // Lag-one polling: the flags of a step go to pinned slot 1 or 2 behind
    // that step's kernels, and the host reads the previous poll's slot while
    // the current step runs, so the stream never drains between steps.  The
    // conditions read that way only ever hold from then on (no live column,
    // no stepping column, a breakdown) until the host itself acts on them, so
    // a stale copy costs at most one idle step.  In the loop k_rr writes the
    // slot itself (host-mapped store, no copy launch).
    int lag_slot = -1;   // slot whose copy is still unread (-1: none)
    Flags* hfl_dev = static_cast<Flags*>(ctx->pinned_dev);
    auto poll = [&]() {
        PKM_HIP(hipMemcpyAsync(hfl, fl, sizeof(Flags), hipMemcpyDeviceToHost, s));
        PKM_HIP(hipStreamSynchronize(s));
        lag_slot = -1;   // in-flight copies completed and are superseded
        return *hfl;
    };
    auto next_slot = [&]() { return lag_slot == 1 ? 2 : 1; };
    // `written`: the slot already holds this step's flags (k_rr's mirror)
    auto poll_lagged = [&](Flags& out, bool written) {
        const int slot = next_slot();
        if (!written)
            PKM_HIP(hipMemcpyAsync(hfl + slot, fl, sizeof(Flags), hipMemcpyDeviceToHost, s));
        PKM_HIP(hipEventRecord(ctx->poll_ev[slot - 1], s));
        const int prev = lag_slot;
        lag_slot = slot;
        if (prev < 0) return false;
        PKM_HIP(hipEventSynchronize(ctx->poll_ev[prev - 1]));
        out = hfl[prev];
        return true;
    };
    int64_t true_count = 0;
    auto true_residual = [&]() {   // r <- b - K_y x in FP64 for live columns
        apply_A(PKM_FP64, X, tmp);
        k_true_res<<<gb, 256, 0, s>>>(n, k, st, B, tmp, r);
        PKM_CHECK_LAUNCH();
        dot_part(ctx, r, r, n, k, partA);
        k_true_final<<<1, 256, 0, s>>>(partA, k, o->tol, st, fl);
        PKM_CHECK_LAUNCH();
        ++true_count;
    };

    // r0 = b - K_y x0, z0 = P^-1 r0, p0 = z0
    if (o->use_x0) {
        apply_A(PKM_FP64, X, tmp);
        k_sub<<<gb, 256, 0, s>>>(tot, B, tmp, r);
        PKM_CHECK_LAUNCH();
        ++true_count;
    } else {
        PKM_HIP(hipMemsetAsync(X, 0, vec, s));
        PKM_HIP(hipMemcpyAsync(r, B, vec, hipMemcpyDeviceToDevice, s));
    }
    precond(r, z);
    PKM_HIP(hipMemcpyAsync(p, z, vec, hipMemcpyDeviceToDevice, s));
    dot_part(ctx, B, B, n, k, partA);
    dot_part(ctx, r, z, n, k, partB);
    k_init_state<<<1, 256, 0, s>>>(partA, partB, k, st);
    PKM_CHECK_LAUNCH();
    // x0 may already satisfy the tolerance
    dot_part(ctx, r, r, n, k, partA);
    k_rr<<<1, 256, 0, s>>>(partA, k, o->tol, st, fl, nullptr);
    PKM_CHECK_LAUNCH();
    Flags f = poll();
    if (f.live > 0 && f.pending == 0) {
        true_residual();
        f = poll();
    }

    // Reduced-precision products carry a perturbation of K.  When the true
    // residual stalls, the columns first switch to refinement mode (restart
    // at every replacement, short inner solves); if it stalls again, or a
    // column breaks down, the product arithmetic is raised (16-bit -> FP32 ->
    // FP64), broken columns resume, and every column restarts from its FP64
    // true residual in plain replacement mode.  An FP32 solve that stalled
    // with a bounded iterate goes on with the int8-digit product instead of
    // FP64 (it certifies where FP32-class products stall, at a fraction of
    // the FP64 cost); after a divergence or breakdown the iterate may be
    // huge, and the fixed-point product's error (2^-30 of each column's
    // largest entry) is then too coarse, so FP64 it is.  The int8-digit
    // product is FP64-class: with it a slow true residual counts as a stall
    // only while the recursion has lost track of it (true / recursive above
    // kStallGap) -- a faithful recursion that converges slowly is PCG's own
    // pace, which FP64 products would not change -- or after
    // kI8PatienceSteps steps without a 0.7 improvement.
    int cur = prec;
    bool refining = false, ever_refined = false;
    // PKM_VERBOSE set reports every FP64 replacement on stderr (long solves)
    // read per call: a caller may switch progress reports on for one long solve
    const bool verbose = std::getenv("PKM_VERBOSE") != nullptr;
    StallMonitor mon;
    int64_t it = 0;   // PCG steps so far
    // bounded: the escalation follows a stall (not a divergence or breakdown)
    auto escalate = [&](bool bounded) {
        if (cur == PKM_BF16X1 || cur == PKM_BF16X3 || cur == PKM_F16X3) cur = PKM_FP32;
        else if (cur == PKM_FP32 && bounded && prob->d <= 32) cur = PKM_I8X;
        else cur = PKM_FP64;
        refining = false;
        k_reactivate<<<1, 256, 0, s>>>(k, st);
        PKM_CHECK_LAUNCH();
        true_residual();
        k_set_restart<<<1, 256, 0, s>>>(k, st, 0.0);
        PKM_CHECK_LAUNCH();
        mon.reset();
        return poll();
    };
    auto assess = [&](Flags fl_now) {   // after an FP64 true residual
        if (cur == PKM_FP64) return fl_now;
        if (fl_now.broke > 0) return escalate(false);
        // a true residual above the right-hand side itself while the
        // recursion believes it is 100 times smaller: the product is far
        // too coarse for lambda (PCG residual norms alone may rise early on)
        if (fl_now.live > 0 && fl_now.max_tru > 1.0 && fl_now.max_gap > 100.0)
            return escalate(false);
        const bool stalled = fl_now.live > 0 && mon.stalled(fl_now.max_tru, it);
        if (stalled && (cur != PKM_I8X || fl_now.max_gap > kStallGap ||
                        it - mon.step_best >= kI8PatienceSteps)) {
            if (refining) return escalate(true);
            refining = true;
            ever_refined = true;
            k_set_restart<<<1, 256, 0, s>>>(k, st, kRefineEta);
            PKM_CHECK_LAUNCH();
            mon.reset();
        }
        return fl_now;
    };

    const int check = o->check_every;
    ReplacementPeriod period(o->reliable_every);
    int64_t last_true = 0;   // step of the last FP64 replacement
    while (f.live > 0 && it < o->max_iter) {
        apply_A(cur, p, Ap);
        dot_part(ctx, p, Ap, n, k, partA);
        k_alpha<<<1, 256, 0, s>>>(partA, k, st);
        PKM_CHECK_LAUNCH();
        k_update_xr_rr<<<NRED, 256, 0, s>>>(n, k, st, p, Ap, X, r, partA);
        PKM_CHECK_LAUNCH();
        // a lagged poll after this step takes its flags from k_rr's mirror
        const int64_t it1 = it + 1;
        const bool lag_poll = !(cur != PKM_FP64 && it1 - last_true >= period.cur) &&
                              it1 % check == 0 && it1 != o->max_iter;
        k_rr<<<1, 256, 0, s>>>(partA, k, o->tol, st, fl,
                               lag_poll ? hfl_dev + next_slot() : nullptr);
        PKM_CHECK_LAUNCH();
        ++it;
        bool do_true = cur != PKM_FP64 && it - last_true >= period.cur;
        if (!do_true && (it % check == 0 || it == o->max_iter)) {
            Flags lagged;
            if (it == o->max_iter) {
                f = poll();
            } else if (poll_lagged(lagged, lag_poll)) {
                f = lagged;
            } else {
                f.broke = 0;   // first poll of the loop: nothing read yet
                f.pending = 1;
            }
            if (f.broke > 0 && cur != PKM_FP64) {
                f = escalate(false);
            } else {
                if (f.live == 0) break;
                if (f.pending == 0) do_true = true;
            }
        }
        if (do_true) {
            true_residual();
            last_true = it;
            f = assess(poll());
            period.update(f.max_gap, f.max_tru);
            if (verbose)
                std::fprintf(stderr, "pkm_solve: step %lld, product %d%s, live columns %d, "
                             "largest true relative residual %.3e, true/recursive %.3g\n",
                             (long long)it, cur, refining ? " (refinement mode)" : "", f.live,
                             f.max_tru, f.max_gap);
            if (f.live == 0) break;
        }
        if (verbose && cur == PKM_FP64 && it % 25 == 0)
            std::fprintf(stderr, "pkm_solve: step %lld, FP64 products, live columns %d\n",
                         (long long)it, f.live);
        if (it == o->max_iter) break;
        precond(r, z);
        dot_part(ctx, r, z, n, k, partB);
        k_beta<<<1, 256, 0, s>>>(partB, k, st);
        PKM_CHECK_LAUNCH();
        if (cur == PKM_F16X3 && !wscale && k <= kBf16MaxCols && ctx->colmax_clean &&
            ctx->colmax.bytes >= kColmaxSlots * sizeof(unsigned long long)) {
            // the next product's column maxima come with the update (the
            // slots are clean: the last product's k_finish32 cleared them)
            const int64_t blocks = std::min<int64_t>(512, cdiv(n, 256 / k));
            k_update_p_cm<<<(unsigned)blocks, 256, 0, s>>>(n, k, st, z, p,
                                                           ctx->colmax.as<unsigned long long>());
            ctx->colmax_clean = false;
            ctx->colmax_src = p;
            ctx->colmax_k = k;
        } else {
            k_update_p<<<gb, 256, 0, s>>>(n, k, st, z, p);
        }
        PKM_CHECK_LAUNCH();
    }
    k_mark_maxiter<<<1, 256, 0, s>>>(k, st);
    PKM_CHECK_LAUNCH();
    ctx->colmax_src = nullptr;
    // final FP64 true residual of every column for the report -- unless every
    // column was accepted by an FP64 true residual of its final x already
    // (no live and no broken column: x has not moved since acceptance)
    if (f.live > 0 || f.broke > 0) {
        apply_A(PKM_FP64, X, tmp);
        k_sub<<<gb, 256, 0, s>>>(tot, B, tmp, tmp);
        PKM_CHECK_LAUNCH();
        dot_part(ctx, tmp, tmp, n, k, partA);
        k_report_true<<<1, 256, 0, s>>>(partA, k, st);
        PKM_CHECK_LAUNCH();
    }
    std::vector<ColState> hs(k);
    PKM_HIP(hipMemcpyAsync(hs.data(), st, sizeof(ColState) * k, hipMemcpyDeviceToHost, s));
    PKM_HIP(hipStreamSynchronize(s));
    auto t_end = std::chrono::steady_clock::now();

    int code = PKM_OK;
    int nbreak = 0, nmax = 0, first_break = -1;
    for (int c = 0; c < k; ++c) {
        if (hs[c].status == PKM_COL_BREAKDOWN) {
            code = PKM_ERR_BREAKDOWN;
            if (nbreak++ == 0) first_break = c;
        } else if (hs[c].status == PKM_COL_MAX_ITER) {
            ++nmax;
            if (code == PKM_OK) code = PKM_NOT_CONVERGED;
        }
    }
    if (nbreak > 0)
        ctx->err = std::to_string(nbreak) + " column(s) broke down (first: column " +
                   std::to_string(first_break) + "): p^T K_y p <= 0, r^T z < 0 or a non-finite "
                   "value; with BF16 products this means the rounded K + lambda I is not "
                   "positive definite (use a more accurate product)";
    else if (nmax > 0)
        ctx->err = std::to_string(nmax) + " column(s) reached max_iter";
    if (info) {
        for (int c = 0; c < k; ++c) {
            if (info->iters) info->iters[c] = hs[c].iters;
            if (info->relres_true) info->relres_true[c] = hs[c].tru;
            if (info->relres_rec) info->relres_rec[c] = hs[c].rec;
            if (info->col_status) info->col_status[c] = hs[c].status;
        }
        info->total_iters = it;
        info->true_residuals = true_count;
        info->prec_final = cur;
        info->refined = ever_refined ? 1 : 0;
        info->solve_ms = std::chrono::duration<double, std::milli>(t_end - t_start).count();
    }
    return code;
}

}  // namespace pkm
