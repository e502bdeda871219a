/*
 * pkm -- preconditioned conjugate gradients on kernel matrices, MI355X (gfx950).
 *
 * C ABI of the library libpkm.so.  Operations follow "Preconditioning Kernel
 * Matrices" (Cutajar, Osborne, Cunningham, Filippone, ICML 2016):
 *
 *   kernel          ARD-RBF, Eq. (1):
 *                   k(x_i, x_j) = sigma2 * exp(-1/2 sum_r (x_ir - x_jr)^2 / l_r^2)
 *   system matrix   K_y = K + lambda I (Section 2.1)
 *   solver          preconditioned CG, Algorithm 1 (textbook reading, see
 *                   pkm_solve), applied independently to every column of a
 *                   right-hand-side block [y, r_1 .. r_N]
 *   preconditioners Nystrom (Section 3.1), FITC (Section 3.1.1) and a
 *                   caller-given factor Phi (Section 3.2), all applied through
 *                   the matrix inversion lemma
 *   gradient        log-marginal-likelihood gradient, Eq. (2), with the trace
 *                   estimated from Rademacher probes (Section 2.1)
 *
 * K is never stored: every product regenerates kernel tiles from X.
 *
 * Conventions shared by every entry point
 *   - Matrices are row-major.  An "n x k block" has element (i, c) at
 *     offset i * k + c.
 *   - "device" pointers are HIP device memory on the context's device,
 *     owned by the caller, and must stay valid until the context's stream
 *     has passed the call.  "host" pointers are ordinary host memory.
 *   - Calls are enqueued on the context's stream.  Calls with host outputs
 *     (pkm_solve's info, gradients, statistics) synchronise that stream
 *     before they return.
 *   - Return value: PKM_OK (0), a positive warning, or a negative error.
 *     On error nothing has been launched unless stated otherwise, and
 *     pkm_last_error() describes the cause.  No C++ exception or abort
 *     crosses this interface.
 *   - Objects created by the library (pkm_ctx, pkm_precond) are owned by it
 *     and released by the matching *_destroy call.
 */
#ifndef PKM_H
#define PKM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define PKM_OK               0
#define PKM_NOT_CONVERGED    1   /* warning: some column hit max_iter      */
#define PKM_ERR_INVALID     -1   /* bad argument; nothing launched          */
#define PKM_ERR_BREAKDOWN   -2   /* p^T K_y p <= 0, r^T z <= 0, or NaN/Inf  */
#define PKM_ERR_HIP         -3   /* a HIP runtime call failed               */
#define PKM_ERR_OOM         -4   /* device allocation failed                */
#define PKM_ERR_UNSUPPORTED -5   /* valid request the library cannot serve  */

/* ---- arithmetic of the kernel product ---------------------------------- */
#define PKM_FP64   0   /* FP64 distances, exp and accumulation             */
#define PKM_FP32   1   /* FP32 MFMA distances and K x V, FP32 accumulation  */
#define PKM_BF16X1 2   /* BF16 MFMA: distances from exact 3-part BF16 splits
                          (FP32-class exponent), K and V rounded to BF16
                          once, FP32 accumulation                          */
#define PKM_BF16X3 3   /* as PKM_BF16X1 with K and V split in two BF16 parts:
                          K_h V_h + K_h V_l + K_l V_h                      */
#define PKM_F16X3  4   /* as PKM_BF16X3 with FP16 parts on FP16 MFMA: K is
                          taken as K / sigma2 in (0, 1]; each V column is
                          scaled by a power of two (largest magnitude in
                          [2^14, 2^15)) and unscaled in the epilogue;
                          relative ~2^-22 per entry.  V must be finite.    */
#define PKM_I8X    5   /* FP64-class product on int8 matrix cores: exponent
                          on FP64 MFMA, FP64 exp2 rounded to the fixed-point
                          integer rint(2^30 K / sigma2), each V column to
                          rint(2^e V) with its largest magnitude in
                          [2^29, 2^30); both in signed base-256 digits whose
                          pair products (all pairs of weight 256^(p+q),
                          p + q >= 2) sum exactly in int32; FP64 epilogue.
                          Errors ~2^-30 of each entry's scale, none of them
                          row- or column-structured (for small lambda against
                          |K|, where FP32-class products cannot certify).
                          d <= 32; V must be finite.                       */

/* ---- preconditioner kinds ---------------------------------------------- */
#define PKM_PC_NONE     0
#define PKM_PC_NYSTROM  1   /* P = K_XU K_UU^-1 K_UX + lambda I  (Section 3.1)   */
#define PKM_PC_FITC     2   /* P = Q + diag(K - Q) + lambda I   (Section 3.1.1) */
#define PKM_PC_LOWRANK  3   /* P = Phi Phi^T + lambda I         (Section 3.2)   */
#define PKM_PC_SKETCH   4   /* P = K S (S^T K S)^-1 S^T K + lambda I: Nystrom
                               with a general n x m sketch S (Section 3.1 is the
                               case S = columns of I at the inducing points)   */
#define PKM_PC_PITC     5   /* P = Q + blockdiag(K - Q) + lambda I over blocks
                               of consecutive rows (Section 3.1.1); set up by
                               pkm_precond_setup_pitc                          */
#define PKM_PC_HYBRID   6   /* SKETCH with S = [columns of I at inducing points,
                               a learned n x r factor U]; set up by
                               pkm_precond_setup_hybrid                        */
#define PKM_PC_SPECTRAL 7   /* P = Phi Phi^T + lambda I with random Fourier
                               features (Section 3.2 spectral approximation);
                               set up by pkm_precond_setup_spectral            */

/* ---- per-column solver status ------------------------------------------ */
#define PKM_COL_CONVERGED  0
#define PKM_COL_MAX_ITER   1
#define PKM_COL_BREAKDOWN  2

typedef struct pkm_ctx pkm_ctx;
typedef struct pkm_precond pkm_precond;
typedef struct pkm_mlp pkm_mlp;

/* One GP regression problem (Section 2): inputs X, kernel hyperparameters
 * theta = (sigma2, l_1 .. l_d) of Eq. (1), and noise variance lambda.
 *   n >= 1, 1 <= d <= 64, sigma2 > 0, lambda > 0, every l_r > 0.          */
typedef struct {
    int64_t       n;
    int32_t       d;
    int32_t       reserved;      /* must be 0 */
    const double* X;             /* device, n x d, FP64                        */
    const double* lengthscales;  /* host, d values l_r                         */
    double        sigma2;
    double        lambda;
} pkm_problem;

/* Solver options.  Zero-initialised fields take the documented default.   */
typedef struct {
    double  tol;             /* relative residual |b - K_y x|_2 / |b|_2 per
                                column; default 1e-6                         */
    int64_t max_iter;        /* default 100000 (the paper's cap, Section 4)  */
    int32_t prec;            /* PKM_FP64, PKM_FP32, PKM_BF16X1, PKM_BF16X3,
                                PKM_F16X3 or PKM_I8X for the product inside
                                the loop;
                                default
                                PKM_FP32                                    */
    int32_t reliable_every;  /* FP64 true-residual replacement period (non-FP64
                                products only); default 25.  Negative: the
                                period adapts (pkm_solve): it starts at
                                -reliable_every, doubles (up to 8x the start)
                                after a replacement whose largest
                                true/recursive residual ratio is at most 2 and
                                whose largest true residual fell below 0.7 of
                                its previous value, and returns to the start
                                after any other;
                                pkm_solve_batched uses the magnitude as a
                                fixed period                                */
    int32_t check_every;     /* host convergence poll period; default 1     */
    int32_t use_x0;          /* nonzero: X holds x0 on entry; else x0 = 0    */
} pkm_solve_opts;

/* Solver report.  Array fields are host arrays of k entries provided by the
 * caller (any may be NULL); scalar fields are written by the library.      */
typedef struct {
    int64_t* iters;          /* CG steps per column                          */
    double*  relres_true;    /* final FP64 |b - K_y x| / |b| per column      */
    double*  relres_rec;     /* final recursive residual per column          */
    int32_t* col_status;     /* PKM_COL_* per column                         */
    int64_t  total_iters;    /* steps of the shared loop                     */
    int64_t  true_residuals; /* FP64 true-residual products performed        */
    double   solve_ms;       /* wall time of the solve on the stream         */
    int32_t  prec_final;     /* product arithmetic in use at the end: the
                                requested one, or a more accurate one if the
                                solve escalated (see pkm_solve)             */
    int32_t  refined;        /* 1 if the columns entered refinement mode (see
                                pkm_solve) at some point, else 0            */
} pkm_solve_info;

/* ---- context ------------------------------------------------------------
 * Binds a HIP device and stream (a hipStream_t passed as void*, NULL for the
 * null stream).  The context owns its scratch buffers.  Not thread-safe: one
 * host thread per context.                                                  */
int pkm_create(pkm_ctx** out, int device, void* stream);
int pkm_destroy(pkm_ctx* ctx);
/* Message for the last failing call on ctx (or on any context when ctx is
 * NULL, per host thread).  Never NULL.                                      */
const char* pkm_last_error(const pkm_ctx* ctx);
/* Library build string (architecture and version).                          */
const char* pkm_version(void);

/* ---- kernel product (Section 2.1: the O(n^2) operation of every CG step) --
 * Y = (K + lambda I) V for V, Y device n x k FP64 (k >= 1).  prec selects
 * the arithmetic of the K V part (the lambda V term is always FP64): any
 * PKM_FP64 .. PKM_I8X; FP32 needs d <= 34, the 16-bit products d <= 36,
 * PKM_I8X d <= 32.
 * Y may not alias V.                                                         */
int pkm_kernel_mvm(pkm_ctx* ctx, const pkm_problem* prob, int32_t k,
                   int32_t prec, const double* V, double* Y);
/* Y = (K + lambda I) V like pkm_kernel_mvm, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the call allocates nothing.  prec must be
 * PKM_I8X (else PKM_ERR_UNSUPPORTED); results equal pkm_kernel_mvm's with
 * PKM_I8X bit for bit.  All scratch (prepared operands, packed V digits,
 * partial sums) lives in one static device array of 128 MiB per device,
 * reserved when the library loads and held until the process ends; its
 * address is looked up by pkm_create.  A problem whose scratch exceeds it is
 * rejected with PKM_ERR_INVALID before any launch (about n <= 65536 at
 * d <= 16, k <= 33).  Every call on a device shares the array: calls that
 * overlap on one device (several streams or contexts) race.               */
int pkm_kernel_mvm_noalloc(pkm_ctx* ctx, const pkm_problem* prob, int32_t k,
                           int32_t prec, const double* V, double* Y);
/* Y = (K + shift I) V with any shift >= 0 (shift = 0: the plain K V, e.g.
 * the probe pairs (Z, K Z) that train the learned factor).                 */
int pkm_kernel_mvm_shift(pkm_ctx* ctx, const pkm_problem* prob, int32_t k,
                         int32_t prec, double shift, const double* V, double* Y);

/* ---- preconditioner setup (Sections 3.1, 3.1.1, 3.2) ----------------------
 * NYSTROM / FITC: inducing points U = X[idx], idx a device array of m
 *   distinct indices in [0, n); jitter >= 0 is added to the diagonal of K_UU.
 * LOWRANK: factor Phi given as a device n x m FP64 array (idx ignored).
 * SKETCH: sketch S given in Phi (device n x m FP64); K S is formed with one
 *   FP32 kernel product, S^T K S gets jitter times its own diagonal added
 *   before its FP64 Cholesky, and the factor is K S L^-T, so the low-rank
 *   part never exceeds K (P <= K_y in the positive semi-definite order).
 * The result represents P^-1 = D^-1 - Psi Psi^T (matrix inversion lemma with
 * the noise, or noise plus FITC diagonal, as D); it is owned by the library.
 * 1 <= m <= min(n, 4096); SKETCH needs d <= 34.                            */
int pkm_precond_setup(pkm_ctx* ctx, const pkm_problem* prob, int32_t kind,
                      int32_t m, const int32_t* idx, const double* Phi,
                      double jitter, pkm_precond** out);
/* Z = P^-1 R for R, Z device n x k FP64 (may not alias).                   */
/* PITC (Section 3.1.1): Nystrom's Q with its error corrected exactly on
 * diagonal blocks of `block` consecutive rows (1 <= block <= 64; the last
 * block may be shorter): P = Q + blockdiag(K - Q) + lambda I.  Block 1 is
 * FITC without its clip at zero.  The blocks are only as useful as the
 * caller's ordering of X makes them (e.g. rows sorted along a space-filling
 * curve).  Inducing points and jitter as for NYSTROM.  Not accepted by
 * pkm_solve_batched (PKM_ERR_UNSUPPORTED).                                 */
int pkm_precond_setup_pitc(pkm_ctx* ctx, const pkm_problem* prob, int32_t m,
                           const int32_t* idx, int32_t block, double jitter,
                           pkm_precond** out);
/* Nystrom on the hybrid sketch S = [E_U, U]: E_U the m columns of the
 * identity at the inducing indices idx (device, m distinct in [0, n)), U a
 * device n x r FP64 array (e.g. the learned factor).  P = K S (S^T K S +
 * jitter * diag(S^T K S))^-1 S^T K + lambda I: the Section 3.1 Nystrom
 * preconditioner enlarged by the span of K U, so its low-rank part never
 * exceeds K and grows monotonically with the sketch.  K_XU and K U (one
 * FP64 product) in FP64.  m, r >= 1, m + r <= min(n, 4096), d <= 34.       */
int pkm_precond_setup_hybrid(pkm_ctx* ctx, const pkm_problem* prob, int32_t m,
                             const int32_t* idx, int32_t r, const double* U,
                             double jitter, pkm_precond** out);
/* Y <- Y - Phi Phi^T V for device n x k FP64 blocks V, Y (distinct), where
 * Phi Phi^T is the low-rank part of P = D + Phi Phi^T (for Nystrom, FITC and
 * PITC: Q = K_XU K_UU^-1 K_UX).  With Y = K V on entry this leaves
 * (K - Q) V, the part of K the preconditioner misses (training pairs for a
 * learned correction).  Two FP64 products with the stored n x m factor.    */
int pkm_precond_sub_lowrank(pkm_ctx* ctx, const pkm_precond* pc, int32_t k,
                            const double* V, double* Y);
/* Spectral approximation (Section 3.2): frequencies s_r ~ N(0, Lambda /
 * (4 pi^2)), Lambda = diag(1 / l_r^2), given through standard normal draws W
 * (device m x d FP64, caller-owned; omega_r = 2 pi s_r = W_r / l).  Features
 * Phi = sqrt(sigma2 / m) [cos(X omega^T), sin(X omega^T)] (n x 2m, FP64), so
 * (Phi Phi^T)_ij = sigma2 / m sum_r cos(omega_r^T (x_i - x_j)) and
 * diag(Phi Phi^T) = sigma2 exactly; P = Phi Phi^T + lambda I through the
 * matrix inversion lemma.  1 <= m <= 2048.                                  */
int pkm_precond_setup_spectral(pkm_ctx* ctx, const pkm_problem* prob, int32_t m,
                               const double* W, pkm_precond** out);
/* Randomised truncated SVD (Section 3.2, partial SVD by random sampling):
 * Omega (device n x l FP64, caller-owned: standard normal draws), q power
 * iterations; Y = K Omega, then q times Q = orth(Y), Y = K Q; Q = orth(Y),
 * B = Q^T K Q = V diag(w) V^T and Phi = Q V_r diag(w_r)^1/2 from the r
 * largest eigenvalues (negatives clipped to 0); P = Phi Phi^T + lambda I
 * through the matrix inversion lemma (a PKM_PC_LOWRANK preconditioner).
 * The products with K use arithmetic prec; orth is shifted Cholesky QR
 * plus two Cholesky QR passes in FP64 on the device; the l x l
 * eigenproblem is solved on the host.  1 <= r <= l <= min(n, 1024),
 * 0 <= q <= 8; PKM_ERR_BREAKDOWN if the sketch is zero or non-finite.    */
int pkm_precond_setup_rsvd(pkm_ctx* ctx, const pkm_problem* prob, int32_t r, int32_t l,
                           const double* Omega, int32_t q, int32_t prec,
                           pkm_precond** out);
/* Rademacher probes for the stochastic trace estimate (Section 2.1) on the
 * device, from the SplitMix64 generator (Steele, Lea and Flood 2014):
 * seeded with `seed`, output t >= 1 is mix(seed + t * 0x9E3779B97F4A7C15
 * mod 2^64) with the reference finaliser (xor-shift 30, multiply by
 * 0xBF58476D1CE4E5B9, xor-shift 27, multiply by 0x94D049BB133111EB,
 * xor-shift 31); Z[i * ldz + c] (device, n x ncols row-major with leading
 * dimension ldz, FP64) is -1 if output i * ncols + c + 1 has its top bit
 * set, else +1.  Asynchronous on the context's stream; entries of a row
 * beyond ncols are not written.  1 <= n <= 2^32, 1 <= ncols <= 4096,
 * ldz >= ncols, else PKM_ERR_INVALID.  (The other calls take probes from
 * the caller; this is an optional source of them.)                       */
int pkm_rademacher(pkm_ctx* ctx, int64_t n, int32_t ncols, uint64_t seed, double* Z,
                   int64_t ldz);
/* Host utility (no device work, no context): eigenvalues w (descending) and
 * eigenvectors (the columns of Z, row-major n x n) of the symmetric n x n
 * host matrix A (row-major; its symmetric part is used), by Householder
 * tridiagonalisation and implicit QR steps with Wilkinson shifts -- the
 * eigensolver of pkm_precond_setup_rsvd.  The eigenvector rotations run on
 * up to 16 host threads (PKM_EIG_THREADS in the environment sets the
 * count).  1 <= n <= 4096, finite A, else PKM_ERR_INVALID.                 */
int pkm_sym_eig(int32_t n, const double* A, double* w, double* Z);
int pkm_precond_apply(pkm_ctx* ctx, const pkm_precond* pc, int32_t k,
                      const double* R, double* Z);
/* Storage of Psi in the apply Z = D^-1 R - Psi (Psi^T R) (the matrix
 * inversion lemma of Section 3.2).  on = 1 rounds Psi to FP32 once (round to
 * nearest) and every later pkm_precond_apply and single-problem solve reads
 * that copy, widening each entry to FP64 before FP64 matrix-core sums: the
 * apply is then exactly that of the symmetric operator D^-1 - Psi~ Psi~^T
 * (Psi~ the rounded copy), at half the bytes of Psi read per apply;
 * |Psi~ Psi~^T - Psi Psi^T| <= (2u + u^2) |Psi| |Psi|^T entrywise, u = 2^-24.
 * on = 0 frees the copy and goes back to Psi.  The batched solver reads the
 * FP64 Psi either way.  The rounding changes the preconditioned operator by
 * up to eta = (2u + u^2) || |Psi| ||^2 ||K + lambda I||, and Psi grows like
 * lambda^-1/2: worth it only while eta << 1 (lambda >= 1e-2 for unit-variance
 * kernels; at lambda = 1e-3 the extra PCG steps outweigh the halved bytes).
 * PKM_ERR_INVALID for another on, or a preconditioner created on another
 * device.                                                                   */
int pkm_precond_psi_f32(pkm_ctx* ctx, pkm_precond* pc, int32_t on);
/* Host copy of the preconditioner's diagonal part D (n values).           */
int pkm_precond_diag(pkm_ctx* ctx, const pkm_precond* pc, double* D_host);
int pkm_precond_destroy(pkm_precond* pc);

/* ---- PCG solve (Algorithm 1) --------------------------------------------
 * Solves K_y X = B for every column of the device n x k FP64 block B; X is a
 * device n x k FP64 block (x0 on entry when opts->use_x0).  pc may be NULL
 * (plain CG).  Textbook recurrences per column; the solution accumulates in
 * FP64.  A column whose recursive residual meets tol stops stepping until
 * an FP64 true residual b - K_y x certifies it (that check runs once every
 * live column has stopped); if it fails, r is replaced by the true residual
 * and the column resumes.  With FP32 or BF16 products the same replacement
 * also runs every reliable_every steps.  A reduced-precision product whose
 * error is too large for lambda shows as a largest true residual that stops
 * decreasing (three replacements in a row without falling below 0.7 of its
 * best value -- and at least 150 steps unless it grew at the latest one), as
 * a true residual above |b| while the recursive one is 100 times smaller, or
 * as a column breakdown.  On the first stall the columns
 * switch to refinement mode: they restart their directions (p = z) at every
 * replacement and stop stepping once the recursive residual is 1e-3 below
 * the last true one (outer FP64 iterative refinement around short inner
 * solves).  With PKM_I8X (FP64-class) a slow true residual counts as a stall
 * only while it exceeds twice the recursive one, or after 1500 steps without
 * falling below 0.7 of its best.  On a second stall, divergence or breakdown
 * the solve raises the product arithmetic (16-bit -> FP32 -> FP64; an FP32
 * solve that stalled rather than diverged or broke down goes on with
 * PKM_I8X when d <= 32, and PKM_I8X -> FP64), resumes broken columns and
 * restarts every column from its FP64 true residual (reported in
 * prec_final).  A column converges when its FP64 true
 * relative residual is <= tol.  Returns PKM_NOT_CONVERGED if a column reached max_iter and
 * PKM_ERR_BREAKDOWN if one broke down; X holds the last iterate either way. */
int pkm_solve(pkm_ctx* ctx, const pkm_problem* prob, const pkm_precond* pc,
              int32_t k, const double* B, double* X,
              const pkm_solve_opts* opts, pkm_solve_info* info);

/* ---- batched solve ----------------------------------------------------------
 * P independent problems (own X, theta, lambda, n and d), each with its own
 * k-column right-hand side B[b] and solution X[b] (device n_b x k FP64;
 * B and X are host arrays of P device pointers) and preconditioner pcs[b]
 * (pcs NULL or pcs[b] NULL: none).  Same recurrences, tolerance handling
 * and per-column reports as pkm_solve (infos: host array of P reports, or
 * NULL).  Every PCG phase runs as one launch over all problems; the kernel
 * product is a work-queue launch per input-dimension class whose tile
 * shape is autotuned on first use: i-tiles per wave (1, 2 or 4; 2 or 4
 * for F16X3) times the work-group count below which a problem is split over
 * column ranges (512, 1024 or 2048), per arithmetic, augmented length,
 * column tiling and power-of-two bucket of the class's work (cached in
 * memory and, if the environment variable PKM_TUNE_CACHE names a file, there
 * as JSON lines; see pkm_tune_cache_load).
 * A problem whose columns all stopped stepping is certified by its own FP64
 * true residual at once; FP64 products run only for problems that need
 * them.  A large problem is split over column ranges of K (partial sums
 * added in a fixed order) when its row blocks alone would leave the chip
 * idle.  Stalls are handled per problem as in pkm_solve (refinement mode,
 * then FP64 products for that problem only; infos[b].prec_final).
 * prec PKM_FP32 or PKM_F16X3 (with FP64 residual replacement; a problem
 * that stalls or breaks down moves to FP64 products directly) or PKM_FP64;
 * 1 <= k <= 33, every d <= 34 for PKM_FP32, d <= 36 for PKM_F16X3.        */
int pkm_solve_batched(pkm_ctx* ctx, int32_t P, const pkm_problem* probs,
                      const pkm_precond* const* pcs, int32_t k, const double* const* B,
                      double* const* X, const pkm_solve_opts* opts, pkm_solve_info* infos);

/* Loads batched-product launch shapes from a tuning cache file (the format
 * pkm_solve_batched writes to PKM_TUNE_CACHE: one JSON object per line with
 * the key s4, kt, kr, work and the shape u, fill).  An entry is kept only if
 * its shape is one the library instantiates for its key; other lines are
 * counted in *rejected and ignored.  Host-only, no context; safe to call from
 * any thread (the cache is shared by all contexts and guarded by a lock).
 * accepted and rejected may be NULL.  PKM_ERR_INVALID for a NULL path.     */
int pkm_tune_cache_load(const char* path, int32_t* accepted, int32_t* rejected);

/* ---- gradient pass (Eq. (2) with the trace estimate of Section 2.1) -------
 * Given alpha = K_y^-1 y and S = K_y^-1 Z for N Rademacher probes Z, writes
 * the d + 2 host values
 *   g_i = 1/2 alpha^T dK_y_i alpha - 1/(2N) sum_c s_c^T dK_y_i z_c
 * for theta = (log sigma2, log l_1 .. log l_d, log lambda), i.e.
 *   dK_y/dlog sigma2 = K,  dK_y/dlog l_r = K o (x_ir - x_jr)^2 / l_r^2,
 *   dK_y/dlog lambda = lambda I.
 * AS = [alpha, S] and YZ = [y-solution alpha, Z] are device n x (1 + N) FP64
 * blocks: column 0 of both is alpha; columns 1..N are s_c and z_c.  N >= 0
 * (N = 0 gives the data-fit term only).  Arithmetic is FP64.               */
int pkm_grad_pass(pkm_ctx* ctx, const pkm_problem* prob, int32_t N,
                  const double* AS, const double* YZ, double* grad_host);

/* ---- solve + gradient --------------------------------------------------
 * Solves K_y [alpha, S] = [y, Z] with pc and opts, then runs the gradient
 * pass.  y is device n, Z device n x N (N >= 1).  Solutions are written to
 * sol (device n x (1 + N), may be NULL).  With opts->use_x0, sol must hold
 * the starting block [alpha_0, S_0] on entry (PKM_ERR_INVALID if sol is
 * NULL).  pc must have been set up for this problem's n on this context's
 * device and opts->prec must suit d, as for pkm_solve.  info arrays, if
 * given, hold 1 + N entries.                                               */
int pkm_lml_grad(pkm_ctx* ctx, const pkm_problem* prob, const pkm_precond* pc,
                 const double* y, int32_t N, const double* Z,
                 const pkm_solve_opts* opts, double* grad_host, double* sol,
                 pkm_solve_info* info);

/* ---- prediction at test inputs ---------------------------------------------
 * The GP predictive equations the paper's Section 2.1 refers to for test
 * data, with every solve a PCG solve (one per test point for the variance).
 * pkm_cross_mvm: Y = K(X_star, X) V, X_star device n_star x d FP64, V device
 * n x k, Y device n_star x k (FP64 MFMA product; d <= 34).
 * pkm_predict: mean (device n_star) = K(X_star, X) K_y^-1 y; if var (device
 * n_star) is not NULL, the latent variances sigma2 - k_*^T K_y^-1 k_* (add
 * lambda for a noisy target), from one block solve with the n_star columns
 * K(X, X_star) as right-hand sides (n_star <= 256 then).  pc and opts as for
 * pkm_solve; info_mean (1 column) and info_var (n_star columns) may be NULL.
 * Returns the worse of the two solves' status.                              */
int pkm_cross_mvm(pkm_ctx* ctx, const pkm_problem* prob, int64_t n_star,
                  const double* X_star, int32_t k, const double* V, double* Y);
int pkm_predict(pkm_ctx* ctx, const pkm_problem* prob, const pkm_precond* pc,
                const double* y, int64_t n_star, const double* X_star,
                const pkm_solve_opts* opts, double* mean, double* var,
                pkm_solve_info* info_mean, pkm_solve_info* info_var);

/* ---- GP classification: Laplace approximation (Section 2.2) --------------
 * Probit likelihood p(y_i | f_i) = Phi(y_i f_i), labels y (device n) in
 * {-1, +1}; prob's X, sigma2 and lengthscales define K (its lambda is not
 * used).  Every linear system is a PCG solve with
 * B = I + W^1/2 K W^1/2 (W = -d^2 log p / df^2, diagonal), with opts as for
 * pkm_solve; pc (NULL or a NYSTROM / FITC / PITC / LOWRANK / SKETCH / HYBRID /
 * SPECTRAL preconditioner of K for the same problem) supplies its low-rank
 * factor Phi for B's preconditioner I + (W^1/2 Phi)(W^1/2 Phi)^T.
 * pkm_laplace_mode: Newton iterations (b = W f + dlog p, B z = W^1/2 K b,
 *   a = b - W^1/2 z, f = K a) from f = 0 until Psi = log p(y|f) - f^T a / 2
 *   changes by <= tol relative; f, a device n outputs (a = K^-1 f).
 * pkm_laplace_grad: the three-term stochastic gradient of the approximate
 *   log-marginal likelihood at the mode f (explicit trace term with the N
 *   probe columns R, device n x N, 1 <= N <= 255; data-fit term; implicit
 *   term through dW/df), grad host d + 1 values for (log sigma2, log l_r).
 * pkm_laplace_predict: at n_star <= 256 test inputs, latent mean, variance
 *   and p(y_* = +1) = Phi(m / sqrt(1 + s^2)) (device n_star each).         */
typedef struct {
    int32_t newton_iters;
    int32_t reserved;
    int64_t pcg_steps;        /* PCG steps of all B solves                  */
    double  psi;              /* log p(y | f_hat) - f_hat^T a / 2           */
    double  ms;
} pkm_laplace_info;
int pkm_laplace_mode(pkm_ctx* ctx, const pkm_problem* prob, const pkm_precond* pc,
                     const double* y, const pkm_solve_opts* opts, int32_t max_newton,
                     double tol, double* f, double* a, pkm_laplace_info* info);
int pkm_laplace_grad(pkm_ctx* ctx, const pkm_problem* prob, const pkm_precond* pc,
                     const double* y, const double* f, int32_t N, const double* R,
                     const pkm_solve_opts* opts, double* grad, int64_t* pcg_steps);
int pkm_laplace_predict(pkm_ctx* ctx, const pkm_problem* prob, const pkm_precond* pc,
                        const double* y, const double* f, int64_t n_star,
                        const double* X_star, const pkm_solve_opts* opts, double* mean,
                        double* var, double* p);

/* ---- learned low-rank factor (Section 3.2 form P = U U^T + lambda I) -------
 * A network maps each scaled input row x_i / l to a row of U (n x rank):
 *   a1 = x W1 + b1, h1 = gelu(a1), a2 = h1 W2 + b2, h2 = gelu(a2),
 *   U = h2 W3 + b3, gelu(a) = a (1 + erf(a / sqrt 2)) / 2,
 * hidden width 128, BF16 weights in the products with FP32 accumulation,
 * FP32 master weights.  params (host, FP32) are laid out W1 (d_in x 128,
 * row-major), b1 (128), W2 (128 x 128), b2, W3 (128 x rank), b3 (rank);
 * 1 <= d_in <= 32, rank a multiple of 16 in [16, 128].  The object owns its
 * device buffers; pkm_mlp_destroy releases them.                            */
int pkm_mlp_create(pkm_ctx* ctx, int32_t d_in, int32_t hidden, int32_t rank,
                   const float* params, pkm_mlp** out);
int pkm_mlp_destroy(pkm_mlp* net);
/* Host copy of the FP32 master weights (same layout as params).             */
int pkm_mlp_params(pkm_ctx* ctx, const pkm_mlp* net, float* params);
/* Training state for checkpoints.  pkm_mlp_nparams reports the parameter
 * count P (no device work).  state (host, 3 P FP32) holds the master
 * weights, Adam's first moments and Adam's second moments, each in params
 * layout, one after the other; t is Adam's step count (bias corrections).
 * pkm_mlp_state_set restores both (t >= 0, every value finite, else
 * PKM_ERR_INVALID and the network is unchanged) and refreshes the BF16
 * copies, so that training continues as if never interrupted.             */
int pkm_mlp_nparams(const pkm_mlp* net, int64_t* nparams);
int pkm_mlp_state_get(pkm_ctx* ctx, const pkm_mlp* net, float* state, int64_t* t);
int pkm_mlp_state_set(pkm_ctx* ctx, pkm_mlp* net, const float* state, int64_t t);
/* U = net(X / l) for the problem's inputs (prob->d == d_in); U device
 * n x rank FP64, ready for pkm_precond_setup(PKM_PC_LOWRANK).               */
int pkm_mlp_forward(pkm_ctx* ctx, pkm_mlp* net, const pkm_problem* prob, double* U);
/* Training loss on probe pairs (Z, KZ = K Z), Z and KZ device n x nz FP64:
 *   L = |U (U^T Z) - K Z|_F^2 / |K Z|_F^2
 * (unbiased for |U U^T - K|_F^2 up to the normaliser since E[Z Z^T] = I).
 * pkm_mlp_loss_grad writes L and, if grads is non-NULL, dL/dparams (host,
 * params layout); pkm_mlp_train_step also applies one Adam step (beta1 0.9,
 * beta2 0.999, eps 1e-8) with learning rate lr.                             */
int pkm_mlp_loss_grad(pkm_ctx* ctx, pkm_mlp* net, const pkm_problem* prob, int32_t nz,
                      const double* Z, const double* KZ, double* loss, float* grads);
int pkm_mlp_train_step(pkm_ctx* ctx, pkm_mlp* net, const pkm_problem* prob, int32_t nz,
                       const double* Z, const double* KZ, double lr, double* loss);

/* ---- hyperparameter step (Section 5) ----------------------------------------
 * ADAGRAD ascent on p host values (log hyperparameters), elementwise:
 *   G <- G + g^2,   theta <- theta + eta g / (sqrt(G) + eps).
 * theta and G are updated in place (G starts at zero); host-only, no device
 * work, no context.  Returns PKM_ERR_INVALID for p < 1, NULL pointers,
 * eta <= 0 or eps < 0, or a non-finite gradient (nothing is updated).      */
int pkm_adagrad_step(int32_t p, double* theta, const double* g, double* G, double eta,
                     double eps);

/* ---- measurement ----------------------------------------------------------
 * When enabled, every kernel-product launch is bracketed by HIP events on
 * the context's stream.  pkm_mvm_stats returns, since the last reset, the
 * launch count, the summed launch time in ms, and the summed algorithmic
 * work: kernel entries n^2 and flops n^2 (2d + 2k) of the products.        */
int pkm_timing_enable(pkm_ctx* ctx, int32_t on);
int pkm_mvm_stats(pkm_ctx* ctx, int32_t prec, int64_t* launches, double* ms,
                  double* pairs, double* flops);
int pkm_mvm_stats_reset(pkm_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* PKM_H */
