"""ctypes binding of libpkm (include/pkm.h).  Argument marshalling only.

Every function keeps the C name and forwards to the library; torch is used
only to own device memory and to name the current HIP stream.  Tensors must
be float64 (int32 for inducing indices), contiguous and on the context's
device.  Errors raise ``PkmError`` carrying the library's status and message.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpkm.so")

PKM_OK = 0
PKM_NOT_CONVERGED = 1
PKM_ERR_INVALID = -1
PKM_ERR_BREAKDOWN = -2
PKM_ERR_HIP = -3
PKM_ERR_OOM = -4
PKM_ERR_UNSUPPORTED = -5

PKM_FP64 = 0
PKM_FP32 = 1
PKM_BF16X1 = 2
PKM_BF16X3 = 3
PKM_F16X3 = 4
PKM_I8X = 5

PKM_PC_NONE = 0
PKM_PC_NYSTROM = 1
PKM_PC_FITC = 2
PKM_PC_LOWRANK = 3
PKM_PC_SKETCH = 4
PKM_PC_PITC = 5
PKM_PC_HYBRID = 6
PKM_PC_SPECTRAL = 7

PKM_COL_CONVERGED = 0
PKM_COL_MAX_ITER = 1
PKM_COL_BREAKDOWN = 2

# every symbol include/pkm.h declares
EXPORTS = (
    "pkm_create", "pkm_destroy", "pkm_last_error", "pkm_version", "pkm_kernel_mvm",
    "pkm_kernel_mvm_shift", "pkm_kernel_mvm_noalloc",
    "pkm_precond_setup", "pkm_precond_setup_pitc",
    "pkm_precond_setup_hybrid", "pkm_precond_setup_spectral", "pkm_precond_sub_lowrank",
    "pkm_precond_apply", "pkm_precond_diag", "pkm_precond_destroy",
    "pkm_solve", "pkm_solve_batched", "pkm_cross_mvm", "pkm_predict",
    "pkm_laplace_mode", "pkm_laplace_grad", "pkm_laplace_predict", "pkm_grad_pass", "pkm_lml_grad", "pkm_timing_enable", "pkm_mvm_stats",
    "pkm_mvm_stats_reset", "pkm_mlp_create", "pkm_mlp_destroy", "pkm_mlp_params",
    "pkm_mlp_forward", "pkm_mlp_loss_grad", "pkm_mlp_train_step", "pkm_adagrad_step",
    "pkm_mlp_nparams", "pkm_mlp_state_get", "pkm_mlp_state_set", "pkm_precond_psi_f32",
    "pkm_precond_setup_rsvd", "pkm_sym_eig", "pkm_rademacher",
    "pkm_tune_cache_load",
)


class pkm_problem(C.Structure):
    _fields_ = [("n", C.c_int64), ("d", C.c_int32), ("reserved", C.c_int32),
                ("X", C.c_void_p), ("lengthscales", C.POINTER(C.c_double)),
                ("sigma2", C.c_double), ("lambda_", C.c_double)]


class pkm_solve_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int64), ("prec", C.c_int32),
                ("reliable_every", C.c_int32), ("check_every", C.c_int32),
                ("use_x0", C.c_int32)]


class pkm_solve_info(C.Structure):
    _fields_ = [("iters", C.POINTER(C.c_int64)), ("relres_true", C.POINTER(C.c_double)),
                ("relres_rec", C.POINTER(C.c_double)), ("col_status", C.POINTER(C.c_int32)),
                ("total_iters", C.c_int64), ("true_residuals", C.c_int64),
                ("solve_ms", C.c_double), ("prec_final", C.c_int32), ("refined", C.c_int32)]


class pkm_laplace_info(C.Structure):
    _fields_ = [("newton_iters", C.c_int32), ("reserved", C.c_int32), ("pcg_steps", C.c_int64),
                ("psi", C.c_double), ("ms", C.c_double)]


class PkmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pkm error {code}: {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load libpkm.so (fails loudly when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with "
                          "`python -m paper_1602_06693_amd.build`")
    lib = C.CDLL(path)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    P = C.POINTER
    sig = {
        "pkm_create": (C.c_int, [P(vp), C.c_int, vp]),
        "pkm_destroy": (C.c_int, [vp]),
        "pkm_last_error": (C.c_char_p, [vp]),
        "pkm_version": (C.c_char_p, []),
        "pkm_kernel_mvm": (C.c_int, [vp, P(pkm_problem), i32, i32, vp, vp]),
        "pkm_kernel_mvm_shift": (C.c_int, [vp, P(pkm_problem), i32, i32, dbl, vp, vp]),
        "pkm_precond_setup": (C.c_int, [vp, P(pkm_problem), i32, i32, vp, vp, dbl, P(vp)]),
        "pkm_precond_setup_pitc": (C.c_int, [vp, P(pkm_problem), i32, vp, i32, dbl, P(vp)]),
        "pkm_precond_setup_hybrid": (C.c_int, [vp, P(pkm_problem), i32, vp, i32, vp, dbl,
                                               P(vp)]),
        "pkm_precond_setup_spectral": (C.c_int, [vp, P(pkm_problem), i32, vp, P(vp)]),
        "pkm_precond_sub_lowrank": (C.c_int, [vp, vp, i32, vp, vp]),
        "pkm_precond_apply": (C.c_int, [vp, vp, i32, vp, vp]),
        "pkm_precond_diag": (C.c_int, [vp, vp, P(dbl)]),
        "pkm_precond_destroy": (C.c_int, [vp]),
        "pkm_precond_psi_f32": (C.c_int, [vp, vp, i32]),
        "pkm_precond_setup_rsvd": (C.c_int, [vp, P(pkm_problem), i32, i32, vp, i32, i32, P(vp)]),
        "pkm_sym_eig": (C.c_int, [i32, P(dbl), P(dbl), P(dbl)]),
        "pkm_rademacher": (C.c_int, [vp, i64, i32, C.c_uint64, vp, i64]),
        "pkm_solve": (C.c_int, [vp, P(pkm_problem), vp, i32, vp, vp, P(pkm_solve_opts),
                                P(pkm_solve_info)]),
        "pkm_solve_batched": (C.c_int, [vp, i32, P(pkm_problem), P(vp), i32, P(vp), P(vp),
                                        P(pkm_solve_opts), P(pkm_solve_info)]),
        "pkm_cross_mvm": (C.c_int, [vp, P(pkm_problem), i64, vp, i32, vp, vp]),
        "pkm_predict": (C.c_int, [vp, P(pkm_problem), vp, vp, i64, vp, P(pkm_solve_opts), vp, vp,
                                  P(pkm_solve_info), P(pkm_solve_info)]),
        "pkm_laplace_mode": (C.c_int, [vp, P(pkm_problem), vp, vp, P(pkm_solve_opts), i32, dbl,
                                       vp, vp, P(pkm_laplace_info)]),
        "pkm_laplace_grad": (C.c_int, [vp, P(pkm_problem), vp, vp, vp, i32, vp,
                                       P(pkm_solve_opts), P(dbl), P(i64)]),
        "pkm_laplace_predict": (C.c_int, [vp, P(pkm_problem), vp, vp, vp, i64, vp,
                                          P(pkm_solve_opts), vp, vp, vp]),
        "pkm_grad_pass": (C.c_int, [vp, P(pkm_problem), i32, vp, vp, P(dbl)]),
        "pkm_lml_grad": (C.c_int, [vp, P(pkm_problem), vp, vp, i32, vp, P(pkm_solve_opts),
                                   P(dbl), vp, P(pkm_solve_info)]),
        "pkm_timing_enable": (C.c_int, [vp, i32]),
        "pkm_mvm_stats": (C.c_int, [vp, i32, P(i64), P(dbl), P(dbl), P(dbl)]),
        "pkm_mvm_stats_reset": (C.c_int, [vp]),
        "pkm_mlp_create": (C.c_int, [vp, i32, i32, i32, P(C.c_float), P(vp)]),
        "pkm_mlp_destroy": (C.c_int, [vp]),
        "pkm_mlp_params": (C.c_int, [vp, vp, P(C.c_float)]),
        "pkm_mlp_forward": (C.c_int, [vp, vp, P(pkm_problem), vp]),
        "pkm_mlp_loss_grad": (C.c_int, [vp, vp, P(pkm_problem), i32, vp, vp, P(dbl),
                                        P(C.c_float)]),
        "pkm_mlp_train_step": (C.c_int, [vp, vp, P(pkm_problem), i32, vp, vp, dbl, P(dbl)]),
        "pkm_mlp_nparams": (C.c_int, [vp, P(i64)]),
        "pkm_mlp_state_get": (C.c_int, [vp, vp, P(C.c_float), P(i64)]),
        "pkm_mlp_state_set": (C.c_int, [vp, vp, P(C.c_float), i64]),
        "pkm_adagrad_step": (C.c_int, [i32, P(dbl), P(dbl), P(dbl), dbl, dbl]),
        "pkm_tune_cache_load": (C.c_int, [C.c_char_p, P(i32), P(i32)]),
        "pkm_kernel_mvm_noalloc": (C.c_int, [vp, P(pkm_problem), i32, i32, vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(rc, ctx=None, allow=(PKM_OK,)):
    if rc in allow:
        return rc
    lib = load()
    msg = lib.pkm_last_error(ctx).decode()
    raise PkmError(rc, msg)


def _ptr(t, dtype="float64"):
    if t is None:
        return None
    import torch
    want = {"float64": torch.float64, "int32": torch.int32}[dtype]
    if t.dtype != want:
        raise TypeError(f"expected {want}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if t.device.type != "cuda":
        raise ValueError("tensor must live on the GPU")
    return C.c_void_p(t.data_ptr())


class Problem:
    """pkm_problem plus the host array it points to (kept alive here)."""

    def __init__(self, X, lengthscales, sigma2, lam):
        self.X = X
        self.ls = np.ascontiguousarray(np.asarray(lengthscales, dtype=np.float64))
        self.struct = pkm_problem(
            n=X.shape[0], d=X.shape[1], reserved=0, X=_ptr(X),
            lengthscales=self.ls.ctypes.data_as(C.POINTER(C.c_double)),
            sigma2=float(sigma2), lambda_=float(lam))

    @property
    def n(self):
        return self.struct.n

    @property
    def d(self):
        return self.struct.d

    @property
    def ref(self):
        return C.byref(self.struct)


def pkm_version():
    return load().pkm_version().decode()


def pkm_create(device=0, stream=None):
    """Create a context bound to ``device`` and a HIP stream handle (int or None)."""
    lib = load()
    out = C.c_void_p()
    s = C.c_void_p(stream) if stream else None
    _check(lib.pkm_create(C.byref(out), int(device), s))
    return out


def current_stream_handle():
    import torch
    return torch.cuda.current_stream().cuda_stream


def pkm_destroy(ctx):
    return load().pkm_destroy(ctx)


def pkm_kernel_mvm(ctx, prob: Problem, V, prec=PKM_FP32, Y=None):
    import torch
    if Y is None:
        Y = torch.empty_like(V)
    k = V.shape[1] if V.dim() == 2 else 1
    _check(load().pkm_kernel_mvm(ctx, prob.ref, k, prec, _ptr(V), _ptr(Y)), ctx)
    return Y


def pkm_kernel_mvm_shift(ctx, prob: Problem, V, shift, prec=PKM_FP32, Y=None):
    import torch
    if Y is None:
        Y = torch.empty_like(V)
    k = V.shape[1] if V.dim() == 2 else 1
    _check(load().pkm_kernel_mvm_shift(ctx, prob.ref, k, prec, float(shift), _ptr(V), _ptr(Y)), ctx)
    return Y


def pkm_precond_setup(ctx, prob: Problem, kind, m, idx=None, Phi=None, jitter=0.0):
    out = C.c_void_p()
    _check(load().pkm_precond_setup(ctx, prob.ref, kind, int(m), _ptr(idx, "int32"),
                                    _ptr(Phi), float(jitter), C.byref(out)), ctx)
    return out


def pkm_precond_setup_pitc(ctx, prob: Problem, m, idx, block, jitter=0.0):
    out = C.c_void_p()
    _check(load().pkm_precond_setup_pitc(ctx, prob.ref, int(m), _ptr(idx, "int32"), int(block),
                                         float(jitter), C.byref(out)), ctx)
    return out


def pkm_precond_setup_hybrid(ctx, prob: Problem, m, idx, U, jitter=0.0):
    out = C.c_void_p()
    _check(load().pkm_precond_setup_hybrid(ctx, prob.ref, int(m), _ptr(idx, "int32"),
                                           int(U.shape[1]), _ptr(U), float(jitter),
                                           C.byref(out)), ctx)
    return out


def pkm_precond_setup_spectral(ctx, prob: Problem, W):
    """W: device (m, d) float64 standard normal draws."""
    out = C.c_void_p()
    _check(load().pkm_precond_setup_spectral(ctx, prob.ref, int(W.shape[0]), _ptr(W),
                                             C.byref(out)), ctx)
    return out


def pkm_precond_sub_lowrank(ctx, pc, V, Y):
    """Y <- Y - Phi Phi^T V in place; returns Y."""
    k = V.shape[1] if V.dim() == 2 else 1
    _check(load().pkm_precond_sub_lowrank(ctx, pc, k, _ptr(V), _ptr(Y)), ctx)
    return Y


def pkm_precond_apply(ctx, pc, R, Z=None):
    import torch
    if Z is None:
        Z = torch.empty_like(R)
    k = R.shape[1] if R.dim() == 2 else 1
    _check(load().pkm_precond_apply(ctx, pc, k, _ptr(R), _ptr(Z)), ctx)
    return Z


def pkm_precond_diag(ctx, pc, n):
    D = np.empty(n)
    _check(load().pkm_precond_diag(ctx, pc, D.ctypes.data_as(C.POINTER(C.c_double))), ctx)
    return D


def pkm_precond_setup_rsvd(ctx, prob: Problem, r, Omega, q=0, prec=PKM_FP32):
    out = C.c_void_p()
    _check(load().pkm_precond_setup_rsvd(ctx, prob.ref, int(r), int(Omega.shape[1]), _ptr(Omega),
                                         int(q), int(prec), C.byref(out)), ctx)
    return out


def pkm_rademacher(ctx, n, ncols, seed, Z=None):
    """n x ncols FP64 +-1 block from the device SplitMix64 generator, written
    into the first ncols columns of Z (contiguous n x ldz, ldz >= ncols)."""
    import torch
    if Z is None:
        Z = torch.empty((n, ncols), dtype=torch.float64, device="cuda")
    _check(load().pkm_rademacher(ctx, int(n), int(ncols), int(seed) & ((1 << 64) - 1), _ptr(Z),
                                 int(Z.shape[1])), ctx)
    return Z


def pkm_sym_eig(A):
    """(w descending, Z with eigenvectors as columns) of a symmetric host matrix."""
    A = np.ascontiguousarray(np.asarray(A, dtype=np.float64))
    n = A.shape[0]
    w = np.zeros(n)
    Z = np.zeros((n, n))
    P = C.POINTER(C.c_double)
    _check(load().pkm_sym_eig(int(n), A.ctypes.data_as(P), w.ctypes.data_as(P),
                              Z.ctypes.data_as(P)))
    return w, Z


def pkm_precond_psi_f32(ctx, pc, on=True):
    _check(load().pkm_precond_psi_f32(ctx, pc, 1 if on else 0), ctx)


def pkm_precond_destroy(pc):
    return load().pkm_precond_destroy(pc)


class SolveInfo:
    def __init__(self, k):
        self.iters = np.zeros(k, np.int64)
        self.relres_true = np.zeros(k)
        self.relres_rec = np.zeros(k)
        self.col_status = np.zeros(k, np.int32)
        self.struct = pkm_solve_info(
            iters=self.iters.ctypes.data_as(C.POINTER(C.c_int64)),
            relres_true=self.relres_true.ctypes.data_as(C.POINTER(C.c_double)),
            relres_rec=self.relres_rec.ctypes.data_as(C.POINTER(C.c_double)),
            col_status=self.col_status.ctypes.data_as(C.POINTER(C.c_int32)))
        self.rc = 0

    @property
    def total_iters(self):
        return self.struct.total_iters

    @property
    def true_residuals(self):
        return self.struct.true_residuals

    @property
    def solve_ms(self):
        return self.struct.solve_ms

    @property
    def prec_final(self):
        return self.struct.prec_final

    @property
    def refined(self):
        return bool(self.struct.refined)


def make_opts(tol=1e-6, max_iter=100000, prec=PKM_FP32, reliable_every=25, check_every=1,
              use_x0=False):
    return pkm_solve_opts(tol=tol, max_iter=max_iter, prec=prec, reliable_every=reliable_every,
                          check_every=check_every, use_x0=1 if use_x0 else 0)


def pkm_solve(ctx, prob: Problem, B, pc=None, X=None, opts=None, allow_warning=True):
    """Returns (X, SolveInfo); PKM_NOT_CONVERGED is returned in info.rc when allowed."""
    import torch
    if X is None:
        X = torch.zeros_like(B)
    k = B.shape[1] if B.dim() == 2 else 1
    info = SolveInfo(k)
    opts = opts or make_opts()
    rc = load().pkm_solve(ctx, prob.ref, pc, k, _ptr(B), _ptr(X), C.byref(opts),
                          C.byref(info.struct))
    info.rc = rc
    _check(rc, ctx, allow=(PKM_OK, PKM_NOT_CONVERGED) if allow_warning else (PKM_OK,))
    return X, info


def pkm_cross_mvm(ctx, prob: Problem, X_star, V):
    """K(X_star, X) V."""
    import torch
    k = V.shape[1] if V.dim() == 2 else 1
    Y = torch.empty((X_star.shape[0], k), dtype=torch.float64, device=V.device)
    _check(load().pkm_cross_mvm(ctx, prob.ref, int(X_star.shape[0]), _ptr(X_star), k, _ptr(V),
                                _ptr(Y)), ctx)
    return Y


def pkm_predict(ctx, prob: Problem, y, X_star, pc=None, opts=None, variance=True):
    """Returns (mean, var or None, SolveInfo of the mean solve, SolveInfo of the
    variance solve or None)."""
    import torch
    ns = X_star.shape[0]
    mean = torch.empty(ns, dtype=torch.float64, device=y.device)
    var = torch.empty(ns, dtype=torch.float64, device=y.device) if variance else None
    im = SolveInfo(1)
    iv = SolveInfo(ns) if variance else None
    opts = opts or make_opts()
    rc = load().pkm_predict(ctx, prob.ref, pc, _ptr(y), int(ns), _ptr(X_star), C.byref(opts),
                            _ptr(mean), _ptr(var) if variance else None, C.byref(im.struct),
                            C.byref(iv.struct) if variance else None)
    _check(rc, ctx, allow=(PKM_OK, PKM_NOT_CONVERGED))
    return mean, var, im, iv


def pkm_laplace_mode(ctx, prob: Problem, y, pc=None, opts=None, max_newton=50, tol=1e-10):
    """Returns (f_hat, a, pkm_laplace_info)."""
    import torch
    f = torch.empty_like(y)
    a = torch.empty_like(y)
    info = pkm_laplace_info()
    opts = opts or make_opts()
    rc = load().pkm_laplace_mode(ctx, prob.ref, pc, _ptr(y), C.byref(opts), int(max_newton),
                                 float(tol), _ptr(f), _ptr(a), C.byref(info))
    _check(rc, ctx, allow=(PKM_OK, PKM_NOT_CONVERGED))
    return f, a, info


def pkm_laplace_grad(ctx, prob: Problem, y, f, R, pc=None, opts=None):
    """Returns (grad (d + 1,), PCG steps)."""
    g = np.zeros(prob.d + 1)
    steps = C.c_int64(0)
    opts = opts or make_opts()
    rc = load().pkm_laplace_grad(ctx, prob.ref, pc, _ptr(y), _ptr(f), int(R.shape[1]), _ptr(R),
                                 C.byref(opts), g.ctypes.data_as(C.POINTER(C.c_double)),
                                 C.byref(steps))
    _check(rc, ctx, allow=(PKM_OK, PKM_NOT_CONVERGED))
    return g, steps.value


def pkm_laplace_predict(ctx, prob: Problem, y, f, X_star, pc=None, opts=None):
    """Returns (mean, var, p) device tensors."""
    import torch
    ns = X_star.shape[0]
    mean = torch.empty(ns, dtype=torch.float64, device=y.device)
    var = torch.empty_like(mean)
    p = torch.empty_like(mean)
    opts = opts or make_opts()
    rc = load().pkm_laplace_predict(ctx, prob.ref, pc, _ptr(y), _ptr(f), int(ns), _ptr(X_star),
                                    C.byref(opts), _ptr(mean), _ptr(var), _ptr(p))
    _check(rc, ctx, allow=(PKM_OK, PKM_NOT_CONVERGED))
    return mean, var, p


def pkm_grad_pass(ctx, prob: Problem, N, AS, YZ):
    g = np.zeros(prob.d + 2)
    _check(load().pkm_grad_pass(ctx, prob.ref, int(N), _ptr(AS), _ptr(YZ),
                                g.ctypes.data_as(C.POINTER(C.c_double))), ctx)
    return g


def pkm_lml_grad(ctx, prob: Problem, y, Z, pc=None, opts=None, sol=None):
    N = Z.shape[1]
    g = np.zeros(prob.d + 2)
    info = SolveInfo(1 + N)
    opts = opts or make_opts()
    rc = load().pkm_lml_grad(ctx, prob.ref, pc, _ptr(y), int(N), _ptr(Z), C.byref(opts),
                             g.ctypes.data_as(C.POINTER(C.c_double)), _ptr(sol),
                             C.byref(info.struct))
    info.rc = rc
    _check(rc, ctx, allow=(PKM_OK, PKM_NOT_CONVERGED))
    return g, info


def pkm_timing_enable(ctx, on=True):
    _check(load().pkm_timing_enable(ctx, 1 if on else 0), ctx)


def pkm_mvm_stats(ctx, prec):
    launches = C.c_int64()
    ms, pairs, flops = C.c_double(), C.c_double(), C.c_double()
    _check(load().pkm_mvm_stats(ctx, prec, C.byref(launches), C.byref(ms), C.byref(pairs),
                                C.byref(flops)), ctx)
    return {"launches": launches.value, "ms": ms.value, "pairs": pairs.value,
            "flops": flops.value}


def pkm_mvm_stats_reset(ctx):
    _check(load().pkm_mvm_stats_reset(ctx), ctx)


MLP_PARAM_NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def mlp_flatten(params):
    """Concatenate a dict of weights into the library's FP32 parameter layout."""
    return np.ascontiguousarray(np.concatenate(
        [np.asarray(params[k], dtype=np.float32).reshape(-1) for k in MLP_PARAM_NAMES]))


def mlp_unflatten(flat, d_in, hidden, rank):
    shapes = {"W1": (d_in, hidden), "b1": (hidden,), "W2": (hidden, hidden), "b2": (hidden,),
              "W3": (hidden, rank), "b3": (rank,)}
    out, o = {}, 0
    for k in MLP_PARAM_NAMES:
        size = int(np.prod(shapes[k]))
        out[k] = np.asarray(flat[o:o + size], dtype=np.float64).reshape(shapes[k])
        o += size
    return out


def pkm_mlp_create(ctx, params, d_in, hidden, rank):
    flat = mlp_flatten(params)
    out = C.c_void_p()
    _check(load().pkm_mlp_create(ctx, int(d_in), int(hidden), int(rank),
                                 flat.ctypes.data_as(C.POINTER(C.c_float)), C.byref(out)), ctx)
    return out


def pkm_mlp_destroy(net):
    return load().pkm_mlp_destroy(net)


def pkm_mlp_params(ctx, net, d_in, hidden, rank):
    n = d_in * hidden + hidden + hidden * hidden + hidden + hidden * rank + rank
    flat = np.zeros(n, np.float32)
    _check(load().pkm_mlp_params(ctx, net, flat.ctypes.data_as(C.POINTER(C.c_float))), ctx)
    return mlp_unflatten(flat, d_in, hidden, rank)


def pkm_mlp_nparams(net):
    n = C.c_int64()
    _check(load().pkm_mlp_nparams(net, C.byref(n)))
    return n.value


def pkm_mlp_state_get(ctx, net):
    """(state, t): FP32 [weights | Adam m | Adam v] and Adam's step count."""
    state = np.zeros(3 * pkm_mlp_nparams(net), np.float32)
    t = C.c_int64()
    _check(load().pkm_mlp_state_get(ctx, net, state.ctypes.data_as(C.POINTER(C.c_float)),
                                    C.byref(t)), ctx)
    return state, t.value


def pkm_mlp_state_set(ctx, net, state, t):
    state = np.ascontiguousarray(np.asarray(state, dtype=np.float32))
    if state.size != 3 * pkm_mlp_nparams(net):
        raise ValueError("state must hold 3 x nparams values")
    _check(load().pkm_mlp_state_set(ctx, net, state.ctypes.data_as(C.POINTER(C.c_float)),
                                    int(t)), ctx)


def pkm_mlp_forward(ctx, net, prob: Problem, rank, U=None):
    import torch
    if U is None:
        U = torch.empty((prob.n, rank), dtype=torch.float64, device=prob.X.device)
    _check(load().pkm_mlp_forward(ctx, net, prob.ref, _ptr(U)), ctx)
    return U


def pkm_mlp_loss_grad(ctx, net, prob: Problem, Z, KZ, d_in, hidden, rank):
    n = d_in * hidden + hidden + hidden * hidden + hidden + hidden * rank + rank
    g = np.zeros(n, np.float32)
    loss = C.c_double()
    _check(load().pkm_mlp_loss_grad(ctx, net, prob.ref, int(Z.shape[1]), _ptr(Z), _ptr(KZ),
                                    C.byref(loss), g.ctypes.data_as(C.POINTER(C.c_float))), ctx)
    return loss.value, mlp_unflatten(g, d_in, hidden, rank)


def pkm_mlp_train_step(ctx, net, prob: Problem, Z, KZ, lr):
    loss = C.c_double()
    _check(load().pkm_mlp_train_step(ctx, net, prob.ref, int(Z.shape[1]), _ptr(Z), _ptr(KZ),
                                     float(lr), C.byref(loss)), ctx)
    return loss.value


def pkm_adagrad_step(theta, g, G, eta=1.0, eps=1e-8):
    """In-place ADAGRAD ascent on float64 numpy arrays theta and G."""
    g = np.ascontiguousarray(np.asarray(g, dtype=np.float64))
    assert theta.dtype == np.float64 and G.dtype == np.float64
    assert theta.flags.c_contiguous and G.flags.c_contiguous
    P = C.POINTER(C.c_double)
    _check(load().pkm_adagrad_step(int(theta.size), theta.ctypes.data_as(P),
                                   g.ctypes.data_as(P), G.ctypes.data_as(P), float(eta),
                                   float(eps)))
    return theta


def pkm_kernel_mvm_noalloc(ctx, prob: Problem, V, Y, prec=PKM_I8X):
    """Y = (K + lambda I) V into the caller's Y without any device allocation."""
    k = V.shape[1] if V.dim() == 2 else 1
    _check(load().pkm_kernel_mvm_noalloc(ctx, prob.ref, k, prec, _ptr(V), _ptr(Y)), ctx)
    return Y


def pkm_tune_cache_load(path):
    """Merge a batched-product tuning cache file; returns (accepted, rejected)."""
    a, r = C.c_int32(), C.c_int32()
    _check(load().pkm_tune_cache_load(None if path is None else str(path).encode(), C.byref(a),
                                      C.byref(r)))
    return a.value, r.value


def pkm_solve_batched(ctx, probs, Bs, pcs=None, Xs=None, opts=None):
    """probs: list of Problem; Bs: list of (n_b, k) device tensors.
    Returns (list of X tensors, list of SolveInfo, rc)."""
    import torch
    P = len(probs)
    k = Bs[0].shape[1]
    Xs = Xs or [torch.zeros_like(b) for b in Bs]
    arr = (pkm_problem * P)(*[p.struct for p in probs])
    VP = C.c_void_p * P
    bptr = VP(*[_ptr(b).value for b in Bs])
    xptr = VP(*[_ptr(x).value for x in Xs])
    pcp = VP(*[(pc.value if pc is not None else None) for pc in pcs]) if pcs else None
    infos = [SolveInfo(k) for _ in range(P)]
    iarr = (pkm_solve_info * P)(*[i.struct for i in infos])
    opts = opts or make_opts()
    rc = load().pkm_solve_batched(ctx, P, arr, pcp, k, bptr, xptr, C.byref(opts), iarr)
    for i, inf in enumerate(infos):
        inf.struct = iarr[i]
        inf.rc = rc
    _check(rc, ctx, allow=(PKM_OK, PKM_NOT_CONVERGED))
    return Xs, infos, rc
