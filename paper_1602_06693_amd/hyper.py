"""Hyperparameter learning loop (Section 5): stochastic-gradient ascent of the
log-marginal likelihood with ADAGRAD, every step's gradient from the library's
preconditioned solve and gradient pass.  Orchestration only: each numeric
step is a libpkm call.

theta = (log sigma2, log l_1 .. log l_d); lambda stays fixed.
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np

from . import binding as pk


def theta_of(sigma2, lengthscales):
    return np.concatenate([[math.log(sigma2)], np.log(np.asarray(lengthscales, float))])


def unpack(theta):
    return float(math.exp(theta[0])), np.exp(np.asarray(theta[1:], float))


def _pack_json(obj):
    return np.frombuffer(json.dumps(obj).encode(), dtype=np.uint8)


def _unpack_json(arr):
    return json.loads(np.asarray(arr, dtype=np.uint8).tobytes().decode())


def _rng_state(rng):
    return _pack_json(rng.bit_generator.state)


def _set_rng_state(rng, arr):
    rng.bit_generator.state = _unpack_json(arr)


class Arm:
    """A preconditioner policy: returns a pkm_precond handle for the current problem.

    state() / restore() carry everything a later step depends on (random
    streams, the network's weights and optimiser state, counters) as numpy
    arrays, so that a checkpointed run resumes exactly."""

    name = "none"

    def setup(self, ctx, prob, step):
        return None

    def state(self, ctx):
        return {}

    def restore(self, ctx, st):
        pass


class NystromArm(Arm):
    """Fresh uniform inducing points every step (Section 5)."""

    def __init__(self, n, m, seed=0, jitter=1e-8, name="nystrom"):
        self.n, self.m, self.jitter, self.name = n, m, jitter, name
        self.rng = np.random.default_rng(seed)

    def setup(self, ctx, prob, step):
        import torch
        idx = np.sort(self.rng.choice(self.n, size=self.m, replace=False)).astype(np.int32)
        return pk.pkm_precond_setup(ctx, prob, pk.PKM_PC_NYSTROM, self.m,
                                    idx=torch.from_numpy(idx).to(prob.X.device),
                                    jitter=self.jitter)

    def state(self, ctx):
        return {"rng": _rng_state(self.rng)}

    def restore(self, ctx, st):
        _set_rng_state(self.rng, st["rng"])


class LearnedArm(Arm):
    """Nystrom enlarged by a learned sketch.  Every step draws the same fresh
    inducing points as a NystromArm with the same seed, forms probe pairs
    (Z, (K - Q) Z) -- the part of K that step's Nystrom approximation Q
    misses -- fine-tunes the factor network on them, and preconditions with
    Nystrom on the sketch [E_U, U(X)] (pkm_precond_setup_hybrid).

    Fallback: the training loss is the share of the probes' residual energy
    ||(K - Q) Z||^2 that the learned columns leave unexplained (1 for a
    network that adds nothing, above 1 for one that adds the wrong
    directions).  When the fine-tuned network leaves at least
    ``fallback_loss`` of it, that step uses plain Nystrom on the same
    inducing points instead (counted in ``fallbacks``).  The threshold sits
    just below 1: a network that explains only a few per cent of the
    residual energy can still take the largest residual directions and cut
    the CG steps by a fifth."""

    name = "learned"

    def __init__(self, ctx, params, d, rank, n, m, n_train_probes=64, first_steps=300,
                 steps_per_theta=50, lr=2e-3, seed=0, jitter=1e-8, log=None,
                 fallback_loss=0.999):
        self.net = pk.pkm_mlp_create(ctx, params, d, 128, rank)
        self.rank, self.nz, self.n, self.m = rank, n_train_probes, n, m
        self.first, self.later, self.lr, self.jitter = first_steps, steps_per_theta, lr, jitter
        self.rng_idx = np.random.default_rng(seed)        # same draws as NystromArm(seed)
        self.rng = np.random.default_rng(seed + 7919)     # probes
        self.train_s = 0.0
        self.losses = []
        self.log = log
        self.fallback_loss = fallback_loss
        self.fallbacks = 0

    def setup(self, ctx, prob, step):
        import torch
        t0 = time.perf_counter()
        dev = prob.X.device
        idx = np.sort(self.rng_idx.choice(self.n, size=self.m, replace=False)).astype(np.int32)
        idx_d = torch.from_numpy(idx).to(dev)
        Z = torch.from_numpy(pk_rademacher(self.rng, prob.n, self.nz)).to(dev)
        R = pk.pkm_kernel_mvm_shift(ctx, prob, Z, 0.0, pk.PKM_FP32)   # K Z
        pcn = pk.pkm_precond_setup(ctx, prob, pk.PKM_PC_NYSTROM, self.m, idx=idx_d,
                                   jitter=self.jitter)
        try:
            pk.pkm_precond_sub_lowrank(ctx, pcn, Z, R)                 # (K - Q) Z
        finally:
            pk.pkm_precond_destroy(pcn)
        iters = self.first if step == 0 else self.later
        for it in range(iters):
            self.losses.append(pk.pkm_mlp_train_step(ctx, self.net, prob, Z, R, self.lr))
            if self.log and (it + 1) % 50 == 0:
                self.log(f"[learned] step {step}: Adam {it + 1}/{iters}, loss {self.losses[-1]:.4e}")
        # the loss after the last update (train_step reports the loss before it)
        final = pk.pkm_mlp_loss_grad(ctx, self.net, prob, Z, R, prob.d, 128, self.rank)[0]
        if final >= self.fallback_loss:
            self.fallbacks += 1
            if self.log:
                self.log(f"[learned] step {step}: loss {final:.3f}, plain Nystrom this step")
            torch.cuda.synchronize()
            self.train_s += time.perf_counter() - t0
            return pk.pkm_precond_setup(ctx, prob, pk.PKM_PC_NYSTROM, self.m, idx=idx_d,
                                        jitter=self.jitter)
        U = pk.pkm_mlp_forward(ctx, self.net, prob, self.rank)
        torch.cuda.synchronize()
        self.train_s += time.perf_counter() - t0
        return pk.pkm_precond_setup_hybrid(ctx, prob, self.m, idx_d, U, jitter=self.jitter)

    def state(self, ctx):
        net, t = pk.pkm_mlp_state_get(ctx, self.net)
        return {"rng_idx": _rng_state(self.rng_idx), "rng": _rng_state(self.rng),
                "net": net, "adam_t": np.int64(t), "losses": np.asarray(self.losses, float),
                "counters": np.array([self.train_s, self.fallbacks], float)}

    def restore(self, ctx, st):
        _set_rng_state(self.rng_idx, st["rng_idx"])
        _set_rng_state(self.rng, st["rng"])
        pk.pkm_mlp_state_set(ctx, self.net, st["net"], int(st["adam_t"]))
        self.losses = [float(v) for v in st["losses"]]
        self.train_s, self.fallbacks = float(st["counters"][0]), int(st["counters"][1])

    def close(self):
        pk.pkm_mlp_destroy(self.net)


class LowRankArm(Arm):
    """The factor form P = U U^T + lambda I (Section 3.2 with the factor
    learned) applied directly: the network is trained on probe pairs
    (Z, K Z) -- loss |U (U^T Z) - K Z|^2 / |K Z|^2 -- and its output is the
    factor of the matrix inversion lemma.  Kept as a comparison for the
    sketch form the learned arm uses; ``max_iter`` caps its solves (a poor
    factor may need many more steps than Nystrom)."""

    name = "lowrank"

    def __init__(self, ctx, params, d, rank, n, n_train_probes=64, first_steps=300,
                 steps_per_theta=50, lr=2e-3, seed=0, log=None, opts=None):
        self.net = pk.pkm_mlp_create(ctx, params, d, 128, rank)
        self.rank, self.nz, self.n = rank, n_train_probes, n
        self.first, self.later, self.lr = first_steps, steps_per_theta, lr
        self.rng = np.random.default_rng(seed + 7919)
        self.losses = []
        self.train_s = 0.0
        self.log = log
        self.opts = opts

    def setup(self, ctx, prob, step):
        import torch
        t0 = time.perf_counter()
        Z = torch.from_numpy(pk_rademacher(self.rng, prob.n, self.nz)).to(prob.X.device)
        R = pk.pkm_kernel_mvm_shift(ctx, prob, Z, 0.0, pk.PKM_FP32)   # K Z
        iters = self.first if step == 0 else self.later
        for _ in range(iters):
            self.losses.append(pk.pkm_mlp_train_step(ctx, self.net, prob, Z, R, self.lr))
        U = pk.pkm_mlp_forward(ctx, self.net, prob, self.rank)
        torch.cuda.synchronize()
        self.train_s += time.perf_counter() - t0
        return pk.pkm_precond_setup(ctx, prob, pk.PKM_PC_LOWRANK, self.rank, Phi=U)

    def state(self, ctx):
        net, t = pk.pkm_mlp_state_get(ctx, self.net)
        return {"rng": _rng_state(self.rng), "net": net, "adam_t": np.int64(t),
                "losses": np.asarray(self.losses, float), "train_s": np.float64(self.train_s)}

    def restore(self, ctx, st):
        _set_rng_state(self.rng, st["rng"])
        pk.pkm_mlp_state_set(ctx, self.net, st["net"], int(st["adam_t"]))
        self.losses = [float(v) for v in st["losses"]]
        self.train_s = float(st["train_s"])

    def close(self):
        pk.pkm_mlp_destroy(self.net)


def pk_rademacher(rng, n, N):
    return rng.integers(0, 2, size=(n, N)).astype(np.float64) * 2.0 - 1.0


def save_checkpoint(path, ctx, step, theta, G, traj, records, arms):
    """Everything ``run`` needs to continue after ``step`` completed steps,
    written atomically (a temporary file renamed over ``path``)."""
    arrays = {"step": np.int64(step), "theta": np.asarray(theta, float),
              "G": np.asarray(G, float), "traj": np.asarray(traj, float),
              "records": _pack_json(records),
              "arm_names": _pack_json([a.name for a in arms])}
    for arm in arms:
        for key, val in arm.state(ctx).items():
            arrays[f"arm.{arm.name}.{key}"] = val
    tmp = path + ".partial.npz"
    np.savez(tmp, **arrays)
    os.replace(tmp, path)


def load_checkpoint(path, ctx, arms):
    """(step, theta, G, traj, records) from ``path``; restores every arm's
    state.  The arms must be the ones the checkpoint was written with."""
    with np.load(path, allow_pickle=False) as f:
        names = _unpack_json(f["arm_names"])
        if names != [a.name for a in arms]:
            raise ValueError(f"checkpoint arms {names} differ from {[a.name for a in arms]}")
        for arm in arms:
            pre = f"arm.{arm.name}."
            arm.restore(ctx, {k[len(pre):]: f[k] for k in f.files if k.startswith(pre)})
        traj = [row.copy() for row in f["traj"]]
        return (int(f["step"]), f["theta"].copy(), f["G"].copy(), traj,
                _unpack_json(f["records"]))


def run(ctx, X, y, Z, theta0, lam, arms, steps, eta=1.0, opts=None, replay=None,
        log=None, checkpoint=None, max_wall_s=None):
    """Run ``steps`` ADAGRAD steps.  The first arm's gradient drives theta
    (or ``replay``, a recorded trajectory); every arm solves the same systems.
    Returns the theta trajectory and per-arm, per-step records.

    With ``checkpoint`` (a path), the state after every step is written
    there, and a run finding the file resumes after its last step.  With
    ``max_wall_s``, the run stops after the first step that ends past that
    many seconds; the trajectory returned is then shorter than steps + 1."""
    import torch
    opts = opts or pk.make_opts(tol=1e-6, prec=pk.PKM_F16X3)
    d = X.shape[1]
    theta = np.array(theta0, dtype=np.float64)
    G = np.zeros_like(theta)
    traj = [theta.copy()]
    records = {a.name: [] for a in arms}
    start = 0
    if checkpoint is not None and os.path.exists(checkpoint):
        start, theta, G, traj, records = load_checkpoint(checkpoint, ctx, arms)
        if log:
            log(f"resumed from {checkpoint} after step {start - 1}")
    N = Z.shape[1]
    sol = torch.zeros((X.shape[0], 1 + N), dtype=torch.float64, device=X.device)
    wall0 = time.perf_counter()
    for t in range(start, steps):
        if replay is not None:
            theta = np.array(replay[t], dtype=np.float64)
        s2, ls = unpack(theta)
        prob = pk.Problem(X, ls, s2, lam)
        grads = {}
        for arm in arms:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pc = arm.setup(ctx, prob, t)
            t1 = time.perf_counter()
            try:
                g, info = pk.pkm_lml_grad(ctx, prob, y, Z, pc=pc,
                                          opts=getattr(arm, "opts", None) or opts, sol=sol)
            finally:
                if pc is not None:
                    pk.pkm_precond_destroy(pc)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            grads[arm.name] = g
            rec = {"step": t, "setup_s": t1 - t0, "solve_grad_s": t2 - t1,
                   "iters": int(info.total_iters), "max_relres": float(info.relres_true.max()),
                   "converged": bool(np.all(info.col_status == pk.PKM_COL_CONVERGED))}
            records[arm.name].append(rec)
            if log:
                log(f"[{arm.name}] step {t}: iters {rec['iters']}, setup {rec['setup_s']:.3f} s, "
                    f"solve+grad {rec['solve_grad_s']:.3f} s, relres {rec['max_relres']:.1e}")
        if replay is None:
            g = grads[arms[0].name][: 1 + d]          # (log sigma2, log l_r); lambda fixed
            pk.pkm_adagrad_step(theta, g, G, eta=eta)
        traj.append(theta.copy())
        if checkpoint is not None:
            save_checkpoint(checkpoint, ctx, t + 1, theta, G, traj, records, arms)
        if max_wall_s is not None and time.perf_counter() - wall0 > max_wall_s:
            break
    return traj, records
