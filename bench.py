"""Benchmark: time to a 1e-6 relative-residual preconditioned CG solve on kernel
matrices, plus kernel-product TFLOP/s, on one MI355X.

One step is the whole hot path on one synthetic problem resident in HBM:
Nystrom preconditioner setup (m inducing points), PCG on the right-hand-side
block [y, Z] (Z: Rademacher probes) to a certified FP64 true relative
residual of 1e-6 with mixed-precision (BF16 MFMA) kernel products and FP64
residual replacement, and the Hutchinson gradient pass of the log-marginal
likelihood.  The same step with plain FP32 MFMA products is timed alongside
("plain") for the mixed-vs-plain comparison.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload block_fp32]

Prints one JSON line (rank 0).  ``value`` is the median step time in seconds
(lower is better).  The ``roofline`` object reports the kernel product (the
dominant kernel) from HIP events around each of its launches during the
timed steps; ``cpu_baseline`` times the FP64 CPU oracle on a
bounded sample of the same work.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("time to 1e-6 rel. residual PCG solve (mixed/learned vs plain); "
          "kernel-MVM TFLOP/s")
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_BF16_MFMA_TFLOPS = 2500.0   # dense
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
# Issue costs on gfx950 measured with throughput probes (cycles per wave64
# instruction at 2.4 GHz): a BF16 16x16x32 MFMA holds the SIMD's vector issue
# for about half of its 17 cycles, v_exp_f32 takes 8, a full-rate VALU op 4.
ISSUE_MFMA_HALF, ISSUE_EXP, ISSUE_VALU, SIMDS, CLOCK_HZ = 8.5, 8.0, 4.0, 1024, 2.4e9


# HBM bytes per launch of the dominant kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE runs, calibrated on a 1 GiB copy (FETCH_SIZE x 2.0, WRITE_SIZE
# x 1.0): (workload, product, n, k) -> bytes.  Valid while the kernel is
# unchanged since the counters were taken.
RECORDED_TRAFFIC = {("block_fp32", "f16x3", 65536, 17): (41858.1 * 2.0 + 34816.0) * 1024,
                    ("mixed", "i8x", 262144, 33): (6650373.9 * 2.0 + 540672.0) * 1024}


def _recorded_traffic(p, prec):
    return RECORDED_TRAFFIC.get((p.name, prec, p.n, p.B.shape[1]))


def bf16_issue_model_ms(n, d, k, prec):
    """Lower bound on a 16-bit product's time from its vector-issue budget:
    per 512 kernel entries (16 rows x 32 columns) and lane, 8 exp2 and the
    split's other VALU ops (BF16 split 3: 24; FP16 split 3: 16; split 1: 4),
    and 2 ceil((6 d + 6) / 32) exponent plus (3 or 1) ceil(k / 16) K V MFMAs
    (FP16 split 3: one fewer when the last 16-column tile holds at most 8
    columns) at half their duration."""
    s6 = -(-(6 * d + 6) // 32)
    kt = -(-k // 16)
    split3 = prec in ("bf16x3", "f16x3")
    mfma = 2 * s6 + (3 if split3 else 1) * kt
    if prec == "f16x3" and k - 16 * (kt - 1) <= 8:
        mfma -= 1   # merged last tile: (K_h + K_l) [V_h | V_l], two MFMAs
    valu = {"bf16x3": 24, "f16x3": 16}.get(prec, 4)
    cycles = 8 * ISSUE_EXP + valu * ISSUE_VALU + mfma * ISSUE_MFMA_HALF
    return (n * n / 512.0) * cycles / (SIMDS * CLOCK_HZ) * 1e3


_INPUTS = {
    "small_fp64": "X~U[0,1]^d, lengthscales 0.5",
    "block_fp32": "X~U[0,1]^d, ARD lengthscales LogU[0.1,1]",
    "mixed": "X~N(0,I_d), ARD lengthscales LogU[2,8]",
    "learned": "X~U[0,1]^d, lengthscales 0.5",
}


def _replacement(reliable):
    if reliable < 0:
        return (f"FP64 residual replacement every {-reliable} steps, doubling while the "
                f"true/recursive residual ratio stays <= 2 (up to {-8 * reliable})")
    return f"FP64 residual replacement every {reliable} steps"


def _describe(p, m, prec, reliable):
    return (f"{p.name}: n={p.n}, d={p.d}, {_INPUTS.get(p.name, '')}, "
            f"sigma2={p.sigma2}, lambda={p.lam}, k=1+{p.Z.shape[1]} (y + Rademacher probes), "
            f"Nystrom m={m}, tol={p.tol} (certified FP64 true residual), {prec} kernel "
            f"products, FP64 vectors, {_replacement(reliable)}; "
            f"step = preconditioner setup + block PCG solve + gradient pass")


def cpu_model():
    """The host CPU's model name (Linux /proc/cpuinfo), for the baseline record."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(p, gpu_iters, budget_rows=1024):
    """FP64 oracle on a bounded sample: product rows, setup, gradient rows."""
    from oracle import gradient as og
    from oracle import kernel as ok
    from oracle import precond as op

    threads = int(os.environ.get("PKM_ORACLE_THREADS", os.cpu_count() or 1))
    rng = np.random.default_rng(0)
    rows = np.sort(rng.choice(p.n, size=budget_rows, replace=False))
    B = p.B
    t0 = time.perf_counter()
    ok.kernel_mvm(p.X, p.sigma2, p.lengthscales, p.lam, B, rows=rows, threads=threads)
    t_rows = time.perf_counter() - t0
    t_mvm = t_rows * p.n / budget_rows
    t0 = time.perf_counter()
    P = op.nystrom(p.X, p.sigma2, p.lengthscales, p.lam, p.idx, jitter=1e-8)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    P(B)
    t_apply = time.perf_counter() - t0
    grows = budget_rows // 4
    t0 = time.perf_counter()
    sub = rows[:grows]
    # the gradient pass's work per row block, scaled to all rows
    og.bilinear_forms(p.X[sub], p.sigma2, p.lengthscales, p.lam, B[sub], B[sub])
    Kb_time = time.perf_counter() - t0
    t_grad = Kb_time * (p.n / grows) * (p.n / grows)
    total = t_setup + gpu_iters * (t_mvm + t_apply) + t_grad
    sample = (f"oracle kernel_mvm on {budget_rows} of {p.n} rows scaled x{p.n / budget_rows:.0f} "
              f"per product, x{gpu_iters} products (the GPU solve's step count); Nystrom setup "
              f"and one preconditioner apply timed in full; gradient forms on a "
              f"{grows}x{grows} block scaled by (n/{grows})^2; extrapolated, FP64")
    return {"value": total, "unit": "s", "cores": threads, "kind": "oracle",
            "sample": sample, "per_product_s": t_mvm, "setup_s": t_setup,
            "cpu_model": cpu_model()}


PEAK_INT8_MFMA_TOPS = 5000.0   # dense


def small_lambda_leg(pk, ctx, a):
    """One step of the 262,144-point mixed-precision workload (d = 16,
    lambda = 1e-4, k = 1 + 32, Nystrom m = 1024): preconditioner setup, block
    PCG to a certified FP64 true residual of 1e-6 and the gradient pass, with
    the FP64-class int8-digit product (PKM_I8X).  FP32-class products cannot
    certify this system (lambda / |K| ~ 1e-9); one step takes minutes, so it
    is timed once, after the headline arms."""
    import torch

    from pkm_inputs import make
    p = make("mixed", seed=a.seed)
    dev = lambda arr: torch.from_numpy(np.ascontiguousarray(arr)).to("cuda:0")
    X, y, Z, idx = dev(p.X), dev(p.y), dev(p.Z), dev(p.idx)
    N = p.Z.shape[1]
    sol = torch.zeros((p.n, 1 + N), dtype=torch.float64, device="cuda:0")
    prob = pk.Problem(X, p.lengthscales, p.sigma2, p.lam)
    opts = pk.make_opts(tol=p.tol, prec=pk.PKM_I8X, reliable_every=a.reliable)
    torch.cuda.synchronize()
    pk.pkm_mvm_stats_reset(ctx)
    pk.pkm_timing_enable(ctx, True)
    t0 = time.perf_counter()
    pc = pk.pkm_precond_setup(ctx, prob, pk.PKM_PC_NYSTROM, len(p.idx), idx=idx, jitter=1e-8)
    try:
        _, info = pk.pkm_lml_grad(ctx, prob, y, Z, pc=pc, opts=opts, sol=sol)
    finally:
        pk.pkm_precond_destroy(pc)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    pk.pkm_timing_enable(ctx, False)
    assert np.all(info.col_status == pk.PKM_COL_CONVERGED), info.col_status
    assert np.all(info.relres_true <= p.tol), info.relres_true.max()
    st = pk.pkm_mvm_stats(ctx, pk.PKM_I8X)
    st64 = pk.pkm_mvm_stats(ctx, pk.PKM_FP64)
    ms = st["ms"] / max(st["launches"], 1)
    fl = st["flops"] / max(st["launches"], 1)
    tf = fl / (ms * 1e-3) / 1e12
    print(f"[small-lambda i8x] step: {t:.1f} s, iters {info.total_iters}, true residuals "
          f"{info.true_residuals}, max relres {info.relres_true.max():.2e}, product {ms:.2f} ms",
          file=sys.stderr, flush=True)
    out = {"workload": _describe(p, len(p.idx), "i8x", a.reliable), "n": p.n, "d": p.d,
           "k": 1 + N, "m": len(p.idx), "product": "i8x", "steps": 1, "warmup": 0,
           "value": t, "unit": "s", "iters": int(info.total_iters),
           "true_residual_products": int(info.true_residuals),
           "prec_final": int(info.prec_final),
           "max_true_relres": float(info.relres_true.max()),
           "mvm_ms": ms, "mvm_tflops": tf,
           "fp64_true_residual_ms": st64["ms"] / max(st64["launches"], 1),
           "product_roofline": {
               "kernel": "k_mvm_i8 (FP64 MFMA exponent + FP64 table exp2 to 30-bit fixed point "
                         "+ int8 MFMA digit pairs, exact int32 sums)",
               "flops_per_launch": fl, "flop_count": "n^2 (2 d + 2 k) per product",
               "achieved": tf, "unit": "TFLOP/s",
               "frac_of_fp64_peak": tf / PEAK_FP64_TFLOPS,
               "frac_of_int8_peak": tf / PEAK_INT8_MFMA_TOPS,
               "traffic": _recorded_traffic(p, "i8x")}}
    if not a.no_cpu_baseline:
        from oracle import kernel as ok
        threads = int(os.environ.get("PKM_ORACLE_THREADS", os.cpu_count() or 1))
        rows = np.sort(np.random.default_rng(0).choice(p.n, size=256, replace=False))
        t1 = time.perf_counter()
        ok.kernel_mvm(p.X, p.sigma2, p.lengthscales, p.lam, p.B, rows=rows, threads=threads)
        per = (time.perf_counter() - t1) * p.n / len(rows)
        out["cpu_baseline"] = {"value": per * int(info.total_iters), "unit": "s",
                               "cores": threads, "kind": "oracle", "cpu_model": cpu_model(),
                               "sample": (f"oracle kernel_mvm on 256 of {p.n} rows, scaled to a "
                                          f"whole product ({per:.1f} s) and by the GPU solve's "
                                          f"{int(info.total_iters)} steps; extrapolated, FP64, "
                                          "setup and gradient not included")}
    return out


def mvm_only(pk, ctx, prob, p, steps, prec_names, ks):
    """Kernel products alone (k-sweep per arithmetic), then a 1 GiB calibration copy."""
    import torch
    precs = {"fp64": pk.PKM_FP64, "fp32": pk.PKM_FP32, "bf16x1": pk.PKM_BF16X1,
             "bf16x3": pk.PKM_BF16X3, "f16x3": pk.PKM_F16X3, "i8x": pk.PKM_I8X}
    rng = np.random.default_rng(1)
    for name in prec_names:
        prec = precs[name]
        for k in ks:
            V = torch.from_numpy(rng.standard_normal((p.n, k))).to("cuda:0")
            Y = torch.empty_like(V)
            pk.pkm_kernel_mvm(ctx, prob, V, prec, Y)
            pk.pkm_mvm_stats_reset(ctx)
            pk.pkm_timing_enable(ctx, True)
            for _ in range(steps):
                pk.pkm_kernel_mvm(ctx, prob, V, prec, Y)
            torch.cuda.synchronize()
            pk.pkm_timing_enable(ctx, False)
            st = pk.pkm_mvm_stats(ctx, prec)
            avg = st["ms"] / max(st["launches"], 1)
            print(json.dumps({"mode": "mvm", "prec": name, "n": p.n, "d": p.d, "k": k,
                              "launches": st["launches"], "avg_ms": avg,
                              "tflops": st["flops"] / max(st["ms"], 1e-9) * 1e-9,
                              "frac_bf16_peak": st["flops"] / max(st["ms"], 1e-9) * 1e-9
                              / PEAK_BF16_MFMA_TFLOPS}), flush=True)
    src = torch.empty(1 << 27, dtype=torch.float64, device="cuda:0")   # 1 GiB
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "copy", "bytes_read": src.numel() * 8,
                      "bytes_written": src.numel() * 8}), flush=True)


def hyper_mode(pk, ctx, p, a):
    """Section 5 loop: ADAGRAD steps on (log sigma2, log l); at every step the
    Nystrom arm (fresh m inducing points), the learned arm (the same inducing
    points enlarged by the factor network's r columns, fine-tuned on probe
    pairs (Z, (K - Q) Z)) and a control Nystrom arm with m + r inducing
    points solve the same systems; the Nystrom arm's gradient drives theta."""
    import torch

    from paper_1602_06693_amd import hyper
    from pkm_inputs import mlp_params
    dev = lambda arr: torch.from_numpy(np.ascontiguousarray(arr)).to("cuda:0")
    precs = {"fp64": pk.PKM_FP64, "fp32": pk.PKM_FP32, "bf16x1": pk.PKM_BF16X1,
             "bf16x3": pk.PKM_BF16X3, "f16x3": pk.PKM_F16X3, "i8x": pk.PKM_I8X}
    opts = pk.make_opts(tol=p.tol, prec=precs[a.prec], reliable_every=a.reliable)
    theta0 = hyper.theta_of(p.sigma2, p.lengthscales)
    log = lambda msg: print(msg, file=sys.stderr, flush=True)
    m = len(p.idx)
    learned = hyper.LearnedArm(ctx, mlp_params(a.seed, d_in=p.d, rank=a.rank, out_scale=0.1),
                               p.d, a.rank, p.n, m, seed=a.seed, log=log)
    arms = [hyper.NystromArm(p.n, m, seed=a.seed), learned]
    if not a.no_control:   # as many extra random inducing points as the learned columns
        arms.append(hyper.NystromArm(p.n, m + a.rank, seed=a.seed, name=f"nystrom_m{m + a.rank}"))
    if a.lowrank_arm:   # the plain factor form P = U U^T + lambda I, capped solves
        arms.append(hyper.LowRankArm(
            ctx, mlp_params(a.seed, d_in=p.d, rank=a.rank, out_scale=0.1), p.d, a.rank, p.n,
            seed=a.seed, log=log,
            opts=pk.make_opts(tol=p.tol, prec=precs[a.prec], reliable_every=a.reliable,
                              max_iter=a.lowrank_max_iter)))
    t0 = time.perf_counter()
    try:
        traj, rec = hyper.run(ctx, dev(p.X), dev(p.y), dev(p.Z), theta0, p.lam, arms,
                              a.hyper_steps, eta=1.0, opts=opts, log=log,
                              checkpoint=a.checkpoint, max_wall_s=a.max_wall)
    finally:
        learned.close()
        if a.lowrank_arm:
            arms[-1].close()
    wall = time.perf_counter() - t0
    out = {"mode": "hyper", "workload": p.name, "n": p.n, "d": p.d, "k": 1 + p.Z.shape[1],
           "lambda": p.lam, "steps": a.hyper_steps, "steps_done": len(traj) - 1,
           "product": a.prec, "wall_s_this_call": wall,
           "theta_final": [float(v) for v in traj[-1]], "learned_rank": a.rank,
           "nystrom_m": len(p.idx), "mlp_train_s": learned.train_s,
           "mlp_loss_first_last": [learned.losses[0], learned.losses[-1]],
           "learned_fallbacks": learned.fallbacks,
           "theta_trajectory": [[float(v) for v in th] for th in traj]}
    for name, rs in rec.items():
        out[name] = {"iters": [r["iters"] for r in rs],
                     "solve_grad_s": sum(r["solve_grad_s"] for r in rs),
                     "setup_s": sum(r["setup_s"] for r in rs),
                     "all_converged": all(r["converged"] for r in rs),
                     "max_relres": max(r["max_relres"] for r in rs)}
    print(json.dumps(out), flush=True)


def batched_mode(pk, ctx, a):
    """Many independent GP problems (uneven n, d, theta, lambda; 1 + 8 columns
    each): Nystrom setup for every problem, then one batched solve, against
    the same problems solved one after another with the single-problem
    solver.  Both to a certified FP64 true relative residual of 1e-6."""
    import torch

    from pkm_inputs import batched_problems
    probs = batched_problems(seed=a.seed, count=a.count)
    dev = lambda arr: torch.from_numpy(np.ascontiguousarray(arr)).to("cuda:0")
    prec = {"fp32": pk.PKM_FP32, "fp64": pk.PKM_FP64, "f16x3": pk.PKM_F16X3}[
        a.prec if a.prec in ("fp32", "fp64", "f16x3") else "fp32"]
    gps = [pk.Problem(dev(p.X), p.lengthscales, p.sigma2, p.lam) for p in probs]
    Bs = [dev(p.B) for p in probs]
    idxs = [dev(p.idx) for p in probs]
    # max_iter 20000: a solve that cannot reach the tolerance ends (and reports
    # it) instead of running the library default of 100000 steps
    # both arms replace every |reliable| steps (the batched solver has no
    # adaptive period), so the comparison is like for like
    opts = pk.make_opts(tol=1e-6, prec=prec, reliable_every=abs(a.reliable), max_iter=20000)
    log = lambda msg: print(msg, file=sys.stderr, flush=True)

    def setups():
        return [pk.pkm_precond_setup(ctx, g, pk.PKM_PC_NYSTROM, len(p.idx), idx=ix, jitter=1e-8)
                for p, g, ix in zip(probs, gps, idxs)]

    def batched_step():
        pcs = setups()
        try:
            Xs, infos, rc = pk.pkm_solve_batched(ctx, gps, Bs, pcs=pcs, opts=opts)
        finally:
            for pc in pcs:
                pk.pkm_precond_destroy(pc)
        return infos, rc

    def sequential_step():
        infos = []
        for p, g, b, ix in zip(probs, gps, Bs, idxs):
            pc = pk.pkm_precond_setup(ctx, g, pk.PKM_PC_NYSTROM, len(p.idx), idx=ix, jitter=1e-8)
            try:
                infos.append(pk.pkm_solve(ctx, g, b, pc=pc, opts=opts)[1])
            finally:
                pk.pkm_precond_destroy(pc)
        return infos

    def timed(fn, label):
        for _ in range(a.warmup):
            fn()
        torch.cuda.synchronize()
        pk.pkm_mvm_stats_reset(ctx)
        pk.pkm_timing_enable(ctx, label == "batched")
        ts, res = [], None
        for i in range(a.steps):
            t0 = time.perf_counter()
            res = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
            log(f"[{label}] step {i + 1}: {ts[-1]:.3f} s")
        pk.pkm_timing_enable(ctx, False)
        return statistics.median(ts), res

    t_b, (infos_b, rc) = timed(batched_step, "batched")
    st = pk.pkm_mvm_stats(ctx, prec)
    t_s, infos_s = timed(sequential_step, "sequential")
    ok_b = all(np.all(i.col_status == pk.PKM_COL_CONVERGED) and np.all(i.relres_true <= 1e-6)
               for i in infos_b)
    ok_s = all(np.all(i.col_status == pk.PKM_COL_CONVERGED) and np.all(i.relres_true <= 1e-6)
               for i in infos_s)
    out = {"mode": "batched", "problems": len(probs), "k": 1 + probs[0].Z.shape[1],
           "product": a.prec, "sum_n": int(sum(p.n for p in probs)),
           "sum_n2": float(sum(float(p.n) ** 2 for p in probs)),
           "dims": sorted({p.d for p in probs}),
           "batched_s": t_b, "sequential_s": t_s, "speedup": t_s / t_b,
           "all_certified_batched": bool(ok_b), "all_certified_sequential": bool(ok_s),
           "max_relres_batched": float(max(i.relres_true.max() for i in infos_b)),
           "raised_to_fp64": int(sum(i.prec_final == pk.PKM_FP64 for i in infos_b))
           if prec != pk.PKM_FP64 else None,
           "iters_batched": [int(i.iters.max()) for i in infos_b],
           "iters_sequential": [int(i.iters.max()) for i in infos_s],
           "batched_product_ms": st["ms"] / max(st["launches"], 1),
           "batched_product_tflops": st["flops"] / max(st["ms"], 1e-9) * 1e-9,
           "batched_product_launches": st["launches"] // max(a.steps, 1)}
    print(json.dumps(out), flush=True)


def laplace_mode(pk, ctx, a):
    """GP classification by the Laplace approximation (probit): Newton mode,
    stochastic gradient (16 Rademacher probes) and predictive probabilities
    at 128 test inputs, with every B = I + W^1/2 K W^1/2 system solved by PCG
    with the Nystrom-derived preconditioner, then by plain CG."""
    import torch

    from pkm_inputs import classification, rademacher
    n = a.n or 16384
    X, y, ls, s2, idx = classification(seed=a.seed, n=n, d=14)
    dev = lambda arr: torch.from_numpy(np.ascontiguousarray(arr)).to("cuda:0")
    prob = pk.Problem(dev(X), ls, s2, 1.0)
    yd = dev(y)
    R = dev(rademacher(np.random.default_rng(a.seed + 1), n, 16))
    Xs = dev(np.random.default_rng(a.seed + 2).random((128, 14)))
    precs = {"fp64": pk.PKM_FP64, "fp32": pk.PKM_FP32, "bf16x3": pk.PKM_BF16X3, "f16x3": pk.PKM_F16X3, "i8x": pk.PKM_I8X}
    # B solves to 1e-8 so that the Newton iterations reach the same mode in
    # both arms (Newton stops when Psi changes by <= 1e-10 relative)
    opts = pk.make_opts(tol=1e-8, prec=precs.get(a.prec, pk.PKM_FP64), reliable_every=a.reliable)
    out = {"mode": "laplace", "n": n, "d": 14, "m": len(idx), "probes": 16, "test_points": 128,
           "product": a.prec if a.prec in precs else "fp64", "tol": 1e-8, "newton_tol": 1e-10}
    for label, use_pc in (("nystrom", True), ("plain", False)):
        for rep in range(a.warmup + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pc = (pk.pkm_precond_setup(ctx, prob, pk.PKM_PC_NYSTROM, len(idx), idx=dev(idx),
                                       jitter=1e-8) if use_pc else None)
            try:
                f, _, info = pk.pkm_laplace_mode(ctx, prob, yd, pc=pc, opts=opts, tol=1e-10)
                t1 = time.perf_counter()
                g, gsteps = pk.pkm_laplace_grad(ctx, prob, yd, f, R, pc=pc, opts=opts)
                t2 = time.perf_counter()
                m, v, p = pk.pkm_laplace_predict(ctx, prob, yd, f, Xs, pc=pc, opts=opts)
                torch.cuda.synchronize()
                t3 = time.perf_counter()
            finally:
                if pc is not None:
                    pk.pkm_precond_destroy(pc)
        out[label] = {"total_s": t3 - t0, "mode_s": t1 - t0, "grad_s": t2 - t1,
                      "predict_s": t3 - t2, "newton_iters": info.newton_iters,
                      "mode_pcg_steps": int(info.pcg_steps), "grad_pcg_steps": int(gsteps),
                      "psi": info.psi, "grad": [float(v) for v in g]}
        print(f"[laplace {label}] {out[label]['total_s']:.3f} s", file=sys.stderr, flush=True)
    out["speedup_nystrom_vs_plain"] = out["plain"]["total_s"] / out["nystrom"]["total_s"]
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="block_fp32")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--prec", default=None, choices=("fp32", "bf16x3", "bf16x1", "f16x3", "fp64",
                                                     "i8x"),
                    help="arithmetic of the kernel product inside the loop (the mixed path); "
                         "default f16x3, fp64 for --mode laplace (its 1e-8 solves sit below "
                         "what 16-bit products refine to quickly)")
    ap.add_argument("--alt", default="none", choices=("fp32", "bf16x3", "bf16x1", "f16x3", "fp64",
                                                        "i8x", "none"),
                    help="also time this mixed arithmetic (reported beside the headline)")
    ap.add_argument("--plain", default="fp32", choices=("fp32", "fp64", "i8x", "none"),
                    help="also time this product arithmetic for the mixed-vs-plain comparison")
    ap.add_argument("--rsvd", action="store_true",
                    help="step mode: also time the step with the randomised truncated SVD "
                         "preconditioner of the same rank (one power iteration, FP32 sketch)")
    ap.add_argument("--fitc", action=argparse.BooleanOptionalAction, default=False,
                    help="step mode: also time the mixed step with FITC (same m and points)")
    ap.add_argument("--small-lambda", action=argparse.BooleanOptionalAction, default=True,
                    help="step mode on the default workload: also time one step of the "
                         "262,144-point lambda = 1e-4 workload with int8-digit products")
    ap.add_argument("--reliable", type=int, default=-50,
                    help="FP64 replacement period; negative: adaptive from its magnitude")
    ap.add_argument("--ks", default="", help="mvm mode: comma-separated column counts")
    ap.add_argument("--mvm-precs", default="f16x3",
                    help="mvm mode: comma-separated arithmetics (fp64,fp32,bf16x1,bf16x3,f16x3)")
    ap.add_argument("--hyper-steps", type=int, default=20)
    ap.add_argument("--n", type=int, default=None, help="override the workload's n")
    ap.add_argument("--rank", type=int, default=128)
    ap.add_argument("--lowrank-arm", action="store_true",
                    help="hyper mode: also solve with P = U U^T + lambda I from the network "
                         "trained on (Z, K Z)")
    ap.add_argument("--lowrank-max-iter", type=int, default=15000)
    ap.add_argument("--psi32", action="store_true",
                    help="step mode: the first arm applies the preconditioner from Psi rounded "
                         "to FP32 (pkm_precond_psi_f32)")
    ap.add_argument("--no-control", action="store_true",
                    help="hyper mode: leave out the Nystrom m + rank control arm")
    ap.add_argument("--checkpoint", default=None,
                    help="hyper mode: .npz written after every step; resumed from if present")
    ap.add_argument("--max-wall", type=float, default=None,
                    help="hyper mode: stop after the first step ending past this many seconds")
    ap.add_argument("--count", type=int, default=64, help="batched mode: number of problems")
    ap.add_argument("--mode", choices=("step", "mvm", "hyper", "batched", "laplace"),
                    default="step",
                    help="mvm: only --steps FP32 kernel products of the workload's size, "
                         "then one 1 GiB device copy (counter calibration for profiles)")
    a = ap.parse_args()
    if a.prec is None:
        a.prec = "fp64" if a.mode == "laplace" else "f16x3"
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the rows of the product would shard over GPUs with an all-gather of V).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1602_06693_amd import binding as pk
    from pkm_inputs import make

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    p = make(a.workload, seed=a.seed, n=a.n)
    m = len(p.idx)
    N = p.Z.shape[1]
    dev = lambda arr: torch.from_numpy(np.ascontiguousarray(arr)).to("cuda:0")
    X, y, Z, idx = dev(p.X), dev(p.y), dev(p.Z), dev(p.idx)
    sol = torch.zeros((p.n, 1 + N), dtype=torch.float64, device="cuda:0")
    ctx = pk.pkm_create(0, pk.current_stream_handle())
    prob = pk.Problem(X, p.lengthscales, p.sigma2, p.lam)
    if a.mode == "hyper":
        hyper_mode(pk, ctx, p, a)
        pk.pkm_destroy(ctx)
        return
    if a.mode == "batched":
        batched_mode(pk, ctx, a)
        pk.pkm_destroy(ctx)
        return
    if a.mode == "laplace":
        laplace_mode(pk, ctx, a)
        pk.pkm_destroy(ctx)
        return
    if a.mode == "mvm":
        ks = [int(v) for v in a.ks.split(",")] if a.ks else [1 + N]
        mvm_only(pk, ctx, prob, p, a.steps, a.mvm_precs.split(","), ks)
        pk.pkm_destroy(ctx)
        return

    precs = {"fp64": pk.PKM_FP64, "fp32": pk.PKM_FP32, "bf16x1": pk.PKM_BF16X1,
             "bf16x3": pk.PKM_BF16X3, "f16x3": pk.PKM_F16X3, "i8x": pk.PKM_I8X}

    def run_variant(prec, steps, warmup, label, kind=None, psi32=False):
        opts = pk.make_opts(tol=p.tol, prec=prec, reliable_every=a.reliable)
        kind = pk.PKM_PC_NYSTROM if kind is None else kind

        setup_s = []

        def step():
            if kind == "rsvd":   # randomised truncated SVD, rank m, 20 oversampling columns
                torch.cuda.synchronize()   # the setup waits for the device itself (host eigensolver)
                t0 = time.perf_counter()
                pc = pk.pkm_precond_setup_rsvd(ctx, prob, m, omega, q=1, prec=pk.PKM_F16X3)
                torch.cuda.synchronize()
                setup_s.append(time.perf_counter() - t0)
            else:
                pc = pk.pkm_precond_setup(ctx, prob, kind, m, idx=idx, jitter=1e-8)
            try:
                if psi32:
                    pk.pkm_precond_psi_f32(ctx, pc, True)
                return pk.pkm_lml_grad(ctx, prob, y, Z, pc=pc, opts=opts, sol=sol)
            finally:
                pk.pkm_precond_destroy(pc)

        all_infos = []   # every step, warmup included, must certify
        for _ in range(warmup):
            all_infos.append(step()[1])
        torch.cuda.synchronize()
        pk.pkm_mvm_stats_reset(ctx)
        pk.pkm_timing_enable(ctx, True)
        times, infos = [], []
        torch.cuda.synchronize()
        t_all = time.perf_counter()
        for _ in range(steps):
            t0 = time.perf_counter()
            g, info = step()
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            infos.append(info)
            print(f"[{label}] step {len(times)}: {times[-1]:.3f} s, iters {info.total_iters}, "
                  f"true residuals {info.true_residuals}, max relres "
                  f"{info.relres_true.max():.2e}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t_all = time.perf_counter() - t_all
        pk.pkm_timing_enable(ctx, False)
        info = infos[-1]
        for i_ in all_infos + infos:
            assert np.all(i_.col_status == pk.PKM_COL_CONVERGED), i_.col_status
            assert np.all(i_.relres_true <= p.tol), i_.relres_true.max()
        max_rel = float(max(i_.relres_true.max() for i_ in all_infos + infos))
        st = pk.pkm_mvm_stats(ctx, prec)
        st64 = pk.pkm_mvm_stats(ctx, pk.PKM_FP64)
        avg_ms = st["ms"] / max(st["launches"], 1)
        return {"times": times, "t_all": t_all, "info": info, "max_rel": max_rel, "mvm_ms": avg_ms,
                "flops_per_launch": st["flops"] / max(st["launches"], 1),
                "tflops": st["flops"] / max(st["launches"], 1) / (avg_ms * 1e-3) / 1e12,
                "fp64_ms": st64["ms"] / max(st64["launches"], 1),
                "fp64_launches": st64["launches"] // max(steps, 1),
                "setup_s": statistics.median(setup_s[warmup:]) if len(setup_s) > warmup else None}

    mixed = run_variant(precs[a.prec], a.steps, a.warmup, a.prec + ("+psi32" if a.psi32 else ""),
                        psi32=a.psi32)
    plain = None
    if a.plain != "none" and a.plain != a.prec:
        plain = run_variant(precs[a.plain], a.steps, a.warmup, a.plain)
    alt = None
    if a.alt != "none" and a.alt not in (a.prec, a.plain):
        alt = run_variant(precs[a.alt], a.steps, a.warmup, a.alt)
    fitc = None
    if a.fitc:   # the same step with the FITC preconditioner (same inducing points)
        fitc = run_variant(precs[a.prec], a.steps, a.warmup, a.prec + "+fitc", pk.PKM_PC_FITC)
    rsvd = None
    if a.rsvd:   # the same step with the randomised truncated SVD of the same rank
        omega = torch.from_numpy(np.random.default_rng(a.seed + 17).standard_normal(
            (p.n, m + 20))).to("cuda:0")
        rsvd = run_variant(precs[a.prec], a.steps, a.warmup, a.prec + "+rsvd", "rsvd")
    small = None
    if a.small_lambda and a.workload == "block_fp32" and a.n is None:
        small = small_lambda_leg(pk, ctx, a)
    pk.pkm_destroy(ctx)

    info = mixed["info"]
    value = statistics.median(mixed["times"])
    bf16 = a.prec in ("bf16x1", "bf16x3", "f16x3")   # 16-bit MFMA products (same dense peak)
    peak = PEAK_BF16_MFMA_TFLOPS if bf16 else (PEAK_FP64_TFLOPS if a.prec == "fp64"
                                                 else PEAK_FP32_MFMA_TFLOPS)
    kname = {"fp32": "k_mvm_f32 (FP32 MFMA distance + exp2 + FP32 MFMA K V)",
             "bf16x3": "k_mvm_bf16<NP=3> (BF16x6-split distance + exp2 + BF16x3 K V, FP32 acc)",
             "bf16x1": "k_mvm_bf16<NP=1> (BF16x6-split distance + exp2 + BF16 K V, FP32 acc)",
             "f16x3": "k_mvm_bf16<NP=4> (BF16x6-split distance + exp2 + FP16x3 K V, FP32 acc)",
             "fp64": "k_mvm_f64x (FP64 MFMA distance + table exp2 + FP64 MFMA K V)"}[a.prec]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * mixed["t_all"] / a.steps,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("f16" if a.prec == "f16x3" else "bf16") if bf16 else (
            "f64" if a.prec == "fp64" else "f32"),
        "data": "synthetic",
        "config": {"workload": _describe(p, m, a.prec, a.reliable), "n": p.n, "d": p.d,
                   "k": 1 + N, "m": m, "preconditioner": "nystrom", "product": a.prec,
                   "psi_storage": "fp32" if a.psi32 else "fp64",
                   "parallelism": "single GPU"},
        "iters": int(info.total_iters),
        "true_residual_products": int(info.true_residuals),
        "max_true_relres": mixed["max_rel"],
        "mvm_tflops": mixed["tflops"],
        "mvm_ms": mixed["mvm_ms"],
        "fp64_true_residual_ms": mixed["fp64_ms"],
        "roofline": {"bound": "mfma", "achieved": mixed["tflops"], "peak": peak,
                     "unit": "TFLOP/s", "frac": mixed["tflops"] / peak,
                     "traffic": _recorded_traffic(p, a.prec),
                     "kernel": kname, "flops_per_launch": mixed["flops_per_launch"],
                     "flop_count": "n^2 (2 d + 2 k) per product"},
    }
    if bf16:   # the product's actual bound: vector-ALU issue (exp2, splits) + MFMA issue
        model = bf16_issue_model_ms(p.n, p.d, p.B.shape[1], a.prec)
        out["roofline"]["issue_bound"] = {
            "model_ms": model, "achieved_ms": mixed["mvm_ms"], "frac": model / mixed["mvm_ms"],
            "model": "per 512 entries and lane: 8 exp2 x 8 cycles + (24|16|4) VALU x 4 "
                     "(BF16x3|FP16x3|x1 splits) + MFMAs x 8.5 (half of 17), over 1024 SIMDs "
                     "at 2.4 GHz"}
    if plain is not None:
        out["plain"] = {"product": a.plain, "value": statistics.median(plain["times"]),
                        "iters": int(plain["info"].total_iters),
                        "true_residual_products": int(plain["info"].true_residuals),
                        "mvm_ms": plain["mvm_ms"], "mvm_tflops": plain["tflops"]}
        out["speedup_vs_plain"] = out["plain"]["value"] / value
    if rsvd is not None:
        out["rsvd"] = {"product": a.prec, "preconditioner": f"randomised SVD r={m}, l={m + 20}, q=1, FP16x3 sketch products",
                       "value": statistics.median(rsvd["times"]),
                       "setup_s": rsvd["setup_s"],
                       "iters": int(rsvd["info"].total_iters),
                       "true_residual_products": int(rsvd["info"].true_residuals),
                       "max_true_relres": rsvd["max_rel"]}
    if fitc is not None:
        out["fitc"] = {"product": a.prec, "preconditioner": "fitc",
                       "value": statistics.median(fitc["times"]),
                       "iters": int(fitc["info"].total_iters),
                       "true_residual_products": int(fitc["info"].true_residuals),
                       "max_true_relres": fitc["max_rel"]}
    if alt is not None:
        out["alt"] = {"product": a.alt, "value": statistics.median(alt["times"]),
                      "iters": int(alt["info"].total_iters),
                      "true_residual_products": int(alt["info"].true_residuals),
                      "max_true_relres": alt["max_rel"],
                      "mvm_ms": alt["mvm_ms"], "mvm_tflops": alt["tflops"]}
    if small is not None:
        out["small_lambda"] = small
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, int(info.total_iters))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
