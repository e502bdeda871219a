"""Hyperparameter loop (Section 5): ADAGRAD steps driven by the library's
gradient match the oracle's trajectory (exact solves, same probes)."""
import math

import numpy as np
import pytest

from gpu_util import ctx, dev  # noqa: F401
from oracle import direct as od
from oracle import gradient as og
from oracle.adagrad import Adagrad
from paper_1602_06693_amd import binding as pk
from paper_1602_06693_amd import hyper
from pkm_inputs import make, mlp_params

pytestmark = pytest.mark.gpu


def test_adagrad_trajectory_matches_oracle(ctx):
    p = make("block_fp32", seed=31, n=1200, n_probes=8)
    d = p.d
    theta0 = hyper.theta_of(1.0, p.lengthscales)
    steps, eta = 3, 0.1
    arms = [hyper.NystromArm(p.n, 60, seed=1)]
    opts = pk.make_opts(tol=1e-10, prec=pk.PKM_FP64)
    traj, rec = hyper.run(ctx, dev(p.X), dev(p.y), dev(p.Z), theta0, p.lam, arms, steps,
                          eta=eta, opts=opts)
    # oracle: exact solves, the same probes, the oracle's ADAGRAD
    th = theta0.copy()
    ada = Adagrad(eta=eta)
    want = [th.copy()]
    for _ in range(steps):
        s2, ls = math.exp(th[0]), np.exp(th[1:])
        alpha = od.solve(p.X, s2, ls, p.lam, p.y)
        S = od.solve(p.X, s2, ls, p.lam, p.Z)
        g = og.hutchinson_gradient(p.X, s2, ls, p.lam, alpha, S, p.Z)[: 1 + d]
        th = ada.step(th, g)
        want.append(th.copy())
    for a, b in zip(traj, want):
        assert np.allclose(a, b, rtol=0, atol=1e-6), (a, b)
    assert all(r["converged"] for r in rec["nystrom"])


def test_learned_and_nystrom_arms_share_a_replayed_trajectory(ctx):
    p = make("learned", seed=2, n=3000, n_probes=4)
    d = p.d
    theta0 = hyper.theta_of(1.0, p.lengthscales)
    learned = hyper.LearnedArm(ctx, mlp_params(3, d_in=d, rank=32), d, 32, p.n, 128,
                               n_train_probes=32, first_steps=60, steps_per_theta=10, lr=3e-3,
                               seed=4)
    try:
        arms = [hyper.NystromArm(p.n, 128, seed=4), learned]
        traj, rec = hyper.run(ctx, dev(p.X), dev(p.y), dev(p.Z), theta0, p.lam, arms, 2,
                              eta=0.1, opts=pk.make_opts(tol=1e-6, prec=pk.PKM_FP32))
        assert learned.losses[-1] < learned.losses[0]
    finally:
        learned.close()
    for name in ("nystrom", "learned"):
        assert all(r["converged"] and r["max_relres"] <= 1e-6 for r in rec[name]), rec[name]
    assert len(traj) == 3


def test_learned_arm_falls_back_to_nystrom(ctx):
    """A network that explains none of the residual (zero output layer, Adam
    steps of 1e-30: loss 1) makes every step use plain Nystrom on the same inducing
    points, so the PCG step counts equal the Nystrom arm's exactly."""
    p = make("learned", seed=5, n=2500, n_probes=4)
    d = p.d
    theta0 = hyper.theta_of(1.0, p.lengthscales)
    learned = hyper.LearnedArm(ctx, mlp_params(3, d_in=d, rank=32, out_scale=0.0), d, 32, p.n,
                               128, n_train_probes=16, first_steps=2, steps_per_theta=2, lr=1e-30,
                               seed=4)
    try:
        arms = [hyper.NystromArm(p.n, 128, seed=4), learned]
        _, rec = hyper.run(ctx, dev(p.X), dev(p.y), dev(p.Z), theta0, p.lam, arms, 2,
                           eta=0.1, opts=pk.make_opts(tol=1e-8, prec=pk.PKM_FP64))
        assert learned.fallbacks == 2
    finally:
        learned.close()
    assert [r["iters"] for r in rec["learned"]] == [r["iters"] for r in rec["nystrom"]]
    assert all(r["converged"] for r in rec["learned"])


def test_checkpoint_resume_matches_uninterrupted_run(ctx, tmp_path):
    """Three ADAGRAD steps with the Nystrom, learned and low-rank arms, once
    straight through and once as 1 step + (fresh arms, resumed from the
    checkpoint) 2 steps: the same theta trajectory, PCG step counts and
    network training losses, bit for bit (the solves are deterministic)."""
    p = make("learned", seed=6, n=2000, n_probes=4)
    d = p.d
    theta0 = hyper.theta_of(1.0, p.lengthscales)
    opts = pk.make_opts(tol=1e-6, prec=pk.PKM_FP32)

    def arms_fresh():
        return [hyper.NystromArm(p.n, 96, seed=8),
                hyper.LearnedArm(ctx, mlp_params(3, d_in=d, rank=32), d, 32, p.n, 96,
                                 n_train_probes=16, first_steps=20, steps_per_theta=5,
                                 lr=3e-3, seed=8),
                hyper.LowRankArm(ctx, mlp_params(4, d_in=d, rank=32), d, 32, p.n,
                                 n_train_probes=16, first_steps=20, steps_per_theta=5,
                                 lr=3e-3, seed=8, opts=pk.make_opts(tol=1e-6, prec=pk.PKM_FP32,
                                                                   max_iter=3000))]

    def go(arms, steps, ckpt=None, max_wall=None):
        try:
            traj, rec = hyper.run(ctx, dev(p.X), dev(p.y), dev(p.Z), theta0, p.lam, arms,
                                  steps, eta=0.1, opts=opts, checkpoint=ckpt,
                                  max_wall_s=max_wall)
            return traj, rec, [list(a.losses) for a in arms[1:]]
        finally:
            for a in arms[1:]:
                a.close()

    traj_a, rec_a, loss_a = go(arms_fresh(), 3)
    ckpt = str(tmp_path / "hyper.npz")
    traj_1, _, _ = go(arms_fresh(), 3, ckpt=ckpt, max_wall=0.0)   # stops after one step
    assert len(traj_1) == 2
    traj_b, rec_b, loss_b = go(arms_fresh(), 3, ckpt=ckpt)
    assert len(traj_b) == 4
    for u, v in zip(traj_a, traj_b):
        assert np.array_equal(u, v), (u, v)
    for name in rec_a:
        assert [r["iters"] for r in rec_a[name]] == [r["iters"] for r in rec_b[name]], name
    assert loss_a == loss_b
