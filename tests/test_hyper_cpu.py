"""Host logic of the hyperparameter loop's checkpoints (no device work):
random streams and the run state survive a save / load round trip."""
import numpy as np
import pytest

from paper_1602_06693_amd import hyper


def test_nystrom_arm_stream_resumes_exactly(tmp_path):
    a = hyper.NystromArm(5000, 64, seed=3)
    for _ in range(3):
        a.rng.choice(a.n, size=a.m, replace=False)
    st = a.state(None)
    b = hyper.NystromArm(5000, 64, seed=99)
    b.restore(None, st)
    for _ in range(2):
        assert np.array_equal(a.rng.choice(a.n, size=a.m, replace=False),
                              b.rng.choice(b.n, size=b.m, replace=False))


def test_checkpoint_round_trip(tmp_path):
    arms = [hyper.NystromArm(100, 8, seed=1), hyper.NystromArm(100, 16, seed=2, name="ctrl")]
    arms[0].rng.random(5)
    theta = np.array([0.1, -0.2, 0.3])
    G = np.array([1.0, 2.0, 3.0])
    traj = [theta - 1.0, theta]
    records = {"nystrom": [{"step": 0, "iters": 12, "max_relres": 9.9e-7, "converged": True}],
               "ctrl": [{"step": 0, "iters": 10, "max_relres": 8.0e-7, "converged": True}]}
    path = str(tmp_path / "c.npz")
    hyper.save_checkpoint(path, None, 1, theta, G, traj, records, arms)
    fresh = [hyper.NystromArm(100, 8, seed=7), hyper.NystromArm(100, 16, seed=8, name="ctrl")]
    step, th, GG, tr, rec = hyper.load_checkpoint(path, None, fresh)
    assert step == 1 and np.array_equal(th, theta) and np.array_equal(GG, G)
    assert all(np.array_equal(u, v) for u, v in zip(tr, traj)) and len(tr) == 2
    assert rec == records
    assert np.array_equal(arms[0].rng.random(4), fresh[0].rng.random(4))
    assert np.array_equal(arms[1].rng.random(4), fresh[1].rng.random(4))
    with pytest.raises(ValueError):
        hyper.load_checkpoint(path, None, [hyper.NystromArm(100, 8, seed=1)])
