"""The allocation-free product entry point (pkm_kernel_mvm_noalloc): the
PKM_I8X product with every scratch byte in the library's static device array.
Checked against pkm_kernel_mvm with PKM_I8X (same kernels and launch shapes:
bit for bit) and against the FP64 oracle, on two calls in a row (the second
with a smaller input, so stale scratch from the first would show)."""
import numpy as np
import pytest

from gpu_util import ctx, dev, host, rel_err, torch_cuda  # noqa: F401
from oracle import kernel as ok
from paper_1602_06693_amd import binding as pk
from pkm_inputs import make

pytestmark = pytest.mark.gpu

TOL_EXACT = 2.0 ** -26   # the PKM_I8X bound against the exact product


def _case(seed, n, k):
    p = make("mixed", seed=seed, n=n, n_probes=k - 1)
    return p, pk.Problem(dev(p.X), p.lengthscales, p.sigma2, p.lam), dev(p.B)


def test_noalloc_matches_allocating_entry_point_twice(ctx):
    torch = torch_cuda()
    # every input and output tensor exists before free memory is first read
    cases = [_case(seed, n, k) for seed, n, k in ((41, 20000, 33), (42, 3001, 17))]
    outs = [torch.full_like(B, np.nan) for _, _, B in cases]
    # warm: first launches may load code objects in the runtime
    p0, prob0, B0 = _case(40, 300, 3)
    Y0 = torch.empty_like(B0)
    pk.pkm_kernel_mvm_noalloc(ctx, prob0, B0, Y0)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for (p, prob, B), Y in zip(cases, outs):   # the second call is the smaller one
        pk.pkm_kernel_mvm_noalloc(ctx, prob, B, Y)
        torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert free1 == free0, (free0, free1)   # the calls allocated nothing
    for (p, prob, B), Y in zip(cases, outs):
        got = host(Y)
        ref = host(pk.pkm_kernel_mvm(ctx, prob, B, pk.PKM_I8X))
        assert np.array_equal(got, ref)
        rows = np.random.default_rng(p.n).choice(p.n, size=48, replace=False)
        want = ok.kernel_mvm(p.X, p.sigma2, p.lengthscales, p.lam, p.B, rows=rows)
        assert rel_err(got[rows], want, axis=None) < TOL_EXACT


def test_noalloc_rejects_oversized_and_other_arithmetic(ctx):
    torch = torch_cuda()
    p, prob, B = _case(43, 200_000, 33)   # scratch far above the 128 MiB limit
    with pytest.raises(pk.PkmError) as e:
        pk.pkm_kernel_mvm_noalloc(ctx, prob, B, torch.empty_like(B))
    assert e.value.code == pk.PKM_ERR_INVALID
    assert "limit" in str(e.value)
    p, prob, B = _case(44, 500, 2)
    with pytest.raises(pk.PkmError) as e:
        pk.pkm_kernel_mvm_noalloc(ctx, prob, B, torch.empty_like(B), prec=pk.PKM_F16X3)
    assert e.value.code == pk.PKM_ERR_UNSUPPORTED


def test_noalloc_column_groups(ctx):
    """k = 70 takes three column groups of at most 33 through the same
    scratch (each group's digits and partial planes overwrite the last's):
    still bit-identical to the allocating entry point."""
    torch = torch_cuda()
    p, prob, B = _case(45, 9000, 70)
    Y = torch.full_like(B, np.nan)
    pk.pkm_kernel_mvm_noalloc(ctx, prob, B, Y)
    torch.cuda.synchronize()
    assert np.array_equal(host(Y), host(pk.pkm_kernel_mvm(ctx, prob, B, pk.PKM_I8X)))
