"""The allocation-free inner-product entry point (its workspace is the
library's fixed per-GPU scratch array) gives the same estimate as
mlmc_inner_product_estimate with a caller workspace, bit for bit: the same
kernels run on the same draws in the same order.  Two calls in a row, the
second on a smaller input (shorter ladder, smaller n, fewer realisations), so
the second call runs on the first call's leftover scratch contents."""
import pytest

from gpu_helpers import flush

pytestmark = pytest.mark.gpu


def _pair(api, torch, dev, n, law, c, prec, seed, **kw):
    ref = api.inner_product_estimate(n, law, law, c, seed=seed, prec=prec, device=dev, level_means=True, **kw)
    out = torch.empty((), dtype=torch.float64, device=dev)
    means = torch.empty((len(c),), dtype=torch.float64, device=dev)
    got = api.inner_product_estimate_noalloc(n, law, law, c, seed=seed, prec=prec, out=out, level_means=means,
                                             **kw)
    torch.cuda.synchronize()
    return ref, got


def test_noalloc_matches_workspace_entry_point():
    import torch

    import paper_1904_00429_amd as api
    from paper_1904_00429_amd import Law
    dev = torch.device("cuda:0")
    cases = [
        # larger first: the 2^20 inner product in target mode (pilot, eq. (28), extension)
        dict(n=1 << 20, law=Law.uniform(0.5, 1.0), c=[64 * 2 ** l for l in range(9)], prec="fp32", seed=3,
             kw=dict(rmse_target=262.144 * 4, pilot=256, index_word32=True)),
        # then smaller: fewer levels, smaller n, fixed N_l, FP64
        dict(n=4099, law=Law.normal(1.0, 0.5), c=[4, 8, 16], prec="fp64", seed=5,
             kw=dict(n_samples=[300, 120, 40])),
    ]
    for case in cases:
        flush(f"noalloc: n={case['n']} levels={len(case['c'])} prec={case['prec']}")
        ref, got = _pair(api, torch, dev, case["n"], case["law"], case["c"], case["prec"], case["seed"],
                         **case["kw"])
        assert float(got.Y) == float(ref.Y)
        assert torch.equal(got.level_means, ref.level_means)
        assert got.n_used == ref.n_used
        assert got.level_var == ref.level_var
        assert got.rmse_est == ref.rmse_est


def test_noalloc_rejects_beyond_limit():
    import torch

    import paper_1904_00429_amd as api
    from paper_1904_00429_amd import Law, MLMCError
    dev = torch.device("cuda:0")
    n = (api._lib.lib().mlmc_inner_product_noalloc_limit() // 8) + 1024   # 8 n bytes of weights exceed it
    w = torch.ones(n, dtype=torch.int32, device=dev)
    out = torch.empty((), dtype=torch.float64, device=dev)
    with pytest.raises(MLMCError, match="allocation-free limit"):
        api.inner_product_estimate_noalloc(n, Law.normal(0.0, 1.0), Law.normal(0.0, 1.0), [4, 8],
                                           n_samples=[10, 10], out=out, index_weights=w)
