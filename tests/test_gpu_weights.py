"""GPU parity of the weighted index draws (eq. (18) with a general xi,
Theorem 3.1's xi**) against the oracle: the weights and the indices
bit-exactly; the matrix and inner-product estimates and the adjoint at the
tolerances of their precisions (FP64 1e-12, FP32 1e-5, BF16 0.05 RMSE_est,
BF16 adjoint 1e-2).  Each side computes its own xi** weights from the same
laws; their equality is tested first."""
import numpy as np
import pytest

from gpu_helpers import flush, laws, rel_frob

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _reparam(seed, n, m, p, spread=3.0):
    """Column-dependent reparameterised laws: A's mean scaled by a ramp over j."""
    rng = np.random.default_rng(seed)
    ramp = np.linspace(0.05, spread, n)[:, None]
    MA = (rng.standard_normal((n, m)) * ramp).astype(np.float32)
    SA = (rng.uniform(0.1, 1.0, (n, m)) * ramp).astype(np.float32)
    MB = rng.standard_normal((n, p)).astype(np.float32)
    SB = rng.uniform(0.1, 1.0, (n, p)).astype(np.float32)
    return MA, SA, MB, SB


def _both(orc, dev, MA, SA, MB, SB):
    oA, gA = laws(orc, ("reparam",), dev, MA, SA)
    oB, gB = laws(orc, ("reparam",), dev, MB, SB)
    return oA, gA, oB, gB


@pytest.mark.parametrize("n, m, p", [(37, 5, 3), (1000, 64, 17), (32768, 8, 8)])
def test_optimal_weights_bit_exact(orc, dev, n, m, p):
    from paper_1904_00429_amd import optimal_index_weights
    flush(f"[weights] optimal n={n} m={m} p={p}")
    oA, gA, oB, gB = _both(orc, dev, *_reparam(n, n, m, p))
    ref = orc.optimal_weights(m, n, p, oA, oB)
    got = optimal_index_weights(m, n, p, gA, gB, device=dev).cpu().numpy().view(np.uint32)
    assert np.array_equal(got, ref)
    # i.i.d. laws: uniform
    from paper_1904_00429_amd import Law
    w = optimal_index_weights(m, n, p, Law.normal(1.0, 2.0), Law.normal(0.0, 1.0), device=dev)
    assert torch.all(w == (1 << 24)).item()


@pytest.mark.parametrize("kind", ["ones", "skewed", "optimal"])
def test_weighted_indices_bit_exact(orc, dev, kind):
    from paper_1904_00429_amd import sample_indices_weighted
    n, c, S = 1234, 37, 50
    rng = np.random.default_rng(3)
    if kind == "ones":
        w = np.ones(n, dtype=np.uint32)
    elif kind == "skewed":
        w = (rng.pareto(1.0, n) * 1000 + 1).astype(np.uint32)
    else:
        oA, _, oB, _ = _both(orc, dev, *_reparam(4, n, 6, 5))
        w = orc.optimal_weights(6, n, 5, oA, oB)
    flush(f"[weights] indices {kind}")
    W = orc.Weights(w)
    got = sample_indices_weighted(9, 3, 2, 100, S, c, torch.from_numpy(w.view(np.int32)).to(dev)).cpu().numpy()
    for s in range(S):
        ref = [orc.draw_index_weighted(9, 3, 2, 100 + s, t, W) for t in range(c)]
        assert list(got[s]) == ref, s
    if kind == "ones":
        assert np.array_equal(got, np.stack([orc.draw_indices(9, 3, 2, 100 + s, c, n) for s in range(S)]))


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_matmul_weighted_matches_oracle(orc, dev, prec):
    from paper_1904_00429_amd import matmul_estimate, optimal_index_weights
    m, n, p, c, N = 37, 300, 45, [2, 4, 8], [200, 100, 50]
    flush(f"[weights] matmul {prec}")
    oA, gA, oB, gB = _both(orc, dev, *_reparam(7, n, m, p))
    ow = orc.Weights(orc.optimal_weights(m, n, p, oA, oB))
    gw = optimal_index_weights(m, n, p, gA, gB, device=dev)
    est = matmul_estimate(m, n, p, gA, gB, c, n_samples=N, seed=5, prec=prec, level_means=True, device=dev,
                          index_weights=gw)
    ref = orc.estimate(m, n, p, oA, oB, c, n_samples=N, seed=5, weights=ow)
    Y = est.Y.cpu().numpy()
    if prec == "bf16":
        err = np.linalg.norm((Y - ref.Y).ravel())
        flush(f"  bf16 error {err:.4g} vs rmse_est {ref.rmse_est:.4g}")
        assert err <= 0.05 * ref.rmse_est
        np.testing.assert_allclose(est.level_var, ref.level_var, rtol=3e-2)
        return
    tol = 1e-12 if prec == "fp64" else 1e-5
    assert rel_frob(Y, ref.Y) <= tol, rel_frob(Y, ref.Y)
    np.testing.assert_allclose(est.level_var, ref.level_var, rtol=1e-10 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_inner_weighted_matches_oracle(orc, dev, prec):
    from paper_1904_00429_amd import inner_product_estimate, optimal_index_weights
    n, c, N = 5000, [4, 8, 16, 32], [2000, 1000, 500, 250]
    flush(f"[weights] inner {prec}")
    rng = np.random.default_rng(11)
    ramp = np.linspace(0.01, 2.0, n)
    mx = (rng.standard_normal(n) * ramp).astype(np.float32)
    sx = (rng.uniform(0.1, 1.0, n) * ramp).astype(np.float32)
    my = rng.standard_normal(n).astype(np.float32)
    sy = rng.uniform(0.1, 1.0, n).astype(np.float32)
    ox, gx = laws(orc, ("reparam",), dev, mx, sx)
    oy, gy = laws(orc, ("reparam",), dev, my, sy)
    ow = orc.Weights(orc.optimal_weights(1, n, 1, ox, oy))
    gw = optimal_index_weights(1, n, 1, gx, gy, device=dev)
    assert np.array_equal(gw.cpu().numpy().view(np.uint32), ow.w)
    est = inner_product_estimate(n, gx, gy, c, n_samples=N, seed=8, prec=prec, level_means=True, device=dev,
                                 index_weights=gw)
    ref = orc.estimate(1, n, 1, ox, oy, c, n_samples=N, seed=8, weights=ow)
    tol = 1e-12 if prec == "fp64" else 1e-5
    Y = est.Y.cpu().numpy().reshape(ref.Y.shape)
    assert rel_frob(Y, ref.Y) <= tol, rel_frob(Y, ref.Y)
    np.testing.assert_allclose(est.level_var, ref.level_var, rtol=1e-10 if prec == "fp64" else 1e-5)


def test_unit_weights_reproduce_the_uniform_estimate(orc, dev):
    from paper_1904_00429_amd import matmul_estimate
    m, n, p, c, N = 200, 3000, 150, [4, 8, 16], [64, 32, 16]
    flush("[weights] unit weights = uniform")
    oA, gA, oB, gB = _both(orc, dev, *_reparam(2, n, m, p))
    ones = torch.ones(n, dtype=torch.int32, device=dev)
    a = matmul_estimate(m, n, p, gA, gB, c, n_samples=N, seed=3, prec="fp64", device=dev)
    b = matmul_estimate(m, n, p, gA, gB, c, n_samples=N, seed=3, prec="fp64", device=dev, index_weights=ones)
    assert torch.equal(a.Y, b.Y)


@pytest.mark.parametrize("prec, tol", [("fp32", 1e-5), ("bf16", 1e-2)])
def test_adjoint_weighted_matches_reference(orc, dev, prec, tol):
    from oracle import grad as og
    from paper_1904_00429_amd import matmul_adjoint_reparam, optimal_index_weights
    m, n, p, c, N = 24, 300, 17, [4, 8, 16], [20, 10, 5]
    flush(f"[weights] adjoint {prec}")
    params = _reparam(13, n, m, p)
    oA, gA, oB, gB = _both(orc, dev, *params)
    ow = orc.Weights(orc.optimal_weights(m, n, p, oA, oB))
    gw = optimal_index_weights(m, n, p, gA, gB, device=dev)
    G = np.random.default_rng(14).standard_normal((m, p))
    _, ref = og.reparam_gradients(*params, c, N, G, seed=2, weights=ow)
    dp = [torch.from_numpy(x).to(dev) for x in params]
    got = matmul_adjoint_reparam(*dp, c, N, torch.from_numpy(G), seed=2, prec=prec, index_weights=gw)
    for name, g, r in zip(("dMA", "dSA", "dMB", "dSB"), got, ref):
        err = rel_frob(g.cpu().numpy(), r)
        flush(f"  {name} rel err {err:.3g}")
        assert err <= tol, (name, err)
