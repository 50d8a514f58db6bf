"""Pins of the gradient reference (oracle/grad.py) for the reparameterised
estimator: its forward equals the C oracle's estimate, its gradients equal
central finite differences (the estimate is affine in every single parameter
and bilinear overall, so central differences are exact up to rounding), and
the seed-average of the gradient of a linear functional <G0, Y> matches the
closed form of grad <G0, E[AB]> = (M_B G0^T, 0, M_A G0, 0) (store layouts:
rows j), E[AB] = M_A M_B being the mean of the product (the estimator is
unbiased, Sec. 3)."""
import math

import numpy as np
import pytest
import torch


@pytest.fixture(scope="module")
def grad_mod(orc):
    from oracle import grad
    return grad


def _params(rng, n, m, p):
    return (rng.normal(size=(n, m)), rng.uniform(0.1, 1, (n, m)),
            rng.normal(size=(n, p)), rng.uniform(0.1, 1, (n, p)))


def test_forward_equals_c_oracle(orc, grad_mod):
    rng = np.random.default_rng(1)
    n, m, p, c, N = 60, 4, 3, [3, 6, 12], [25, 12, 6]
    MA, SA, MB, SB = _params(rng, n, m, p)
    Y = grad_mod.reparam_estimate(*[torch.from_numpy(x) for x in (MA, SA, MB, SB)], c, N, seed=9)
    est = orc.estimate(m, n, p, orc.Law.reparam(MA.ravel(), SA.ravel(), m),
                       orc.Law.reparam(MB.ravel(), SB.ravel(), p), c, n_samples=N, seed=9)
    np.testing.assert_allclose(Y.numpy(), est.Y, rtol=1e-13, atol=1e-13 * np.abs(est.Y).max())


def test_gradients_match_finite_differences(grad_mod):
    rng = np.random.default_rng(2)
    n, m, p, c, N = 30, 3, 2, [2, 4], [10, 5]
    params = list(_params(rng, n, m, p))
    G = rng.normal(size=(m, p))
    _, grads = grad_mod.reparam_gradients(*params, c, N, G, seed=4)

    def L(ps):
        Y = grad_mod.reparam_estimate(*[torch.from_numpy(x) for x in ps], c, N, seed=4)
        return float((Y.numpy() * G).sum())

    h = 1e-3
    for which in range(4):
        for _ in range(4):
            idx = tuple(rng.integers(0, s) for s in params[which].shape)
            plus = [x.copy() for x in params]
            minus = [x.copy() for x in params]
            plus[which][idx] += h
            minus[which][idx] -= h
            fd = (L(plus) - L(minus)) / (2 * h)
            assert abs(fd - grads[which][idx]) <= 1e-7 * (1 + abs(fd)), (which, idx, fd, grads[which][idx])
    # one random direction through all four parameters (second order, still exact for central FD)
    d = [rng.normal(size=x.shape) for x in params]
    plus = [x + h * dx for x, dx in zip(params, d)]
    minus = [x - h * dx for x, dx in zip(params, d)]
    fd = (L(plus) - L(minus)) / (2 * h)
    an = sum(float((g * dx).sum()) for g, dx in zip(grads, d))
    assert abs(fd - an) <= 1e-7 * (1 + abs(fd))


def test_expected_gradient_of_linear_functional(grad_mod):
    rng = np.random.default_rng(3)
    n, m, p, c, N = 12, 3, 2, [2, 4], [12, 6]
    MA, SA, MB, SB = _params(rng, n, m, p)
    G0 = rng.normal(size=(m, p))
    seeds = 300
    acc = [[] for _ in range(4)]
    for s in range(seeds):
        _, g = grad_mod.reparam_gradients(MA, SA, MB, SB, c, N, G0, seed=1000 + s)
        for i in range(4):
            acc[i].append(g[i])
    expected = [MB @ G0.T, np.zeros_like(SA), MA @ G0, np.zeros_like(SB)]
    for i in range(4):
        a = np.array(acc[i])
        mean = a.mean(axis=0)
        se = a.std(axis=0, ddof=1) / math.sqrt(seeds) + 1e-12
        z = np.abs(mean - expected[i]) / se
        assert z.max() < 5.0, (i, z.max())


@pytest.mark.parametrize("coupling", ["prefix", "stride"])
def test_restricted_gradient_equals_full_rows(coupling):
    """The entry-restricted gradient equals the full autograd gradient at the
    chosen rows (including rows no draw hit, whose gradient is 0)."""
    from oracle import grad as og
    rng = np.random.default_rng(5)
    m, n, p, c, N = 7, 23, 5, [2, 4, 8], [12, 6, 3]
    MA, MB = rng.standard_normal((n, m)), rng.standard_normal((n, p))
    SA, SB = rng.uniform(0.1, 1, (n, m)), rng.uniform(0.1, 1, (n, p))
    G = rng.standard_normal((m, p))
    _, full = og.reparam_gradients(MA, SA, MB, SB, c, N, G, seed=4, coupling=coupling)
    cols = [0, 5, 9, 22, 13]
    part = og.reparam_gradients_at(MA, SA, MB, SB, c, N, G, cols, seed=4, coupling=coupling)
    for f, g in zip(full, part):
        np.testing.assert_allclose(g, f[cols], rtol=1e-12, atol=1e-12 * np.abs(f).max())
