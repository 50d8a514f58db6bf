"""Pins of the oracle's non-uniform index probabilities xi_j = w_j / W
(eq. (18) with a general xi; Theorem 3.1's xi** for reparameterised laws):

  - all weights 1 reproduce the uniform draw index for index;
  - the draws follow w_j / W (chi-square);
  - unbiasedness: the xi-weighted average of the sketch over every index
    tuple is AB (brute force on tiny fixed matrices);
  - the exact expected squared error for any xi, (1/c)(sum_j ||A_j||^2 ||B_j||^2
    / xi_j - ||AB||^2), by brute force, and at xi** Theorem 3.1's minimum
    (1/c)((sum_j ||A_j|| ||B_j||)^2 - ||AB||^2) up to the weights' 2^-24
    quantisation, below the uniform sampler's error;
  - the MLMC estimate with xi** converges to E[AB] within its error bar.
"""
import itertools

import numpy as np
import pytest

import oracle as orc


def test_unit_weights_are_the_uniform_draw():
    n = 77
    ones = orc.Weights(np.ones(n, dtype=np.uint32))
    for k in range(5):
        r = orc.draw_indices(3, 2, 1, k, 40, n)
        for t in range(40):
            assert orc.draw_index_weighted(3, 2, 1, k, t, ones) == r[t]


def test_weighted_draws_follow_the_weights():
    w = np.array([5, 1, 3, 1, 10, 20], dtype=np.uint32)
    W = orc.Weights(w)
    counts = np.zeros(w.size)
    for k in range(2000):
        for t in range(8):
            counts[orc.draw_index_weighted(11, 0, 0, k, t, W)] += 1
    expect = counts.sum() * W.xi
    chi2 = float(((counts - expect) ** 2 / expect).sum())
    assert chi2 < 25.0, chi2      # 5 degrees of freedom: p ~ 1e-4 at 25


def _fixed_laws(M, Wm):
    m, n = M.shape
    p = Wm.shape[1]
    A = orc.Law.reparam(M.T.copy(), np.zeros((n, m)), m)
    B = orc.Law.reparam(Wm.copy(), np.zeros((n, p)), p)
    return A, B


@pytest.mark.parametrize("w", [[1, 2, 5], [7, 7, 7], [1, 1, 30]])
def test_weighted_sketch_is_unbiased_with_exact_error(w):
    rng = np.random.default_rng(8)
    m, n, p, c = 2, 3, 3, 2
    M = rng.normal(size=(m, n))
    Wm = rng.normal(size=(n, p))
    weights = orc.Weights(np.array(w, dtype=np.uint32))
    xi = weights.xi
    AB = M @ Wm
    mean = np.zeros((m, p))
    err2 = 0.0
    for tup in itertools.product(range(n), repeat=c):
        prob = np.prod([xi[r] for r in tup])
        AS = np.stack([M[:, r] for r in tup])
        BS = np.stack([Wm[r, :] for r in tup])
        factor = [weights.total / float(weights.w[r]) for r in tup]
        Zf, _ = orc.sketch_pair_weighted(c, 0, factor, AS, BS)
        mean += prob * Zf
        err2 += prob * float(((Zf - AB) ** 2).sum())
    assert np.abs(mean - AB).max() <= 1e-13 * np.abs(AB).max()
    colsq = (M ** 2).sum(axis=0) * (Wm ** 2).sum(axis=1)
    exact = (float((colsq / xi).sum()) - float((AB ** 2).sum())) / c
    assert err2 == pytest.approx(exact, rel=1e-12)


def test_optimal_weights_reach_theorem_3_1():
    rng = np.random.default_rng(3)
    m, n, p, c = 3, 6, 2, 2
    # columns of very different sizes, so xi** differs from uniform
    M = rng.normal(size=(m, n)) * (1.0 + 5.0 * np.arange(n))
    Wm = rng.normal(size=(n, p))
    A, B = _fixed_laws(M.astype(np.float32).astype(np.float64), Wm.astype(np.float32).astype(np.float64))
    w = orc.optimal_weights(m, n, p, A, B)
    assert int(w.max()) == 1 << 24
    weights = orc.Weights(w)
    M = M.astype(np.float32).astype(np.float64)
    Wm = Wm.astype(np.float32).astype(np.float64)
    AB = M @ Wm
    norms = np.sqrt((M ** 2).sum(axis=0)) * np.sqrt((Wm ** 2).sum(axis=1))
    mu_bar = float(norms.sum()) ** 2 - float((AB ** 2).sum())
    colsq = (M ** 2).sum(axis=0) * (Wm ** 2).sum(axis=1)
    err_opt = (float((colsq / weights.xi).sum()) - float((AB ** 2).sum())) / c
    err_uni = (float((colsq * n).sum()) - float((AB ** 2).sum())) / c
    assert err_opt == pytest.approx(mu_bar / c, rel=1e-6)
    assert err_opt < err_uni


def test_optimal_weights_are_uniform_for_iid_laws():
    w = orc.optimal_weights(4, 9, 3, orc.Law.normal(1.0, 2.0), orc.Law.uniform(0.0, 1.0))
    assert np.all(w == 1 << 24)


def test_weighted_mlmc_converges_to_the_mean():
    rng = np.random.default_rng(5)
    m, n, p = 4, 60, 3
    MA = rng.normal(size=(n, m)) * np.linspace(0.1, 3.0, n)[:, None]
    SA = rng.uniform(0.1, 1.0, size=(n, m))
    MB = rng.normal(size=(n, p))
    SB = rng.uniform(0.1, 1.0, size=(n, p))
    A = orc.Law.reparam(MA, SA, m)
    B = orc.Law.reparam(MB, SB, p)
    weights = orc.Weights(orc.optimal_weights(m, n, p, A, B))
    c, N = [2, 4, 8], [4000, 2000, 1000]
    est = orc.estimate(m, n, p, A, B, c, n_samples=N, seed=4, weights=weights)
    uni = orc.estimate(m, n, p, A, B, c, n_samples=N, seed=4)
    exact = MA.T @ MB
    assert np.linalg.norm(est.Y - exact) <= 5.0 * est.rmse_est
    # importance sampling lowers every level's variance for these laws
    assert np.all(est.level_var < uni.level_var)


def test_gradient_reference_with_weights_matches_the_c_oracle():
    import torch
    from oracle import grad as og
    rng = np.random.default_rng(9)
    m, n, p = 3, 40, 2
    MA = rng.normal(size=(n, m)) * np.linspace(0.2, 2.0, n)[:, None]
    SA = rng.uniform(0.1, 1.0, size=(n, m))
    MB = rng.normal(size=(n, p))
    SB = rng.uniform(0.1, 1.0, size=(n, p))
    A, B = orc.Law.reparam(MA, SA, m), orc.Law.reparam(MB, SB, p)
    weights = orc.Weights(orc.optimal_weights(m, n, p, A, B))
    c, N = [2, 4], [30, 15]
    ref = orc.estimate(m, n, p, A, B, c, n_samples=N, seed=6, weights=weights)
    Y = og.reparam_estimate(*[torch.from_numpy(x) for x in (MA, SA, MB, SB)], c, N, seed=6, weights=weights)
    assert np.abs(Y.numpy() - ref.Y).max() <= 1e-12 * np.abs(ref.Y).max()
