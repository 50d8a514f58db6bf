"""Pins of the oracle's target function f (Sec. 3: the estimator of
E[f(AB)] maps both sketches of a realisation entrywise by f before the
difference).  Each pin holds independently of the oracle's own code path:

  - special cases: constant matrices make every sketch equal to n a b exactly,
    so every level mean is f(n a b) at level 0 and exactly 0 above it, with
    f evaluated by hand from its definition on both sides of each step;
  - telescoping on shared realisations: with the same realisations and index
    prefixes at every level, the level means of f(Z_l) - f(Z_{l-1}) sum to
    the mean of f(Z_L) (a wrong coarse scale or f applied to the difference
    breaks this);
  - brute force: for fixed matrices (zero standard deviation) on tiny n the
    telescoped estimate converges to the exact average of f(Z_L) over every
    index tuple, within the estimator's own error bar.
"""
import itertools
import math

import numpy as np
import pytest

import oracle as orc


def test_func_values_at_the_steps():
    # f(x) = |x| H(2 - x), H(0) = 1 (Sec. 4.2)
    f = orc.Func.abs_step(2.0)
    assert f(-3.0) == 3.0
    assert f(1.5) == 1.5
    assert f(2.0) == 2.0
    assert f(2.5) == 0.0
    # f(x) = 1 / (|x| H(x + 0.4) + 0.01) (Sec. 4.1)
    g = orc.Func.inv_abs_step(0.4, 0.01)
    assert g(-0.5) == pytest.approx(100.0, rel=1e-15)
    assert g(-0.4) == pytest.approx(1.0 / 0.41, rel=1e-15)
    assert g(3.0) == pytest.approx(1.0 / 3.01, rel=1e-15)
    assert orc.Func()(-7.25) == -7.25


@pytest.mark.parametrize("func, x, expect", [
    (orc.Func.abs_step(2.0), 1.5, 1.5),      # below the step
    (orc.Func.abs_step(2.0), 2.0, 2.0),      # at the step, H(0) = 1
    (orc.Func.abs_step(2.0), 3.0, 0.0),      # above the step
    (orc.Func.abs_step(2.0), -1.0, 1.0),     # negative: |x|
    (orc.Func.inv_abs_step(0.4, 0.01), -0.5, 100.0),
    (orc.Func.inv_abs_step(0.4, 0.01), 0.25, 1.0 / 0.26),
])
def test_constant_matrices(func, x, expect):
    # A = a, B = b everywhere (scale 0): every sketch is (n / c) c a b = n a b
    # exactly (powers of two), so D_0 = f(n a b) and D_l = 0 for l > 0.
    n, m, p = 64, 3, 2
    b = 0.25 if x >= 0 else -0.25
    a = x / (n * b)
    A, B = orc.Law.normal(a, 0.0), orc.Law.normal(b, 0.0)
    est = orc.estimate(m, n, p, A, B, [2, 4, 8], n_samples=[5, 4, 3], seed=1, func=func)
    assert np.all(est.level_means[0] == pytest.approx(expect, rel=1e-15))
    assert np.all(est.level_means[1:] == 0.0)
    assert np.all(est.level_var == 0.0)


@pytest.mark.parametrize("func", [orc.Func.abs_step(2.0), orc.Func.inv_abs_step(0.4, 0.01),
                                  orc.Func.abs_step(1e300)])
def test_telescoping_with_func(func):
    # Shared realisations, equal N_l: the prefix coupling makes the coarse
    # sketch of level l the fine sketch of level l - 1, so the level means of
    # f(Z_l) - f(Z_{l-1}) telescope to the mean of f(Z_L).
    m, n, p, N = 3, 40, 4, 30
    c = [2, 4, 8, 16]
    A, B = orc.Law.normal(0.05, 0.1), orc.Law.uniform(0.1, 0.2)
    est = orc.estimate(m, n, p, A, B, c, n_samples=[N] * 4, seed=6, shared=True, func=func)
    fin = orc.LevelState.empty(m, p)
    orc.level_estimation(fin, m, n, p, A, B, c[-1], 0, 6, 0, orc.SHARED_LEVEL_FIELD, 0, N, func=func)
    scale = np.abs(fin.mean).max()
    assert np.abs(est.Y.ravel() - fin.mean).max() <= 1e-12 * scale
    # and the level samples really are nonlinear: f(Zf) - f(Zc) differs from f(Zf - Zc)
    if func.kind != orc.F_ABS_STEP or func.theta0 < 1e10:
        lin = orc.estimate(m, n, p, A, B, c, n_samples=[N] * 4, seed=6, shared=True)
        assert np.abs(lin.level_means[1:] - est.level_means[1:]).max() > 1e-6 * scale


def test_identity_func_is_the_plain_estimator():
    m, n, p = 4, 50, 3
    A, B = orc.Law.normal(0.3, 1.0), orc.Law.normal(-0.2, 0.5)
    a = orc.estimate(m, n, p, A, B, [2, 4], n_samples=[20, 10], seed=9)
    b = orc.estimate(m, n, p, A, B, [2, 4], n_samples=[20, 10], seed=9, func=orc.Func())
    assert np.array_equal(a.level_means, b.level_means)
    assert np.array_equal(a.level_var, b.level_var)


@pytest.mark.parametrize("func", [orc.Func.abs_step(1.0), orc.Func.inv_abs_step(0.4, 0.01)])
def test_brute_force_expectation_of_f(func):
    # Fixed A = M (2 x 3), B = W (3 x 2) (zero standard deviation): the only
    # randomness is the index draws.  E[f(Z_L)] is the average of f over all
    # n^{c_L} index tuples; the MLMC estimate converges to it (Sec. 3: the
    # telescoping sum estimates E[f(Z_L)]).
    m, n, p = 2, 3, 2
    rng = np.random.default_rng(4)
    M = rng.normal(size=(m, n)) * 0.4
    W = rng.normal(size=(n, p)) * 0.4
    c = [1, 2]
    # reparam laws: A column-major (element (i, j) at j * ld + i), B row-major
    A = orc.Law.reparam(M.T.copy(), np.zeros((n, m)), m)
    B = orc.Law.reparam(W.copy(), np.zeros((n, p)), p)
    exact = np.zeros((m, p))
    for tup in itertools.product(range(n), repeat=c[-1]):
        Z = sum(np.outer(M[:, r], W[r, :]) for r in tup) * (n / c[-1])
        exact += np.vectorize(func)(Z)
    exact /= n ** c[-1]
    N = [20000, 20000]
    est = orc.estimate(m, n, p, A, B, c, n_samples=N, seed=12, func=func)
    # per-entry standard error from the level variances of the entries
    err = np.abs(est.Y - exact)
    assert err.max() <= 5.0 * est.rmse_est, (err.max(), est.rmse_est)
    # the level means themselves are the exact level expectations' estimates
    e0 = np.zeros((m, p))
    for r in range(n):
        e0 += np.vectorize(func)(n * np.outer(M[:, r], W[r, :]))
    e0 /= n
    assert np.abs(est.level_means[0] - e0).max() <= 5.0 * math.sqrt(est.level_var[0] / N[0])
