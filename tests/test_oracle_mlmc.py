"""Pins of the MLMC layer of the oracle (Sec. 2-3, eqs. (9), (10), (28)).

- Telescoping (eq. (10)): on shared realisations with equal N_l the level
  means sum to the finest-level sample mean, exactly up to rounding.
- Level variances: the closed forms of Thm 3.2 with xi = 1/n, specialised to
  the synthetic laws, checked by z-tests on the oracle's V_l.
- Special cases: n = 1, deterministic matrices, identical columns.
- Scheduler (eq. (28)): the continuous allocation meets the variance budget
  eps^2 / 2 with equality and is cost-optimal (Lagrange conditions).
"""
import math

import numpy as np
import pytest


def test_telescoping_shared_realisations(orc):
    m, n, p = 5, 40, 4
    c = [2, 4, 8, 16]
    A, B = orc.Law.normal(1, 1), orc.Law.uniform(0.2, 1.5)
    est = orc.estimate(m, n, p, A, B, c, n_samples=[30] * 4, seed=3, shared=True)
    st = orc.LevelState.empty(m, p)
    orc.level_estimation(st, m, n, p, A, B, c[-1], 0, 3, 0, orc.SHARED_LEVEL_FIELD, 0, 30)
    finest = st.mean.reshape(m, p)
    np.testing.assert_allclose(est.Y, finest, rtol=1e-12, atol=1e-12 * np.abs(finest).max())


def _z_check(orc, m, n, p, A, B, c, N, V_true, seed=11):
    for l in range(len(c)):
        st = orc.LevelState.empty(m, p)
        D = orc.level_estimation(st, m, n, p, A, B, c[l], c[l - 1] if l else 0, seed, 0, l,
                                 0, N, want_samples=True)
        dev = ((D - st.mean.reshape(m, p)) ** 2).reshape(N, -1).sum(axis=1)
        se = dev.std() / math.sqrt(N)
        assert abs(st.variance - V_true[l]) < 5 * se, (l, st.variance, V_true[l], se)


def test_level_variance_normal_closed_form(orc):
    m, n, p, c = 4, 64, 3, [4, 8, 16]
    A, B = orc.Law.normal(1, 1), orc.Law.normal(0.5, 2)
    E, V = orc.closed_form_iid(m, n, p, A, B, c)
    _z_check(orc, m, n, p, A, B, c, 20000, V)


def test_level_variance_uniform_closed_form(orc):
    m, n, p, c = 1, 4096, 1, [64, 128, 256]
    A, B = orc.Law.uniform(0.5, 1), orc.Law.uniform(0.5, 1)
    E, V = orc.closed_form_iid(m, n, p, A, B, c)
    _z_check(orc, m, n, p, A, B, c, 20000, V)


def test_level_variance_reparam_closed_form(orc):
    m, n, p, c = 3, 50, 2, [2, 4, 8]
    rng = np.random.default_rng(5)
    MA, SA = rng.normal(size=(m, n)), rng.uniform(0.1, 1, size=(m, n))
    MB, SB = rng.normal(size=(n, p)), rng.uniform(0.1, 1, size=(n, p))
    A = orc.Law.reparam(MA.T.ravel(), SA.T.ravel(), m)
    B = orc.Law.reparam(MB.ravel(), SB.ravel(), p)
    E, V = orc.closed_form_reparam(MA, SA, MB, SB, c)
    _z_check(orc, m, n, p, A, B, c, 20000, V)


def test_mean_unbiased_against_closed_form(orc):
    m, n, p, c = 3, 64, 2, [4, 8, 16]
    A, B = orc.Law.normal(1, 1), orc.Law.normal(1, 1)
    E, V = orc.closed_form_iid(m, n, p, A, B, c)
    N = [4000, 2000, 1000]
    est = orc.estimate(m, n, p, A, B, c, n_samples=N, seed=21)
    sd_entry = math.sqrt(sum(V[l] / N[l] for l in range(3)) / (m * p))
    assert np.all(np.abs(est.Y - E) < 5 * sd_entry)


def test_special_case_n_equals_one(orc):
    m, p = 3, 2
    A, B = orc.Law.normal(1, 1), orc.Law.normal(2, 1)
    est = orc.estimate(m, 1, p, A, B, [2, 4, 8], n_samples=[10, 10, 10], seed=1)
    # every index is 0: fine and coarse sketches are the same product up to
    # the rounding of summing c identical terms
    scale = np.abs(est.Y).max()
    assert est.level_var[1] < (1e-14 * scale) ** 2 and est.level_var[2] < (1e-14 * scale) ** 2
    np.testing.assert_allclose(est.level_means[1:], 0, atol=1e-14 * scale)


def test_special_case_deterministic_entries(orc):
    # scale 0: every sketch equals n loc_a loc_b exactly, so D_l = 0, V_0 = 0
    A, B = orc.Law.normal(1.5, 0.0), orc.Law.uniform(-2.0, 0.0)
    est = orc.estimate(2, 37, 3, A, B, [3, 6], n_samples=[5, 5], seed=2)
    np.testing.assert_allclose(est.Y, 37 * 1.5 * -2.0, rtol=1e-14)
    assert est.level_var[0] < 1e-20 and est.level_var[1] < 1e-20


def test_special_case_identical_columns(orc):
    # A = M with identical columns, B = M_B with identical rows (S = 0):
    # every sketch equals AB, so D_l = 0 for l >= 1
    m, n, p = 3, 10, 2
    col = np.array([1.0, -2.0, 0.5]); row = np.array([3.0, -1.0])
    MA = np.tile(col[:, None], (1, n)); MB = np.tile(row[None, :], (n, 1))
    A = orc.Law.reparam(MA.T.ravel(), np.zeros(m * n), m)
    B = orc.Law.reparam(MB.ravel(), np.zeros(n * p), p)
    est = orc.estimate(m, n, p, A, B, [2, 4], n_samples=[4, 4], seed=0)
    np.testing.assert_allclose(est.Y, MA @ MB, rtol=1e-13)
    np.testing.assert_allclose(est.level_means[1], 0, atol=1e-12)


def test_scheduler_lagrange_optimal(orc):
    rng = np.random.default_rng(0)
    for _ in range(20):
        L1 = rng.integers(2, 9)
        V = rng.uniform(0.1, 10, size=L1) * 2.0 ** -np.arange(L1)
        C = 2.0 ** np.arange(L1) * rng.integers(1, 64)
        eps = rng.uniform(0.01, 0.2)
        N = np.array(orc.schedule(V, C, eps), dtype=float)
        # ceil'd allocation meets the budget eps^2 / 2
        assert np.sum(V / N) <= eps ** 2 / 2 * (1 + 1e-12)
        # continuous optimum: equality in the constraint, N_l C_l / sqrt(V_l C_l) constant
        Nc = 2 / eps ** 2 * np.sqrt(V / C) * np.sum(np.sqrt(V * C))
        assert np.all(N >= Nc) and np.all(N < Nc + 1)
        assert abs(np.sum(V / Nc) - eps ** 2 / 2) < 1e-9 * eps ** 2
        # any feasible perturbation along the constraint costs more
        cost = np.sum(Nc * C)
        for _ in range(10):
            d = rng.normal(size=L1)
            g = V / Nc ** 2                      # gradient of sum V/N is -g
            d -= (d @ g) / (g @ g) * g           # first order on the constraint
            Np = Nc * (1 + 1e-3 * d / np.abs(d).max())
            Np *= np.sum(V / Np) / (eps ** 2 / 2)  # rescale back onto the constraint
            assert np.sum(Np * C) >= cost * (1 - 1e-12)


def test_target_mode_meets_rmse(orc):
    m, n, p, c = 1, 2048, 1, [16, 32, 64, 128]
    A, B = orc.Law.uniform(0.5, 1), orc.Law.uniform(0.5, 1)
    E, V = orc.closed_form_iid(m, n, p, A, B, c)
    eps = 0.02 * abs(E)
    est = orc.estimate(m, n, p, A, B, c, rmse_target=eps, pilot=200, seed=4)
    assert est.rmse_est <= eps / math.sqrt(2) * 1.2
    assert np.all(est.n_used >= 200)
    assert abs(est.Y[0, 0] - E) < 5 * est.rmse_est


@pytest.mark.parametrize("law", ["normal", "uniform", "reparam"])
def test_entries_restriction_equals_full_estimate(orc, law):
    """The entry-restricted evaluation reproduces the full estimate at the
    chosen entries bit for bit (same realisations, same arithmetic order),
    including repeated and unsorted rows/columns."""
    m, n, p, c, N = 7, 90, 6, [3, 6, 12], [25, 12, 6]
    rng = np.random.default_rng(5)
    if law == "reparam":
        # A column-major: row j of the (n, m) arrays is column j of A
        MA, SA = rng.standard_normal((n, m)), rng.uniform(0.1, 1, (n, m))
        MB, SB = rng.standard_normal((n, p)), rng.uniform(0.1, 1, (n, p))
        A, B = orc.Law.reparam(MA.ravel(), SA.ravel(), m), orc.Law.reparam(MB.ravel(), SB.ravel(), p)
    elif law == "uniform":
        A, B = orc.Law.uniform(0.3, 1.2), orc.Law.uniform(-0.4, 2.0)
    else:
        A, B = orc.Law.normal(1.0, 0.5), orc.Law.normal(-0.2, 1.5)
    rows, cols = [6, 0, 3, 3], [5, 1]
    for shared in (False, True):
        full = orc.estimate(m, n, p, A, B, c, n_samples=N, seed=8, problem=4, shared=shared)
        sub = orc.estimate_entries(m, n, p, A, B, c, N, rows, cols, seed=8, problem=4, shared=shared)
        ix = np.ix_(rows, cols)
        assert np.array_equal(sub.Y, full.Y[ix])
        for l in range(len(c)):
            assert np.array_equal(sub.level_means[l], full.level_means[l][ix])
        # the entry variances sum (over all entries) to V_l
        every = orc.estimate_entries(m, n, p, A, B, c, N, range(m), range(p), seed=8, problem=4,
                                     shared=shared)
        np.testing.assert_allclose(every.entry_var.sum(axis=(1, 2)), full.level_var, rtol=1e-12)
