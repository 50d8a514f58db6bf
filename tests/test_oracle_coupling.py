"""Pins of the oracle's stride coupling (Sec. 3.1: the coarse sketch of level
l takes every M-th fine index, r_{jM} for j = 1 .. c_{l-1}, M = c_l / c_{l-1};
the prefix coupling takes the first c_{l-1} draws):

  - which draws: with a_t the t-th unit vector (1-based positions as in the
    paper) the coarse sketch is nonzero exactly at positions M, 2M, ...;
  - brute force over every index tuple: E[D] = 0 and Var(D_iq) =
    s2_iq (1/c_{l-1} - 1/c_l), the same law as the prefix coupling (any fixed
    subset of i.i.d. draws), which a repeated or missing coarse draw breaks;
  - the level variance of i.i.d. laws against the closed form by z-test;
  - Alg. 1 on one realisation equals the stride sketches of the materialised
    A^(k), B^(k), and the gradient reference's forward equals the C oracle.
"""
import itertools

import numpy as np
import pytest

import oracle as orc


@pytest.mark.parametrize("cf, cc", [(4, 2), (6, 2), (6, 3), (8, 1)])
def test_coarse_draws_are_every_M_th(cf, cc):
    M = cf // cc
    n = 10
    AS = np.eye(cf)                    # a_t = e_t
    BS = np.ones((cf, 1))
    _, Zc = orc.sketch_pair(n, cf, cc, AS, BS, stride=M)
    picked = [t + 1 for t in range(cf) if Zc[t, 0] != 0.0]     # 1-based positions
    assert picked == [j * M for j in range(1, cc + 1)]
    assert np.all(Zc[[j * M - 1 for j in range(1, cc + 1)], 0] == n / cc)
    _, Zp = orc.sketch_pair(n, cf, cc, AS, BS)                 # prefix: 1 .. cc
    assert [t + 1 for t in range(cf) if Zp[t, 0] != 0.0] == list(range(1, cc + 1))


@pytest.mark.parametrize("m,n,p,cc,cf", [(2, 3, 2, 2, 4), (2, 3, 1, 2, 6), (1, 4, 2, 1, 4)])
def test_bruteforce_moments_stride(m, n, p, cc, cf):
    A, B = orc.realisation(7, 0, 0, 1, m, n, p, orc.Law.normal(0.3, 1.1), orc.Law.uniform(-0.2, 0.9))
    AB = A @ B
    s2 = n * (A ** 2) @ (B ** 2) - AB ** 2
    M = cf // cc
    sum_d = np.zeros((m, p)); sq_d = np.zeros((m, p)); sum_c = np.zeros((m, p))
    count = 0
    for tup in itertools.product(range(n), repeat=cf):
        idx = list(tup)
        Zf, Zc = orc.sketch_pair(n, cf, cc, A[:, idx].T, B[idx, :], stride=M)
        D = Zf - Zc
        sum_d += D; sq_d += D ** 2; sum_c += Zc
        count += 1
    scale = np.abs(AB).max() + 1
    np.testing.assert_allclose(sum_c / count, AB, atol=1e-12 * scale * n)
    np.testing.assert_allclose(sum_d / count, 0, atol=1e-12 * scale * n)
    np.testing.assert_allclose(sq_d / count, s2 * (1 / cc - 1 / cf), rtol=1e-9, atol=1e-9 * s2.max())


def test_level_variance_closed_form_stride():
    # i.i.d. laws: the closed-form V_l (Theorem 3.2, uniform xi) holds for any
    # fixed coarse subset; z-test on the per-sample squared deviations
    import math
    m, n, p, c, N = 4, 64, 3, [4, 8, 16], 20000
    A, B = orc.Law.normal(1, 1), orc.Law.normal(0.5, 2)
    _, V_true = orc.closed_form_iid(m, n, p, A, B, c)
    for l in (1, 2):
        st = orc.LevelState.empty(m, p)
        D = orc.level_estimation(st, m, n, p, A, B, c[l], c[l - 1], 3, 0, l, 0, N, want_samples=True,
                                 coupling="stride")
        dev = ((D - st.mean.reshape(m, p)) ** 2).reshape(N, -1).sum(axis=1)
        se = dev.std() / math.sqrt(N)
        assert abs(st.variance - V_true[l]) < 5 * se, (l, st.variance, V_true[l], se)


def test_level_estimation_stride_uses_the_realisation_columns():
    m, n, p, c, cp = 3, 11, 2, 9, 3
    A_law, B_law = orc.Law.normal(1, 1), orc.Law.normal(-0.5, 2)
    st = orc.LevelState.empty(m, p)
    D = orc.level_estimation(st, m, n, p, A_law, B_law, c, cp, 9, 0, 2, 5, 6, want_samples=True,
                             coupling="stride")
    A, B = orc.realisation(9, 0, 2, 5, m, n, p, A_law, B_law)
    r = orc.draw_indices(9, 0, 2, 5, c, n)
    rc = r[[2, 5, 8]]                  # r_3, r_6, r_9 (1-based): every third
    Zf = n / c * A[:, r] @ B[r, :]
    Zc = n / cp * A[:, rc] @ B[rc, :]
    np.testing.assert_allclose(D[0], Zf - Zc, rtol=1e-12, atol=1e-12)


def test_gradient_reference_stride_matches_the_c_oracle():
    import torch
    from oracle import grad as og
    rng = np.random.default_rng(2)
    m, n, p = 3, 30, 2
    MA, SA = rng.normal(size=(n, m)), rng.uniform(0.1, 1.0, size=(n, m))
    MB, SB = rng.normal(size=(n, p)), rng.uniform(0.1, 1.0, size=(n, p))
    c, N = [2, 6, 12], [20, 10, 5]
    ref = orc.estimate(m, n, p, orc.Law.reparam(MA, SA, m), orc.Law.reparam(MB, SB, p), c, n_samples=N, seed=4,
                       coupling="stride")
    Y = og.reparam_estimate(*[torch.from_numpy(x) for x in (MA, SA, MB, SB)], c, N, seed=4, coupling="stride")
    assert np.abs(Y.numpy() - ref.Y).max() <= 1e-12 * np.abs(ref.Y).max()
