"""Brute-force pins of the sketch (Sec. 3, eq. (18)) and of Alg. 1's coupling.

For a fixed realisation and every one of the n^c equally likely index tuples,
the oracle's sketches are averaged exactly.  The mathematics fixes:
  E[Z_c] = AB for any c (unbiasedness, Sec. 3),
  E[D] = 0 for D = Z_{c_l} - Z_{c_{l-1}} on shared indices,
  Var(D_iq) = s2_iq (1/c_{l-1} - 1/c_l), Var(Z_c,iq) = s2_iq / c,
  with s2_iq = n sum_j A_ij^2 B_jq^2 - (AB)_iq^2 (Drineas et al. 2006, uniform
  probabilities).
"""
import itertools

import numpy as np
import pytest


def _tuples(n, c):
    return itertools.product(range(n), repeat=c)


@pytest.mark.parametrize("m,n,p,cc,cf", [(3, 5, 2, 2, 4), (2, 4, 3, 1, 3), (1, 6, 1, 2, 4)])
def test_bruteforce_moments(orc, m, n, p, cc, cf):
    A, B = orc.realisation(42, 0, 0, 3, m, n, p, orc.Law.normal(0.3, 1.1),
                           orc.Law.uniform(-0.2, 0.9))
    AB = A @ B
    s2 = n * (A ** 2) @ (B ** 2) - AB ** 2
    sum_f = np.zeros((m, p)); sum_c = np.zeros((m, p)); sum_d = np.zeros((m, p))
    sq_f = np.zeros((m, p)); sq_d = np.zeros((m, p))
    count = 0
    for tup in _tuples(n, cf):
        idx = list(tup)
        AS = A[:, idx].T
        BS = B[idx, :]
        Zf, Zc = orc.sketch_pair(n, cf, cc, AS, BS)
        D = Zf - Zc
        sum_f += Zf; sum_c += Zc; sum_d += D
        sq_f += Zf ** 2; sq_d += D ** 2
        count += 1
    Ef, Ec, Ed = sum_f / count, sum_c / count, sum_d / count
    scale = np.abs(AB).max() + 1
    np.testing.assert_allclose(Ef, AB, atol=1e-12 * scale * n)
    np.testing.assert_allclose(Ec, AB, atol=1e-12 * scale * n)
    np.testing.assert_allclose(Ed, 0, atol=1e-12 * scale * n)
    var_f = sq_f / count - Ef ** 2
    var_d = sq_d / count
    np.testing.assert_allclose(var_f, s2 / cf, rtol=1e-9, atol=1e-9 * s2.max())
    np.testing.assert_allclose(var_d, s2 * (1 / cc - 1 / cf), rtol=1e-9, atol=1e-9 * s2.max())


def test_sketch_matches_definition_on_one_tuple(orc):
    # the definition written with matrices: Z = (n/c) A S S^T B with S the
    # n x c selection matrix (eq. (18), xi = 1/n)
    m, n, p = 4, 9, 3
    A, B = orc.realisation(1, 0, 0, 0, m, n, p, orc.Law.normal(0, 1), orc.Law.normal(0, 1))
    idx = [3, 3, 8, 0, 5, 1]
    S = np.zeros((n, len(idx)))
    for t, j in enumerate(idx):
        S[j, t] = 1.0
    Zf, Zc = orc.sketch_pair(n, 6, 2, A[:, idx].T, B[idx, :])
    ref_f = n / 6 * A @ S @ S.T @ B
    ref_c = n / 2 * A @ S[:, :2] @ S[:, :2].T @ B
    np.testing.assert_allclose(Zf, ref_f, rtol=1e-13, atol=1e-13 * np.abs(ref_f).max())
    np.testing.assert_allclose(Zc, ref_c, rtol=1e-13, atol=1e-13 * np.abs(ref_c).max())


def test_level_estimation_uses_the_realisation_columns(orc):
    # Alg. 1 on one realisation equals the sketch of the materialised A^(k), B^(k)
    m, n, p, c = 3, 11, 2, 8
    A_law, B_law = orc.Law.normal(1, 1), orc.Law.normal(-0.5, 2)
    st = orc.LevelState.empty(m, p)
    D = orc.level_estimation(st, m, n, p, A_law, B_law, c, 4, 9, 0, 2, 5, 6, want_samples=True)
    A, B = orc.realisation(9, 0, 2, 5, m, n, p, A_law, B_law)
    r = orc.draw_indices(9, 0, 2, 5, c, n)
    Zf = n / c * A[:, r] @ B[r, :]
    Zc = n / 4 * A[:, r[:4]] @ B[r[:4], :]
    np.testing.assert_allclose(D[0], Zf - Zc, rtol=1e-12, atol=1e-12)
