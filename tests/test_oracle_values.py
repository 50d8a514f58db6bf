"""Pin of the oracle's value generation: the laws of the synthetic matrices.

Checked against the distributions they must follow (Kolmogorov-Smirnov and
moment tests), against the keying rule (a column of one realisation is fixed:
a repeated index reuses it, Alg. 1 draws the pair A^(k), B^(k) before the
indices) and the uniform map's exactness.
"""
import numpy as np
from scipy import stats


def _many(orc, law_a, law_b, m=6, p=5, ks=200, js=40, lev=0):
    a_all, b_all = [], []
    for k in range(ks):
        for j in range(js):
            a, b = orc.column(77, 0, lev, k, 1000 + j, m, p, law_a, law_b)
            a_all.append(a)
            b_all.append(b)
    return np.array(a_all), np.array(b_all)


def test_normal_law(orc):
    A = orc.Law.normal(0.5, 2.0)
    B = orc.Law.normal(-1.0, 0.25)
    a, b = _many(orc, A, B)
    for x, loc, sc in ((a, 0.5, 2.0), (b, -1.0, 0.25)):
        z = (x.ravel() - loc) / sc
        assert stats.kstest(z, "norm").pvalue > 1e-4
        assert abs(z.mean()) < 5 / np.sqrt(z.size)
        assert abs(z.var() - 1) < 5 * np.sqrt(2 / z.size)
    # both members of a Box-Muller pair are standard normal and uncorrelated
    z = (a - 0.5) / 2.0
    r = np.corrcoef(z[:, 0], z[:, 1])[0, 1]
    assert abs(r) < 5 / np.sqrt(z.shape[0])


def test_uniform_law(orc):
    A = orc.Law.uniform(0.5, 1.0)
    B = orc.Law.uniform(-2.0, 3.0)
    a, b = _many(orc, A, B, m=1, p=1, ks=400, js=100)
    assert stats.kstest(a.ravel(), "uniform", args=(-0.5, 2.0)).pvalue > 1e-4
    assert stats.kstest(b.ravel(), "uniform", args=(-5.0, 6.0)).pvalue > 1e-4
    assert a.min() > -0.5 and a.max() < 1.5


def test_uniform_map_exact_and_open(orc):
    for w in (0, 1, 511, 512, 2**31, 2**32 - 1):
        u = orc.uniform(w)
        assert 0.0 < u < 1.0
        assert np.float32(u) == u                     # representable in FP32
        assert u == ((w >> 9) + 0.5) / 2.0**23
    assert orc.uniform(0) == 2.0**-24
    assert orc.uniform(2**32 - 1) == 1 - 2.0**-24


def test_reparam_law(orc):
    m, n, p = 3, 7, 2
    rng = np.random.default_rng(0)
    MA, SA = rng.normal(size=(m, n)), rng.uniform(0.1, 1, size=(m, n))
    MB, SB = rng.normal(size=(n, p)), rng.uniform(0.1, 1, size=(n, p))
    A = orc.Law.reparam(MA.T.ravel(), SA.T.ravel(), m)      # column-major A
    B = orc.Law.reparam(MB.ravel(), SB.ravel(), p)          # row-major B
    Z = []
    for k in range(3000):
        j = k % n
        a, b = orc.column(3, 0, 0, k, j, m, p, A, B)
        Z.append(np.concatenate([(a - MA[:, j]) / SA[:, j], (b - MB[j, :]) / SB[j, :]]))
    Z = np.array(Z).ravel()
    assert stats.kstest(Z, "norm").pvalue > 1e-4


def test_column_keyed_not_draw_keyed(orc):
    A = orc.Law.normal(0, 1)
    a1, b1 = orc.column(5, 0, 2, 9, 123, 4, 3, A, A)
    a2, b2 = orc.column(5, 0, 2, 9, 123, 4, 3, A, A)
    np.testing.assert_array_equal(a1, a2)
    np.testing.assert_array_equal(b1, b2)
    a3, _ = orc.column(5, 0, 2, 10, 123, 4, 3, A, A)      # other realisation
    a4, _ = orc.column(5, 0, 3, 9, 123, 4, 3, A, A)       # other level
    assert not np.array_equal(a1, a3) and not np.array_equal(a1, a4)
    # column vector layout: A part first, B part continues the same stream
    a5, b5 = orc.column(5, 0, 2, 9, 123, 7, 0, A, A)
    np.testing.assert_array_equal(a5[:4], a1)
    np.testing.assert_array_equal(a5[4:], b1)
