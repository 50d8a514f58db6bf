"""Pins of the oracle's 32-bit index words (four draws per Philox call, draw t
from word t % 4 of the call (t / 4, k, 0, index stream), r = floor(w n / 2^32);
the library offers it for power-of-two n, where it is exactly uniform):

  - for n = 2^b the index is the top b bits of the (rocRAND-pinned) Philox
    word, and n = 1 gives 0;
  - exact integer arithmetic for other n, and chi-square uniformity;
  - the inner-product level variances of i.i.d. laws match the closed form
    (Theorem 3.2 with uniform xi) by z-test, so the draws are independent and
    uniform as the estimator needs.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle as orc


def _words(seed, tagword, call, k):
    return orc.philox(np.array([[call, k, 0, tagword]], np.uint32), seed)[0]


@pytest.mark.parametrize("b", [0, 1, 10, 20, 31])
def test_power_of_two_is_top_bits(b):
    seed, problem, lev, n = 77, 5, 3, 1 << b
    tagword = (1 << 28) | (lev << 20) | problem
    for k in (0, 9):
        r = orc.draw_indices(seed, problem, lev, k, 13, n, word32=True)
        for t in range(13):
            w = int(_words(seed, tagword, t >> 2, k)[t & 3])
            assert r[t] == (w >> (32 - b) if b else 0)


@pytest.mark.parametrize("n", [3, 1000, 65537])
def test_exact_integer_map(n):
    seed, tagword = 4, (1 << 28)
    r = orc.draw_indices(seed, 0, 0, 2, 12, n, word32=True)
    for t in range(12):
        w = int(_words(seed, tagword, t >> 2, 2)[t & 3])
        assert r[t] == (w * n) >> 32 and 0 <= r[t] < n


@pytest.mark.parametrize("n", [256, 4096])
def test_uniformity_chi_square(n):
    draws = np.concatenate([orc.draw_indices(31, 0, 1, k, 512, n, word32=True) for k in range(300)])
    _, pval = stats.chisquare(np.bincount(draws, minlength=n))
    assert pval > 1e-4


def test_differs_from_the_64_bit_draw():
    a = orc.draw_indices(1, 0, 0, 0, 64, 1 << 20)
    b = orc.draw_indices(1, 0, 0, 0, 64, 1 << 20, word32=True)
    assert not np.array_equal(a, b)


def test_inner_level_variance_closed_form():
    m, n, p, c, N = 1, 4096, 1, [16, 64, 128], 20000
    A = orc.Law.uniform(0.5, 1.0)
    _, V_true = orc.closed_form_iid(m, n, p, A, A, c)
    for l in range(3):
        st = orc.LevelState.empty(m, p)
        D = orc.level_estimation(st, m, n, p, A, A, c[l], c[l - 1] if l else 0, 6, 0, l, 0, N,
                                 want_samples=True, index_word32=True)
        dev = ((D - st.mean.reshape(m, p)) ** 2).reshape(N, -1).sum(axis=1)
        se = dev.std() / math.sqrt(N)
        assert abs(st.variance - V_true[l]) < 5 * se, (l, st.variance, V_true[l], se)
