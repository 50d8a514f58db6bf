"""Pins of the oracle's 16-bit value uniforms (element e of column j: half
(e odd: high, e even: low) of word (e/2) % 4 of the value-stream call
(e/8, k, j, 2 << 28 | level << 20 | problem), u = (h + 1/2) 2^-16; normals by
Box-Muller on the pair (e & ~1, e | 1)):

  - the uniform law's values are exactly loc + scale (2u - 1) with h the
    corresponding half of the rocRAND-pinned Philox word;
  - the normal law's pairs satisfy the Box-Muller identities
    z_e^2 + z_{e+1}^2 = -2 ln u_e and atan2(z_{e+1}, z_e) = 2 pi u_{e+1} (mod 2 pi);
  - sample moments of both laws;
  - the matrix estimator's level variances against the closed form (Theorem
    3.2, uniform xi) by z-test: the truncation of the normal at 4.85 sigma
    changes the variance by about 1e-5 relative, far below the test's reach.
"""
import math

import numpy as np
import pytest

import oracle as orc


def _half(seed, problem, lev, k, j, e):
    tag = (2 << 28) | (lev << 20) | problem
    w = int(orc.philox(np.array([[e >> 3, k, j, tag]], np.uint32), seed)[0][(e >> 1) & 3])
    return (w >> 16) if (e & 1) else (w & 0xFFFF)


def test_uniform_values_are_the_word_halves():
    seed, problem, lev, k, j = 17, 3, 2, 9, 41
    m, p = 13, 6
    law = orc.Law.uniform(0.25, 1.5).with_value16()
    a, b = orc.column(seed, problem, lev, k, j, m, p, law, law)
    v = np.concatenate([a, b])
    for e in range(m + p):
        u = (_half(seed, problem, lev, k, j, e) + 0.5) / 65536.0
        assert v[e] == 0.25 + 1.5 * (2.0 * u - 1.0)


def test_normal_pairs_are_box_muller_of_the_halves():
    seed, problem, lev, k, j = 5, 0, 1, 2, 7
    law = orc.Law.normal(0.0, 1.0).with_value16()
    a, _ = orc.column(seed, problem, lev, k, j, 16, 1, law, law)
    for e in range(0, 16, 2):
        u1 = (_half(seed, problem, lev, k, j, e) + 0.5) / 65536.0
        u2 = (_half(seed, problem, lev, k, j, e + 1) + 0.5) / 65536.0
        assert a[e] ** 2 + a[e + 1] ** 2 == pytest.approx(-2.0 * math.log(u1), rel=1e-13)
        ang = math.atan2(a[e + 1], a[e]) % (2 * math.pi)
        assert ang == pytest.approx(2 * math.pi * u2, abs=1e-12)


def test_moments():
    law = orc.Law.normal(1.0, 2.0).with_value16()
    x = np.concatenate([orc.column(8, 0, 0, k, 3, 8, 0 + 1, law, law)[0] for k in range(4000)])
    sd = x.std(ddof=1)
    assert abs(x.mean() - 1.0) < 5 * sd / math.sqrt(x.size)
    assert abs(sd / 2.0 - 1.0) < 5 * math.sqrt(0.5 / x.size)
    u = orc.Law.uniform(0.0, 1.0).with_value16()
    y = np.concatenate([orc.column(8, 0, 0, k, 3, 8, 1, u, u)[0] for k in range(4000)])
    assert abs(y.mean()) < 5 * math.sqrt(1 / 3 / y.size)
    assert abs(y.var() - 1 / 3) < 5 * math.sqrt(4 / 45 / y.size)


def test_level_variance_closed_form_value16():
    m, n, p, c, N = 4, 64, 3, [4, 8, 16], 20000
    A, B = orc.Law.normal(1, 1).with_value16(), orc.Law.normal(0.5, 2).with_value16()
    _, V_true = orc.closed_form_iid(m, n, p, orc.Law.normal(1, 1), orc.Law.normal(0.5, 2), c)
    for l in range(3):
        st = orc.LevelState.empty(m, p)
        D = orc.level_estimation(st, m, n, p, A, B, c[l], c[l - 1] if l else 0, 4, 0, l, 0, N, want_samples=True)
        dev = ((D - st.mean.reshape(m, p)) ** 2).reshape(N, -1).sum(axis=1)
        se = dev.std() / math.sqrt(N)
        assert abs(st.variance - V_true[l]) < 5 * se, (l, st.variance, V_true[l], se)


def test_gradient_reference_value16_matches_the_c_oracle():
    import torch
    from oracle import grad as og
    rng = np.random.default_rng(3)
    m, n, p = 3, 30, 2
    MA, SA = rng.normal(size=(n, m)), rng.uniform(0.1, 1.0, size=(n, m))
    MB, SB = rng.normal(size=(n, p)), rng.uniform(0.1, 1.0, size=(n, p))
    c, N = [2, 4, 8], [20, 10, 5]
    A = orc.Law.reparam(MA, SA, m).with_value16()
    B = orc.Law.reparam(MB, SB, p).with_value16()
    ref = orc.estimate(m, n, p, A, B, c, n_samples=N, seed=7)
    Y = og.reparam_estimate(*[torch.from_numpy(x) for x in (MA, SA, MB, SB)], c, N, seed=7, value16=True)
    assert np.abs(Y.numpy() - ref.Y).max() <= 1e-12 * np.abs(ref.Y).max()
