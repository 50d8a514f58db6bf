"""Pins of the oracle's generators for the laws of the experiments of Sec. 4
(column index j counted from 1 as in the paper): sample moments against
closed forms derived from characteristic functions,
  E[cos(K + 2E)] = Re(exp(lam (e^i - 1)) / (1 - 2i)),
  E[cos^2(K + 2E)] = (1 + Re(exp(lam (e^2i - 1)) / (1 - 4i))) / 2
(K ~ Poisson(lam), E ~ Exp(1)), E[sin x] = sin(mu) exp(-s^2 / 2) for
x ~ N(mu, s^2), finite Poisson sums for the step law, and the Poisson
probabilities themselves (chi-square), each by a 5-sigma z-test."""
import cmath
import math

import numpy as np
import pytest

import oracle as orc


def _samples(law, j, count, seed=1, e=0):
    """`count` independent values of column j's element e (one per realisation)."""
    other = orc.Law.normal(0.0, 1.0)
    out = np.empty(count)
    for k in range(count):
        a, b = orc.column(seed, 0, 0, k, j, 1, 1, law, other)
        out[k] = a[0]
    return out


def _ztest(x, mean):
    sd = x.std(ddof=1) / math.sqrt(x.size)
    assert abs(x.mean() - mean) <= 5.0 * sd + 1e-15, (x.mean(), mean, sd)


@pytest.mark.parametrize("j", [0, 49, 999])
def test_ramp_normal(j):
    law = orc.Law.experiment(orc.LAW_RAMP_NORMAL, 0.4, 1.0 / 50)
    x = _samples(law, j, 20000)
    J = j + 1
    _ztest(x, J / 50 * 0.4)
    _ztest(x ** 2, (J / 50) ** 2 * (1.0 + 0.4 ** 2))


def test_cos_poisson_exp():
    lam, beta = 10.0, 0.05
    law = orc.Law.experiment(orc.LAW_COS_POISSON_EXP, lam, beta)
    x = _samples(law, 3, 40000)
    m1 = beta * (cmath.exp(lam * (cmath.exp(1j) - 1)) / (1 - 2j)).real
    m2 = beta * (1 + (cmath.exp(lam * (cmath.exp(2j) - 1)) / (1 - 4j)).real) / 2
    _ztest(x, m1)
    _ztest(x ** 2, m2)
    # the Bernoulli factor: the zero fraction is 1 - beta
    frac = float((x != 0).mean())
    assert abs(frac - beta) <= 5 * math.sqrt(beta * (1 - beta) / x.size)


@pytest.mark.parametrize("j", [0, 4999, 9999])
def test_sin_ramp(j):
    s = (j + 1) * 1e-4
    law = orc.Law.experiment(orc.LAW_SIN_RAMP, 0.5, 1e-4)
    x = _samples(law, j, 30000)
    mu, var = s * 0.5, s * s
    _ztest(x, math.sin(mu) * math.exp(-var / 2))
    _ztest(x ** 2, (1 - math.cos(2 * mu) * math.exp(-2 * var)) / 2 + var + mu * mu)


def test_cos_poisson_step_and_poisson_probabilities():
    lam, beta = 2.0, 0.2
    law = orc.Law.experiment(orc.LAW_COS_POISSON_STEP, lam, beta)
    x = _samples(law, 7, 40000)
    pmf = [math.exp(-lam) * lam ** k / math.factorial(k) for k in range(6)]
    _ztest(x, beta * sum(math.cos(k) * pk for k, pk in enumerate(pmf)))
    _ztest(x ** 2, beta * sum(math.cos(k) ** 2 * pk for k, pk in enumerate(pmf)))
    # with beta = 1 every value is cos(K) for K <= 5 (distinct values) or 0:
    # the counts of K = 0..5 follow the Poisson probabilities
    x1 = _samples(orc.Law.experiment(orc.LAW_COS_POISSON_STEP, lam, 1.0), 7, 20000, seed=3)
    counts = np.array([np.sum(np.isclose(x1, math.cos(k), rtol=0, atol=1e-12)) for k in range(6)], dtype=float)
    expect = x1.size * np.array(pmf)
    chi2 = float(((counts - expect) ** 2 / expect).sum())
    assert chi2 < 30.0, chi2     # 6 bins
    assert int(counts.sum() + np.sum(x1 == 0.0)) == x1.size
