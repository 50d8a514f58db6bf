"""Pins of the oracle's adaptive-L driver (Alg. 2's loop over L with the
stopping tests of Sec. 2, eq. (15), and Remark 3.5, eq. (27)):

  - at least three levels: with constant matrices every correction is exactly
    zero, so the test holds as soon as it may be applied, after level 2, and
    every level keeps its pilot (V_l = 0);
  - reuse of earlier realisations: realisations are never redrawn, so the
    result equals a fixed-N run with the final N_l, bit for bit;
  - the stopping test: a run that stops early stopped on a finest level whose
    mean (which no later step changed) is below the bound; a run that used
    every level without passing has a finest mean at or above it;
  - the two bounds differ only by the sign of 1 (inner product sqrt(M) - 1,
    matrix sqrt(M) + 1).
"""
import math

import numpy as np
import pytest

import oracle as orc


@pytest.mark.parametrize("kind", ["matrix", "inner"])
def test_constant_laws_stop_after_three_levels(kind):
    m, p = (3, 2) if kind == "matrix" else (1, 1)
    n = 64
    A, B = orc.Law.normal(0.125, 0.0), orc.Law.normal(0.5, 0.0)
    est = orc.estimate(m, n, p, A, B, [2, 4, 8, 16, 32], rmse_target=0.1, pilot=6, seed=3, adaptive=kind)
    assert est.levels_used == 3 and est.bias_test_passed
    assert list(est.n_used) == [6, 6, 6, 0, 0]
    assert np.all(est.Y == n * 0.125 * 0.5)
    assert np.all(est.level_means[1:] == 0.0)


def test_bounds():
    c = [4, 16, 64]
    assert orc.bias_bound(c, 2, 1.0, "matrix") == pytest.approx(3.0 / math.sqrt(2.0), rel=1e-15)
    assert orc.bias_bound(c, 2, 1.0, "inner") == pytest.approx(1.0 / math.sqrt(2.0), rel=1e-15)
    assert orc.bias_bound([3, 6], 1, 2.0, "matrix") == pytest.approx((math.sqrt(2.0) + 1.0) * math.sqrt(2.0))


@pytest.mark.parametrize("kind, func, eps", [
    ("matrix", None, 2.0),
    ("matrix", orc.Func.abs_step(2.0), 0.3),          # stops after four levels
    ("inner", orc.Func.inv_abs_step(0.4, 0.01), 0.2),  # uses every level
    ("inner", None, 0.5),
])
def test_adaptive_reuses_realisations_and_stops_on_the_test(kind, func, eps):
    m, p = (6, 5) if kind == "matrix" else (1, 1)
    n = 100
    A = orc.Law.normal(0.1, 0.1)
    c = [2, 4, 8, 16, 32]
    est = orc.estimate(m, n, p, A, A, c, rmse_target=eps, pilot=20, seed=5, func=func, adaptive=kind)
    used = est.levels_used
    assert 3 <= used <= len(c)
    assert all(x >= 20 for x in est.n_used[:used]) and all(x == 0 for x in est.n_used[used:])
    # a fixed-N run over the same realisations gives the same numbers
    fixed = orc.estimate(m, n, p, A, A, c[:used], n_samples=list(est.n_used[:used]), seed=5, func=func)
    assert np.array_equal(fixed.level_means, est.level_means[:used])
    assert np.array_equal(fixed.Y, est.Y)
    norm = float(np.linalg.norm(fixed.level_means[used - 1]))
    bound = orc.bias_bound(c, used - 1, eps, kind)
    if est.bias_test_passed:
        assert norm < bound
    else:
        assert used == len(c) and norm >= bound


def test_adaptive_uses_every_level_when_the_bias_stays_large():
    # f = |x| H(2 - x) with sketches straddling the step: E[f(Z_l)] moves with
    # l, and a tiny eps keeps the finest correction above the bound
    A = orc.Law.normal(0.1, 0.1)
    est = orc.estimate(4, 100, 3, A, A, [2, 4, 8, 16], rmse_target=0.05, pilot=10, seed=2,
                       func=orc.Func.abs_step(2.0), adaptive="matrix", max_total_draws=0)
    assert est.levels_used == 4
    assert not est.bias_test_passed
