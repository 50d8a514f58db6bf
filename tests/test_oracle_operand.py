"""Pins of the oracle's operand formats (the precision form: the contraction
reads every generated value rounded to BF16, or to FP8 e4m3 under a
power-of-two scale) and of the FP8 scale rule.

The roundings are pinned to PyTorch's own conversions (float32 -> bfloat16
and float32 -> float8_e4m3fn, both round-to-nearest-even), on random values,
exact ties, the subnormal range and the ends of e4m3's range; the scale rule
to its defining inequality 2^s bound <= 256 < 2^(s+1) bound; the operand mode
of Alg. 1 to the materialised realisation rounded by PyTorch and sketched
with NumPy."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")


def _vals(rng):
    x = np.concatenate([
        rng.standard_normal(20000) * 10.0 ** rng.uniform(-8, 3, 20000),
        rng.uniform(-500, 500, 5000),
        rng.uniform(-0.02, 0.02, 5000),            # e4m3 subnormals (below 2^-6)
    ]).astype(np.float32)
    return x


def _bf16_ties():
    # halfway between neighbouring bfloat16 values: 1 + 2^-8 (to 1), 1 + 3 2^-8 (to 1 + 2^-6), ...
    k = np.arange(1, 200, 2, dtype=np.float64)
    return np.concatenate([1.0 + k * 2.0 ** -8, -(3.0 + k * 2.0 ** -7), 2.0 ** -120 * (1 + k * 2.0 ** -8)])


def _e4m3_ties():
    k = np.arange(1, 31, 2, dtype=np.float64)
    return np.concatenate([1.0 + k * 2.0 ** -4, 64.0 + k * 4.0, -(k * 2.0 ** -10), 2.0 ** -6 + k * 2.0 ** -10])


def test_bf16_rounding_matches_torch(orc):
    law = orc.Law.normal(0, 1).with_operand(orc.OPERAND_BF16)
    x = np.concatenate([_vals(np.random.default_rng(1)).astype(np.float64), _bf16_ties()])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    got = np.array([orc.operand_value(law, 0, v) for v in x])
    np.testing.assert_array_equal(got, ref)


def test_e4m3_rounding_matches_torch(orc):
    law = orc.Law.normal(0, 1).with_operand(orc.OPERAND_FP8_E4M3)   # no scale array: s = 0
    x = _vals(np.random.default_rng(2)).astype(np.float64)
    x = np.concatenate([x[np.abs(x) <= 448.0], _e4m3_ties(), [448.0, -448.0, 447.9, 432.0, 2.0 ** -9, 2.0 ** -10]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    got = np.array([orc.operand_value(law, 0, v) for v in x])
    np.testing.assert_array_equal(got, ref)
    # beyond the largest finite value: saturated
    assert orc.operand_value(law, 0, 1e6) == 448.0 and orc.operand_value(law, 0, -500.0) == -448.0


def test_e4m3_scale_is_undone_exactly(orc):
    s = np.array([5, -3, 0], dtype=np.int32)
    law = orc.Law.normal(0, 1).with_operand(orc.OPERAND_FP8_E4M3, s)
    rng = np.random.default_rng(3)
    for v in rng.standard_normal(2000) * 3:
        for i, e in enumerate(s):
            scaled = torch.tensor([math.ldexp(v, int(e))], dtype=torch.float32).clamp(-448, 448)
            ref = math.ldexp(float(scaled.to(torch.float8_e4m3fn).to(torch.float64)), -int(e))
            assert orc.operand_value(law, i, v) == ref


@pytest.mark.parametrize("bound", [1e-9, 0.013, 1.0, 3.0, 6.5, 8.0, 255.9, 256.0, 256.1, 1e4, 7.3e8])
def test_fp8_scale_rule(orc, bound):
    s = orc.fp8_scale_exponent(bound)
    if -20 < s < 20:
        assert math.ldexp(bound, s) <= 256.0 < math.ldexp(bound, s + 1)
    assert orc.fp8_scale_exponent(0.0) == 0
    assert orc.fp8_scale_exponent(1e-30) == 20 and orc.fp8_scale_exponent(1e30) == -20


def test_fp8_exponents_per_law(orc):
    assert list(orc.fp8_scale_exponents(orc.Law.normal(0.5, 1.0), 3, "A")) == [5, 5, 5]   # 6.5 -> 2^5
    assert list(orc.fp8_scale_exponents(orc.Law.uniform(-3.0, 1.0), 2, "B")) == [6, 6]    # 4 -> 2^6
    rng = np.random.default_rng(4)
    n, m = 7, 5
    mean = rng.standard_normal((n, m)) * 4       # A column-major: element (i, j) at j*m + i
    sd = rng.uniform(0.1, 2, (n, m))
    law = orc.Law.reparam(mean.ravel(), sd.ravel(), m)
    got = orc.fp8_scale_exponents(law, m, "A")
    for i in range(m):
        bound = max(abs(mean[j, i]) + 6 * sd[j, i] for j in range(n))
        assert got[i] == orc.fp8_scale_exponent(bound) or abs(bound * 2.0 ** got[i] - 256) < 1e-9


@pytest.mark.parametrize("operand", ["bf16", "fp8"])
def test_level_estimation_reads_rounded_operands(orc, operand):
    """Alg. 1 in an operand format equals the sketch of the materialised
    realisation with every entry rounded by PyTorch (FP8: under the scales)."""
    m, n, p, c = 5, 13, 4, 8
    la, lb = orc.Law.normal(0.7, 1.3), orc.Law.uniform(-0.4, 2.0)
    if operand == "bf16":
        ga, gb = la.with_operand(orc.OPERAND_BF16), lb.with_operand(orc.OPERAND_BF16)
    else:
        sa, sb = orc.fp8_scale_exponents(la, m, "A"), orc.fp8_scale_exponents(lb, p, "B")
        ga, gb = la.with_operand(orc.OPERAND_FP8_E4M3, sa), lb.with_operand(orc.OPERAND_FP8_E4M3, sb)
    st = orc.LevelState.empty(m, p)
    D = orc.level_estimation(st, m, n, p, ga, gb, c, 4, 9, 0, 2, 5, 6, want_samples=True)
    A, B = orc.realisation(9, 0, 2, 5, m, n, p, la, lb)

    def rnd(X, exps, axis):
        t = torch.from_numpy(X.astype(np.float32))
        if operand == "bf16":
            return t.to(torch.bfloat16).to(torch.float64).numpy()
        e = torch.from_numpy(exps.astype(np.float64))
        sc = torch.pow(2.0, e).unsqueeze(axis)
        q = (t.double() * sc).float().clamp(-448, 448).to(torch.float8_e4m3fn).to(torch.float64)
        return (q / sc).numpy()
    Aq = rnd(A, sa if operand == "fp8" else None, 1)
    Bq = rnd(B, sb if operand == "fp8" else None, 0)
    assert not np.array_equal(Aq, A)       # the rounding did something
    r = orc.draw_indices(9, 0, 2, 5, c, n)
    Zf = n / c * Aq[:, r] @ Bq[r, :]
    Zc = n / 4 * Aq[:, r[:4]] @ Bq[r[:4], :]
    np.testing.assert_allclose(D[0], Zf - Zc, rtol=1e-12, atol=1e-12 * np.abs(Zf).max())


def test_exact_operand_is_the_plain_estimator(orc):
    m, n, p, c, N = 6, 40, 5, [2, 4], [30, 15]
    la = orc.Law.normal(0.2, 1.0)
    a = orc.estimate(m, n, p, la, la, c, n_samples=N, seed=3)
    b = orc.estimate(m, n, p, la.with_operand(orc.OPERAND_EXACT), la.with_operand(orc.OPERAND_EXACT), c,
                     n_samples=N, seed=3)
    np.testing.assert_array_equal(a.Y, b.Y)
    np.testing.assert_array_equal(a.level_var, b.level_var)


def test_entry_variances_sum_to_level_variances(orc):
    m, n, p, c, N = 4, 30, 3, [2, 4, 8], [40, 20, 10]
    la = orc.Law.normal(1.0, 1.0)
    est = orc.estimate(m, n, p, la, la, c, n_samples=N, seed=8)
    np.testing.assert_allclose(est.entry_var.reshape(len(c), -1).sum(axis=1), est.level_var, rtol=1e-12)
    # per entry: the sample variance of the level samples themselves
    st = orc.LevelState.empty(m, p)
    D = orc.level_estimation(st, m, n, p, la, la, c[1], c[0], 8, 0, 1, 0, N[1], want_samples=True)
    np.testing.assert_allclose(est.entry_var[1], D.var(axis=0, ddof=1), rtol=1e-10)
    sd = est.entry_sd
    assert sd.shape == (m, p) and np.all(sd > 0)


def test_e4m3_round_to_nearest_bias_of_the_scaled_normal_law(orc):
    """Round-to-nearest on e4m3's grid is biased where the density falls
    across a power of two (the cell of 2^k reaches a quarter of the lower
    spacing below it and half of the upper one above it).  For N(0.5, 1)
    under its FP8 scale 2^5 (mean 16, sd 32) the rounded mean is low by about
    7.1e-4 relative, computed here by quadrature of the rounding against the
    normal density; A and B independent, a product's mean is low by twice
    that: 23 per entry of E[AB] = n mu^2 = 16384 at n = 65536, the size of the
    FP8 form's measured rounding error on that workload."""
    s = int(orc.fp8_scale_exponents(orc.Law.normal(0.5, 1.0), 1, "A")[0])
    assert s == 5
    mu, sd = 0.5 * 2.0 ** s, 2.0 ** s
    h = 2.0 ** -12
    x = np.arange(mu - 14 * sd, mu + 14 * sd, h)
    dens = np.exp(-0.5 * ((x - mu) / sd) ** 2) / (sd * math.sqrt(2.0 * math.pi))
    r = torch.from_numpy(np.clip(x, -448.0, 448.0).astype(np.float32)).to(torch.float8_e4m3fn).to(
        torch.float64).numpy()
    mean_x = float(np.sum(x * dens) * h)
    mean_r = float(np.sum(r * dens) * h)
    beta = (mean_r - mean_x) / mean_x
    assert abs(mean_x - mu) < 1e-9 * mu
    assert -7.4e-4 < beta < -6.8e-4
    per_entry = 65536 * 0.25 * (1.0 - (1.0 + beta) ** 2)
    assert 22.0 < per_entry < 24.5
