"""GPU parity of the MLMC estimators against the oracle on the same seeded
inputs: estimate Y (eq. (10)), level means Ybar_l (eq. (9)), level variances
V_l (Remark 3.6) and, in target mode, the scheduled N_l (eq. (28)).

Tolerances: gpu_helpers.check_estimate (FP64 1e-12 for Y and the level
means, 1e-10 for V_l; FP32 1e-5; BF16 against the oracle on the same rounded
operands at 1e-4, and against the exact oracle within 0.05 RMSE_est overall
and 0.1 of the estimator's standard deviation at every entry).
"""
import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from gpu_helpers import check_estimate, flush, laws, operand_law, rel_frob

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def pool():
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 4)) as ex:
        yield ex


def _compare(est, ref, prec, ref_q=None, label=""):
    check_estimate(est, ref, prec, ref_q, label)


# ----------------------------------------------------------------- inner product
INNER_CASES = [
    # n, law x, law y, ladder, N
    (4096, ("uniform", 0.5, 1.0), ("uniform", 0.5, 1.0), [16, 32, 64, 128], [3000, 1500, 700, 300]),
    (100003, ("normal", 1.0, 2.0), ("normal", -0.5, 1.0), [3, 6, 12, 24, 48], [2000, 900, 500, 200, 77]),
    (2**20, ("uniform", 0.5, 1.0), ("normal", 2.0, 1.0), [64, 128, 256, 512, 1024, 2048], [4000, 2000, 800, 400, 130, 65]),
    (5000, ("reparam",), ("reparam",), [1, 2, 4, 8], [1000, 500, 300, 101]),
    (1, ("uniform", 0.5, 1.0), ("normal", 1.0, 1.0), [1, 2, 4], [50, 20, 10]),
    (7, ("normal", 0.0, 1.0), ("uniform", 0.0, 2.0), [5, 10, 40, 80, 1280], [3, 2, 2, 5, 2]),
]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", range(len(INNER_CASES)))
def test_inner_fixed(orc, dev, pool, prec, case):
    from paper_1904_00429_amd import inner_product_estimate
    n, lx, ly, c, N = INNER_CASES[case]
    flush(f"inner fixed case={case} prec={prec} n={n} c={c} N={N}")
    rng = np.random.default_rng(case)
    mx = rng.standard_normal(n).astype(np.float32) if lx[0] == "reparam" else None
    sx = rng.uniform(0.1, 1, n).astype(np.float32) if lx[0] == "reparam" else None
    ox, gx = laws(orc, lx, dev, mx, sx)
    oy, gy = laws(orc, ly, dev, mx, sx)
    est = inner_product_estimate(n, gx, gy, c, n_samples=N, seed=5, prec=prec, level_means=True, device=dev)
    ref = orc.estimate(1, n, 1, ox, oy, c, n_samples=N, seed=5, pool=pool)
    _compare(est, ref, prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_inner_target_mode(orc, dev, pool, prec):
    from paper_1904_00429_amd import inner_product_estimate
    n, c = 2**16, [32 * 2**l for l in range(6)]
    flush(f"inner target prec={prec}")
    ox, gx = laws(orc, ("uniform", 0.5, 1.0), dev)
    eps = 5e-3 * n * 0.25
    est = inner_product_estimate(n, gx, gx, c, rmse_target=eps, pilot=500, seed=11, prec=prec,
                                 level_means=True, device=dev)
    ref = orc.estimate(1, n, 1, ox, ox, c, rmse_target=eps, pilot=500, seed=11, pool=pool)
    if prec == "fp64":
        _compare(est, ref, prec)
    else:
        # FP32 pilot variances differ from FP64 at ~1e-6 relative: the ceiling
        # in eq. (28) may move by one realisation
        assert all(abs(a - b) <= 1 for a, b in zip(est.n_used, ref.n_used)), (est.n_used, ref.n_used)
    assert est.rmse_est <= eps / math.sqrt(2) * 1.1


def test_inner_shared_telescoping(orc, dev):
    """Property: with shared realisations and equal N_l the level means sum to
    the finest-level sample mean (eq. (10)); computed on the GPU path alone."""
    from paper_1904_00429_amd import inner_product_estimate
    n, c, N = 10007, [4, 8, 16, 32], 700
    _, gx = laws(orc, ("normal", 1.0, 1.0), dev)
    est = inner_product_estimate(n, gx, gx, c, n_samples=[N] * 4, seed=3, shared=True, prec="fp64",
                                 level_means=True, device=dev)
    fin = inner_product_estimate(n, gx, gx, [c[-1]], n_samples=[N], seed=3, shared=True, prec="fp64", device=dev)
    y, f = float(est.Y.cpu()), float(fin.Y.cpu())
    assert abs(y - f) <= 1e-12 * abs(f)


# ------------------------------------------------------------------ matrix product
MATMUL_CASES = [
    # m, n, p, law A, law B, ladder, N, precisions
    (64, 256, 64, ("normal", 1.0, 1.0), ("normal", 1.0, 1.0), [4, 8, 16, 32], [1000, 500, 250, 125], ["fp64", "fp32"]),
    (37, 500, 45, ("normal", 0.5, 1.0), ("uniform", 0.2, 1.5), [5, 10, 20], [700, 300, 100], ["fp64", "fp32", "bf16", "fp8"]),
    (300, 1000, 200, ("normal", 0.5, 1.0), ("normal", 0.5, 1.0), [8, 16, 32], [1000, 300, 90], ["fp64", "fp32", "bf16"]),
    (70, 3000, 129, ("reparam",), ("reparam",), [16, 32, 64, 128], [400, 200, 100, 50], ["fp64", "fp32", "bf16", "fp8"]),
    (1, 2000, 1, ("uniform", 0.5, 1.0), ("uniform", 0.5, 1.0), [2, 4, 8], [500, 200, 100], ["fp64", "fp32"]),
    # at least 512 x 512 (the FP64 128 x 128 tiles of 4 x 4 waves), ragged
    (520, 700, 600, ("normal", 0.5, 1.0), ("normal", 0.3, 1.0), [4, 8], [60, 30], ["fp64"]),
    # |E[D_0]| far above its spread (mean^2 / variance ~ 1e3 per entry), ragged tiles:
    # the level-0 statistics must not cancel
    (100, 600, 37, ("normal", 5.0, 0.1), ("uniform", -3.0, 0.05), [4, 8, 16], [400, 200, 100], ["fp64", "fp32"]),
]


@pytest.mark.parametrize("case,prec", [(i, pr) for i, cs in enumerate(MATMUL_CASES) for pr in cs[7]])
def test_matmul_fixed(orc, dev, pool, case, prec):
    from paper_1904_00429_amd import matmul_estimate
    m, n, p, la, lb, c, N, _ = MATMUL_CASES[case]
    flush(f"matmul fixed case={case} prec={prec} m={m} n={n} p={p} c={c} N={N}")
    rng = np.random.default_rng(100 + case)
    ma = rng.standard_normal((n, m)).astype(np.float32)
    sa = rng.uniform(0.1, 1, (n, m)).astype(np.float32)
    mb = rng.standard_normal((n, p)).astype(np.float32)
    sb = rng.uniform(0.1, 1, (n, p)).astype(np.float32)
    oA, gA = laws(orc, la, dev, ma, sa)
    oB, gB = laws(orc, lb, dev, mb, sb)
    est = matmul_estimate(m, n, p, gA, gB, c, n_samples=N, seed=21, prec=prec, level_means=True, device=dev)
    ref = orc.estimate(m, n, p, oA, oB, c, n_samples=N, seed=21, pool=pool)
    ref_q = None
    if prec in ("bf16", "fp8"):
        ref_q = orc.estimate(m, n, p, operand_law(orc, oA, prec, m, "A"), operand_law(orc, oB, prec, p, "B"), c,
                             n_samples=N, seed=21, pool=pool)
    _compare(est, ref, prec, ref_q, f"case {case}")


def test_matmul_many_passes(orc, dev, pool, monkeypatch):
    """A gather budget far below one level forces many passes per level and
    several realisations per sketch group."""
    from paper_1904_00429_amd import matmul_estimate
    monkeypatch.setenv("MLMC_GATHER_BUDGET", str(200 * 1024))
    m, n, p, c, N = 130, 777, 70, [6, 12, 24], [900, 400, 150]
    flush("matmul many passes")
    oA, gA = laws(orc, ("normal", 0.3, 1.0), dev)
    oB, gB = laws(orc, ("normal", -0.2, 2.0), dev)
    for prec in ("fp64", "fp32"):
        est = matmul_estimate(m, n, p, gA, gB, c, n_samples=N, seed=8, prec=prec, level_means=True, device=dev)
        ref = orc.estimate(m, n, p, oA, oB, c, n_samples=N, seed=8, pool=pool)
        _compare(est, ref, prec)


def test_matmul_target_mode(orc, dev, pool):
    from paper_1904_00429_amd import matmul_estimate
    m, n, p, c = 20, 4096, 24, [8, 16, 32, 64]
    flush("matmul target mode")
    oA, gA = laws(orc, ("normal", 1.0, 1.0), dev)
    eps = 2e-2 * n * math.sqrt(m * p)
    est = matmul_estimate(m, n, p, gA, gA, c, rmse_target=eps, pilot=64, seed=2, prec="fp64",
                          level_means=True, device=dev)
    ref = orc.estimate(m, n, p, oA, oA, c, rmse_target=eps, pilot=64, seed=2, pool=pool)
    _compare(est, ref, "fp64")
    assert est.rmse_est <= eps / math.sqrt(2) * 1.2


def test_matmul_shared_telescoping(orc, dev, pool):
    from paper_1904_00429_amd import matmul_estimate
    m, n, p, c, N = 33, 300, 17, [2, 4, 8, 16], 200
    oA, gA = laws(orc, ("normal", 1.0, 1.0), dev)
    est = matmul_estimate(m, n, p, gA, gA, c, n_samples=[N] * 4, seed=4, shared=True, prec="fp64",
                          level_means=True, device=dev)
    st = orc.LevelState.empty(m, p)
    orc.level_estimation(st, m, n, p, oA, oA, c[-1], 0, 4, 0, orc.SHARED_LEVEL_FIELD, 0, N)
    assert rel_frob(est.Y.cpu().numpy(), st.mean.reshape(m, p)) <= 1e-12


def test_budget_error(dev):
    from paper_1904_00429_amd import MLMCError, Law, matmul_estimate
    with pytest.raises(MLMCError) as ei:
        matmul_estimate(8, 1000, 8, Law.normal(1, 1), Law.normal(1, 1), [4, 8], rmse_target=1e-3,
                        pilot=16, max_total_draws=10**6, device=dev)
    assert ei.value.status == 3
