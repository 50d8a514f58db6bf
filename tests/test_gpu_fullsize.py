"""Parity at the full sizes of the benchmarked workloads, in the launch
configurations bench.py times.

Inner product: x, y in R^(2^20), i.i.d. 0.5 + U(-1, 1), c_l = 64 * 2^l
(l = 0..8), target RMSE 1e-3 |E[x^T y]|, pilot 1024.

The oracle runs the same target-mode estimate (pilot, eq. (28), extension)
on the host, one thread per level (about 7e8 index draws).  FP64: the
scheduled N_l must agree exactly and the estimate to 1e-12.  FP32: the pilot
variances differ at ~1e-6 relative, so each N_l may move by one realisation;
the estimate and variances agree to 1e-5.
"""
import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from gpu_helpers import ENTRY_SD, QTOL, flush, rel_frob

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_inner_2pow20_target_mode_full(orc, dev, prec):
    from paper_1904_00429_amd import Law, inner_product_estimate, workloads
    wl = workloads.INNER_2POW20
    flush(f"full-size inner product prec={prec} n={wl.n} levels={len(wl.c)}")
    g = Law.uniform(wl.law_a[1], wl.law_a[2])
    est = inner_product_estimate(wl.n, g, g, wl.c, rmse_target=wl.rmse_target, pilot=wl.pilot,
                                 seed=wl.seed, prec=prec, level_means=True, device=dev)
    o = orc.Law.uniform(wl.law_a[1], wl.law_a[2])
    with ThreadPoolExecutor(max_workers=min(len(wl.c), os.cpu_count() or 4)) as pool:
        ref = orc.estimate(1, wl.n, 1, o, o, wl.c, rmse_target=wl.rmse_target, pilot=wl.pilot,
                           seed=wl.seed, pool=pool)
    flush(f"  gpu N={est.n_used}\n  orc N={list(ref.n_used)}")
    y = float(est.Y.cpu())
    V = np.array(est.level_var)
    if prec == "fp64":
        assert list(est.n_used) == list(ref.n_used)
        assert abs(y - ref.Y[0, 0]) <= 1e-12 * abs(ref.Y[0, 0])
        np.testing.assert_allclose(V, ref.level_var, rtol=1e-10)
    else:
        assert all(abs(a - b) <= 1 for a, b in zip(est.n_used, ref.n_used))
        assert abs(y - ref.Y[0, 0]) <= 1e-5 * abs(ref.Y[0, 0])
        np.testing.assert_allclose(V, ref.level_var, rtol=1e-5)
    # the target is met: predicted RMSE within the eps^2 / 2 variance budget
    assert est.rmse_est <= wl.rmse_target / math.sqrt(2) * 1.05


@pytest.mark.parametrize("prec, value16", [("fp64", False), ("bf16", True), ("bf16", False), ("fp32", False)])
def test_matmul_1024x65536x1024_target_mode_sampled_entries(orc, dev, prec, value16):
    """The precision-form workload at its full size and in the benchmark's
    launch configuration (target mode: 64-realisation pilot, eq. (28), then
    extension), checked at an 8 x 8 grid of output entries that the oracle
    computes one by one with the N_l the GPU used.

    FP64 1e-12 and FP32 1e-5 relative over the sampled entries; level means
    against their spread there (the sum of the sampled entries' level-sample
    variances).  BF16 against the oracle on the same BF16-rounded operands at
    1e-4, and against the exact oracle: RMS error over the sampled entries
    <= 5% of the estimator's own standard deviation there, every entry within
    0.1 of its standard deviation.  BF16 is timed with 16-bit value uniforms
    (eight per Philox call); the oracle then draws from the same 16-bit
    streams."""
    from paper_1904_00429_amd import Law, matmul_estimate, workloads
    wl = workloads.MATMUL_LARGE
    flush(f"full-size target-mode matmul prec={prec} value16={value16} m={wl.m} n={wl.n} p={wl.p}")
    g = Law.normal(wl.law_a[1], wl.law_a[2])
    est = matmul_estimate(wl.m, wl.n, wl.p, g, g, wl.c, rmse_target=wl.rmse_target, pilot=wl.pilot,
                          seed=3, prec=prec, level_means=True, device=dev, value16=value16)
    N = [int(x) for x in est.n_used]
    flush(f"  N_l = {N}")
    rows = list(range(3, wl.m, wl.m // 8))
    cols = list(range(wl.p - 1, 0, -(wl.p // 8)))
    o = orc.Law.normal(wl.law_a[1], wl.law_a[2])
    if value16:
        o = o.with_value16()
    with ThreadPoolExecutor(max_workers=min(len(wl.c), os.cpu_count() or 4)) as pool:
        ref = orc.estimate_entries(wl.m, wl.n, wl.p, o, o, wl.c, N, rows, cols, seed=3, pool=pool)
        ref_q = None
        if prec == "bf16":
            oq = o.with_operand(orc.OPERAND_BF16)
            ref_q = orc.estimate_entries(wl.m, wl.n, wl.p, oq, oq, wl.c, N, rows, cols, seed=3, pool=pool)
    ix = np.ix_(rows, cols)
    Y = est.Y.cpu().numpy()[ix]
    means = est.level_means.cpu().numpy()[(slice(None),) + ix]

    def close(ref, tol):
        r = rel_frob(Y, ref.Y)
        flush(f"  rel err {r:.3g}")
        assert r <= tol, r
        for l in range(len(wl.c)):
            d = float(np.linalg.norm(means[l] - ref.level_means[l]))
            spread = float(np.linalg.norm(ref.level_means[l])) if l == 0 else math.sqrt(float(ref.entry_var[l].sum()))
            assert d <= tol * spread, (l, d, spread)

    if prec in ("fp64", "fp32"):
        close(ref, 1e-12 if prec == "fp64" else 1e-5)
    else:
        sd2 = (ref.entry_var / ref.n_used[:, None, None]).sum(axis=0)
        rms = math.sqrt(float(np.mean((Y - ref.Y) ** 2)))
        worst = float(np.max(np.abs(Y - ref.Y) / np.sqrt(sd2)))
        flush(f"  bf16 RMS error {rms:.4g}, estimator sd {math.sqrt(float(np.mean(sd2))):.4g}, "
              f"max entry |dY| / sd {worst:.3g}")
        assert rms <= 0.05 * math.sqrt(float(np.mean(sd2)))
        assert worst <= ENTRY_SD["bf16"]
        close(ref_q, QTOL["bf16"])
