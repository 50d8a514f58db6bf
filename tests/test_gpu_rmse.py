"""End-to-end check of the target-RMSE mode on the GPU: eq. (28) allocates
N_l so that sum_l V_l / N_l = eps^2 / 2, and with f = identity the estimator
is unbiased (E[Y] = E[AB], telescoping), so over many independent estimates
the observed RMSE is eps / sqrt(2) up to the spread of a sample RMSE and the
pilot's error in V_l, and the mean has no bias.  The exact E[x^T y] and E[AB]
of i.i.d. laws are closed forms (n E[a] E[b] per entry).  A factor-2 error in
N_l, a wrong V_l or a missing level would move the observed RMSE outside the
band."""
import math

import numpy as np
import pytest

from gpu_helpers import flush

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _check(ys, exact, eps, name):
    ys = np.asarray(ys, dtype=np.float64)
    err2 = ((ys - exact) ** 2).reshape(len(ys), -1).sum(axis=1)
    rmse = math.sqrt(err2.mean())
    flush(f"  {name}: observed RMSE {rmse:.4g}, eps / sqrt(2) = {eps / math.sqrt(2):.4g}")
    # a sample RMSE over R estimates spreads by about 1 / sqrt(2 R) relative
    # (more for a sum over entries with heavier tails); the pilot adds ~10%
    assert 0.5 * eps / math.sqrt(2) < rmse < 1.35 * eps / math.sqrt(2), rmse
    bias = (ys - exact).reshape(len(ys), -1).mean(axis=0)
    assert np.linalg.norm(bias) < 5 * rmse / math.sqrt(len(ys)), np.linalg.norm(bias)


@pytest.mark.parametrize("word32", [False, True])
def test_inner_product_meets_eps(dev, word32):
    from paper_1904_00429_amd import Law, inner_product_estimate
    n, R = 1 << 16, 300
    exact = n * 0.5 * 0.5
    eps = 1e-2 * exact
    c = [16 << l for l in range(6)]
    flush(f"[rmse] inner n={n} {R} estimates word32={word32}")
    x = Law.uniform(0.5, 1.0)
    ys = [float(inner_product_estimate(n, x, x, c, rmse_target=eps, pilot=256, seed=1000 + r, prec="fp32",
                                       device=dev, index_word32=word32).Y.cpu()) for r in range(R)]
    _check(ys, exact, eps, "inner")


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_matrix_product_meets_eps(dev, prec):
    from paper_1904_00429_amd import Law, matmul_estimate
    m, n, p, R = 48, 2048, 40, 120
    exact = n * 0.5 * 0.5
    eps = 2e-2 * exact * math.sqrt(m * p)
    c = [8 << l for l in range(5)]
    flush(f"[rmse] matrix {m}x{n}x{p} {R} estimates {prec}")
    A = Law.normal(0.5, 1.0)
    ys = [matmul_estimate(m, n, p, A, A, c, rmse_target=eps, pilot=64, seed=2000 + r, prec=prec,
                          device=dev).Y.cpu().numpy() for r in range(R)]
    _check(ys, exact, eps, "matrix")
