"""GPU parity at the largest n the library accepts (n < 2^32): the index
draw floor(x n / 2^64) and the value stream's column counter j = r at their
ends of range.  The laws are generated, so no operand of that length is ever
stored.  Inner product with 64-bit index words at n = 2^32 - 1 (prefix and
stride coupling), with 32-bit index words at n = 2^31 (the largest power of
two below 2^32), and a ragged matrix product at n = 2^32 - 1; FP64 1e-12,
FP32 1e-5, against the oracle on the same seeded streams."""
import numpy as np
import pytest

from gpu_helpers import flush, laws, rel_frob

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

N_MAX = 2 ** 32 - 1


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


INNER = [
    # n, law, ladder, N, precision, coupling, 32-bit index words
    (N_MAX, ("uniform", 0.5, 1.0), [4, 16, 64], [4000, 2000, 1000], "fp64", "prefix", False),
    (N_MAX, ("normal", 0.3, 1.0), [3, 9, 27], [4000, 2000, 1000], "fp64", "stride", False),
    (N_MAX, ("uniform", 0.5, 1.0), [64, 128, 512], [2000, 1000, 500], "fp32", "prefix", False),
    (2 ** 31, ("uniform", 0.5, 1.0), [6, 12, 48], [4000, 2000, 1000], "fp64", "prefix", True),
    (2 ** 31, ("normal", 0.5, 1.0), [64, 128, 256], [2000, 1000, 500], "fp32", "prefix", True),
]


@pytest.mark.parametrize("case", range(len(INNER)))
def test_inner_at_maximum_n(orc, dev, case):
    from paper_1904_00429_amd import inner_product_estimate
    n, law, c, N, prec, coupling, w32 = INNER[case]
    flush(f"[max n] inner n={n} c={c} {prec} {coupling} word32={w32}")
    ox, gx = laws(orc, law, dev)
    est = inner_product_estimate(n, gx, gx, c, n_samples=N, seed=41, prec=prec, level_means=True, device=dev,
                                 coupling=coupling, index_word32=w32)
    ref = orc.estimate(1, n, 1, ox, ox, c, n_samples=N, seed=41, coupling=coupling, index_word32=w32)
    tol = 1e-12 if prec == "fp64" else 1e-5
    y = float(est.Y.cpu())
    scale = abs(ref.Y[0, 0]) + float(np.sqrt(np.sum(np.asarray(ref.level_var) / np.asarray(N))))
    assert abs(y - ref.Y[0, 0]) <= tol * scale, (y, ref.Y[0, 0])
    np.testing.assert_allclose(est.level_var, ref.level_var, rtol=1e-10 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("prec, coupling", [("fp64", "prefix"), ("fp64", "stride"), ("fp32", "prefix")])
def test_matmul_at_maximum_n(orc, dev, prec, coupling):
    from paper_1904_00429_amd import matmul_estimate
    m, p, c, N = 33, 20, [2, 6, 18], [300, 150, 75]
    flush(f"[max n] matmul {m}x{N_MAX}x{p} c={c} {prec} {coupling}")
    oA, gA = laws(orc, ("normal", 0.5, 1.0), dev)
    est = matmul_estimate(m, N_MAX, p, gA, gA, c, n_samples=N, seed=43, prec=prec, level_means=True, device=dev,
                          coupling=coupling)
    ref = orc.estimate(m, N_MAX, p, oA, oA, c, n_samples=N, seed=43, coupling=coupling)
    tol = 1e-12 if prec == "fp64" else 1e-5
    assert rel_frob(est.Y.cpu().numpy(), ref.Y) <= tol, rel_frob(est.Y.cpu().numpy(), ref.Y)
    np.testing.assert_allclose(est.level_var, ref.level_var, rtol=1e-10 if prec == "fp64" else 1e-5)
