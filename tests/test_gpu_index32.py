"""GPU parity of the 32-bit index words of the inner-product kernel (four
draws per Philox call, r = floor(w n / 2^32), power-of-two n) against the
oracle's word32 mode on the same seeded inputs: ladders whose c_l and c_{l-1}
are and are not multiples of four (the quad that straddles the coarse
boundary, the partial last quad), n = 1, a target function, the stride
coupling, target mode; FP64 1e-12, FP32 1e-5."""
import numpy as np
import pytest

from gpu_helpers import flush, laws

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


CASES = [
    # n, law, ladder, N, precision, f, coupling
    (4096, ("uniform", 0.5, 1.0), [16, 64, 128], [4000, 2000, 1000], "fp64", None, "prefix"),
    (1024, ("normal", 0.3, 1.0), [3, 6, 18, 54], [4000, 2000, 1000, 500], "fp64", None, "prefix"),
    (1, ("normal", 0.3, 1.0), [1, 2, 6], [1000, 500, 200], "fp64", None, "prefix"),
    (2048, ("normal", 0.1, 0.1), [2, 6, 12, 36], [4000, 2000, 1000, 500], "fp64", "inv_abs_step", "prefix"),
    (1024, ("uniform", 0.5, 1.0), [1, 3, 9, 27], [4000, 2000, 1000, 500], "fp64", None, "stride"),
    (2 ** 20, ("uniform", 0.5, 1.0), [64, 128, 256, 512], [800, 400, 200, 100], "fp32", None, "prefix"),
    (2 ** 16, ("normal", 0.5, 1.0), [5, 10, 40, 120], [2000, 1000, 500, 250], "fp32", None, "prefix"),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_inner_index32_matches_oracle(orc, dev, case):
    from paper_1904_00429_amd import Func, inner_product_estimate
    n, law, c, N, prec, fname, coupling = CASES[case]
    flush(f"[index32] n={n} c={c} {prec} {fname} {coupling}")
    ox, gx = laws(orc, law, dev)
    of = orc.Func.inv_abs_step(0.4, 0.01) if fname else None
    gf = Func.inv_abs_step(0.4, 0.01) if fname else None
    est = inner_product_estimate(n, gx, gx, c, n_samples=N, seed=29, prec=prec, level_means=True, device=dev,
                                 func=gf, coupling=coupling, index_word32=True)
    ref = orc.estimate(1, n, 1, ox, ox, c, n_samples=N, seed=29, func=of, coupling=coupling, index_word32=True)
    tol = 1e-12 if prec == "fp64" else 1e-5
    y = float(est.Y.cpu())
    scale = abs(ref.Y[0, 0]) + float(np.sqrt(np.sum(np.asarray(ref.level_var) / np.asarray(N))))
    assert abs(y - ref.Y[0, 0]) <= tol * scale, (y, ref.Y[0, 0])
    # (n = 1: D_l = 0 for l >= 1 up to rounding, which the two sides leave differently)
    np.testing.assert_allclose(est.level_var, ref.level_var, rtol=1e-10 if prec == "fp64" else 1e-5,
                               atol=1e-20 * max(ref.level_var))
    if n > 1:
        # a different index stream from the 64-bit draws
        other = orc.estimate(1, n, 1, ox, ox, c, n_samples=N, seed=29, func=of, coupling=coupling)
        assert other.Y[0, 0] != ref.Y[0, 0]


def test_inner_index32_target_mode(orc, dev):
    from paper_1904_00429_amd import inner_product_estimate
    n, c = 4096, [8, 16, 32, 64]
    flush("[index32] target mode")
    ox, gx = laws(orc, ("uniform", 0.5, 1.0), dev)
    eps = 2.0
    est = inner_product_estimate(n, gx, gx, c, rmse_target=eps, pilot=64, seed=3, prec="fp64", device=dev,
                                 index_word32=True)
    ref = orc.estimate(1, n, 1, ox, ox, c, rmse_target=eps, pilot=64, seed=3, index_word32=True)
    assert list(est.n_used) == [int(x) for x in ref.n_used]
    assert abs(float(est.Y.cpu()) - ref.Y[0, 0]) <= 1e-12 * abs(ref.Y[0, 0])
