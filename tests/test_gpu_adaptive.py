"""GPU parity of the adaptive number of levels (Alg. 2's loop over L with the
bias tests of eq. (15) and eq. (27)) against the oracle's driver: the same
levels are run with the same N_l and the same stopping decision, and the
estimate agrees at the FP64 tolerance (1e-12); at a size the oracle is not
run on, the adaptive estimate equals a fixed-N run over the same
realisations (only the order of the statistics' merges differs)."""
import numpy as np
import pytest

from gpu_helpers import flush, laws, rel_frob

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _func(orc, name):
    from paper_1904_00429_amd import Func
    if name == "abs_step":
        return orc.Func.abs_step(2.0), Func.abs_step(2.0)
    if name == "inv_abs_step":
        return orc.Func.inv_abs_step(0.4, 0.01), Func.inv_abs_step(0.4, 0.01)
    return None, None


CASES = [
    ("matrix", None, 2.0),
    ("matrix", "abs_step", 0.3),
    ("inner", "inv_abs_step", 0.2),
    ("inner", None, 0.5),
]


@pytest.mark.parametrize("kind, fname, eps", CASES)
def test_adaptive_matches_oracle(orc, dev, kind, fname, eps):
    from paper_1904_00429_amd import inner_product_estimate, matmul_estimate
    m, n, p = (6, 100, 5) if kind == "matrix" else (1, 100, 1)
    c = [2, 4, 8, 16, 32]
    flush(f"[adaptive] {kind} {fname} eps {eps}")
    oA, gA = laws(orc, ("normal", 0.1, 0.1), dev)
    of, gf = _func(orc, fname)
    ref = orc.estimate(m, n, p, oA, oA, c, rmse_target=eps, pilot=20, seed=5, func=of, adaptive=kind)
    if kind == "matrix":
        est = matmul_estimate(m, n, p, gA, gA, c, rmse_target=eps, pilot=20, seed=5, prec="fp64", device=dev,
                              func=gf, adaptive=True, level_means=True)
    else:
        est = inner_product_estimate(n, gA, gA, c, rmse_target=eps, pilot=20, seed=5, prec="fp64", device=dev,
                                     func=gf, adaptive=True, level_means=True)
    flush(f"  levels {est.levels_used} (oracle {ref.levels_used}), N {est.n_used}")
    assert est.levels_used == ref.levels_used
    assert est.bias_test_passed == ref.bias_test_passed
    assert list(est.n_used) == [int(x) for x in ref.n_used]
    Y = est.Y.cpu().numpy().reshape(ref.Y.shape)
    assert rel_frob(Y, ref.Y) <= 1e-12
    np.testing.assert_allclose(est.level_var[:est.levels_used], ref.level_var[:ref.levels_used], rtol=1e-10)


def test_adaptive_equals_fixed_run_on_the_same_realisations(orc, dev):
    from paper_1904_00429_amd import matmul_estimate
    m, n, p = 200, 3000, 150
    c = [4, 8, 16, 32, 64, 128]
    flush("[adaptive] 200 x 3000 x 150 against fixed N")
    _, gA = laws(orc, ("normal", 0.02, 0.05), dev)
    _, gf = _func(orc, "abs_step")
    est = matmul_estimate(m, n, p, gA, gA, c, rmse_target=5.0, pilot=16, seed=8, prec="fp64", device=dev,
                          func=gf, adaptive=True)
    used = est.levels_used
    flush(f"  levels {used}, N {est.n_used}, passed {est.bias_test_passed}")
    assert 3 <= used <= len(c)
    fixed = matmul_estimate(m, n, p, gA, gA, c[:used], n_samples=est.n_used[:used], seed=8, prec="fp64",
                            device=dev, func=gf)
    assert rel_frob(est.Y.cpu().numpy(), fixed.Y.cpu().numpy()) <= 1e-12
    np.testing.assert_allclose(est.level_var[:used], fixed.level_var, rtol=1e-10)
