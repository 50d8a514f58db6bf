"""Run-to-run reproducibility of the optional forms: the same seed gives the
same estimate bit for bit (the statistics merge in a fixed order), and a
captured batched graph replays its eager result, with the stride coupling
and the 16-bit values, with the laws of Sec. 4, and for the inner product
with 32-bit index words."""
import pytest

from gpu_helpers import flush

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.mark.parametrize("kw", [dict(coupling="stride"), dict(value16=True), dict(coupling="stride", value16=True)])
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_matmul_twice_is_bitwise_equal(dev, kw, prec):
    from paper_1904_00429_amd import Law, matmul_estimate
    flush(f"[repro] matmul {prec} {kw}")
    A = Law.normal(0.5, 1.0)
    runs = [matmul_estimate(200, 3000, 130, A, A, [4, 8, 16, 32], rmse_target=200.0, pilot=32, seed=11, prec=prec,
                            device=dev, **kw) for _ in range(2)]
    assert torch.equal(runs[0].Y, runs[1].Y)
    assert runs[0].n_used == runs[1].n_used


@pytest.mark.parametrize("kw", [dict(index_word32=True), dict(index_word32=True, coupling="stride")])
def test_inner_twice_is_bitwise_equal(dev, kw):
    from paper_1904_00429_amd import Law, inner_product_estimate
    flush(f"[repro] inner {kw}")
    x = Law.uniform(0.5, 1.0)
    runs = [inner_product_estimate(1 << 20, x, x, [64, 128, 256, 512], rmse_target=300.0, pilot=256, seed=3,
                                   prec="fp32", device=dev, **kw) for _ in range(2)]
    assert torch.equal(runs[0].Y, runs[1].Y)


def test_experiment_laws_twice_is_bitwise_equal(dev):
    from paper_1904_00429_amd import Func, Law, matmul_estimate
    flush("[repro] laws of Sec. 4.2")
    A, B = Law.sin_ramp(1e-3, 0.5), Law.cos_poisson_step(2.0, 0.2)
    runs = [matmul_estimate(100, 1000, 70, A, B, [1, 10, 100], n_samples=[2000, 500, 100], seed=2, prec="fp32",
                            device=dev, func=Func.abs_step(2.0)) for _ in range(2)]
    assert torch.equal(runs[0].Y, runs[1].Y)


@pytest.mark.parametrize("kw", [dict(coupling="stride"), dict(value16=True)])
def test_graph_replays_match_eager(dev, kw):
    from paper_1904_00429_amd import BatchedEstimate, BatchProblem, Law
    flush(f"[repro] graph {kw}")
    shapes = [(64, 500, 64), (128, 900, 37), (100, 2000, 192)]
    probs = [BatchProblem(m, n, p, Law.normal(0.2 * i, 1.0), Law.normal(0.5, 1.0), i)
             for i, (m, n, p) in enumerate(shapes)]
    est = BatchedEstimate(probs, [8, 16, 32], [200, 100, 50], seed=4, prec="fp32", device=dev, **kw)
    est.run()
    torch.cuda.synchronize()
    eager = [y.clone() for y in est.Y]
    est.capture()
    for r in range(3):
        for y in est.Y:
            y.fill_(float("nan"))
        junk = torch.randn(1 << 20, device=dev).sum()
        torch.cuda.synchronize()
        est.replay()
        torch.cuda.synchronize()
        for y, e in zip(est.Y, eager):
            assert torch.equal(y, e), f"replay {r} differs"
        del junk
    est.release()
