"""GPU parity of the batching form (one pipeline over many uneven products,
hipGraph replay, autotuner) and of the FP8 precision form, against the oracle
run product by product with the same stream ids.

Tolerances: FP64 1e-12, FP32 1e-5 (relative Frobenius); BF16 0.05 RMSE_est;
FP8 e4m3: ||Y - Y_oracle||_F <= 0.25 RMSE_est and V_l within 15% (each operand
carries up to 2^-4 relative rounding, about 4-7% of the sampling spread of a
single level sample for these laws, shrinking with N_l in the estimate)."""
import json
import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from gpu_helpers import ENTRY_SD, QTOL, check_estimate, flush, laws, operand_law, rel_frob

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SHAPES = [(64, 500, 64), (128, 1234, 192), (64, 4096, 320), (256, 777, 64), (192, 2000, 128), (100, 999, 37)]
MUS = [0.1, 0.7, 1.3, 1.9, 0.4, 1.0]
C, N = [16, 32, 64], [60, 30, 15]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def refs(orc):
    def one(i):
        m, n, p = SHAPES[i]
        law = orc.Law.normal(MUS[i], 1.0)
        return orc.estimate(m, n, p, law, law, C, n_samples=N, seed=17, problem=100 + i)
    with ThreadPoolExecutor(max_workers=min(len(SHAPES), os.cpu_count() or 4)) as ex:
        return list(ex.map(one, range(len(SHAPES))))


def _batch(dev, prec, tuning=None):
    from paper_1904_00429_amd import BatchedEstimate, BatchProblem, Law
    probs = [BatchProblem(m, n, p, Law.normal(mu, 1.0), Law.normal(mu, 1.0), 100 + i)
             for i, ((m, n, p), mu) in enumerate(zip(SHAPES, MUS))]
    return BatchedEstimate(probs, C, N, seed=17, prec=prec, tuning=tuning, device=dev)


class _BatchEntry:
    """One product of a batch in the shape check_estimate reads."""
    def __init__(self, Y, V, ref):
        self.Y, self.level_var, self.level_means = Y, list(V), None
        self.n_used, self.rmse_est = list(ref.n_used), float(np.sqrt(np.sum(np.asarray(V) / ref.n_used)))


def _rounded_refs(orc, prec):
    def one(i):
        m, n, p = SHAPES[i]
        law = orc.Law.normal(MUS[i], 1.0)
        return orc.estimate(m, n, p, operand_law(orc, law, prec, m, "A"), operand_law(orc, law, prec, p, "B"),
                            C, n_samples=N, seed=17, problem=100 + i)
    with ThreadPoolExecutor(max_workers=min(len(SHAPES), os.cpu_count() or 4)) as ex:
        return list(ex.map(one, range(len(SHAPES))))


def _check(est, V, refs, prec, refs_q=None):
    for i, ref in enumerate(refs):
        check_estimate(_BatchEntry(est.Y[i], V[:, i], ref), ref, prec, None if refs_q is None else refs_q[i],
                       f"product {i}")


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16", "fp8"])
@pytest.mark.parametrize("tile", [64, 128])
def test_batched_matches_oracle(orc, dev, refs, prec, tile):
    flush(f"batched prec={prec} tile={tile}")
    est = _batch(dev, prec, {"tile": tile})
    V = est.run(level_var=True)
    _check(est, V, refs, prec, _rounded_refs(orc, prec) if prec in ("bf16", "fp8") else None)


def test_graph_replays_match_eager(orc, dev, refs):
    """A captured graph replayed several times, with other device work and
    synchronisations in between, reproduces the eager result every time."""
    est = _batch(dev, "fp32", {"tile": 64})
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
    V = est.run(level_var=True)
    _check(est, V, refs, "fp32")


def test_fp8_single_product(orc, dev):
    from paper_1904_00429_amd import matmul_estimate
    m, n, p, c, N = 96, 3000, 160, [16, 32, 64, 128], [400, 200, 100, 50]
    oA, gA = laws(orc, ("normal", 1.5, 1.0), dev)
    oB, gB = laws(orc, ("uniform", 0.3, 2.0), dev)
    est = matmul_estimate(m, n, p, gA, gB, c, n_samples=N, seed=4, prec="fp8", level_means=True, device=dev)
    ref = orc.estimate(m, n, p, oA, oB, c, n_samples=N, seed=4)
    ref_q = orc.estimate(m, n, p, operand_law(orc, oA, "fp8", m, "A"), operand_law(orc, oB, "fp8", p, "B"), c,
                         n_samples=N, seed=4)
    check_estimate(est, ref, "fp8", ref_q, "fp8 single")


def test_batched_rejects_duplicate_streams(dev):
    from paper_1904_00429_amd import BatchedEstimate, BatchProblem, Law, MLMCError
    probs = [BatchProblem(64, 100, 64, Law.normal(0, 1), Law.normal(0, 1), 5) for _ in range(2)]
    with pytest.raises(MLMCError):
        BatchedEstimate(probs, [4, 8], [10, 5], device=dev)


def test_autotuner_picks_and_caches(dev, tmp_path, monkeypatch):
    from paper_1904_00429_amd import BatchProblem, Law, autotune
    monkeypatch.setenv("MLMC_AUTOTUNE_CACHE", str(tmp_path / "cache.json"))
    probs = [BatchProblem(m, n, p, Law.normal(mu, 1.0), Law.normal(mu, 1.0), i)
             for i, ((m, n, p), mu) in enumerate(zip(SHAPES, MUS))]
    best = autotune.tune(probs, C, N, prec="fp8", device=dev)
    assert best in autotune.CANDIDATES
    cached = json.load(open(tmp_path / "cache.json"))
    assert len(cached) == 1 and list(cached.values())[0]["best"] == best
    assert autotune.tune(probs, C, N, prec="fp8", device=dev) == best


def _full_batch(orc, value16, operand=None):
    """The benchmarked batch (256 uneven products, c_l = 16 * 2^l, l = 0..6,
    N_l = 2048 * 2^-l); the oracle evaluates every 4th product at a 4 x 4 grid
    of entries, with the 16-bit value uniforms when value16 is set, on
    operands rounded to `operand` when given."""
    from paper_1904_00429_amd import workloads
    shapes, mus, c, N = workloads.batched_products()
    picked = list(range(0, len(shapes), 4))

    def one(i):
        m, n, p = shapes[i]
        law = orc.Law.normal(mus[i], 1.0)
        if value16:
            law = law.with_value16()
        la = lb = law
        if operand:
            la, lb = operand_law(orc, law, operand, m, "A"), operand_law(orc, law, operand, p, "B")
        rows = [0, m // 3, (2 * m) // 3, m - 1]
        cols = [p - 1, p // 2, 1, p // 4]
        return rows, cols, orc.estimate_entries(m, n, p, la, lb, c, N, rows, cols, seed=0, problem=i)
    with ThreadPoolExecutor(max_workers=os.cpu_count() or 4) as ex:
        refs = list(ex.map(one, picked))
    return shapes, mus, c, N, picked, refs


@pytest.fixture(scope="module")
def full_batch(orc):
    return _full_batch(orc, False)


@pytest.fixture(scope="module")
def full_batch16(orc):
    return _full_batch(orc, True)


@pytest.fixture(scope="module")
def full_batch_fp8(orc):
    return _full_batch(orc, False, "fp8")


@pytest.fixture(scope="module")
def full_batch16_fp8(orc):
    return _full_batch(orc, True, "fp8")


@pytest.mark.parametrize("prec, value16", [("fp8", True), ("fp8", False), ("fp32", False)])
@pytest.mark.parametrize("tile", [64, 128])
def test_full_batch_sampled_entries(request, dev, prec, value16, tile):
    """The benchmarked batch in its launch configuration (one captured graph
    per estimate, both tile shapes the autotuner chooses between; FP8 is timed
    with 16-bit value uniforms), checked at sampled entries of sampled
    products."""
    from paper_1904_00429_amd import BatchedEstimate, BatchProblem, Law
    shapes, mus, c, N, picked, refs = request.getfixturevalue("full_batch16" if value16 else "full_batch")
    flush(f"full batch prec={prec} value16={value16} tile={tile} products={len(shapes)}")
    probs = [BatchProblem(m, n, p, Law.normal(mu, 1.0), Law.normal(mu, 1.0), i)
             for i, ((m, n, p), mu) in enumerate(zip(shapes, mus))]
    est = BatchedEstimate(probs, c, N, seed=0, prec=prec, tuning={"tile": tile}, device=dev, value16=value16)
    est.capture()
    est.replay()
    torch.cuda.synchronize()
    refs_q = None
    if prec == "fp8":
        refs_q = request.getfixturevalue("full_batch16_fp8" if value16 else "full_batch_fp8")[5]
    err2 = var2 = ref2 = 0.0
    worst = worst_q = 0.0
    for t, (i, (rows, cols, ref)) in enumerate(zip(picked, refs)):
        Y = est.Y[i].cpu().numpy()[np.ix_(rows, cols)]
        err2 += float(np.sum((Y - ref.Y) ** 2))
        ref2 += float(np.sum(ref.Y ** 2))
        sd2 = (ref.entry_var / ref.n_used[:, None, None]).sum(axis=0)
        var2 += float(np.sum(sd2))
        if prec == "fp32":
            assert rel_frob(Y, ref.Y) <= 1e-5, (i, rel_frob(Y, ref.Y))
        else:
            worst = max(worst, float(np.max(np.abs(Y - ref.Y) / np.sqrt(sd2))))
            yq = refs_q[t][2].Y
            worst_q = max(worst_q, float(np.linalg.norm(Y - yq)) / (float(np.linalg.norm(yq)) + math.sqrt(float(np.sum(sd2)))))
    est.release()
    flush(f"  RMS error / estimator sd = {np.sqrt(err2 / var2):.4g}, rel = {np.sqrt(err2 / ref2):.3g}, "
          f"max entry |dY| / sd = {worst:.3g}, rel vs rounded-operand oracle {worst_q:.3g}")
    if prec == "fp8":
        assert np.sqrt(err2 / var2) <= 0.25
        assert worst <= ENTRY_SD["fp8"]
        assert worst_q <= QTOL["fp8"]


@pytest.mark.parametrize("prec,tile", [("fp64", 64), ("fp32", 64), ("fp32", 128), ("fp8", 64)])
def test_batched_large_mean_ragged(orc, dev, prec, tile):
    """Products whose level-0 mean is far above its spread, with ragged tiles:
    the statistics shifted by E[D] (i.i.d. laws) must match the oracle."""
    from paper_1904_00429_amd import BatchedEstimate, BatchProblem, Law
    shapes = [(100, 600, 37), (64, 300, 64), (130, 450, 70)]
    c, N = [4, 8, 16], [300, 150, 60]
    la, lb = (5.0, 0.1), (-3.0, 0.25)
    flush(f"batched large mean prec={prec} tile={tile}")
    probs = [BatchProblem(m, n, p, Law.normal(*la), Law.normal(*lb), 40 + i) for i, (m, n, p) in enumerate(shapes)]
    est = BatchedEstimate(probs, c, N, seed=5, prec=prec, tuning={"tile": tile}, device=dev)
    V = est.run(level_var=True)
    for i, (m, n, p) in enumerate(shapes):
        ref = orc.estimate(m, n, p, orc.Law.normal(*la), orc.Law.normal(*lb), c, n_samples=N, seed=5, problem=40 + i)
        Y = est.Y[i].cpu().numpy()
        if prec == "fp8":
            # e4m3 keeps 4 significant bits: 5 +- 0.1 and -3 +- 0.25 lose most of
            # their spread, so the estimate is compared with the oracle on the
            # same rounded operands (V_l included), and its mean level with the
            # exact oracle
            la_o, lb_o = orc.Law.normal(*la), orc.Law.normal(*lb)
            ref_q = orc.estimate(m, n, p, operand_law(orc, la_o, "fp8", m, "A"), operand_law(orc, lb_o, "fp8", p, "B"),
                                 c, n_samples=N, seed=5, problem=40 + i)
            rq = rel_frob(Y, ref_q.Y)
            flush(f"  product {i}: rel err vs rounded-operand oracle {rq:.3g}, V_l {V[:, i]} vs {ref_q.level_var}")
            assert rq <= QTOL["fp8"], (i, rq)
            np.testing.assert_allclose(V[:, i], ref_q.level_var, rtol=QTOL["fp8"])
            assert rel_frob(Y, ref.Y) <= 0.02, (i, rel_frob(Y, ref.Y))
            continue
        tol = 1e-12 if prec == "fp64" else 1e-5
        assert rel_frob(Y, ref.Y) <= tol, (i, rel_frob(Y, ref.Y))
        np.testing.assert_allclose(V[:, i], ref.level_var, rtol=1e-10 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batched_one_group_per_pass(orc, dev, refs, prec):
    """target_blocks = 1 leaves one realisation group per tile and pass, so
    each pass is merged into the level state by the sketch epilogue itself."""
    flush(f"batched one group per pass prec={prec}")
    est = _batch(dev, prec, {"tile": 64, "target_blocks": 1})
    V = est.run(level_var=True)
    _check(est, V, refs, prec)
