"""GPU parity of the set form of a realisation (the note after Alg. 1 in
Sec. 3.1: the index tuple as distinct indices with multiplicities, each
distinct column generated once) against the oracle's set form, on workloads
where repeats are the rule (c_l up to several times n): FP64 1e-12 and FP32
1e-5 (relative Frobenius, V_l likewise), single products and a batch, both
couplings.  The set form must also equal the default tuple form up to the
order of the sums."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from gpu_helpers import check_estimate, flush, rel_frob

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


CASES = [
    dict(m=40, n=37, p=52, c=[8, 32, 128], N=[40, 20, 10], law="normal", coupling="prefix"),
    dict(m=33, n=50, p=20, c=[4, 16, 64, 256], N=[30, 20, 12, 6], law="uniform", coupling="stride"),
    dict(m=16, n=1000, p=24, c=[256, 1024, 4096], N=[12, 8, 4], law="normal", coupling="prefix"),
    dict(m=70, n=9, p=65, c=[3, 9, 27], N=[25, 15, 10], law="normal", coupling="stride"),
]


def _laws(mod, law):
    L = mod.Law
    return (L.normal(0.5, 1.0), L.normal(-0.3, 2.0)) if law == "normal" else (L.uniform(0.2, 1.0), L.uniform(1.0, 0.5))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_set_form_matches_oracle(orc, dev, prec, case):
    from paper_1904_00429_amd import matmul_estimate
    import paper_1904_00429_amd as pkg
    cs = CASES[case]
    flush(f"set form prec={prec} case={cs}")
    gA, gB = _laws(pkg, cs["law"])
    oA, oB = _laws(orc, cs["law"])
    est = matmul_estimate(cs["m"], cs["n"], cs["p"], gA, gB, cs["c"], n_samples=cs["N"], seed=21, prec=prec,
                          level_means=True, device=dev, coupling=cs["coupling"], set_form=True)
    ref = orc.estimate(cs["m"], cs["n"], cs["p"], oA, oB, cs["c"], n_samples=cs["N"], seed=21,
                       coupling=cs["coupling"], as_set=True)
    check_estimate(est, ref, prec, label=f"case {case}")
    if prec == "fp64":
        tup = matmul_estimate(cs["m"], cs["n"], cs["p"], gA, gB, cs["c"], n_samples=cs["N"], seed=21, prec=prec,
                              device=dev, coupling=cs["coupling"])
        r = rel_frob(est.Y.cpu().numpy(), tup.Y.cpu().numpy())
        flush(f"  set vs tuple form {r:.3g}")
        assert r <= 1e-12


def test_set_form_batched(orc, dev):
    from paper_1904_00429_amd import BatchedEstimate, BatchProblem, Law
    shapes = [(40, 37, 52), (64, 20, 64), (17, 100, 33)]
    c, N = [8, 32, 128], [30, 15, 8]
    flush("set form batched fp64")
    probs = [BatchProblem(m, n, p, Law.normal(0.4 + 0.3 * i, 1.0), Law.normal(0.4 + 0.3 * i, 1.0), 70 + i)
             for i, (m, n, p) in enumerate(shapes)]
    est = BatchedEstimate(probs, c, N, seed=9, prec="fp64", device=dev, set_form=True)
    V = est.run(level_var=True)
    torch.cuda.synchronize()

    def one(i):
        m, n, p = shapes[i]
        law = orc.Law.normal(0.4 + 0.3 * i, 1.0)
        return orc.estimate(m, n, p, law, law, c, n_samples=N, seed=9, problem=70 + i, as_set=True)

    with ThreadPoolExecutor(max_workers=min(len(shapes), os.cpu_count() or 4)) as ex:
        refs = list(ex.map(one, range(len(shapes))))
    for i, ref in enumerate(refs):
        r = rel_frob(est.Y[i].cpu().numpy(), ref.Y)
        flush(f"  product {i}: rel err {r:.3g}")
        assert r <= 1e-12
        np.testing.assert_allclose(V[:, i], ref.level_var, rtol=1e-10)
