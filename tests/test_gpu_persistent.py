"""The single-launch (persistent) form of the batched estimate: every pass of
every level in one kernel whose phases overlap the gather of one pass with the
sketch of the previous one.

It runs the same device arithmetic on the same passes as the launch-per-pass
form with one realisation group per pass (tuning target_blocks = 1), so the
two must agree bit for bit; and against the oracle product by product (FP32
1e-5; BF16 / FP8 against the oracle on the same rounded operands at 1e-4 of
||Y|| + RMSE_est, and against the exact oracle within their precision's
bounds).  tuning single_launch = 1 selects it; its workspace holds a second
gather buffer, which shows that a call planned it."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from gpu_helpers import check_estimate, flush, operand_law

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# products in whole tiles of 64 (m, p multiples of 64), of 128, and ragged
# ones (at tile 128 the single launch takes any shape, with Welford statistics)
SHAPES64 = [(64, 500, 64), (128, 1234, 192), (64, 4096, 320), (256, 777, 64), (192, 2000, 128), (128, 3000, 256)]
SHAPES128 = [(128, 700, 128), (256, 2100, 128), (128, 999, 384)]
RAGGED = [(100, 999, 37), (64, 500, 64), (200, 1500, 130), (37, 3000, 45)]
MUS = [0.1, 0.7, 1.3, 1.9, 0.4, 1.0]
C, N = [16, 32, 64], [60, 30, 15]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _laws(law, i):
    from paper_1904_00429_amd import Law
    mu = MUS[i % len(MUS)]
    return (Law.normal(mu, 1.0), Law.normal(mu, 1.0)) if law == "normal" else \
        (Law.uniform(mu, 1.5), Law.uniform(-mu, 0.5))


def _orc_laws(orc, law, i):
    mu = MUS[i % len(MUS)]
    return (orc.Law.normal(mu, 1.0), orc.Law.normal(mu, 1.0)) if law == "normal" else \
        (orc.Law.uniform(mu, 1.5), orc.Law.uniform(-mu, 0.5))


def _run(dev, shapes, law, prec, tile, value16, persistent, graph=False):
    from paper_1904_00429_amd import BatchedEstimate, BatchProblem
    probs = [BatchProblem(m, n, p, *_laws(law, i), 300 + i) for i, (m, n, p) in enumerate(shapes)]
    est = BatchedEstimate(probs, C, N, seed=23, prec=prec, device=dev, value16=value16,
                          tuning={"tile": tile, "target_blocks": 1, "single_launch": int(persistent)})
    if graph:
        est.capture()
        outs = []
        for _ in range(3):
            est.replay()
            torch.cuda.synchronize()
            outs.append([y.cpu().numpy().copy() for y in est.Y])
            # eager work of the program between replays
            torch.ones(1 << 20, device=dev).sum().item()
        est.release()
        return est, outs, None
    V = est.run(level_var=True)
    torch.cuda.synchronize()
    return est, [y.cpu().numpy() for y in est.Y], V


@pytest.mark.parametrize("prec,value16", [("fp32", False), ("bf16", True), ("fp8", True), ("fp8", False)])
@pytest.mark.parametrize("tile", [64, 128, "128-ragged"])
@pytest.mark.parametrize("law", ["normal", "uniform"])
def test_persistent_equals_launch_per_pass(dev, prec, value16, tile, law):
    shapes = {64: SHAPES64, 128: SHAPES128, "128-ragged": RAGGED}[tile]
    tile = 128 if tile == "128-ragged" else tile
    flush(f"persistent vs per-pass prec={prec} value16={value16} tile={tile} law={law}")
    est_p, Yp, Vp = _run(dev, shapes, law, prec, tile, value16, True)
    est_l, Yl, Vl = _run(dev, shapes, law, prec, tile, value16, False)
    # the persistent plan holds a second gather buffer: it was the one used
    assert est_p.ws_bytes > est_l.ws_bytes
    for i in range(len(shapes)):
        np.testing.assert_array_equal(Yp[i], Yl[i], err_msg=f"product {i}")
    np.testing.assert_array_equal(Vp, Vl)


class _Entry:
    def __init__(self, Y, V, ref):
        self.Y, self.level_var, self.level_means = torch.from_numpy(Y), list(V), None
        self.n_used, self.rmse_est = list(ref.n_used), float(np.sqrt(np.sum(np.asarray(V) / ref.n_used)))


@pytest.mark.parametrize("prec,value16", [("fp32", False), ("bf16", True), ("fp8", True)])
def test_persistent_matches_oracle(orc, dev, prec, value16):
    shapes = SHAPES64
    flush(f"persistent vs oracle prec={prec} value16={value16}")
    _, Y, V = _run(dev, shapes, "normal", prec, 64, value16, True)

    def one(i, rounded):
        m, n, p = shapes[i]
        la, lb = _orc_laws(orc, "normal", i)
        if value16:
            la, lb = la.with_value16(), lb.with_value16()
        if rounded:
            la, lb = operand_law(orc, la, prec, m, "A"), operand_law(orc, lb, prec, p, "B")
        return orc.estimate(m, n, p, la, lb, C, n_samples=N, seed=23, problem=300 + i)

    with ThreadPoolExecutor(max_workers=min(len(shapes), os.cpu_count() or 4)) as ex:
        refs = list(ex.map(lambda i: one(i, False), range(len(shapes))))
        refs_q = list(ex.map(lambda i: one(i, True), range(len(shapes)))) if prec in ("bf16", "fp8") else None
    for i, ref in enumerate(refs):
        check_estimate(_Entry(Y[i], V[:, i], ref), ref, prec, None if refs_q is None else refs_q[i], f"product {i}")


@pytest.mark.parametrize("prec,value16", [("fp32", False), ("fp8", True)])
def test_persistent_graph_replays(dev, prec, value16):
    """The persistent launch captured in a hipGraph: every replay (with eager
    work between them) gives the eager estimate."""
    flush(f"persistent graph prec={prec}")
    _, Y, _ = _run(dev, SHAPES64, "normal", prec, 64, value16, True)
    _, outs, _ = _run(dev, SHAPES64, "normal", prec, 64, value16, True, graph=True)
    for r, Yr in enumerate(outs):
        for i in range(len(SHAPES64)):
            np.testing.assert_array_equal(Yr[i], Y[i], err_msg=f"replay {r} product {i}")
