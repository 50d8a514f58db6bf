"""GPU parity of the adjoint (mlmc_matmul_adjoint_reparam) and of the autograd
Function built on it, against the FP64 torch-CPU gradient reference on the
same seeds; finite differences of the GPU's own FP64 forward; and the
seed-average against the closed-form gradient of a linear functional.

Tolerance: FP32 adjoint, 1e-5 relative Frobenius per gradient array.  BF16
adjoint (values and G rounded to BF16, FP32 accumulation): 1e-2.  Each
gradient entry is a sum of kappa_t (G b_t)_i terms; rounding both operands of
a dot product by at most 2^-9 relative gives it a relative error of about
2^-9 sqrt(2/3) (0.16%) for these random operands, and summing independent
terms keeps that ratio, so 1e-2 leaves a margin of about 5."""
import math

import numpy as np
import pytest

from gpu_helpers import flush, rel_frob

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _params(seed, n, m, p):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((n, m)).astype(np.float32), rng.uniform(0.1, 1, (n, m)).astype(np.float32),
            rng.standard_normal((n, p)).astype(np.float32), rng.uniform(0.1, 1, (n, p)).astype(np.float32)]


CASES = [
    (5, 40, 3, [2, 4, 8], [40, 20, 10]),
    (70, 300, 33, [16, 32, 64], [30, 12, 5]),
    (64, 500, 130, [5, 10, 20, 40], [20, 10, 6, 3]),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_adjoint_matches_reference(orc, dev, case):
    from oracle import grad as og
    from paper_1904_00429_amd import matmul_adjoint_reparam
    m, n, p, c, N = CASES[case]
    flush(f"adjoint case={case} m={m} n={n} p={p} c={c} N={N}")
    params = _params(case, n, m, p)
    G = np.random.default_rng(50 + case).standard_normal((m, p))
    _, ref = og.reparam_gradients(*params, c, N, G, seed=7)
    dp = [torch.from_numpy(x).to(dev) for x in params]
    got = matmul_adjoint_reparam(*dp, c, N, torch.from_numpy(G), seed=7)
    for name, g, r in zip(("dMA", "dSA", "dMB", "dSB"), got, ref):
        err = rel_frob(g.cpu().numpy(), r)
        flush(f"  {name} rel err {err:.3g}")
        assert err <= 1e-5, (name, err)


def test_autograd_loss_gradient(orc, dev):
    from oracle import grad as og
    from paper_1904_00429_amd import mlmc_matmul
    m, n, p, c, N = 24, 400, 17, [8, 16, 32], [30, 15, 8]
    flush("autograd end to end")
    params = _params(11, n, m, p)
    T = np.random.default_rng(12).standard_normal((m, p))
    leaves = [torch.from_numpy(x).to(dev).requires_grad_(True) for x in params]
    Y = mlmc_matmul(*leaves, c, N, seed=3, prec="fp32")
    loss = ((Y - torch.from_numpy(T).to(dev)) ** 2).sum()
    loss.backward()
    # reference: gradient of the same loss, G = 2 (Y - T) at the oracle's Y
    Y_ref = og.reparam_estimate(*[torch.from_numpy(x.astype(np.float64)) for x in params], c, N, seed=3).numpy()
    assert rel_frob(Y.detach().cpu().numpy(), Y_ref) <= 1e-5
    _, ref = og.reparam_gradients(*params, c, N, 2 * (Y_ref - T), seed=3)
    for g, r in zip(leaves, ref):
        assert rel_frob(g.grad.cpu().numpy(), r) <= 1e-5


def test_adjoint_full_shape_few_realisations(orc, dev):
    """The differentiation workload's shapes (512 x 32768 x 512, c_l = 32 * 2^l,
    l = 0..6) with a handful of realisations per level, against the reference."""
    from oracle import grad as og
    from paper_1904_00429_amd import matmul_adjoint_reparam
    m, n, p = 512, 32768, 512
    c = [32 * 2 ** l for l in range(7)]
    N = [3, 2, 2, 1, 1, 1, 1]
    flush("adjoint full shape")
    params = _params(21, n, m, p)
    G = np.random.default_rng(22).standard_normal((m, p))
    _, ref = og.reparam_gradients(*params, c, N, G, seed=5)
    dp = [torch.from_numpy(x).to(dev) for x in params]
    got = matmul_adjoint_reparam(*dp, c, N, torch.from_numpy(G), seed=5)
    for g, r in zip(got, ref):
        assert rel_frob(g.cpu().numpy(), r) <= 1e-5


def test_adjoint_matches_finite_differences_of_gpu_forward(dev):
    """Y is affine in each single mean or scale entry, so a central difference of
    the GPU's FP64 forward is exact up to rounding."""
    from paper_1904_00429_amd import Law, matmul_adjoint_reparam, matmul_estimate
    m, n, p, c, N = 9, 50, 7, [2, 4, 8], [40, 20, 10]
    params = _params(31, n, m, p)
    G = np.random.default_rng(32).standard_normal((m, p))
    dp = [torch.from_numpy(x).to(dev) for x in params]
    got = [g.cpu().numpy() for g in matmul_adjoint_reparam(*dp, c, N, torch.from_numpy(G), seed=9)]

    def L(ps):
        t = [torch.from_numpy(x).to(dev) for x in ps]
        est = matmul_estimate(m, n, p, Law.reparam(t[0], t[1]), Law.reparam(t[2], t[3]), c, n_samples=N,
                              seed=9, prec="fp64", device=dev)
        return float((est.Y.cpu().numpy() * G).sum())

    rng = np.random.default_rng(33)
    checked = 0
    for which in range(4):
        # entries whose row was drawn carry a gradient; pick those
        rows = np.nonzero(np.abs(got[which]).sum(axis=1))[0]
        for _ in range(3):
            j = int(rng.choice(rows))
            i = int(rng.integers(0, params[which].shape[1]))
            plus = [x.copy() for x in params]
            minus = [x.copy() for x in params]
            plus[which][j, i] = np.float32(params[which][j, i] + 0.25)
            minus[which][j, i] = np.float32(params[which][j, i] - 0.25)
            step = float(plus[which][j, i]) - float(minus[which][j, i])
            fd = (L(plus) - L(minus)) / step
            assert abs(fd - got[which][j, i]) <= 1e-5 * (1 + abs(fd)), (which, j, i, fd, got[which][j, i])
            checked += 1
    assert checked == 12


def test_adjoint_seed_average_matches_closed_form(dev):
    """E over seeds of grad <G0, Y> equals grad <G0, M_A M_B>:
    (M_B G0^T, 0, M_A G0, 0) in the row-j layouts."""
    from paper_1904_00429_amd import matmul_adjoint_reparam
    m, n, p, c, N = 6, 16, 5, [2, 4], [8, 4]
    params = _params(41, n, m, p)
    G0 = np.random.default_rng(42).standard_normal((m, p))
    dp = [torch.from_numpy(x).to(dev) for x in params]
    seeds = 400
    acc = [np.zeros((seeds,) + x.shape) for x in params]
    for s in range(seeds):
        g = matmul_adjoint_reparam(*dp, c, N, torch.from_numpy(G0), seed=10_000 + s)
        for i in range(4):
            acc[i][s] = g[i].cpu().numpy()
    MA, SA, MB, SB = [x.astype(np.float64) for x in params]
    expected = [MB @ G0.T, np.zeros_like(SA), MA @ G0, np.zeros_like(SB)]
    for i in range(4):
        mean = acc[i].mean(axis=0)
        se = acc[i].std(axis=0, ddof=1) / math.sqrt(seeds) + 1e-9
        z = np.abs(mean - expected[i]) / se
        assert z.max() < 5.5, (i, z.max())


@pytest.mark.parametrize("case", range(len(CASES)))
def test_adjoint_bf16_matches_reference(orc, dev, case):
    from oracle import grad as og
    from paper_1904_00429_amd import matmul_adjoint_reparam
    m, n, p, c, N = CASES[case]
    flush(f"adjoint bf16 case={case} m={m} n={n} p={p} c={c} N={N}")
    params = _params(case, n, m, p)
    G = np.random.default_rng(50 + case).standard_normal((m, p))
    _, ref = og.reparam_gradients(*params, c, N, G, seed=7)
    dp = [torch.from_numpy(x).to(dev) for x in params]
    got = matmul_adjoint_reparam(*dp, c, N, torch.from_numpy(G), seed=7, prec="bf16")
    for name, g, r in zip(("dMA", "dSA", "dMB", "dSB"), got, ref):
        err = rel_frob(g.cpu().numpy(), r)
        flush(f"  {name} rel err {err:.3g}")
        assert err <= 1e-2, (name, err)


def test_adjoint_bf16_full_shape_few_realisations(orc, dev):
    from oracle import grad as og
    from paper_1904_00429_amd import matmul_adjoint_reparam
    m, n, p = 512, 32768, 512
    c = [32 * 2 ** l for l in range(7)]
    N = [3, 2, 2, 1, 1, 1, 1]
    flush("adjoint bf16 full shape")
    params = _params(21, n, m, p)
    G = np.random.default_rng(22).standard_normal((m, p))
    _, ref = og.reparam_gradients(*params, c, N, G, seed=5)
    dp = [torch.from_numpy(x).to(dev) for x in params]
    got = matmul_adjoint_reparam(*dp, c, N, torch.from_numpy(G), seed=5, prec="bf16")
    for name, g, r in zip(("dMA", "dSA", "dMB", "dSB"), got, ref):
        err = rel_frob(g.cpu().numpy(), r)
        flush(f"  {name} rel err {err:.3g}")
        assert err <= 1e-2, (name, err)


def test_autograd_bf16_forward_and_adjoint(orc, dev):
    # BF16 forward and BF16 adjoint; the reference gradient is taken at the
    # GPU's own estimate (G = 2 (Y - T)) so that only the adjoint's rounding
    # is measured against the 1e-2 bound
    from oracle import grad as og
    from paper_1904_00429_amd import mlmc_matmul
    m, n, p, c, N = 24, 400, 17, [8, 16, 32], [30, 15, 8]
    flush("autograd bf16 end to end")
    params = _params(11, n, m, p)
    T = np.random.default_rng(12).standard_normal((m, p))
    leaves = [torch.from_numpy(x).to(dev).requires_grad_(True) for x in params]
    Y = mlmc_matmul(*leaves, c, N, seed=3, prec="bf16")
    loss = ((Y - torch.from_numpy(T).to(dev)) ** 2).sum()
    loss.backward()
    Yg = Y.detach().cpu().numpy()
    Y_ref = og.reparam_estimate(*[torch.from_numpy(x.astype(np.float64)) for x in params], c, N, seed=3).numpy()
    assert rel_frob(Yg, Y_ref) <= 1e-2
    _, ref = og.reparam_gradients(*params, c, N, 2 * (Yg - T), seed=3)
    for g, r in zip(leaves, ref):
        assert rel_frob(g.grad.cpu().numpy(), r) <= 1e-2


@pytest.mark.parametrize("prec, tol", [("fp32", 1e-5), ("bf16", 1e-2)])
def test_adjoint_full_workload_sampled_columns(orc, dev, prec, tol):
    """The differentiation workload as benchmarked: 512 x 32768 x 512,
    c_l = 32 * 2^l (l = 0..6), N_l = 4096 * 2^-l (about 28 draws hit each
    column, so every column's sum runs over many draws), checked
    at eight columns j against the entry-restricted gradient reference."""
    from oracle import grad as og
    from paper_1904_00429_amd import matmul_adjoint_reparam, workloads
    wl = workloads.DIFF_512x32768x512
    m, n, p = wl.m, wl.n, wl.p
    flush(f"adjoint full workload {prec}: N={wl.n_samples}")
    params = _params(61, n, m, p)
    G = np.random.default_rng(62).standard_normal((m, p))
    dp = [torch.from_numpy(x).to(dev) for x in params]
    got = [g.cpu().numpy() for g in matmul_adjoint_reparam(*dp, wl.c, wl.n_samples, torch.from_numpy(G), seed=8,
                                                           prec=prec)]
    cols = sorted(np.random.default_rng(63).choice(n, 8, replace=False).tolist())
    ref = og.reparam_gradients_at(*params, wl.c, wl.n_samples, G, cols, seed=8)
    for name, g, r in zip(("dMA", "dSA", "dMB", "dSB"), got, ref):
        assert np.abs(r).max() > 0, name            # the sampled columns were drawn
        err = rel_frob(g[cols], r)
        flush(f"  {name} rel err at columns {cols}: {err:.3g}")
        assert err <= tol, (name, err)


# Few columns, many draws: each column's draws run through many 64-draw tiles
# (carried partial sums, the fix-up chain), and n = 1 (no sort digit at all,
# one segment per pass) and n above 2^16 (three 8-bit digits).
HEAVY = [
    (20, 3, 30, [64, 256, 1024], [12, 6, 3]),
    (33, 1, 17, [100, 400], [10, 5]),
    (16, 70000, 24, [256, 1024], [6, 3]),
    (130, 7, 70, [32, 96, 288], [20, 8, 4]),
]


@pytest.mark.parametrize("prec, tol", [("fp32", 1e-5), ("bf16", 1e-2)])
@pytest.mark.parametrize("case", range(len(HEAVY)))
def test_adjoint_repeated_columns(orc, dev, case, prec, tol):
    from oracle import grad as og
    from paper_1904_00429_amd import matmul_adjoint_reparam
    m, n, p, c, N = HEAVY[case]
    flush(f"adjoint repeated columns {prec} m={m} n={n} p={p} c={c} N={N}")
    params = _params(80 + case, n, m, p)
    G = np.random.default_rng(90 + case).standard_normal((m, p))
    dp = [torch.from_numpy(x).to(dev) for x in params]
    got = [g.cpu().numpy() for g in matmul_adjoint_reparam(*dp, c, N, torch.from_numpy(G), seed=4, prec=prec)]
    if n > 1000:
        # columns the first top-level realisation drew (the oracle's own draws),
        # and two chosen at random
        hit = [int(j) for j in np.unique(orc.draw_indices(4, 0, len(c) - 1, 0, c[-1], n))[:4]]
        cols = sorted(set(hit) | set(np.random.default_rng(95).choice(n, 2, replace=False).tolist()))
        ref = og.reparam_gradients_at(*params, c, N, G, cols, seed=4)
        got = [g[cols] for g in got]
    else:
        _, ref = og.reparam_gradients(*params, c, N, G, seed=4)
    for name, g, r in zip(("dMA", "dSA", "dMB", "dSB"), got, ref):
        err = rel_frob(g, r)
        flush(f"  {name} rel err {err:.3g}")
        assert err <= tol, (name, err)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_adjoint_is_deterministic(dev, prec):
    """The gradients are formed without atomics (draws sorted by column, each
    column summed in draw order by one owner), so two calls give the same
    bits, at the differentiation workload's full size."""
    from paper_1904_00429_amd import matmul_adjoint_reparam, workloads
    wl = workloads.DIFF_512x32768x512
    flush(f"adjoint determinism {prec}")
    params = _params(71, wl.n, wl.m, wl.p)
    G = torch.from_numpy(np.random.default_rng(72).standard_normal((wl.m, wl.p)))
    dp = [torch.from_numpy(x).to(dev) for x in params]
    a = matmul_adjoint_reparam(*dp, wl.c, wl.n_samples, G, seed=3, prec=prec)
    b = matmul_adjoint_reparam(*dp, wl.c, wl.n_samples, G, seed=3, prec=prec)
    for name, x, y in zip(("dMA", "dSA", "dMB", "dSB"), a, b):
        assert torch.equal(x, y), name
        assert bool(torch.isfinite(x).all()), name


@pytest.mark.parametrize("prec, tol", [("fp32", 1e-5), ("bf16", 1e-2)])
def test_adjoint_small_workspace_many_passes(orc, dev, prec, tol):
    """A workspace far below the one-pass size: the draws of all levels go in
    passes of a few hundred, which cut through levels, realisations and
    column segments; the gradients stay within the tolerance of the
    reference, and agree with the one-pass call up to the summation order."""
    from oracle import grad as og
    from paper_1904_00429_amd import matmul_adjoint_reparam
    m, n, p, c, N = 20, 5, 30, [8, 32, 128], [30, 12, 5]
    flush(f"adjoint many passes {prec}")
    params = _params(77, n, m, p)
    G = np.random.default_rng(78).standard_normal((m, p))
    dp = [torch.from_numpy(x).to(dev) for x in params]
    one = [g.cpu().numpy() for g in matmul_adjoint_reparam(*dp, c, N, torch.from_numpy(G), seed=6, prec=prec)]
    # about 300 draws per pass (G's two operand buffers, then 64-draw steps)
    small = [g.cpu().numpy() for g in matmul_adjoint_reparam(*dp, c, N, torch.from_numpy(G), seed=6, prec=prec,
                                                             max_workspace_bytes=400 << 10)]
    _, ref = og.reparam_gradients(*params, c, N, G, seed=6)
    for name, a, b, r in zip(("dMA", "dSA", "dMB", "dSB"), one, small, ref):
        flush(f"  {name} one pass {rel_frob(a, r):.3g}, many passes {rel_frob(b, r):.3g}")
        assert rel_frob(b, r) <= tol, name
        assert rel_frob(b, a) <= (1e-6 if prec == "fp32" else 1e-3), name
