"""GPU parity of the building blocks against the oracle: Philox words and
index draws bit-exact, sampled columns within the rounding of their precision."""
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


@pytest.mark.parametrize("seed", [0, 12345, 2**64 - 3])
def test_philox_bit_exact(orc, dev, seed):
    from paper_1904_00429_amd import philox
    flush(f"philox seed={seed}")
    rng = np.random.default_rng(seed % 1000)
    ctr = rng.integers(0, 2**32, size=(20000, 4), dtype=np.uint64).astype(np.uint32)
    got = philox(torch.from_numpy(ctr.view(np.int32)).to(dev), seed).cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(got, orc.philox(ctr, seed))


@pytest.mark.parametrize("n,c,lev,k0,S", [(1, 5, 0, 0, 3), (7, 1, 3, 10, 50), (4099, 64, 1, 7, 40),
                                          (2**20, 1000, 8, 123456, 6), (2**31 + 11, 33, 0xFF, 0, 9),
                                          (65536, 4096, 7, 2**32 - 20, 5)])
def test_indices_bit_exact(orc, dev, n, c, lev, k0, S):
    from paper_1904_00429_amd import sample_indices
    flush(f"indices n={n} c={c} lev={lev} k0={k0} S={S}")
    seed, problem = 99, 17
    got = sample_indices(seed, problem, lev, k0, S, c, n, device=dev).cpu().numpy().astype(np.int64)
    for s in range(S):
        np.testing.assert_array_equal(got[s], orc.draw_indices(seed, problem, lev, k0 + s, c, n))


@pytest.mark.parametrize("prec,rtol,atol", [("fp64", 1e-13, 1e-13), ("fp32", 4e-6, 4e-6), ("bf16", 8e-3, 1e-6)])
@pytest.mark.parametrize("law", ["normal", "uniform", "reparam", "mixed"])
def test_gather_columns(orc, dev, prec, rtol, atol, law):
    from paper_1904_00429_amd import gather_columns
    flush(f"gather prec={prec} law={law}")
    m, n, p, c, S, k0, lev = 5, 300, 3, 24, 4, 9, 2
    rng = np.random.default_rng(1)
    if law == "reparam":
        ma, sa = rng.standard_normal((n, m)), rng.uniform(0.1, 1, (n, m))
        mb, sb = rng.standard_normal((n, p)), rng.uniform(0.1, 1, (n, p))
        oA, gA = laws(orc, ("reparam",), dev, ma, sa)
        oB, gB = laws(orc, ("reparam",), dev, mb, sb)
    elif law == "mixed":
        oA, gA = laws(orc, ("normal", 0.5, 2.0), dev)
        oB, gB = laws(orc, ("uniform", -1.0, 3.0), dev)
    else:
        oA, gA = laws(orc, (law, 0.5, 2.0), dev)
        oB, gB = laws(orc, (law, -1.0, 3.0), dev)
    AS, BS = gather_columns(m, n, p, gA, gB, 7, 0, lev, k0, S, c, prec=prec, device=dev)
    AS, BS = AS.cpu().numpy(), BS.cpu().numpy()
    for s in range(S):
        r = orc.draw_indices(7, 0, lev, k0 + s, c, n)
        for t in range(c):
            a, b = orc.column(7, 0, lev, k0 + s, r[t], m, p, oA, oB)
            np.testing.assert_allclose(AS[s, t], a, rtol=rtol, atol=atol)
            np.testing.assert_allclose(BS[s, t], b, rtol=rtol, atol=atol)


def test_fp64_normals_to_a_few_ulp(orc, dev):
    """The FP64 Box-Muller pairs (series for ln, cos and sin after exact range
    reductions of the grid uniforms) against the oracle's libm on about 3e5
    values.  The oracle rounds its angle 2 pi v to FP64 before the cosine (up
    to 2^-51 absolute for angles in [4, 8)), so its z carries up to
    rho 2^-51 <= 5.8 2^-51 (rho = sqrt(-2 ln u), u >= 2^-24) of its own:
    bound 16 units in the last place of max(1, |z|)."""
    from paper_1904_00429_amd import gather_columns
    flush("gather fp64 normals, many values")
    m, n, p, c, S = 300, 100003, 300, 64, 8
    oA, gA = laws(orc, ("normal", 0.0, 1.0), dev)
    AS, BS = gather_columns(m, n, p, gA, gA, 11, 0, 3, 0, S, c, prec="fp64", device=dev)
    AS, BS = AS.cpu().numpy(), BS.cpu().numpy()
    worst = 0.0
    for s in range(S):
        r = orc.draw_indices(11, 0, 3, s, c, n)
        for t in range(c):
            a, b = orc.column(11, 0, 3, s, r[t], m, p, oA, oA)
            for got, ref in ((AS[s, t], a), (BS[s, t], b)):
                worst = max(worst, float(np.max(np.abs(got - ref) / np.maximum(1.0, np.abs(ref)))))
    flush(f"  max |dz| / max(1, |z|) = {worst:.3g} = {worst / 2.0 ** -52:.2f} ulp")
    assert worst <= 16 * 2.0 ** -52
