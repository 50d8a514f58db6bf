"""The oracle's set form of a realisation (the note after Alg. 1 in Sec. 3.1:
the index tuple (r_1, ..., r_{M^l}) taken as a set of distinct indices with
multiplicities, every distinct column read once).

Pinned two ways: the multiset mapping against collections.Counter on random
tuples and both couplings, and the whole estimate in the set form against the
tuple form of Alg. 1 (the plain definition: every draw's column read and
summed, fine and coarse sketches formed apart), which it must equal up to the
order of the sums, on workloads where repeats are the rule (c_l up to several
times n)."""
import collections

import numpy as np
import pytest


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("M", [0, 2, 3])
def test_multiset_counts_brute_force(orc, seed, M):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 13))
    c_c = int(rng.integers(1, 20))
    c_f = c_c * M if M else int(rng.integers(c_c, 3 * c_c + 1))
    r = rng.integers(0, n, size=c_f)
    j, mf, mc = orc.multiset(r, c_c, M)
    coarse = [M * (i + 1) - 1 for i in range(c_c)] if M else list(range(c_c))
    cf = collections.Counter(int(x) for x in r)
    cc = collections.Counter(int(r[t]) for t in coarse)
    assert list(j) == sorted(cf)
    assert list(mf) == [cf[int(x)] for x in j]
    assert list(mc) == [cc.get(int(x), 0) for x in j]
    assert mf.sum() == c_f and mc.sum() == c_c


def _close(a, b, rtol=1e-12):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    scale = max(float(np.max(np.abs(b))), 1e-300)
    assert float(np.max(np.abs(a - b))) <= rtol * scale, (float(np.max(np.abs(a - b))), scale)


@pytest.mark.parametrize("case", [
    dict(m=3, n=5, p=4, c=[2, 8, 32], N=[30, 20, 10], law=("normal", 0.5, 1.0)),
    dict(m=3, n=5, p=4, c=[2, 8, 32], N=[30, 20, 10], law=("uniform", -0.2, 1.0), coupling="stride"),
    dict(m=2, n=7, p=3, c=[3, 9, 27, 81], N=[40, 20, 10, 6], law=("normal", 1.0, 0.5), coupling="stride"),
    dict(m=4, n=9, p=2, c=[4, 16, 64], N=[20, 10, 5], law=("normal", 0.0, 1.0), func=("abs_step", 2.0)),
    dict(m=3, n=6, p=3, c=[2, 8, 32], N=[20, 10, 5], law=("normal", 0.3, 1.0), weights=True),
    dict(m=1, n=6, p=1, c=[4, 16, 64], N=[50, 30, 20], law=("uniform", 0.5, 1.0)),
    dict(m=5, n=40, p=5, c=[8, 32, 128], N=[16, 8, 4], law=("normal", 0.5, 1.0)),
])
def test_set_form_equals_tuple_form(orc, case):
    kind, loc, scale = case["law"]
    A = getattr(orc.Law, kind)(loc, scale)
    B = getattr(orc.Law, kind)(-0.5 * loc, 2.0 * scale)
    kw = dict(n_samples=case["N"], seed=11, problem=3, coupling=case.get("coupling", "prefix"))
    if "func" in case:
        kw["func"] = getattr(orc.Func, case["func"][0])(case["func"][1])
    if case.get("weights"):
        kw["weights"] = orc.Weights(np.random.default_rng(5).integers(1, 6, size=case["n"]))
    m, n, p, c = case["m"], case["n"], case["p"], case["c"]
    tup = orc.estimate(m, n, p, A, B, c, **kw)
    st = orc.estimate(m, n, p, A, B, c, as_set=True, **kw)
    _close(st.Y, tup.Y)
    for l in range(len(c)):
        _close(st.level_means[l], tup.level_means[l])
        _close(st.level_var[l], tup.level_var[l], rtol=1e-10)
    # the top level repeats indices: c_L exceeds n, or is close to it
    r = orc.draw_indices(11, 3, len(c) - 1, 0, c[-1], n)
    assert len(np.unique(r)) < c[-1]
