"""The C ABI library loads, exports every declared symbol, and rejects bad
arguments before touching the device (CPU only: no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_1904_00429_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1904_00429_amd import build
        build.build()
    return _lib.lib()


def declared_functions():
    text = open(os.path.join(ROOT, "include", "mlmc.h")).read()
    return sorted(set(re.findall(r"\b(mlmc_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 9
    for name in names:
        assert hasattr(L, name), name
    from paper_1904_00429_amd import _lib
    assert sorted(_lib.EXPORTED) == names


def test_status_strings(L):
    for code, name in [(0, b"MLMC_OK"), (1, b"MLMC_EINVAL"), (2, b"MLMC_EDEVICE"),
                       (3, b"MLMC_EBUDGET"), (4, b"MLMC_EWORKSPACE")]:
        assert L.mlmc_status_string(code) == name


def _levels(c, n_samples=None, eps=0.0, pilot=0, prec=0):
    from paper_1904_00429_amd._lib import Levels
    ca = (ctypes.c_int64 * len(c))(*c)
    lv = Levels()
    lv.num_levels = len(c)
    lv.c = ctypes.cast(ca, ctypes.POINTER(ctypes.c_int64))
    keep = [ca]
    if n_samples is not None:
        na = (ctypes.c_int64 * len(n_samples))(*n_samples)
        lv.n_samples = ctypes.cast(na, ctypes.POINTER(ctypes.c_int64))
        keep.append(na)
    lv.rmse_target = eps
    lv.pilot_samples = pilot
    lv.prec = prec
    return lv, keep


def _dist(law=0, loc=0.0, scale=1.0):
    from paper_1904_00429_amd._lib import Dist
    d = Dist()
    d.law, d.loc, d.scale = law, loc, scale
    return d


@pytest.mark.parametrize("case", [
    dict(m=0), dict(p=0), dict(n=0), dict(n=2**32), dict(c=[]), dict(c=[4, 6]), dict(c=[4, 4]),
    dict(c=[2, 2**31]), dict(c=[2**32 - 1]), dict(c=[2**27, 2**28]),
    dict(c=[0, 4]), dict(N=[1, 0]), dict(N=None), dict(eps=1.0, pilot=1, N=None),
    dict(eps=1.0, pilot=10), dict(prec=7), dict(lawA=2), dict(out=False),
])
def test_matmul_rejects_invalid(L, case):
    m, n, p = case.get("m", 4), case.get("n", 16), case.get("p", 3)
    c = case.get("c", [2, 4])
    N = case.get("N", [4, 4]) if "N" in case else [4, 4]
    lv, keep = _levels(c if c else [1], N, case.get("eps", 0.0), case.get("pilot", 0), case.get("prec", 0))
    if not c:
        lv.num_levels = 0
    A = _dist(case.get("lawA", 0))
    B = _dist()
    st = L.mlmc_matmul_estimate(m, n, p, ctypes.byref(A), ctypes.byref(B), ctypes.byref(lv),
                                None if case.get("out", True) is False else 8, None, 16, 1 << 40,
                                None, None)
    assert st == 1, L.mlmc_last_error()
    assert L.mlmc_last_error()


def test_workspace_too_small(L):
    lv, keep = _levels([2, 4], [4, 4])
    A, B = _dist(), _dist()
    need = L.mlmc_matmul_workspace_size(4, 16, 3, ctypes.byref(lv))
    assert need > 0
    st = L.mlmc_matmul_estimate(4, 16, 3, ctypes.byref(A), ctypes.byref(B), ctypes.byref(lv), 8, None,
                                16, need - 1, None, None)
    assert st == 4
    st = L.mlmc_inner_product_estimate(16, ctypes.byref(A), ctypes.byref(B), ctypes.byref(lv), 8, None,
                                       None, 0, None, None)
    assert st == 4


def test_inner_rejects_bf16(L):
    lv, keep = _levels([2, 4], [4, 4], prec=2)
    A, B = _dist(), _dist()
    st = L.mlmc_inner_product_estimate(16, ctypes.byref(A), ctypes.byref(B), ctypes.byref(lv), 8, None,
                                       16, 1 << 30, None, None)
    assert st == 1


@pytest.mark.parametrize("c", [[2**31], [3, 3 * 2**30], [2**32 - 1]])
def test_inner_rejects_ladders_from_2pow31(L, c):
    # the kernels count draws, pairs and quads of a realisation in 32 bits
    lv, keep = _levels(c, [4] * len(c), prec=0)
    A, B = _dist(), _dist()
    st = L.mlmc_inner_product_estimate(16, ctypes.byref(A), ctypes.byref(B), ctypes.byref(lv), 8, None,
                                       16, 1 << 30, None, None)
    assert st == 1
    assert b"2^31" in L.mlmc_last_error()


def test_workspace_size_scales_with_shape(L):
    lv, keep = _levels([32, 64, 128], [10, 10, 10], prec=1)
    small = L.mlmc_matmul_workspace_size(64, 1000, 64, ctypes.byref(lv))
    big = L.mlmc_matmul_workspace_size(1024, 1000, 1024, ctypes.byref(lv))
    assert 0 < small < big


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1904_00429_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        _lib.lib()


@pytest.mark.parametrize("func, params", [(3, (0.0, 0.0)), (-1, (0.0, 0.0)), (1, (float("inf"), 0.0)),
                                          (2, (0.4, 0.0)), (2, (0.4, -1.0)), (2, (float("nan"), 0.01))])
def test_rejects_bad_target_function(L, func, params):
    lv, keep = _levels([2, 4], [4, 4])
    lv.func = func
    lv.func_param[0], lv.func_param[1] = params
    A, B = _dist(), _dist()
    st = L.mlmc_matmul_estimate(4, 16, 3, ctypes.byref(A), ctypes.byref(B), ctypes.byref(lv), 8, None,
                                16, 1 << 40, None, None)
    assert st == 1, L.mlmc_last_error()
    st = L.mlmc_inner_product_estimate(16, ctypes.byref(A), ctypes.byref(B), ctypes.byref(lv), 8, None,
                                       16, 1 << 40, None, None)
    assert st == 1
    assert L.mlmc_matmul_workspace_size(4, 16, 3, ctypes.byref(lv)) == 0


def test_adjoint_rejects_target_function(L):
    lv, keep = _levels([2, 4], [4, 4], prec=1)
    lv.func = 1
    lv.func_param[0] = 2.0
    A = _dist(2)
    B = _dist(2)
    A.mean = A.stdev = B.mean = B.stdev = 16
    A.ld, B.ld = 4, 3
    st = L.mlmc_matmul_adjoint_reparam(4, 16, 3, ctypes.byref(A), ctypes.byref(B), ctypes.byref(lv), 16, 16, 16,
                                       16, 16, 16, 1 << 40, None)
    assert st == 1
    assert b"identity" in L.mlmc_last_error()


def test_adaptive_levels_need_target_mode(L):
    lv, keep = _levels([2, 4, 8], [4, 4, 4])
    lv.flags = 4
    A, B = _dist(), _dist()
    st = L.mlmc_matmul_estimate(4, 16, 3, ctypes.byref(A), ctypes.byref(B), ctypes.byref(lv), 8, None,
                                16, 1 << 40, None, None)
    assert st == 1 and b"adaptive" in L.mlmc_last_error()
    st = L.mlmc_inner_product_estimate(16, ctypes.byref(A), ctypes.byref(B), ctypes.byref(lv), 8, None,
                                       16, 1 << 40, None, None)
    assert st == 1


def test_matrix_ladder_cap_in_workspace_size(L):
    # c_L < 2^28 for matrix products (gather grid and 32-bit position counts),
    # checked without a device call through the workspace query
    for c, ok in (([2**26, 2**27], True), ([2**27, 2**28], False), ([3, 2**29 * 3], False)):
        lv, keep = _levels(c, [4, 4], prec=1)
        assert (L.mlmc_matmul_workspace_size(4, 16, 3, ctypes.byref(lv)) > 0) == ok, c
        assert (L.mlmc_matmul_adjoint_workspace_size(4, 16, 3, ctypes.byref(lv)) > 0) == ok, c


def test_adjoint_rejects_fp64_and_fp8(L):
    for prec in (0, 3):
        lv, keep = _levels([2, 4], [4, 4], prec=prec)
        A = _dist(2)
        B = _dist(2)
        A.mean = A.stdev = B.mean = B.stdev = 16
        A.ld, B.ld = 4, 3
        st = L.mlmc_matmul_adjoint_reparam(4, 16, 3, ctypes.byref(A), ctypes.byref(B), ctypes.byref(lv), 16, 16,
                                           16, 16, 16, 16, 1 << 40, None)
        assert st == 1


def test_weighted_draws_rejected_with_fp8_and_in_batches(L):
    from paper_1904_00429_amd._lib import Problem
    lv, keep = _levels([2, 4], [4, 4], prec=3)
    lv.index_weights = 16
    A, B = _dist(), _dist()
    st = L.mlmc_matmul_estimate(4, 16, 3, ctypes.byref(A), ctypes.byref(B), ctypes.byref(lv), 8, None,
                                16, 1 << 40, None, None)
    assert st == 1 and b"FP8" in L.mlmc_last_error()
    lv.prec = 1
    probs = (Problem * 1)()
    probs[0].m, probs[0].n, probs[0].p = 4, 16, 3
    probs[0].A, probs[0].B = _dist(), _dist()
    probs[0].out = 8
    st = L.mlmc_matmul_estimate_batched(1, probs, ctypes.byref(lv), None, 16, 1 << 40, None, None)
    assert st == 1 and b"uniformly" in L.mlmc_last_error()


@pytest.mark.parametrize("lawA, lawB, prec, locB, scaleB, words", [
    (3, 0, 0, 0.0, 1.0, b"pair only"),          # an experiment law with a classic one
    (0, 4, 1, 10.0, 0.05, b"pair only"),
    (5, 6, 3, 2.0, 0.2, b"FP8"),                # not with FP8 operands
    (3, 4, 0, 0.0, 0.05, b"Poisson rate"),      # rate must be positive
    (3, 4, 0, 600.0, 0.05, b"Poisson rate"),
    (5, 6, 0, 2.0, 1.5, b"Bernoulli rate"),
    (7, 6, 0, 2.0, 0.2, b"unknown law"),
])
def test_experiment_laws_validated(L, lawA, lawB, prec, locB, scaleB, words):
    lv, keep = _levels([2, 4], [4, 4], prec=prec)
    A, B = _dist(lawA, 0.4, 0.02), _dist(lawB, locB, scaleB)
    st = L.mlmc_matmul_estimate(4, 16, 3, ctypes.byref(A), ctypes.byref(B), ctypes.byref(lv), 8, None,
                                16, 1 << 40, None, None)
    assert st == 1 and words in L.mlmc_last_error(), L.mlmc_last_error()


def test_experiment_laws_rejected_by_xi_star_and_mixed_batches(L):
    from paper_1904_00429_amd._lib import Problem
    A, B = _dist(5, 0.5, 1e-4), _dist(6, 2.0, 0.2)
    st = L.mlmc_optimal_index_weights(4, 16, 3, ctypes.byref(A), ctypes.byref(B), 16, 16, None)
    assert st == 1 and b"xi**" in L.mlmc_last_error()
    lv, keep = _levels([2, 4], [4, 4], prec=1)
    probs = (Problem * 2)()
    for i in range(2):
        probs[i].m, probs[i].n, probs[i].p = 4, 16, 3
        probs[i].out = 8
        probs[i].problem = i
    probs[0].A, probs[0].B = A, B
    probs[1].A, probs[1].B = _dist(), _dist()
    st = L.mlmc_matmul_estimate_batched(2, probs, ctypes.byref(lv), None, 16, 1 << 40, None, None)
    assert st == 1 and b"every product or none" in L.mlmc_last_error()


def test_index_word32_validated(L):
    from paper_1904_00429_amd._lib import Problem
    lv, keep = _levels([2, 4], [4, 4], prec=1)
    lv.flags = 16
    A = _dist(0, 0.5, 1.0)
    # inner product: n must be a power of two
    st = L.mlmc_inner_product_estimate(1000, ctypes.byref(A), ctypes.byref(A), ctypes.byref(lv), 8, None,
                                       16, 1 << 40, None, None)
    assert st == 1 and b"power-of-two" in L.mlmc_last_error()
    # laws of the experiments
    X, Y = _dist(3, 0.4, 0.02), _dist(4, 10.0, 0.05)
    st = L.mlmc_inner_product_estimate(1024, ctypes.byref(X), ctypes.byref(Y), ctypes.byref(lv), 8, None,
                                       16, 1 << 40, None, None)
    assert st == 1
    # weighted draws
    lv.index_weights = 16
    st = L.mlmc_inner_product_estimate(1024, ctypes.byref(A), ctypes.byref(A), ctypes.byref(lv), 8, None,
                                       16, 1 << 40, None, None)
    assert st == 1 and b"32-bit index words" in L.mlmc_last_error()
    lv.index_weights = None
    # matrix products
    st = L.mlmc_matmul_estimate(4, 16, 3, ctypes.byref(A), ctypes.byref(A), ctypes.byref(lv), 8, None,
                                16, 1 << 40, None, None)
    assert st == 1 and b"32-bit index words" in L.mlmc_last_error()


def test_value16_validated(L):
    lv, keep = _levels([2, 4], [4, 4], prec=1)
    lv.flags = 32
    A = _dist(0, 0.5, 1.0)
    st = L.mlmc_inner_product_estimate(1024, ctypes.byref(A), ctypes.byref(A), ctypes.byref(lv), 8, None,
                                       16, 1 << 40, None, None)
    assert st == 1 and b"16-bit value" in L.mlmc_last_error()
    X, Y = _dist(5, 0.5, 1e-4), _dist(6, 2.0, 0.2)
    st = L.mlmc_matmul_estimate(4, 16, 3, ctypes.byref(X), ctypes.byref(Y), ctypes.byref(lv), 8, None,
                                16, 1 << 40, None, None)
    assert st == 1 and b"own stream" in L.mlmc_last_error()


def test_noalloc_limit_checked_before_the_device(L):
    # weighted draws need 8 n bytes of scratch: beyond the fixed array -> EINVAL,
    # decided on the host before any device call
    limit = L.mlmc_inner_product_noalloc_limit()
    assert limit == 4 << 20
    lv, keep = _levels([4, 8], [10, 10], prec=0)
    lv.index_weights = 8   # never dereferenced: the size check comes first
    A, B = _dist(), _dist()
    n = limit // 8 + 1024
    st = L.mlmc_inner_product_estimate_noalloc(n, ctypes.byref(A), ctypes.byref(B), ctypes.byref(lv), 8, None,
                                               None, None)
    assert st == 1
    assert b"allocation-free limit" in L.mlmc_last_error()
    bad, keep2 = _levels([4, 8], [10, 10], prec=0)
    bad.num_levels = 0
    st = L.mlmc_inner_product_estimate_noalloc(16, ctypes.byref(A), ctypes.byref(B), ctypes.byref(bad), 8, None,
                                               None, None)
    assert st == 1


@pytest.mark.parametrize("prec, func, weights, inner, what", [
    (2, 0, False, False, b"FP64 or FP32"), (3, 0, False, False, b"FP64 or FP32"),
    (0, 1, False, False, b"f = identity"), (1, 0, True, False, b"uniform index draws"),
    (0, 0, False, True, b"matrix products"),
])
def test_set_form_validated(L, prec, func, weights, inner, what):
    lv, keep = _levels([2, 4], [4, 4], prec=prec)
    lv.flags = 64
    lv.func = func
    lv.func_param[0] = 2.0
    if weights:
        lv.index_weights = 8   # never dereferenced: the flag check comes first
    A = _dist(0, 0.5, 1.0)
    if inner:
        st = L.mlmc_inner_product_estimate(1024, ctypes.byref(A), ctypes.byref(A), ctypes.byref(lv), 8, None,
                                           16, 1 << 40, None, None)
    else:
        st = L.mlmc_matmul_estimate(4, 16, 3, ctypes.byref(A), ctypes.byref(A), ctypes.byref(lv), 8, None,
                                    16, 1 << 40, None, None)
    assert st == 1 and what in L.mlmc_last_error()


def test_set_form_and_single_launch_workspace(L):
    """The set form adds its tables to the workspace; single_launch = 1 adds
    the second and third gather buffers where the single-launch kernel is
    built (FP32, i.i.d. normal laws, whole tiles) and nothing elsewhere
    (FP64); an out-of-range single_launch is rejected."""
    from paper_1904_00429_amd._lib import Problem, Tuning
    lv, keep = _levels([2, 4], [4, 4], prec=1)
    base = L.mlmc_matmul_workspace_size(64, 1000, 64, ctypes.byref(lv))
    lv.flags = 64
    assert L.mlmc_matmul_workspace_size(64, 1000, 64, ctypes.byref(lv)) > base
    lv.flags = 0
    arr = (Problem * 2)()
    for i in range(2):
        arr[i].m, arr[i].n, arr[i].p = 64, 1000 + i, 128
        arr[i].A, arr[i].B = _dist(0, 0.5, 1.0), _dist(0, 0.5, 1.0)
        arr[i].problem = i
        arr[i].out = 8
    t = Tuning()
    t.tile = 64
    plain = L.mlmc_matmul_batched_workspace_size(2, arr, ctypes.byref(lv), ctypes.byref(t))
    t.single_launch = 1
    assert L.mlmc_matmul_batched_workspace_size(2, arr, ctypes.byref(lv), ctypes.byref(t)) > plain
    lv.prec = 0
    t.single_launch = 0
    plain64 = L.mlmc_matmul_batched_workspace_size(2, arr, ctypes.byref(lv), ctypes.byref(t))
    t.single_launch = 1
    assert L.mlmc_matmul_batched_workspace_size(2, arr, ctypes.byref(lv), ctypes.byref(t)) == plain64
    t.single_launch = 2
    assert L.mlmc_matmul_batched_workspace_size(2, arr, ctypes.byref(lv), ctypes.byref(t)) == 0


def test_adjoint_workspace_follows_the_draws(L):
    # room for every draw of the call (one pass), so the size grows with N_l,
    # up to 4 GiB of pass buffers (plus G's two operand buffers)
    sizes = []
    for N in ([4, 4], [40, 40], [4000, 4000]):
        lv, keep = _levels([32, 64], N, prec=1)
        sizes.append(L.mlmc_matmul_adjoint_workspace_size(512, 32768, 512, ctypes.byref(lv)))
    assert 0 < sizes[0] < sizes[1] < sizes[2]
    # the differentiation workload (917504 draws) fits one pass; ten and a
    # hundred times its N_l are capped
    c = [32 * 2 ** l for l in range(7)]
    caps = []
    for scale in (1, 10, 100):
        lv, keep = _levels(c, [scale * (4096 >> l) for l in range(7)], prec=1)
        caps.append(L.mlmc_matmul_adjoint_workspace_size(512, 32768, 512, ctypes.byref(lv)))
    assert caps[0] < caps[1] == caps[2]
    assert (4 << 30) < caps[1] < (4 << 30) + (8 << 20)


def test_adjoint_workspace_below_one_pass_rejected(L):
    # any workspace from one 64-draw pass up is taken (more passes); below
    # that EWORKSPACE, with both sizes in the message, before any device call
    lv, keep = _levels([2, 4], [4, 4], prec=1)
    A, B = _dist(2), _dist(2)
    A.mean = A.stdev = B.mean = B.stdev = 16
    A.ld, B.ld = 4, 3
    st = L.mlmc_matmul_adjoint_reparam(4, 16, 3, ctypes.byref(A), ctypes.byref(B), ctypes.byref(lv), 16, 16, 16,
                                       16, 16, 16, 4096, None)
    assert st == 4
    msg = L.mlmc_last_error()
    assert b"at least" in msg and b"fewest passes" in msg


def test_inner_graph_arguments_checked_before_the_device(L):
    """mlmc_inner_product_graph_create refuses a NULL graph or stream, the
    adaptive loop (its bias test runs on the host), kernel timing and a short
    workspace before any device call; the report call checks its own."""
    lv, keep = _levels([4, 8], [10, 10], prec=0)
    x = _dist(1, 0.5, 1.0)
    need = L.mlmc_inner_product_workspace_size(1024, ctypes.byref(lv))
    g = ctypes.c_void_p()
    st = L.mlmc_inner_product_graph_create(1024, ctypes.byref(x), ctypes.byref(x), ctypes.byref(lv), 8, None,
                                           16, need, 8, None)
    assert st == 1 and b"graph is NULL" in L.mlmc_last_error()
    st = L.mlmc_inner_product_graph_create(1024, ctypes.byref(x), ctypes.byref(x), ctypes.byref(lv), 8, None,
                                           16, need, None, ctypes.byref(g))
    assert st == 1 and b"stream" in L.mlmc_last_error() and not g.value
    st = L.mlmc_inner_product_graph_create(1024, ctypes.byref(x), ctypes.byref(x), ctypes.byref(lv), 8, None,
                                           16, need - 1, 8, ctypes.byref(g))
    assert st == 4
    lv.flags = 2                                      # timing
    st = L.mlmc_inner_product_graph_create(1024, ctypes.byref(x), ctypes.byref(x), ctypes.byref(lv), 8, None,
                                           16, need, 8, ctypes.byref(g))
    assert st == 1 and b"timing" in L.mlmc_last_error()
    ad, keep2 = _levels([4, 8, 16], None, eps=1.0, pilot=10, prec=0)
    ad.flags = 4                                      # adaptive levels
    need_ad = L.mlmc_inner_product_workspace_size(1024, ctypes.byref(ad))
    st = L.mlmc_inner_product_graph_create(1024, ctypes.byref(x), ctypes.byref(x), ctypes.byref(ad), 8, None,
                                           16, need_ad, 8, ctypes.byref(g))
    assert st == 1 and b"adaptive" in L.mlmc_last_error() and not g.value
    st = L.mlmc_inner_product_graph_report(1024, ctypes.byref(ad), 16, need_ad, None, None)
    assert st == 1
    lv.flags = 0
    st = L.mlmc_inner_product_graph_report(1024, ctypes.byref(lv), 16, need - 1, None, None)
    assert st == 4
    st = L.mlmc_inner_product_graph_report(0, ctypes.byref(lv), 16, need, None, None)
    assert st == 1
