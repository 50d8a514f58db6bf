"""The inner-product estimate captured into a hipGraph
(mlmc_inner_product_graph_create) gives, replay after replay, the estimate of
the direct call bit for bit: the same kernels on the same draws in the same
order, in fixed-N_l and in target mode (pilot, eq. (28) and extension on the
device).  Replays are separated by other device work and synchronisations,
and the report call reads N_l, V_l and the schedule's status as the direct
call returns them (EBUDGET included)."""
import pytest

from gpu_helpers import flush

pytestmark = pytest.mark.gpu

CASES = [
    # ragged n, four levels, fixed N_l, both precisions
    dict(n=65539, law=("normal", 1.0, 0.5), c=[4, 8, 16, 32], prec="fp64", seed=7,
         kw=dict(n_samples=[400, 200, 100, 50])),
    dict(n=65539, law=("uniform", 0.5, 1.0), c=[4, 8, 16, 32], prec="fp32", seed=8,
         kw=dict(n_samples=[400, 200, 100, 50])),
    # the 2^20 inner product in target mode with 32-bit index words
    dict(n=1 << 20, law=("uniform", 0.5, 1.0), c=[64 * 2 ** l for l in range(9)], prec="fp32", seed=3,
         kw=dict(rmse_target=262.144 * 4, pilot=256, index_word32=True)),
    # target mode in FP64 with the stride coupling
    dict(n=4099, law=("normal", 1.0, 0.5), c=[4, 8, 16], prec="fp64", seed=5,
         kw=dict(rmse_target=2.0, pilot=64, coupling="stride")),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"n{c['n']}-{c['prec']}-{'target' if 'rmse_target' in c['kw'] else 'fixed'}")
def test_graph_replays_match_direct_call(case):
    import torch

    import paper_1904_00429_amd as api
    from paper_1904_00429_amd import Law
    dev = torch.device("cuda:0")
    kind, a, b = case["law"]
    law = getattr(Law, kind)(a, b)
    flush(f"inner graph: n={case['n']} levels={len(case['c'])} prec={case['prec']} kw={case['kw']}")
    ref = api.inner_product_estimate(case["n"], law, law, case["c"], seed=case["seed"], prec=case["prec"],
                                     device=dev, level_means=True, **case["kw"])
    g = api.InnerProductGraph(case["n"], law, law, case["c"], seed=case["seed"], prec=case["prec"], device=dev,
                              level_means=True, **case["kw"])
    scratch = torch.randn(1 << 20, device=dev)
    for replay in range(3):
        g.out.fill_(float("nan"))
        g.means.fill_(float("nan"))
        g.replay()
        rep = g.report()
        assert float(g.out) == float(ref.Y), replay
        assert torch.equal(g.means, ref.level_means), replay
        assert rep.n_used == ref.n_used
        assert rep.level_var == ref.level_var
        assert rep.rmse_est == ref.rmse_est
        # other device work between replays
        scratch = torch.sin(scratch) * 2.0
        torch.cuda.synchronize()
    g.release()


def test_graph_report_raises_the_schedule_budget():
    import torch

    import paper_1904_00429_amd as api
    from paper_1904_00429_amd import Law, MLMCError
    dev = torch.device("cuda:0")
    law = Law.normal(1.0, 0.5)
    kw = dict(rmse_target=1e-3, pilot=32, max_total_draws=100000)
    flush("inner graph: budget")
    with pytest.raises(MLMCError) as direct:
        api.inner_product_estimate(4099, law, law, [4, 8, 16], seed=2, prec="fp64", device=dev, **kw)
    g = api.InnerProductGraph(4099, law, law, [4, 8, 16], seed=2, prec="fp64", device=dev, **kw)
    g.replay()
    with pytest.raises(MLMCError) as graph:
        g.report()
    assert graph.value.status == direct.value.status == 3
    g.release()
