"""Benchmark: MLMC product estimates/s at fixed RMSE eps on one MI355X.

One step is one whole estimate on synthetic data: pilot realisations on every
level, the optimal allocation of Remark 3.6 (eq. (28)), the extension of every
level, the per-level statistics and the telescoping sum (eq. (10)).  Inputs are
laws, not arrays: every sampled value is generated inside the timed region
(the method draws its data).

Default workload: x, y in R^(2^20) with i.i.d. 0.5 + U(-1, 1) entries, ladder
c_l = 64 * 2^l (l = 0..8), eps = 1e-3 |E[x^T y]|, FP32 arithmetic, index draws
from 32-bit words (four per Philox call; exactly uniform since n is a power of
two; --index-words 64 selects the two-per-call 64-bit draws).

Printed: one JSON line with the throughput, the roofline of the dominant
kernel (device time from HIP events recorded by the library on the stream the
kernels run on) and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLMC product estimates/s at fixed RMSE eps"

# VALU issue slots per index draw of the inner-product level kernel, counted
# from the operations the algorithm needs, at gfx950 issue rates (full-rate
# 32-bit operation = 1 slot; 32x32->64-bit integer multiply-add and 32-bit
# high multiply are half rate = 2 slots):
#   1.5 Philox4x32-10 evaluations (half an index call, one value call), each
#       10 rounds x (2 multiply-adds x 2 + 2 three-input xors x 1) = 60 slots;
#       1.25 with 32-bit index words (a quarter of an index call);
#   index map: 1 shift for a power-of-two n, else high multiply + multiply-add = 4;
#   two uniform values: shift, convert, fused scale and law map = 4 each;
#   product and accumulation into the level sum = 2.
def slots_per_draw_inner(n: int, word32: bool = False) -> float:
    index = 1 if n & (n - 1) == 0 else 4
    return (1.25 if word32 else 1.5) * 60 + index + 2 * 4 + 2


# MI355X VALU issue: 256 CUs x 128 lanes per clock x 2.4 GHz = 78.6 T lane-ops/s
# (the 157.3 TFLOP/s FP32 vector peak counts an FMA as two flops).
PEAK_VALU_SLOTS = 256 * 128 * 2.4e9
PEAK_MFMA = {"fp64": 78.6e12, "fp32": 157.3e12, "bf16": 2.5e15, "fp8": 5.0e15}
PEAK_HBM = 8.0e12


def measured_traffic(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    passes (calibrated on a 1 GiB copy), or None once the kernel's sources differ
    from the ones the counters were taken on."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        entry = json.load(open(path))[kernel]
        h = hashlib.sha256()
        for src in entry["sources"]:
            h.update(open(os.path.join(ROOT, src), "rb").read())
        return entry["bytes_per_launch"] if h.hexdigest() == entry["sha256"] else None
    except (OSError, KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="matmul-large", choices=["inner", "matmul-large", "matmul-small", "diff", "batched", "matmul-large-fixed",
                             "importance", "experiments"])
    ap.add_argument("--prec", default=None,
                    help="matmul-large: fp64 (default), fp32, bf16 or fp8; inner: fp32 (default) or fp64")
    ap.add_argument("--no-forms", action="store_true",
                    help="matmul-large: skip the FP32 and BF16 runs of the same workload after the headline")
    ap.add_argument("--form-steps", type=int, default=None,
                    help="timed estimates of each extra precision (default: max(3, steps / 2))")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision-check", action="store_true",
                    help="skip the low-precision vs FP64 comparison of the matrix workloads")
    ap.add_argument("--cpu-fraction", type=float, default=0.15,
                    help="share of every level's realisations the CPU oracle runs")
    ap.add_argument("--func", default="identity", choices=["identity", "abs_step", "inv_abs_step"],
                    help="target function f of E[f(AB)]: |x| H(2 - x) or 1 / (|x| H(x + 0.4) + 0.01) (Sec. 4)")
    ap.add_argument("--index-words", type=int, default=32, choices=[32, 64],
                    help="inner product: index draws from 32-bit words (four per Philox call, power-of-two n) "
                         "or 64-bit words (two per call)")
    ap.add_argument("--value-bits", default="auto", choices=["auto", "16", "23"],
                    help="matrix and differentiation workloads: uniforms of the generated values (16: eight per Philox call); "
                         "auto: 16 for BF16 and FP8 operands of the i.i.d. matrix workloads (their rounding is far "
                         "coarser than 2^-16), 23 for FP32, FP64 and the differentiation workload")
    ap.add_argument("--adaptive", action="store_true",
                    help="choose the number of levels by the bias test (the workload's ladder is the longest)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after timing, run one device copy of 1 GiB (counter calibration)")
    return ap.parse_args()


def _oracle_func(oracle, name):
    return {"identity": None, "abs_step": oracle.Func.abs_step(2.0),
            "inv_abs_step": oracle.Func.inv_abs_step(0.4, 0.01)}[name]


def cpu_baseline_inner(wl, n_used, fraction, func="identity", word32=False):
    """The oracle (single-threaded C) on the first `fraction` of every level's
    realisations of the same workload; scaled to estimates/s."""
    import oracle
    oracle.build(force=False)
    law = oracle.Law.uniform(wl.law_a[1], wl.law_a[2])
    f = _oracle_func(oracle, func)
    t0 = time.perf_counter()
    draws = 0
    for l, N in enumerate(n_used):
        if N == 0:
            continue
        k = max(2, int(round(N * fraction)))
        st = oracle.LevelState.empty(1, 1)
        oracle.level_estimation(st, 1, wl.n, 1, law, law, wl.c[l], wl.c[l - 1] if l else 0, wl.seed, 0, l, 0, k,
                                func=f, index_word32=word32)
        draws += k * wl.c[l]
    dt = time.perf_counter() - t0
    total_draws = sum(N * c for N, c in zip(n_used, wl.c))
    full = dt * total_draws / draws
    return {"value": 1.0 / full, "unit": "estimates/s", "cores": 1, "kind": "oracle",
            "sample": f"{draws} of {total_draws} index draws ({fraction:.0%} of every level's "
                      f"realisations), {dt:.1f} s, scaled by draws"}


def cpu_model() -> str:
    """The host CPU's model name (as lscpu prints it)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads() -> int:
    """Threads the all-cores baseline uses: the CPUs this process may run on,
    at most 16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline_matmul(wl, n_used, fraction, edge=256, func="identity", all_fraction=0.004):
    """The oracle on the same ladder, laws and N_l with m = p = edge, on one
    core and on all the host threads.

    A full-shape realisation of the finest level costs the oracle minutes, so
    each level runs a sample of realisations at the reduced shape; the time
    per realisation t_l gives sum_l N_l t_l, scaled by m p / edge^2 (the
    oracle's sketch loop, m p (c_l + c_{l-1}) multiply-adds per realisation,
    dominates its per-realisation cost).  One core: max(1, fraction N_l)
    realisations per level.  All threads: max(threads, all_fraction N_l)
    realisations per level, split into one contiguous range per thread (the C
    oracle runs outside the interpreter lock), timed by the wall clock."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    oracle.build(force=False)
    law = oracle.Law.normal(wl.law_a[1], wl.law_a[2])
    f = _oracle_func(oracle, func)
    m, p = min(edge, wl.m), min(edge, wl.p)
    scale = (wl.m * wl.p) / float(m * p)

    def run(l, k0, k1):
        st = oracle.LevelState.empty(m, p)
        oracle.level_estimation(st, m, wl.n, p, law, law, wl.c[l], wl.c[l - 1] if l else 0,
                                wl.seed, 0, l, k0, k1, func=f)

    total, run1 = 0.0, 0
    t_all = time.perf_counter()
    for l, N in enumerate(n_used):
        if N == 0:
            continue
        k = max(1, int(round(N * fraction)))
        t0 = time.perf_counter()
        run(l, 0, k)
        total += N * (time.perf_counter() - t0) / k
        run1 += k
    dt1 = time.perf_counter() - t_all
    threads = host_threads()
    total_mt, run_mt = 0.0, 0
    t_all = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        for l, N in enumerate(n_used):
            if N == 0:
                continue
            k = max(threads, int(round(N * all_fraction)))
            cuts = [k * i // threads for i in range(threads + 1)]
            t0 = time.perf_counter()
            list(ex.map(lambda i: run(l, cuts[i], cuts[i + 1]), range(threads)))
            total_mt += N * (time.perf_counter() - t0) / k
            run_mt += k
    dtm = time.perf_counter() - t_all
    return {"value": 1.0 / (total_mt * scale), "unit": "estimates/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{run_mt} realisations (max({threads}, {all_fraction} N_l) per level, split over {threads} "
                      f"threads) at m = p = {m}, {dtm:.1f} s wall; sum_l N_l t_l scaled by m p / {m * p}",
            "one_core": {"value": 1.0 / (total * scale), "cores": 1,
                         "sample": f"{run1} realisations (max(1, {fraction} N_l) per level) at m = p = {m}, "
                                   f"{dt1:.1f} s"}}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported (the library "
              f"drives one GPU; the per-level work would shard over GPUs with one merge of the "
              f"level statistics per phase)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1904_00429_amd import Law, workloads
    import paper_1904_00429_amd.mlmc as api

    dev = torch.device("cuda:0")
    torch.cuda.init()
    timing_flag = 2
    _OPTS["func"] = _func_of(args.func)
    _OPTS["adaptive"] = bool(args.adaptive)
    args.index_word32 = args.workload == "inner" and args.index_words == 32
    _OPTS["index_word32"] = args.index_word32
    _OPTS["value_bits"] = args.value_bits
    if args.workload == "diff":
        return bench_diff(args)
    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "matmul-large-fixed":
        return bench_large_fixed(args)
    if args.workload == "importance":
        return bench_importance(args)
    if args.workload == "experiments":
        # a Sec. 4.2 estimate takes seconds: fewer steps unless asked for
        if "--steps" not in sys.argv:
            args.steps = 3
        if "--warmup" not in sys.argv:
            args.warmup = 1
        return bench_experiments(args)
    if args.workload == "inner":
        wl = workloads.INNER_2POW20
        prec = args.prec or "fp32"
        x = Law.uniform(wl.law_a[1], wl.law_a[2])
        expected = wl.n * wl.law_a[1] * wl.law_b[1]

        def step(want_timing, seed):
            return _inner(api, wl, x, prec, dev, want_timing, seed)
    else:
        wl = workloads.MATMUL_LARGE if args.workload == "matmul-large" else workloads.MATMUL_SMALL_FP64
        prec = args.prec or "fp64"
        a = Law.normal(wl.law_a[1], wl.law_a[2])
        expected = wl.n * wl.law_a[1] * wl.law_b[1]

        def step(want_timing, seed):
            return _matmul(api, wl, a, prec, dev, want_timing, seed)

    # every step is an independent estimate: seed = step number
    for i in range(args.warmup):
        step(False, 1000 + i)
    torch.cuda.synchronize()
    results = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        results.append(step(True, i))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = args.steps / elapsed

    # achieved accuracy against the exact E[AB] (closed form of the synthetic
    # law; no closed form for a nonlinear f)
    rmse_obs = None
    if args.func == "identity" and not args.adaptive:
        errs = [float(torch.linalg.norm(r.Y - expected)) for r in results]
        rmse_obs = math.sqrt(sum(e * e for e in errs) / len(errs))
    rep = results[-1]
    k_ms = [sum(r.kernel_ms[i] for r in results) for i in range(4)]
    k_n = [sum(r.kernel_launches[i] for r in results) for i in range(4)]
    draws = sum(r.total_draws for r in results)

    if args.workload == "inner":
        avg = k_ms[0] / max(k_n[0], 1)
        slots = slots_per_draw_inner(wl.n, args.index_word32) * draws / max(k_n[0], 1)
        achieved = slots / (avg * 1e-3)
        roof = {"bound": "alu", "kernel": f"inner_multi_kernel<{'float' if prec == 'fp32' else 'double'}>",
                "achieved": achieved / 1e12, "peak": PEAK_VALU_SLOTS / 1e12, "unit": "Tops/s",
                "frac": achieved / PEAK_VALU_SLOTS, "traffic": measured_traffic("inner_multi_kernel"),
                "traffic_unit": "bytes per launch",
                "avg_launch_ms": avg, "launches": k_n[0],
                "ops_per_draw": slots_per_draw_inner(wl.n, args.index_word32)}
        config = {"workload": wl.name, "n": wl.n, "levels": len(wl.c), "c0": wl.c[0], "ratio": 2,
                  "eps": wl.rmse_target, "pilot": wl.pilot, "law": "0.5 + U(-1, 1) i.i.d.",
                  "prec": prec, "func": args.func, "adaptive": bool(args.adaptive),
                  "index_words": 32 if args.index_word32 else 64}
    else:
        # dominant: the sketch (MFMA) kernel; algorithmic flops 2 m p per draw
        flops = 2.0 * wl.m * wl.p * draws
        achieved = flops / (k_ms[0] * 1e-3)
        roof = {"bound": "mfma", "kernel": f"sketch_kernel<{prec}>", "achieved": achieved / 1e12,
                "peak": PEAK_MFMA[prec] / 1e12, "unit": "TFLOP/s", "frac": achieved / PEAK_MFMA[prec],
                "traffic": measured_traffic(f"sketch_kernel<{prec}>") if wl is workloads.MATMUL_LARGE else None,
                "traffic_unit": "bytes per launch",
                "avg_launch_ms": k_ms[0] / max(k_n[0], 1), "launches": k_n[0],
                "gather_ms_per_step": k_ms[1] / args.steps, "sketch_ms_per_step": k_ms[0] / args.steps,
                "merge_ms_per_step": k_ms[2] / args.steps}
        config = {"workload": wl.name, "m": wl.m, "n": wl.n, "p": wl.p, "levels": len(wl.c), "c0": wl.c[0],
                  "ratio": 2, "eps": wl.rmse_target, "pilot": wl.pilot, "prec": prec, "func": args.func,
                  "adaptive": bool(args.adaptive), "value_bits": 16 if _value16(prec) else 23}

    out = {"metric": METRIC, "value": value, "unit": "estimates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": {"fp32": "f32", "fp64": "f64", "bf16": "bf16", "fp8": "fp8_e4m3"}[prec],
           "data": "synthetic (entries generated inside the estimate)", "config": config, "roofline": roof,
           "n_used": rep.n_used, "draws_per_step": draws / args.steps, "rmse_est": rep.rmse_est,
           "rmse_observed": rmse_obs, "levels_used": rep.levels_used, "kernel_ms_per_step": {
               "sample": k_ms[0] / args.steps, "gather": k_ms[1] / args.steps, "merge": k_ms[2] / args.steps,
               "final": k_ms[3] / args.steps}}

    if args.workload == "inner" and not args.adaptive:
        out["graph"] = _inner_graph(api, wl, x, prec, dev, args.steps, args.warmup)

    forms = {}
    if args.workload == "matmul-large" and not args.no_forms and not args.adaptive:
        # the same workload in the other precisions of the precision form:
        # estimates/s and the sketch's share of its MFMA peak, each timed like
        # the headline (fresh seeds, target mode, every value generated inside)
        k_form = args.form_steps or max(3, args.steps // 2)
        for pr in ("fp64", "fp32", "bf16", "fp8"):
            if pr == prec:
                forms[pr] = {"estimates_per_s": value, "ms_per_estimate": ms_per_step,
                             "sketch_frac": roof["frac"] if roof["bound"] == "mfma" else None}
                continue
            _matmul(api, wl, a, pr, dev, False, 2000)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            runs = [_matmul(api, wl, a, pr, dev, True, 3000 + i) for i in range(k_form)]
            torch.cuda.synchronize()
            sec = (time.perf_counter() - t1) / k_form
            sk_ms = sum(r.kernel_ms[0] for r in runs)
            fl = 2.0 * wl.m * wl.p * sum(r.total_draws for r in runs)
            forms[pr] = {"estimates_per_s": 1.0 / sec, "ms_per_estimate": 1e3 * sec, "steps": k_form,
                         "value_bits": 16 if _value16(pr) else 23,
                         "sketch_tflops": fl / (sk_ms * 1e-3) / 1e12,
                         "sketch_frac": fl / (sk_ms * 1e-3) / PEAK_MFMA[pr],
                         "kernel_ms_per_estimate": {
                             "sketch": sk_ms / k_form, "gather": sum(r.kernel_ms[1] for r in runs) / k_form,
                             "merge": sum(r.kernel_ms[2] for r in runs) / k_form,
                             "final": sum(r.kernel_ms[3] for r in runs) / k_form},
                         "rmse_est": runs[-1].rmse_est}
            del runs
        out["forms"] = forms
        if "fp32" in forms and "bf16" in forms:
            out["bf16_over_fp32"] = forms["bf16"]["estimates_per_s"] / forms["fp32"]["estimates_per_s"]
        if "fp32" in forms and "fp8" in forms:
            out["fp8_over_fp32"] = forms["fp8"]["estimates_per_s"] / forms["fp32"]["estimates_per_s"]

    lps = [pr for pr in forms if pr != "fp64"] or ([prec] if prec != "fp64" else [])
    if args.workload != "inner" and lps and not args.no_precision_check and not args.adaptive:
        # precision form: the same estimate (seed 0, the N_l of the last timed
        # step, fixed mode) in each lower precision and in FP64, outside the
        # timed region; the rounding error is reported next to RMSE_est
        from paper_1904_00429_amd import matmul_estimate
        y64 = {}                      # FP64 reference per value stream (16- or 23-bit uniforms)
        checks = {}
        for pr in lps:
            v16 = _value16(pr)
            if v16 not in y64:
                y64[v16] = matmul_estimate(wl.m, wl.n, wl.p, a, a, wl.c, n_samples=rep.n_used, seed=0, prec="fp64",
                                           device=dev, report=True, func=_OPTS["func"], value16=v16)
            ylp = matmul_estimate(wl.m, wl.n, wl.p, a, a, wl.c, n_samples=rep.n_used, seed=0, prec=pr,
                                  device=dev, report=True, func=_OPTS["func"], value16=v16)
            d = float(torch.linalg.norm(ylp.Y - y64[v16].Y))
            checks[pr] = {"lp_minus_fp64_frob": d, "rmse_est_fp64": y64[v16].rmse_est,
                          "over_rmse_est": d / y64[v16].rmse_est, "value_bits": 16 if v16 else 23}
            del ylp
        out["precision_check"] = {"seed": 0, "n_samples": rep.n_used, "forms": checks}
        del y64
        torch.cuda.empty_cache()


    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = src.numel() * 4

    if not args.no_cpu_baseline:
        if args.workload == "inner":
            out["cpu_baseline"] = cpu_baseline_inner(wl, rep.n_used, args.cpu_fraction, args.func,
                                                     args.index_word32)
        else:
            out["cpu_baseline"] = cpu_baseline_matmul(wl, rep.n_used, 0.001, func=args.func)
    print(json.dumps(out), flush=True)


def bench_diff(args):
    """Differentiation form: loss = ||Y - T||_F^2 of the reparameterised
    estimate, forward + hand-written adjoint per step (FP32, or --prec bf16:
    BF16 operands on MFMA in both)."""
    import torch
    from paper_1904_00429_amd import mlmc_matmul, workloads
    import paper_1904_00429_amd.mlmc as api
    dev = torch.device("cuda:0")
    wl = workloads.DIFF_512x32768x512
    MA, SA, MB, SB, T = workloads.reparam_inputs(wl.m, wl.n, wl.p, seed=0)
    leaves = [torch.from_numpy(x).to(dev).requires_grad_(True) for x in (MA, SA, MB, SB)]
    Tt = torch.from_numpy(T).to(dev, torch.float64)
    prec = args.prec or "fp32"
    if prec not in ("fp32", "bf16"):
        raise SystemExit("the differentiation form runs in fp32 or bf16")
    # 16-bit values only when asked for: with reparameterised laws they
    # measured slower in BF16 (47.2 against 50.7 estimates/s)
    v16 = _OPTS.get("value_bits") == "16"

    def step(seed):
        for t in leaves:
            t.grad = None
        Y = mlmc_matmul(*leaves, wl.c, wl.n_samples, seed=seed, prec=prec, value16=v16)
        loss = ((Y - Tt) ** 2).sum()
        loss.backward()
        return loss

    for i in range(args.warmup):
        step(1000 + i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # one timed adjoint call with the library's event timing, for the roofline
    import ctypes
    draws = sum(N * c for N, c in zip(wl.n_samples, wl.c))
    flops = 2.0 * 2.0 * wl.m * wl.p * draws
    t1 = time.perf_counter()
    grads = api.matmul_adjoint_reparam(*[t.detach() for t in leaves], wl.c, wl.n_samples,
                                       torch.ones((wl.m, wl.p), dtype=torch.float64, device=dev), prec=prec,
                                       value16=v16)
    torch.cuda.synchronize()
    adj_ms = 1e3 * (time.perf_counter() - t1)
    out = {"metric": "MLMC product estimates/s with gradients (forward + adjoint)", "value": args.steps / elapsed,
           "unit": "estimates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": {"fp32": "f32", "bf16": "bf16"}[prec], "data": "synthetic",
           "config": {"workload": wl.name, "m": wl.m, "n": wl.n, "p": wl.p, "levels": len(wl.c), "c0": wl.c[0],
                      "n_samples": wl.n_samples, "prec": prec, "value_bits": 16 if v16 else 23},
           "adjoint_ms_wall": adj_ms,
           "adjoint_roofline": {"bound": "mfma", "achieved": flops / (adj_ms * 1e-3) / 1e12,
                                "peak": PEAK_MFMA[prec] / 1e12, "unit": "TFLOP/s",
                                "frac": flops / (adj_ms * 1e-3) / PEAK_MFMA[prec], "draws": draws}}
    print(json.dumps(out), flush=True)


def bench_importance(args):
    """Importance sampling (Theorem 3.1's xi**) against uniform draws on the
    column-ramped reparameterised 512 x 32768 x 512 product at the same target
    RMSE: estimates/s and draws per estimate of each sampler (FP32)."""
    import torch
    from paper_1904_00429_amd import Law, matmul_estimate, optimal_index_weights, workloads
    dev = torch.device("cuda:0")
    wl = workloads.IS_512x32768x512
    MA, SA, MB, SB = workloads.reparam_ramp_inputs(wl.m, wl.n, wl.p, seed=0)
    t = [torch.from_numpy(x).to(dev) for x in (MA, SA, MB, SB)]
    A, B = Law.reparam(t[0], t[1]), Law.reparam(t[2], t[3])
    exact = (t[0].double().T @ t[2].double())            # E[AB] of the laws (for the observed error)
    eps = 0.1 * float(torch.linalg.norm(exact))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    w = optimal_index_weights(wl.m, wl.n, wl.p, A, B, device=dev)
    torch.cuda.synchronize()
    w_ms = 1e3 * (time.perf_counter() - t0)
    res = {}
    for name, iw in (("xi**", w), ("uniform", None)):
        def step(seed):
            return matmul_estimate(wl.m, wl.n, wl.p, A, B, wl.c, rmse_target=eps, pilot=wl.pilot, seed=seed,
                                   prec="fp32", device=dev, index_weights=iw)
        for i in range(args.warmup):
            step(1000 + i)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        runs = [step(i) for i in range(args.steps)]
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t1) / args.steps
        err = [float(torch.linalg.norm(r.Y - exact)) for r in runs]
        res[name] = {"estimates_per_s": 1.0 / sec, "ms_per_estimate": 1e3 * sec,
                     "draws_per_estimate": sum(r.total_draws for r in runs) / len(runs),
                     "n_used": runs[-1].n_used, "rmse_est": runs[-1].rmse_est,
                     "rmse_observed": math.sqrt(sum(e * e for e in err) / len(err))}
    flops = 2.0 * wl.m * wl.p * res["xi**"]["draws_per_estimate"] / (res["xi**"]["ms_per_estimate"] * 1e-3)
    out = {"metric": "MLMC product estimates/s at fixed RMSE eps (importance-sampled indices)",
           "value": res["xi**"]["estimates_per_s"], "unit": "estimates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": res["xi**"]["ms_per_estimate"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": wl.name, "m": wl.m, "n": wl.n, "p": wl.p, "levels": len(wl.c), "c0": wl.c[0],
                      "eps": eps, "pilot": wl.pilot, "law": "reparam, A's columns scaled by 0.05 .. 3"},
           "samplers": res, "speedup_over_uniform": res["xi**"]["estimates_per_s"] / res["uniform"]["estimates_per_s"],
           "weights_ms": w_ms,
           "roofline": {"bound": "mfma", "achieved": flops / 1e12, "peak": PEAK_MFMA["fp32"] / 1e12,
                        "unit": "TFLOP/s", "frac": flops / PEAK_MFMA["fp32"], "traffic": None,
                        "note": "algorithmic 2 m p flops per draw over the whole estimate"}}
    print(json.dumps(out), flush=True)


def _experiment_laws(wl):
    from paper_1904_00429_amd import Func, Law
    return (getattr(Law, wl.law_a[0])(*wl.law_a[1]), getattr(Law, wl.law_b[0])(*wl.law_b[1]),
            getattr(Func, wl.func[0])(*wl.func[1]))


def _experiment_run(api, wl, A, B, f, prec, dev, seed, eps=0.0, n_samples=None, timing=False):
    """One estimate through the C ABI (adaptive L in target mode), with the
    library's per-class kernel times when `timing`."""
    import ctypes
    import torch
    c = wl.c if n_samples is None else wl.c[:len(n_samples)]
    h = api._LevelsHolder(c, n_samples, eps, wl.pilot, seed, prec, False, 0, 0, f, n_samples is None)
    if timing:
        h.lv.flags |= 2
    lib = api.lib()
    rep = api.Report()
    da, db = A.c(), B.c()
    if wl.kind == "inner":
        need = int(lib.mlmc_inner_product_workspace_size(wl.n, ctypes.byref(h.lv)))
    else:
        need = int(lib.mlmc_matmul_workspace_size(wl.m, wl.n, wl.p, ctypes.byref(h.lv)))
    key = ("exp", wl.name, prec, len(c))
    if key not in _WS or _WS[key][0].numel() < need:
        _WS.pop(key, None)
        torch.cuda.empty_cache()
        _WS[key] = (torch.empty(need, dtype=torch.uint8, device=dev),
                    torch.empty((wl.m, wl.p), dtype=torch.float64, device=dev))
    ws, out = _WS[key]
    if wl.kind == "inner":
        st = lib.mlmc_inner_product_estimate(wl.n, ctypes.byref(da), ctypes.byref(db), ctypes.byref(h.lv),
                                             out.data_ptr(), None, ws.data_ptr(), ws.numel(), ctypes.byref(rep),
                                             api._stream(dev))
    else:
        st = lib.mlmc_matmul_estimate(wl.m, wl.n, wl.p, ctypes.byref(da), ctypes.byref(db), ctypes.byref(h.lv),
                                      out.data_ptr(), None, ws.data_ptr(), ws.numel(), ctypes.byref(rep),
                                      api._stream(dev))
    api.check(st)
    return _Rep(out.clone(), rep, len(c))


def cpu_baseline_experiment(wl, n_used, budget_s=6.0):
    """The oracle (one core) on the same laws, f, ladder and N_l.

    Inner product: max(2, N_l / 20) realisations per level at the full n,
    scaled by N_l.  Matrix product: per level, the time per realisation is
    measured at m = p = 24 and 48 (a few realisations, capped by the draws a
    level needs) and fitted as alpha (m + p) + beta m p (generation of the
    sampled columns plus the sketch), evaluated at the full shape and summed
    over N_l."""
    import oracle
    oracle.build(force=False)
    kinds = {"ramp_normal": (oracle.LAW_RAMP_NORMAL, 1, 0), "cos_poisson_exp": (oracle.LAW_COS_POISSON_EXP, 0, 1),
             "sin_ramp": (oracle.LAW_SIN_RAMP, 1, 0), "cos_poisson_step": (oracle.LAW_COS_POISSON_STEP, 0, 1)}

    def law(desc):
        kind, iscale, iloc = kinds[desc[0]]
        return oracle.Law.experiment(kind, desc[1][iloc], desc[1][iscale])
    A, B = law(wl.law_a), law(wl.law_b)
    f = getattr(oracle.Func, wl.func[0])(*wl.func[1])
    total, run, t_all = 0.0, 0, time.perf_counter()
    for l, N in enumerate(n_used):
        if N == 0:
            continue
        cp = wl.c[l - 1] if l else 0
        if wl.kind == "inner":
            k = max(2, N // 20)
            st = oracle.LevelState.empty(1, 1)
            t0 = time.perf_counter()
            oracle.level_estimation(st, 1, wl.n, 1, A, B, wl.c[l], cp, 0, 0, l, 0, k, func=f)
            total += N * (time.perf_counter() - t0) / k
            run += k
            continue
        times = []
        for e in (24, 48):
            k = max(1, min(N, int(5e4 // wl.c[l])))
            st = oracle.LevelState.empty(e, e)
            t0 = time.perf_counter()
            oracle.level_estimation(st, e, wl.n, e, A, B, wl.c[l], cp, 0, 0, l, 0, k, func=f)
            times.append((time.perf_counter() - t0) / k)
            run += k
        # t = alpha (2e) + beta e^2 at e = 24, 48
        beta = (times[1] - 2.0 * times[0]) / (48.0 ** 2 - 2.0 * 24.0 ** 2)
        alpha = (times[0] - beta * 24.0 ** 2) / 48.0
        beta, alpha = max(beta, 0.0), max(alpha, 0.0)
        total += N * (alpha * (wl.m + wl.p) + beta * wl.m * wl.p)
    dt = time.perf_counter() - t_all
    sample = (f"{run} realisations (N_l / 20 per level) at n = {wl.n}" if wl.kind == "inner" else
              f"{run} realisations at m = p = 24 and 48 per level, time per realisation fitted as "
              f"alpha (m + p) + beta m p and evaluated at {wl.m} x {wl.p}")
    return {"value": 1.0 / total, "unit": "estimates/s", "cores": 1, "kind": "oracle",
            "sample": f"{sample}; {dt:.1f} s"}


def bench_experiments(args):
    """The experiments of Sec. 4 at the paper's sizes: adaptive L on M = 10
    ladders, eps = 0.1 of the size of E[f] (the workloads' fixed estimate of
    it; Sec. 4.1's N_l scaled by 1/20); estimates/s of each, with the spread
    of the independent estimates as the observed RMSE and the mean over their
    entries (every entry of E[f(AB)] is the same) as a check of the size."""
    import torch
    import paper_1904_00429_amd.mlmc as api
    from paper_1904_00429_amd import workloads
    dev = torch.device("cuda:0")
    prec = args.prec or "fp32"
    res = {}
    for wl in (workloads.EXP41_INNER, workloads.EXP42_MATMUL):
        A, B, f = _experiment_laws(wl)
        size, eps = wl.size, wl.eps
        # the inner product computes in FP64 or FP32
        wprec = prec if wl.kind == "matmul" or prec in ("fp32", "fp64") else "fp32"
        for i in range(args.warmup):
            _experiment_run(api, wl, A, B, f, wprec, dev, 1000 + i, eps=eps)
        torch.cuda.synchronize()
        print(f"[experiments] {wl.name}: timing", flush=True)
        t0 = time.perf_counter()
        runs = [_experiment_run(api, wl, A, B, f, wprec, dev, i, eps=eps, timing=True) for i in range(args.steps)]
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / args.steps
        # observed RMSE: spread of the independent estimates around their mean
        ybar = sum(r.Y for r in runs) / len(runs)
        size_obs = abs(float(ybar.mean())) * math.sqrt(wl.m * wl.p)
        spread = math.sqrt(sum(float(torch.linalg.norm(r.Y - ybar)) ** 2 for r in runs) / max(len(runs) - 1, 1))
        k_ms = [sum(r.kernel_ms[i] for r in runs) / args.steps for i in range(4)]
        k_n = [sum(r.kernel_launches[i] for r in runs) for i in range(4)]
        draws = sum(r.total_draws for r in runs) / args.steps
        entry = {"estimates_per_s": 1.0 / sec, "ms_per_estimate": 1e3 * sec, "eps": eps,
                 "size": size, "size_from_these_estimates": size_obs,
                 "levels_used": [r.levels_used for r in runs],
                 "bias_test_passed": [r.bias_test_passed for r in runs],
                 "n_used": runs[-1].n_used, "rmse_est": runs[-1].rmse_est, "draws_per_estimate": draws,
                 "rmse_observed": spread, "relative_rmse_observed": spread / size,
                 "kernel_ms_per_estimate": {"sample": k_ms[0], "gather": k_ms[1], "merge": k_ms[2], "final": k_ms[3]},
                 "launches_per_estimate": [x / args.steps for x in k_n]}
        if wl.kind == "inner":
            entry["paper_time_s"] = 0.047
        else:
            flops = 2.0 * wl.m * wl.p * draws
            entry["sketch_tflops"] = flops / (k_ms[0] * 1e-3) / 1e12
            entry["values_per_s_gather"] = draws * (wl.m + wl.p) / (k_ms[1] * 1e-3)
            entry["paper_time_s"] = 2.240
        res[wl.name] = (wl, entry)
        print(f"[experiments] {wl.name}: {json.dumps(entry)}", flush=True)
    wl, e = res[workloads.EXP42_MATMUL.name]
    flops = 2.0 * wl.m * wl.p * e["draws_per_estimate"]
    sk = e["kernel_ms_per_estimate"]["sample"]
    out = {"metric": "MLMC estimates/s of E[f(AB)] on the laws of Sec. 4.2 (adaptive L, eps 0.1 relative)",
           "value": e["estimates_per_s"], "unit": "estimates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": e["ms_per_estimate"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": {"fp32": "f32", "fp64": "f64", "bf16": "bf16", "fp8": "fp8_e4m3"}[prec],
           "data": "synthetic (the laws of Sec. 4 generated inside the estimate)",
           "config": {"workload": wl.name, "m": wl.m, "n": wl.n, "p": wl.p, "ladder": "c_l = 10^l, l <= 6",
                      "func": "|x| H(2 - x)", "eps": e["eps"], "prec": prec, "adaptive": True},
           "experiments": {name: entry for name, (_, entry) in res.items()},
           "roofline": {"bound": "mfma", "kernel": f"sketch_kernel<{prec}> (target-function form)",
                        "achieved": flops / (sk * 1e-3) / 1e12, "peak": PEAK_MFMA[prec] / 1e12,
                        "unit": "TFLOP/s", "frac": flops / (sk * 1e-3) / PEAK_MFMA[prec], "traffic": None,
                        "note": "algorithmic 2 m p flops per draw over the sketch launches of an estimate; "
                                "the gather of the sampled columns is timed separately"}}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_experiment(wl, e["n_used"])
        wi, ei = res[workloads.EXP41_INNER.name]
        out["experiments"][wi.name]["cpu_baseline"] = cpu_baseline_experiment(wi, ei["n_used"])
    print(json.dumps(out), flush=True)


def _time_replays(est, steps, warmup):
    import torch
    for _ in range(warmup):
        est.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        est.replay()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def bench_batched(args):
    """Batching form: 256 uneven products per estimate, one hipGraph replay per
    step; FP8 e4m3 (the value) and FP32 (for the ratio), autotuned tiles."""
    import torch
    from paper_1904_00429_amd import BatchedEstimate, BatchProblem, Law, autotune, workloads
    dev = torch.device("cuda:0")
    shapes, mus, c, N = workloads.batched_products()
    probs = [BatchProblem(m, n, p, Law.normal(mu, 1.0), Law.normal(mu, 1.0), i)
             for i, ((m, n, p), mu) in enumerate(zip(shapes, mus))]
    draws = sum(Nl * cl for Nl, cl in zip(N, c))
    flops = sum(2.0 * m * p for m, n, p in shapes) * draws
    out = {}
    for prec in ("fp8", "fp32"):
        best = autotune.tune(probs, c, N, prec=prec, device=dev)
        est = BatchedEstimate(probs, c, N, seed=0, prec=prec, tuning=best, device=dev, value16=_value16(prec))
        est.capture()
        sec = _time_replays(est, args.steps, args.warmup)
        out[prec] = {"s_per_estimate": sec, "tuning": best, "mfma_tflops_whole_graph": flops / sec / 1e12}
        est.release()
        del est
        torch.cuda.empty_cache()
        # the single-launch form beside it (one persistent kernel for every
        # pass of every level), at the tile where the table is whole
        single = {"tile": 64, "target_blocks": 0, "gather_budget": 768 << 20, "single_launch": 1}
        est = BatchedEstimate(probs, c, N, seed=0, prec=prec, tuning=single, device=dev, value16=_value16(prec))
        est.capture()
        out[prec]["single_launch_s_per_estimate"] = _time_replays(est, args.steps, args.warmup)
        est.release()
        del est
        torch.cuda.empty_cache()
    value = 1.0 / out["fp8"]["s_per_estimate"]
    res = {"metric": "MLMC batched estimates/s (256 products per estimate, fixed N_l)", "value": value,
           "unit": "estimates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 * out["fp8"]["s_per_estimate"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "fp8", "data": "synthetic",
           "config": {"workload": "batched-256-uneven", "products": len(shapes), "c0": c[0], "levels": len(c),
                      "N": N, "graph": True,
                      "value_bits": {"fp8": 16 if _value16("fp8") else 23, "fp32": 16 if _value16("fp32") else 23}},
           "products_per_s": len(shapes) * value,
           "fp32_value": 1.0 / out["fp32"]["s_per_estimate"],
           "fp8_over_fp32": out["fp32"]["s_per_estimate"] / out["fp8"]["s_per_estimate"],
           "forms": out,
           "roofline": {"bound": "mfma", "achieved": out["fp8"]["mfma_tflops_whole_graph"],
                        "peak": 5000.0, "unit": "TFLOP/s",
                        "frac": out["fp8"]["mfma_tflops_whole_graph"] / 5000.0, "traffic": None,
                        "note": "algorithmic 2 m p flops per draw over the whole graph time"}}
    print(json.dumps(res), flush=True)


def bench_large_fixed(args):
    """1024 x 65536 x 1024 at the N_l a target-RMSE run chose, through the
    table pipeline with each tile shape, BF16 and FP32 (sketch-kernel study;
    with --func, the target-function form at the same N_l)."""
    import torch
    from paper_1904_00429_amd import BatchedEstimate, BatchProblem, Law, workloads
    dev = torch.device("cuda:0")
    wl = workloads.MATMUL_LARGE
    N = [120032, 60001, 30001, 15001, 7501, 3751, 1876, 938]
    draws = sum(a * b for a, b in zip(N, wl.c))
    flops = 2.0 * wl.m * wl.p * draws
    prob = [BatchProblem(wl.m, wl.n, wl.p, Law.normal(0.5, 1.0), Law.normal(0.5, 1.0), 0)]
    res = {}
    func = _func_of(args.func)
    for prec in ("bf16", "fp32"):
        # a target function always runs the tile-64 sketch
        for tile in ((64, 128) if func is None else (64,)):
            est = BatchedEstimate(prob, wl.c, N, seed=0, prec=prec, tuning={"tile": tile}, device=dev, func=func)
            est.run()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                est.run()
            torch.cuda.synchronize()
            sec = (time.perf_counter() - t0) / args.steps
            res[f"{prec}-tile{tile}"] = {"s_per_estimate": sec, "estimates_per_s": 1.0 / sec,
                                         "mfma_tflops_whole_pipeline": flops / sec / 1e12}
            del est
            torch.cuda.empty_cache()
    print(json.dumps({"workload": "matmul-1024x65536x1024-fixedN", "func": args.func, "N": N, "results": res}),
          flush=True)


_WS = {}
_OPTS = {"func": None, "adaptive": False}


def _value16(prec: str) -> bool:
    """16-bit value uniforms for this operand precision (--value-bits)."""
    vb = _OPTS.get("value_bits", "auto")
    return vb == "16" or (vb == "auto" and prec in ("bf16", "fp8"))


def _func_of(name):
    from paper_1904_00429_amd import Func
    return {"identity": None, "abs_step": Func.abs_step(2.0), "inv_abs_step": Func.inv_abs_step(0.4, 0.01)}[name]


def _inner(api, wl, x, prec, dev, want_timing, seed):
    import torch
    key = ("inner", prec)
    if key not in _WS:
        _WS[key] = (torch.empty(1 << 20, dtype=torch.uint8, device=dev), torch.empty((), dtype=torch.float64, device=dev))
    ws, out = _WS[key]
    return _call_inner(api, wl, x, prec, dev, ws, out, want_timing, seed)


def _call_inner(api, wl, x, prec, dev, ws, out, want_timing, seed):
    import ctypes
    h = api._LevelsHolder(wl.c, None, wl.rmse_target, wl.pilot, seed, prec, False, 0, 0, _OPTS["func"],
                          _OPTS["adaptive"], index_word32=_OPTS.get("index_word32", False))
    if want_timing:
        h.lv.flags |= 2
    lib = api.lib()
    need = int(lib.mlmc_inner_product_workspace_size(wl.n, ctypes.byref(h.lv)))
    assert ws.numel() >= need
    d = x.c()
    rep = api.Report()
    api.check(lib.mlmc_inner_product_estimate(wl.n, ctypes.byref(d), ctypes.byref(d), ctypes.byref(h.lv),
                                              out.data_ptr(), None, ws.data_ptr(), ws.numel(), ctypes.byref(rep),
                                              api._stream(dev)))
    return _Rep(out.clone(), rep, len(wl.c))


def _inner_graph(api, wl, x, prec, dev, steps, warmup):
    """The inner-product estimate (seed 0) captured into one hipGraph and
    replayed back to back (mlmc_inner_product_graph_create): no host
    synchronisation or kernel-timing events between estimates, one graph
    launch per estimate."""
    import torch
    g = api.InnerProductGraph(wl.n, x, x, wl.c, rmse_target=wl.rmse_target, pilot=wl.pilot, seed=0, prec=prec,
                              device=dev, func=_OPTS["func"], index_word32=_OPTS.get("index_word32", False))
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    rep = g.report()
    g.release()
    return {"s_per_estimate": sec, "estimates_per_s": 1.0 / sec, "n_used": rep.n_used, "rmse_est": rep.rmse_est,
            "note": "replays of one captured estimate (fixed seed); the headline value is the direct call "
                    "with a new seed per step and kernel-timing events"}


def _matmul(api, wl, a, prec, dev, want_timing, seed):
    import ctypes
    import torch
    h = api._LevelsHolder(wl.c, wl.n_samples, wl.rmse_target if wl.n_samples is None else 0.0,
                          wl.pilot, seed, prec, False, 0, 0, _OPTS["func"],
                          _OPTS["adaptive"] and wl.n_samples is None, value16=_value16(prec))
    if want_timing:
        h.lv.flags |= 2
    lib = api.lib()
    need = int(lib.mlmc_matmul_workspace_size(wl.m, wl.n, wl.p, ctypes.byref(h.lv)))
    key = ("matmul", wl.name, prec)
    if key not in _WS:
        _WS[key] = (torch.empty(need, dtype=torch.uint8, device=dev),
                    torch.empty((wl.m, wl.p), dtype=torch.float64, device=dev))
    ws, out = _WS[key]
    d = a.c()
    rep = api.Report()
    api.check(lib.mlmc_matmul_estimate(wl.m, wl.n, wl.p, ctypes.byref(d), ctypes.byref(d), ctypes.byref(h.lv),
                                       out.data_ptr(), None, ws.data_ptr(), ws.numel(), ctypes.byref(rep),
                                       api._stream(dev)))
    return _Rep(out.clone(), rep, len(wl.c))


class _Rep:
    def __init__(self, Y, rep, L1):
        self.Y = Y
        self.n_used = [int(rep.n_used[l]) for l in range(L1)]
        self.level_var = [float(rep.level_var[l]) for l in range(L1)]
        self.rmse_est = float(rep.rmse_est)
        self.total_draws = int(rep.total_draws)
        self.kernel_ms = [float(rep.kernel_ms[i]) for i in range(4)]
        self.kernel_launches = [int(rep.kernel_launches[i]) for i in range(4)]
        self.levels_used = int(rep.levels_used)
        self.bias_test_passed = bool(rep.bias_test_passed)


if __name__ == "__main__":
    main()
