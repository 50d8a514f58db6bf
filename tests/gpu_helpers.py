"""Shared helpers of the GPU parity tests: the same law description is turned
into the oracle's law and the binding's law (inputs only, no arithmetic)."""
import sys

import numpy as np


def flush(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def laws(orc, desc, device, mean=None, stdev=None):
    """desc: ("normal"|"uniform", loc, scale) or ("reparam",) with FP32 numpy
    mean/stdev in the binding's layout ((n, m) for A, (n, p) for B)."""
    import torch
    from paper_1904_00429_amd import Law
    if desc[0] == "normal":
        return orc.Law.normal(desc[1], desc[2]), Law.normal(desc[1], desc[2])
    if desc[0] == "uniform":
        return orc.Law.uniform(desc[1], desc[2]), Law.uniform(desc[1], desc[2])
    mean = np.ascontiguousarray(mean, dtype=np.float32)
    stdev = np.ascontiguousarray(stdev, dtype=np.float32)
    ld = mean.shape[1] if mean.ndim == 2 else 1
    o = orc.Law.reparam(mean.astype(np.float64).ravel(), stdev.astype(np.float64).ravel(), ld)
    g = Law.reparam(torch.from_numpy(mean).to(device), torch.from_numpy(stdev).to(device))
    return o, g


def rel_frob(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


# ----------------------------------------------------------------------------
# Parity tolerances, in one place.
#
# FP64 / FP32 paths against the FP64 oracle (relative Frobenius):
#   Y and the level-0 mean: TOL (1e-12 / 1e-5);
#   level means l >= 1 (about 0): ||dYbar_l|| <= TOL sqrt(V_l);
#   V_l and RMSE_est: relative VTOL (1e-10 / 1e-5).
#   A level whose oracle variance is itself rounding (D_l = 0 in exact
#   arithmetic: n = 1, or every draw the same column) has no spread to measure
#   against: its mean is held to TOL ||Y|| and its V_l to (TOL ||Y||)^2.
# BF16 / FP8 paths:
#   against the oracle reading the same rounded operands (operand_law), the
#   only difference left is FP32 accumulation and the rare value whose FP32
#   evaluation lands on the other side of a rounding boundary: ||dY||_F at
#   QTOL (||Y||_F + RMSE_est), level means at QTOL sqrt(V_l), V_l at QTOL
#   relative;
#   against the exact FP64 oracle (the rounding error of the precision form,
#   reported next to the sampling error): ||dY||_F <= FROB_RMSE RMSE_est and
#   every entry |dY_iq| <= ENTRY_SD sd_iq (the estimator's own standard
#   deviation there), V_l within VREL.
# ----------------------------------------------------------------------------
TOL = {"fp64": 1e-12, "fp32": 1e-5}
VTOL = {"fp64": 1e-10, "fp32": 1e-5}
DEGENERATE = 1e-10          # V_l <= (DEGENERATE ||Y||)^2: rounding only
QTOL = {"bf16": 1e-4, "fp8": 1e-4}
FROB_RMSE = {"bf16": 0.05, "fp8": 0.25}
ENTRY_SD = {"bf16": 0.1, "fp8": 0.75}
VREL = {"bf16": 3e-2, "fp8": 0.15}


def operand_law(orc, law, prec, count, side):
    """The oracle's law read by the contraction in the operand format of
    `prec` (count: m for A's rows, p for B's columns)."""
    if prec == "bf16":
        return law.with_operand(orc.OPERAND_BF16)
    if prec == "fp8":
        return law.with_operand(orc.OPERAND_FP8_E4M3, orc.fp8_scale_exponents(law, count, side))
    return law


def _levels_close(means, ref_means, V, ref_V, ynorm, tol, vtol, what):
    for l in range(len(ref_V)):
        d = float(np.linalg.norm((means[l] - ref_means[l]).ravel()))
        degenerate = ref_V[l] <= (DEGENERATE * ynorm) ** 2
        if l == 0 and not degenerate:
            bound = tol * max(float(np.linalg.norm(ref_means[0].ravel())), 1e-300)
        elif degenerate:
            bound = tol * ynorm
        else:
            bound = tol * np.sqrt(ref_V[l])
        assert d <= bound, (what, "level mean", l, d, bound)
        if degenerate:
            assert abs(V[l] - ref_V[l]) <= (tol * ynorm) ** 2, (what, "V", l, V[l], ref_V[l])
        else:
            assert abs(V[l] - ref_V[l]) <= vtol * ref_V[l], (what, "V", l, V[l], ref_V[l],
                                                             abs(V[l] / ref_V[l] - 1))


def check_estimate(est, ref, prec, ref_q=None, label=""):
    """Parity of a GPU estimate with the oracle's (same N_l) at the tolerances
    above; ref_q: the oracle on the rounded operands (BF16 / FP8)."""
    Y = est.Y.cpu().numpy().reshape(ref.Y.shape)
    V = np.asarray(est.level_var, dtype=np.float64)
    means = None if est.level_means is None else est.level_means.cpu().numpy().reshape(ref.level_means.shape)
    assert list(est.n_used) == list(ref.n_used), (label, est.n_used, ref.n_used)
    ynorm = float(np.linalg.norm(ref.Y.ravel()))
    if prec in TOL:
        tol, vtol = TOL[prec], VTOL[prec]
        r = rel_frob(Y, ref.Y)
        flush(f"  {label} {prec}: rel err {r:.3g}")
        assert r <= tol, (label, r)
        if means is not None:
            _levels_close(means, ref.level_means, V, ref.level_var, ynorm, tol, vtol, label)
        else:
            np.testing.assert_allclose(V, ref.level_var, rtol=vtol, atol=(tol * ynorm) ** 2)
        assert abs(est.rmse_est - ref.rmse_est) <= vtol * ref.rmse_est + tol * ynorm
        return
    # rounding error of the precision form against the exact oracle
    err = float(np.linalg.norm((Y - ref.Y).ravel()))
    sd = ref.entry_sd
    worst = float(np.max(np.abs(Y - ref.Y) / np.maximum(sd, 1e-300)))
    flush(f"  {label} {prec}: |Y - Y_fp64| = {err:.4g} = {err / ref.rmse_est:.3g} RMSE_est; "
          f"max entry |dY| / sd = {worst:.3g}")
    assert err <= FROB_RMSE[prec] * ref.rmse_est, (label, err, ref.rmse_est)
    assert worst <= ENTRY_SD[prec], (label, worst)
    np.testing.assert_allclose(V, ref.level_var, rtol=VREL[prec])
    if ref_q is not None:
        # against the estimate's size plus its sampling error: a product whose
        # mean is small against its spread is not held to a relative bound on
        # a near-zero mean
        rq = float(np.linalg.norm((Y - ref_q.Y).ravel())) / (float(np.linalg.norm(ref_q.Y.ravel())) + ref_q.rmse_est)
        flush(f"  {label} {prec}: rel err vs rounded-operand oracle {rq:.3g}")
        assert rq <= QTOL[prec], (label, rq)
        if means is not None:
            _levels_close(means, ref_q.level_means, V, ref_q.level_var, float(np.linalg.norm(ref_q.Y.ravel())),
                          QTOL[prec], QTOL[prec], label + " (rounded operands)")
