"""Gradient reference for the reparameterised matrix estimator (test
infrastructure only).

The estimate of Alg. 1 / eq. (10) is rewritten with plain PyTorch CPU FP64
operations on the same index draws and standard normals as the C oracle
(taken from it), so torch's autograd gives the exact gradient of
<G, Y> with respect to the means and scales at a fixed seed.  Pinned to the
C oracle's forward and to finite differences in the tests."""
from __future__ import annotations

from typing import Sequence

import numpy as np
import torch

from . import Law, column, coupling_stride, draw_index_weighted, draw_indices, level_field


def standard_normals(seed, problem, lfield, k, cols, m, p, value16=False):
    """z (len(cols) x m) and w (len(cols) x p) of the draws of realisation k
    (value16: the 16-bit value uniforms)."""
    unit = Law.normal(0.0, 1.0)
    if value16:
        unit = unit.with_value16()
    Z = np.empty((len(cols), m))
    W = np.empty((len(cols), p))
    for t, j in enumerate(cols):
        Z[t], W[t] = column(seed, problem, lfield, k, int(j), m, p, unit, unit)
    return torch.from_numpy(Z), torch.from_numpy(W)


def reparam_estimate(MA: torch.Tensor, SA: torch.Tensor, MB: torch.Tensor, SB: torch.Tensor,
                     c: Sequence[int], N: Sequence[int], seed: int = 0, problem: int = 0,
                     shared: bool = False, weights=None, coupling: str = "prefix",
                     value16: bool = False) -> torch.Tensor:
    """Y = sum_l (1/N_l) sum_k (Z_l^(k) - Z_{l-1}^(k)) for A = MA^T + SA^T o Z
    (MA, SA: n x m, row j = column j of A) and B = MB + SB o W (n x p).  With
    `weights` (oracle.Weights) the indices are drawn with xi_j = w_j / W and
    Z_l = (1/c_l) sum_t a_t b_t^T / xi_{r_t} (eq. (18)).  coupling "stride": the
    coarse sketch takes draws M - 1, 2M - 1, ... (M = c_l / c_{l-1})."""
    n, m = MA.shape
    p = MB.shape[1]
    Y = torch.zeros((m, p), dtype=torch.float64)
    for l, (cl, Nl) in enumerate(zip(c, N)):
        cp = c[l - 1] if l > 0 else 0
        lf = level_field(l, shared)
        M = coupling_stride(cl, cp, coupling)
        ci = torch.arange(cp) if M == 0 else M * (torch.arange(cp) + 1) - 1   # coarse draws
        acc = torch.zeros((m, p), dtype=torch.float64)
        for k in range(Nl):
            if weights is None:
                r = draw_indices(seed, problem, lf, k, cl, n)
            else:
                r = np.array([draw_index_weighted(seed, problem, lf, k, t, weights) for t in range(cl)],
                             dtype=np.int64)
            Z, W = standard_normals(seed, problem, lf, k, r, m, p, value16)
            idx = torch.from_numpy(r)
            AS = MA[idx] + SA[idx] * Z          # c x m: row t = a_t
            BS = MB[idx] + SB[idx] * W          # c x p: row t = b_t
            if weights is None:
                Zf = (n / cl) * (AS.T @ BS)
                Zc = (n / cp) * (AS[ci].T @ BS[ci]) if cp > 0 else None
            else:
                f = torch.from_numpy(weights.total / weights.w[r].astype(np.float64))[:, None]
                Zf = ((AS * f).T @ BS) / cl
                Zc = ((AS[ci] * f[ci]).T @ BS[ci]) / cp if cp > 0 else None
            acc = acc + (Zf - Zc if Zc is not None else Zf)
        Y = Y + acc / Nl
    return Y


def reparam_gradients(MA, SA, MB, SB, c, N, G, seed=0, problem=0, shared=False, weights=None,
                      coupling="prefix", value16=False):
    """Gradients of <G, Y> (FP64) with respect to MA, SA, MB, SB (weights held fixed)."""
    leaves = [torch.as_tensor(np.asarray(x, dtype=np.float64)).clone().requires_grad_(True)
              for x in (MA, SA, MB, SB)]
    Y = reparam_estimate(*leaves, c, N, seed, problem, shared, weights, coupling, value16)
    (Y * torch.as_tensor(np.asarray(G, dtype=np.float64))).sum().backward()
    return Y.detach().numpy(), [t.grad.numpy() for t in leaves]


def reparam_gradients_at(MA, SA, MB, SB, c, N, G, cols, seed=0, problem=0, coupling="prefix", value16=False):
    """The same gradients restricted to the rows `cols` of MA, SA, MB, SB
    (columns j of A and rows j of B), for products whose full gradient the
    CPU cannot afford.

    Only the terms a_t b_t^T whose draw r_t is one of `cols` depend on those
    rows, so <G, Y> restricted to them has the same gradient there: every
    index of every realisation is drawn (as reparam_estimate does), and only
    the hit draws' columns are generated and entered into the restricted
    objective sum_l (1/N_l) sum_k <G, Z_l^hits - Z_{l-1}^hits>.  Returns the
    four gradients as arrays of shape (len(cols), m) and (len(cols), p)."""
    cols = [int(j) for j in cols]
    n, m = np.asarray(MA).shape
    p = np.asarray(MB).shape[1]
    pos = {j: i for i, j in enumerate(cols)}
    J = torch.tensor(cols)
    leaves = [torch.as_tensor(np.asarray(x, dtype=np.float64))[J].clone().requires_grad_(True)
              for x in (MA, SA, MB, SB)]
    mA, sA, mB, sB = leaves
    Gt = torch.as_tensor(np.asarray(G, dtype=np.float64))
    obj = torch.zeros((), dtype=torch.float64)
    for l, (cl, Nl) in enumerate(zip(c, N)):
        cp = c[l - 1] if l > 0 else 0
        M = coupling_stride(cl, cp, coupling)
        coarse = set(range(cp)) if M == 0 else {M * (i + 1) - 1 for i in range(cp)}
        lf = level_field(l, False)
        for k in range(Nl):
            r = draw_indices(seed, problem, lf, k, cl, n)
            hits = [t for t in range(cl) if int(r[t]) in pos]
            if not hits:
                continue
            Z, W = standard_normals(seed, problem, lf, k, r[hits], m, p, value16)
            idx = torch.tensor([pos[int(r[t])] for t in hits])
            a = mA[idx] + sA[idx] * Z            # hit draws' a_t
            b = mB[idx] + sB[idx] * W            # and b_t
            wt = torch.tensor([n / cl - (n / cp if t in coarse else 0.0) for t in hits], dtype=torch.float64)
            # <G, sum_t w_t a_t b_t^T> = sum_t w_t a_t^T G b_t
            obj = obj + ((a @ Gt) * b).sum(dim=1).mul(wt).sum() / Nl
    obj.backward()
    return [t.grad.numpy() if t.grad is not None else np.zeros(tuple(t.shape)) for t in leaves]
