"""torch.autograd.Function over the MLMC matrix estimator with reparameterised
laws A = M_A + S_A o Z, B = M_B + S_B o W: the forward is
mlmc_matmul_estimate, the backward the hand-written adjoint
(mlmc_matmul_adjoint_reparam), which regenerates the forward's indices and
normals from the seed instead of storing them."""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from .mlmc import Law, matmul_adjoint_reparam, matmul_estimate


class MLMCMatmul(torch.autograd.Function):
    @staticmethod
    def forward(ctx, MA, SA, MB, SB, c, n_samples, seed, prec, problem, index_weights, coupling, value16):
        n, m = MA.shape
        p = MB.shape[1]
        res = matmul_estimate(m, n, p, Law.reparam(MA.detach(), SA.detach()),
                              Law.reparam(MB.detach(), SB.detach()), list(c),
                              n_samples=list(n_samples), seed=seed, prec=prec, problem=problem,
                              report=False, device=MA.device, index_weights=index_weights, coupling=coupling,
                              value16=value16)
        ctx.save_for_backward(MA, SA, MB, SB)
        ctx.cfg = (list(c), list(n_samples), seed, problem, prec, index_weights, coupling, value16)
        return res.Y

    @staticmethod
    def backward(ctx, grad_out):
        MA, SA, MB, SB = ctx.saved_tensors
        c, n_samples, seed, problem, prec, index_weights, coupling, value16 = ctx.cfg
        # a BF16 forward gets the BF16-operand adjoint; every other form the FP32 one
        dMA, dSA, dMB, dSB = matmul_adjoint_reparam(MA.detach(), SA.detach(), MB.detach(), SB.detach(),
                                                    c, n_samples, grad_out, seed=seed, problem=problem,
                                                    prec="bf16" if prec == "bf16" else "fp32",
                                                    index_weights=index_weights, coupling=coupling,
                                                    value16=value16)
        # the index weights are inputs of the estimator, held fixed: the
        # gradient is that of the estimate at the given xi (its mean, E[AB],
        # does not depend on xi)
        return dMA, dSA, dMB, dSB, None, None, None, None, None, None, None, None


def mlmc_matmul(MA: torch.Tensor, SA: torch.Tensor, MB: torch.Tensor, SB: torch.Tensor,
                c: Sequence[int], n_samples: Sequence[int], seed: int = 0, prec: str = "fp32",
                problem: int = 0, index_weights: Optional[torch.Tensor] = None,
                coupling: str = "prefix", value16: bool = False) -> torch.Tensor:
    """Differentiable MLMC estimate of E[AB] (m x p, FP64).  MA, SA: (n, m) FP32
    device tensors (row j = column j of A); MB, SB: (n, p).  index_weights:
    optional int32 device weights of the index draws (held fixed); coupling:
    "prefix" or "stride"; value16: values from 16-bit uniforms."""
    return MLMCMatmul.apply(MA, SA, MB, SB, tuple(c), tuple(n_samples), seed, prec, problem, index_weights,
                            coupling, value16)
