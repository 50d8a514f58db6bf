"""Python binding of libmlmc (include/mlmc.h): argument marshalling only.

Every step of the estimator runs in the HIP kernels of libmlmc.so; PyTorch
only provides device memory (outputs, workspace, reparameterised inputs) and
the stream the work is enqueued on.  There is no CPU fallback: calling into a
missing library raises.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

from ._lib import Dist, Levels, MLMCError, Problem, Report, Tuning, check, lib

PREC = {"fp64": 0, "fp32": 1, "bf16": 2, "fp8": 3}
FLAG_SHARED_SAMPLES = 1
FLAG_STRIDE_COUPLING = 8
FLAG_INDEX_WORD32 = 16
FLAG_VALUE16 = 32
FLAG_SET_FORM = 64
COUPLINGS = ("prefix", "stride")   # coarse draws: the first c_{l-1}, or every M-th (Sec. 3.1)
FLAG_ADAPTIVE_LEVELS = 4
SHARED_LEVEL_FIELD = 0xFF


@dataclass
class Law:
    """Entry law of A (m x n), B (n x p), x or y (length n).

    normal: loc + scale N(0, 1); uniform: loc + scale U(-1, 1);
    reparam: mean + stdev N(0, 1), entrywise, with FP32 device tensors of shape
    (n, m) for A (row j = column j of A, i.e. A stored column-major),
    (n, p) for B (row-major), (n,) for x and y.
    The laws of the experiments of Sec. 4 (both operands take one of them, or
    neither does; column j counted from 1, K ~ Poisson, E ~ Exp(1)):
    ramp_normal (j scale)(loc - z), cos_poisson_exp cos(K + 2E) Bern(beta),
    sin_ramp sin(x) + z' x with x = (j scale)(loc - z), cos_poisson_step
    cos(K) H(5 - K) Bern(beta)."""
    kind: int
    loc: float = 0.0
    scale: float = 1.0
    mean: Optional[torch.Tensor] = None
    stdev: Optional[torch.Tensor] = None

    @staticmethod
    def normal(loc: float, scale: float) -> "Law":
        return Law(0, float(loc), float(scale))

    @staticmethod
    def uniform(loc: float, scale: float) -> "Law":
        return Law(1, float(loc), float(scale))

    @staticmethod
    def ramp_normal(scale: float, loc: float) -> "Law":
        """(j scale)(loc - N(0, 1)); Sec. 4.1's x: ramp_normal(1 / 50, 0.4)."""
        return Law(3, float(loc), float(scale))

    @staticmethod
    def cos_poisson_exp(lam: float, beta: float) -> "Law":
        """cos(Poi(lam) + 2 Exp(1)) Bern(beta); Sec. 4.1's y: cos_poisson_exp(10, 0.05)."""
        return Law(4, float(lam), float(beta))

    @staticmethod
    def sin_ramp(scale: float, loc: float) -> "Law":
        """sin(x) + N(0, 1) x, x = (j scale)(loc - N(0, 1)); Sec. 4.2's A: sin_ramp(1e-4, 0.5)."""
        return Law(5, float(loc), float(scale))

    @staticmethod
    def cos_poisson_step(lam: float, beta: float) -> "Law":
        """cos(K) H(5 - K) Bern(beta), K ~ Poi(lam); Sec. 4.2's B: cos_poisson_step(2, 0.2)."""
        return Law(6, float(lam), float(beta))

    @staticmethod
    def reparam(mean: torch.Tensor, stdev: torch.Tensor) -> "Law":
        if mean.dtype != torch.float32 or stdev.dtype != torch.float32:
            raise TypeError("reparam mean/stdev must be float32")
        if mean.shape != stdev.shape or not mean.is_contiguous() or not stdev.is_contiguous():
            raise ValueError("reparam mean/stdev must be contiguous and of the same shape")
        if not mean.is_cuda:
            raise ValueError("reparam mean/stdev must be device tensors")
        return Law(2, 0.0, 0.0, mean, stdev)

    def c(self) -> Dist:
        d = Dist()
        d.law = self.kind
        d.loc = self.loc
        d.scale = self.scale
        if self.kind == 2:
            d.mean = self.mean.data_ptr()
            d.stdev = self.stdev.data_ptr()
            d.ld = self.mean.shape[1] if self.mean.dim() == 2 else 1
        return d


@dataclass
class Func:
    """Target function f of E[f(AB)] (mlmc_func), applied entrywise to both
    sketches of every realisation: identity; abs_step f(x) = |x| H(theta0 - x);
    inv_abs_step f(x) = 1 / (|x| H(x + theta0) + theta1); H(0) = 1."""
    kind: int = 0
    theta0: float = 0.0
    theta1: float = 0.0

    @staticmethod
    def identity() -> "Func":
        return Func()

    @staticmethod
    def abs_step(theta0: float = 2.0) -> "Func":
        return Func(1, float(theta0), 0.0)

    @staticmethod
    def inv_abs_step(theta0: float = 0.4, theta1: float = 0.01) -> "Func":
        return Func(2, float(theta0), float(theta1))


@dataclass
class Result:
    Y: torch.Tensor                        # m x p (or scalar) FP64 on the device
    level_means: Optional[torch.Tensor]    # (L+1) x m x p, if requested
    n_used: list
    level_var: list
    rmse_est: float
    total_draws: int
    levels_used: int = 0                   # levels run (all unless adaptive)
    bias_test_passed: bool = True          # adaptive: stopped on the bias test


class _LevelsHolder:
    """Keeps the ctypes arrays of a Levels struct alive."""

    def __init__(self, c, n_samples, rmse_target, pilot, seed, prec, shared, problem, max_total_draws,
                 func: Optional[Func] = None, adaptive: bool = False,
                 index_weights: Optional[torch.Tensor] = None, coupling: str = "prefix",
                 index_word32: bool = False, value16: bool = False, set_form: bool = False):
        if prec not in PREC:
            raise ValueError(f"prec must be one of {sorted(PREC)}")
        if coupling not in COUPLINGS:
            raise ValueError(f"coupling must be one of {COUPLINGS}")
        self.c = (ctypes.c_int64 * len(c))(*[int(v) for v in c])
        self.n = None if n_samples is None else (ctypes.c_int64 * len(n_samples))(*[int(v) for v in n_samples])
        lv = Levels()
        lv.num_levels = len(c)
        lv.c = ctypes.cast(self.c, ctypes.POINTER(ctypes.c_int64))
        lv.n_samples = ctypes.cast(self.n, ctypes.POINTER(ctypes.c_int64)) if self.n is not None else None
        lv.rmse_target = float(rmse_target)
        lv.pilot_samples = int(pilot)
        lv.max_total_draws = int(max_total_draws)
        lv.seed = int(seed) & (2**64 - 1)
        lv.prec = PREC[prec]
        lv.flags = ((FLAG_SHARED_SAMPLES if shared else 0) | (FLAG_ADAPTIVE_LEVELS if adaptive else 0)
                    | (FLAG_STRIDE_COUPLING if coupling == "stride" else 0)
                    | (FLAG_INDEX_WORD32 if index_word32 else 0)
                    | (FLAG_VALUE16 if value16 else 0) | (FLAG_SET_FORM if set_form else 0))
        lv.problem = int(problem)
        f = func or Func()
        lv.func = int(f.kind)
        lv.func_param[0] = float(f.theta0)
        lv.func_param[1] = float(f.theta1)
        if index_weights is not None:
            if index_weights.dtype != torch.int32 or not index_weights.is_cuda or not index_weights.is_contiguous():
                raise TypeError("index_weights must be a contiguous int32 device tensor of positive weights")
            lv.index_weights = index_weights.data_ptr()
        self.index_weights = index_weights
        self.lv = lv


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _result(Y, means, rep: Report, num_levels: int) -> Result:
    return Result(Y, means, [int(rep.n_used[l]) for l in range(num_levels)],
                  [float(rep.level_var[l]) for l in range(num_levels)], float(rep.rmse_est),
                  int(rep.total_draws), int(rep.levels_used), bool(rep.bias_test_passed))


def matmul_workspace_size(m, n, p, c, prec="fp64", n_samples=None, rmse_target=0.0, pilot=0,
                          func: Optional[Func] = None) -> int:
    h = _LevelsHolder(c, n_samples, rmse_target, pilot, 0, prec, False, 0, 0, func)
    return int(lib().mlmc_matmul_workspace_size(int(m), int(n), int(p), ctypes.byref(h.lv)))


def matmul_estimate(m: int, n: int, p: int, A: Law, B: Law, c: Sequence[int],
                    n_samples: Optional[Sequence[int]] = None, rmse_target: float = 0.0,
                    pilot: int = 0, seed: int = 0, prec: str = "fp64", shared: bool = False,
                    problem: int = 0, max_total_draws: int = 0, level_means: bool = False,
                    report: bool = True, device=None, workspace: Optional[torch.Tensor] = None,
                    out: Optional[torch.Tensor] = None, func: Optional[Func] = None,
                    adaptive: bool = False, index_weights: Optional[torch.Tensor] = None,
                    coupling: str = "prefix", value16: bool = False, set_form: bool = False) -> Result:
    """MLMC estimate of E[f(AB)] on the GPU (mlmc_matmul_estimate; f = identity
    unless func is given; adaptive: number of levels chosen by the bias test,
    c being the longest ladder allowed; index_weights: int32 device tensor of n
    positive weights, xi_j = w_j / sum w, e.g. optimal_index_weights;
    coupling: "prefix" or "stride", the coarse draws of each level sample;
    value16: values from 16-bit uniforms, eight per Philox call; set_form:
    each realisation's index tuple as a set with multiplicities)."""
    device = torch.device(device or "cuda")
    h = _LevelsHolder(c, n_samples, rmse_target, pilot, seed, prec, shared, problem, max_total_draws, func,
                      adaptive, index_weights, coupling, value16=value16, set_form=set_form)
    ws_bytes = int(lib().mlmc_matmul_workspace_size(int(m), int(n), int(p), ctypes.byref(h.lv)))
    if ws_bytes == 0:
        raise MLMCError(1, "invalid problem: no workspace size")
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=device)
    if out is None:
        out = torch.empty((m, p), dtype=torch.float64, device=device)
    means = torch.empty((len(c), m, p), dtype=torch.float64, device=device) if level_means else None
    da, db = A.c(), B.c()
    rep = Report()
    check(lib().mlmc_matmul_estimate(int(m), int(n), int(p), ctypes.byref(da), ctypes.byref(db),
                                     ctypes.byref(h.lv), out.data_ptr(),
                                     means.data_ptr() if means is not None else None,
                                     workspace.data_ptr(), ws_bytes,
                                     ctypes.byref(rep) if report else None, _stream(device)))
    return _result(out, means, rep, len(c))


def inner_product_estimate(n: int, x: Law, y: Law, c: Sequence[int],
                           n_samples: Optional[Sequence[int]] = None, rmse_target: float = 0.0,
                           pilot: int = 0, seed: int = 0, prec: str = "fp64", shared: bool = False,
                           problem: int = 0, max_total_draws: int = 0, level_means: bool = False,
                           report: bool = True, device=None,
                           workspace: Optional[torch.Tensor] = None,
                           out: Optional[torch.Tensor] = None, func: Optional[Func] = None,
                           adaptive: bool = False, index_weights: Optional[torch.Tensor] = None,
                           coupling: str = "prefix", index_word32: bool = False) -> Result:
    """MLMC estimate of E[f(x^T y)] on the GPU (mlmc_inner_product_estimate;
    f = identity unless func is given; adaptive, index_weights and coupling
    as for matmul_estimate; index_word32: four index draws per Philox call
    from 32-bit words, for power-of-two n)."""
    device = torch.device(device or "cuda")
    h = _LevelsHolder(c, n_samples, rmse_target, pilot, seed, prec, shared, problem, max_total_draws, func,
                      adaptive, index_weights, coupling, index_word32)
    ws_bytes = int(lib().mlmc_inner_product_workspace_size(int(n), ctypes.byref(h.lv)))
    if ws_bytes == 0:
        raise MLMCError(1, "invalid problem: no workspace size")
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=device)
    if out is None:
        out = torch.empty((), dtype=torch.float64, device=device)
    means = torch.empty((len(c),), dtype=torch.float64, device=device) if level_means else None
    dx, dy = x.c(), y.c()
    rep = Report()
    check(lib().mlmc_inner_product_estimate(int(n), ctypes.byref(dx), ctypes.byref(dy),
                                            ctypes.byref(h.lv), out.data_ptr(),
                                            means.data_ptr() if means is not None else None,
                                            workspace.data_ptr(), ws_bytes,
                                            ctypes.byref(rep) if report else None, _stream(device)))
    return _result(out, means, rep, len(c))


def inner_product_estimate_noalloc(n: int, x: Law, y: Law, c: Sequence[int],
                                   n_samples: Optional[Sequence[int]] = None, rmse_target: float = 0.0,
                                   pilot: int = 0, seed: int = 0, prec: str = "fp64", out: torch.Tensor = None,
                                   level_means: Optional[torch.Tensor] = None, report: bool = True,
                                   func: Optional[Func] = None, adaptive: bool = False,
                                   index_weights: Optional[torch.Tensor] = None, coupling: str = "prefix",
                                   index_word32: bool = False) -> Result:
    """mlmc_inner_product_estimate_noalloc: the inner-product estimate with
    the library's fixed per-GPU scratch array as its workspace.  The caller
    passes the output (a device FP64 scalar) and, optionally, the level-means
    vector; nothing is allocated here."""
    if out is None:
        raise ValueError("out (a device FP64 scalar tensor) is required")
    h = _LevelsHolder(c, n_samples, rmse_target, pilot, seed, prec, False, 0, 0, func,
                      adaptive, index_weights, coupling, index_word32)
    dx, dy = x.c(), y.c()
    rep = Report()
    check(lib().mlmc_inner_product_estimate_noalloc(int(n), ctypes.byref(dx), ctypes.byref(dy),
                                                    ctypes.byref(h.lv), out.data_ptr(),
                                                    level_means.data_ptr() if level_means is not None else None,
                                                    ctypes.byref(rep) if report else None, _stream(out.device)))
    return _result(out, level_means, rep, len(c))


class InnerProductGraph:
    """One inner-product estimate (fixed N_l, or target mode with eq. (28) on
    the device) captured into a hipGraph (mlmc_inner_product_graph_create)
    and replayed on the current stream; after a replay `out` (and `means`)
    hold the estimate, and report() reads V_l, N_l and the schedule's status
    (mlmc_inner_product_graph_report, which synchronises the stream)."""

    def __init__(self, n: int, x: Law, y: Law, c: Sequence[int], n_samples: Optional[Sequence[int]] = None,
                 rmse_target: float = 0.0, pilot: int = 0, seed: int = 0, prec: str = "fp64",
                 max_total_draws: int = 0, level_means: bool = False, device=None, func: Optional[Func] = None,
                 index_weights: Optional[torch.Tensor] = None, coupling: str = "prefix",
                 index_word32: bool = False, stream: Optional[torch.cuda.Stream] = None):
        self.device = torch.device(device or "cuda")
        self.n = int(n)
        self.num_levels = len(c)
        self.h = _LevelsHolder(c, n_samples, rmse_target, pilot, seed, prec, False, 0, max_total_draws, func,
                               False, index_weights, coupling, index_word32)
        self.ws_bytes = int(lib().mlmc_inner_product_workspace_size(self.n, ctypes.byref(self.h.lv)))
        if self.ws_bytes == 0:
            raise MLMCError(1, "invalid problem: no workspace size")
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.out = torch.empty((), dtype=torch.float64, device=self.device)
        self.means = torch.empty((len(c),), dtype=torch.float64, device=self.device) if level_means else None
        self._dx, self._dy = x.c(), y.c()
        self.graph = None
        stream = stream or torch.cuda.Stream(device=self.device)
        handle = ctypes.c_void_p()
        check(lib().mlmc_inner_product_graph_create(self.n, ctypes.byref(self._dx), ctypes.byref(self._dy),
                                                    ctypes.byref(self.h.lv), self.out.data_ptr(),
                                                    self.means.data_ptr() if self.means is not None else None,
                                                    self.workspace.data_ptr(), self.ws_bytes, stream.cuda_stream,
                                                    ctypes.byref(handle)))
        self.graph = handle

    def replay(self):
        """Launch the captured estimate on the current stream."""
        if self.graph is None:
            raise RuntimeError("the graph has been released")
        check(lib().mlmc_graph_launch(self.graph, _stream(self.device)))

    def report(self) -> Result:
        """N_l, V_l and the RMSE estimate of the last replay; raises the
        schedule's status (EBUDGET) like the direct call."""
        rep = Report()
        check(lib().mlmc_inner_product_graph_report(self.n, ctypes.byref(self.h.lv), self.workspace.data_ptr(),
                                                    self.ws_bytes, ctypes.byref(rep), _stream(self.device)))
        return _result(self.out, self.means, rep, self.num_levels)

    def release(self):
        if self.graph is not None:
            check(lib().mlmc_graph_destroy(self.graph))
            self.graph = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


def philox(ctr: torch.Tensor, seed: int) -> torch.Tensor:
    """Philox4x32-10 of device counters (count x 4, int32 holding uint32 bits)."""
    ctr = ctr.contiguous()
    out = torch.empty_like(ctr)
    check(lib().mlmc_philox4x32_10(ctr.shape[0], ctr.data_ptr(), int(seed) & (2**64 - 1),
                                   out.data_ptr(), _stream(ctr.device)))
    return out


def sample_indices(seed: int, problem: int, level_field: int, k0: int, num_samples: int,
                   c: int, n: int, device=None) -> torch.Tensor:
    device = torch.device(device or "cuda")
    out = torch.empty((num_samples, c), dtype=torch.int32, device=device)
    check(lib().mlmc_sample_indices(int(seed) & (2**64 - 1), problem, level_field, k0, num_samples,
                                    c, n, out.data_ptr(), _stream(device)))
    return out


def sample_indices_weighted(seed: int, problem: int, level_field: int, k0: int, num_samples: int,
                            c: int, weights: torch.Tensor) -> torch.Tensor:
    """Index draws with probabilities w_j / sum w (mlmc_sample_indices_weighted)."""
    n = weights.numel()
    device = weights.device
    cum = torch.empty(n, dtype=torch.int64, device=device)
    out = torch.empty((num_samples, c), dtype=torch.int32, device=device)
    check(lib().mlmc_sample_indices_weighted(int(seed) & (2**64 - 1), problem, level_field, k0, num_samples, c, n,
                                             weights.data_ptr(), cum.data_ptr(), out.data_ptr(), _stream(device)))
    return out


def optimal_index_weights(m: int, n: int, p: int, A: Law, B: Law, device=None) -> torch.Tensor:
    """Theorem 3.1's xi** as integer weights (mlmc_optimal_index_weights):
    an int32 device tensor of n entries for index_weights."""
    device = torch.device(device or "cuda")
    w = torch.empty(n, dtype=torch.int32, device=device)
    scratch = torch.empty(n + 1, dtype=torch.float64, device=device)
    da, db = A.c(), B.c()
    check(lib().mlmc_optimal_index_weights(int(m), int(n), int(p), ctypes.byref(da), ctypes.byref(db),
                                           w.data_ptr(), scratch.data_ptr(), _stream(device)))
    return w


def gather_columns(m: int, n: int, p: int, A: Law, B: Law, seed: int, problem: int,
                   level_field: int, k0: int, num_samples: int, c: int, prec: str = "fp64",
                   device=None):
    """Sampled columns (num_samples x c x m) and rows (num_samples x c x p), FP64."""
    device = torch.device(device or "cuda")
    AS = torch.empty((num_samples, c, m), dtype=torch.float64, device=device)
    BS = torch.empty((num_samples, c, p), dtype=torch.float64, device=device)
    da, db = A.c(), B.c()
    check(lib().mlmc_gather_columns(m, n, p, ctypes.byref(da), ctypes.byref(db),
                                    int(seed) & (2**64 - 1), problem, level_field, k0, num_samples,
                                    c, PREC[prec], AS.data_ptr(), BS.data_ptr(), _stream(device)))
    return AS, BS


def matmul_adjoint_reparam(MA: torch.Tensor, SA: torch.Tensor, MB: torch.Tensor, SB: torch.Tensor,
                           c: Sequence[int], n_samples: Sequence[int], grad_out: torch.Tensor,
                           seed: int = 0, problem: int = 0, shared: bool = False,
                           workspace: Optional[torch.Tensor] = None, prec: str = "fp32",
                           index_weights: Optional[torch.Tensor] = None, coupling: str = "prefix",
                           value16: bool = False, max_workspace_bytes: Optional[int] = None):
    """Gradients of <grad_out, Y> with respect to M_A, S_A, M_B, S_B
    (mlmc_matmul_adjoint_reparam).  MA, SA: (n, m) FP32 device tensors (row j =
    column j of A); MB, SB: (n, p).  prec: "fp32" or "bf16" (BF16 operands
    on MFMA, FP32 accumulation).  max_workspace_bytes: use at most this much
    workspace (the draws then go in more passes).  Returns (dMA, dSA, dMB,
    dSB), FP32."""
    n, m = MA.shape
    p = MB.shape[1]
    device = MA.device
    A, B = Law.reparam(MA, SA), Law.reparam(MB, SB)
    h = _LevelsHolder(c, n_samples, 0.0, 0, seed, prec, shared, problem, 0, None, False, index_weights, coupling,
                      value16=value16)
    ws_bytes = int(lib().mlmc_matmul_adjoint_workspace_size(int(m), int(n), int(p), ctypes.byref(h.lv)))
    if ws_bytes == 0:
        raise MLMCError(1, "invalid problem: no workspace size")
    if max_workspace_bytes is not None:
        ws_bytes = min(ws_bytes, int(max_workspace_bytes))
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=device)
    g = grad_out.to(device=device, dtype=torch.float64).contiguous()
    grads = [torch.zeros_like(t) for t in (MA, SA, MB, SB)]
    da, db = A.c(), B.c()
    check(lib().mlmc_matmul_adjoint_reparam(int(m), int(n), int(p), ctypes.byref(da), ctypes.byref(db),
                                            ctypes.byref(h.lv), g.data_ptr(), *[t.data_ptr() for t in grads],
                                            workspace.data_ptr(), ws_bytes, _stream(device)))
    return tuple(grads)


# ------------------------------------------------------------------ batching
@dataclass
class BatchProblem:
    """One product of a batched estimate: shapes, laws, Philox stream id."""
    m: int
    n: int
    p: int
    A: Law
    B: Law
    problem: int


class BatchedEstimate:
    """Many independent products through one pipeline (mlmc_matmul_estimate_batched),
    optionally captured once into a hipGraph and replayed.  Outputs live in
    `self.Y` (one m x p FP64 device tensor per product)."""

    def __init__(self, problems: Sequence[BatchProblem], c: Sequence[int], n_samples: Sequence[int],
                 seed: int = 0, prec: str = "fp32", tuning: Optional[dict] = None, device=None,
                 func: Optional[Func] = None, coupling: str = "prefix", value16: bool = False,
                 set_form: bool = False):
        self.device = torch.device(device or "cuda")
        self.problems = list(problems)
        self.h = _LevelsHolder(c, n_samples, 0.0, 0, seed, prec, False, 0, 0, func, coupling=coupling,
                               value16=value16, set_form=set_form)
        self.Y = [torch.empty((pr.m, pr.p), dtype=torch.float64, device=self.device) for pr in self.problems]
        arr = (Problem * len(self.problems))()
        for i, pr in enumerate(self.problems):
            arr[i].m, arr[i].n, arr[i].p = pr.m, pr.n, pr.p
            arr[i].A, arr[i].B = pr.A.c(), pr.B.c()
            arr[i].problem = pr.problem
            arr[i].out = self.Y[i].data_ptr()
            arr[i].level_means = None
        self.table = arr
        self.tuning = Tuning()
        t = tuning or {}
        self.tuning.tile = int(t.get("tile", 0))
        self.tuning.target_blocks = int(t.get("target_blocks", 0))
        self.tuning.gather_budget = int(t.get("gather_budget", 0))
        self.tuning.single_launch = int(t.get("single_launch", 0))
        self.ws_bytes = int(lib().mlmc_matmul_batched_workspace_size(len(arr), arr, ctypes.byref(self.h.lv),
                                                                     ctypes.byref(self.tuning)))
        if self.ws_bytes == 0:
            raise MLMCError(1, lib().mlmc_last_error().decode(errors="replace") or "invalid batch")
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.graph = None
        self.num_levels = len(c)

    def run(self, level_var: bool = False):
        """Enqueue one batched estimate; with level_var, return V_l per product
        (num_levels x nprob, synchronises)."""
        out = (ctypes.c_double * (self.num_levels * len(self.problems)))() if level_var else None
        check(lib().mlmc_matmul_estimate_batched(len(self.table), self.table, ctypes.byref(self.h.lv),
                                                 ctypes.byref(self.tuning), self.workspace.data_ptr(),
                                                 self.ws_bytes, out, _stream(self.device)))
        if level_var:
            import numpy as np
            return np.array(out[:]).reshape(self.num_levels, len(self.problems))
        return None

    def capture(self, stream: Optional[torch.cuda.Stream] = None):
        """Capture the whole estimate into a hipGraph on a side stream."""
        self.release()
        stream = stream or torch.cuda.Stream(device=self.device)
        handle = ctypes.c_void_p()
        check(lib().mlmc_matmul_batched_graph_create(len(self.table), self.table, ctypes.byref(self.h.lv),
                                                     ctypes.byref(self.tuning), self.workspace.data_ptr(),
                                                     self.ws_bytes, stream.cuda_stream, ctypes.byref(handle)))
        self.graph = handle
        self.graph_stream = stream
        return self

    def replay(self):
        """Launch the captured graph on the current stream."""
        if self.graph is None:
            raise RuntimeError("capture() first")
        check(lib().mlmc_graph_launch(self.graph, _stream(self.device)))

    def release(self):
        if self.graph is not None:
            check(lib().mlmc_graph_destroy(self.graph))
            self.graph = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass
