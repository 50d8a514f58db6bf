"""Synthetic workloads: shapes, laws, level ladders and seeded inputs.

Holds no arithmetic of the estimator: only the configurations and the seeded
generators of the inputs that both the GPU path and the oracle receive.
Every input is synthetic (the paper's own experiments are synthetic too).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional

import numpy as np


@dataclass
class Workload:
    name: str
    kind: str                 # "matmul" or "inner"
    m: int
    n: int
    p: int
    law_a: tuple              # ("normal"|"uniform", loc, scale) or ("reparam",)
    law_b: tuple
    c: list
    n_samples: Optional[list] = None
    rmse_target: float = 0.0  # total-Frobenius eps
    pilot: int = 0
    prec: str = "fp64"
    seed: int = 0


def ladder(c0: int, levels: int, ratio: int = 2) -> list:
    return [c0 * ratio ** l for l in range(levels)]


# A 64 x 256, B 256 x 64, i.i.d. N(1, 1); c_l = 4 * 2^l, l = 0..3; fixed N_l; FP64.
MATMUL_SMALL_FP64 = Workload("matmul-64x256x64-fp64", "matmul", 64, 256, 64, ("normal", 1.0, 1.0),
                             ("normal", 1.0, 1.0), ladder(4, 4), [1000, 500, 250, 125])

# x, y in R^(2^20), i.i.d. 0.5 + U(-1, 1); c_l = 64 * 2^l, l = 0..8;
# target RMSE eps = 1e-3 |E[x^T y]| with E[x^T y] = n * 0.5 * 0.5.
_N2 = 2 ** 20
INNER_2POW20 = Workload("inner-2^20-uniform", "inner", 1, _N2, 1, ("uniform", 0.5, 1.0),
                        ("uniform", 0.5, 1.0), ladder(64, 9), None, 1e-3 * _N2 * 0.25, 1024, "fp32")

# A 1024 x 65536, B 65536 x 1024, i.i.d. N(0.5, 1); c_l = 32 * 2^l, l = 0..7;
# eps per entry = 1e-2 ||E[AB]||_F / sqrt(m p) = 1e-2 * n * 0.25; the estimator
# takes the total-Frobenius eps = sqrt(m p) times that.
_N3 = 65536
MATMUL_LARGE = Workload("matmul-1024x65536x1024", "matmul", 1024, _N3, 1024, ("normal", 0.5, 1.0),
                        ("normal", 0.5, 1.0), ladder(32, 8), None,
                        1e-2 * _N3 * 0.25 * math.sqrt(1024 * 1024), 64, "bf16")


# Differentiation form: A = M_A + S_A o Z (512 x 32768), B = M_B + S_B o W
# (32768 x 512); c_l = 32 * 2^l, l = 0..6; fixed N_l = 4096 * 2^-l.
DIFF_512x32768x512 = Workload("diff-512x32768x512", "matmul", 512, 32768, 512, ("reparam",), ("reparam",),
                              ladder(32, 7), [4096 >> l for l in range(7)], prec="fp32")


def reparam_inputs(m: int, n: int, p: int, seed: int = 0):
    """M_A, M_B ~ N(0, 1), S_A, S_B ~ U(0.1, 1), T ~ N(0, 1) (m x p), FP32.

    Returned as A's in (n, m) layout (row j = column j of A) and B's in (n, p)."""
    rng = np.random.default_rng(seed)
    MA = rng.standard_normal((n, m), dtype=np.float32)
    SA = rng.uniform(0.1, 1.0, size=(n, m)).astype(np.float32)
    MB = rng.standard_normal((n, p), dtype=np.float32)
    SB = rng.uniform(0.1, 1.0, size=(n, p)).astype(np.float32)
    T = rng.standard_normal((m, p), dtype=np.float32)
    return MA, SA, MB, SB, T


# Importance sampling: A = M_A + S_A o Z (512 x 32768) whose column j is
# scaled by r_j = 0.05 + 2.95 j / (n - 1) (column-dependent laws, as in the
# experiments of Sec. 4), B = M_B + S_B o W; c_l = 32 * 2^l, l = 0..6; target
# RMSE 10% of ||E[AB]||_F (set at run time from the inputs), pilot 64, FP32.
IS_512x32768x512 = Workload("is-512x32768x512", "matmul", 512, 32768, 512, ("reparam",), ("reparam",),
                            ladder(32, 7), None, 0.0, 64, "fp32")


def reparam_ramp_inputs(m: int, n: int, p: int, seed: int = 0):
    """M_A ~ N(0, 1) r_j, S_A ~ U(0.1, 1) r_j with r_j = 0.05 + 2.95 j / (n - 1),
    M_B ~ N(0, 1), S_B ~ U(0.1, 1), FP32; A's in (n, m) layout, B's in (n, p)."""
    rng = np.random.default_rng(seed)
    r = (0.05 + 2.95 * np.arange(n) / max(n - 1, 1)).astype(np.float32)[:, None]
    MA = rng.standard_normal((n, m), dtype=np.float32) * r
    SA = rng.uniform(0.1, 1.0, size=(n, m)).astype(np.float32) * r
    MB = rng.standard_normal((n, p), dtype=np.float32)
    SB = rng.uniform(0.1, 1.0, size=(n, p)).astype(np.float32)
    return MA, SA, MB, SB


def batched_products(count: int = 256, seed: int = 0):
    """The batching workload: `count` independent products, m and p uniform on
    {64, 128, ..., 512}, n log-uniform on [4096, 131072] (rounded), entries
    i.i.d. N(mu, 1) with mu uniform on (0, 2) per product; c_l = 16 * 2^l,
    l = 0..6; N_l = 2048 * 2^-l.  Returns (shapes, mus, c, N)."""
    rng = np.random.default_rng(seed)
    m = rng.integers(1, 9, size=count) * 64
    p = rng.integers(1, 9, size=count) * 64
    n = np.rint(np.exp(rng.uniform(np.log(4096), np.log(131072), size=count))).astype(np.int64)
    mu = rng.uniform(0.0, 2.0, size=count)
    shapes = [(int(a), int(b), int(c)) for a, b, c in zip(m, n, p)]
    return shapes, [float(x) for x in mu], ladder(16, 7), [2048 >> l for l in range(7)]


# The experiments of Sec. 4 at the paper's sizes, with M = 10 ladders
# c_l = 10^l, l = 0..6 (the adaptive loop chooses L):
#   Sec. 4.1: n = 1e4, x_j = (j/50)(0.4 - z), y_j = cos(Poi(10) + 2 Exp(1)) Bern(0.05),
#             f(x) = 1 / (|x| H(x + 0.4) + 0.01);
#   Sec. 4.2: m = p = 1e3, n = 1e4, A_ij = sin(s) + z' s with s = (j/1e4)(0.5 - z),
#             B_jk = cos(Poi(2)) H(5 - Poi(2)) Bern(0.2), f(x) = |x| H(2 - x).
# Target RMSE: 0.1 of the size of E[f] (|.| or Frobenius), fixed from
# estimates of it: |E f(x^T y)| = 52.2 (an FP64 estimate with RMSE 1.3), so
# eps = 5.22, times sqrt(20) for the 1/20 scaling of N_l in Sec. 4.1; every
# entry of E[f(AB)] is the same, about 26.8 (the mean over the entries of
# FP32 estimates of it), so ||E f(AB)||_F = 26.8 * 1e3 = 2.68e4 and
# eps = 2680.
@dataclass
class ExperimentWorkload:
    name: str
    kind: str
    m: int
    n: int
    p: int
    law_a: tuple              # (binding constructor, arguments)
    law_b: tuple
    func: tuple               # (binding constructor, arguments)
    c: list
    size: float               # |E f| or ||E f||_F (see above)
    rel_eps: float
    n_scale: float            # N_l scale of eq. (28): eps is divided by sqrt(n_scale)
    pilot: int

    @property
    def eps(self) -> float:
        return self.rel_eps * self.size / math.sqrt(self.n_scale)


EXP41_INNER = ExperimentWorkload("sec4.1-inner-n1e4", "inner", 1, 10000, 1, ("ramp_normal", (1 / 50, 0.4)),
                                 ("cos_poisson_exp", (10.0, 0.05)), ("inv_abs_step", (0.4, 0.01)),
                                 ladder(1, 7, 10), 52.2, 0.1, 1 / 20, 100)
EXP42_MATMUL = ExperimentWorkload("sec4.2-matmul-1000x1e4x1000", "matmul", 1000, 10000, 1000,
                                  ("sin_ramp", (1e-4, 0.5)), ("cos_poisson_step", (2.0, 0.2)),
                                  ("abs_step", (2.0,)), ladder(1, 7, 10), 2.68e4, 0.1, 1.0, 100)
