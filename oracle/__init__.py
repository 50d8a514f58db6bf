"""Reference oracle for the MLMC estimator of E[AB] (Wu & Polydorides, arXiv:1904.00429).

TEST INFRASTRUCTURE ONLY.  Nothing in the product imports this package: only
``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
do.  It shares no code with the HIP library.

The per-realisation work (random numbers, index draws, sketches, Welford
updates) is plain sequential FP64 C in ``mlmc_oracle.c``; this module drives it
the way Alg. 2 of Sec. 3.1 does, for a fixed finest level L, and adds the
closed-form moments that pin it (Theorem 3.2 specialised to the synthetic
laws) and the optimal-allocation rule of Remark 3.6, eq. (28).

Parity pins and where they are tested (``tests/test_oracle_*.py``):
  Philox4x32-10      against rocRAND's open-source engine (a third-party
                     implementation of the same published generator);
  index map          against exact big-integer arithmetic and chi-square;
  sketch (18)        brute force over every index tuple on tiny n and c;
  Alg. 1 / (10)      telescoping identity on shared realisations;
  level variances    closed forms (Thm 3.2 with uniform xi) by z-tests;
  scheduler (28)     Lagrange optimality of the continuous allocation;
  target function f  hand-evaluated steps, constant matrices, telescoping,
                     brute force over index tuples;
  adaptive L         constant laws, reuse of realisations, the stopping test;
  weighted xi        unit weights = uniform draws, chi-square, unbiasedness
                     and exact error by brute force, Theorem 3.1's minimum;
  Sec. 4 laws        sample moments against closed forms (characteristic
                     functions of Poisson, exponential and normal variables)
                     and the Poisson probabilities by chi-square;
  stride coupling    unit-vector probe of the coarse draws (r_{jM}), brute
                     force over index tuples, closed-form V_l by z-test;
  32-bit index words top bits of the rocRAND-pinned Philox words for
                     power-of-two n, exact integers, chi-square, closed-form
                     V_l of the inner product by z-test;
  16-bit values      the halves of the rocRAND-pinned words, the Box-Muller
                     identities, moments, closed-form V_l by z-test.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mlmc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_mlmc_oracle.so")

LAW_NORMAL = 0
LAW_UNIFORM = 1
LAW_REPARAM = 2
LAW_RAMP_NORMAL = 3         # Sec. 4.1's a_j: (j scale)(loc - z)
LAW_COS_POISSON_EXP = 4     # Sec. 4.1's b_j: cos(K + 2E) [u < scale], K ~ Poisson(loc)
LAW_SIN_RAMP = 5            # Sec. 4.2's A_ij: sin(x) + z' x, x = (j scale)(loc - z)
LAW_COS_POISSON_STEP = 6    # Sec. 4.2's B_jk: cos(K) H(5 - K) [u < scale], K ~ Poisson(loc)
SHARED_LEVEL_FIELD = 0xFF


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (IEEE FP64, no contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
            "-fno-fast-math", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Law(ctypes.Structure):
    _fields_ = [("law", ctypes.c_int32), ("loc", ctypes.c_double),
                ("scale", ctypes.c_double), ("mean", ctypes.c_void_p),
                ("stdev", ctypes.c_void_p), ("ld", ctypes.c_int64),
                ("exp_neg_loc", ctypes.c_double), ("value16", ctypes.c_int32),
                ("operand", ctypes.c_int32), ("scale_exp", ctypes.c_void_p)]


class _Weights(ctypes.Structure):
    _fields_ = [("w", ctypes.c_void_p), ("cum", ctypes.c_void_p), ("total", ctypes.c_uint64)]


class _Func(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("theta0", ctypes.c_double), ("theta1", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_philox_batch.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_uint64,
                                       ctypes.c_void_p]
        L.orc_draw_index.restype = ctypes.c_int64
        L.orc_draw_index.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                     ctypes.c_uint32, ctypes.c_int64, ctypes.c_int64]
        L.orc_draw_indices.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                       ctypes.c_uint32, ctypes.c_int64, ctypes.c_int64,
                                       ctypes.c_void_p]
        L.orc_draw_indices_mode.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                            ctypes.c_uint32, ctypes.c_int64, ctypes.c_int64,
                                            ctypes.c_int32, ctypes.c_void_p]
        L.orc_uniform.restype = ctypes.c_double
        L.orc_uniform.argtypes = [ctypes.c_uint32]
        L.orc_column.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                 ctypes.c_uint32, ctypes.c_int64, ctypes.c_int64,
                                 ctypes.c_int64, ctypes.POINTER(_Law), ctypes.POINTER(_Law),
                                 ctypes.c_void_p, ctypes.c_void_p]
        L.orc_sketch_pair.argtypes = [ctypes.c_int64] * 6 + [ctypes.c_void_p] * 4
        L.orc_level_estimation.restype = ctypes.c_int
        L.orc_level_estimation.argtypes = (
            [ctypes.c_int64] * 3 + [ctypes.POINTER(_Law)] * 2 + [ctypes.c_int64] * 3 + [ctypes.c_int32]
            + [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int64,
               ctypes.c_int64, ctypes.POINTER(_Func), ctypes.POINTER(_Weights), ctypes.c_int32, ctypes.c_void_p,
               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p])
        L.orc_multiset.restype = ctypes.c_int64
        L.orc_multiset.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.orc_weights_cumulative.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
        L.orc_draw_index_weighted.restype = ctypes.c_int64
        L.orc_draw_index_weighted.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                              ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(_Weights)]
        L.orc_optimal_weights.argtypes = ([ctypes.c_int64] * 3 + [ctypes.POINTER(_Law)] * 2 + [ctypes.c_void_p])
        L.orc_sketch_pair_weighted.argtypes = [ctypes.c_int64] * 5 + [ctypes.c_void_p] * 5
        L.orc_operand_value.restype = ctypes.c_double
        L.orc_operand_value.argtypes = [ctypes.POINTER(_Law), ctypes.c_int64, ctypes.c_double]
        L.orc_reparam_bounds.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                         ctypes.c_int64, ctypes.c_void_p]
        L.orc_apply_func.restype = ctypes.c_double
        L.orc_apply_func.argtypes = [ctypes.POINTER(_Func), ctypes.c_double]
        L.orc_level_entries.argtypes = (
            [ctypes.c_int64] * 3 + [ctypes.POINTER(_Law)] * 2 + [ctypes.c_int64] * 3
            + [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int64,
               ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p])
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


# --------------------------------------------------------------------------
# Laws of the random matrices (the "pre-defined" L_A, L_B of Alg. 1 / Alg. 2)
# --------------------------------------------------------------------------
@dataclass
class Law:
    """Entry law of A (m x n) or B (n x p).

    normal:  loc + scale * N(0, 1);  uniform: loc + scale * U(-1, 1);
    reparam: mean + stdev * N(0, 1) with A column-major (m x n, element (i, j)
    at j*ld + i) and B row-major (n x p, element (j, q) at j*ld + q)."""
    law: int
    loc: float = 0.0
    scale: float = 1.0
    mean: Optional[np.ndarray] = None
    stdev: Optional[np.ndarray] = None
    ld: int = 0
    value16: bool = False     # laws 0-2: 16-bit uniforms, eight per Philox call
    operand: int = 0          # OPERAND_*: the format the contraction reads the values in
    scale_exp: Optional[np.ndarray] = None   # FP8: exponent s of 2^s per row of A / column of B
    _keep: list = field(default_factory=list, repr=False)

    @staticmethod
    def normal(loc: float, scale: float) -> "Law":
        return Law(LAW_NORMAL, float(loc), float(scale))

    @staticmethod
    def uniform(loc: float, scale: float) -> "Law":
        return Law(LAW_UNIFORM, float(loc), float(scale))

    @staticmethod
    def experiment(kind: int, loc: float, scale: float) -> "Law":
        """One of the laws of the experiments of Sec. 4 (LAW_RAMP_NORMAL ...)."""
        return Law(int(kind), float(loc), float(scale))

    @staticmethod
    def reparam(mean: np.ndarray, stdev: np.ndarray, ld: int) -> "Law":
        return Law(LAW_REPARAM, 0.0, 0.0, np.ascontiguousarray(mean, dtype=np.float64),
                   np.ascontiguousarray(stdev, dtype=np.float64), int(ld))

    def with_value16(self) -> "Law":
        """The same law with values from 16-bit uniforms: element e of column
        j takes the low (even e) or high (odd e) half h of word (e/2) % 4 of
        the call (e/8, k, j, value stream), u = (h + 1/2) 2^-16; normals by
        Box-Muller on the pair (e & ~1, e | 1), which shares one word."""
        return Law(self.law, self.loc, self.scale, self.mean, self.stdev, self.ld, True, self.operand,
                   self.scale_exp)

    def with_operand(self, operand: int, scale_exp: Optional[np.ndarray] = None) -> "Law":
        """The same law read by the contraction in a narrower format
        (orc_operand_value): OPERAND_BF16, or OPERAND_FP8_E4M3 with the
        exponents s of the power-of-two scales 2^s of every row of A (or
        column of B), e.g. from fp8_scale_exponents."""
        se = None if scale_exp is None else np.ascontiguousarray(scale_exp, dtype=np.int32)
        return Law(self.law, self.loc, self.scale, self.mean, self.stdev, self.ld, self.value16, int(operand), se)

    def c(self) -> _Law:
        s = _Law()
        s.law = self.law
        s.loc = self.loc
        s.scale = self.scale
        s.exp_neg_loc = math.exp(-self.loc) if self.law in (LAW_COS_POISSON_EXP, LAW_COS_POISSON_STEP) else 0.0
        s.value16 = 1 if self.value16 else 0
        s.operand = self.operand
        s.scale_exp = _ptr(self.scale_exp) if self.scale_exp is not None else None
        if self.law == LAW_REPARAM:
            s.mean = _ptr(self.mean)
            s.stdev = _ptr(self.stdev)
            s.ld = self.ld
        return s


OPERAND_EXACT, OPERAND_BF16, OPERAND_FP8_E4M3 = 0, 1, 2


def operand_value(law: Law, idx: int, v: float) -> float:
    """orc_operand_value: v as the contraction reads it under law.operand."""
    return float(lib().orc_operand_value(ctypes.byref(law.c()), int(idx), float(v)))


def fp8_scale_exponent(bound: float) -> int:
    """The exponent s of the FP8 operand scale 2^s: the largest s with
    2^s bound <= 256 (entries up to the bound then sit in e4m3's top binades,
    below its largest value 448), clamped to [-20, 20]; 0 for a zero bound.
    Exact: bound = f 2^E with f in [1/2, 1) gives s = 8 - E, or 9 - E when
    f = 1/2."""
    if not bound > 0.0:
        return 0
    f, E = math.frexp(bound)
    s = 8 - E + (1 if f == 0.5 else 0)
    return max(-20, min(20, s))


def fp8_scale_exponents(law: Law, count: int, side: str) -> np.ndarray:
    """Scale exponents of the rows of A (side "A", count = m) or the columns
    of B (side "B", count = p).  The bound of an entry is |loc| + 6 |scale|
    (normal), |loc| + |scale| (uniform), fma(6, |stdev|, |mean|) per entry
    (reparameterised; the maximum over the n columns of A's row or rows of
    B's column)."""
    if law.law == LAW_NORMAL:
        return np.full(count, fp8_scale_exponent(abs(law.loc) + 6.0 * abs(law.scale)), dtype=np.int32)
    if law.law == LAW_UNIFORM:
        return np.full(count, fp8_scale_exponent(abs(law.loc) + abs(law.scale)), dtype=np.int32)
    if law.law != LAW_REPARAM:
        raise ValueError("FP8 operands take the normal, uniform or reparameterised laws")
    n = law.mean.size // law.ld
    bound = np.empty(count)
    lib().orc_reparam_bounds(_ptr(law.mean), _ptr(law.stdev), n, law.ld, count, _ptr(bound))
    return np.array([fp8_scale_exponent(b) for b in bound], dtype=np.int32)


# --------------------------------------------------------------------------
# Target function f of Sec. 3 (entrywise on every sketch)
# --------------------------------------------------------------------------
F_IDENTITY, F_ABS_STEP, F_INV_ABS_STEP = 0, 1, 2


@dataclass
class Func:
    """f(x) = x (identity); |x| H(theta0 - x) (abs_step, Sec. 4.2 with
    theta0 = 2); 1 / (|x| H(x + theta0) + theta1) (inv_abs_step, Sec. 4.1 with
    theta0 = 0.4, theta1 = 0.01).  H(0) = 1."""
    kind: int = F_IDENTITY
    theta0: float = 0.0
    theta1: float = 0.0

    @staticmethod
    def abs_step(theta0: float = 2.0) -> "Func":
        return Func(F_ABS_STEP, float(theta0), 0.0)

    @staticmethod
    def inv_abs_step(theta0: float = 0.4, theta1: float = 0.01) -> "Func":
        return Func(F_INV_ABS_STEP, float(theta0), float(theta1))

    def c(self) -> _Func:
        s = _Func()
        s.kind = self.kind
        s.theta0 = self.theta0
        s.theta1 = self.theta1
        return s

    def __call__(self, x: float) -> float:
        fc = self.c()
        return float(lib().orc_apply_func(ctypes.byref(fc), float(x)))


# --------------------------------------------------------------------------
# Index probabilities xi_j = w_j / W (eq. (18) with a general xi)
# --------------------------------------------------------------------------
class Weights:
    """Integer column weights w_j >= 1 and their cumulative sums."""

    def __init__(self, w):
        self.w = np.ascontiguousarray(w, dtype=np.uint32)
        if self.w.ndim != 1 or self.w.size == 0 or int(self.w.min()) < 1:
            raise ValueError("weights must be a non-empty vector of integers >= 1")
        self.cum = np.empty(self.w.size, dtype=np.uint64)
        lib().orc_weights_cumulative(_ptr(self.w), self.w.size, _ptr(self.cum))
        self.total = int(self.cum[-1])

    @property
    def xi(self) -> np.ndarray:
        return self.w.astype(np.float64) / float(self.total)

    def c(self) -> _Weights:
        s = _Weights()
        s.w = _ptr(self.w)
        s.cum = _ptr(self.cum)
        s.total = self.total
        return s


def optimal_weights(m: int, n: int, p: int, A: Law, B: Law) -> np.ndarray:
    """Theorem 3.1's xi** as integer weights (orc_optimal_weights)."""
    w = np.empty(n, dtype=np.uint32)
    la, lb = A.c(), B.c()
    lib().orc_optimal_weights(int(m), int(n), int(p), ctypes.byref(la), ctypes.byref(lb), _ptr(w))
    return w


def draw_index_weighted(seed: int, problem: int, lfield: int, k: int, t: int, weights: Weights) -> int:
    wc = weights.c()
    return int(lib().orc_draw_index_weighted(int(seed), int(problem), int(lfield), int(k), int(t),
                                             weights.w.size, ctypes.byref(wc)))


def sketch_pair_weighted(c_f: int, c_c: int, factor, AS: np.ndarray, BS: np.ndarray, stride: int = 0):
    """Zf, Zc of eq. (18) with per-draw factors 1 / xi_{r_t} (coarse draws:
    the first c_c, or with stride M > 0 draws M - 1, 2M - 1, ...)."""
    AS = np.ascontiguousarray(AS, dtype=np.float64)
    BS = np.ascontiguousarray(BS, dtype=np.float64)
    factor = np.ascontiguousarray(factor, dtype=np.float64)
    m, p = AS.shape[1], BS.shape[1]
    Zf = np.zeros((m, p))
    Zc = np.zeros((m, p))
    lib().orc_sketch_pair_weighted(m, p, int(c_f), int(c_c), int(stride), _ptr(factor), _ptr(AS), _ptr(BS),
                                   _ptr(Zf), _ptr(Zc))
    return Zf, Zc


# --------------------------------------------------------------------------
# Random numbers, index draws, columns, sketches
# --------------------------------------------------------------------------
def philox(ctr: np.ndarray, seed: int) -> np.ndarray:
    """Philox4x32-10 of counters ctr (count x 4 uint32) under key = seed."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    out = np.empty_like(ctr)
    lib().orc_philox_batch(ctr.shape[0], _ptr(ctr), int(seed), _ptr(out))
    return out


def level_field(level: int, shared: bool = False) -> int:
    return SHARED_LEVEL_FIELD if shared else int(level)


def draw_indices(seed: int, problem: int, lfield: int, k: int, c: int, n: int,
                 word32: bool = False) -> np.ndarray:
    """Draws 0 .. c-1 of realisation k; word32: four draws per Philox call,
    r = floor(w n / 2^32) from one 32-bit word (exact for power-of-two n)."""
    r = np.empty(int(c), dtype=np.int64)
    lib().orc_draw_indices_mode(int(seed), int(problem), int(lfield), int(k), int(c), int(n), int(bool(word32)),
                                _ptr(r))
    return r


def uniform(w: int) -> float:
    return lib().orc_uniform(int(w))


def column(seed: int, problem: int, lfield: int, k: int, j: int, m: int, p: int,
           A: Law, B: Law):
    a = np.empty(m, dtype=np.float64)
    b = np.empty(p, dtype=np.float64)
    la, lb = A.c(), B.c()
    lib().orc_column(int(seed), int(problem), int(lfield), int(k), int(j), int(m), int(p),
                     ctypes.byref(la), ctypes.byref(lb), _ptr(a), _ptr(b))
    return a, b


def realisation(seed: int, problem: int, lfield: int, k: int, m: int, n: int, p: int,
                A: Law, B: Law):
    """The whole realisation A^(k) (m x n), B^(k) (n x p) -- tiny n only."""
    Am = np.empty((m, n))
    Bm = np.empty((n, p))
    for j in range(n):
        Am[:, j], Bm[j, :] = column(seed, problem, lfield, k, j, m, p, A, B)
    return Am, Bm


def sketch_pair(n: int, c_f: int, c_c: int, AS: np.ndarray, BS: np.ndarray, stride: int = 0):
    """Fine and coarse sketches (eq. (18), xi = 1/n) of gathered columns.

    AS is (c_f, m): row t is the sampled column a_t; BS is (c_f, p).  The
    coarse sketch takes the first c_c draws, or with stride M > 0 the draws
    M - 1, 2M - 1, ... (r_{jM} of Sec. 3.1)."""
    AS = np.ascontiguousarray(AS, dtype=np.float64)
    BS = np.ascontiguousarray(BS, dtype=np.float64)
    m, p = AS.shape[1], BS.shape[1]
    Zf = np.zeros((m, p))
    Zc = np.zeros((m, p))
    lib().orc_sketch_pair(m, p, int(n), int(c_f), int(c_c), int(stride), _ptr(AS), _ptr(BS), _ptr(Zf), _ptr(Zc))
    return Zf, Zc


@dataclass
class LevelState:
    """Welford state of one level: count, per-entry mean and M2."""
    count: int
    mean: np.ndarray
    m2: np.ndarray

    @staticmethod
    def empty(m: int, p: int) -> "LevelState":
        return LevelState(0, np.zeros(m * p), np.zeros(m * p))

    @property
    def variance(self) -> float:
        """V_l of Remark 3.6: vectorised variance of one level sample
        (sum over entries of the unbiased entry variances)."""
        if self.count < 2:
            return 0.0
        return float(self.m2.sum()) / (self.count - 1)


def coupling_stride(c_l: int, c_prev: int, coupling: str) -> int:
    """M = c_l / c_prev for the stride coupling (0: prefix, or level 0)."""
    if coupling not in ("prefix", "stride"):
        raise ValueError("coupling must be 'prefix' or 'stride'")
    return int(c_l) // int(c_prev) if coupling == "stride" and c_prev > 0 else 0


def level_estimation(state: LevelState, m: int, n: int, p: int, A: Law, B: Law,
                     c_l: int, c_prev: int, seed: int, problem: int, lfield: int,
                     k_begin: int, k_end: int, want_samples: bool = False,
                     func: Optional[Func] = None, weights: Optional["Weights"] = None,
                     coupling: str = "prefix", index_word32: bool = False, as_set: bool = False):
    """Alg. 1 for realisations [k_begin, k_end), continuing `state` in place;
    level samples f(Zf) - f(Zc) (identity when func is None).  coupling:
    "prefix" (the coarse sketch takes the first c_prev draws) or "stride"
    (every M-th draw, M = c_l / c_prev, Sec. 3.1).  index_word32: the indices
    from 32-bit words (draw_indices(word32=True)).  as_set: each index tuple
    is taken as a set with multiplicities (the note after Alg. 1), every
    distinct column read once."""
    cnt = ctypes.c_int64(state.count)
    samples = np.empty((max(k_end - k_begin, 0), m, p)) if want_samples else None
    la, lb = A.c(), B.c()
    fc = (func or Func()).c()
    if weights is not None and weights.w.size != n:
        raise ValueError("one weight per column")
    wc = weights.c() if weights is not None else None
    rc = lib().orc_level_estimation(
        int(m), int(n), int(p), ctypes.byref(la), ctypes.byref(lb), int(c_l), int(c_prev),
        coupling_stride(c_l, c_prev, coupling), int(bool(index_word32)), int(seed), int(problem), int(lfield), int(k_begin), int(k_end), ctypes.byref(fc),
        ctypes.byref(wc) if wc is not None else None, int(bool(as_set)),
        ctypes.byref(cnt), _ptr(state.mean), _ptr(state.m2), _ptr(samples) if want_samples else None)
    if rc != 0:
        raise ValueError("orc_level_estimation rejected its arguments")
    state.count = cnt.value
    return samples


def multiset(r: Sequence[int], c_c: int = 0, stride: int = 0):
    """The index tuple r as a set with multiplicities (the note after Alg. 1):
    (distinct values ascending, draws per value, coarse draws per value) for
    the c_c coarse draws of the coupling (stride 0: the first c_c)."""
    r = np.ascontiguousarray(r, dtype=np.int64)
    c_f = len(r)
    j = np.empty(c_f, dtype=np.int64)
    mf = np.empty(c_f, dtype=np.int64)
    mc = np.empty(c_f, dtype=np.int64)
    u = lib().orc_multiset(c_f, _ptr(r), int(c_c), int(stride), _ptr(j), _ptr(mf), _ptr(mc))
    if u < 0:
        raise ValueError("orc_multiset rejected its arguments")
    return j[:u].copy(), mf[:u].copy(), mc[:u].copy()


# --------------------------------------------------------------------------
# Optimal number of realisations per level: Remark 3.6, eq. (28)
# --------------------------------------------------------------------------
def schedule(V: Sequence[float], C: Sequence[float], eps: float) -> list:
    """N_l = ceil(2 eps^-2 sqrt(V_l / C_l) sum_j sqrt(V_j C_j)).

    Reading: the summand is indexed by j (the printed sqrt(V_l M^l) under a
    sum over j is a typo) and C_l is the cost of one level-l realisation,
    proportional to the number of sampled indices (M^l in the paper).  With
    this choice the variance of the estimator, sum_l V_l / N_l, is at most
    eps^2 / 2 (the budget of the proof of Theorem 2.3)."""
    V = np.asarray(V, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    total = float(np.sum(np.sqrt(V * C)))
    out = []
    for v, c in zip(V, C):
        out.append(int(math.ceil(2.0 / (eps * eps) * math.sqrt(v / c) * total)))
    return out


# --------------------------------------------------------------------------
# The estimator (Alg. 2 with a fixed finest level L)
# --------------------------------------------------------------------------
@dataclass
class Estimate:
    Y: np.ndarray                 # sum_l Ybar_l, m x p (eq. (10))
    level_means: np.ndarray       # (L+1) x m x p
    level_var: np.ndarray         # V_l
    n_used: np.ndarray            # N_l
    rmse_est: float               # sqrt(sum_l V_l / N_l)
    levels_used: int = 0          # adaptive mode: levels that were run
    bias_test_passed: bool = True  # adaptive mode: the stopping test held
    entry_var: Optional[np.ndarray] = None  # (L+1) x m x p: unbiased variance of one level sample per entry

    @property
    def entry_sd(self) -> np.ndarray:
        """Standard deviation of every entry of Y: sqrt(sum_l var_l / N_l)
        (levels are independent, eq. (10)); levels with no realisation add 0."""
        N = np.maximum(np.asarray(self.n_used, dtype=np.float64), 1.0)
        return np.sqrt(np.sum(self.entry_var / N[:, None, None], axis=0))


def bias_bound(c: Sequence[int], L: int, eps: float, kind: str) -> float:
    """The finest correction Ybar_L is small enough when its norm is below
    (sqrt(M) + 1) eps / sqrt(2) for a matrix product (Remark 3.5, eq. (27),
    Frobenius norm) or (sqrt(M) - 1) eps / sqrt(2) for the inner product
    (Sec. 2, eq. (15), absolute value); M is read as the ladder's ratio at the
    finest level, c_L / c_{L-1}."""
    M = c[L] / c[L - 1]
    return (math.sqrt(M) + (1.0 if kind == "matrix" else -1.0)) * eps / math.sqrt(2.0)


def estimate(m: int, n: int, p: int, A: Law, B: Law, c: Sequence[int],
             n_samples: Optional[Sequence[int]] = None, rmse_target: float = 0.0,
             pilot: int = 0, seed: int = 0, problem: int = 0, shared: bool = False,
             max_total_draws: int = 0, pool=None, func: Optional[Func] = None,
             adaptive: Optional[str] = None, weights: Optional[Weights] = None,
             coupling: str = "prefix", index_word32: bool = False, as_set: bool = False) -> Estimate:
    """MLMC estimate of E[f(AB)] (f entrywise, identity by default) over the
    ladder c_0 < c_1 < ... < c_L.

    Adaptive mode (adaptive = "matrix" or "inner", the entry point whose
    stopping test applies; Alg. 2's loop over L, target mode only; c is the
    longest ladder allowed): levels are added one at a time.  A new level first runs
    `pilot` realisations (its V_l must be estimated before eq. (28) can give
    N_l), then eq. (28) over the levels so far gives every N_l, and each level
    is extended to max(N_l, the realisations it already has), reusing them.
    From three levels on, the loop stops once the finest level mean passes
    the test of Remark 3.5 (bias_bound).

    Fixed-N mode: n_samples gives N_l.  Target mode (rmse_target > 0): `pilot`
    realisations per level estimate V_l, eq. (28) gives N_l, and every level
    is extended to max(N_l, pilot) realisations, reusing the pilot ones (the
    reuse of earlier evaluations in Alg. 2).  `pool` (a ThreadPoolExecutor)
    runs levels concurrently; each level's arithmetic is unchanged."""
    L1 = len(c)
    states = [LevelState.empty(m, p) for _ in range(L1)]

    def run(l, k0, k1):
        level_estimation(states[l], m, n, p, A, B, c[l], c[l - 1] if l > 0 else 0,
                         seed, problem, level_field(l, shared), k0, k1, func=func, weights=weights,
                         coupling=coupling, index_word32=index_word32, as_set=as_set)

    def run_all(ranges):
        if pool is None:
            for l, (k0, k1) in enumerate(ranges):
                run(l, k0, k1)
        else:
            list(pool.map(lambda a: run(*a), [(l, r[0], r[1]) for l, r in enumerate(ranges)]))

    if adaptive:
        if adaptive not in ("matrix", "inner"):
            raise ValueError("adaptive must be 'matrix' or 'inner'")
        if rmse_target <= 0 or pilot < 2:
            raise ValueError("adaptive mode needs rmse_target > 0 and a pilot of at least 2 realisations")
        used, passed = 0, False
        for L in range(L1):
            run(L, 0, pilot)
            used = L + 1
            V = [s.variance for s in states[:used]]
            N = [max(x, pilot) for x in schedule(V, c[:used], rmse_target)]
            if max_total_draws and sum(x * cl for x, cl in zip(N, c)) > max_total_draws:
                raise RuntimeError("draw budget exceeded")
            run_all([(states[l].count, max(N[l], states[l].count)) for l in range(used)])
            if used >= 3 and float(np.linalg.norm(states[L].mean)) < bias_bound(c, L, rmse_target, adaptive):
                passed = True
                break
        means = np.stack([s.mean.reshape(m, p) for s in states])
        V = np.array([s.variance for s in states])
        N = np.array([s.count for s in states], dtype=np.int64)
        rmse = math.sqrt(float(np.sum(V[:used] / N[:used])))
        return Estimate(means.sum(axis=0), means, V, N, rmse, used, passed, _entry_var(states, m, p))
    if rmse_target > 0:
        if pilot < 2:
            raise ValueError("target mode needs a pilot of at least 2 realisations")
        run_all([(0, pilot)] * L1)
        V = [s.variance for s in states]
        N = [max(x, pilot) for x in schedule(V, c, rmse_target)]
        if max_total_draws and sum(x * cl for x, cl in zip(N, c)) > max_total_draws:
            raise RuntimeError("draw budget exceeded")
        run_all([(pilot, N[l]) for l in range(L1)])
    else:
        if n_samples is None or len(n_samples) != L1:
            raise ValueError("fixed mode needs one N_l per level")
        run_all([(0, int(x)) for x in n_samples])
    means = np.stack([s.mean.reshape(m, p) for s in states])
    V = np.array([s.variance for s in states])
    N = np.array([s.count for s in states], dtype=np.int64)
    rmse = math.sqrt(float(np.sum(V / N)))
    return Estimate(means.sum(axis=0), means, V, N, rmse, L1, True, _entry_var(states, m, p))


def _entry_var(states, m: int, p: int) -> np.ndarray:
    """Per-entry unbiased variance of one level sample, M2 / (N_l - 1) (0 below two realisations)."""
    return np.stack([s.m2.reshape(m, p) / (s.count - 1) if s.count >= 2 else np.zeros((m, p)) for s in states])


@dataclass
class EntriesEstimate:
    Y: np.ndarray                 # sum_l Ybar_l at the chosen entries (nr x nc)
    level_means: np.ndarray       # (L+1) x nr x nc
    entry_var: np.ndarray         # (L+1) x nr x nc: unbiased variance of one level sample
    n_used: np.ndarray            # N_l


def estimate_entries(m: int, n: int, p: int, A: Law, B: Law, c: Sequence[int],
                     n_samples: Sequence[int], rows: Sequence[int], cols: Sequence[int],
                     seed: int = 0, problem: int = 0, shared: bool = False,
                     pool=None, coupling: str = "prefix") -> EntriesEstimate:
    """The fixed-N estimate of eq. (10) at the entries rows x cols only.

    Level l runs realisations 0 .. N_l - 1 exactly as `estimate` does, so its
    values at these entries equal the full estimate's (same arithmetic and
    order); products whose full sketch the CPU cannot afford are checked this
    way.  A target-mode run is reproduced by passing the N_l it used."""
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    nr, nc = len(rows), len(cols)
    L1 = len(c)
    if len(n_samples) != L1:
        raise ValueError("one N_l per level expected")
    means = np.zeros((L1, nr * nc))
    m2s = np.zeros((L1, nr * nc))
    la, lb = A.c(), B.c()

    def run(l):
        cnt = ctypes.c_int64(0)
        rc = lib().orc_level_entries(
            int(m), int(n), int(p), ctypes.byref(la), ctypes.byref(lb), int(c[l]),
            int(c[l - 1]) if l > 0 else 0, coupling_stride(c[l], c[l - 1] if l > 0 else 0, coupling), int(seed), int(problem), level_field(l, shared), 0,
            int(n_samples[l]), nr, _ptr(rows), nc, _ptr(cols), ctypes.byref(cnt),
            _ptr(means[l]), _ptr(m2s[l]))
        if rc != 0:
            raise ValueError("orc_level_entries rejected its arguments")

    if pool is None:
        for l in range(L1):
            run(l)
    else:
        list(pool.map(run, range(L1)))
    N = np.asarray(n_samples, dtype=np.int64)
    var = m2s / np.maximum(N - 1, 1)[:, None]
    shape = (L1, nr, nc)
    return EntriesEstimate(means.sum(axis=0).reshape(nr, nc), means.reshape(shape),
                           var.reshape(shape), N)


# --------------------------------------------------------------------------
# Closed forms (Theorem 3.2 with xi = 1/n, specialised to the synthetic laws)
# --------------------------------------------------------------------------
def _moments(law: Law):
    """(E x, E x^2) of one entry of an i.i.d. law."""
    if law.law == LAW_NORMAL:
        return law.loc, law.loc ** 2 + law.scale ** 2
    if law.law == LAW_UNIFORM:
        return law.loc, law.loc ** 2 + law.scale ** 2 / 3.0
    raise ValueError("i.i.d. law expected")


def closed_form_iid(m: int, n: int, p: int, A: Law, B: Law, c: Sequence[int]):
    """E[AB] (every entry) and V_l for i.i.d. entries.

    With kappa = E a^2 E b^2 - (E a E b)^2 and the prefix coupling,
      V_0 = m p (n (n-1) kappa / c_0 + n kappa),
      V_l = m p n (n-1) kappa (1/c_{l-1} - 1/c_l), l >= 1."""
    ma, a2 = _moments(A)
    mb, b2 = _moments(B)
    kappa = a2 * b2 - (ma * mb) ** 2
    V = [m * p * (n * (n - 1) * kappa / c[0] + n * kappa)]
    for l in range(1, len(c)):
        V.append(m * p * n * (n - 1) * kappa * (1.0 / c[l - 1] - 1.0 / c[l]))
    return n * ma * mb, np.array(V)


def closed_form_reparam(MA, SA, MB, SB, c: Sequence[int]):
    """E[AB] and V_l for A = MA + SA o Z, B = MB + SB o W (Z, W standard normal).

    With Q = M^2 + S^2 (entrywise),
      sigma2 = (n-1) QA QB + MA^2 MB^2 - (MA MB)^2   (entrywise squares),
      V_0 = sum(sigma2 / c_0 + QA QB - MA^2 MB^2),  V_l = (1/c_{l-1} - 1/c_l) sum(sigma2)."""
    MA, SA, MB, SB = (np.asarray(x, dtype=np.float64) for x in (MA, SA, MB, SB))
    n = MA.shape[1]
    QA, QB = MA ** 2 + SA ** 2, MB ** 2 + SB ** 2
    QQ = QA @ QB
    MM2 = (MA ** 2) @ (MB ** 2)
    EAB = MA @ MB
    sigma2 = (n - 1) * QQ + MM2 - EAB ** 2
    V = [float(np.sum(sigma2 / c[0] + QQ - MM2))]
    for l in range(1, len(c)):
        V.append(float((1.0 / c[l - 1] - 1.0 / c[l]) * np.sum(sigma2)))
    return EAB, np.array(V)
