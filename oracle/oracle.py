"""Test-only reference CPU implementation of the sparse permanent (Python side).

This module is test infrastructure.  Only the test suite, the smoke check and
the benchmark's CPU-baseline leg may import it; the product path never does.
It wraps ``perm_oracle.c`` (plain C, long double / exact integer arithmetic)
through ctypes and shares no code with the HIP library.

Functions (each follows the passage named in ``perm_oracle.c``):

* ``perm_brute(A)``          Eq. (1), permutations, dense input, n <= 12.
* ``perm_ryser(A)``          Eq. (2), all 2^n subsets, dense input, n <= 24.
* ``nw_range(ccs, b, e)``    Alg. 1 terms g in [b, e), long double.
* ``perm_nw(ccs)``           Alg. 1 full range times the final factor.
* ``perm_int(ccs)``          exact integer permanent of a 0/1 pattern via the
                             integer form of Alg. 1 (terms mod 2^128).
* ``gray(g)``, ``changed_bit(g)``  Alg. 1's Gray-code step, from the XOR definition.
* ``permanent_ordering(ccs)``  Alg. 4.
* ``partitioning(ccs, tau, grratio)``  Alg. 5.
* ``structural_rank(ccs)``   maximum bipartite matching size.

A CCS here is a tuple ``(n, colptr, rowidx, val)`` of an int, two int32 arrays
and one float64 array.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import threading
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "perm_oracle.c")
_LIB_DIR = os.path.join(_HERE, "_build")
_LIB = os.path.join(_LIB_DIR, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile ``perm_oracle.c`` with gcc into ``oracle/_build/liboracle.so``."""
    os.makedirs(_LIB_DIR, exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-pthread",
                        "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            lib = ctypes.CDLL(_LIB)
            P = ctypes.POINTER
            i32p, f64p, u64p = P(ctypes.c_int32), P(ctypes.c_double), P(ctypes.c_uint64)
            lib.oracle_gray.restype = ctypes.c_uint64
            lib.oracle_gray.argtypes = [ctypes.c_uint64]
            lib.oracle_changed_bit.argtypes = [ctypes.c_uint64, i32p, i32p]
            lib.oracle_perm_brute.argtypes = [ctypes.c_int, f64p, f64p, f64p]
            lib.oracle_perm_ryser.argtypes = [ctypes.c_int, f64p, f64p, f64p]
            lib.oracle_nw_range.argtypes = [ctypes.c_int, i32p, i32p, f64p, ctypes.c_uint64,
                                            ctypes.c_uint64, ctypes.c_int, f64p]
            lib.oracle_perm_nw.argtypes = [ctypes.c_int, i32p, i32p, f64p, ctypes.c_int, f64p]
            lib.oracle_nw_int_range.argtypes = [ctypes.c_int, i32p, i32p, ctypes.c_uint64,
                                                ctypes.c_uint64, ctypes.c_int, u64p]
            lib.oracle_permanent_ordering.argtypes = [ctypes.c_int, i32p, i32p, i32p, i32p]
            lib.oracle_partitioning.argtypes = [ctypes.c_int, i32p, i32p, f64p, ctypes.c_double,
                                                i32p, i32p, f64p]
            lib.oracle_structural_rank.argtypes = [ctypes.c_int, i32p, i32p]
            _lib = lib
    return _lib


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def default_threads() -> int:
    return max(1, len(os.sched_getaffinity(0)))


# --------------------------------------------------------------------------
# Gray code (Alg. 1's Gray-code step)
# --------------------------------------------------------------------------

def gray(g: int) -> int:
    return int(_load().oracle_gray(g))


def changed_bit(g: int) -> tuple[int, int]:
    """(j, s) of step g >= 1: the flipped column and +1/-1 direction."""
    j, s = ctypes.c_int32(), ctypes.c_int32()
    if _load().oracle_changed_bit(g, ctypes.byref(j), ctypes.byref(s)) != 0:
        raise ValueError("step index must be >= 1")
    return j.value, s.value


# --------------------------------------------------------------------------
# Dense definitions, Eq. (1) and Eq. (2)
# --------------------------------------------------------------------------

def _dense_call(fn, A):
    A = _f64(A)
    n = A.shape[0]
    assert A.shape == (n, n)
    hi, lo = ctypes.c_double(), ctypes.c_double()
    if fn(n, _ptr(A, ctypes.c_double), ctypes.byref(hi), ctypes.byref(lo)) != 0:
        raise ValueError("size out of range for this oracle")
    return hi.value + lo.value, (hi.value, lo.value)


def perm_brute(A) -> float:
    """Eq. (1): sum over all permutations, long double; n <= 12."""
    return _dense_call(_load().oracle_perm_brute, A)[0]


def perm_ryser(A) -> float:
    """Eq. (2): Ryser inclusion-exclusion over all subsets, long double; n <= 24."""
    return _dense_call(_load().oracle_perm_ryser, A)[0]


# --------------------------------------------------------------------------
# Alg. 1, sparse (CCS) input
# --------------------------------------------------------------------------

def _ccs_args(ccs):
    n, colptr, rowidx, val = ccs
    colptr, rowidx, val = _i32(colptr), _i32(rowidx), _f64(val)
    if len(colptr) != n + 1:
        raise ValueError("colptr must have n+1 entries")
    return n, colptr, rowidx, val


def nw_range(ccs, g_begin: int, g_end: int, threads: int | None = None):
    """Alg. 1 terms for Gray indices g in [g_begin, g_end), without the final factor.

    Returns ``(sum, abs_sum)`` where each is a ``(hi, lo)`` pair of doubles that
    represents the long double result exactly.
    """
    n, colptr, rowidx, val = _ccs_args(ccs)
    out = np.zeros(4, dtype=np.float64)
    rc = _load().oracle_nw_range(n, _ptr(colptr, ctypes.c_int32), _ptr(rowidx, ctypes.c_int32),
                                 _ptr(val, ctypes.c_double), g_begin, g_end,
                                 threads or default_threads(), _ptr(out, ctypes.c_double))
    if rc != 0:
        raise ValueError("bad CCS or range")
    return (out[0], out[1]), (out[2], out[3])


def perm_nw(ccs, threads: int | None = None):
    """Permanent by Alg. 1 in long double.

    Returns ``(value, abs_sum)``: value as a Python float (hi + lo rounded) and
    ``abs_sum`` = 2 * sum_g |term_g|, the scale of the cancellation.
    """
    n, colptr, rowidx, val = _ccs_args(ccs)
    out = np.zeros(4, dtype=np.float64)
    rc = _load().oracle_perm_nw(n, _ptr(colptr, ctypes.c_int32), _ptr(rowidx, ctypes.c_int32),
                                _ptr(val, ctypes.c_double), threads or default_threads(),
                                _ptr(out, ctypes.c_double))
    if rc != 0:
        raise ValueError("bad CCS")
    return out[0] + out[1], out[2] + out[3]


def perm_nw_hilo(ccs, threads: int | None = None):
    """As ``perm_nw`` but returns the long double value as an exact Fraction."""
    n, colptr, rowidx, val = _ccs_args(ccs)
    out = np.zeros(4, dtype=np.float64)
    rc = _load().oracle_perm_nw(n, _ptr(colptr, ctypes.c_int32), _ptr(rowidx, ctypes.c_int32),
                                _ptr(val, ctypes.c_double), threads or default_threads(),
                                _ptr(out, ctypes.c_double))
    if rc != 0:
        raise ValueError("bad CCS")
    return Fraction(out[0]) + Fraction(out[1]), out[2] + out[3]


def nw_int_range(ccs, g_begin: int, g_end: int, threads: int | None = None):
    """Integer Alg. 1 terms 2^n * term_g summed over [g_begin, g_end), mod 2^128.

    Only the pattern of the CCS is used (every stored entry counts as a 1).
    Returns ``(sum_mod_2^128, nonzero_terms)``.
    """
    n, colptr, rowidx, _ = _ccs_args(ccs)
    out = np.zeros(3, dtype=np.uint64)
    rc = _load().oracle_nw_int_range(n, _ptr(colptr, ctypes.c_int32), _ptr(rowidx, ctypes.c_int32),
                                     g_begin, g_end, threads or default_threads(),
                                     _ptr(out, ctypes.c_uint64))
    if rc != 0:
        raise ValueError("bad CCS or range")
    return int(out[0]) | (int(out[1]) << 64), int(out[2])


def bregman_bound(ccs) -> int:
    """An integer upper bound on the permanent of a 0/1 pattern.

    Bregman-Minc: perm <= prod_i (d_i!)^(1/d_i) over row degrees d_i; rounded up
    generously (times 2) so that the float evaluation cannot undercut it.
    """
    n, colptr, rowidx, _ = _ccs_args(ccs)
    deg = np.bincount(rowidx, minlength=n)
    logb = sum(math.lgamma(int(d) + 1) / int(d) for d in deg if d > 0)
    if np.any(deg == 0):
        return 0
    return int(math.exp(logb)) * 2 + 2


def perm_int(ccs, threads: int | None = None) -> int:
    """Exact permanent (number of perfect matchings) of a 0/1 pattern.

    Recovers T = sum_g (-1)^g prod_i (2 x_i) = (-1)^(n-1) 2^(n-1) perm from its
    value mod 2^128.  This is exact when |T| < 2^127, which is checked against
    the Bregman-Minc bound.
    """
    n = ccs[0]
    T, _ = nw_int_range(ccs, 0, 1 << (n - 1), threads)
    bound = bregman_bound(ccs)
    if bound * (1 << (n - 1)) >= (1 << 127):
        raise OverflowError("permanent bound too large for 128-bit recovery")
    if T >= 1 << 127:
        T -= 1 << 128
    if (n - 1) % 2 == 1:
        T = -T
    q, r = divmod(T, 1 << (n - 1))
    if r != 0:
        raise ArithmeticError("integer sum not divisible by 2^(n-1): oracle inconsistency")
    return q


# --------------------------------------------------------------------------
# Alg. 4, Alg. 5, structural rank
# --------------------------------------------------------------------------

def permanent_ordering(ccs):
    """Alg. 4: returns (rowPerm, colPerm) as int lists (new position -> old index)."""
    n, colptr, rowidx, _ = _ccs_args(ccs)
    rp = np.zeros(n, dtype=np.int32)
    cp = np.zeros(n, dtype=np.int32)
    rc = _load().oracle_permanent_ordering(n, _ptr(colptr, ctypes.c_int32), _ptr(rowidx, ctypes.c_int32),
                                           _ptr(rp, ctypes.c_int32), _ptr(cp, ctypes.c_int32))
    if rc != 0:
        raise ValueError("bad CCS")
    return rp.tolist(), cp.tolist()


def partitioning(ccs, tau, grratio: float = 16.0):
    """Alg. 5 on an ordered CCS.  ``tau[r]`` for r = 0..2n is the thread-count
    model.  Returns (k, c, best_score)."""
    n, colptr, rowidx, _ = _ccs_args(ccs)
    tau = _f64(tau)
    if len(tau) < 2 * n + 1:
        raise ValueError("tau needs 2n+1 entries")
    k, c, best = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    rc = _load().oracle_partitioning(n, _ptr(colptr, ctypes.c_int32), _ptr(rowidx, ctypes.c_int32),
                                     _ptr(tau, ctypes.c_double), grratio, ctypes.byref(k), ctypes.byref(c),
                                     ctypes.byref(best))
    if rc != 0:
        raise ValueError("bad CCS")
    return k.value, c.value, best.value


def structural_rank(ccs) -> int:
    n, colptr, rowidx, _ = _ccs_args(ccs)
    r = _load().oracle_structural_rank(n, _ptr(colptr, ctypes.c_int32), _ptr(rowidx, ctypes.c_int32))
    if r < 0:
        raise ValueError("bad CCS")
    return int(r)


# --------------------------------------------------------------------------
# small helpers for tests (format conversions only, no method arithmetic)
# --------------------------------------------------------------------------

def dense_to_ccs(A):
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    colptr = [0]
    rowidx, val = [], []
    for j in range(n):
        for i in range(n):
            if A[i, j] != 0.0:
                rowidx.append(i)
                val.append(A[i, j])
        colptr.append(len(rowidx))
    return n, np.array(colptr, np.int32), np.array(rowidx, np.int32), np.array(val, np.float64)


def ccs_to_dense(ccs):
    n, colptr, rowidx, val = ccs
    A = np.zeros((n, n))
    for j in range(n):
        for p in range(colptr[j], colptr[j + 1]):
            A[rowidx[p], j] = val[p]
    return A
