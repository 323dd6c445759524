"""Seeded synthetic inputs (sparse n x n matrices in CCS form).

This module only draws random matrices.  It holds none of the permanent's
arithmetic, imports nothing from the HIP path or from the oracle, and is the
one piece of code that both sides of every parity test share.

A CCS is a tuple ``(n, colptr, rowidx, val)``: ``colptr`` int32[n+1],
``rowidx`` int32[nnz] (ascending inside each column), ``val`` float64[nnz].

Workloads (the paper's synthetic model is Erdos-Renyi with U[0,1] values,
Sec. VI-C; its real-life matrices are SuiteSparse matrices that are not used
here -- these seeded generators stand in for them):

* ``single_01(n, p, seed)``       a random permutation matrix OR'd with
  Bernoulli(p) entries, values 1.0 (n=24 p=0.15 and n=40 p=0.10 workloads).
* ``single_real(n, p, seed)``     the same pattern, values U(0,1) (n=36 p=0.30).
* ``batch_matrix(seed, i)``       one matrix of the 2000-matrix batch:
  n ~ U{16..30}, p ~ U[0.15,0.40], Bernoulli(p) pattern, values U(-1,1),
  no forced diagonal.
* ``serving_trace(seed, ...)``    Poisson arrivals with mixed-size requests.
* ``erdos_renyi(n, p, seed)``     the paper's own synthetic model: Bernoulli(p)
  pattern, U[0,1] values, rejected until structurally nonsingular.

Draw order for every generator is fixed: permutation (if any), then the n x n
uniform matrix for the pattern (row-major), then one value per stored entry in
CCS order (column by column, ascending row).
"""
from __future__ import annotations

import numpy as np


def _pattern_to_ccs(mask: np.ndarray, values: np.ndarray | None):
    n = mask.shape[0]
    colptr = np.zeros(n + 1, dtype=np.int32)
    rows = []
    for j in range(n):
        r = np.nonzero(mask[:, j])[0]
        rows.append(r)
        colptr[j + 1] = colptr[j] + len(r)
    rowidx = np.concatenate(rows).astype(np.int32) if n else np.zeros(0, np.int32)
    if values is None:
        val = np.ones(len(rowidx), dtype=np.float64)
    else:
        val = np.asarray(values, dtype=np.float64)
        assert len(val) == len(rowidx)
    return n, colptr, rowidx, val


def _pattern(rng: np.random.Generator, n: int, p: float, diag: bool) -> np.ndarray:
    pi = rng.permutation(n) if diag else None
    mask = rng.random((n, n)) < p
    if diag:
        mask[np.arange(n), pi] = True
    return mask


def single_01(n: int, p: float, seed: int):
    """Permutation matrix OR Bernoulli(p), all stored values 1.0."""
    rng = np.random.default_rng(seed)
    mask = _pattern(rng, n, p, diag=True)
    return _pattern_to_ccs(mask, None)


def single_real(n: int, p: float, seed: int):
    """Permutation matrix OR Bernoulli(p), values U(0,1)."""
    rng = np.random.default_rng(seed)
    mask = _pattern(rng, n, p, diag=True)
    nnz = int(mask.sum())
    return _pattern_to_ccs(mask, rng.random(nnz))


def random_sparse(n: int, p: float, seed: int, kind: str = "real", diag: bool = True,
                  lo: float = 0.0, hi: float = 1.0):
    """General helper: kind in {"01", "real", "signed"}; signed draws U(-1,1)."""
    rng = np.random.default_rng(seed)
    mask = _pattern(rng, n, p, diag=diag)
    nnz = int(mask.sum())
    if kind == "01":
        return _pattern_to_ccs(mask, None)
    if kind == "signed":
        return _pattern_to_ccs(mask, rng.uniform(-1.0, 1.0, nnz))
    return _pattern_to_ccs(mask, rng.uniform(lo, hi, nnz))


def batch_matrix(seed: int, i: int):
    """Matrix i of the batch workload: n ~ U{16..30}, density ~ U[0.15, 0.40],
    values U(-1, 1), no forced diagonal (structurally singular draws occur)."""
    rng = np.random.default_rng([seed, i])
    n = int(rng.integers(16, 31))
    d = float(rng.uniform(0.15, 0.40))
    mask = rng.random((n, n)) < d
    nnz = int(mask.sum())
    return _pattern_to_ccs(mask, rng.uniform(-1.0, 1.0, nnz))


def batch(seed: int, count: int = 2000):
    return [batch_matrix(seed, i) for i in range(count)]


def serving_request(seed: int, i: int):
    """Request i of the serving workload: n ~ U{12..36}, density ~ U[0.10, 0.35],
    0/1 values with probability 0.7 else U(0,1), no forced diagonal."""
    rng = np.random.default_rng([seed, 1_000_003, i])
    n = int(rng.integers(12, 37))
    d = float(rng.uniform(0.10, 0.35))
    binary = bool(rng.random() < 0.7)
    mask = rng.random((n, n)) < d
    nnz = int(mask.sum())
    vals = None if binary else rng.random(nnz)
    return _pattern_to_ccs(mask, vals)


def serving_trace(seed: int, rate_hz: float = 200.0, duration_s: float = 60.0):
    """Poisson arrival times (seconds) for the serving workload."""
    rng = np.random.default_rng([seed, 7])
    t, out = 0.0, []
    while True:
        t += float(rng.exponential(1.0 / rate_hz))
        if t >= duration_s:
            return np.array(out)
        out.append(t)


def _structurally_nonsingular(mask: np.ndarray) -> bool:
    # Kuhn's augmenting paths; used only to reject draws, as the paper does.
    n = mask.shape[0]
    match = [-1] * n

    def try_col(j, seen):
        for i in np.nonzero(mask[:, j])[0]:
            if not seen[i]:
                seen[i] = True
                if match[i] < 0 or try_col(match[i], seen):
                    match[i] = j
                    return True
        return False

    return all(try_col(j, [False] * n) for j in range(n))


def erdos_renyi(n: int, p: float, seed: int):
    """The paper's synthetic model: Bernoulli(p) pattern with U[0,1] values,
    redrawn until structurally nonsingular."""
    rng = np.random.default_rng(seed)
    while True:
        mask = rng.random((n, n)) < p
        if _structurally_nonsingular(mask):
            return _pattern_to_ccs(mask, rng.random(int(mask.sum())))


# The paper's synthetic grid (Sec. VI-C, Table 3): n in {40, 45, 48}, p in
# {0.1, ..., 0.5}, U[0,1] values, structurally nonsingular.
ER_GRID = [(n, p) for n in (40, 45, 48) for p in (0.1, 0.2, 0.3, 0.4, 0.5)]


def er_grid_matrix(n: int, p: float, seed: int = 1):
    """Cell (n, p) of the grid; the generator is seeded with [seed, n, 10 p]."""
    return erdos_renyi(n, p, [seed, n, int(round(10 * p))])


# The single-matrix workloads at full size, keyed by a descriptive name.
WORKLOADS = {
    "n24_p0.15_01": lambda seed=1: single_01(24, 0.15, seed),
    "n36_p0.30_real": lambda seed=1: single_real(36, 0.30, seed),
    "n40_p0.10_01": lambda seed=1: single_01(40, 0.10, seed),
    # a 0/1 matrix whose FP64 rounding error reaches units (exact-mode test case)
    "n36_p0.15_01": lambda seed=1: single_01(36, 0.15, seed),
}
