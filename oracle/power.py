"""Powers of a square matrix over a semiring, by repeated products of the
CPU oracle.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle``): used by the tests and
the CPU-baseline leg of ``bench.py``, never by the GPU library.

What it computes (paper, Section 2.2): over (min,+) the k-th power of a
weighted adjacency matrix W holds the lightest walk of exactly k edges
between two vertices; with the semiring one (+0.0) on the diagonal, i.e. the
powers of I (+) W, walks may stay put, so the k-th power holds the shortest
path of at most k edges, and the powers stop changing once k reaches the
longest shortest path: that fixed point is the distance matrix.  The same
construction over (or,and) gives reachability within k steps (the transitive
closure at the fixed point) and over (+,x) the number of walks of k edges.

Steps, in the order the definition gives them:
  W' = I (+) W      (merge with the identity, when self loops are asked for)
  D_1 = W'
  D_{h+1} = D_h (x).(+) W'          (linear: one more edge per product), or
  D_{2h}  = D_h (x).(+) D_h         (squaring: W'^(2h) = W'^h W'^h)
until h reaches max_hops, or, when asked, until a product equals its left
operand (pattern and value bits), which is then the fixed point.

For (+,x) float32 each product is computed by the oracle in float64 and
rounded to float32 before the next one.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import IN_DTYPE, Oracle

# test-only planted mistakes (tests/test_oracle_mutants.py): 0 = none
MUTANT = 0

# the multiplicative identity of each semiring
ONE = {1: 1, 2: 1.0, 3: 1.0, 4: 1, 5: 0.0}


@dataclass
class Mat:
    nrows: int
    ncols: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray


@dataclass
class PowerResult:
    D: Mat
    hops: int
    products: int
    converged: bool


def identity(n: int, sr: int) -> Mat:
    return Mat(n, n, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32),
               np.full(n, ONE[sr], dtype=IN_DTYPE[sr]))


def _mat(res, n: int, sr: int) -> Mat:
    return Mat(n, n, res.rowptr, res.col, res.val.astype(IN_DTYPE[sr]))


def same(X: Mat, Y: Mat) -> bool:
    """Equal pattern and equal value bits."""
    if not (np.array_equal(X.rowptr, Y.rowptr) and np.array_equal(X.col, Y.col)):
        return False
    if MUTANT == 3:
        return True
    return X.val.tobytes() == Y.val.tobytes()


def power(orc: Oracle, sr: int, W, max_hops: int, self_loops: bool = False, squaring: bool = False,
          fixpoint: bool = False) -> PowerResult:
    """D = W'^h for the h described above; max_hops <= 0 means twice the
    matrix size: a shortest path has fewer than n edges, so with self loops
    the powers are final by then and one more product shows it."""
    n = W.nrows
    if W.ncols != n:
        raise ValueError("W must be square")
    Wv = Mat(n, n, W.rowptr, W.col, np.asarray(W.val, dtype=IN_DTYPE[sr]))
    if self_loops and MUTANT != 2:
        Wp = _mat(orc.merge(sr, [identity(n, sr), Wv]), n, sr)
    else:
        Wp = Wv
    limit = max_hops if max_hops > 0 else 2 * max(n, 1)
    D, hops, products, converged = Wp, 1, 0, False
    while hops < limit:
        right = D if (squaring or MUTANT == 1) else Wp
        X = _mat(orc.spgemm(sr, D, right), n, sr)
        products += 1
        hops = 2 * hops if squaring else hops + 1
        stop = fixpoint and same(X, D)
        D = X
        if stop:
            converged = True
            break
    return PowerResult(D, hops, products, converged)
