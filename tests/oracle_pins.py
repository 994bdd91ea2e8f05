"""Pins for the CPU oracle: checks against what the paper and the mathematics
fix, independent of the oracle's own code.  Each function takes an oracle
instance and raises AssertionError on a mismatch; test_oracle_pins runs them
on the real oracle, test_oracle_mutants on builds with planted mistakes.

Sources of truth used here:
  * the semiring definition itself (paper, Section 2.2), written out as a
    dense brute force with the same ascending-k order, so float results are
    bit-exact;
  * library routines that compute special cases independently: scipy.sparse
    products for (+,x) over float64/int64 and for the boolean pattern, and
    scipy.sparse.csgraph shortest paths for (min,+) powers (the paper,
    Section 2.2, states that min-plus powers of the adjacency matrix give
    shortest paths and the distance matrix);
  * algebraic identities: multiplicative identity, empty operands,
    associativity, the transpose identity (AB)^T = B^T A^T (Section 4.1) and
    the block (SUMMA) identity C_IJ = (+)_K A_IK B_KJ (Section 2.1);
  * hand-worked examples stored under tests/golden/.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

import synth
from helpers import (ALL, BOOL, EXACT, F32, F64, I64, MINPLUS, IN_DTYPE, assert_exact, assert_same_pattern, brute,
                     brute_merge, dense_to_rows, identity, rand_values, with_vals)

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

TINY_SHAPES = [(1, 1, 1), (5, 7, 3), (12, 12, 12), (24, 9, 17), (30, 30, 30), (3, 40, 2)]
DENSITIES = [0.0, 0.08, 0.3, 0.6]


def _tiny_pairs(seed0: int):
    s = seed0
    for (n, k, m) in TINY_SHAPES:
        for dens in DENSITIES:
            A = synth.random_small(n, k, dens, s)
            B = synth.random_small(k, m, min(1.0, dens * 1.3 + 0.02), s + 1)
            yield A, B, s
            s += 2


def pin_bruteforce(orc, sr: int):
    """Oracle == dense brute force, bit-exact (values, pattern, |.|-sums)."""
    for A, B, s in _tiny_pairs(1000 + 97 * sr):
        A = with_vals(A, sr, s + 11)
        B = with_vals(B, sr, s + 12)
        C, P, M = brute(sr, A, B)
        rp, cl, vl = dense_to_rows(C, P)
        r = orc.spgemm(sr, A, B)
        assert_same_pattern(r.rowptr, r.col, rp, cl, f"sr{sr} seed{s} pattern")
        assert_exact(r.val, vl, f"sr{sr} seed{s} values")
        if sr in (F32, F64):
            assert_exact(r.mag, M[P], f"sr{sr} seed{s} |products| sums")


def pin_row_selection(orc, sr: int):
    """Selected rows equal the same rows of the full product."""
    A = with_vals(synth.random_small(40, 30, 0.2, 5), sr, 6)
    B = with_vals(synth.random_small(30, 35, 0.2, 7), sr, 8)
    full = orc.spgemm(sr, A, B)
    rows = np.array([39, 0, 17, 17, 3], dtype=np.int64)
    part = orc.spgemm(sr, A, B, rows=rows)
    for q, i in enumerate(rows):
        a, b = full.rowptr[i], full.rowptr[i + 1]
        c, d = part.rowptr[q], part.rowptr[q + 1]
        assert np.array_equal(full.col[a:b], part.col[c:d])
        assert_exact(full.val[a:b], part.val[c:d], "row selection")


def pin_scipy_plus_times(orc):
    """(+,x) float64, float32 (as float64) and int64 against scipy.sparse on
    positive values (no cancellation, so scipy keeps the full pattern)."""
    A = synth.rmat(9, 8, seed=3)
    B = synth.er(512, 700, 6, 4)
    for sr in (F64, F32, I64):
        Av = with_vals(A, sr, 21, "positive")
        Bv = with_vals(B, sr, 22, "positive")
        dt = np.int64 if sr == I64 else np.float64
        SA = sp.csr_matrix((Av.val.astype(dt), Av.col, Av.rowptr), shape=(A.nrows, A.ncols))
        SB = sp.csr_matrix((Bv.val.astype(dt), Bv.col, Bv.rowptr), shape=(B.nrows, B.ncols))
        SC = (SA @ SB).tocsr()
        SC.sort_indices()
        r = orc.spgemm(sr, Av, Bv)
        assert_same_pattern(r.rowptr, r.col, SC.indptr, SC.indices, f"scipy sr{sr}")
        if sr == I64:
            assert np.array_equal(r.val, SC.data)
        else:
            np.testing.assert_allclose(r.val, SC.data, rtol=1e-13, atol=0)


def pin_scipy_bool(orc):
    """(or,and) pattern = structural product; value = 1 iff some product of
    true entries exists (scipy integer product of the 0/1 values > 0)."""
    A = with_vals(synth.rmat(8, 8, seed=5), BOOL, 31)
    B = with_vals(synth.rmat(8, 8, seed=6), BOOL, 32)
    ones = lambda X, v: sp.csr_matrix((v, X.col, X.rowptr), shape=(X.nrows, X.ncols))
    S = (ones(A, np.ones(A.nnz, np.int64)) @ ones(B, np.ones(B.nnz, np.int64))).tocsr()
    S.sort_indices()
    T = (ones(A, A.val.astype(np.int64)) @ ones(B, B.val.astype(np.int64))).tocsr()
    r = orc.spgemm(BOOL, A, B)
    assert_same_pattern(r.rowptr, r.col, S.indptr, S.indices, "bool pattern")
    truth = (np.asarray(T[np.repeat(np.arange(A.nrows), np.diff(r.rowptr)), r.col]).ravel() > 0).astype(np.uint8)
    assert np.array_equal(r.val, truth)


def pin_identity(orc, sr: int):
    """A (x).(+) I = I (x).(+) A = A exactly (x (x) 1 = x, one term per entry)."""
    A = with_vals(synth.rmat(7, 6, seed=40 + sr), sr, 41)
    for left in (False, True):
        r = orc.spgemm(sr, identity(A.nrows, sr), A) if left else orc.spgemm(sr, A, identity(A.ncols, sr))
        assert_same_pattern(r.rowptr, r.col, A.rowptr, A.col, "identity")
        ref = A.val
        if sr == BOOL:
            ref = (A.val != 0).astype(np.uint8)
        if sr == F32:
            ref = A.val.astype(np.float64)
        assert_exact(r.val, ref, "identity values")


def pin_empty(orc, sr: int):
    """Empty operands give an empty product of the right shape; empty rows of
    A and empty rows of B contribute nothing."""
    A = with_vals(synth.rmat(6, 4, seed=50), sr, 51)
    Z = synth.CSR(A.ncols, 33, np.zeros(A.ncols + 1, np.int64), np.zeros(0, np.int32),
                  np.zeros(0, IN_DTYPE[sr]))
    r = orc.spgemm(sr, A, Z)
    assert r.nnz == 0 and len(r.rowptr) == A.nrows + 1
    Z2 = synth.CSR(5, A.nrows, np.zeros(6, np.int64), np.zeros(0, np.int32), np.zeros(0, IN_DTYPE[sr]))
    r = orc.spgemm(sr, Z2, A)
    assert r.nnz == 0 and len(r.rowptr) == 6
    # a 0 x 0 product
    E = synth.CSR(0, 0, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, IN_DTYPE[sr]))
    r = orc.spgemm(sr, E, E)
    assert r.nnz == 0 and len(r.rowptr) == 1


def _csr_from(res, nrows, ncols):
    return synth.CSR(nrows, ncols, res.rowptr, res.col, res.val)


def pin_associativity(orc, sr: int):
    """(AB)C = A(BC), exact for int64, bool and (min,+) with integer weights."""
    style = "int" if sr == MINPLUS else "wide"
    A = with_vals(synth.random_small(20, 25, 0.15, 60), sr, 61, style)
    B = with_vals(synth.random_small(25, 18, 0.2, 62), sr, 63, style)
    C = with_vals(synth.random_small(18, 22, 0.2, 64), sr, 65, style)
    AB = _csr_from(orc.spgemm(sr, A, B), 20, 18)
    BC = _csr_from(orc.spgemm(sr, B, C), 25, 22)
    L = orc.spgemm(sr, AB, C)
    R = orc.spgemm(sr, A, BC)
    assert_same_pattern(L.rowptr, L.col, R.rowptr, R.col, "assoc")
    assert_exact(L.val, R.val, "assoc values")


def pin_transpose(orc, sr: int):
    """(AB)^T = B^T A^T for commutative (x) (paper, Section 4.1), exact for
    int64, bool and (min,+)."""
    A = with_vals(synth.rmat(7, 6, seed=70), sr, 71)
    B = with_vals(synth.er(128, 90, 5, 72), sr, 73)
    AB = _csr_from(orc.spgemm(sr, A, B), A.nrows, B.ncols)
    BtAt = orc.spgemm(sr, synth.transpose(B), synth.transpose(A))
    T = synth.transpose(AB)
    assert_same_pattern(T.rowptr, T.col, BtAt.rowptr, BtAt.col, "transpose")
    assert_exact(T.val, BtAt.val, "transpose values")


def pin_block(orc, sr: int):
    """Block identity (Sparse SUMMA, Section 2.1): with A, B cut into a g x g
    grid, C_IJ = (+)_K A_IK B_KJ; exact for int64, bool and (min,+)."""
    A = with_vals(synth.rmat(8, 8, seed=80), sr, 81)
    B = with_vals(synth.rmat(8, 8, seed=82), sr, 83)
    full = _csr_from(orc.spgemm(sr, A, B), A.nrows, B.ncols)
    g = 3
    Ab, Bb, Cb = synth.block_split(A, g), synth.block_split(B, g), synth.block_split(full, g)
    for I in range(g):
        for J in range(g):
            parts = [_csr_from(orc.spgemm(sr, Ab[I][K], Bb[K][J]), Ab[I][K].nrows, Bb[K][J].ncols) for K in range(g)]
            m = orc.merge(sr, parts)
            assert_same_pattern(m.rowptr, m.col, Cb[I][J].rowptr, Cb[I][J].col, f"block {I},{J}")
            assert_exact(m.val, Cb[I][J].val, f"block {I},{J} values")


def pin_invariants(orc):
    """Cheap whole-matrix invariants: int64 C.1 = A.(B.1) with wrap-around;
    all-ones int64 row sums = products per row; (min,+) row minima
    min_j C_ij = min_k (a_ik + min_j b_kj); bool row non-empty iff some
    k in A_i has a non-empty B_k."""
    A = synth.rmat(9, 8, seed=90)
    B = synth.rmat(9, 8, seed=91)
    rows_of = lambda X: np.repeat(np.arange(X.nrows), np.diff(X.rowptr))
    # int64 row sums
    Av, Bv = with_vals(A, I64, 92), with_vals(B, I64, 93)
    r = orc.spgemm(I64, Av, Bv)
    with np.errstate(over="ignore"):
        b1 = np.zeros(B.nrows, np.uint64)
        np.add.at(b1, rows_of(Bv), Bv.val.view(np.uint64))
        ab1 = np.zeros(A.nrows, np.uint64)
        np.add.at(ab1, rows_of(Av), Av.val.view(np.uint64) * b1[Av.col])
        c1 = np.zeros(A.nrows, np.uint64)
        np.add.at(c1, np.repeat(np.arange(A.nrows), np.diff(r.rowptr)), r.val.view(np.uint64))
    assert np.array_equal(c1, ab1), "int64 row sums"
    # all-ones: row sums equal products per row
    ones = lambda X: X.with_values(np.ones(X.nnz, np.int64))
    r = orc.spgemm(I64, ones(A), ones(B))
    p = np.zeros(A.nrows, np.int64)
    np.add.at(p, rows_of(A), np.diff(B.rowptr)[A.col])
    c1 = np.zeros(A.nrows, np.int64)
    np.add.at(c1, np.repeat(np.arange(A.nrows), np.diff(r.rowptr)), r.val)
    assert np.array_equal(c1, p), "all-ones row sums"
    # (min,+) row minima
    Av, Bv = with_vals(A, MINPLUS, 94), with_vals(B, MINPLUS, 95)
    r = orc.spgemm(MINPLUS, Av, Bv)
    bmin = np.full(B.nrows, np.inf, np.float32)
    np.minimum.at(bmin, rows_of(Bv), Bv.val)
    cand = (Av.val + bmin[Av.col]).astype(np.float32)
    amin = np.full(A.nrows, np.inf, np.float32)
    np.minimum.at(amin, rows_of(Av), cand)
    cmin = np.full(A.nrows, np.inf, np.float32)
    np.minimum.at(cmin, np.repeat(np.arange(A.nrows), np.diff(r.rowptr)), r.val)
    assert np.array_equal(cmin, amin), "(min,+) row minima"
    # bool row non-empty
    Av, Bv = with_vals(A, BOOL, 96), with_vals(B, BOOL, 97)
    r = orc.spgemm(BOOL, Av, Bv)
    has = np.zeros(A.nrows, bool)
    np.logical_or.at(has, rows_of(A), np.diff(B.rowptr)[A.col] > 0)
    assert np.array_equal(np.diff(r.rowptr) > 0, has), "bool non-empty rows"


def pin_shortest_paths(orc):
    """(min,+) powers: with the identity (0 on the diagonal) merged into W,
    repeated squaring of (I (+) W) reaches the all-pairs distance matrix
    (paper, Section 2.2), checked against scipy's shortest paths."""
    n = 70
    W = synth.random_small(n, n, 0.05, 100)
    W = W.with_values(rand_values(MINPLUS, W.nnz, 101, "int"))
    I = identity(n, MINPLUS)
    X = _csr_from(orc.merge(MINPLUS, [I, W]), n, n)
    steps = 1
    while steps < n - 1:
        X = _csr_from(orc.spgemm(MINPLUS, X, X), n, n)
        steps *= 2
    dense = sp.csr_matrix((W.val.astype(np.float64), W.col, W.rowptr), shape=(n, n))
    D = shortest_path(dense, method="FW", directed=True)
    got = np.full((n, n), np.inf)
    rr = np.repeat(np.arange(n), np.diff(X.rowptr))
    got[rr, X.col] = X.val
    assert np.array_equal(got, D), "min-plus powers vs shortest paths"


def pin_merge(orc, sr: int):
    """Merge == dense brute-force fold over the parts in order; a single part
    merges to itself; scipy sum for float64."""
    parts = [with_vals(synth.random_small(26, 31, d, 110 + q), sr, 120 + q) for q, d in
             enumerate([0.1, 0.0, 0.3, 0.05, 0.2])]
    C, P = brute_merge(sr, parts)
    rp, cl, vl = dense_to_rows(C, P)
    m = orc.merge(sr, parts)
    assert_same_pattern(m.rowptr, m.col, rp, cl, f"merge sr{sr}")
    assert_exact(m.val, vl, f"merge sr{sr} values")
    one = orc.merge(sr, parts[:1])
    assert_same_pattern(one.rowptr, one.col, parts[0].rowptr, parts[0].col, "merge of one")
    if sr == F64:
        S = sum(sp.csr_matrix((p.val, p.col, p.rowptr), shape=(p.nrows, p.ncols)) for p in parts).tocsr()
        S.sort_indices()
        dense_s = S.toarray()
        rr = np.repeat(np.arange(26), np.diff(m.rowptr))
        np.testing.assert_allclose(m.val, dense_s[rr, m.col], rtol=1e-14, atol=1e-15)


def _read_golden(name):
    mats = {}
    cur = None
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            if line.startswith("["):
                cur = line.strip("[]")
                mats[cur] = []
            else:
                mats[cur].append([float("inf") if t == "." else float(t) for t in line.split()])
    return {k: np.array(v) for k, v in mats.items()}


def _dense_to_csr(D, absent):
    present = ~np.isinf(D) if absent == "inf" else (D != 0)
    rowptr = np.zeros(D.shape[0] + 1, np.int64)
    np.cumsum(present.sum(axis=1), out=rowptr[1:])
    r, c = np.nonzero(present)
    return synth.CSR(D.shape[0], D.shape[1], rowptr, c.astype(np.int32), D[r, c]), present


def pin_golden(orc):
    """Hand-worked examples (tests/golden/*.txt)."""
    g = _read_golden("minplus_4node.txt")
    W, _ = _dense_to_csr(g["W"], "inf")
    W = W.with_values(W.val.astype(np.float32))
    r = orc.spgemm(MINPLUS, W, W)
    got = np.full(g["W2"].shape, np.inf)
    got[np.repeat(np.arange(4), np.diff(r.rowptr)), r.col] = r.val
    assert np.array_equal(got, g["W2"]), "hand-worked W^2"
    g = _read_golden("plus_times_3x3.txt")
    A, _ = _dense_to_csr(g["A"], "zero")
    B, _ = _dense_to_csr(g["B"], "zero")
    r = orc.spgemm(I64, A.with_values(A.val.astype(np.int64)), B.with_values(B.val.astype(np.int64)))
    got = np.zeros(g["C"].shape)
    got[np.repeat(np.arange(3), np.diff(r.rowptr)), r.col] = r.val
    assert np.array_equal(got, g["C"]), "hand-worked 3x3 product"
    # pattern of the 3x3 example is structural: the (1,1) entry cancels to 0
    # yet stays stored
    assert r.nnz == int(g["PATTERN_NNZ"][0][0])


def all_pins():
    """(name, callable(orc)) for every pin."""
    out = []
    for sr in ALL:
        out.append((f"bruteforce_sr{sr}", lambda o, sr=sr: pin_bruteforce(o, sr)))
        out.append((f"rowsel_sr{sr}", lambda o, sr=sr: pin_row_selection(o, sr)))
        out.append((f"identity_sr{sr}", lambda o, sr=sr: pin_identity(o, sr)))
        out.append((f"empty_sr{sr}", lambda o, sr=sr: pin_empty(o, sr)))
        out.append((f"merge_sr{sr}", lambda o, sr=sr: pin_merge(o, sr)))
    for sr in EXACT:
        out.append((f"assoc_sr{sr}", lambda o, sr=sr: pin_associativity(o, sr)))
        out.append((f"transpose_sr{sr}", lambda o, sr=sr: pin_transpose(o, sr)))
        out.append((f"block_sr{sr}", lambda o, sr=sr: pin_block(o, sr)))
    out.append(("scipy_plus_times", pin_scipy_plus_times))
    out.append(("scipy_bool", pin_scipy_bool))
    out.append(("invariants", pin_invariants))
    out.append(("shortest_paths", pin_shortest_paths))
    out.append(("golden", pin_golden))
    out.append(("power_minplus", pin_power_minplus))
    out.append(("power_bool_int", pin_power_bool_int))
    out.append(("dcsc", pin_dcsc))
    out.append(("user_semirings", pin_user_semirings))
    return out


# ---- powers (paper, Section 2.2) -------------------------------------------------

def _bellman_ford_rounds(n, W, rounds):
    """All-pairs lightest paths of at most `rounds` edges by synchronous
    Bellman-Ford relaxation over W's edge list (a textbook algorithm, not a
    matrix product): distance 0 to itself, +inf elsewhere, then `rounds`
    rounds in which every edge (u, v, w) offers d[s, u] + w to d[s, v]."""
    u = np.repeat(np.arange(n), np.diff(W.rowptr))
    v = W.col.astype(np.int64)
    w = W.val.astype(np.float64)
    d = np.full((n, n), np.inf)
    np.fill_diagonal(d, 0.0)
    for _ in range(rounds):
        nd = d.copy()
        for e in range(len(u)):
            np.minimum(nd[:, v[e]], d[:, u[e]] + w[e], out=nd[:, v[e]])
        d = nd
    return d


def _dense_of(M, absent):
    d = np.full((M.nrows, M.ncols), absent, dtype=np.float64)
    d[np.repeat(np.arange(M.nrows), np.diff(M.rowptr)), M.col] = M.val
    return d


def pin_power_minplus(orc):
    """(min,+) powers of I (+) W: k linear steps equal k rounds of
    Bellman-Ford; squaring to the fixed point equals scipy's all-pairs
    shortest paths (the distance matrix) and agrees with linear steps."""
    from oracle import power as pw
    n = 48
    W = synth.random_small(n, n, 0.06, 500)
    W = W.with_values(rand_values(MINPLUS, W.nnz, 501, "int"))
    for k in (1, 2, 3, 5):
        r = pw.power(orc, MINPLUS, W, k, self_loops=True)
        assert r.hops == k and r.products == k - 1
        assert np.array_equal(_dense_of(r.D, np.inf), _bellman_ford_rounds(n, W, k)), f"(min,+) {k} hops"
    fix = pw.power(orc, MINPLUS, W, 0, self_loops=True, squaring=True, fixpoint=True)
    assert fix.converged
    dense = sp.csr_matrix((W.val.astype(np.float64), W.col, W.rowptr), shape=(n, n))
    assert np.array_equal(_dense_of(fix.D, np.inf), shortest_path(dense, method="D", directed=True))
    lin = pw.power(orc, MINPLUS, W, 0, self_loops=True, fixpoint=True)
    assert lin.converged and pw.same(lin.D, fix.D)
    sq4 = pw.power(orc, MINPLUS, W, 4, self_loops=True, squaring=True)
    assert sq4.hops == 4 and sq4.products == 2
    assert pw.same(sq4.D, pw.power(orc, MINPLUS, W, 4, self_loops=True).D)
    # every pair i < j joined directly (heavy edge, weight 10 (j - i)^2) and
    # through the chain of unit edges: the pattern of the powers is final at
    # once, the values keep falling until paths of 7 edges are allowed
    m = 8
    iu, ju = np.triu_indices(m, 1)
    Wt = synth.CSR(m, m, np.concatenate([[0], np.cumsum(np.bincount(iu, minlength=m))]).astype(np.int64),
                   ju.astype(np.int32), np.where(ju - iu == 1, 1.0, 10.0 * (ju - iu) ** 2).astype(np.float32))
    fix = pw.power(orc, MINPLUS, Wt, 0, self_loops=True, squaring=True, fixpoint=True)
    ref = np.where(np.arange(m)[None, :] >= np.arange(m)[:, None], np.arange(m)[None, :] - np.arange(m)[:, None], np.inf)
    assert fix.converged and np.array_equal(_dense_of(fix.D, np.inf), ref), "values fall after the pattern is final"
    # without self loops: walks of exactly two edges (the hand-worked golden)
    g = _read_golden("minplus_4node.txt")
    W4, _ = _dense_to_csr(g["W"], "inf")
    r = pw.power(orc, MINPLUS, W4.with_values(W4.val.astype(np.float32)), 2)
    assert np.array_equal(_dense_of(r.D, np.inf), g["W2"])


def pin_power_bool_int(orc):
    """(or,and) closure of I (+) W = reachability (scipy breadth-first
    shortest paths are finite); (+,x) int64 W^k = numpy's integer matrix
    power (walk counts); float64 W^3 = scipy's sparse product chain."""
    from oracle import power as pw
    n = 40
    W = synth.random_small(n, n, 0.05, 510)
    Wb = W.with_values(np.ones(W.nnz, np.uint8))
    fix = pw.power(orc, BOOL, Wb, 0, self_loops=True, squaring=True, fixpoint=True)
    assert fix.converged
    reach = np.isfinite(shortest_path(sp.csr_matrix((np.ones(W.nnz), W.col, W.rowptr), shape=(n, n)),
                                      unweighted=True, directed=True))
    got = _dense_of(fix.D, 0) != 0
    assert np.array_equal(got, reach), "(or,and) closure"
    assert fix.D.nrows == n and len(fix.D.col) == int(reach.sum())
    Wi = W.with_values(rand_values(I64, W.nnz, 511, "positive"))
    r = pw.power(orc, I64, Wi, 4)
    dense = np.zeros((n, n), np.int64)
    dense[np.repeat(np.arange(n), np.diff(W.rowptr)), W.col] = Wi.val
    ref = np.linalg.matrix_power(dense, 4)
    got = np.zeros((n, n), np.int64)
    got[np.repeat(np.arange(n), np.diff(r.D.rowptr)), r.D.col] = r.D.val
    assert np.array_equal(got, ref), "(+,x) int64 W^4"
    Wf = W.with_values(rand_values(F64, W.nnz, 512, "positive"))
    r = pw.power(orc, F64, Wf, 3)
    S = sp.csr_matrix((Wf.val, W.col, W.rowptr), shape=(n, n))
    S3 = (S @ S @ S).tocsr()
    S3.sort_indices()
    assert np.array_equal(r.D.rowptr, S3.indptr) and np.array_equal(r.D.col, S3.indices)
    np.testing.assert_allclose(r.D.val, S3.data, rtol=1e-13)


# ---- DCSC / CSC adapter (paper, Section 4.1) -------------------------------------

def pin_dcsc(orc):
    """Decompression and compression against the hand-worked example and
    against scipy's column pointers of a hypersparse matrix (non-empty
    columns taken from its coordinate list); CSC products against scipy."""
    from oracle import dcsc as dc
    g = _read_golden("dcsc_4x7.txt")
    jc = g["JC"][0].astype(np.int32)
    cp = g["CP"][0].astype(np.int64)
    assert np.array_equal(dc.decompress(7, jc, cp), g["COLPTR"][0].astype(np.int64))
    j2, c2 = dc.compress(g["COLPTR"][0].astype(np.int64))
    assert np.array_equal(j2, jc) and np.array_equal(c2, cp)
    A = sp.csc_matrix(g["A"])
    assert np.array_equal(A.indptr, g["COLPTR"][0]) and np.array_equal(A.indices, g["IR"][0])
    # hypersparse: 60 x 3000 with ~90 entries, most columns empty
    H = sp.random(60, 3000, density=0.0005, format="coo", random_state=np.random.RandomState(7))
    Hc = H.tocsc()
    Hc.sort_indices()
    cols, counts = np.unique(H.col, return_counts=True)
    cp_h = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    assert np.array_equal(dc.decompress(3000, cols.astype(np.int32), cp_h), Hc.indptr)
    j3, c3 = dc.compress(Hc.indptr)
    assert np.array_equal(j3, cols) and np.array_equal(c3, cp_h)
    # CSC products (A is 50 x 70, B is 70 x 40, positive values: no cancellation)
    rs = np.random.RandomState(8)
    Ad = sp.random(50, 70, density=0.08, format="csc", random_state=rs, data_rvs=lambda k: rs.uniform(0.5, 2, k))
    Bd = sp.random(70, 40, density=0.08, format="csc", random_state=rs, data_rvs=lambda k: rs.uniform(0.5, 2, k))
    for M in (Ad, Bd):
        M.sort_indices()
    Acsc = dc.Csc(50, 70, Ad.indptr.astype(np.int64), Ad.indices.astype(np.int32), Ad.data)
    Bcsc = dc.Csc(70, 40, Bd.indptr.astype(np.int64), Bd.indices.astype(np.int32), Bd.data)
    Ar = dc.csc_to_csr(Acsc)
    Acr = Ad.tocsr()
    Acr.sort_indices()
    assert np.array_equal(Ar.rowptr, Acr.indptr) and np.array_equal(Ar.col, Acr.indices)
    C = dc.csc_spgemm(orc, F64, Acsc, Bcsc)
    R = (Ad @ Bd).tocsc()
    R.sort_indices()
    assert np.array_equal(C.colptr, R.indptr) and np.array_equal(C.row, R.indices)
    np.testing.assert_allclose(C.val, R.data, rtol=1e-14)
    Ci = dc.csc_spgemm(orc, I64, dc.Csc(50, 70, Acsc.colptr, Acsc.row, np.round(Ad.data * 4).astype(np.int64)),
                       dc.Csc(70, 40, Bcsc.colptr, Bcsc.row, np.round(Bd.data * 4).astype(np.int64)))
    Ri = (sp.csc_matrix((np.round(Ad.data * 4), Ad.indices, Ad.indptr), shape=(50, 70)) @
          sp.csc_matrix((np.round(Bd.data * 4), Bd.indices, Bd.indptr), shape=(70, 40))).tocsc()
    Ri.sort_indices()
    assert np.array_equal(Ci.colptr, Ri.indptr) and np.array_equal(Ci.val, Ri.data.astype(np.int64))
    # a square pair: A.B differs from B.A, so operand order is pinned too
    Sq = sp.random(30, 30, density=0.1, format="csc", random_state=rs, data_rvs=lambda k: rs.uniform(0.5, 2, k))
    Tq = sp.random(30, 30, density=0.1, format="csc", random_state=rs, data_rvs=lambda k: rs.uniform(0.5, 2, k))
    for M in (Sq, Tq):
        M.sort_indices()
    C = dc.csc_spgemm(orc, F64, dc.Csc(30, 30, Sq.indptr.astype(np.int64), Sq.indices.astype(np.int32), Sq.data),
                      dc.Csc(30, 30, Tq.indptr.astype(np.int64), Tq.indices.astype(np.int32), Tq.data))
    R = (Sq @ Tq).tocsc()
    R.sort_indices()
    assert np.array_equal(C.colptr, R.indptr) and np.array_equal(C.row, R.indices)
    np.testing.assert_allclose(C.val, R.data, rtol=1e-14)


# ---- semirings a user defines (paper, Section 2.2) ---------------------------------

def _dense_pair(A, B, absent):
    da = np.full((A.nrows, A.ncols), absent, dtype=np.float64)
    db = np.full((B.nrows, B.ncols), absent, dtype=np.float64)
    da[np.repeat(np.arange(A.nrows), np.diff(A.rowptr)), A.col] = A.val
    db[np.repeat(np.arange(B.nrows), np.diff(B.rowptr)), B.col] = B.val
    ma = np.zeros(da.shape, bool)
    mb = np.zeros(db.shape, bool)
    ma[np.repeat(np.arange(A.nrows), np.diff(A.rowptr)), A.col] = True
    mb[np.repeat(np.arange(B.nrows), np.diff(B.rowptr)), B.col] = True
    return da, db, ma, mb


def pin_user_semirings(orc):
    """(max,+) f32 is (min,+) of the negated operands, negated, bit for bit
    (negation commutes with rounding and swaps min and max); (max,x) f64 and
    (min,max) int64 equal numpy's dense reductions over k (maximum of the
    rounded products; minimum of the pairwise maxima) on the stored pairs."""
    import oracle as o
    A = synth.rmat(9, 8, seed=600)
    B = synth.er(512, 300, 5, 601)
    av = synth.values(synth.VAL_F32_UNIFORM, A.nnz, -50.0, 100.0, 602)
    bv = synth.values(synth.VAL_F32_UNIFORM, B.nnz, -50.0, 100.0, 603)
    mx = orc.spgemm(o.MAX_PLUS_F32, A.with_values(av), B.with_values(bv))
    mn = orc.spgemm(MINPLUS, A.with_values(-av), B.with_values(-bv))
    assert_same_pattern(mx.rowptr, mx.col, mn.rowptr, mn.col, "(max,+) pattern")
    assert np.array_equal((-mn.val).view(np.uint32), mx.val.view(np.uint32)), "(max,+) = -(min,+)(-A,-B)"
    # tiny dense checks
    for s, (n, k, m) in enumerate([(7, 9, 6), (12, 5, 11), (20, 20, 20)]):
        At = synth.random_small(n, k, 0.3, 610 + s)
        Bt = synth.random_small(k, m, 0.3, 620 + s)
        At = At.with_values(synth.values(synth.VAL_F64_UNIFORM, At.nnz, 0.5, 2.0, 630 + s))
        Bt = Bt.with_values(synth.values(synth.VAL_F64_UNIFORM, Bt.nnz, 0.5, 2.0, 640 + s))
        da, db, ma, mb = _dense_pair(At, Bt, 0.0)
        pair = ma[:, :, None] & mb[None, :, :]
        prod = np.where(pair, da[:, :, None] * db[None, :, :], -np.inf)
        ref = prod.max(axis=1)
        r = orc.spgemm(o.MAX_TIMES_F64, At, Bt)
        got = np.full((n, m), -np.inf)
        got[np.repeat(np.arange(n), np.diff(r.rowptr)), r.col] = r.val
        assert np.array_equal(got, ref), "(max,x) f64 dense"
        Ai = At.with_values(synth.values(synth.VAL_I64_UNIFORM, At.nnz, -1000, 1000, 650 + s))
        Bi = Bt.with_values(synth.values(synth.VAL_I64_UNIFORM, Bt.nnz, -1000, 1000, 660 + s))
        da, db, ma, mb = _dense_pair(Ai, Bi, 0)
        big = np.iinfo(np.int64).max
        mm = np.where(pair, np.maximum(da[:, :, None], db[None, :, :]), np.inf)
        ref = mm.min(axis=1)
        r = orc.spgemm(o.MIN_MAX_I64, Ai, Bi)
        got = np.full((n, m), np.inf)
        got[np.repeat(np.arange(n), np.diff(r.rowptr)), r.col] = r.val
        assert np.array_equal(got, ref) and big > 0, "(min,max) int64 dense"
    # merges fold with the semiring's (+)
    parts = [synth.random_small(15, 17, 0.3, 670 + q) for q in range(3)]
    parts = [p.with_values(synth.values(synth.VAL_I64_UNIFORM, p.nnz, -9, 9, 680 + q)) for q, p in enumerate(parts)]
    m = orc.merge(o.MIN_MAX_I64, parts)
    dense = np.full((3, 15, 17), np.inf)
    for q, p in enumerate(parts):
        dense[q][np.repeat(np.arange(15), np.diff(p.rowptr)), p.col] = p.val
    ref = dense.min(axis=0)
    got = np.full((15, 17), np.inf)
    got[np.repeat(np.arange(15), np.diff(m.rowptr)), m.col] = m.val
    assert np.array_equal(got, ref), "(min,max) merge"
