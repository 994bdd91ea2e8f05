"""GPU parity of the column-major adapter (paper, Section 4.1, Algorithm 1)
and of the power driver (Section 2.2) against the CPU oracle: DCSC column
pointers decompressed and compressed exactly, products of CSC operands, and
semiring powers (k hops, squarings, the distance matrix / transitive closure
at the fixed point)."""
import numpy as np
import pytest

import oracle
import synth
from oracle import dcsc as odc
from oracle import power as opw
from helpers import ALL, BOOL, EXACT, F32, F64, I64, IN_DTYPE, MINPLUS, assert_exact, with_vals

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import paper_2504_06408_amd as sg
    hd = sg.Handle(0)
    yield hd
    hd.close()


def _t(a, dtype=None):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a if dtype is None else np.asarray(a, dtype=dtype))).to("cuda")


def _csc_of(A):
    """Host CSC (oracle transposition) of a synth CSR."""
    return odc.csr_to_csc(A)


def _hypersparse_block(scale, grid, bi, bj, sr, seed):
    """One block of an R-MAT matrix cut into a grid x grid block grid
    (block-local columns): most of its columns are empty."""
    A = synth.rmat(scale, 16, seed=seed)
    blocks = synth.block_split(A, grid)
    B = blocks[bi][bj]
    return with_vals(B, sr, seed + 1, "positive")


@pytest.mark.parametrize("case", ["rmat_block", "empty_cols", "one_col", "all_full"])
def test_dcsc_decompress_compress(h, case):
    if case == "rmat_block":
        M = _hypersparse_block(14, 8, 6, 7, F64, 40)
    elif case == "empty_cols":
        M = synth.CSR(5, 9, np.zeros(6, np.int64), np.zeros(0, np.int32), np.zeros(0))
    elif case == "one_col":
        M = synth.random_small(40, 1, 0.5, 41)
        M = M.with_values(np.ones(M.nnz))
    else:
        M = synth.random_small(30, 25, 0.9, 42)
        M = M.with_values(np.ones(M.nnz))
    C = _csc_of(M)
    jc, cp = odc.compress(C.colptr)
    assert np.array_equal(odc.decompress(M.ncols, jc, cp), C.colptr)
    got = h.dcsc_decompress(M.nrows, M.ncols, _t(jc, np.int32), _t(cp, np.int64), _t(C.row, np.int32),
                            _t(C.val, np.float64))
    assert np.array_equal(got.colptr.cpu().numpy(), odc.decompress(M.ncols, jc, cp)), "decompressed column pointers"
    gjc, gcp = h.dcsc_compress(_t(C.colptr, np.int64))
    assert np.array_equal(gjc.cpu().numpy(), jc) and np.array_equal(gcp.cpu().numpy(), cp), "compressed columns"


def _close(sr, got, ref, what):
    if sr in EXACT:
        assert_exact(np.asarray(got), np.asarray(ref, dtype=IN_DTYPE[sr]), what)
    else:
        tol = 1e-12 if sr == F64 else 1e-5
        np.testing.assert_allclose(np.asarray(got, np.float64), np.asarray(ref, np.float64), rtol=tol, err_msg=what)


@pytest.mark.parametrize("sr", ALL)
def test_csc_product(h, sr):
    """C = A.B with A (R-MAT s11, rows spanning every path) and B (ER,
    20,000 columns: two column tiles) given in CSC; C comes out in CSC."""
    import paper_2504_06408_amd as sg
    A = with_vals(synth.rmat(11, 16, seed=50), sr, 51, "positive")
    B = with_vals(synth.er(2048, 20000, 24, 52), sr, 53, "positive")
    Ac, Bc = _csc_of(A), _csc_of(B)
    dA = sg.DeviceCSC(A.nrows, A.ncols, _t(Ac.colptr, np.int64), _t(Ac.row, np.int32), _t(Ac.val))
    dB = sg.DeviceCSC(B.nrows, B.ncols, _t(Bc.colptr, np.int64), _t(Bc.row, np.int32), _t(Bc.val))
    C = h.spgemm_csc(sr, dA, dB)
    h.check()
    ref = odc.csc_spgemm(oracle.get(), sr, Ac, Bc)
    cp, rw, vl = C.to_numpy()
    assert np.array_equal(cp, ref.colptr) and np.array_equal(rw, ref.row), "CSC pattern"
    _close(sr, vl, ref.val, "CSC values")


@pytest.mark.parametrize("sr", EXACT)
def test_dcsc_pipeline(h, sr):
    """Hypersparse SUMMA-style blocks in DCSC: decompress both operands,
    multiply in CSC, compress the result (paper, Algorithm 1 and the
    transposition identity of Section 4.1)."""
    import paper_2504_06408_amd as sg
    A = _hypersparse_block(15, 8, 0, 5, sr, 60)
    B = _hypersparse_block(15, 8, 5, 2, sr, 60)
    Ac, Bc = _csc_of(A), _csc_of(B)
    dev = []
    for M, Mc in ((A, Ac), (B, Bc)):
        jc, cp = odc.compress(Mc.colptr)
        dev.append(h.dcsc_decompress(M.nrows, M.ncols, _t(jc, np.int32), _t(cp, np.int64), _t(Mc.row, np.int32),
                                     _t(np.asarray(Mc.val, IN_DTYPE[sr]))))
    C = h.spgemm_csc(sr, dev[0], dev[1])
    jc, cp = h.dcsc_compress(C.colptr)
    h.check()
    ref = odc.csc_spgemm(oracle.get(), sr, Ac, Bc)
    rjc, rcp = odc.compress(ref.colptr)
    assert np.array_equal(jc.cpu().numpy(), rjc) and np.array_equal(cp.cpu().numpy(), rcp)
    assert np.array_equal(C.row.cpu().numpy(), ref.row)
    _close(sr, C.val.cpu().numpy(), ref.val, "DCSC pipeline values")
    assert len(rjc) < C.ncols, "the result should have empty columns"


def _graph(scale, sr, seed, style):
    W = synth.rmat(scale, 8, seed=seed)
    return with_vals(W, sr, seed + 1, style)


def _cmp_power(h, sr, W, max_hops, **kw):
    from gpu_helpers import to_dev
    D, hops, prods, conv = h.power(sr, to_dev(W), max_hops, **kw)
    ref = opw.power(oracle.get(), sr, W, max_hops, **kw)
    assert (hops, prods, conv) == (ref.hops, ref.products, ref.converged), ((hops, prods, conv), ref)
    rp, cl, vl = D.to_numpy()
    assert np.array_equal(rp, ref.D.rowptr) and np.array_equal(cl, ref.D.col), f"power pattern {kw}"
    _close(sr, vl, ref.D.val, f"power values {kw}")
    return ref


@pytest.mark.parametrize("squaring", [False, True])
def test_power_minplus_distance_matrix(h, squaring):
    """(min,+) powers of I (+) W to the fixed point: the distance matrix."""
    W = _graph(9, MINPLUS, 70, "int")
    ref = _cmp_power(h, MINPLUS, W, 0, self_loops=True, squaring=squaring, fixpoint=True)
    assert ref.converged


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_power_minplus_k_hops(h, k):
    W = _graph(10, MINPLUS, 80, "positive")
    _cmp_power(h, MINPLUS, W, k, self_loops=True)
    _cmp_power(h, MINPLUS, W, k)  # walks of exactly k edges


def test_power_bool_closure(h):
    W = _graph(10, BOOL, 90, "positive")
    ref = _cmp_power(h, BOOL, W, 0, self_loops=True, squaring=True, fixpoint=True)
    assert ref.converged


@pytest.mark.parametrize("sr", [I64, F64])
def test_power_walk_counts(h, sr):
    W = _graph(8, sr, 95, "positive")
    _cmp_power(h, sr, W, 3)
    _cmp_power(h, sr, W, 4, squaring=True)


def test_power_errors(h):
    import paper_2504_06408_amd as sg
    from gpu_helpers import to_dev
    W = _graph(6, MINPLUS, 99, "int")
    with pytest.raises(sg.SgError) as e:
        h.power(MINPLUS, to_dev(W), 0, fixpoint=True)  # a fixed point needs self loops
    assert e.value.status == -1
    with pytest.raises(sg.SgError) as e:
        h.power(F64, to_dev(with_vals(W, F64, 3)), 0, self_loops=True, fixpoint=True)
    assert e.value.status == -1
    R = synth.er(10, 12, 2, 5).with_values(np.ones(20, np.float32))
    with pytest.raises(sg.SgError) as e:
        h.power(MINPLUS, to_dev(R), 2)
    assert e.value.status == -2
    # one hop without self loops: a copy of W
    _cmp_power(h, MINPLUS, W, 1)
