"""GPU parity: the HIP library (called through its C ABI) against the CPU
oracle, element by element, on seeded inputs.  Bit-exact for int64, bool and
(min,+); within the gated relative tolerance (1e-12 float64, 1e-5 float32
against the float64 oracle) for float sums; patterns exact everywhere."""
import numpy as np
import pytest

import synth
from helpers import ALL, BOOL, EXACT, F32, F64, I64, MINPLUS, with_vals
from gpu_helpers import check_product, gpu_product

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import paper_2504_06408_amd as sg
    hd = sg.Handle(0)
    yield hd
    hd.close()


def _fresh(h):
    h.set_option("force_path", "auto")
    h.set_option("hash_max_products", 4096)


def test_er_4096_fp64(h):
    """Erdos-Renyi n=4096, 8 per row, float64 (+,x)."""
    _fresh(h)
    A = synth.er(4096, 4096, 8, 1).with_values(synth.values(synth.VAL_F64_UNIFORM, 4096 * 8, 0, 1, 11))
    B = synth.er(4096, 4096, 8, 2).with_values(synth.values(synth.VAL_F64_UNIFORM, 4096 * 8, 0, 1, 12))
    check_product(h, F64, A, B, what="ER 4096")


@pytest.mark.parametrize("sr", ALL)
@pytest.mark.parametrize("scale", [10, 12])
def test_rmat_auto(h, sr, scale):
    """R-MAT A.A: rows span every path (small, hash, dense)."""
    _fresh(h)
    A = with_vals(synth.rmat(scale, 16, seed=scale), sr, 100 + sr)
    check_product(h, sr, A, A, what=f"rmat s{scale}")


@pytest.mark.parametrize("sr", ALL)
@pytest.mark.parametrize("path", ["small", "hash", "dense"])
def test_forced_path(h, sr, path):
    """Each kernel family alone (rows it cannot take fall through)."""
    _fresh(h)
    h.set_option("force_path", path)
    try:
        A = with_vals(synth.rmat(10, 8, seed=3), sr, 5)
        B = with_vals(synth.er(1024, 1024, 6, 4), sr, 6)
        check_product(h, sr, A, B, what=f"forced {path}")
        check_product(h, sr, A, A, what=f"forced {path} A.A")
    finally:
        _fresh(h)


@pytest.mark.parametrize("hm", [0, 64, 300, 1024, 4096])
def test_hash_threshold(h, hm):
    _fresh(h)
    h.set_option("hash_max_products", hm)
    try:
        A = with_vals(synth.rmat(11, 16, seed=21), MINPLUS, 22)
        check_product(h, MINPLUS, A, A, what=f"hash_max {hm}")
    finally:
        _fresh(h)


@pytest.mark.parametrize("sr", ALL)
def test_wide_tiles(h, sr):
    """B with 1.2M columns: 74 column tiles, so dense rows need two bitmap
    passes in the symbolic kernel and tile offsets in the numeric one."""
    _fresh(h)
    A = with_vals(synth.er(96, 160, 40, 31), sr, 32)
    B = with_vals(synth.er(160, 1_200_000, 700, 33), sr, 34)
    check_product(h, sr, A, B, what="wide")


@pytest.mark.parametrize("sr", ALL)
def test_rectangular_and_ragged(h, sr):
    _fresh(h)
    A = with_vals(synth.random_small(37, 501, 0.03, 41), sr, 42)
    B = with_vals(synth.er(501, 70000, 9, 43), sr, 44)
    check_product(h, sr, A, B, what="rect")
    A1 = with_vals(synth.random_small(1, 1, 1.0, 45), sr, 46)
    check_product(h, sr, A1, A1, what="1x1")


@pytest.mark.parametrize("sr", ALL)
def test_empty_operands(h, sr):
    _fresh(h)
    import torch
    A = with_vals(synth.rmat(8, 4, seed=50), sr, 51)
    Z = synth.CSR(A.ncols, 33, np.zeros(A.ncols + 1, np.int64), np.zeros(0, np.int32),
                  np.zeros(0, with_vals(synth.er(1, 1, 1, 1), sr, 1).val.dtype))
    C = gpu_product(h, sr, A, Z)
    assert C.nnz == 0 and C.nrows == A.nrows and int(C.rowptr.abs().sum()) == 0
    E = synth.CSR(0, 0, np.zeros(1, np.int64), np.zeros(0, np.int32), Z.val)
    C = gpu_product(h, sr, E, E)
    assert C.nnz == 0 and C.rowptr.numel() == 1


@pytest.mark.parametrize("sr", EXACT)
def test_repeat_bit_identical(h, sr):
    _fresh(h)
    A = with_vals(synth.rmat(11, 16, seed=60), sr, 61)
    c1 = gpu_product(h, sr, A, A).to_numpy()
    c2 = gpu_product(h, sr, A, A).to_numpy()
    for x, y in zip(c1, c2):
        assert np.array_equal(x, y)


def test_compensated_beats_plain(h):
    """float32 (+,x) with N(0,1) values: compensated and plain accumulation
    both pass the gate; compensated has the smaller worst-case error."""
    _fresh(h)
    import paper_2504_06408_amd as sg
    A = with_vals(synth.rmat(12, 16, seed=70), F32, 71)
    e_comp, _ = check_product(h, F32, A, A, acc=sg.ACC_COMPENSATED, what="compensated")
    e_plain, _ = check_product(h, F32, A, A, acc=sg.ACC_PLAIN, what="plain")
    e_def, _ = check_product(h, F32, A, A, acc=sg.ACC_DEFAULT, what="default")
    assert e_comp[0] <= e_plain[0]


def test_numeric_without_symbolic_cache(h):
    """A second handle runs numeric on a C sized by the first handle's
    symbolic pass: the dense-row tile offsets are recomputed, not reused."""
    import torch
    import paper_2504_06408_amd as sg
    from gpu_helpers import to_dev
    import oracle
    _fresh(h)
    A = with_vals(synth.rmat(11, 16, seed=80), I64, 81)
    dA = to_dev(A)
    rowptr, nnz = h.symbolic(dA, dA)
    C = sg.DeviceCSR(A.nrows, A.ncols, rowptr, torch.empty(nnz, dtype=torch.int32, device="cuda"),
                     torch.empty(nnz, dtype=torch.int64, device="cuda"))
    h2 = sg.Handle(0)
    h2.numeric(sg.semiring(I64), dA, dA, C)
    torch.cuda.synchronize()
    h2.check()
    h2.close()
    ref = oracle.get().spgemm(I64, A, A)
    rp, cl, vl = C.to_numpy()
    assert np.array_equal(rp, ref.rowptr) and np.array_equal(cl, ref.col) and np.array_equal(vl, ref.val)


def test_errors(h):
    import paper_2504_06408_amd as sg
    from gpu_helpers import to_dev
    _fresh(h)
    A = with_vals(synth.er(10, 12, 3, 1), F64, 2)
    dA = to_dev(A)
    with pytest.raises(sg.SgError) as e:
        h.symbolic(dA, dA)
    assert e.value.status == -2
    bad = sg.semiring(F64)
    bad.id = 9
    B = with_vals(synth.er(12, 10, 3, 3), F64, 4)
    dB = to_dev(B)
    rowptr, nnz = h.symbolic(dA, dB)
    import torch
    C = sg.DeviceCSR(10, 10, rowptr, torch.empty(nnz, dtype=torch.int32, device="cuda"),
                     torch.empty(nnz, dtype=torch.float64, device="cuda"))
    with pytest.raises(sg.SgError) as e:
        h.numeric(bad, dA, dB, C)
    assert e.value.status == -3
    # unsorted input is caught when validation is on
    U = synth.CSR(A.nrows, A.ncols, A.rowptr.copy(), A.col.copy(), A.val)
    U.col[0], U.col[1] = U.col[1], U.col[0]
    h.set_option("validate", 1)
    try:
        with pytest.raises(sg.SgError) as e:
            h.symbolic(to_dev(U), dB)
        assert e.value.status == -6
    finally:
        h.set_option("validate", 0)
    with pytest.raises(sg.SgError):
        h.set_option("force_path", "sideways")
