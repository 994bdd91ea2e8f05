"""The no-allocation entry point (sg_spgemm_numeric_noalloc) against the
ordinary numeric pass and the oracle: two calls in a row on one GPU, the
second on a smaller input, for every semiring and for the column-slab and
whole-row tile paths; a product too large for the fixed array is refused
with SG_ERR_NOMEM before the output is touched."""
import numpy as np
import pytest

import oracle
import synth
from helpers import ALL, with_vals
from gpu_helpers import compare, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import paper_2504_06408_amd as sg
    hd = sg.Handle(0)
    yield hd
    hd.close()


def _both(h, sr, A, B):
    """The product through sg_spgemm_numeric and through the no-allocation
    variant on the same row pointers; host copies of both."""
    import torch
    import paper_2504_06408_amd as sg
    dA = to_dev(A)
    dB = dA if B is A else to_dev(B)
    s = sg.semiring(sr)
    rowptr, nnz = h.symbolic(dA, dB)
    dt = sg._torch_dtype(sr)
    C1 = sg.DeviceCSR(A.nrows, B.ncols, rowptr, torch.empty(nnz, dtype=torch.int32, device="cuda"),
                      torch.empty(nnz, dtype=dt, device="cuda"))
    C2 = sg.DeviceCSR(A.nrows, B.ncols, rowptr, torch.full((nnz,), -7, dtype=torch.int32, device="cuda"),
                      torch.zeros(nnz, dtype=dt, device="cuda"))
    h.numeric(s, dA, dB, C1)
    h.numeric_noalloc(s, dA, dB, C2)
    torch.cuda.synchronize()
    h.check()
    return C1.to_numpy(), C2.to_numpy()


def _check(h, sr, A, B, what):
    (rp1, c1, v1), (rp2, c2, v2) = _both(h, sr, A, B)
    ref = oracle.get().spgemm(sr, A, B)
    compare(sr, rp2, c2, v2, ref, what + " (no-allocation entry point)")
    compare(sr, rp1, c1, v1, ref, what + " (ordinary entry point)")
    assert np.array_equal(c1, c2), what + ": column ids differ between the two entry points"


@pytest.mark.parametrize("sr", ALL)
@pytest.mark.parametrize("slab", [1, 0])
def test_noalloc_matches_numeric_twice(h, sr, slab):
    """R-MAT s12 A.A (rows on every path, 4096 columns: one tile) and then the
    smaller R-MAT s10 A.A through the same fixed array; then an s11 x ER
    product over 20000 columns (two tiles, ragged) and again s10."""
    h.set_option("dense_slab", slab)
    h.set_option("hash_max_products", 1024)
    try:
        big = with_vals(synth.rmat(12, 16, seed=21), sr, 40 + sr)
        small = with_vals(synth.rmat(10, 8, seed=22), sr, 50 + sr)
        _check(h, sr, big, big, f"s12 slab={slab}")
        _check(h, sr, small, small, f"s10 after s12 slab={slab}")
        A = with_vals(synth.rmat(11, 16, seed=23), sr, 60 + sr)
        B = with_vals(synth.er(2048, 20000, 48, 24), sr, 70 + sr)
        _check(h, sr, A, B, f"s11 x ER 20000 columns slab={slab}")
        _check(h, sr, small, small, f"s10 after the wide product slab={slab}")
    finally:
        h.set_option("dense_slab", 1)
        h.set_option("hash_max_products", 4096)


def test_noalloc_refuses_too_large(h):
    """R-MAT s18 needs far more than the fixed array: SG_ERR_NOMEM, and C's
    arrays keep what they held."""
    import torch
    import paper_2504_06408_amd as sg
    A = with_vals(synth.rmat(18, 16, seed=1), 5, 2, style="positive")
    dA = to_dev(A)
    rowptr, nnz = h.symbolic(dA, dA)
    C = sg.DeviceCSR(A.nrows, A.ncols, rowptr, torch.full((nnz,), -7, dtype=torch.int32, device="cuda"),
                     torch.full((nnz,), 3.0, dtype=torch.float32, device="cuda"))
    with pytest.raises(sg.SgError) as e:
        h.numeric_noalloc(sg.semiring(5), dA, dA, C)
    assert e.value.status == -4 and "fixed" in str(e.value)
    torch.cuda.synchronize()
    assert int((C.col != -7).sum()) == 0 and int((C.val != 3.0).sum()) == 0
    # the handle still works afterwards, through either entry point
    small = with_vals(synth.rmat(10, 8, seed=22), 5, 55)
    _check(h, 5, small, small, "s10 after a refused call")
