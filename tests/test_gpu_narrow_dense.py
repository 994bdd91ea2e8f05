"""GPU parity of dense rows over narrow B (at most 65,536 columns: the blocks
of a SUMMA grid, the products of a batch) against the CPU oracle.

Outside the column-slab path, such a row with at most a workgroup's LDS
capacity of entries (12,544 with 8-byte accumulators, 21,504 with 4-byte
ones, 44,288 for bool) is folded whole over a bitmap of the columns; a
fuller row stays on the tile and range tasks.  Each case here holds rows on
both sides of every cap, so both kinds of task run in one call: a single
product with the slab path switched off, a batch of such products merged
into one block (checked against the oracle's product of the concatenated
operands, the block identity of the paper's SUMMA, Section 2.1), and a
merge of narrow parts."""
import numpy as np
import pytest

import oracle
import synth
from helpers import ALL, with_vals
from gpu_helpers import check_product, compare, hcat, to_dev, vcat

pytestmark = pytest.mark.gpu

NCOLS = 65536


@pytest.fixture(scope="module")
def h():
    import paper_2504_06408_amd as sg
    hd = sg.Handle(0)
    yield hd
    hd.close()


def _reset(h):
    h.set_option("force_path", "auto")
    h.set_option("hash_max_products", 4096)
    h.set_option("dense_slab", 1)


def _rows_of_lengths(lengths, ncols, seed):
    """CSR structure whose row r holds lengths[r] distinct random columns."""
    rng = np.random.default_rng(seed)
    rowptr = np.zeros(len(lengths) + 1, np.int64)
    cols = []
    for r, k in enumerate(lengths):
        c = np.sort(rng.choice(ncols, size=int(k), replace=False)).astype(np.int32)
        cols.append(c)
        rowptr[r + 1] = rowptr[r] + len(c)
    col = np.concatenate(cols) if cols else np.zeros(0, np.int32)
    return synth.CSR(len(lengths), ncols, rowptr, col, np.zeros(len(col), np.float64))


def _a_rows(n_inner, seed):
    """64 rows of 150 .. 4000 entries (geometric): times a B of 24 entries a
    row over 65,536 columns they make rows of ~4k to ~50k entries."""
    return _rows_of_lengths(np.geomspace(150, 4000, 64).astype(np.int64), n_inner, seed)


@pytest.mark.parametrize("sr", ALL)
def test_single_product_both_sides_of_cap(h, sr):
    _reset(h)
    h.set_option("dense_slab", 0)
    try:
        A = with_vals(_a_rows(4096, 800), sr, 801)
        B = with_vals(synth.er(4096, NCOLS, 24, 802), sr, 803)
        _, C = check_product(h, sr, A, B, what="narrow dense rows")
        st = h.stats()
        m = np.diff(C.rowptr.cpu().numpy())
        assert m.min() < 12544 and m.max() > 44288, (m.min(), m.max())
        assert st["slab_tasks"] > 0 and st["tile_tasks"] + st["range_tasks"] > 0, st
    finally:
        _reset(h)


@pytest.mark.parametrize("sr", ALL)
def test_batch_products_and_merge(h, sr):
    """Four narrow products and their merge in one plan."""
    import paper_2504_06408_amd as sg
    _reset(h)
    As = [with_vals(_a_rows(4096, 810 + q), sr, 820 + q) for q in range(4)]
    Bs = [with_vals(synth.er(4096, NCOLS, 6 + 6 * q, 830 + q), sr, 840 + q) for q in range(4)]
    plan = h.batch_plan(sg.semiring(sr), [to_dev(a) for a in As], [to_dev(b) for b in Bs], [0, 4])
    try:
        # the block identity: sum_q A_q B_q = [A_1 .. A_4] [B_1; ..; B_4]
        Acat = hcat(As)
        Bcat = vcat(Bs)
        ref_m = oracle.get().spgemm(sr, Acat, Bcat)
        for rep in range(2):
            plan.execute()
            res = plan.results_numpy()
            for q in range(4):
                compare(sr, *res[q], oracle.get().spgemm(sr, As[q], Bs[q]), f"batch product {q} rep {rep}")
            compare(sr, *res[4], ref_m, f"batch merge rep {rep}")
        m = np.diff(res[4][0])
        assert m.min() < 12544 and m.max() > 44288, (m.min(), m.max())
    finally:
        plan.destroy()


@pytest.mark.parametrize("sr", ALL)
def test_merge_of_narrow_parts(h, sr):
    """Four parts of rows of 500 .. 15000 random columns each: merged rows
    of ~2k to ~42k entries."""
    import torch
    import paper_2504_06408_amd as sg
    _reset(h)
    lengths = np.geomspace(500, 15000, 48).astype(np.int64)
    parts = [with_vals(_rows_of_lengths(lengths, NCOLS, 850 + q), sr, 860 + q) for q in range(4)]
    C = h.merge(sg.semiring(sr), [to_dev(p) for p in parts])
    torch.cuda.synchronize()
    h.check()
    rp, cl, vl = C.to_numpy()
    compare(sr, rp, cl, vl, oracle.get().merge(sr, parts), "narrow merge")
    m = np.diff(rp)
    assert m.min() < 11776 and m.max() > 39168, (m.min(), m.max())
