"""GPU parity of the batched path when B spans more than one 16384-column
tile, and of the single-product whole-row tile path (dense_slab = 0) on
such B.

Every product of a multi-product plan runs the whole-row dense kernels
(per-B-row tile offsets, tile and range tasks); with blocks of 32768
columns each dense row spans two tiles, so the tasks start and end inside
B rows and merges cut their parts by column.  Each stage product and each
merged block is compared with the oracle element by element: the merge
against the same block of the oracle's full product (paper, Section 2.1:
C_IJ = (+)_K A_IK B_KJ)."""
import numpy as np
import pytest

import oracle
import synth
from helpers import ALL, EXACT, F32, F64, I64, MINPLUS, BOOL, assert_close_gated, with_vals
from gpu_helpers import TOL, check_product, compare, to_dev

pytestmark = pytest.mark.gpu

_FULL = {}


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


def _summa_inputs(sr):
    """R-MAT scale 16 (edge factor 8) cut 2x2: 32768-column blocks, so T = 2
    for every stage product; the oracle's full A.A cut the same way."""
    if sr not in _FULL:
        A = with_vals(synth.rmat(16, 8, seed=5), sr, 6)
        g = 2
        blk = synth.block_split(A, g)
        full = oracle.get().spgemm(sr, A, A)
        Cb = synth.block_split(synth.CSR(A.nrows, A.ncols, full.rowptr, full.col, full.val), g)
        Mb = None if full.mag is None else synth.block_split(
            synth.CSR(A.nrows, A.ncols, full.rowptr, full.col, full.mag), g)
        stage = [oracle.get().spgemm(sr, blk[I][K], blk[K][J]) for I in range(g) for J in range(g) for K in range(g)]
        _FULL[sr] = (A, g, blk, Cb, Mb, stage)
    return _FULL[sr]


@pytest.mark.parametrize("sr", ALL)
@pytest.mark.parametrize("path", ["auto", "dense"])
def test_batch_summa_two_tiles(h, sr, path):
    import paper_2504_06408_amd as sg
    _reset(h)
    h.set_option("force_path", path)
    try:
        A, g, blk, Cb, Mb, stage = _summa_inputs(sr)
        assert blk[0][0].ncols == 32768
        As, Bs, go = [], [], [0]
        for I in range(g):
            for J in range(g):
                for K in range(g):
                    As.append(blk[I][K])
                    Bs.append(blk[K][J])
                go.append(len(As))
        dA = [to_dev(x) for x in As]
        dB = [to_dev(x) for x in Bs]
        plan = h.batch_plan(sg.semiring(sr), dA, dB, go)
        for rep in range(2):
            plan.execute()
            res = plan.results_numpy()
            for q in range(len(As)):
                compare(sr, *res[q], stage[q], f"2x2 stage product {q} ({path}, rep {rep})")
            for q in range(g * g):
                I, J = divmod(q, g)
                rp, cl, vl = res[len(As) + q]
                ref = Cb[I][J]
                what = f"2x2 merged block {I},{J} ({path}, rep {rep})"
                assert np.array_equal(rp, ref.rowptr) and np.array_equal(cl, ref.col), what
                if sr in (F32, F64):
                    assert_close_gated(vl, ref.val, Mb[I][J].val, TOL[sr], what)
                else:
                    assert np.array_equal(vl.view(np.uint8), ref.val.view(np.uint8)), what
        plan.destroy()
    finally:
        _reset(h)


@pytest.mark.parametrize("sr", ALL)
@pytest.mark.parametrize("path", ["auto", "dense"])
def test_batch_er_wide(h, sr, path):
    """A batch of ER products with n log-uniform in [16k, 64k] (up to four
    column tiles per product, different tile counts in one plan)."""
    import paper_2504_06408_amd as sg
    _reset(h)
    h.set_option("force_path", path)
    try:
        ns, ds = synth.batch_params(6, 16384, 65536, 4, 12, 17)
        As = [with_vals(synth.er(int(n), int(n), int(d), 500 + q), sr, 600 + q) for q, (n, d) in enumerate(zip(ns, ds))]
        Bs = [with_vals(synth.er(int(n), int(n), int(d), 700 + q), sr, 800 + q) for q, (n, d) in enumerate(zip(ns, ds))]
        assert max(a.ncols for a in As) > 2 * 16384
        plan = h.batch_plan(sg.semiring(sr), [to_dev(a) for a in As], [to_dev(b) for b in Bs])
        plan.execute()
        res = plan.results_numpy()
        for q, (a, b) in enumerate(zip(As, Bs)):
            compare(sr, *res[q], oracle.get().spgemm(sr, a, b), f"ER wide product {q} n={a.nrows} ({path})")
        plan.destroy()
    finally:
        _reset(h)


@pytest.mark.parametrize("sr", ALL)
@pytest.mark.parametrize("path", ["auto", "dense"])
def test_tile_path_two_tiles_single(h, sr, path):
    """One product through the whole-row tile path (dense_slab = 0) with B of
    32768 columns: tile and range tasks read B rows through their per-row
    tile offsets."""
    _reset(h)
    h.set_option("dense_slab", 0)
    h.set_option("force_path", path)
    try:
        A = with_vals(synth.rmat(15, 8, seed=12), sr, 13)
        assert A.ncols == 32768
        check_product(h, sr, A, A, what=f"tile path s15 ({path})")
    finally:
        _reset(h)
