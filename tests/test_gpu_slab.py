"""GPU parity of the column-slab dense path against the CPU oracle.

The dense rows of a single product run per (row, column slab) tasks over a
slab partition of B; slabs holding more entries than a task's LDS value
array go to the tile and range tasks.  These cases make every kind of task
appear: slabs under and over the cap, dense and sparse tiles inside
over-cap slabs, a ragged last slab, and values that change between the
symbolic and the numeric pass (the cached partition structure with fresh
values)."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from helpers import ALL, EXACT, F64, I64, MINPLUS, with_vals
from gpu_helpers import check_product, compare, to_dev

pytestmark = pytest.mark.gpu


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


def _hstack(blocks, sr, seed):
    """Column concatenation of synth CSR blocks (structure only), values per
    semiring drawn afterwards."""
    mats = [sp.csr_matrix((np.ones(b.nnz), np.asarray(b.col), np.asarray(b.rowptr)), shape=(b.nrows, b.ncols))
            for b in blocks]
    M = sp.hstack(mats, format="csr")
    M.sort_indices()
    S = synth.CSR(M.shape[0], M.shape[1], M.indptr.astype(np.int64), M.indices.astype(np.int32),
                  np.zeros(M.nnz, np.float64))
    return with_vals(S, sr, seed)


@pytest.mark.parametrize("sr", ALL)
@pytest.mark.parametrize("slab", [0, 1])
def test_slab_and_tile_paths(h, sr, slab):
    """R-MAT s12 A.A with every row forced dense, through each dense path."""
    _reset(h)
    h.set_option("dense_slab", slab)
    h.set_option("force_path", "dense")
    try:
        A = with_vals(synth.rmat(12, 16, seed=90), sr, 91)
        check_product(h, sr, A, A, what=f"rmat12 dense slab={slab}")
    finally:
        _reset(h)


@pytest.mark.parametrize("sr", ALL)
def test_over_cap_slabs_mix_all_tasks(h, sr):
    """B = [dense 16384-column block | sparse 180000-column block]: C's rows
    hold ~10k entries in the first tile (over the slab cap: dense-tile task)
    and a few hundred spread over the other tiles (slab tasks, and range
    tasks inside the over-cap slab)."""
    _reset(h)
    A = with_vals(synth.er(64, 160, 40, 200), sr, 201)
    B = _hstack([synth.er(160, 16384, 3000, 202), synth.er(160, 180000, 40, 203)], sr, 204)
    check_product(h, sr, A, B, what="over-cap mix")


@pytest.mark.parametrize("sr", [MINPLUS, F64])
def test_ragged_last_slab_wide(h, sr):
    """1,200,001 columns: slabs of 2^17 columns, the last one holds a single
    column tile's remainder."""
    _reset(h)
    A = with_vals(synth.er(80, 300, 60, 210), sr, 211)
    B = with_vals(synth.er(300, 1_200_001, 900, 212), sr, 213)
    check_product(h, sr, A, B, what="ragged wide")


@pytest.mark.parametrize("sr", EXACT)
def test_values_change_between_passes(h, sr):
    """Numeric after symbolic on the same arrays with new values: the slab
    partition's structure is reused and its values rebuilt."""
    import torch
    import paper_2504_06408_amd as sg
    import oracle
    _reset(h)
    A = with_vals(synth.rmat(11, 16, seed=220), sr, 221)
    dA = to_dev(A)
    rowptr, nnz = h.symbolic(dA, dA)
    A2 = with_vals(A, sr, 222)
    dA.val.copy_(torch.from_numpy(np.ascontiguousarray(A2.val)).to(dA.val.device))
    vdt = dA.val.dtype
    C = sg.DeviceCSR(A.nrows, A.ncols, rowptr, torch.empty(nnz, dtype=torch.int32, device="cuda"),
                     torch.empty(nnz, dtype=vdt, device="cuda"))
    h.numeric(sg.semiring(sr), dA, dA, C)
    torch.cuda.synchronize()
    h.check()
    rp, cl, vl = C.to_numpy()
    compare(sr, rp, cl, vl, oracle.get().spgemm(sr, A2, A2), "values changed")


def test_dense_slab_option_errors(h):
    import paper_2504_06408_amd as sg
    with pytest.raises(sg.SgError):
        h.set_option("dense_slab", 2)


@pytest.mark.parametrize("sr", ALL)
def test_many_sources_per_row(h, sr):
    """Rows of A with ~700 stored entries: more sources than one workgroup
    chunk, so the symbolic, light and heavy slab kernels load sources chunk
    by chunk (and the heavy kernel per tile)."""
    _reset(h)
    A = with_vals(synth.er(24, 2000, 700, 230), sr, 231)
    B = _hstack([synth.er(2000, 16384, 40, 232), synth.er(2000, 300000, 6, 233)], sr, 234)
    check_product(h, sr, A, B, what="many sources")


@pytest.mark.parametrize("sr", ALL)
def test_heavy_tile_span_counts(h, sr):
    """One dense row over 2^20 columns whose first slab is heavy for every
    semiring (34,815 entries).  Tile 0 is full (2048 entries in each of its
    eight 2048-column spans, the largest span count), tile 1 holds exactly
    1024 entries, all in its last span (the least count for which the
    symbolic pass records span counts), tile 2 holds 1023 (heavy tasks count
    such a tile themselves), tile 3 is full.  A second source repeats every
    third column, so entries also fold two products."""
    _reset(h)
    c0 = np.concatenate([np.arange(16384), 16384 + 14336 + np.arange(1024), 32768 + 2 * np.arange(1023),
                         49152 + np.arange(16384)]).astype(np.int32)
    c1 = c0[::3]
    B = synth.CSR(2, 1 << 20, np.array([0, c0.size, c0.size + c1.size], np.int64), np.concatenate([c0, c1]),
                  np.zeros(c0.size + c1.size, np.float64))
    B = with_vals(B, sr, 240)
    A = with_vals(synth.CSR(1, 2, np.array([0, 2], np.int64), np.array([0, 1], np.int32), np.zeros(2)), sr, 241)
    check_product(h, sr, A, B, what="heavy span counts")
    st = h.stats()
    assert st["tile_tasks"] == 1 and st["tile_entries"] == c0.size, st


@pytest.mark.parametrize("sr", ALL)
def test_heavy_tiles_staged_and_dense(h, sr):
    """Heavy tasks whose tiles alternate between the dense accumulator and
    the LDS-staged path (products and entries of a sparse tile staged in the
    accumulator's LDS), so a dense tile follows a staged one inside a task
    and across tasks.  One slab of 2^17 columns, light cap 64: per row, tile
    0 folds 4 x 3000 products (dense), tile 1 2 x 1500 (staged), tile 2 300
    (one round in registers), tile 3 4 x 5000 (dense), tile 4 2000
    (staged), tile 5 nothing, tile 6 1100 (staged, with span counts), tile 7
    4 x 8000 (dense)."""
    _reset_knobs(h)
    rng = np.random.default_rng(260)

    def cols(t, k):
        return (t << 14) + np.sort(rng.choice(1 << 14, size=k, replace=False))

    t0, t1, t2, t3, t4, t6, t7 = cols(0, 3000), cols(1, 1500), cols(2, 300), cols(3, 5000), cols(4, 2000), \
        cols(6, 1100), cols(7, 8000)
    rows = [np.concatenate([t0, t1, t2, t3, t7]), np.concatenate([t0, t1, t3, t7]),
            np.concatenate([t0, t3, t4, t7]), np.concatenate([t0, t3, t6, t7])]
    B = synth.CSR(4, 1 << 17, np.concatenate([[0], np.cumsum([r.size for r in rows])]).astype(np.int64),
                  np.concatenate(rows).astype(np.int32), np.zeros(sum(r.size for r in rows)))
    A = synth.CSR(3, 4, np.array([0, 4, 8, 10], np.int64), np.array([0, 1, 2, 3, 0, 1, 2, 3, 1, 3], np.int32),
                  np.zeros(10))
    h.set_option("slab_log", 17)
    h.set_option("light_cap", 64)
    try:
        check_product(h, sr, with_vals(A, sr, 261), with_vals(B, sr, 262), what="staged and dense tiles")
        st = h.stats()
        assert st["tile_tasks"] == 3 and st["slab_tasks"] == 0, st
    finally:
        _reset_knobs(h)


@pytest.mark.parametrize("sr", [MINPLUS, I64])
@pytest.mark.parametrize("g32", [0, 1])
def test_symbolic_gather_widths(h, sr, g32):
    """The symbolic slab pass with 32-bit gathers (the default below 2^30
    entries of B) and with 64-bit gathers (forced), on a product whose rows
    are all dense."""
    _reset(h)
    h.set_option("force_path", "dense")
    h.set_option("gather32", g32)
    try:
        A = with_vals(synth.rmat(12, 16, seed=250), sr, 251)
        check_product(h, sr, A, A, what=f"gather32={g32}")
    finally:
        h.set_option("gather32", 1)
        _reset(h)


def test_gather32_option_errors(h):
    import paper_2504_06408_amd as sg
    with pytest.raises(sg.SgError):
        h.set_option("gather32", 2)


def _reset_knobs(h):
    h.set_option("slab_log", 0)
    h.set_option("light_cap", 0)
    _reset(h)


@pytest.mark.parametrize("sr", ALL)
@pytest.mark.parametrize("ls", [14, 15, 17])
@pytest.mark.parametrize("cap", [0, 200])
def test_slab_width_and_light_cap(h, sr, ls, cap):
    """The tunable slab width and light-task cap: an s11 R-MAT times a B of
    70,000 columns (five column tiles, the last one ragged) with every row
    dense, so slab widths of 1, 2 and 8 tiles (one slab wider than B) and a cap
    that sends most slabs to the heavy kernel all meet the oracle."""
    _reset_knobs(h)
    h.set_option("force_path", "dense")
    h.set_option("slab_log", ls)
    h.set_option("light_cap", cap)
    try:
        A = with_vals(synth.rmat(11, 16, seed=300), sr, 301)
        B = with_vals(synth.er(2048, 70000, 40, 302), sr, 303)
        check_product(h, sr, A, B, what=f"slab_log={ls} light_cap={cap}")
        check_product(h, sr, A, A, what=f"A.A slab_log={ls} light_cap={cap}")
    finally:
        _reset_knobs(h)


@pytest.mark.parametrize("sr", ALL)
def test_light_cap_moves_tasks_to_heavy(h, sr):
    """A smaller light cap turns light slab tasks into heavy ones (the task
    statistics of the numeric pass), with the same result.  The heavy tasks
    made so hold mostly sparse tiles (under 1024 entries, products of one
    round), which the heavy kernel compacts by bitmap and rank in LDS
    borrowed from its accumulator; denser tiles keep the sweep."""
    _reset_knobs(h)
    h.set_option("force_path", "dense")
    try:
        A = with_vals(synth.rmat(12, 16, seed=310), sr, 311)
        check_product(h, sr, A, A, what="light_cap default")
        s0 = h.stats()
        h.set_option("light_cap", 64)
        check_product(h, sr, A, A, what="light_cap 64")
        s1 = h.stats()
        assert s1["tile_tasks"] > s0["tile_tasks"] and s1["slab_tasks"] < s0["slab_tasks"], (s0, s1)
        assert s0["slab_entries"] + s0["tile_entries"] == s1["slab_entries"] + s1["tile_entries"]
    finally:
        _reset_knobs(h)


def test_knob_option_errors(h):
    import paper_2504_06408_amd as sg
    for name, bad in [("slab_log", 13), ("slab_log", 18), ("light_cap", -1), ("light_cap", 40000)]:
        with pytest.raises(sg.SgError):
            h.set_option(name, bad)
