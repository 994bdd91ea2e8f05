"""GPU parity of hash-bin rows over wide B (more than 65,536 columns): a row
of 65 to 4096 products is merged in LDS from its sources' sorted segments
(option merge_rows, default on) instead of going through an LDS hash table
and a sort.  Each case runs with the option on and off against the CPU
oracle, on rows of one to several hundred sources whose columns repeat
across sources (a hot column range), including rows whose products all fall
on one or three columns; the merge of parts (paper, Section 4.4) and a
batch with a merged block (Section 2.1, checked by the block identity
sum_q A_q B_q = [A_1 .. A_n][B_1; ..; B_n]) take the same kernel."""
import numpy as np
import pytest

import oracle
import synth
from helpers import ALL, F32, with_vals
from gpu_helpers import check_product, compare, hcat, to_dev, vcat

pytestmark = pytest.mark.gpu

NCOLS = 200_000
HOT = 4096


@pytest.fixture(scope="module")
def h():
    import paper_2504_06408_amd as sg
    hd = sg.Handle(0)
    yield hd
    hd.close()


def _reset(h):
    h.set_option("force_path", "auto")
    h.set_option("hash_max_products", 4096)
    h.set_option("merge_rows", 1)


def _csr(rows, ncols):
    rowptr = np.zeros(len(rows) + 1, np.int64)
    rowptr[1:] = np.cumsum([len(r) for r in rows])
    col = np.concatenate(rows).astype(np.int32) if rows else np.zeros(0, np.int32)
    return synth.CSR(len(rows), ncols, rowptr, col, np.zeros(len(col), np.float64))


def _wide_rows(lengths, rng):
    """Sorted distinct columns: half from the hot range, half from all."""
    out = []
    for k in lengths:
        k = int(k)
        hot = rng.choice(HOT, size=k // 2, replace=False)
        cold = rng.choice(NCOLS, size=k - k // 2, replace=False)
        out.append(np.unique(np.concatenate([hot, cold])))
    return out


def _operands(seed):
    """B: 6000 rows of 1 .. 4000 entries (log-uniform) plus 400 rows {7} and
    400 rows {7, 8, 9}.  A: rows of 1 .. 300 sources, each row aiming at 300
    .. 4000 products (70 .. 256 for 60 rows of at most 12 sources) from B
    rows of about equal length, and rows of 100 to 400 sources on the one-
    and three-column B rows."""
    rng = np.random.default_rng(seed)
    lens = np.exp(rng.uniform(0, np.log(4000), 6000)).astype(np.int64) + 1
    brows = _wide_rows(lens, rng)
    one0 = len(brows)
    brows += [np.array([7])] * 400
    three0 = len(brows)
    brows += [np.array([7, 8, 9])] * 400
    B = _csr(brows, NCOLS)
    blen = np.array([len(r) for r in brows])
    order = np.argsort(blen[:one0])
    arows = []
    for r in range(420):
        s = [1, 1, 2, 2, 3, 4, 6, 8, 12, 20, 40, 100, 300][r % 13]
        # rows of 65 .. 256 products (one wavefront per row) after 360 larger ones
        target = int(rng.integers(300, 4000)) if r < 360 else int(rng.integers(70, 256))
        s = s if r < 360 else min(s, 12)
        per = max(1, target // s)
        # B rows of length in (per/2, per]
        lo = np.searchsorted(blen[order], per // 2 + 1)
        hi = np.searchsorted(blen[order], per, side="right")
        pool = order[lo:hi] if hi - lo >= s else order[:max(hi, s)]
        arows.append(np.sort(rng.choice(pool, size=s, replace=False)))
    arows.append(np.arange(one0, one0 + 300))
    arows.append(np.arange(one0, one0 + 400))
    arows.append(np.arange(three0, three0 + 300))
    arows.append(np.concatenate([np.arange(one0, one0 + 200), np.arange(three0, three0 + 200)]))
    # rows of one-wavefront bins whose sources fill several chunks of 64
    arows.append(np.arange(one0, one0 + 200))
    arows.append(np.arange(one0, one0 + 100))
    arows.append(np.concatenate([np.arange(one0, one0 + 70), np.arange(three0, three0 + 40)]))
    A = _csr(arows, B.nrows)
    return A, B


def _products(A, B):
    deg = np.diff(B.rowptr)
    return np.array([deg[A.col[A.rowptr[r]:A.rowptr[r + 1]]].sum() for r in range(A.nrows)])


_OPS = {}


def _ops(seed):
    if seed not in _OPS:
        _OPS[seed] = _operands(seed)
    return _OPS[seed]


def test_operands_reach_the_merge_bins():
    A, B = _ops(900)
    p = _products(A, B)
    assert B.ncols > 65536
    assert ((p > 64) & (p <= 4096)).mean() > 0.8, np.percentile(p, [5, 50, 95])
    assert (p > 2048).sum() > 50 and ((p > 256) & (p <= 512)).sum() > 10 and ((p > 64) & (p <= 256)).sum() > 30


@pytest.mark.parametrize("sr", ALL)
@pytest.mark.parametrize("merge", [1, 0])
def test_single_product(h, sr, merge):
    _reset(h)
    h.set_option("merge_rows", merge)
    try:
        A, B = _ops(900)
        A = with_vals(A, sr, 901)
        B = with_vals(B, sr, 902)
        check_product(h, sr, A, B, what=f"merge_rows={merge}")
    finally:
        _reset(h)


@pytest.mark.parametrize("acc", ["compensated", "plain"])
def test_fp32_accumulation_modes(h, acc):
    """fp32 sums with every row compensated (8-byte (hi, lo) accumulators,
    which the merge kernel folds group by group in registers) or none,
    merge rows on and off."""
    import paper_2504_06408_amd as sg
    mode = sg.ACC_COMPENSATED if acc == "compensated" else sg.ACC_PLAIN
    A, B = _ops(900)
    A, B = with_vals(A, F32, 961), with_vals(B, F32, 962)
    for merge in (1, 0):
        _reset(h)
        h.set_option("merge_rows", merge)
        try:
            check_product(h, F32, A, B, acc=mode, what=f"fp32 {acc}, merge_rows={merge}")
        finally:
            _reset(h)


@pytest.mark.parametrize("sr", ALL)
def test_forced_hash_path(h, sr):
    """Every row that the hash bins can take (up to 4096 products) through
    them, so rows of the small bins sit beside the merge bins."""
    _reset(h)
    h.set_option("force_path", "hash")
    try:
        A, B = _ops(910)
        check_product(h, sr, with_vals(A, sr, 911), with_vals(B, sr, 912), what="forced hash")
    finally:
        _reset(h)


@pytest.mark.parametrize("sr", ALL)
def test_merge_of_wide_parts(h, sr):
    """Five parts of rows of 60 .. 900 entries (hot and wide columns):
    merged rows of ~300 to ~4500 entries."""
    import torch
    import paper_2504_06408_amd as sg
    _reset(h)
    rng = np.random.default_rng(920)
    parts = []
    for q in range(5):
        lens = np.exp(rng.uniform(np.log(60), np.log(900), 300)).astype(np.int64)
        parts.append(with_vals(_csr(_wide_rows(lens, rng), NCOLS), sr, 921 + q))
    for merge in (1, 0):
        h.set_option("merge_rows", merge)
        C = h.merge(sg.semiring(sr), [to_dev(p) for p in parts])
        torch.cuda.synchronize()
        h.check()
        rp, cl, vl = C.to_numpy()
        compare(sr, rp, cl, vl, oracle.get().merge(sr, parts), f"wide merge, merge_rows={merge}")
    _reset(h)


@pytest.mark.parametrize("sr", ALL)
def test_batch_with_merged_block(h, sr):
    """Three wide products and their merge in one plan, replayed twice."""
    import paper_2504_06408_amd as sg
    _reset(h)
    As, Bs = [], []
    for q in range(3):
        A, B = _ops(930 + q)
        As.append(with_vals(A, sr, 940 + q))
        Bs.append(with_vals(B, sr, 950 + q))
    ref_m = oracle.get().spgemm(sr, hcat(As), vcat(Bs))
    plan = h.batch_plan(sg.semiring(sr), [to_dev(a) for a in As], [to_dev(b) for b in Bs], [0, 3])
    try:
        for rep in range(2):
            plan.execute()
            res = plan.results_numpy()
            for q in range(3):
                compare(sr, *res[q], oracle.get().spgemm(sr, As[q], Bs[q]), f"batch product {q} rep {rep}")
            compare(sr, *res[3], ref_m, f"batch merge rep {rep}")
    finally:
        plan.destroy()


def test_merge_rows_option_errors(h):
    import paper_2504_06408_amd as sg
    with pytest.raises(sg.SgError):
        h.set_option("merge_rows", 2)
    _reset(h)
