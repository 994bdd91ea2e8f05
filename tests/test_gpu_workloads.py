"""GPU parity on the benchmark workloads at reduced scale plus the sampled
full-scale checks: the (min,+) 3-hop panel, the float32 precision path
against float64, the autotuner, and sampled rows + invariants of the full
R-MAT scale-18 products."""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from helpers import BOOL, F32, F64, I64, MINPLUS, rel_error_stats, with_vals
from gpu_helpers import check_product, compare, rows_of, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import paper_2504_06408_amd as sg
    hd = sg.Handle(0)
    yield hd
    hd.close()


def test_three_hop_panel(h):
    """(min,+) 3-hop on a seeded row panel S: X1 = A[S,:].A, X2 = X1.A equal
    rows S of (A.A).A bit for bit (rows are independent)."""
    import torch
    import paper_2504_06408_amd as sg
    h.set_option("force_path", "auto")
    A = synth.rmat(13, 16, seed=1)
    A = A.with_values(synth.values(synth.VAL_F32_UNIFORM, A.nnz, 1.0, 100.0, 2))
    nonempty = np.nonzero(np.diff(A.rowptr) > 0)[0]
    S = nonempty[synth.select(len(nonempty), 256, 9)]
    AS = synth.take_rows(A, S)
    semi = sg.semiring(MINPLUS)
    dA = to_dev(A)
    X1 = h.spgemm(semi, to_dev(AS), dA)
    X2 = h.spgemm(semi, X1, dA)
    torch.cuda.synchronize()
    h.check()
    orc = oracle.get()
    r1 = orc.spgemm(MINPLUS, AS, A)
    X1h = synth.CSR(AS.nrows, A.ncols, r1.rowptr, r1.col, r1.val)
    r2 = orc.spgemm(MINPLUS, X1h, A)
    compare(MINPLUS, *X1.to_numpy(), r1, "3-hop X1")
    compare(MINPLUS, *X2.to_numpy(), r2, "3-hop X2")


def test_precision_fp32_vs_fp64(h):
    """(+,x) with N(0,1) values: fp32 (compensated by the default rule, and
    plain) and fp64 runs on the same (fp32-representable) values against the
    fp64 oracle.  The gated comparisons are the bar; on top, compensation must
    not lose to plain summation: the median plain relative error over all
    sampled entries, and the worst error relative to sum|a*b| (the gate's
    scale, bounded even where entries cancel) over the rows the rule
    compensates (more than 64 terms), are no larger than plain fp32's."""
    import paper_2504_06408_amd as sg
    h.set_option("force_path", "auto")
    A = synth.rmat(13, 16, seed=1)
    v32 = synth.values(synth.VAL_F32_NORMAL, A.nnz, 0, 1, 2)
    A32 = A.with_values(v32)
    A64 = A.with_values(v32.astype(np.float64))
    rows = np.sort(synth.select(A.nrows, 600, 4))
    terms = np.diff(A.rowptr)[rows]
    ref = oracle.get().spgemm(F32, A32, A32, rows=rows)
    comp_entry = np.repeat(terms > 64, np.diff(ref.rowptr))
    assert comp_entry.sum() > 1000
    scale = np.maximum(np.abs(ref.val), ref.mag)
    e_c, C = check_product(h, F32, A32, A32, acc=sg.ACC_DEFAULT, rows=rows, what="fp32 compensated")
    g_c = np.abs(rows_of(C, rows)[2].astype(np.float64) - ref.val) / scale
    e_p, C = check_product(h, F32, A32, A32, acc=sg.ACC_PLAIN, rows=rows, what="fp32 plain")
    g_p = np.abs(rows_of(C, rows)[2].astype(np.float64) - ref.val) / scale
    e_64, _ = check_product(h, F64, A64, A64, rows=rows, what="fp64")
    assert e_c[1] <= e_p[1], (e_c, e_p)
    assert g_c[comp_entry].max() <= g_p[comp_entry].max(), (g_c[comp_entry].max(), g_p[comp_entry].max())
    print(json.dumps({"max_rel_fp32_comp": e_c[0], "median_rel_fp32_comp": e_c[1], "max_rel_fp32_plain": e_p[0],
                      "median_rel_fp32_plain": e_p[1], "max_rel_fp64": e_64[0],
                      "max_gated_comp_rows_fp32_comp": float(g_c[comp_entry].max()),
                      "max_gated_comp_rows_fp32_plain": float(g_p[comp_entry].max())}))


def test_autotuner_writes_table(h, tmp_path):
    """The tuner searches the knobs the slab path reads and keys its table by
    semiring and value width; a tuned handle (and a new handle made from the
    table) still meets the oracle; a table made for another semiring is
    refused."""
    import paper_2504_06408_amd as sg
    h.set_option("force_path", "auto")
    A = with_vals(synth.rmat(12, 16, seed=3), MINPLUS, 4)
    dA = to_dev(A)
    path = os.path.join(str(tmp_path), "tune.json")
    h.tune(sg.semiring(MINPLUS), dA, dA, path)
    t = json.load(open(path))
    assert t["semiring"] == MINPLUS and t["value_bytes"] == 4
    assert t["hash_max_products"] in (1024, 2048, 4096)
    assert 14 <= t["slab_log"] <= 17
    assert t["light_cap"] in (7168, 3584, 1792)  # the 4-byte light cap and its halves
    assert t["tuned_ms"] <= t["default_ms"] and len(t["timings_ms"]) >= 5
    check_product(h, MINPLUS, A, A, what="tuned")
    h2 = sg.Handle(0, tuning=path)
    try:
        check_product(h2, MINPLUS, A, A, what="handle made from the table")
        h2.tune_load(MINPLUS, path)
        with pytest.raises(sg.SgError) as e:
            h2.tune_load(F64, path)
        assert e.value.status == -3
    finally:
        h2.close()
    # the autotuner leaves the handle on the tuned settings; restore the defaults
    h.set_option("hash_max_products", 4096)
    h.set_option("slab_log", 0)
    h.set_option("light_cap", 0)


@pytest.mark.parametrize("sr", [BOOL, I64])
def test_rmat18_full_scale(h, sr):
    """R-MAT scale 18 A.A (config sizes): stratified sampled rows against the
    oracle plus whole-matrix invariants computed on the GPU with torch."""
    import torch
    import paper_2504_06408_amd as sg
    h.set_option("force_path", "auto")
    A = synth.rmat(18, 16, seed=1)
    if sr == BOOL:
        A = A.with_values(synth.values(synth.VAL_ONES, A.nnz, 0, 0, 2))
    else:
        A = A.with_values(synth.values(synth.VAL_I64_UNIFORM, A.nnz, 1, 9, 2))
    dA = to_dev(A)
    C = h.spgemm(sg.semiring(sr), dA, dA)
    torch.cuda.synchronize()
    h.check()
    # stratified sample: rows from every product-count decade
    p = np.zeros(A.nrows, np.int64)
    np.add.at(p, np.repeat(np.arange(A.nrows), np.diff(A.rowptr)), np.diff(A.rowptr)[A.col])
    rows = []
    for lo, hi in [(1, 64), (65, 4096), (4097, 65536), (65537, 1 << 40)]:
        cand = np.nonzero((p >= lo) & (p <= hi))[0]
        if len(cand):
            rows.extend(cand[synth.select(len(cand), min(12, len(cand)), lo)])
    rows = np.sort(np.array(rows, np.int64))
    got = rows_of(C, rows)
    ref = oracle.get().spgemm(sr, A, A, rows=rows)
    compare(sr, *got, ref, "s18 sampled rows")
    # invariants over all rows
    rp = C.rowptr.cpu().numpy()
    if sr == BOOL:
        has = np.zeros(A.nrows, bool)
        np.logical_or.at(has, np.repeat(np.arange(A.nrows), np.diff(A.rowptr)), np.diff(A.rowptr)[A.col] > 0)
        assert np.array_equal(np.diff(rp) > 0, has)
        assert int(C.val.min()) == 1
    else:
        # row sums C.1 = A.(A.1): sums of int64 per row via a GPU segment sum
        counts = torch.from_numpy(np.diff(rp)).to("cuda")
        ids = torch.repeat_interleave(torch.arange(A.nrows, device="cuda"), counts)
        csum = torch.zeros(A.nrows, dtype=torch.int64, device="cuda").index_add_(0, ids, C.val).cpu().numpy()
        a1 = np.zeros(A.nrows, np.int64)
        rows_of_a = np.repeat(np.arange(A.nrows), np.diff(A.rowptr))
        np.add.at(a1, rows_of_a, A.val)
        aa1 = np.zeros(A.nrows, np.int64)
        np.add.at(aa1, rows_of_a, A.val * a1[A.col])
        assert np.array_equal(csum, aa1)
