"""GPU parity of the batched persistent path (one recorded graph over many
products and merges) against the oracle and against per-call products."""
import numpy as np
import pytest

import oracle
import synth
from helpers import ALL, BOOL, EXACT, F64, I64, MINPLUS, assert_close_gated, with_vals
from gpu_helpers import compare, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import paper_2504_06408_amd as sg
    hd = sg.Handle(0)
    yield hd
    hd.close()


def _check_results(sr, res, refs, what):
    for k, ((rp, cl, vl), ref) in enumerate(zip(res, refs)):
        compare(sr, rp, cl, vl, ref, f"{what} result {k}")


@pytest.mark.parametrize("sr", [F64, I64, MINPLUS])
def test_batch_er_products(h, sr):
    """A batch of ER products of uneven sizes (n log-uniform, d uniform)."""
    import paper_2504_06408_amd as sg
    h.set_option("force_path", "auto")
    ns, ds = synth.batch_params(12, 64, 4096, 4, 32, 5)
    As = [with_vals(synth.er(int(n), int(n), int(d), 100 + q), sr, 200 + q) for q, (n, d) in enumerate(zip(ns, ds))]
    Bs = [with_vals(synth.er(int(n), int(n), int(d), 300 + q), sr, 400 + q) for q, (n, d) in enumerate(zip(ns, ds))]
    dA = [to_dev(a) for a in As]
    dB = [to_dev(b) for b in Bs]
    plan = h.batch_plan(sg.semiring(sr), dA, dB)
    for rep in range(3):  # graph replays, each checked
        plan.execute()
        res = plan.results_numpy()
        _check_results(sr, res, [oracle.get().spgemm(sr, a, b) for a, b in zip(As, Bs)], f"ER batch rep {rep}")
    plan.destroy()


@pytest.mark.parametrize("sr", [F64, I64, MINPLUS, BOOL])
@pytest.mark.parametrize("path", ["auto", "dense"])
def test_batch_summa_grid(h, sr, path):
    """Sparse SUMMA on a 4x4 block grid (paper Section 2.1): 64 block
    products and 16 merges in one plan; each merged block equals the same
    block of the oracle's full product."""
    import paper_2504_06408_amd as sg
    h.set_option("force_path", path)
    try:
        A = with_vals(synth.rmat(11, 16, seed=5), sr, 6)
        g = 4
        blk = synth.block_split(A, g)
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
        full = oracle.get().spgemm(sr, A, A)
        Cb = synth.block_split(synth.CSR(A.nrows, A.ncols, full.rowptr, full.col, full.val), g)
        Mb = None if full.mag is None else synth.block_split(synth.CSR(A.nrows, A.ncols, full.rowptr, full.col,
                                                                         full.mag), g)
        for rep in range(2):
            plan.execute()
            res = plan.results_numpy()
            # products
            _check_results(sr, res[:8], [oracle.get().spgemm(sr, a, b) for a, b in zip(As[:8], Bs[:8])],
                           f"SUMMA products rep {rep}")
            # merges against the oracle's full product, block by block
            for q in range(g * g):
                I, J = divmod(q, g)
                rp, cl, vl = res[len(As) + q]
                ref = Cb[I][J]
                assert np.array_equal(rp, ref.rowptr) and np.array_equal(cl, ref.col), (I, J, rep)
                if sr == F64:
                    assert_close_gated(vl, ref.val, Mb[I][J].val, 1e-12, f"SUMMA merge {I},{J}")
                else:
                    assert np.array_equal(vl.view(np.uint8), ref.val.view(np.uint8)), (I, J, rep)
        plan.destroy()
    finally:
        h.set_option("force_path", "auto")


@pytest.mark.parametrize("sr", EXACT)
def test_batch_matches_per_call_bitwise(h, sr):
    import torch
    import paper_2504_06408_amd as sg
    h.set_option("force_path", "auto")
    As = [with_vals(synth.rmat(10, 16, seed=50 + q), sr, 60 + q) for q in range(3)]
    dA = [to_dev(a) for a in As]
    plan = h.batch_plan(sg.semiring(sr), dA, dA)
    plan.execute()
    res = plan.results_numpy()
    # eager work between replays, then replay again
    for q in range(3):
        C = h.spgemm(sg.semiring(sr), dA[q], dA[q])
        torch.cuda.synchronize()
        rp, cl, vl = C.to_numpy()
        assert np.array_equal(rp, res[q][0]) and np.array_equal(cl, res[q][1])
        assert np.array_equal(vl.view(np.uint8), res[q][2].view(np.uint8))
    plan.execute()
    res2 = plan.results_numpy()
    for a, b in zip(res, res2):
        for x, y in zip(a, b):
            assert np.array_equal(x.view(np.uint8), y.view(np.uint8))
    plan.destroy()


def test_batch_pool_too_small(h):
    import paper_2504_06408_amd as sg
    A = with_vals(synth.rmat(9, 16, seed=70), F64, 71)
    dA = to_dev(A)
    with pytest.raises(sg.SgError) as e:
        h.batch_plan(sg.semiring(F64), [dA], [dA], pool_bytes=1024)
    assert e.value.status == -4


def test_batch_shape_errors(h):
    import paper_2504_06408_amd as sg
    A = with_vals(synth.er(20, 30, 3, 1), F64, 2)
    dA = to_dev(A)
    with pytest.raises(sg.SgError) as e:
        h.batch_plan(sg.semiring(F64), [dA], [dA])
    assert e.value.status == -2


@pytest.mark.parametrize("sr", ALL)
@pytest.mark.parametrize("path", ["auto", "dense"])
def test_batch_single_product(h, sr, path):
    """A plan of one product and no merges is recorded on the column-slab
    path: results match the oracle, replays pick up new values, and repeated
    replays agree bit for bit on exact semirings."""
    import torch
    import paper_2504_06408_amd as sg
    import oracle
    from gpu_helpers import compare
    h.set_option("force_path", path)
    try:
        A = with_vals(synth.rmat(11, 16, seed=80), sr, 81)
        dA = to_dev(A)
        plan = h.batch_plan(sg.semiring(sr), [dA], [dA])
        plan.execute()
        rp, cl, vl = plan.results_numpy()[0]
        compare(sr, rp, cl, vl, oracle.get().spgemm(sr, A, A), "single product")
        A2 = with_vals(A, sr, 82)
        dA.val.copy_(torch.from_numpy(np.ascontiguousarray(A2.val)).to(dA.val.device))
        plan.execute()
        rp2, cl2, vl2 = plan.results_numpy()[0]
        compare(sr, rp2, cl2, vl2, oracle.get().spgemm(sr, A2, A2), "single product, new values")
        plan.execute()
        rp3, cl3, vl3 = plan.results_numpy()[0]
        assert np.array_equal(rp2, rp3) and np.array_equal(cl2, cl3)
        if sr in EXACT:
            assert np.array_equal(vl2.view(np.uint8), vl3.view(np.uint8))
        plan.destroy()
    finally:
        h.set_option("force_path", "auto")
