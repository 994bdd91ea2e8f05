"""GPU parity of the semiring merge C = P_0 (+) ... (+) P_{S-1} against the
oracle, and the block (Sparse SUMMA) identity C_IJ = (+)_K A_IK B_KJ computed
entirely on the GPU."""
import numpy as np
import pytest

import oracle
import synth
from helpers import ALL, EXACT, with_vals
from gpu_helpers import compare, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import paper_2504_06408_amd as sg
    hd = sg.Handle(0)
    yield hd
    hd.close()


def _gpu_merge(h, sr, parts, acc=0):
    import torch
    import paper_2504_06408_amd as sg
    C = h.merge(sg.semiring(sr, acc), [to_dev(p) for p in parts])
    torch.cuda.synchronize()
    h.check()
    return C


def _parts(sr, n, ncols, specs, seed):
    out = []
    for q, (kind, x) in enumerate(specs):
        if kind == "er":
            P = synth.er(n, ncols, x, seed + q)
        else:
            P = synth.rmat(x, 16, seed=seed + q)
            assert P.nrows == n
        out.append(with_vals(P, sr, seed + 50 + q))
    return out


@pytest.mark.parametrize("sr", ALL)
@pytest.mark.parametrize("path", ["auto", "small", "hash", "dense"])
def test_merge_paths(h, sr, path):
    h.set_option("force_path", path)
    try:
        parts = _parts(sr, 2048, 2048, [("rmat", 11), ("er", 3), ("rmat", 11), ("er", 40), ("rmat", 11)], 7)
        C = _gpu_merge(h, sr, parts)
        ref = oracle.get().merge(sr, parts)
        compare(sr, *C.to_numpy(), ref, f"merge {path}")
    finally:
        h.set_option("force_path", "auto")


@pytest.mark.parametrize("sr", ALL)
def test_merge_wide_and_single(h, sr):
    parts = _parts(sr, 300, 1_100_000, [("er", 900), ("er", 2000), ("er", 5)], 17)
    C = _gpu_merge(h, sr, parts)
    compare(sr, *C.to_numpy(), oracle.get().merge(sr, parts), "merge wide")
    one = _gpu_merge(h, sr, parts[:1])
    compare(sr, *one.to_numpy(), oracle.get().merge(sr, parts[:1]), "merge single")


@pytest.mark.parametrize("sr", EXACT)
def test_block_identity_on_gpu(h, sr):
    """Paper Section 2.1: with A and B cut into a 4x4 grid, merging the four
    GPU block products of each output block gives that block of A.B."""
    import paper_2504_06408_amd as sg
    A = with_vals(synth.rmat(11, 16, seed=90), sr, 91)
    g = 4
    Ab = synth.block_split(A, g)
    full = oracle.get().spgemm(sr, A, A)
    Cfull = synth.CSR(A.nrows, A.ncols, full.rowptr, full.col, full.val)
    Cb = synth.block_split(Cfull, g)
    semi = sg.semiring(sr)
    for I in range(g):
        for J in range(g):
            parts = [h.spgemm(semi, to_dev(Ab[I][K]), to_dev(Ab[K][J])) for K in range(g)]
            M = h.merge(semi, parts)
            ref = Cb[I][J]
            rp, cl, vl = M.to_numpy()
            assert np.array_equal(rp, ref.rowptr) and np.array_equal(cl, ref.col), (I, J)
            assert np.array_equal(vl.view(np.uint8), ref.val.view(np.uint8)), (I, J)
