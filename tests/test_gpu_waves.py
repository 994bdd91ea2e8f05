"""GPU parity of memory-budgeted waves (sg_waves_*): a SUMMA grid whose
merge groups are cut into several waves, each a batched plan of its own;
every merged block of every wave equals the same block of the oracle's full
product (paper, Section 2.1: C_IJ = (+)_K A_IK B_KJ), and every stage
product equals the oracle's."""
import numpy as np
import pytest

import oracle
import synth
from helpers import EXACT, F64, I64, MINPLUS, with_vals
from gpu_helpers import compare, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import paper_2504_06408_amd as sg
    hd = sg.Handle(0)
    yield hd
    hd.close()


def _grid(sr, scale, g, seed):
    A = with_vals(synth.rmat(scale, 16, seed=seed), sr, seed + 1)
    blk = synth.block_split(A, g)
    full = oracle.get().spgemm(sr, A, A)
    Cb = synth.block_split(synth.CSR(A.nrows, A.ncols, full.rowptr, full.col, full.val), g)
    Mb = None if full.mag is None else synth.block_split(synth.CSR(A.nrows, A.ncols, full.rowptr, full.col, full.mag), g)
    As, Bs, go = [], [], [0]
    for I in range(g):
        for J in range(g):
            for K in range(g):
                As.append(blk[I][K])
                Bs.append(blk[K][J])
            go.append(len(As))
    return As, Bs, go, Cb, Mb


@pytest.mark.parametrize("sr", [I64, MINPLUS, F64])
def test_waves_match_oracle(h, sr):
    """R-MAT s13 cut 4x4 (64 stage products, 16 merges) under a budget that
    forces several waves; waves run out of order and one twice."""
    import paper_2504_06408_amd as sg
    from oracle import OracleResult
    g = 4
    As, Bs, go, Cb, Mb = _grid(sr, 13, g, 31)
    dA, dB = [to_dev(x) for x in As], [to_dev(x) for x in Bs]
    probe = h.waves(sg.semiring(sr), dA, dB, go, 1 << 40)
    assert probe.count == 1
    per_group = [2 * sum(probe.product_nnz[go[x]:go[x + 1]]) * (4 + sg.semiring(sr).value_bytes) for x in range(g * g)]
    probe.destroy()
    budget = max(per_group) + max(per_group) // 2
    W = h.waves(sg.semiring(sr), dA, dB, go, budget)
    assert W.count >= 3, (W.count, W.wave_bytes)
    assert all(b <= budget for b in W.wave_bytes)
    order = list(range(W.count))[::-1] + [0]
    for w in order:
        W.run(w)
        res = W.results()
        g0, g1 = W.wave_groups[w], W.wave_groups[w + 1]
        q0, q1 = go[g0], go[g1]
        assert len(res) == (q1 - q0) + (g1 - g0)
        for k, q in enumerate(range(q0, q1)):
            r = res[k]
            got = (sg._to_numpy(r.rowptr, r.nrows + 1, np.int64), sg._to_numpy(r.col, r.nnz, np.int32),
                   sg._to_numpy(r.val, r.nnz, sg.NP_DTYPE[sr]))
            assert r.nnz == W.product_nnz[q]
            compare(sr, *got, oracle.get().spgemm(sr, As[q], Bs[q]), f"wave {w} stage product {q}")
        for k, grp in enumerate(range(g0, g1)):
            r = res[(q1 - q0) + k]
            I, J = divmod(grp, g)
            got = (sg._to_numpy(r.rowptr, r.nrows + 1, np.int64), sg._to_numpy(r.col, r.nnz, np.int32),
                   sg._to_numpy(r.val, r.nnz, sg.NP_DTYPE[sr]))
            ref = Cb[I][J]
            refr = OracleResult(ref.rowptr, ref.col, ref.val, None if Mb is None else Mb[I][J].val)
            compare(sr, *got, refr, f"wave {w} merged block ({I},{J})")
    W.destroy()


def test_waves_group_over_budget(h):
    import paper_2504_06408_amd as sg
    As, Bs, go, _, _ = _grid(I64, 10, 2, 33)
    with pytest.raises(sg.SgError) as e:
        h.waves(sg.semiring(I64), [to_dev(x) for x in As], [to_dev(x) for x in Bs], go, 1024)
    assert e.value.status == -4
