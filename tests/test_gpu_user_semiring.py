"""GPU parity of semirings defined at run time (paper, Section 2.2: the user
redefines the entry type, (+), (x), zero and one).  Each definition is
compiled with hipRTC into the library's own numeric kernels and compared with
the oracle's definition of the same semiring, element by element: (max,+)
float32, (max,x) float64 and (min,max) int64 bit for bit, a run-time (min,+)
bit for bit against the built-in one, a run-time (+,x) float64 within the
gated tolerance, and (+,x) over uint32 against the int64 oracle modulo 2^32;
on every row path (small, hash, column slab, whole-row tiles), merges, CSC
operands, the no-allocation entry point and the power driver."""
import numpy as np
import pytest

import oracle
import synth
from helpers import F64, I64, MINPLUS, assert_exact, with_vals
from gpu_helpers import compare, rows_of, to_dev

pytestmark = pytest.mark.gpu

DEFS = {
    "max_plus_f32": dict(value_type="float", add="a > b ? a : b", mul="a + b", zero="-__builtin_huge_valf()",
                         one="0.0f", idempotent=True),
    "max_times_f64": dict(value_type="double", add="a > b ? a : b", mul="a * b", zero="0.0", one="1.0",
                          idempotent=True),
    "min_max_i64": dict(value_type="int64_t", add="a < b ? a : b", mul="a > b ? a : b", zero="INT64_MAX",
                        one="INT64_MIN", idempotent=True),
    "min_plus_f32": dict(value_type="float", add="a < b ? a : b", mul="a + b", zero="__builtin_huge_valf()",
                         one="0.0f", idempotent=True),
    "plus_times_f64": dict(value_type="double", add="a + b", mul="a * b", zero="0.0", one="1.0"),
    "plus_times_u32": dict(value_type="uint32_t", add="a + b", mul="a * b", zero="0u", one="1u"),
}
# oracle semiring and value recipe of each definition
ORACLE = {"max_plus_f32": (oracle.MAX_PLUS_F32, "maxplus"), "max_times_f64": (oracle.MAX_TIMES_F64, "pos64"),
          "min_max_i64": (oracle.MIN_MAX_I64, "i64"), "min_plus_f32": (oracle.MIN_PLUS_F32, "maxplus"),
          "plus_times_f64": (oracle.PLUS_TIMES_F64, "wide64")}


@pytest.fixture(scope="module")
def h():
    import paper_2504_06408_amd as sg
    hd = sg.Handle(0)
    yield hd
    hd.close()


_SR = {}


def _sr(h, name):
    if name not in _SR:
        _SR[name] = h.define_semiring(**DEFS[name])
    return _SR[name]


def _vals(kind, n, seed):
    if kind == "maxplus":
        return synth.values(synth.VAL_F32_UNIFORM, n, -50.0, 100.0, seed)
    if kind == "pos64":
        return synth.values(synth.VAL_F64_UNIFORM, n, 0.5, 2.0, seed)
    if kind == "wide64":
        return synth.values(synth.VAL_F64_UNIFORM, n, -1.0, 1.0, seed)
    return synth.values(synth.VAL_I64_UNIFORM, n, -(2 ** 40), 2 ** 40, seed)


def _reset(h):
    h.set_option("force_path", "auto")
    h.set_option("hash_max_products", 4096)
    h.set_option("dense_slab", 1)


def _run(h, s, A, B):
    import torch
    C = h.spgemm(s, to_dev(A), to_dev(B))
    torch.cuda.synchronize()
    h.check()
    return C


@pytest.mark.parametrize("name", ["max_plus_f32", "max_times_f64", "min_max_i64", "min_plus_f32", "plus_times_f64"])
@pytest.mark.parametrize("path", ["auto", "hash", "dense", "tiles"])
def test_user_semiring_matches_oracle(h, name, path):
    osr, kind = ORACLE[name]
    s = _sr(h, name)
    _reset(h)
    if path == "tiles":
        h.set_option("dense_slab", 0)
        h.set_option("force_path", "dense")
    elif path != "auto":
        h.set_option("force_path", path)
    try:
        A = synth.rmat(12, 16, seed=700)
        A = A.with_values(_vals(kind, A.nnz, 701))
        B = synth.er(4096, 20000, 24, 702)
        B = B.with_values(_vals(kind, B.nnz, 703))
        for L, R, what in ((A, A, "A.A"), (A, B, "A.B over 20000 columns")):
            C = _run(h, s, L, R)
            ref = oracle.get().spgemm(osr, L, R)
            compare(osr if osr <= 5 else {6: MINPLUS, 7: I64, 8: I64}[osr], *C.to_numpy(), ref, f"{name} {path} {what}")
    finally:
        _reset(h)


def test_runtime_min_plus_equals_builtin(h):
    """The run-time (min,+) and the built-in one give the same bits."""
    import paper_2504_06408_amd as sg
    A = synth.rmat(13, 16, seed=710)
    A = A.with_values(synth.values(synth.VAL_F32_UNIFORM, A.nnz, 1.0, 100.0, 711))
    C1 = _run(h, _sr(h, "min_plus_f32"), A, A)
    C2 = _run(h, sg.semiring(sg.MIN_PLUS_F32), A, A)
    r1, c1, v1 = C1.to_numpy()
    r2, c2, v2 = C2.to_numpy()
    assert np.array_equal(r1, r2) and np.array_equal(c1, c2)
    assert np.array_equal(v1.view(np.uint32), v2.view(np.uint32))


def test_uint32_ring_is_int64_mod_2_32(h):
    """(+,x) over uint32 wraps modulo 2^32: the int64 oracle's result reduced
    modulo 2^32 (wrapping arithmetic is a ring homomorphism)."""
    A = synth.rmat(12, 16, seed=720)
    v = synth.values(synth.VAL_I64_UNIFORM, A.nnz, -(2 ** 40), 2 ** 40, 721)
    C = _run(h, _sr(h, "plus_times_u32"), A.with_values(v.astype(np.uint32)), A.with_values(v.astype(np.uint32)))
    ref = oracle.get().spgemm(I64, A.with_values(v), A.with_values(v))
    rp, cl, vl = C.to_numpy()
    assert np.array_equal(rp, ref.rowptr) and np.array_equal(cl, ref.col)
    assert np.array_equal(vl.astype(np.uint64), (ref.val.astype(np.uint64) & np.uint64(0xFFFFFFFF)))


@pytest.mark.parametrize("name", ["max_plus_f32", "min_max_i64"])
def test_user_semiring_merge(h, name):
    import torch
    osr, kind = ORACLE[name]
    s = _sr(h, name)
    parts = [synth.er(3000, 5000, d, 730 + d) for d in (3, 7, 12)]
    parts = [p.with_values(_vals(kind, p.nnz, 740 + q)) for q, p in enumerate(parts)]
    C = h.merge(s, [to_dev(p) for p in parts])
    torch.cuda.synchronize()
    ref = oracle.get().merge(osr, parts)
    rp, cl, vl = C.to_numpy()
    assert np.array_equal(rp, ref.rowptr) and np.array_equal(cl, ref.col)
    assert_exact(vl, ref.val, f"{name} merge")


def test_user_semiring_noalloc_and_csc(h):
    """The no-allocation entry point and the CSC entry points with a run-time
    semiring."""
    import torch
    import paper_2504_06408_amd as sg
    from oracle import dcsc as odc
    s = _sr(h, "max_plus_f32")
    A = synth.rmat(11, 16, seed=750)
    A = A.with_values(_vals("maxplus", A.nnz, 751))
    dA = to_dev(A)
    rowptr, nnz = h.symbolic(dA, dA)
    C = sg.DeviceCSR(A.nrows, A.ncols, rowptr, torch.empty(nnz, dtype=torch.int32, device="cuda"),
                     torch.empty(nnz, dtype=torch.float32, device="cuda"))
    h.numeric_noalloc(s, dA, dA, C)
    torch.cuda.synchronize()
    ref = oracle.get().spgemm(oracle.MAX_PLUS_F32, A, A)
    rp, cl, vl = C.to_numpy()
    assert np.array_equal(cl, ref.col)
    assert_exact(vl, ref.val, "no-allocation (max,+)")
    Ac = odc.csr_to_csc(A)
    dAc = sg.DeviceCSC(A.nrows, A.ncols, torch.from_numpy(Ac.colptr).cuda(), torch.from_numpy(Ac.row).cuda(),
                       torch.from_numpy(np.ascontiguousarray(Ac.val)).cuda())
    Cc = h.spgemm_csc(s, dAc, dAc)
    refc = odc.csc_spgemm(oracle.get(), oracle.MAX_PLUS_F32, Ac, Ac)
    cp, rw, vc = Cc.to_numpy()
    assert np.array_equal(cp, refc.colptr) and np.array_equal(rw, refc.row)
    assert_exact(vc, np.asarray(refc.val, np.float32), "CSC (max,+)")


def test_user_semiring_power(h):
    """sg_power_run with a run-time (min,+): the distance matrix, the
    identity's one read from the definition."""
    from oracle import power as opw
    W = synth.rmat(9, 8, seed=760)
    W = W.with_values(synth.values(synth.VAL_I64_UNIFORM, W.nnz, 1, 20, 761).astype(np.float32))
    D, hops, prods, conv = h.power(_sr(h, "min_plus_f32"), to_dev(W), 0, self_loops=True, squaring=True,
                                   fixpoint=True)
    ref = opw.power(oracle.get(), MINPLUS, W, 0, self_loops=True, squaring=True, fixpoint=True)
    assert (hops, prods, conv) == (ref.hops, ref.products, ref.converged)
    rp, cl, vl = D.to_numpy()
    assert np.array_equal(rp, ref.D.rowptr) and np.array_equal(cl, ref.D.col)
    assert_exact(vl, ref.D.val, "run-time (min,+) distance matrix")


def test_user_semiring_errors_and_cache(h):
    import paper_2504_06408_amd as sg
    with pytest.raises(sg.SgError) as e:
        h.define_semiring("float", "a +* b", "a * b", "0.0f", "1.0f")
    assert e.value.status == -3 and "compile" in str(e.value)
    with pytest.raises(sg.SgError) as e:
        h.define_semiring("half", "a + b", "a * b", "0", "1")
    assert e.value.status == -1
    again = h.define_semiring(**DEFS["max_plus_f32"])
    assert again.id == _sr(h, "max_plus_f32").id and again.id >= 64
    A = to_dev(with_vals(synth.rmat(8, 8, seed=770), MINPLUS, 771))
    with pytest.raises(sg.SgError) as e:
        h.batch_plan(again, [A], [A])
    assert e.value.status == -3
