#!/usr/bin/env python3
"""Benchmark of the semiring sparse product on one MI355X.

Default workload: R-MAT scale 20 (2^20 vertices, 16 edge draws per vertex,
quadrant probabilities (0.57, 0.19, 0.19, 0.05), duplicates removed), float32
weights uniform in [1, 100), C = A.A over the (min,+) semiring.  One step is
the whole two-pass product through the C ABI: row analysis, binning,
symbolic pass (with its one host read-back of nnz(C)), and numeric pass into
a pre-reserved output buffer.  Inputs are resident in HBM before timing.

Prints one JSON line: semiring products per second (value), the HBM GB/s of
the algorithmic byte model, the roofline of the dominant kernel (timed live
with HIP events on the library's stream) and the CPU oracle's throughput on a
bounded sample of the same rows.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "semiring products/s + HBM GB/s, R-MAT s20 A·A; batched vs per-call"
PEAK_HBM_GBPS = 8000.0

WORKLOADS = {
    # name: (generator, semiring, value kind, lo, hi, description)
    "rmat20_minplus": ("rmat", 20, 5, "f32u", 1.0, 100.0,
                       "R-MAT scale 20, edge factor 16, (a,b,c,d)=(0.57,0.19,0.19,0.05), dedup, fp32 weights "
                       "U[1,100), (min,+) C=A.A"),
    "rmat18_bool": ("rmat", 18, 4, "ones", 0, 0,
                    "R-MAT scale 18, edge factor 16, (or,and) C=A.A, all-true values"),
    "rmat18_i64": ("rmat", 18, 1, "i64u", 1, 9, "R-MAT scale 18, edge factor 16, (+,x) int64 C=A.A, values U{1..9}"),
    "rmat20_f32": ("rmat", 20, 2, "f32n", 0, 1,
                   "R-MAT scale 20, edge factor 16, (+,x) fp32 values N(0,1), compensated accumulation, C=A.A"),
    "er4096_f64": ("er", 4096, 3, "f64u", 0, 1, "Erdos-Renyi n=4096, 8 per row, (+,x) fp64 U[0,1), C=A.B"),
}
VAL_BYTES = {1: 8, 2: 4, 3: 8, 4: 1, 5: 4}
DTYPE = {1: "int64", 2: "f32", 3: "f64", 4: "u8", 5: "f32"}


def make_inputs(name):
    import synth
    kind, size, sr, vk, lo, hi, desc = WORKLOADS[name]
    vmap = {"f32u": synth.VAL_F32_UNIFORM, "ones": synth.VAL_ONES, "i64u": synth.VAL_I64_UNIFORM,
            "f32n": synth.VAL_F32_NORMAL, "f64u": synth.VAL_F64_UNIFORM}
    if kind == "rmat":
        A = synth.rmat(size, 16, seed=1)
        A = A.with_values(synth.values(vmap[vk], A.nnz, lo, hi, 2))
        B = A
    else:
        A = synth.er(size, size, 8, 1).with_values(synth.values(vmap[vk], size * 8, lo, hi, 11))
        B = synth.er(size, size, 8, 2).with_values(synth.values(vmap[vk], size * 8, lo, hi, 12))
    return A, B, sr, desc


HERE = os.path.dirname(os.path.abspath(__file__))
COUNTERS = os.path.join(HERE, "profiles", "rmat20_minplus_hbm_counters.md")


def kernel_sources_sha256() -> str:
    """Digest of the HIP sources of the library (any edit changes it)."""
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "paper_2504_06408_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp", ".cpp")):
            h.update(f.encode())
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` (rocprofv3 FETCH_SIZE + WRITE_SIZE,
    scaled by a plain copy kernel) from the committed counter summary, when
    that summary was taken on the current kernel sources; otherwise None."""
    if workload != "rmat20_minplus" or not os.path.exists(COUNTERS):
        return None
    text = open(COUNTERS).read()
    sha = re.search(r"^kernel_sources_sha256: (\S+)$", text, re.M)
    per = dict(re.findall(r"^traffic_bytes_per_launch\.(\w+): (\d+)$", text, re.M))
    if not sha or sha.group(1) != kernel_sources_sha256() or kernel not in per:
        return None
    return int(per[kernel])


def products_per_row(A, B):
    lens = np.diff(B.rowptr)[A.col]
    p = np.zeros(A.nrows, dtype=np.int64)
    np.add.at(p, np.repeat(np.arange(A.nrows), np.diff(A.rowptr)), lens)
    return p


def cpu_baseline(A, B, sr, p, target_s):
    """The oracle, as it is, on a growing uniform sample of rows until one
    run takes about target_s seconds on all host threads."""
    import oracle
    import synth
    orc = oracle.get()
    rng_rows = synth.select(A.nrows, min(A.nrows, 1 << 20), 3)  # a fixed random order of rows
    order = np.argsort(synth.values(synth.VAL_F64_UNIFORM, len(rng_rows), 0, 1, 4))
    rows_all = rng_rows[order]
    k = 256
    while True:
        rows = np.sort(rows_all[:k])
        t0 = time.perf_counter()
        orc.spgemm(sr, A, B, rows=rows)
        dt = time.perf_counter() - t0
        if dt >= target_s or k >= len(rows_all):
            break
        k = min(len(rows_all), int(k * max(2.0, min(8.0, 0.9 * target_s / max(dt, 1e-3)))))
    prods = int(p[rows].sum())
    return {"value": prods / dt, "unit": "semiring products/s", "cores": orc.num_threads(), "kind": "oracle",
            "sample": f"{k} rows drawn uniformly (seed 3) of the same product, {prods} products, {dt:.2f} s"}


def _device_rows(C, rows):
    """Host copies (rowptr, col, val) of rows `rows` of a device CSR."""
    import torch
    rp = C.rowptr.cpu().numpy()
    rows = np.asarray(rows, dtype=np.int64)
    g_rp = np.zeros(len(rows) + 1, np.int64)
    np.cumsum(rp[rows + 1] - rp[rows], out=g_rp[1:])
    if g_rp[-1] == 0:
        return g_rp, np.zeros(0, np.int32), C.val[:0].cpu().numpy()
    idx = np.concatenate([np.arange(rp[r], rp[r + 1]) for r in rows])
    ti = torch.from_numpy(idx).to(C.col.device)
    return g_rp, C.col[ti].cpu().numpy(), C.val[ti].cpu().numpy()


def compare_rows(sr, g_rp, g_col, g_val, ref):
    """GPU rows against oracle rows: the pattern exactly; values bit for bit
    (int64, bool, (min,+)) or within the gated tolerance with plain max /
    median relative error (float sums)."""
    out = {"rows": int(len(g_rp) - 1), "entries": int(g_rp[-1]),
           "pattern_equal": bool(np.array_equal(g_rp, ref.rowptr) and np.array_equal(g_col, ref.col))}
    if not out["pattern_equal"]:
        return out
    if sr in (1, 4, 5):
        a, b = g_val, ref.val
        same = (a.view(np.uint8).reshape(len(a), -1) == b.view(np.uint8).reshape(len(b), -1)).all(axis=1)
        if a.dtype.kind == "f":
            same |= (a == 0) & (b == 0)
        out["bit_exact"] = bool(same.all())
    else:
        tol = 1e-12 if sr == 3 else 1e-5
        got, r = g_val.astype(np.float64), ref.val
        scale = np.maximum(np.abs(r), ref.mag)
        out["within_tol"] = bool((np.abs(got - r) <= tol * scale).all())
        nz = r != 0
        rel = np.abs(got[nz] - r[nz]) / np.abs(r[nz])
        out["max_rel_err"] = float(rel.max()) if len(rel) else 0.0
        out["median_rel_err"] = float(np.median(rel)) if len(rel) else 0.0
    return out


def merge_reports(reps):
    """One summary of several compare_rows reports."""
    out = {"rows": sum(r["rows"] for r in reps), "entries": sum(r["entries"] for r in reps),
           "pattern_equal": all(r["pattern_equal"] for r in reps)}
    if "bit_exact" in reps[0]:
        out["bit_exact"] = all(r.get("bit_exact", False) for r in reps)
    if "within_tol" in reps[0]:
        out["within_tol"] = all(r.get("within_tol", False) for r in reps)
        out["max_rel_err"] = max(r.get("max_rel_err", 0.0) for r in reps)
    return out


def stratified_rows(p, per_bin, seed_base=0):
    """Up to per_bin rows from each product-count decade."""
    import synth
    rows = []
    edges = [1, 64, 4096, 65536, 1 << 20, 1 << 62]
    for lo, hi in zip(edges[:-1], edges[1:]):
        cand = np.nonzero((p >= lo) & (p < hi))[0]
        if len(cand):
            rows.extend(cand[synth.select(len(cand), min(per_bin, len(cand)), lo + seed_base)].tolist())
    return np.sort(np.array(rows, dtype=np.int64))


def parity_sample(A, B, sr, p, C, per_bin=12, rows=None):
    """Rows of the timed result against the oracle: a stratified sample over
    product-count decades, or the given rows."""
    import oracle
    if rows is None:
        rows = stratified_rows(p, per_bin)
    rows = np.sort(np.asarray(rows, dtype=np.int64))
    ref = oracle.get().spgemm(sr, A, B, rows=rows)
    return compare_rows(sr, *_device_rows(C, rows), ref)


def batched_leg(sg, torch, h, sr, dA, dB, P, steps, ms_per_call):
    """The same product through the batched path: one plan (sized once),
    then whole-pipeline graph replays with no host round trip."""
    t0 = time.perf_counter()
    plan = h.batch_plan(sr, [dA], [dB])
    t_plan = time.perf_counter() - t0
    plan.execute()
    torch.cuda.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.execute()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    plan.results()  # raises on pool overflow or a consistency error
    plan.destroy()
    return {"ms_per_step": round(ms, 4), "value": P / (ms * 1e-3), "unit": "semiring products/s",
            "speedup_vs_per_call": round(ms_per_call / ms, 4), "plan_s": round(t_plan, 3)}


def summa_leg(sg, torch, h, scale, steps):
    """Sparse SUMMA emulation on one GPU: R-MAT A cut into an 8x8 block grid;
    all 512 stage products A_IK.A_KJ (fp64 (+,x)) and the 64 merges of each
    output block, batched (one graph) against per-call (one symbolic +
    numeric call per product and per merge)."""
    import synth
    A = synth.rmat(scale, 16, seed=1)
    A = A.with_values(synth.values(synth.VAL_F64_UNIFORM, A.nnz, 0, 1, 2))
    g = 8
    blk = synth.block_split(A, g)
    dblk = [[sg.DeviceCSR.from_host(blk[I][J]) for J in range(g)] for I in range(g)]
    As, Bs, go = [], [], [0]
    for I in range(g):
        for J in range(g):
            for K in range(g):
                As.append(dblk[I][K])
                Bs.append(dblk[K][J])
            go.append(len(As))
    sr = sg.semiring(sg.PLUS_TIMES_F64)
    nb = np.diff(A.rowptr)
    prods = 0
    for I in range(g):
        for J in range(g):
            for K in range(g):
                a, b = blk[I][K], blk[K][J]
                prods += int(np.diff(b.rowptr)[a.col].sum())

    def per_call():
        outs = []
        for I in range(g):
            for J in range(g):
                parts = [h.spgemm(sr, dblk[I][K], dblk[K][J]) for K in range(g)]
                outs.append(h.merge(sr, parts))
        return outs

    per_call()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        per_call()
    torch.cuda.synchronize()
    ms_pc = (time.perf_counter() - t0) * 1e3 / steps
    plan = h.batch_plan(sr, As, Bs, go)
    plan.execute()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.execute()
    torch.cuda.synchronize()
    ms_b = (time.perf_counter() - t0) * 1e3 / steps
    par = summa_parity(sg, A, g, plan, len(As), per_bin=8)
    plan.destroy()
    return {"workload": f"R-MAT s{scale} cut 8x8, 512 fp64 (+,x) stage products + 64 merges", "products": prods,
            "ms_per_call_path": round(ms_pc, 3), "ms_batched": round(ms_b, 3),
            "batched_speedup": round(ms_pc / ms_b, 3), "batched_products_per_s": prods / (ms_b * 1e-3),
            "parity_sample": par}


def summa_parity(sg, A, g, plan, nprod, per_bin=8):
    """Block identity (paper, Section 2.1) on sampled rows: row i of output
    block row I, read across the g merged blocks (I, J) with their column
    offsets, equals row I*rb + i of the oracle's full A.A.  Rows are
    stratified by product count over the whole matrix."""
    import oracle
    p = products_per_row(A, A)
    rows = stratified_rows(p, per_bin, 7)
    rb = -(-A.nrows // g)
    cb = -(-A.ncols // g)
    sid = 3
    res = plan.results()
    views = [sg.view_results(r, sid) for r in res[nprod:]]
    g_rp = np.zeros(len(rows) + 1, np.int64)
    cols, vals = [], []
    for k, r in enumerate(rows):
        I, i = divmod(int(r), rb)
        n_r = 0
        for J in range(g):
            brp, bcl, bvl = _device_rows(views[I * g + J], [i])
            cols.append(bcl.astype(np.int64) + J * cb)
            vals.append(bvl)
            n_r += len(bcl)
        g_rp[k + 1] = g_rp[k] + n_r
    ref = oracle.get().spgemm(sid, A, A, rows=rows)
    out = compare_rows(sid, g_rp, np.concatenate(cols).astype(np.int32), np.concatenate(vals), ref)
    out["check"] = "merged blocks across each sampled row vs the oracle's full A.A"
    return out


def summa_waves_leg(sg, torch, h, scale, budget_frac=0.9, per_bin=4):
    """The 8x8 Sparse SUMMA emulation at a scale whose 512 stage outputs do
    not fit the GPU together (scale 22: ~1.1 TB of fp64 stage outputs): every
    product is sized by a symbolic pass, the 64 output blocks are cut into
    waves whose outputs fit a budget, and each wave runs as one batched plan
    (graph replay) that is checked and freed before the next.  Time: the sum
    of the waves' replays (each plan's one-off build is reported apart).
    Check: the block identity (paper, Section 2.1) on stratified rows."""
    import oracle
    import synth
    t0 = time.perf_counter()
    A = synth.rmat(scale, 16, seed=1)
    A = A.with_values(synth.values(synth.VAL_F64_UNIFORM, A.nnz, 0, 1, 2))
    g = 8
    blk = synth.block_split(A, g)
    t_gen = time.perf_counter() - t0
    dblk = [[sg.DeviceCSR.from_host(blk[I][J]) for J in range(g)] for I in range(g)]
    As, Bs, go = [], [], [0]
    prods = 0
    for I in range(g):
        for J in range(g):
            for K in range(g):
                As.append(dblk[I][K])
                Bs.append(dblk[K][J])
                prods += int(np.diff(blk[K][J].rowptr)[blk[I][K].col].sum())
            go.append(len(As))
    free, _ = torch.cuda.mem_get_info()
    budget = int(budget_frac * free)
    sr = sg.semiring(sg.PLUS_TIMES_F64)
    t0 = time.perf_counter()
    W = h.waves(sr, As, Bs, go, budget)
    t_size = time.perf_counter() - t0
    print(f"# s{scale} waves: {W.count} waves, {sum(W.product_nnz)} stage-output entries, sized in {t_size:.1f}s",
          file=sys.stderr, flush=True)
    # sampled rows of the whole product: per row, its pieces from the g merged
    # blocks of its block row, collected wave by wave
    p = products_per_row(A, A)
    rows = stratified_rows(p, per_bin, 7)
    rb = -(-A.nrows // g)
    cb = -(-A.ncols // g)
    pieces = {}
    waves, t_plan = [], 0.0
    for w in range(W.count):
        t0 = time.perf_counter()
        W.run(w)  # builds the plan (one eager pass) and replays it once
        torch.cuda.synchronize()
        t_plan += time.perf_counter() - t0
        t0 = time.perf_counter()
        W.run(w)  # the timed replay
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        res = W.results()
        g0, g1 = W.wave_groups[w], W.wave_groups[w + 1]
        nprod = go[g1] - go[g0]
        wp = 0
        for grp in range(g0, g1):
            I, J = divmod(grp, g)
            wp += sum(int(np.diff(blk[K][J].rowptr)[blk[I][K].col].sum()) for K in range(g))
            view = sg.view_results(res[nprod + grp - g0], 3)
            for r in rows:
                if int(r) // rb == I:
                    _, bcl, bvl = _device_rows(view, [int(r) % rb])
                    pieces[(int(r), J)] = (bcl.astype(np.int64) + J * cb, bvl)
        waves.append({"groups": g1 - g0, "products": wp, "out_bytes_bound": int(W.wave_bytes[w]),
                      "ms": round(ms, 3)})
        print(f"# wave {w}: {g1 - g0} blocks, {wp:.3e} products, {ms:.1f} ms", file=sys.stderr, flush=True)
    W.destroy()
    del dblk, As, Bs
    torch.cuda.empty_cache()
    g_rp = np.zeros(len(rows) + 1, np.int64)
    cols, vals = [], []
    for k, r in enumerate(rows):
        n_r = 0
        for J in range(g):
            c, v = pieces[(int(r), J)]
            cols.append(c)
            vals.append(v)
            n_r += len(c)
        g_rp[k + 1] = g_rp[k] + n_r
    ref = oracle.get().spgemm(3, A, A, rows=rows)
    par = compare_rows(3, g_rp, np.concatenate(cols).astype(np.int32), np.concatenate(vals), ref)
    par["check"] = "merged blocks across each sampled row vs the oracle's full A.A"
    ms_total = sum(x["ms"] for x in waves)
    return {"workload": f"R-MAT s{scale} cut 8x8, 512 fp64 (+,x) stage products + 64 merges, in waves",
            "products": prods, "stage_output_entries": int(sum(W.product_nnz)), "waves": waves,
            "wave_budget_bytes": budget, "ms_batched": round(ms_total, 3),
            "batched_products_per_s": prods / (ms_total * 1e-3), "plan_s": round(t_plan, 2),
            "sizing_s": round(t_size, 2), "generation_s": round(t_gen, 2), "parity_sample": par}


def three_hop_leg(sg, torch, h, A, dA, steps):
    """(min,+) 3-hop on a seeded panel S of 4096 non-empty rows of the s20
    graph: X1 = A[S,:].A, X2 = X1.A (rows S of (A.A).A).  Timed as the two
    products back to back; X2 rows sampled against the oracle bit for bit."""
    import oracle
    import synth
    nonempty = np.nonzero(np.diff(A.rowptr) > 0)[0]
    S = nonempty[synth.select(len(nonempty), min(4096, len(nonempty)), 9)]
    AS = synth.take_rows(A, S)
    dAS = sg.DeviceCSR.from_host(AS)
    sr = sg.semiring(sg.MIN_PLUS_F32)

    def run():
        X1 = h.spgemm(sr, dAS, dA)
        X2 = h.spgemm(sr, X1, dA)
        return X1, X2

    X1, X2 = run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        del X1, X2
        X1, X2 = run()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    h.check()
    deg = dA.rowptr[1:] - dA.rowptr[:-1]
    p1 = int(np.diff(A.rowptr)[AS.col].sum())
    p2 = int(deg[X1.col.long()].sum().item())
    orc = oracle.get()
    r1 = orc.spgemm(5, AS, A)
    X1h = synth.CSR(AS.nrows, A.ncols, r1.rowptr, r1.col, r1.val)
    x1n = X1.to_numpy()
    rows = np.sort(synth.select(AS.nrows, 24, 10))
    p_x1 = np.zeros(X1h.nrows, np.int64)
    par = parity_sample(X1h, A, 5, p_x1 + 1, X2, per_bin=0, rows=rows)
    out = {"workload": "R-MAT s20 (min,+) 3-hop panel: X1 = A[S,:].A, X2 = X1.A, |S| = 4096 seeded non-empty rows",
           "products": p1 + p2, "nnz_X1": int(X1.nnz), "nnz_X2": int(X2.nnz), "ms": round(ms, 3),
           "value": (p1 + p2) / (ms * 1e-3), "unit": "semiring products/s",
           "X1_equal_oracle": bool(np.array_equal(x1n[0], r1.rowptr) and np.array_equal(x1n[1], r1.col)
                                   and np.array_equal(x1n[2].view(np.uint32), r1.val.view(np.uint32))),
           "X2_parity_sample": par}
    del X1, X2, dAS
    return out


def precision_leg(sg, torch, h, scale):
    """(+,x) with N(0,1) values on the s20 pattern: fp32 storage with the
    default (compensated by rule) and plain fp32 accumulation, and a plain
    fp64 run on the same values, each against the fp64 oracle on stratified
    rows (max / median relative error, gated tolerance)."""
    import synth
    A = synth.rmat(scale, 16, seed=1)
    v32 = synth.values(synth.VAL_F32_NORMAL, A.nnz, 0, 1, 2)
    A32 = A.with_values(v32)
    A64 = A.with_values(v32.astype(np.float64))
    p = products_per_row(A, A)
    out = {"workload": f"R-MAT s{scale}, values N(0,1) stored in fp32, (+,x) C = A.A", "products": int(p.sum())}
    for name, M, sid, acc in (("fp32_compensated", A32, 2, sg.ACC_DEFAULT), ("fp32_plain", A32, 2, sg.ACC_PLAIN),
                              ("fp64_plain", A64, 3, 0)):
        dM = sg.DeviceCSR.from_host(M)
        sr = sg.semiring(sid, acc)
        C = h.spgemm(sr, dM, dM)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        del C
        C = h.spgemm(sr, dM, dM)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        h.check()
        res = parity_sample(M, M, sid, p, C)
        res["ms"] = round(ms, 3)
        res["value"] = int(p.sum()) / (ms * 1e-3)
        out[name] = res
        del C, dM
        torch.cuda.empty_cache()
    return out


def er_batch_leg(sg, torch, h, count, steps):
    """A batch of ER products (fp64 (+,x)): per instance n log-uniform in
    [1k, 64k], d uniform in {4..32} for A and B; one batched plan (graph
    replays) against a per-call loop."""
    import synth
    n, d = synth.batch_params(count, 1024, 65536, 4, 32, 5)
    As, Bs, hosts, prods = [], [], [], 0
    for i in range(count):
        a = synth.er(int(n[i]), int(n[i]), int(d[i]), 1000 + 2 * i)
        b = synth.er(int(n[i]), int(n[i]), int(d[i]), 1001 + 2 * i)
        a = a.with_values(synth.values(synth.VAL_F64_UNIFORM, a.nnz, 0, 1, 3000 + 2 * i))
        b = b.with_values(synth.values(synth.VAL_F64_UNIFORM, b.nnz, 0, 1, 3001 + 2 * i))
        prods += int(np.diff(b.rowptr)[a.col].sum())
        hosts.append((a, b))
        As.append(sg.DeviceCSR.from_host(a))
        Bs.append(sg.DeviceCSR.from_host(b))
    sr = sg.semiring(sg.PLUS_TIMES_F64)

    def per_call():
        return [h.spgemm(sr, a, b) for a, b in zip(As, Bs)]

    per_call()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        per_call()
    torch.cuda.synchronize()
    ms_pc = (time.perf_counter() - t0) * 1e3 / steps
    torch.cuda.empty_cache()
    plan = h.batch_plan(sr, As, Bs)
    plan.execute()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.execute()
    torch.cuda.synchronize()
    ms_b = (time.perf_counter() - t0) * 1e3 / steps
    # parity: every instance's largest row plus 4 random rows of 16
    # instances (the 8 largest and 8 drawn at random) against the oracle
    import oracle
    res = plan.results()
    pick = sorted(set(np.argsort(n)[-8:].tolist()) | set(synth.select(count, min(8, count), 21).tolist()))
    reps = []
    for q in pick:
        a, b = hosts[q]
        pq = products_per_row(a, b)
        rows = np.unique(np.concatenate([[int(np.argmax(pq))], synth.select(a.nrows, 4, 22 + q)]))
        Cq = sg.view_results(res[q], 3)
        reps.append(compare_rows(3, *_device_rows(Cq, rows), oracle.get().spgemm(3, a, b, rows=rows)))
    plan.destroy()
    par = merge_reports(reps)
    par["instances"] = len(pick)
    return {"workload": f"{count} ER fp64 (+,x) products, n log-uniform in [1k, 64k], d in {{4..32}}",
            "products": prods, "ms_per_call_path": round(ms_pc, 3), "ms_batched": round(ms_b, 3),
            "batched_speedup": round(ms_pc / ms_b, 3), "batched_products_per_s": prods / (ms_b * 1e-3),
            "parity_sample": par}


def measure_product(sg, torch, h, A, B, sr_id, steps, warmup, hash_max=None, workload=None):
    """Time `steps` whole two-pass products C = A.B (symbolic with its nnz
    read-back, then numeric into a pre-reserved output) after `warmup`
    untimed ones; return the figures, the roofline of the dominant
    single-kernel phase and the last result C (device)."""
    dev = "cuda:0"
    p = products_per_row(A, B)
    P = int(p.sum())
    dA = sg.DeviceCSR.from_host(A, dev)
    dB = dA if B is A else sg.DeviceCSR.from_host(B, dev)
    sr = sg.semiring(sr_id)
    vb = VAL_BYTES[sr_id]
    # pre-reserved output: sized by one symbolic pass before timing
    rowptr, nnzC = h.symbolic(dA, dB)
    col = torch.empty(nnzC, dtype=torch.int32, device=dev)
    val = torch.empty(nnzC, dtype={1: torch.int64, 2: torch.float32, 3: torch.float64, 4: torch.uint8,
                                   5: torch.float32}[sr_id], device=dev)

    def step():
        rp, nz = h.symbolic(dA, dB)
        C = sg.DeviceCSR(A.nrows, B.ncols, rp, col[:nz], val[:nz])
        h.numeric(sr, dA, dB, C)
        return C, nz

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    h.check()
    phase_runs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        C, nz = step()
        phase_runs.append(h.timings())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    h.check()
    assert nz == nnzC
    ms = (t1 - t0) * 1e3 / steps

    n, nnzA, nnzB = A.nrows, A.nnz, B.nnz
    b_sym = 8 * (n + 1) + 4 * nnzA + 8 * (B.nrows + 1) + 4 * nnzB + 8 * (n + 1)
    b_num = 8 * (n + 1) + (4 + vb) * nnzA + 8 * (B.nrows + 1) + (4 + vb) * nnzB + 8 * (n + 1) + (4 + vb) * nnzC
    b_alg = b_sym + b_num
    phases = {k: float(np.mean([r[k] for r in phase_runs])) for k in phase_runs[0]}
    stats = h.stats()
    # Roofline of the dominant single-kernel phase.  Algorithmic bytes per
    # launch: the output entries that kernel writes ((4 + value bytes) each)
    # plus one read of its inputs: the A rows it handles (col + value), B
    # (col + value; col only in the symbolic pass) and 8 B of row offsets per
    # dense row.
    hm = 4096 if hash_max is None else hash_max
    dense = p > hm
    nd = int(dense.sum())
    a_dense = int(np.diff(A.rowptr)[dense].sum())
    kernels = {
        "sym_dense_bitmap": 4 * a_dense + 4 * nnzB + 8 * nd,
        "num_dense_slab": (4 + vb) * (stats["slab_entries"] + a_dense + nnzB) + 8 * nd,
        "num_dense_tiles": (4 + vb) * (stats["tile_entries"] + a_dense + nnzB) + 8 * nd,
        "num_dense_ranges": (4 + vb) * (stats["range_entries"] + a_dense + nnzB) + 8 * nd,
    }
    dom = max(kernels, key=lambda k: phases.get(k, 0.0))
    kb = kernels[dom]
    achieved = kb / (phases[dom] * 1e-3) / 1e9 if phases[dom] > 0 else 0.0
    roof = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBPS, 4), "traffic": measured_traffic(workload, dom),
            "bytes_per_launch": int(kb), "ms_per_launch": round(phases[dom], 4)}
    res = {"products": P, "nnz_C": int(nnzC), "ms_per_step": round(ms, 4), "value": P / (ms * 1e-3),
           "unit": "semiring products/s",
           "hbm_gbps_model": round(b_alg / (ms * 1e-3) / 1e9, 1),
           "hbm_frac_model": round(b_alg / (ms * 1e-3) / 1e9 / PEAK_HBM_GBPS, 4), "bytes_alg": int(b_alg),
           "phases_ms": {k: round(v, 4) for k, v in phases.items()}, "dense_stats": stats, "roofline": roof}
    return res, C, dA, dB, p


def product_leg(sg, torch, h, name, steps, warmup):
    """Another workload of the configuration list through the same per-call
    two-pass product, with its own roofline and parity sample."""
    A, B, sr_id, desc = make_inputs(name)
    res, C, dA, dB, p = measure_product(sg, torch, h, A, B, sr_id, steps, warmup, workload=name)
    out = {"workload": desc, "semiring": sg.SEMIRING_NAMES[sr_id], "dtype": DTYPE[sr_id]}
    out.update(res)
    out["parity_sample"] = parity_sample(A, B, sr_id, p, C)
    del C, dA, dB
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat20_minplus", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--hash-max", type=int, default=None)
    ap.add_argument("--slab-log", type=int, default=None, help="slab width 2^k columns of the dense path (14..17)")
    ap.add_argument("--light-cap", type=int, default=None, help="most entries of a light slab task")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched legs")
    ap.add_argument("--summa-scale", type=int, default=18, help="R-MAT scale of the 8x8 SUMMA leg (0: skip)")
    ap.add_argument("--summa-waves-scale", type=int, default=22,
                    help="R-MAT scale of the 8x8 SUMMA leg run in memory-budgeted waves (0: skip)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the s18, 3-hop, precision and ER-batch legs")
    ap.add_argument("--er-batch", type=int, default=256, help="ER products in the batch leg (0: skip)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 512 MiB copy kernel (scales rocprofv3 FETCH_SIZE/WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the product is the per-GPU local multiply and this library has no "
              "multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2504_06408_amd as sg

    t_gen = time.perf_counter()
    A, B, sr_id, desc = make_inputs(args.workload)
    print(f"# inputs ready in {time.perf_counter() - t_gen:.1f}s: n={A.nrows} nnz(A)={A.nnz}",
          file=sys.stderr, flush=True)
    h = sg.Handle(0)
    h.set_option("timing", 1)
    if args.hash_max is not None:
        h.set_option("hash_max_products", args.hash_max)
    if args.slab_log is not None:
        h.set_option("slab_log", args.slab_log)
    if args.light_cap is not None:
        h.set_option("light_cap", args.light_cap)
    sr = sg.semiring(sr_id)
    res, C, dA, dB, p = measure_product(sg, torch, h, A, B, sr_id, args.steps, args.warmup, args.hash_max,
                                        args.workload)
    P, ms = res["products"], res["ms_per_step"]
    print(f"# {args.steps} steps: {ms:.3f} ms/step", file=sys.stderr, flush=True)
    out = {
        "metric": METRIC,
        "value": res["value"],
        "unit": "semiring products/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": DTYPE[sr_id],
        "data": "synthetic",
        "config": {"workload": desc, "name": args.workload, "semiring": sg.SEMIRING_NAMES[sr_id], "n": int(A.nrows),
                   "nnz_A": int(A.nnz), "products": P, "nnz_C": res["nnz_C"], "path": "per-call symbolic+numeric"},
    }
    for k in ("hbm_gbps_model", "hbm_frac_model", "bytes_alg", "phases_ms", "dense_stats", "roofline"):
        out[k] = res[k]
    t_par = time.perf_counter()
    out["parity_sample"] = parity_sample(A, B, sr_id, p, C)
    print(f"# parity sample {out['parity_sample']} in {time.perf_counter() - t_par:.1f}s", file=sys.stderr, flush=True)
    del C
    torch.cuda.empty_cache()
    if not args.no_batched:
        out["batched"] = batched_leg(sg, torch, h, sr, dA, dB, P, args.steps, ms)
        print(f"# batched leg {out['batched']['ms_per_step']} ms", file=sys.stderr, flush=True)
        if args.summa_scale > 0:
            out["summa"] = summa_leg(sg, torch, h, args.summa_scale, args.steps)
            print(f"# summa leg {out['summa']['ms_batched']} ms", file=sys.stderr, flush=True)
        if args.summa_waves_scale > 0:
            t_w = time.perf_counter()
            try:
                out["summa_waves"] = summa_waves_leg(sg, torch, h, args.summa_waves_scale)
            except sg.SgError as e:
                out["summa_waves"] = {"error": str(e)}
            torch.cuda.empty_cache()
            print(f"# summa waves leg in {time.perf_counter() - t_w:.1f}s", file=sys.stderr, flush=True)
    if not args.no_extra and args.workload == "rmat20_minplus":
        t_x = time.perf_counter()
        for name in ("rmat18_bool", "rmat18_i64"):
            out[name] = product_leg(sg, torch, h, name, args.steps, args.warmup)
            print(f"# {name} leg {out[name]['ms_per_step']} ms", file=sys.stderr, flush=True)
        out["three_hop"] = three_hop_leg(sg, torch, h, A, dA, args.steps)
        torch.cuda.empty_cache()
        out["precision"] = precision_leg(sg, torch, h, 20)
        torch.cuda.empty_cache()
        if args.er_batch > 0:
            out["er_batch"] = er_batch_leg(sg, torch, h, args.er_batch, args.steps)
            torch.cuda.empty_cache()
        print(f"# extra legs in {time.perf_counter() - t_x:.1f}s", file=sys.stderr, flush=True)
    if args.calibrate_copy:
        n = 1 << 27
        src = torch.ones(n, dtype=torch.int32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.mul(src, 1, out=dst)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = {"read": 4 * n, "write": 4 * n, "kernel": "torch mul int32 (elementwise)"}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A, B, sr_id, p, args.cpu_seconds)
    h.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
