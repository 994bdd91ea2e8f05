/*
 * spgemm.h -- semiring sparse x sparse product C = A (x).(+) B and the
 * semiring merge of partial products on one AMD Instinct MI355X (gfx950).
 *
 * The operation (paper, Section 2.2 "Semiring Abstraction"): for a semiring
 * (S, (+), (x), 0, 1) with commutative, associative (+) and associative (x),
 *     C_ij = (+)_{k : A_ik and B_kj stored} A_ik (x) B_kj .
 * C's pattern is structural: (i, j) is stored iff at least one product
 * reaches it, even when the folded value equals the semiring zero.  This is
 * the local multiply that every stage of the paper's distributed Sparse SUMMA
 * runs (Section 2.1; Section 4.3 "GALATIC SpGEMM"), and the merge is the
 * combination of those stage outputs into one matrix (Section 2.1, last
 * paragraph; Section 4.4 "Merging Operation"), done here on the GPU.
 *
 * Conventions shared by every call
 *  - Matrices are CSR.  rowptr: int64[nrows+1], rowptr[0] = 0; col: int32[nnz];
 *    val: nnz values of the semiring's value type (int64, float, double,
 *    uint8 0/1, float).  All matrix arrays are DEVICE pointers.  Columns in a
 *    row must be strictly ascending (unique, sorted); with the environment
 *    variable SG_VALIDATE=1 every call checks this and returns
 *    SG_ERR_UNSORTED otherwise.  nrows = 0 and nnz = 0 are legal.
 *  - Ownership: the caller allocates and frees every matrix array.  The
 *    library never frees caller memory.  A handle owns its scratch memory
 *    (grown on demand, freed by sg_handle_destroy); a plan owns its pool.
 *  - Streams: `stream` is a hipStream_t (NULL = the null stream).  Work is
 *    queued on it; only the *_symbolic calls and sg_batch_plan wait for it.
 *  - Errors: every call returns an sg_status and never aborts or throws.
 *    sg_last_error() gives a message.  An asynchronous HIP fault surfaces as
 *    SG_ERR_HIP on a later call that waits for the device.  The kernels'
 *    own consistency check (a numeric pass that filled a different number of
 *    entries than its symbolic pass counted, or B with unsorted or
 *    out-of-range columns) sets a device flag that the next *_symbolic call
 *    on the handle, or sg_handle_check, reports as SG_ERR_INVALID (and
 *    clears).  On failure no output array holds a partial result that the
 *    caller may rely on.
 *  - A and B may alias (A.A).  C must not alias A or B.
 *  - One handle serves one host thread at a time.
 */
#ifndef SG_SPGEMM_H
#define SG_SPGEMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SG_OK = 0,
  SG_ERR_INVALID = -1,  /* null pointer, negative size, bad option */
  SG_ERR_SHAPE = -2,    /* A.ncols != B.nrows, or parts of unequal shape */
  SG_ERR_SEMIRING = -3, /* unknown semiring id or accumulation flag */
  SG_ERR_NOMEM = -4,    /* device allocation failed or pool too small */
  SG_ERR_OVERFLOW = -5, /* a size exceeds the index types (ncols > 2^31-1) */
  SG_ERR_UNSORTED = -6, /* validation found an unsorted or duplicate column */
  SG_ERR_HIP = -7       /* a HIP runtime call or a kernel failed */
} sg_status;

/* The five semirings (paper, Section 2.2; Section 5.1 uses (+,x) on floats
 * and (min,+)).
 *  SG_PLUS_TIMES_I64 : int64, (+) and (x) wrap modulo 2^64, 0 = 0, 1 = 1
 *  SG_PLUS_TIMES_F32 : float, IEEE binary32 (x) and (+); see acc_flags
 *  SG_PLUS_TIMES_F64 : double, IEEE binary64
 *  SG_OR_AND_BOOL    : uint8 (nonzero = true), (+) = or, (x) = and; C holds 0/1
 *  SG_MIN_PLUS_F32   : float, (x) = binary32 addition, (+) = minimum,
 *                      0 = +inf, 1 = +0.0.  Inputs must not be NaN and no
 *                      product may be +inf + -inf.                         */
typedef enum {
  SG_PLUS_TIMES_I64 = 1,
  SG_PLUS_TIMES_F32 = 2,
  SG_PLUS_TIMES_F64 = 3,
  SG_OR_AND_BOOL = 4,
  SG_MIN_PLUS_F32 = 5
} sg_semiring_id;

/* Accumulation of SG_PLUS_TIMES_F32 sums (ignored by the other semirings).
 *  SG_ACC_DEFAULT     : compensated (two-sum plus exact product error, kept
 *                       as a float pair per accumulator slot) for hash rows
 *                       (at most hash_max_products products) with more than
 *                       comp_min_terms stored entries in A's row and more
 *                       than comp_min_products products, and for every dense
 *                       row (more than hash_max_products products); plain
 *                       binary32 otherwise.
 *  SG_ACC_COMPENSATED : compensated for every row that is not a small row
 *                       (at most 64 products).
 *  SG_ACC_PLAIN       : plain binary32 everywhere.                          */
enum { SG_ACC_DEFAULT = 0, SG_ACC_COMPENSATED = 1, SG_ACC_PLAIN = 2 };

typedef struct {
  int32_t id;                /* sg_semiring_id */
  int32_t value_bytes;       /* size of one value: 8, 4, 8, 1, 4 */
  uint32_t acc_flags;        /* SG_ACC_* */
  int32_t comp_min_terms;    /* default 64 */
  int64_t comp_min_products; /* default 0 */
} sg_semiring;

/* Semirings defined at run time (paper, Section 2.2: the user redefines the
 * entry type, (+), (x), zero and one).  value_type is one of "float",
 * "double", "int32_t", "uint32_t", "int64_t", "uint64_t"; add and mul are
 * HIP device expressions in the two values a and b (of value_type) that
 * give a (+) b and a (x) b; zero and one are expressions giving the
 * identities of (+) and (x) (zero starts every accumulator, so
 * zero (+) x = x must hold; one is used by sg_power's self loops).  The
 * expressions may call device math functions (fminf, fmax, ...) and use
 * INT32_MAX, INT64_MAX, UINT64_MAX and the like.  (+) must be commutative
 * and associative; any order of folds may occur.  flags: SG_SR_IDEMPOTENT
 * declares a (+) a = a (then repeated folds of one product are allowed and
 * sg_power may stop at a fixed point). */
enum { SG_SR_IDEMPOTENT = 1 };
typedef struct {
  const char* value_type;
  const char* add;
  const char* mul;
  const char* zero;
  const char* one;
  uint32_t flags;
} sg_semiring_def;

typedef struct {
  int64_t nrows, ncols, nnz;
  int64_t* rowptr; /* device, nrows+1 */
  int32_t* col;    /* device, nnz */
  void* val;       /* device, nnz values */
} sg_csr;

typedef struct sg_handle sg_handle;
typedef struct sg_plan sg_plan;

/* Fill *out (host memory) with the descriptor of semiring `id`.
 * Returns SG_ERR_SEMIRING for an unknown id or flag, SG_ERR_INVALID for
 * out == NULL. */
sg_status sg_semiring_make(sg_semiring_id id, uint32_t acc_flags, sg_semiring* out);

/* Define a semiring at run time: the library's numeric kernels (small,
 * hash, column-slab and tile paths) are compiled for it with hipRTC (once
 * per distinct definition in the process, loaded on each device that uses
 * it) and *out receives a descriptor (id >= 64, value_bytes of value_type)
 * for sg_spgemm_numeric, sg_spgemm_numeric_noalloc,
 * sg_spgemm_merge_numeric, the CSC entry points and sg_power_run; batched
 * plans (sg_batch_plan, sg_waves_plan) take the five built-in semirings
 * only.  A definition that does not compile gives SG_ERR_SEMIRING with the
 * compiler's messages in sg_last_error.  Waits for the device. */
sg_status sg_semiring_define(sg_handle* h, const sg_semiring_def* def, sg_semiring* out);

/* Create a handle bound to HIP device `device` (made current by every call
 * that uses the handle).  tuning_json: path to a tuning table written by
 * sg_tune, or NULL for the built-in defaults (the environment variable
 * SG_TUNING names a table when tuning_json is NULL).  *out receives the
 * handle. */
sg_status sg_handle_create(int device, const char* tuning_json, sg_handle** out);
sg_status sg_handle_destroy(sg_handle* h);

/* Set a tuning option by name (host strings): "hash_max_products" (rows with
 * more products take the column-tiled dense path; <= 4096), "force_path"
 * ("auto", "small", "hash", "dense": route every row that the path can take
 * through it), "validate" (0/1), "timing" (0/1: record per-phase HIP events,
 * see sg_handle_timings), "dense_slab" (0/1, default 1: dense rows of a single
 * product run per column slab of B over a slab partition of B; 0: per
 * column tile through a per-B-row tile offset table), "gather32" (0/1,
 * default 1: the slab path's gathers use 32-bit offsets when its partition of
 * B spans less than 4 GiB; 0: always 64-bit), "merge_rows" (0/1, default 1:
 * in the numeric pass a row of 65 to 4096 products over B of more than
 * 65,536 columns, in the symbolic pass such a row of 1025 to 4096, is
 * merged in LDS from its sources' sorted segments; 0: LDS hash tables, and
 * a sort in the numeric pass), "slab_log" (0 = chosen from
 * B's width, or 14..17: the slab path cuts B's columns into slabs of
 * 2^slab_log columns), "light_cap" (0 = the light kernel's LDS capacity, or
 * 1..32768: a dense row's slab with at most this many output entries is a
 * light task, a fuller one a heavy task; set here it applies to every
 * semiring), "dense_tile_min" (1..2048, default 2048; whole-row tile path of
 * batches and dense_slab=0 only: a dense row's column tile with at least
 * this many output entries is accumulated in a dense LDS array, runs of
 * smaller ones (at most four tiles and 2048 entries) on an LDS column bitmap,
 * or for run-time semirings in an LDS hash table).  Returns SG_ERR_INVALID
 * for an unknown
 * name or a bad value. */
sg_status sg_handle_set_option(sg_handle* h, const char* name, const char* value);

/* Pass 1 of C = A (x).(+) B (structure only; independent of the semiring).
 * Writes C_rowptr[0..A.nrows] (device, int64, caller-allocated) and stores
 * nnz(C) in *nnzC (host).  Waits for `stream`.  A.val and B.val are not
 * read.  The row analysis is kept in the handle for the next
 * sg_spgemm_numeric on the same A and B. */
sg_status sg_spgemm_symbolic(sg_handle* h, const sg_csr* A, const sg_csr* B, int64_t* C_rowptr, int64_t* nnzC,
                             void* stream);

/* Pass 2: fills C->col and C->val (device, caller-allocated with nnz(C)
 * entries) given C->rowptr from pass 1 on the same A and B.  Rows of C come
 * out sorted by column.  Does not wait for `stream`.  C->nrows must equal
 * A.nrows, C->ncols B.ncols, C->nnz the value pass 1 returned.  When A and B
 * are the arrays of the handle's last pass 1, their row offsets and column
 * ids must be unchanged since then (values may change): the saved per-row
 * product counts and dense-row tile offsets are reused. */
sg_status sg_spgemm_numeric(sg_handle* h, const sg_semiring* sr, const sg_csr* A, const sg_csr* B, sg_csr* C,
                            void* stream);

/* Variant of sg_spgemm_numeric for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc): same arguments, same result, same stream semantics
 * (no wait for the stream), but it calls no hipMalloc, hipFree or other
 * allocating routine.  Its scratch (row bins, B's column-slab partition, the
 * dense-row tile offsets and task lists) comes from one fixed device array of
 * SG_NOALLOC_SCRATCH_BYTES per GPU, bound when a handle is created on that
 * GPU and held until the process ends.  It never reuses the structure saved
 * by the handle's last symbolic pass (everything is rebuilt from A, B and
 * C->rowptr), so it does not depend on which call came before, but C->rowptr
 * must still come from sg_spgemm_symbolic on the same A and B.  A product
 * whose scratch exceeds the array returns SG_ERR_NOMEM before any kernel
 * writes to C.  Every call on one GPU shares that GPU's array: calls that
 * overlap in time on one GPU (two streams, two host threads) race and must
 * be serialised by the caller; consecutive calls on one stream are safe. */
#define SG_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
sg_status sg_spgemm_numeric_noalloc(sg_handle* h, const sg_semiring* sr, const sg_csr* A, const sg_csr* B, sg_csr* C,
                                    void* stream);

/* Merge (paper, Section 4.4): C = parts[0] (+) ... (+) parts[nparts-1],
 * entry by entry, pattern = union.  parts is a host array of nparts
 * descriptors (device arrays) of one shape.  Same two-pass convention as the
 * product: merge_symbolic writes C_rowptr and *nnzC (host) and waits for the
 * stream; merge_numeric fills C->col, C->val.  1 <= nparts <= 4096. */
sg_status sg_spgemm_merge_symbolic(sg_handle* h, int nparts, const sg_csr* parts, int64_t* C_rowptr,
                                   int64_t* nnzC, void* stream);
sg_status sg_spgemm_merge_numeric(sg_handle* h, const sg_semiring* sr, int nparts, const sg_csr* parts, sg_csr* C,
                                  void* stream);

/* Batched path (the many block products of a 2D Sparse SUMMA, Section 2.1,
 * plus batches of small products): nprob products C_q = A[q] (x).(+) B[q]
 * (host arrays of descriptors) and ngroups merges, group g combining the
 * products group_offsets[g] .. group_offsets[g+1]-1 (host int32 array of
 * ngroups+1 ascending entries; ngroups = 0 means no merges).  The plan sizes
 * and owns a device pool (pool_bytes = 0: sized exactly from a symbolic
 * pass at plan time; otherwise that many bytes) and records one graph of
 * persistent kernels over a global work queue; sg_batch_plan waits for its
 * own work.  sg_batch_execute replays the graph on `stream` with no host
 * round trip; it recomputes every product and merge from the current values
 * (the patterns of A[q], B[q] must not change after planning).
 * sg_batch_results fills out_C (host array) with views into the pool: nprob
 * product results followed by ngroups merge results; they stay valid until
 * the plan is destroyed or executed again.  A pool overflow on execute sets
 * SG_ERR_NOMEM on the next sg_batch_results. */
sg_status sg_batch_plan(sg_handle* h, const sg_semiring* sr, int nprob, const sg_csr* A, const sg_csr* B,
                        int ngroups, const int32_t* group_offsets, size_t pool_bytes, sg_plan** out);
sg_status sg_batch_execute(sg_plan* plan, void* stream);
sg_status sg_batch_results(sg_plan* plan, sg_csr* out_C);
sg_status sg_plan_destroy(sg_plan* plan);

/* Memory-budgeted waves of a batch (Section 2.1, at a scale whose stage
 * outputs exceed the GPU: e.g. the 512 stage products of an 8 x 8 SUMMA grid
 * at R-MAT scale 22 hold ~1.1 TB).  group_offsets (host, ngroups+1, from 0
 * to nprob, ascending) cuts the products into merge groups, as in
 * sg_batch_plan; every product belongs to one group.  sg_waves_plan sizes
 * each product's output with a symbolic pass and cuts the groups, in order,
 * into waves whose output bytes (each group: its products' entries twice --
 * the stage outputs and their merge, which holds at most as many -- times
 * 4 + value_bytes) stay within budget_bytes; a group above the budget gives
 * SG_ERR_NOMEM.  sg_waves_info reports the wave count, each product's nnz
 * (product_nnz: nprob entries), the wave offsets over the groups
 * (wave_groups: nwaves+1 entries) and each wave's output bytes (wave_bytes:
 * nwaves entries); any of them may be NULL.  sg_waves_run makes wave w
 * current -- freeing the previous wave's plan and building this wave's with
 * sg_batch_plan when w is not already current -- and replays its graph on
 * `stream`; sg_waves_results fills out_C with the current wave's results as
 * sg_batch_results does: its products, then its merges.  The operands must
 * stay unchanged and alive until sg_waves_destroy. */
typedef struct sg_waves sg_waves;
sg_status sg_waves_plan(sg_handle* h, const sg_semiring* sr, int nprob, const sg_csr* A, const sg_csr* B,
                        int ngroups, const int32_t* group_offsets, size_t budget_bytes, sg_waves** out);
sg_status sg_waves_info(const sg_waves* w, int* nwaves, int64_t* product_nnz, int32_t* wave_groups,
                        size_t* wave_bytes);
sg_status sg_waves_run(sg_waves* w, int wave, void* stream);
sg_status sg_waves_results(sg_waves* w, sg_csr* out_C);
sg_status sg_waves_destroy(sg_waves* w);

/* Autotuner (paper, Section 4.3: the tunable parameters of the local
 * multiply): times the whole two-pass product C = A (x).(+) B with semiring
 * sr under candidate settings of the knobs the default path reads --
 * "hash_max_products", "slab_log" and "light_cap" (see
 * sg_handle_set_option) -- walking them one at a time from the defaults, and
 * writes the fastest as a tuning table (JSON, host path out_json) keyed by
 * sr's semiring id and value width, with the default and tuned times.  The
 * handle adopts the result.  Waits for its own work; allocates and frees its
 * own output buffers. */
sg_status sg_tune(sg_handle* h, const sg_semiring* sr, const sg_csr* A, const sg_csr* B, const char* out_json);

/* Adopt the tuning table at host path `path` (written by sg_tune).  With
 * sr != NULL a table made for another semiring id or value width is refused
 * with SG_ERR_SEMIRING.  The structural knobs (hash_max_products, slab_log)
 * apply to every product of the handle; the table's light_cap applies only
 * to numeric calls with the table's semiring.  sg_handle_create loads its
 * tuning_json through this call with sr = NULL. */
sg_status sg_tune_load(sg_handle* h, const sg_semiring* sr, const char* path);

/* ---- Column-major operands (paper, Section 4.1 and Algorithm 1) ----------
 * CSC: colptr int64[ncols+1], row int32[nnz] (ascending within a column),
 * val[nnz].  DCSC keeps only the nzc non-empty columns: jc int32[nzc]
 * (their ids, ascending), cp int64[nzc+1] (cp[i] = first entry of column
 * jc[i], cp[nzc] = nnz), row and val as in CSC.  All arrays are device
 * pointers owned by the caller. */
typedef struct {
  int64_t nrows, ncols, nnz;
  int64_t* colptr; /* device, ncols+1 */
  int32_t* row;    /* device, nnz */
  void* val;       /* device, nnz values */
} sg_csc;

typedef struct {
  int64_t nrows, ncols, nzc, nnz;
  int32_t* jc;  /* device, nzc */
  int64_t* cp;  /* device, nzc+1 */
  int32_t* row; /* device, nnz */
  void* val;    /* device, nnz values */
} sg_dcsc;

/* Decompress DCSC column pointers (Algorithm 1): colptr[j] (device,
 * caller-allocated, ncols+1) = the entries of the columns before j, so every
 * column the compressed list skips gets an empty segment.  The row and
 * value arrays need no change: with colptr they form A in CSC.  Does not
 * wait for the stream. */
sg_status sg_dcsc_decompress(sg_handle* h, const sg_dcsc* A, int64_t* colptr, void* stream);

/* Compress CSC column pointers colptr[0..ncols] (device) to DCSC: jc (device,
 * capacity ncols) and cp (device, capacity ncols+1) receive the non-empty
 * columns and their offsets, *nzc (host) their count.  Waits for the
 * stream. */
sg_status sg_dcsc_compress(sg_handle* h, int64_t ncols, const int64_t* colptr, int32_t* jc, int64_t* cp,
                           int64_t* nzc, void* stream);

/* C = A (x).(+) B for CSC operands, C in CSC (Section 4.1: the CSC arrays of
 * a matrix are the CSR arrays of its transpose and AB = (B^T A^T)^T, so the
 * product runs as the CSR product of the swapped operands with no copy or
 * transposition).  Each product is formed as b_kj (x) a_ik, which equals
 * a_ik (x) b_kj for the five semirings (all have commutative (x)).  Same
 * two-pass convention as sg_spgemm_symbolic/numeric, with column pointers in
 * place of row pointers. */
sg_status sg_spgemm_csc_symbolic(sg_handle* h, const sg_csc* A, const sg_csc* B, int64_t* C_colptr, int64_t* nnzC,
                                 void* stream);
sg_status sg_spgemm_csc_numeric(sg_handle* h, const sg_semiring* sr, const sg_csc* A, const sg_csc* B, sg_csc* C,
                                void* stream);

/* ---- Powers of a square matrix (paper, Section 2.2) ------------------------
 * Over (min,+) the k-th power of a weighted adjacency matrix W holds the
 * lightest walks of exactly k edges; with the semiring one on the diagonal
 * (W' = I (+) W, flag SG_POWER_SELF_LOOPS) the shortest paths of at most k
 * edges, which stop changing at the distance matrix.  Over (or,and) the
 * powers of I (+) W give reachability, over (+,x) walk counts.
 * sg_power_run computes D_1 = W' and then D_{h+1} = D_h W' (linear steps)
 * or D_{2h} = D_h D_h (SG_POWER_SQUARING) with the product entry points,
 * until h >= max_hops (max_hops <= 0: twice the matrix size), or, with
 * SG_POWER_FIXPOINT (needs SG_POWER_SELF_LOOPS and (min,+) or (or,and)),
 * until a product equals its left operand in pattern and value bits.  The
 * result lives in memory the power object owns (until sg_power_destroy);
 * sg_power_result gives a descriptor of it, the exponent h it holds, the
 * number of products run and whether the fixed point was reached.  Waits
 * for the stream. */
enum { SG_POWER_SELF_LOOPS = 1, SG_POWER_SQUARING = 2, SG_POWER_FIXPOINT = 4 };
typedef struct sg_power sg_power;
sg_status sg_power_run(sg_handle* h, const sg_semiring* sr, const sg_csr* W, int32_t max_hops, uint32_t flags,
                       void* stream, sg_power** out);
sg_status sg_power_result(const sg_power* p, sg_csr* D, int32_t* hops, int32_t* products, int32_t* converged);
sg_status sg_power_destroy(sg_power* p);

/* Phases timed when the handle option "timing" is "1" (a pair of HIP events
 * is recorded on the call's stream around each phase).  Phases 10..13 are
 * single kernels nested inside phases 4 and 9. */
enum {
  SG_PHASE_SYM_ANALYZE = 0, /* row analysis + binning of the symbolic pass */
  SG_PHASE_SYM_BOUNDS = 1,  /* per-B-row column-tile offsets and the column-slab partition of B */
  SG_PHASE_SYM_SMALL = 2,   /* wavefront rows */
  SG_PHASE_SYM_HASH = 3,    /* LDS hash rows */
  SG_PHASE_SYM_DENSE = 4,   /* bitmap rows: bitmap kernel + per-row tile offsets */
  SG_PHASE_SYM_SCAN = 5,    /* prefix sum into C.rowptr */
  SG_PHASE_NUM_ANALYZE = 6, /* row binning of the numeric pass (+ value partition of B) */
  SG_PHASE_NUM_SMALL = 7,
  SG_PHASE_NUM_HASH = 8,
  SG_PHASE_NUM_DENSE = 9,         /* dense rows: task building + the three task kernels */
  SG_PHASE_SYM_DENSE_BITMAP = 10, /* the dense-row bitmap kernel alone */
  SG_PHASE_NUM_DENSE_SLAB = 11,   /* slab tasks (bitmap + rank accumulator) */
  SG_PHASE_NUM_DENSE_TILES = 12,  /* dense-tile tasks */
  SG_PHASE_NUM_DENSE_RANGES = 13, /* range tasks (hash + sort) */
  SG_NPHASES = 14
};

/* Device milliseconds of each phase of the most recent symbolic and numeric
 * calls (product or merge) on this handle: ms[0..n) receives
 * min(n, SG_NPHASES) values; a phase that did not run reports 0.  Waits for
 * the recorded events.  Requires the "timing" option. */
sg_status sg_handle_timings(sg_handle* h, double* ms, int n);

/* Dense-row work of the most recent numeric call on this handle (waits for
 * the device): out[0..n) receives min(n, SG_NSTATS) values, in this order:
 * dense rows, slab tasks, dense-tile tasks, range tasks, and the output
 * entries written by each of the three task kinds (slab, tile, range). */
enum { SG_NSTATS = 7 };
sg_status sg_handle_stats(sg_handle* h, int64_t* out, int n);

/* Wait for all work of the handle's device, then report any device-side
 * consistency error (a numeric pass that filled a different number of
 * entries than its symbolic pass counted) as SG_ERR_INVALID. */
sg_status sg_handle_check(sg_handle* h);

const char* sg_status_string(sg_status s);
const char* sg_last_error(const sg_handle* h);

#ifdef __cplusplus
}
#endif

#endif /* SG_SPGEMM_H */
