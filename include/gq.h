/*
 * gq.h -- C-ABI of libgq.so: columnar query operators on AMD Instinct MI355X
 * (gfx950): filter, hash partition, hash-join build and probe, hash group-by
 * over int64 fixed-point decimals, and a fused filter -> probe -> group-by
 * pipeline.
 *
 * Operator model (paper "Accelerating Presto with GPUs"):
 *  - Operators consume and produce batches of rows held column-wise in device
 *    memory in an Arrow-compatible layout (Section 3.1 describes a RowVector as
 *    a batch of typically thousands of rows; Section 3.2 the cuDF table it wraps
 *    on the GPU).
 *  - Each batch travels with a stream; an operator enqueues its work on that
 *    stream and returns at once without blocking the calling thread, and
 *    streams are synchronised only at pipeline boundaries such as join build ->
 *    probe (Section 3, "asynchronous execution model" and "cross-pipeline
 *    synchronization"; Section 3.2).
 *  - Expressions are evaluated fused into one pass where possible (Section 3.2,
 *    AST execution versus standalone functions): here predicates and aggregate
 *    input products are fused into the scanning kernel.
 *  - Hash aggregation is a batch operator (Section 3.2, HashAggregation).
 *  - The partitioned output operator splits a batch into per-destination
 *    packed contiguous buffers (Section 3.3): gq_hash_partition writes every
 *    partition contiguously plus an offsets array.
 *
 * Conventions shared by every call:
 *  - All data pointers in gq_column / gq_batch are DEVICE pointers.  Arrays of
 *    descriptors (gq_batch, gq_column, gq_pred, gq_agg, key and projection
 *    lists, gq_plan) are HOST memory read during the call only.
 *  - Inputs are borrowed: they must stay valid until the stream has passed the
 *    call.  Outputs are caller-allocated at the caller's capacity.
 *  - Every compute call enqueues on `stream` and returns without waiting.
 *    Errors detectable on the host are returned at once (negative gq_status)
 *    and nothing is enqueued.  Conditions found on the device (output capacity
 *    exceeded, hash table full) are OR-ed into the context's device status word
 *    and read with gq_ctx_sync_status; the required size is still written to
 *    the call's device count so the caller can retry.  No kernel ever writes
 *    past a caller's capacity.
 *  - Calls never call hipMemset*, never synchronise, and allocate only through
 *    the context allocator (stream ordered), so they can be captured in a HIP
 *    graph.
 *  - Row indices are int32: a batch holds at most 2^31-1 rows.
 *  - A context is used by one host thread at a time.  Different contexts may be
 *    used concurrently, on different streams.
 *  - No C++ exception crosses this interface.
 */
#ifndef GQ_H
#define GQ_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
typedef enum gq_status {
  GQ_OK = 0,
  GQ_ERR_INVALID = -1,     /* bad descriptor, type mismatch, size out of range */
  GQ_ERR_UNSUPPORTED = -2, /* valid request outside what the library implements */
  GQ_ERR_NOMEM = -3,       /* the allocator returned NULL */
  GQ_ERR_HIP = -4,         /* a HIP runtime call failed; text in gq_last_error */
  GQ_ERR_CAPACITY = -5,    /* device: output capacity too small (count = required) */
  GQ_ERR_TABLE_FULL = -6   /* device: hash table could not hold every key */
} gq_status;

/* Device status word bits (see gq_ctx_sync_status). */
#define GQ_DEV_CAPACITY 1
#define GQ_DEV_TABLE_FULL 2

/* ---- columns and batches -------------------------------------------------- */
typedef enum gq_type { GQ_I8 = 1, GQ_I16 = 2, GQ_I32 = 3, GQ_I64 = 4 } gq_type;

/*
 * One fixed-width signed integer column, Arrow layout.
 *  type      GQ_I8 .. GQ_I64, little-endian values.
 *  scale     fixed-point decimal digits (metadata only; 0 = plain integer).
 *  length    rows (input) or capacity in rows (output).
 *  offset    first row: row i lives at data + (offset + i) * width and at bit
 *            (offset + i) of the validity bitmap (Arrow slice offset).
 *  data      device pointer.
 *  validity  device pointer to an LSB-first bitmap, bit = 1 means valid, or
 *            NULL = all rows valid.  Output bitmaps must be 4-byte aligned and
 *            are written for exactly the output rows (other bits untouched).
 */
typedef struct gq_column {
  int32_t type;
  int32_t scale;
  int64_t length;
  int64_t offset;
  void* data;
  uint8_t* validity;
} gq_column;

/* A batch: `ncols` columns of `nrows` rows each. */
typedef struct gq_batch {
  int64_t nrows;
  int32_t ncols;
  int32_t reserved;
  gq_column* cols;
} gq_batch;

/* ---- predicates and aggregate expressions --------------------------------- */
typedef enum gq_pred_op {
  GQ_RANGE = 1, /* lo <= x <= hi, compared as int64 after sign extension */
  GQ_NE = 2     /* x != lo */
} gq_pred_op;

/* An array of predicates is a conjunction; a NULL value never passes (SQL
 * three-valued logic drops UNKNOWN rows).  An empty array keeps every row. */
typedef struct gq_pred {
  int32_t col;
  int32_t op;
  int64_t lo;
  int64_t hi;
} gq_pred;

typedef enum gq_factor_kind {
  GQ_F_COL = 1,         /* x          */
  GQ_F_K_MINUS_COL = 2, /* k - x      */
  GQ_F_K_PLUS_COL = 3,  /* k + x      */
  GQ_F_CONST = 4        /* k          */
} gq_factor_kind;

typedef struct gq_factor {
  int32_t kind;
  int32_t col;
  int64_t k;
} gq_factor;

typedef enum gq_agg_op {
  GQ_SUM = 1,        /* wrapping int64 sum of non-NULL inputs; NULL if none  */
  GQ_COUNT_STAR = 2, /* rows in the group                                    */
  GQ_COUNT = 3,      /* non-NULL inputs                                      */
  GQ_MIN = 4,        /* NULL if no non-NULL input                            */
  GQ_MAX = 5
} gq_agg_op;

/* Aggregate over an input expression: the product of `nfactors` (0..3)
 * factors in wrapping int64 arithmetic, NULL if any referenced column is NULL.
 * Fixed-point scale of a product is the sum of its factors' scales. */
typedef struct gq_agg {
  int32_t op;
  int32_t nfactors;
  gq_factor f[3];
} gq_agg;

#define GQ_MAX_COLS 16
#define GQ_MAX_PREDS 8
#define GQ_MAX_AGGS 8
#define GQ_MAX_KEYS 4

/* ---- context --------------------------------------------------------------- */
typedef struct gq_ctx gq_ctx;

/* Stream-ordered allocator.  alloc returns device memory usable by work
 * enqueued on `stream` after the call, or NULL.  free releases it once work
 * enqueued on `stream` before the call has finished. */
typedef struct gq_allocator {
  void* (*alloc)(size_t bytes, hipStream_t stream, void* user);
  void (*free)(void* ptr, size_t bytes, hipStream_t stream, void* user);
  void* user;
} gq_allocator;

/* Create a context on `device`.  `alloc` may be NULL: hipMallocAsync /
 * hipFreeAsync on the device's default memory pool.  The allocator struct is
 * copied.  Returns GQ_ERR_INVALID for a bad device, GQ_ERR_HIP on a runtime
 * failure, GQ_ERR_NOMEM if the status word cannot be allocated. */
int gq_ctx_create(int device, const gq_allocator* alloc, gq_ctx** out);
/* Destroy a context; waits for the device first.  NULL is a no-op. */
int gq_ctx_destroy(gq_ctx* ctx);
/* Text of the last host-side error on this context ("" if none).  The pointer
 * stays valid until the next call on the context. */
const char* gq_last_error(gq_ctx* ctx);
/* Synchronise `stream`, read and clear the device status word.  Writes the raw
 * GQ_DEV_* bits to *bits (if not NULL) and returns GQ_OK, GQ_ERR_CAPACITY or
 * GQ_ERR_TABLE_FULL (capacity first if both). */
int gq_ctx_sync_status(gq_ctx* ctx, hipStream_t stream, int32_t* bits);
/* Device address of the context's status word (int32), for callers that read
 * it themselves without a synchronisation. */
int32_t* gq_ctx_status_ptr(gq_ctx* ctx);

/* Per-kernel timing, a profiling aid.  While enabled, every kernel the context
 * launches is bracketed by two HIP events recorded on the kernel's own stream.
 * Not for use under HIP graph capture. */
int gq_ctx_set_timing(gq_ctx* ctx, int enable);
/* Restrict that timing to the launches named `name` (the names the report
 * lists), so that a timed region carries events around one kernel only; NULL
 * or "" times every launch again.  The name is copied.  Returns GQ_OK, or
 * GQ_ERR_INVALID for a NULL context. */
int gq_ctx_set_timing_only(gq_ctx* ctx, const char* name);
/* Wait for the recorded events, then report the totals per kernel name since
 * the last report, largest first: up to `cap` entries of `names` (each
 * name_len bytes, NUL-terminated), total_ms and launches.  Returns the number
 * of distinct kernels (may exceed cap) or a negative gq_status.  Clears the
 * records. */
int gq_ctx_timing_report(gq_ctx* ctx, char* names, int name_len, double* total_ms, int64_t* launches,
                         int cap);

/* ---- filter -----------------------------------------------------------------
 * Stable stream compaction (Section 3.2, filter and projection on the GPU):
 * rows of `in` for which every predicate holds, in input order, projected to
 * the input columns listed in `proj` (nproj entries, 0..GQ_MAX_COLS).
 *  out     nproj columns; out->cols[j] must have the type of in->cols[proj[j]];
 *          its `length` is the capacity in rows.  If the input column has a
 *          validity bitmap the output column must have one too.
 *  d_count device int64: number of kept rows (written even when it exceeds the
 *          capacity, in which case GQ_DEV_CAPACITY is raised and rows beyond
 *          the capacity are not written).
 * Errors: GQ_ERR_INVALID (bad column index, type mismatch, too many columns or
 * predicates, more than 2^31-1 rows). */
int gq_filter(gq_ctx* ctx, const gq_batch* in, const gq_pred* preds, int npreds,
              const int32_t* proj, int nproj, gq_batch* out, int64_t* d_count,
              hipStream_t stream);

/* gq_filter for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and results, with the workspace (a ticket word and one status
 * word per 4,096-row tile) taken from a fixed 512 KiB array that the library
 * holds on each device for the life of the process, instead of the context
 * allocator.  No allocation of any kind happens in the call.  Inputs of more
 * than 268,435,456 rows (65,536 tiles) give GQ_ERR_INVALID.  Every call on a
 * device shares that device's array (the call clears it first): calls that
 * may overlap on one device, on any streams or contexts, race and must be
 * ordered by the caller. */
int gq_filter_noalloc(gq_ctx* ctx, const gq_batch* in, const gq_pred* preds, int npreds,
                      const int32_t* proj, int nproj, gq_batch* out, int64_t* d_count,
                      hipStream_t stream);

/* ---- hash partition -----------------------------------------------------------
 * Split `in` into `nparts` partitions by a hash of its key columns (the
 * partitioned-output operator of Section 3.3; the packed per-destination
 * layout of the same section).
 *  hash       h = seed; for each key column in order h = fmix64(h ^ x) with x
 *             the value sign-extended to 64 bits, 0 for NULL; fmix64 is the
 *             MurmurHash3 64-bit finaliser.
 *  partition  p = floor(h * nparts / 2^64).
 *  out        same column count and types as `in`, capacity >= in->nrows; rows
 *             grouped by ascending p and in input order within a partition.
 *  d_offsets  device int64[nparts + 1]: partition q occupies rows
 *             [d_offsets[q], d_offsets[q+1]); d_offsets[0] = 0.
 * 1 <= nparts <= 1024.  Errors: GQ_ERR_INVALID. */
int gq_hash_partition(gq_ctx* ctx, const gq_batch* in, const int32_t* keys, int nkeys,
                      int32_t nparts, uint64_t seed, gq_batch* out, int64_t* d_offsets,
                      hipStream_t stream);

/* ---- hash join ----------------------------------------------------------------
 * Inner equi-join on one integer key column (Section 3.1 names Join among the
 * relational operators run on the GPU; the build -> probe hand-over is the
 * pipeline boundary of Section 3).  NULL keys never match.  Duplicate build
 * keys are allowed. */
typedef struct gq_join_table gq_join_table;

typedef struct gq_join_opts {
  float load_factor; /* target keys / slots, (0, 0.9]; 0 = 0.5 */
  int32_t acc_slots; /* 8-byte accumulator words reserved per slot for a fused
                        group-by on the join key (0, 2 or 6); see gq_pipeline */
  int32_t regions_log2; /* build inputs of at least 2^20 rows are partitioned into
                           2^regions_log2 key-hash regions for the radix group-join
                           of gq_pipeline: 0 = chosen from the row count, else 4..12 */
} gq_join_opts;

/* Build a table over the rows of `build` that pass `preds` and have a non-NULL
 * key.  The table (library-owned, allocated through the context allocator)
 * records an event on `stream` after its build work; every call that reads it
 * (gq_join_probe, gq_pipeline / gq_groupby_agg with a join,
 * gq_join_table_free) makes its own stream wait for that event, and
 * gq_pipeline's radix group-join waits only after partitioning its probe side.
 * So a build enqueued on one stream overlaps the probe side of a pipeline
 * enqueued on another (the build -> probe hand-over of Section 3 is the only
 * synchronisation); the build input must stay unchanged until the build's work
 * has run.  Its capacity is sized on the device from the number of passing
 * rows.  A table over at least 2^20 build rows is stored partitioned; the
 * first call that needs its probe index (gq_join_probe, or a pipeline that
 * does not take the radix group-join) builds the index on its own stream and
 * re-records the table's event there, so every later reader, on any stream,
 * is ordered after the index build too.
 * Keys: 1 to GQ_MAX_KEYS integer columns.  With more than one, their values
 * are packed into one 64-bit word per row (first column most significant,
 * each field as wide as its build column's type), which must fit: more than
 * 64 bits of key types gives GQ_ERR_UNSUPPORTED.  Rows with a NULL in any key
 * column are not inserted.  Such a table serves gq_join_probe and
 * gq_join_groupby; gq_pipeline and gq_pipeline_shared group by their one
 * probe key and take single-key tables only (GQ_ERR_UNSUPPORTED otherwise). */
int gq_join_build(gq_ctx* ctx, const gq_batch* build, const int32_t* keys, int nkeys,
                  const gq_pred* preds, int npreds, const gq_join_opts* opts,
                  hipStream_t stream, gq_join_table** out);

/* Probe: for each row of `probe` that passes `preds` and has a non-NULL key,
 * emit one (probe row, build row) pair per matching build row.  Pairs are
 * ordered by probe row, then build row, ascending (a canonical order of the
 * SQL result).  `probe_idx`/`build_idx` are device int32[out_cap]; *d_count
 * receives the number of pairs (GQ_DEV_CAPACITY if above out_cap).  `nkeys`
 * must equal the build's (GQ_ERR_INVALID otherwise); the probe's key columns
 * may be of other integer types, and a row whose value in a key column lies
 * outside the range of the build column's type, or is NULL, matches nothing. */
int gq_join_probe(gq_ctx* ctx, const gq_join_table* table, const gq_batch* probe,
                  const int32_t* keys, int nkeys, const gq_pred* preds, int npreds,
                  int32_t* probe_idx, int32_t* build_idx, int64_t out_cap, int64_t* d_count,
                  hipStream_t stream);

/* Number of build rows inserted (device int64 inside the table), for callers
 * that size outputs; valid once the build has run. */
const int64_t* gq_join_table_count_ptr(const gq_join_table* table);

/* Stream-ordered release of a table. */
int gq_join_table_free(gq_ctx* ctx, gq_join_table* table, hipStream_t stream);

/* Gather: out column j row r = in column cols[j] row idx[r] (with validity),
 * for r < n.  idx is device int32[n]; each output needs capacity >= n.  Used
 * after a probe to materialise payload columns (late materialisation,
 * Section 2.3). */
int gq_gather(gq_ctx* ctx, const gq_batch* in, const int32_t* cols, int ncols,
              const int32_t* idx, int64_t n, gq_batch* out, hipStream_t stream);

/* ---- hash group-by ------------------------------------------------------------
 * SQL GROUP BY over the rows that pass `preds` (by default the Single
 * aggregation mode of Section 3.2; see gq_agg_mode).  Up to GQ_MAX_KEYS key columns whose combined width plus one
 * NULL flag bit per nullable column fits 64 bits, or one int64 key column of
 * any nullability.  NULL keys form one group.  nkeys = 0 gives one global row,
 * also for an empty input (COUNT = 0, SUM NULL).
 *  out       nkeys key columns (the key types) followed by naggs int64 columns;
 *            capacity in each `length`; key and aggregate validity written when
 *            the output column has a bitmap (required where NULL can occur).
 *  d_groups  device int64: groups found (GQ_DEV_CAPACITY if above capacity).
 * Output order is the hash table's slot order unless flags has GQ_SORTED, in
 * which case groups come in ascending key order, NULL first. */
#define GQ_SORTED 1

typedef enum gq_strategy {
  GQ_STRATEGY_AUTO = 0,
  GQ_STRATEGY_LDS = 1,   /* block-private tables in LDS, merged into HBM */
  GQ_STRATEGY_GLOBAL = 2 /* one table in HBM, device-scope atomics */
} gq_strategy;

/* Aggregation modes (Section 3.2: the aggregation operator runs Single,
 * Partial, Intermediate or Final, so that one aggregation can be split across
 * batches and exchange stages).  A partial state of SUM, COUNT(*), COUNT, MIN
 * and MAX is one int64 value with validity, the aggregate of the rows seen so
 * far (SUM, MIN, MAX NULL when no non-NULL input was seen), so:
 *  SINGLE, PARTIAL      raw rows in, predicates apply; out: values (= states)
 *  INTERMEDIATE, FINAL  state rows in (key columns, then one state column per
 *                       aggregate): aggs[i] names aggregate i's state column
 *                       with one GQ_F_COL factor and keeps its original op;
 *                       SUM, COUNT(*) and COUNT states are merged by SUM, MIN
 *                       and MAX by MIN and MAX.  No predicates.
 * For these aggregates Partial equals Single and Intermediate equals Final;
 * they differ in the streaming object below, where Partial and Intermediate
 * may emit before the input ends. */
typedef enum gq_agg_mode {
  GQ_MODE_SINGLE = 0,
  GQ_MODE_PARTIAL = 1,
  GQ_MODE_INTERMEDIATE = 2,
  GQ_MODE_FINAL = 3
} gq_agg_mode;

typedef struct gq_groupby_opts {
  float load_factor;       /* 0 = 0.5 */
  int32_t strategy;        /* gq_strategy */
  int32_t flags;           /* GQ_SORTED */
  int32_t block_size;      /* 0 = library choice; else 256 or 512 */
  int64_t expected_groups; /* sizing hint; 0 = number of input rows.  Fewer
                              slots than groups raises GQ_DEV_TABLE_FULL. */
  int32_t mode;            /* gq_agg_mode; 0 = GQ_MODE_SINGLE */
  int32_t reserved;
} gq_groupby_opts;

int gq_groupby_agg(gq_ctx* ctx, const gq_batch* in, const int32_t* keys, int nkeys,
                   const gq_pred* preds, int npreds, const gq_agg* aggs, int naggs,
                   const gq_groupby_opts* opts, gq_batch* out, int64_t* d_groups,
                   hipStream_t stream);

/* Late materialisation (Section 2.3): group-by over the inner join of the rows
 * of `probe` passing probe_preds with the table's build rows, computed as the
 * paper's late-materialising join does it: the join on the key columns alone
 * gives (probe row, build row) gather maps, the columns the group-by needs are
 * gathered through them from either side, then grouped.  Column c of the
 * joined rows is probe column c for c < probe->ncols, else column
 * c - probe->ncols of `build`, the batch the table was built from (it must
 * still be valid).  group_keys and aggregate factor columns index joined
 * columns.  pair_capacity bounds the joined rows (0 = probe->nrows, enough
 * when the build keys are unique); more raise GQ_DEV_CAPACITY and only the
 * first pair_capacity are grouped.  Output as for gq_groupby_agg; opts.mode
 * must be single or partial.  At most 16 joined columns. */
int gq_join_groupby(gq_ctx* ctx, const gq_join_table* table, const gq_batch* build, const gq_batch* probe,
                    const int32_t* probe_keys, int nprobe_keys, const gq_pred* probe_preds, int nprobe_preds,
                    const int32_t* group_keys, int ngroup_keys, const gq_agg* aggs, int naggs,
                    const gq_groupby_opts* opts, int64_t pair_capacity, gq_batch* out, int64_t* d_groups,
                    hipStream_t stream);

/* ---- expression programs ------------------------------------------------------
 * An integer expression over the columns of a batch, evaluated for every row
 * by one kernel for the whole expression (Section 3.2: fused expression
 * evaluation, as cuDF's AST compute_column, rather than one kernel per
 * operation).  A program is a list of instructions in postfix order;
 * instruction i produces value i from earlier values (operand indices a, b, c
 * below i); the program's result is its last value.  Arithmetic wraps modulo
 * 2^64.  A NULL operand makes ADD, SUB, MUL, NEG and the comparisons NULL;
 * CASE takes value b where value a is non-NULL and non-zero, else value c
 * (SQL CASE WHEN ... THEN ... ELSE ... END). */
typedef enum gq_expr_op {
  GQ_E_COL = 1,   /* column a, sign-extended to int64, NULL where its bitmap says so */
  GQ_E_CONST = 2, /* the constant k */
  GQ_E_ADD = 3,   /* a + b */
  GQ_E_SUB = 4,   /* a - b */
  GQ_E_MUL = 5,   /* a * b */
  GQ_E_NEG = 6,   /* -a */
  GQ_E_LT = 7,    /* a < b: 1 or 0 */
  GQ_E_LE = 8,
  GQ_E_EQ = 9,
  GQ_E_NE = 10,
  GQ_E_GT = 11,
  GQ_E_GE = 12,
  GQ_E_CASE = 13  /* a (non-NULL, non-zero) ? b : c */
} gq_expr_op;

typedef struct gq_expr_instr {
  int32_t op;
  int32_t a;
  int32_t b;
  int32_t c;
  int64_t k;
} gq_expr_instr;

#define GQ_MAX_EXPR 32  /* instructions per program */

typedef struct gq_expr {
  int32_t ninstr;
  int32_t reserved;
  const gq_expr_instr* instr;  /* host array, read during the call */
} gq_expr;

/* out: int64 column of capacity >= in->nrows; its validity bitmap, when
 * present, receives the result's NULLs. */
int gq_compute_column(gq_ctx* ctx, const gq_batch* in, const gq_expr* expr, gq_column* out, hipStream_t stream);

/* gq_filter whose conjunction also holds every expression in `exprs` (a row
 * passes an expression that is non-NULL and non-zero). */
int gq_filter_expr(gq_ctx* ctx, const gq_batch* in, const gq_pred* preds, int npreds, const gq_expr* exprs,
                   int nexprs, const int32_t* proj, int nproj, gq_batch* out, int64_t* d_count, hipStream_t stream);

/* gq_groupby_agg over the rows passing preds and every expression in `exprs`,
 * where aggregate i is agg_ops[i] (SUM, COUNT(*), COUNT, MIN, MAX) over the
 * expression agg_exprs[i] (ignored for COUNT(*)). */
int gq_groupby_expr(gq_ctx* ctx, const gq_batch* in, const int32_t* keys, int nkeys, const gq_pred* preds,
                    int npreds, const gq_expr* exprs, int nexprs, const int32_t* agg_ops, const gq_expr* agg_exprs,
                    int naggs, const gq_groupby_opts* opts, gq_batch* out, int64_t* d_groups, hipStream_t stream);

/* ---- ORDER BY / top-k -------------------------------------------------------------
 * Row ids of `in` in ORDER BY order (Section 3.1 lists OrderBy among the
 * operators moved to the GPU): keys compared in turn, each ascending unless
 * desc[j] != 0, NULLs first where nulls_first[j] != 0 else last; ties keep
 * input order (stable).  With limit >= 0 only the first min(limit, nrows) ids
 * are written (top-k).  out_rows: device int32[min(limit, nrows)] (all rows
 * when limit < 0).  desc and nulls_first may be NULL (all 0). */
int gq_order_by(gq_ctx* ctx, const gq_batch* in, const int32_t* keys, int nkeys, const int32_t* desc,
                const int32_t* nulls_first, int64_t limit, int32_t* out_rows, hipStream_t stream);

/* ---- streaming aggregation ------------------------------------------------------
 * One aggregation over a sequence of batches (Section 3.2: a streaming
 * group-by that holds its result across input batches and, in the Partial and
 * Intermediate modes, emits it once it reaches a size threshold).  The paper's
 * operator concatenates each batch's result with the held one and aggregates
 * the concatenation again; here the held groups stay in one HBM hash table
 * that every batch is aggregated into directly, which gives the same result
 * without re-reading the held groups per batch.
 *  push    aggregate the batch's rows (Single, Partial: raw rows passing
 *          preds; Intermediate, Final: state rows, no preds) into the held
 *          groups.  In the Partial and Intermediate modes with emit_groups > 0,
 *          once the held groups number at least emit_groups they are written
 *          to `out` and the stream starts over; *d_emitted (device int64)
 *          receives the number of groups written (0: nothing emitted).
 *  finish  write the held groups to `out` and start over.  d_groups is device
 *          int64[2]: [0] groups written, [1] 1 if a result was emitted, 0 if no
 *          batch was pushed since the last emission (then nothing is written).
 * Outputs as for gq_groupby_agg (slot order), capacity >= max_groups (one row
 * for nkeys = 0).  Every batch has the same key column types and the
 * aggregates read the same columns (by index) of every batch.  Decisions are
 * taken on the device: no call blocks.  Groups beyond the table raise
 * GQ_DEV_TABLE_FULL. */
typedef struct gq_agg_stream gq_agg_stream;

typedef struct gq_agg_stream_spec {
  int32_t mode;               /* gq_agg_mode */
  int32_t nkeys;              /* key columns (0: one global group) */
  const int32_t* keys;        /* key column indices of every batch */
  const int32_t* key_nullable;/* nkeys flags: key j may be NULL in some batch
                                 (a key column with a bitmap must be flagged) */
  const gq_agg* aggs;         /* as for gq_groupby_agg in this mode */
  int32_t naggs;
  int32_t reserved;
  int64_t max_groups;         /* most groups the stream holds at once; sizes the table */
  int64_t emit_groups;        /* Partial / Intermediate: emit once this many groups are held; 0 = never early */
  float load_factor;          /* 0 = 0.5 */
  int32_t reserved2;
} gq_agg_stream_spec;

int gq_agg_stream_create(gq_ctx* ctx, const gq_agg_stream_spec* spec, hipStream_t stream, gq_agg_stream** out);
int gq_agg_stream_push(gq_agg_stream* s, const gq_batch* in, const gq_pred* preds, int npreds, gq_batch* out,
                       int64_t* d_emitted, hipStream_t stream);
int gq_agg_stream_finish(gq_agg_stream* s, gq_batch* out, int64_t* d_groups, hipStream_t stream);
/* Stream-ordered release. */
int gq_agg_stream_free(gq_agg_stream* s, hipStream_t stream);

/* ---- shared scan ------------------------------------------------------------------
 * Up to GQ_MAX_SHARED filter + group-by queries over the same batch in one
 * pass: every column is read once and each query aggregates its own kept rows
 * into its own table.  The queries share key columns, aggregates and predicate
 * columns and ops; only predicate bounds differ.  (Serving many queries
 * against resident tables, Section 2 and Section 3.3.)
 *  preds     nqueries * npreds predicates: query q's conjunction is
 *            preds[q*npreds .. q*npreds + npreds)
 *  outs      nqueries output batches, each as for gq_groupby_agg
 *  d_groups  device int64[nqueries]
 * Results equal one gq_groupby_agg call per query. */
#define GQ_MAX_SHARED 8

int gq_groupby_shared(gq_ctx* ctx, const gq_batch* in, const int32_t* keys, int nkeys, const gq_pred* preds,
                      int npreds, int nqueries, const gq_agg* aggs, int naggs, const gq_groupby_opts* opts,
                      gq_batch* outs, int64_t* d_groups, hipStream_t stream);

/* ---- fused pipeline -------------------------------------------------------------
 * filter(in) [-> probe `join` on probe_key] -> group-by, in one pass over `in`
 * with nothing materialised between the steps (the fused per-batch operator
 * chain of Section 3.2).  Group keys and aggregate inputs are columns of `in`.
 * With a join, a probe row matching m build rows counts m times (SUM adds
 * m * value, COUNT adds m), exactly as aggregating the materialised join.
 * When the single group key is the probe key and the table reserved
 * accumulators (gq_join_opts.acc_slots), groups are accumulated inside the join
 * table itself (a group-join).  Output as for gq_groupby_agg. */
typedef struct gq_plan {
  const gq_pred* preds;
  int32_t npreds;
  int32_t probe_key;           /* column of `in`, used when join != NULL */
  const gq_join_table* join;   /* NULL: filter -> group-by only */
  const int32_t* group_keys;
  int32_t ngroup_keys;
  int32_t naggs;
  const gq_agg* aggs;
  gq_groupby_opts opts;
} gq_plan;

int gq_pipeline(gq_ctx* ctx, const gq_plan* plan, const gq_batch* in, gq_batch* out,
                int64_t* d_groups, hipStream_t stream);

/* Shared probe side: nq filter -> group-join pipelines over one probe input
 * that differ only in their join table and in one range predicate on the
 * probe side (Section 3: the pipelines of concurrent queries run side by side
 * over the same resident tables; here they also share the probe side's scan
 * and partition).  Query i equals gq_pipeline with preds = plan->preds plus
 * ranges[i] and join = tables[i], output outs[i] and group count d_groups[i]
 * (device int64).  The probe side is partitioned once, keeping the rows that
 * pass plan->preds and lie in the hull of the ranges, each kept row's value of
 * the range column carried in its tuple; each query's join takes only the
 * tuples whose carried value lies in its own range.
 *  plan     preds, probe_key, group_keys = {probe_key} (the group-join shape),
 *           aggs, opts (single mode; GQ_SORTED honoured); plan->join must be
 *           NULL (the tables are per query).
 *  tables   nq tables from gq_join_build, each partitioned (built over at
 *           least 2^20 rows) with the same region count (same build input row
 *           count and regions_log2).
 *  ranges   nq GQ_RANGE predicates, all on the same column of `in`.
 * Everything runs on `stream`; each query's join waits for its own table's
 * build.  Errors: GQ_ERR_INVALID (arguments), GQ_ERR_UNSUPPORTED (shape,
 * unpartitioned or mismatched tables; nothing enqueued), GQ_ERR_NOMEM. */
int gq_pipeline_shared(gq_ctx* ctx, const gq_plan* plan, const gq_batch* in, int32_t nq,
                       const gq_join_table* const* tables, const gq_pred* ranges, gq_batch* const* outs,
                       int64_t* const* d_groups, hipStream_t stream);

/* ---- batched fragments ----------------------------------------------------------
 * Many independent filter + group-by fragments of very different sizes run as
 * one plan: one persistent launch over tiles of all fragments, captured once in
 * a HIP graph and replayed by gq_batch_plan_launch.  (Section 2.3 finds that
 * the largest batch that fits memory runs fastest; Section 3.3 that millions
 * of small vectors degrade GPU libraries until merged.)  Every fragment has the
 * same key and aggregate shape (spec) and its own columns, predicate bounds,
 * output and cardinality hint.  Results equal one gq_groupby_agg call per
 * fragment (output in slot order).  The fragments' key columns must have the
 * same types and nullability, and every aggregate input column must be
 * nullable (has a validity bitmap) in all fragments or in none; otherwise
 * plan creation returns GQ_ERR_INVALID. */
typedef struct gq_fragment {
  gq_batch in;              /* the fragment's rows (device columns) */
  const gq_pred* preds;     /* host array, read during plan creation */
  int32_t npreds;
  int32_t reserved;
  int64_t expected_groups;  /* cardinality hint sizing the fragment's table;
                               0 = its row count */
  gq_batch out;             /* nkeys key columns then naggs int64 columns */
  int64_t* d_groups;        /* device int64: the fragment's group count */
} gq_fragment;

typedef struct gq_batch_spec {
  const int32_t* keys;
  int32_t nkeys;
  int32_t naggs;
  const gq_agg* aggs;
  float load_factor;        /* 0 = 0.5 */
  int32_t lds_max_groups;   /* fragments expecting at most this many groups
                               aggregate in LDS first; 0 = 256, -1 = never */
  int32_t tile_rows;        /* rows per work item, multiple of 1024; 0 = 8192 */
  int32_t blocks_per_cu;    /* persistent blocks per compute unit; 0 = 4 */
  int32_t radix_min_groups; /* fragments expecting at least this many groups are
                               partitioned by key hash and aggregated in LDS
                               region by region (no per-row HBM atomics);
                               0 = one more than lds_max_groups, -1 = never */
} gq_batch_spec;

typedef struct gq_batch_plan gq_batch_plan;

/* Validate the fragments, allocate every fragment's table in one arena (via
 * the context allocator), upload the descriptors and capture the graph.
 * Synchronises `stream` once.  Inputs and outputs must stay valid while the
 * plan is launched. */
int gq_batch_plan_create(gq_ctx* ctx, const gq_fragment* frags, int nfrags, const gq_batch_spec* spec,
                         hipStream_t stream, gq_batch_plan** out);
/* Enqueue one execution of the plan (a graph launch) on `stream`. */
int gq_batch_plan_launch(gq_batch_plan* plan, hipStream_t stream);
/* Plan statistics (any pointer may be NULL). */
int gq_batch_plan_info(const gq_batch_plan* plan, int64_t* total_rows, int64_t* tiles, int64_t* table_slots,
                       int64_t* bytes);
/* Wait for the device, then release the plan. */
int gq_batch_plan_free(gq_batch_plan* plan);

#ifdef __cplusplus
}
#endif

#endif /* GQ_H */
