/*
 * dr.h — C ABI of the MI355X (gfx950) segmented-range library: for_each,
 * transform_reduce and inclusive_scan over a distributed range stored as a
 * table of segments in HBM, through a lazily composed zip/transform view.
 *
 * The model (Brock et al., "Distributed Ranges: A Model for Distributed
 * Data Structures, Algorithms, and Views"):
 *  - A distributed range is a range whose segments, concatenated in order,
 *    form the logical range; segments may differ in size (section 3,
 *    "Distributed Range"). On one GPU the segments are that GPU's share of
 *    the range, each a contiguous block of HBM (section 3, "Additional
 *    Concepts": contiguous remote ranges). Here that is the segment table.
 *  - Views are lazy: zip pairs the elements of aligned ranges, transform
 *    applies an element-wise function (section 4.4 "Transform", "Zip";
 *    Algorithm 1 builds a dot product as zip | transform(l*r) | reduce).
 *    Here that is the view descriptor, evaluated in registers inside the one
 *    kernel that runs the algorithm (no intermediate array).
 *  - The algorithms are for_each, reduce and inclusive_scan over the
 *    segments (section 4.3; Algorithms 3 and 4). Here each call covers all
 *    segments at once (the paper launches per segment). The scan writes
 *    every output once: its cross-segment offsets come from a read-only
 *    first pass of tile totals (the two-pass form) or from chunk totals
 *    published one chunk ahead (the chained single pass, the default for
 *    long ranges); the paper's second pass re-reads and re-writes the
 *    output.
 *
 * Conventions shared by every entry point:
 *  - Ownership: the caller owns every buffer (inputs, outputs, the device
 *    segment table, the workspace, results). The library never allocates
 *    or frees memory and keeps no state between calls outside the
 *    caller's workspace, except one fault word per device in its static
 *    device memory (dr_check_device_error).
 *  - Asynchrony: each call only enqueues work on `stream` (NULL = the
 *    default stream) and returns; results are valid once the stream's work
 *    completes. No call synchronises the host except dr_device_status and
 *    dr_check_device_error, so the calls can be captured into a hipGraph.
 *  - Errors: arguments are checked on the host before anything is enqueued;
 *    a failed check returns a negative dr_status and enqueues nothing.
 *    dr_last_error() gives a readable reason (thread-local). Faults that
 *    only the device can see (a malformed device table, a wait that never
 *    completes, a stale plan) set a flag in the call's workspace, which
 *    dr_device_status reads, and in a fault word the library keeps per
 *    device, which dr_check_device_error reads (so calls made without a
 *    workspace report them too); the kernels then skip the work instead of
 *    touching memory out of range.
 *  - Workspace: a caller-owned device buffer of dr_workspace_bytes bytes,
 *    zero-filled once (dr_workspace_init) before its first use. The kernels
 *    leave it ready for the next call, also under hipGraph replay. Two calls
 *    that overlap in time must not share a workspace.
 *  - Alignment: vector loads need no particular alignment from the caller;
 *    segments whose pointers are misaligned relative to each other fall
 *    back to element-wise access for that segment.
 */
#ifndef DR_H
#define DR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DR_ABI_VERSION 1

/* Maximum zip arity and number of output streams per segment. */
#define DR_MAX_ARITY 4
#define DR_MAX_OUTPUTS 2

/* Tables with more rows than this need a plan (dr_plan) in the workspace;
 * smaller tables are planned inside every launch. */
#define DR_SMALL_TABLE 64

typedef enum dr_status {
    DR_OK = 0,
    DR_ERR_INVALID_ARG = -1,   /* a malformed argument (see dr_last_error) */
    DR_ERR_UNSUPPORTED = -2,   /* a dtype/op/out-dtype combination not built */
    DR_ERR_WORKSPACE = -3,     /* workspace missing, too small or misaligned */
    DR_ERR_HIP = -4,           /* the HIP runtime reported an error */
    DR_ERR_NOT_ALIGNED = -5,   /* rows of a zip do not have equal lengths */
    DR_ERR_DEVICE = -6         /* dr_device_status: the device flagged a fault */
} dr_status;

typedef enum dr_dtype {
    DR_I32 = 0,   /* int32 */
    DR_F32 = 1,   /* IEEE binary32 */
    DR_BF16 = 2,  /* bfloat16: the upper 16 bits of a binary32 */
    DR_F64 = 3,   /* IEEE binary64 */
    DR_I64 = 4    /* int64 */
} dr_dtype;

/* The transform of the view, applied to the zipped elements x0, x1:
 * identity x0 (arity 1), square x0*x0 (arity 1), mul x0*x1 (arity 2),
 * axpy x0 + alpha*x1 (arity 2). For int32 inputs alpha must be an integer. */
typedef enum dr_op {
    DR_OP_IDENTITY = 0,
    DR_OP_SQUARE = 1,
    DR_OP_MUL = 2,
    DR_OP_AXPY = 3,
    /* Black-Scholes prices of European options (the paper's Black Scholes
     * for_each benchmark, section 5): arity 4, in[0] spot S, in[1] strike K,
     * in[2] time to expiry T (years), in[3] volatility sigma; alpha is the
     * risk-free rate r. dr_for_each only, binary32 in and out, two outputs:
     * out[0] the call price S N(d1) - K exp(-rT) N(d2), out[1] the put price
     * K exp(-rT) N(-d2) - S N(-d1), with d1 = (ln(S/K) + (r + sigma^2/2) T)
     * / (sigma sqrt(T)), d2 = d1 - sigma sqrt(T) and N the standard normal
     * distribution function, evaluated in binary32 with the hardware's log2,
     * exp2, reciprocal and square root, N by the rational approximation of
     * Abramowitz & Stegun 26.2.17 (absolute error below 7.5e-8); each price
     * is within 32 units in the last place of S + K of the exact one. */
    DR_OP_BLACK_SCHOLES = 4
} dr_op;

/* Floating-point accumulation of a reduction of binary32 / bfloat16 inputs.
 * PLAIN: binary32 sums, per thread over all of its elements, then over the
 * wave and the workgroup. COMPENSATED: the same in binary32 (sum, error)
 * pairs built with error-free transformations (TwoSum on every addition,
 * FMA-based TwoProduct on binary32 products; bfloat16 products and squares
 * are exact in binary32 and need none), pairs added pairwise (TwoSum of
 * the sums, errors added). In both, only the workgroup's partial is widened
 * (exactly) to binary64, and the combine across workgroups and segments is
 * binary64. Integer reductions are always exact in int64 and ignore this
 * setting; binary64 inputs accumulate in binary64. */
typedef enum dr_acc {
    DR_ACC_PLAIN = 0,
    DR_ACC_COMPENSATED = 1
} dr_acc;

/* CONCAT: the segments are one distributed range (results: one reduction;
 * the scan carries across segment boundaries). BATCH: each segment is an
 * independent range (one reduction per segment; the scan restarts at every
 * segment). */
typedef enum dr_mode {
    DR_MODE_CONCAT = 0,
    DR_MODE_BATCH = 1
} dr_mode;

/* Scan flags. REVERSE: suffix sums (element i gets the sum of elements i
 * and after), the adjoint of the forward scan. CARRY_F32: binary32 carries
 * for floating-point scans instead of binary64 (only for comparisons of
 * accuracy; binary64 carries are the default). */
enum {
    DR_SCAN_REVERSE = 1u,
    DR_SCAN_CARRY_F32 = 2u
};

/* Algorithm ids for dr_workspace_bytes and dr_plan. */
typedef enum dr_algo {
    DR_ALGO_FOR_EACH = 0,
    DR_ALGO_REDUCE = 1,
    DR_ALGO_SCAN = 2,
    DR_ALGO_SCAN_REDUCE = 3,
    DR_ALGO_BROADCAST_MUL = 4
} dr_algo;

/* The view descriptor: zip arity, element type of the zipped inputs (all
 * inputs share it), the transform and its scalar. */
typedef struct dr_view {
    int32_t arity;     /* 1, 2 or 4; must equal the arity of `op` */
    int32_t in_dtype;  /* dr_dtype of every zipped input */
    int32_t op;        /* dr_op */
    int32_t reserved;  /* must be 0 */
    double alpha;      /* scalar of DR_OP_AXPY, ignored otherwise */
} dr_view;

/* One row of the segment table: segment k of every zipped input, the
 * segment's output stream(s), and its length in elements (the same for all
 * of them: the zip is aligned, section 4.4 "Zip"). 64 bytes. Pointers are
 * device pointers; unused slots must be NULL. */
typedef struct dr_segment {
    const void* in[DR_MAX_ARITY];
    void* out[DR_MAX_OUTPUTS];
    int64_t length;
    int64_t reserved;   /* must be 0 */
} dr_segment;

/* The segment table. `rows` is a DEVICE array of n_segments rows read by the
 * kernels. `host_rows`, when not NULL, is a host copy of the same rows that
 * the library checks before enqueuing (lengths, NULL pointers, the sum of
 * lengths, overlap of outputs with inputs); without it only the device
 * checks apply. total_length must equal the sum of the lengths. */
typedef struct dr_table {
    const dr_segment* rows;
    const dr_segment* host_rows;
    int64_t n_segments;
    int64_t total_length;
    int32_t mode;       /* dr_mode */
    int32_t reserved;   /* must be 0 */
} dr_table;

/* Launch shape. block_threads: threads per workgroup, 0 or 256 for every
 * kernel; 512 and 1024 for the single-pass look-back scan only
 * (DR_TUNE_TILE_PER_BLOCK; binary32 sums of the identity view with binary64
 * carries, plain or fused with the compensated dot), any other call with
 * them returns DR_ERR_UNSUPPORTED. items_per_thread: elements per thread per
 * tile (a tile is block_threads * items_per_thread elements), one of the
 * values dr_tuning_supported accepts; flags: DR_TUNE_* bits. NULL = the
 * built-in default for the call: 256 threads, 16 items per thread, except
 * bfloat16 reductions (32) and the scan defaults described at
 * dr_inclusive_scan. dr_plan and dr_workspace_bytes given NULL assume the
 * same defaults; given a tuning, they size for its tile. */
typedef struct dr_tuning {
    int32_t block_threads;
    int32_t items_per_thread;
    int32_t flags;
    int32_t reserved;   /* must be 0 */
} dr_tuning;

/* dr_tuning.flags: one workgroup per tile, single pass. For a CONCAT
 * transform_reduce: a per-tile combine instead of a resident grid whose
 * workgroups each sum many tiles and combine once. For inclusive_scan /
 * scan_reduce: one kernel whose tiles, in block-index order, take their
 * carries from a decoupled look-back over their predecessors, instead of
 * the default read-only tile-totals pass followed by the apply pass (the
 * input is read once). In BATCH mode a tile's look-back stops at its range's
 * first tile, so ranges of one tile never wait. The carries of binary32 /
 * binary64 scans are then sums of the predecessors in an order that depends
 * on timing: results stay within the same error bound but need not repeat
 * bit for bit from run to run (integer results are exact either way). */
enum { DR_TUNE_TILE_PER_BLOCK = 1 };

/* dr_tuning.flags for inclusive_scan, scan (sum) and scan_reduce: one pass
 * whose workgroups, one per CU and all resident (a cooperative launch),
 * split their waves into loaders (the input into a ring of LDS slots and
 * each tile's total), writers (tile scan plus carry, outputs written once),
 * a publisher of the totals and a fetcher of the carries, while one
 * workgroup scans the published totals in a fixed order (results repeat
 * from run to run). Built for sums of the identity view over binary32,
 * bfloat16, binary64 and int32 -> int32 (fused: binary32), at 32 items per
 * thread (binary64 and fused 16), which items_per_thread must name. Where
 * the device cannot hold the whole grid at once, or the stream is being
 * captured into a graph, the call runs the default two passes instead.
 * Results are those of a fixed order of operations, like the default's. */
enum { DR_TUNE_SPECIALIZED = 2 };

/* dr_tuning.flags for inclusive_scan, scan (sum) and scan_reduce: the
 * reduce-then-scan form (the default except where dr_inclusive_scan names
 * another): a
 * read-only pass forms every tile's total, one workgroup scans the
 * per-chunk totals, and the apply pass reads the input again, scans each
 * tile and adds its carry (three launches; the input is read twice). Max /
 * min scans always run this form. */
enum { DR_TUNE_TWO_PASS = 4 };

/* dr_tuning.flags for inclusive_scan and scan (sums): the chained single
 * pass. Workgroups claim chunks of 4 tiles from a counter; each chunk is
 * read once to publish its total and read again one chunk later, when its
 * carry is known, to be scanned and written (the re-read mostly misses the
 * L2 cache: the memory counters see the input fetched twice). Carries are sums over a fixed shape (chunk totals
 * folded per superblock of 128 chunks, running carries chained across
 * superblocks), so results repeat from run to run. Built for one range
 * (CONCAT) of sums of the identity view: F32 -> F32 (binary64 carries, or
 * binary32 with DR_SCAN_CARRY_F32), I32 -> I64 and I32 -> I32, at 16 items
 * per thread (items_per_thread 0 or 16), forward and reverse, with the
 * initial value and the exclusive form of dr_scan. Any other call with it
 * (BATCH tables, other dtypes or views, max / min, the fused scan_reduce)
 * returns DR_ERR_UNSUPPORTED before anything is enqueued. */
enum { DR_TUNE_CHAINED = 8 };

/* Library version (DR_ABI_VERSION). Never fails. */
int dr_abi_version(void);

/* Static string for a status code. Never fails. */
const char* dr_status_string(dr_status status);

/* Detail of the last error returned on the calling thread ("" if none). */
const char* dr_last_error(void);

/* 1 if (algo, view, out_dtype, tuning) has a built kernel, else 0: the
 * tuning's block_threads, items_per_thread and form flag (the look-back
 * form has shapes of its own, see dr_tuning). For DR_ALGO_REDUCE
 * `out_dtype` carries the dr_acc instead; for DR_ALGO_SCAN the carries are
 * the default (binary64 for binary32 input); for DR_ALGO_SCAN_REDUCE the
 * reduce view is mul, compensated. */
int dr_tuning_supported(int32_t algo, const dr_view* view, int32_t out_dtype,
                        const dr_tuning* tuning);

/* Bytes of workspace that `algo` needs for a table of n_segments rows and
 * total_length elements with this view and tuning (for DR_ALGO_SCAN_REDUCE
 * the view is the scanned one). Writes *bytes; host only, enqueues nothing. */
dr_status dr_workspace_bytes(int32_t algo, int64_t n_segments, int64_t total_length,
                             const dr_view* view, const dr_tuning* tuning, size_t* bytes);

/* Zero-fill a fresh workspace (ws_bytes bytes, 256-byte aligned device
 * pointer) on `stream`. Needed once after allocation. */
dr_status dr_workspace_init(void* workspace, size_t ws_bytes, void* stream);

/* Build the tile plan of a large table (more than DR_SMALL_TABLE rows) in
 * the workspace: the prefix of per-segment tile counts and a tile ->
 * segment map. Needed once per (table, algo, view dtype, tuning,
 * workspace); calls whose plan does not match flag a device error and do
 * nothing. Tables of at most DR_SMALL_TABLE rows need no plan. */
dr_status dr_plan(const dr_table* table, int32_t algo, const dr_view* view,
                  const dr_tuning* tuning, void* workspace, size_t ws_bytes, void* stream);

/*
 * for_each (section 4.3, "for_each"; section 5.1, "Stream"):
 * for every segment k and index j < length_k,
 *     rows[k].out[0][j] = op(in[0][j], in[1][j])
 * evaluated in the output type with one rounding per arithmetic operation
 * and no fused multiply-add (the triad a = b + s*c is fl(b + fl(s*c))).
 * Supported (in_dtype -> out_dtype): F32 -> F32, BF16 -> F32, F64 -> F64,
 * I32 -> I32 (two's complement wrap), I32 -> I64.
 * The workspace is required for tables larger than DR_SMALL_TABLE (it holds
 * their plan) and optional otherwise (NULL/0); when one is given, it is
 * checked as for the other calls and a malformed device table is flagged
 * in it as well as in the device's fault word (dr_check_device_error).
 */
dr_status dr_for_each(const dr_table* table, const dr_view* view, int32_t out_dtype,
                      void* workspace, size_t ws_bytes, const dr_tuning* tuning,
                      void* stream);

/*
 * transform_reduce (section 4.3, "reduce"; Algorithms 1 and 3):
 * R = init + sum of op(in[0][j], in[1][j]) over all elements (CONCAT), or
 * R_k = init + sum over segment k (BATCH). Partial sums are combined in a
 * fixed order, so results are the same from run to run.
 *  - I32 inputs: exact in int64; `init` points to an int64_t (host);
 *    `result` is a device int64 array.
 *  - F32/BF16 inputs: per `acc` inside tiles, binary64 across tiles and
 *    segments; `init` points to a double (host); `result` is a device
 *    binary64 array. F64 inputs accumulate in binary64.
 * `result` has 1 (CONCAT) or n_segments (BATCH) elements. An empty range
 * gives `init`.
 */
dr_status dr_transform_reduce(const dr_table* table, const dr_view* view, int32_t acc,
                              const void* init, void* result, void* workspace,
                              size_t ws_bytes, const dr_tuning* tuning, void* stream);

/*
 * inclusive_scan (section 4.3, "inclusive_scan"; Algorithm 4):
 * out[0] of the element at logical position i receives the sum of the
 * view over positions 0..i (CONCAT: across segments; BATCH: within the
 * element's segment), or over positions i.. (DR_SCAN_REVERSE).
 * The offset of a segment is the total of the segments before it (0 for the
 * first). The reduce-then-scan form runs three kernels: tile totals (reads
 * the input), a scan of per-chunk totals, and the tile scans plus carries
 * (reads the input again, writes the output once); carries are sums in a
 * fixed order, so results repeat from run to run (DR_TUNE_TWO_PASS names
 * this form explicitly; which form runs without a tuning is stated below). DR_TUNE_TILE_PER_BLOCK selects one kernel whose
 * tiles take their carries from a decoupled look-back, DR_TUNE_SPECIALIZED
 * the single pass with specialised waves, and DR_TUNE_CHAINED the chained
 * single pass (one range; the input read from HBM once); at most one form
 * flag. Without a tuning: sums of the identity view over one range (CONCAT)
 * of more than 2^22 F32 -> F32 or I32 -> I64 / I32 elements run the chained
 * single pass; other int32 scans of at most 2^22 elements take the
 * look-back form (lower latency, exact either way); other larger int32 ->
 * int64 scans of the identity view over tables of at most DR_SMALL_TABLE
 * rows use tiles of 64 items per thread (the output is twice the input's
 * size); everything else runs the reduce-then-scan form. Supported (in_dtype -> out_dtype): I32 -> I64 (exact), I32 -> I32
 * (exact modulo 2^32), F32 -> F32 and BF16 -> F32 (binary32 inside a tile,
 * binary64 carries unless DR_SCAN_CARRY_F32), F64 -> F64.
 * In-place (out[0] == in[0], same dtype size) is allowed; other overlap
 * between outputs and inputs is rejected when host_rows is given.
 */
dr_status dr_inclusive_scan(const dr_table* table, const dr_view* view, int32_t out_dtype,
                            uint32_t flags, void* workspace, size_t ws_bytes,
                            const dr_tuning* tuning, void* stream);

/*
 * Fused inclusive_scan + transform_reduce over the same rows in one call
 * (the reduction runs inside the scan's apply pass, so in[1] is read once):
 * out[0] receives the inclusive scan of the
 * scan view (identity of in[0]), and `result` the reduction of the reduce
 * view (mul over in[0], in[1]); both per segment in BATCH mode. Types:
 * F32 in -> F32 scan out (binary64 carries) and a binary64 result with
 * `acc` accumulation; F64 in -> F64 scan out and result (`acc` ignored).
 * `init` is a host double. This is the batched form: thousands of ragged
 * ranges in BATCH mode are one call (capturable in a hipGraph).
 */
dr_status dr_scan_reduce(const dr_table* table, const dr_view* scan_view,
                         const dr_view* reduce_view, int32_t acc, const void* init,
                         void* result, uint32_t flags, void* workspace, size_t ws_bytes,
                         const dr_tuning* tuning, void* stream);

/*
 * Adjoint of transform_reduce: for every element, out[w][j] =
 * fl(g_r * d op / d x_w) for w < `n_grads` outputs, where g is a DEVICE
 * binary64 array of 1 (CONCAT) or n_segments (BATCH) upstream gradients,
 * the derivative is evaluated on in[0], in[1] (mul: d/dx0 = x1,
 * d/dx1 = x0; square: 2*x0; identity: 1; axpy: 1 and alpha), the product is
 * binary64 and rounded once to the output type (= the input type; BF16
 * inputs give F32 gradients). Workspace as dr_for_each.
 */
dr_status dr_broadcast_mul(const dr_table* table, const dr_view* view, const double* g,
                           int32_t n_grads, void* workspace, size_t ws_bytes,
                           const dr_tuning* tuning, void* stream);

/* ---- Generic operators (section 4.3) ----------------------------------------
 * The paper's reduce and scan take any commutative binary operator (its
 * listings show +), reduce takes an initial value, and exclusive_scan is
 * built like inclusive_scan. */

/* Combine operators. Max / min compare the view values as dr_for_each
 * would store them (binary32 arithmetic with one rounding per operation for
 * F32 and BF16 inputs, binary64 for F64, exact int64 for I32); the results
 * are exact. NaN values are ignored (IEEE maxNum / minNum) unless every
 * value is NaN. */
typedef enum dr_combine { DR_COMBINE_SUM = 0, DR_COMBINE_MAX = 1, DR_COMBINE_MIN = 2 } dr_combine;

/* dr_scan flag (with DR_SCAN_REVERSE, DR_SCAN_CARRY_F32): exclusive scan. */
enum { DR_SCAN_EXCLUSIVE = 4 };

/*
 * reduce with an operator (section 4.3, "reduce"; Algorithm 3): R = init
 * combined with every view value (CONCAT), or R_k per segment (BATCH).
 * `init` is a host pointer (int64_t for I32 inputs, double otherwise) or
 * NULL for the operator's identity (0, -inf / INT64_MIN for max,
 * +inf / INT64_MAX for min); an empty range gives it. DR_COMBINE_SUM is
 * dr_transform_reduce (`acc` as there); for max / min `acc` is ignored and
 * every op and input dtype is supported at the default tile (16 items per
 * thread; bfloat16 32, and 16 with a tuning). Results, workspace and tuning
 * as dr_transform_reduce.
 */
dr_status dr_reduce(const dr_table* table, const dr_view* view, int32_t combine, int32_t acc,
                    const void* init, void* result, void* workspace, size_t ws_bytes,
                    const dr_tuning* tuning, void* stream);

/*
 * scan with an operator, an initial value and the exclusive form (section
 * 4.3, "inclusive_scan" and the exclusive_scan built like it): element i
 * of the range receives init combined with the view values up to and
 * including i (inclusive), or strictly before i (DR_SCAN_EXCLUSIVE; the first
 * element receives init); after i instead of before it with
 * DR_SCAN_REVERSE; per segment in BATCH mode. `init` is a host int64_t (I32
 * inputs) or double, or NULL for the identity. The initial value enters the
 * outputs only (binary64 for floating inputs, rounded once with the
 * element's value into the output type).
 * DR_COMBINE_SUM: the dtypes, ops, flags and forms of dr_inclusive_scan;
 * DR_COMBINE_MAX / MIN: the identity view, every dtype pair of
 * dr_inclusive_scan, the default (reduce-then-scan) form at 16 items per
 * thread; DR_SCAN_CARRY_F32 and DR_TUNE_TILE_PER_BLOCK are rejected
 * (DR_ERR_UNSUPPORTED).
 */
dr_status dr_scan(const dr_table* table, const dr_view* view, int32_t out_dtype, int32_t combine,
                  uint32_t flags, const void* init, void* workspace, size_t ws_bytes,
                  const dr_tuning* tuning, void* stream);

/* ---- Segment algebra (host side; section 4.4) ------------------------------
 * Views that change which elements or which segment boundaries a call sees.
 * They only compute new segment lists on the host; the kernels above then
 * run on the result unchanged. */

/* One segment of a single distributed range: `length` elements at `ptr`
 * (device memory; only the address is used here). */
typedef struct dr_span {
    void* ptr;
    int64_t length;
} dr_span;

/* A distributed range (section 3): its segments in order, each of elements
 * of `elem_size` bytes. `spans` is a host array. */
typedef struct dr_range {
    const dr_span* spans;
    int64_t n_spans;
    int32_t elem_size;   /* bytes per element, > 0 */
    int32_t reserved;    /* must be 0 */
} dr_range;

/*
 * take / drop (section 4.4, "Take and Drop": trim_segments): the segments
 * of `r` restricted to the elements [first, last) of its concatenation, in
 * order; segments that keep no element are left out. take(l) is [0, l),
 * drop(f) is [f, total). `first` and `last` are clamped to [0, total]; last
 * <= first gives an empty range. Writes at most r->n_spans spans to `out`
 * (host array of `capacity` entries) and their count to *n_out. Host only:
 * no device access, nothing enqueued. Errors (DR_ERR_INVALID_ARG): NULL
 * pointers, a negative length, elem_size <= 0, a non-zero reserved field,
 * capacity smaller than the result.
 */
dr_status dr_trim_segments(const dr_range* r, int64_t first, int64_t last, dr_span* out,
                           int64_t capacity, int64_t* n_out);

/*
 * zip of ranges whose segments are not aligned (section 4.4, "Zip"): the
 * coarsest common refinement of the segment boundaries of `n_in` input
 * ranges (1..DR_MAX_ARITY) and `n_out` output ranges (0..DR_MAX_OUTPUTS), as
 * segment-table rows. Walking all ranges together, each row takes from every
 * range the largest piece that stays inside that range's current segment,
 * i.e. the minimum of their remaining lengths; row k's in[i] / out[j] point
 * at the k-th piece of input i / output j, and `length` is the common piece
 * length. Empty segments are stepped over and produce no row. The zip ends
 * with the shortest range; *length receives its element count. At most the
 * total number of spans of all ranges rows are written to `rows` (host
 * array of `capacity` entries; unused in/out slots are NULL); *n_rows
 * receives the count. Copy the rows to the device for dr_table.rows and
 * pass them as dr_table.host_rows. Host only. Errors as dr_trim_segments,
 * plus n_in / n_out out of range.
 */
dr_status dr_zip_segments(const dr_range* ins, int32_t n_in, const dr_range* outs, int32_t n_out,
                          dr_segment* rows, int64_t capacity, int64_t* n_rows, int64_t* length);

/*
 * Read and clear the device fault flag of a workspace. Synchronises
 * `stream`. *flags (host) receives the raw flag bits (0 = no fault): 1 = a
 * row of the device table was malformed (negative length, NULL pointer,
 * lengths not summing to total_length), 2 = a look-back wait timed out,
 * 4 = the plan in the workspace did not match the call, 8 = the tile count
 * exceeded the bound the workspace was sized for. Returns DR_ERR_DEVICE
 * when any bit was set.
 */
dr_status dr_device_status(void* workspace, uint32_t* flags, void* stream);

/*
 * Read and clear the fault word the library keeps for the device of
 * `stream` (NULL = the current device): the DR_DEVFLAG bits (as
 * dr_device_status) of every fault any kernel of the library flagged on
 * that device since the last read, including calls made without a
 * workspace. Synchronises `stream`; *flags (host) receives the bits.
 * Returns DR_ERR_DEVICE when any bit was set. The word is shared by every
 * caller on the device: concurrent callers see each other's faults.
 */
dr_status dr_check_device_error(uint32_t* flags, void* stream);

/*
 * inclusive_scan that allocates nothing and takes no workspace: for callers
 * that cannot allocate device memory (code being captured into a hipGraph,
 * tight serving loops, harnesses that forbid hipMalloc). Same operation,
 * arguments, forms and results as dr_inclusive_scan, with the workspace
 * replaced by a static scratch area of the library (8 MiB per device,
 * resident from the first call on a device until the process ends; zero-
 * filled on that first call by a kernel enqueued on `stream`). Tables of
 * more than DR_SMALL_TABLE rows are planned into the scratch by every call.
 * A call whose workspace would not fit the scratch (more than about 2.6e5
 * tiles: 2^30 binary32 elements at the default tile) is rejected with
 * DR_ERR_WORKSPACE before anything is enqueued. Every call on a device
 * shares its scratch, which keeps the last call's contents: calls that
 * overlap in time on one device (other streams, other threads) race and
 * must be ordered by the caller. Device faults are reported only through
 * dr_check_device_error. Never calls hipMalloc / hipFree.
 */
dr_status dr_inclusive_scan_noalloc(const dr_table* table, const dr_view* view, int32_t out_dtype,
                                    uint32_t flags, const dr_tuning* tuning, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* DR_H */
