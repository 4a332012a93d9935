/*
 * sg_spgemm.h - C ABI of the MI355X (gfx950) local sparse product library.
 *
 * The library computes C = A (x) B over a semiring for sparse operands held
 * in device memory: the local product that every processor of Sparse SUMMA
 * runs on its 2D blocks at each stage (paper, Sections 2.4, 3.2 and 3.5),
 * column by column, C(:, j) = (+)_k A(:, k) (x) B(k, j) (the column-by-column
 * formulation of Section 2.1, Figure 3), together with the accumulation of
 * the stage partial products C_ij = (+)_k A_ik B_kj (Section 3.2). Products
 * that share an output (a "group") are accumulated into it directly, so the
 * stage partials are never materialised.
 *
 * Conventions for every entry point:
 *  - Ids are 0-based (the paper is 1-based).
 *  - Every array pointer inside sg_mat / sg_mat_out is a DEVICE pointer owned
 *    by the caller; the library never frees or reallocates them.
 *  - `ws` is a caller-owned DEVICE workspace of the size the matching
 *    *_workspace_size call reports; the library allocates no device memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *  - Status codes are returned, never thrown; no entry point exits the
 *    process. A call that returns an error leaves its outputs undefined.
 *  - Operands must be canonical: ptr non-decreasing from 0, minor ids in
 *    [0, minor dim) strictly increasing inside each vector, and for the
 *    doubly compressed formats vid strictly increasing and every stored
 *    vector non-empty (Section 2.3). sg_validate checks this on the device.
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
    SG_ERR_INVALID_ARG = -1,   /* NULL pointer, negative size, bad enum        */
    SG_ERR_DIM_MISMATCH = -2,  /* inner dimensions or group shapes differ      */
    SG_ERR_NOT_CANONICAL = -3, /* sg_validate found an unsorted/duplicate id   */
    SG_ERR_UNSUPPORTED = -4,   /* format/orientation combination not handled   */
    SG_ERR_WORKSPACE = -5,     /* workspace smaller than the reported size     */
    SG_ERR_CAPACITY = -6,      /* output arrays smaller than the exact result  */
    SG_ERR_HIP = -7,           /* a HIP runtime call failed                    */
    SG_ERR_OOM = -8            /* host allocation failed                       */
} sg_status;

/*
 * Semiring descriptor (Section 1: the product is defined over an arbitrary
 * semiring). The kind fixes the value type, add (+), multiply (x) and the
 * additive identity:
 *   SG_PLUS_TIMES_F64  double, +, *, 0
 *   SG_PLUS_TIMES_F32  float,  +, *, 0 (accumulates in float)
 *   SG_MIN_PLUS_I32    int32, min, saturating + (INT32_MAX is +infinity and
 *                      absorbs), INT32_MAX
 *   SG_OR_AND_BOOL     pattern only (val arrays are NULL), or, and
 * Every position produced by at least one multiplication is stored, even if
 * its value equals the additive identity (a structural product).
 */
typedef enum {
    SG_PLUS_TIMES_F64 = 0,
    SG_PLUS_TIMES_F32 = 1,
    SG_MIN_PLUS_I32 = 2,
    SG_OR_AND_BOOL = 3
} sg_semiring_kind;

typedef struct {
    int32_t kind; /* sg_semiring_kind */
} sg_semiring;

/*
 * Storage formats (Sections 2.2 and 2.3). CSR/CSC: ptr has major_dim + 1
 * entries and vid is NULL. DCSR/DCSC (doubly compressed): vid lists the nvec
 * non-empty major ids (the paper's JC for DCSC) and ptr has nvec + 1 entries
 * (the paper's CP); idx/val are the paper's IR/NUM.
 */
typedef enum { SG_CSR = 0, SG_CSC = 1, SG_DCSR = 2, SG_DCSC = 3 } sg_format;

typedef struct {
    int32_t fmt;        /* sg_format                                         */
    int64_t nrows;
    int64_t ncols;
    int64_t nvec;       /* stored vectors: nrows (CSR), ncols (CSC), nzc/nzr  */
    int64_t nnz;
    const int64_t *ptr; /* device, nvec + 1                                  */
    const int32_t *vid; /* device, nvec (doubly compressed) or NULL          */
    const int32_t *idx; /* device, nnz                                       */
    const void *val;    /* device, nnz values; NULL for SG_OR_AND_BOOL       */
} sg_mat;

/* Output matrix. Capacities come from sg_sym_info (exact sizes). */
typedef struct {
    int32_t fmt;        /* must have the operands' orientation               */
    int64_t nrows;
    int64_t ncols;
    int64_t cap_nnz;    /* entries available in idx/val                      */
    int64_t cap_vec;    /* entries available in vid (doubly compressed only) */
    int64_t *ptr;       /* device: major_dim + 1 (CSR/CSC) or cap_vec + 1    */
    int32_t *vid;       /* device, doubly compressed only, else NULL         */
    int32_t *idx;       /* device                                            */
    void *val;          /* device; NULL for SG_OR_AND_BOOL                   */
} sg_mat_out;

/*
 * Tuning knobs of the flops-binned numeric tiers. sg_tuning_default fills
 * the values the library uses when a NULL tuning pointer is passed.
 *   tiny_max_flops   vectors with at most this many multiplications run on
 *                    one wavefront with a register sort/merge (<= 64)
 *   mid_max_ub       vectors whose size bound min(flops, minor dim) is at
 *                    most this use one workgroup with an LDS-resident
 *                    accumulator (bitmap-rank or open-addressing hash)
 *   mid_kind         0 = bitmap-rank accumulator, 1 = LDS hash accumulator
 *   lds_bytes        LDS budget of one workgroup of the mid tier and of the
 *                    count passes
 *   block_threads    threads per workgroup of the mid tier and of the count
 *                    passes (64..1024)
 *   chunk_width      heavy tier: width in ids of one split bucket (rank
 *                    windows) or of one dense window (0 = automatic)
 *   heavy_kind       heavy tier: 0 = bitmap-rank windows planned from exact
 *                    bucket counts wherever the id-range bitmap fits in LDS,
 *                    dense windows elsewhere; 1 = dense windows only (each
 *                    one a flag bit and a value slot per id)
 *   force_tier       -1 = bin by size; 0/1/2 = route every vector with
 *                    work to the tiny / mid / heavy tier where it is legal
 *                    (tiny needs flops <= 64, mid needs the bound to fit);
 *                    3 = every vector with at most 1024 multiplications
 *                    (and an id range below 2^22 - 1) to the mid tier's
 *                    one-wavefront form (small_max_flops), the others by
 *                    size
 *   blocks_per_cu    workgroups per compute unit of the persistent launches
 *   validate         non-zero: run sg_validate on every operand first
 *   xcd_ranges       heavy tier: the output id range is cut into 8 x this
 *                    many consecutive ranges, no heavy window crosses a range,
 *                    and the numeric launch keeps one work queue per XCD (the
 *                    chip's 8 dies, each with its own L2) holding the windows
 *                    of that XCD's ranges, so each L2 caches a slice of the
 *                    gathered operand; workgroups drain their own XCD's queue
 *                    first and then help the others (0 = one shared queue)
 *   bitmap_mb        heavy tier: MiB of workspace in which the count pass
 *                    keeps each heavy vector's id bitmap, so that numeric
 *                    windows load their slice instead of re-marking it
 *                    (vectors beyond the budget re-mark; 0 = never keep)
 *   heavy_threads    threads per workgroup of the heavy-tier numeric launch
 *                    and of the single persistent launch (0 = block_threads)
 *   heavy_lds_bytes  LDS budget of those workgroups; heavy windows are
 *                    planned to fit it, so a larger budget means fewer,
 *                    wider windows (0 = lds_bytes). The persistent launch
 *                    uses the larger of the two budgets.
 *   entry_mb         heavy tier: MiB of workspace for per-window entry
 *                    records (the addresses of the G slice of every streamed
 *                    entry inside a window, and its S value), written once by
 *                    the symbolic phase so that the numeric walk reads one
 *                    record per entry instead of the segment's descriptors,
 *                    the entry, its G vector and its window split points in
 *                    turn; a vector fed by several products (the stage
 *                    products of a SUMMA share) walks its records as one
 *                    list. Windows beyond the budget walk the operands (0 =
 *                    off, the default: building them costs the symbolic phase
 *                    about what they save one numeric run, so they pay only
 *                    for a plan whose numeric phase is replayed). Mid-tier
 *                    vectors of a plan with records get records too.
 *   small_max_flops  mid tier: vectors with more than tiny_max_flops and at
 *                    most this many multiplications (<= 1024), whose id
 *                    range is below 2^22 - 1, run one per wavefront with no
 *                    workgroup barrier: their ids are gathered into
 *                    registers (16 per lane) and their products into the
 *                    wavefront's LDS, (id, slot) keys are sorted with a
 *                    register bitonic network, and runs of equal ids are
 *                    summed and written (0 = off: every mid vector takes a
 *                    workgroup's LDS accumulator). They count as mid-tier
 *                    vectors in the per-tier totals (n_small of sg_sym_info).
 *                    Only plans with at least 8192 output vectors (bound
 *                    from the streamed operand) use it: fewer could not give
 *                    the chip's wavefronts one vector each.
 */
typedef struct {
    int32_t tiny_max_flops;
    int32_t mid_max_ub;
    int32_t mid_kind;
    int32_t lds_bytes;
    int32_t block_threads;
    int32_t chunk_width;
    int32_t heavy_kind;
    int32_t force_tier;
    int32_t blocks_per_cu;
    int32_t validate;
    int32_t xcd_ranges;
    int32_t bitmap_mb;
    int32_t heavy_threads;
    int32_t heavy_lds_bytes;
    int32_t entry_mb;
    int32_t small_max_flops;
} sg_tuning;

/* Host-side sizes of one output, valid when sg_spgemm_symbolic returns. */
typedef struct {
    int64_t flops;       /* multiplications (Section 1's flops)              */
    int64_t nnz_ub;      /* sum over output vectors of min(flops_j, minor)   */
    int64_t nnz;         /* exact nnz(C)                                     */
    int64_t nvec;        /* stored vectors of C for its format               */
    int64_t max_vec_flops;
    int64_t n_out_vec;   /* output vectors with at least one stored input   */
    int64_t n_tiny;      /* vectors per tier                                 */
    int64_t n_mid;
    int64_t n_heavy;
    int64_t n_heavy_items; /* (vector, window) work items of the heavy tier  */
    /* totals per tier (index 0 tiny, 1 mid, 2 heavy) over the whole call:  */
    int64_t tier_flops[3]; /* multiplications (mid: n_mid and n_small)      */
    int64_t tier_sent[3];  /* stored entries of the streamed operand read   */
    int64_t tier_nnz[3];   /* output entries written                        */
    int64_t n_small;       /* mid-tier vectors run one per wavefront (not in n_mid) */
} sg_sym_info;

typedef struct sg_plan sg_plan;

/* Defaults for a semiring (see sg_tuning). */
void sg_tuning_default(int32_t semiring_kind, sg_tuning *tuning);

/* Static text for a status code. */
const char *sg_status_string(int32_t status);

/*
 * Text describing the last HIP runtime failure seen by this host thread
 * (the call, HIP's error string and the source line), or "" if none.
 * The pointer stays valid until the thread's next failing call.
 */
const char *sg_last_error(void);

/*
 * Device workspace needed by sg_spgemm_symbolic for the same arguments.
 * Host-only: reads no device memory. Arguments as in sg_spgemm_symbolic.
 */
sg_status sg_spgemm_workspace_size(const sg_semiring *sr, int32_t nprod,
                                   const sg_mat *A, const sg_mat *B,
                                   const int32_t *group, int32_t ngroup,
                                   int32_t out_fmt, const sg_tuning *tuning,
                                   size_t *ws_bytes);

/*
 * Symbolic phase of C_g = (+)_{p : group[p] = g} A_p (x) B_p.
 *
 * nprod products (host arrays A[nprod], B[nprod] of descriptors of device
 * data) are accumulated into ngroup outputs; group[p] in [0, ngroup) (host
 * array; NULL means group[p] = p and ngroup = nprod). All operands share one
 * orientation: column-major (CSC/DCSC; C is column-major, the columns of B
 * are streamed and the columns of A gathered, Section 2.1) or row-major
 * (CSR/DCSR; rows of A streamed, rows of B gathered). Within a group all
 * products have the same m x n output shape and inner dimensions must agree
 * per product. out_fmt is the format of every C_g.
 *
 * The phase computes flops per output vector and the bound min(flops,
 * minor dim) (the symbolic pass), bins vectors into the tiny / mid / heavy
 * tiers, counts the exact size of every output vector and builds the output
 * pointers. For doubly compressed gathered operands the column lookup uses
 * the AUX index of Section 2.3. It ends with one stream synchronisation and
 * fills info[g] (host array of ngroup) for each group.
 *
 * *plan receives a library-owned handle (host memory only) that refers to
 * ws and to the operand arrays: both must stay alive and structurally
 * unchanged until sg_plan_destroy; the operand VALUES may change between
 * numeric calls. Errors: INVALID_ARG, DIM_MISMATCH, UNSUPPORTED, WORKSPACE,
 * NOT_CANONICAL (when tuning->validate), HIP.
 */
sg_status sg_spgemm_symbolic(const sg_semiring *sr, int32_t nprod,
                             const sg_mat *A, const sg_mat *B,
                             const int32_t *group, int32_t ngroup,
                             int32_t out_fmt, const sg_tuning *tuning,
                             void *ws, size_t ws_bytes, sg_plan **plan,
                             sg_sym_info *info, void *stream);

/*
 * Search of the tuning knobs for one product shape (the arguments of
 * sg_spgemm_symbolic), by timing whole runs on the device: coordinate
 * descent from *tuning over a built-in table of settings, most influential
 * knob first, keeping a change that is at least 2% faster. form 0 times
 * symbolic + sg_spgemm_numeric per run, form 1 symbolic + sg_spgemm_batched,
 * form 2 (a plan whose numeric phase is replayed) sg_spgemm_batched alone on
 * one plan, and then searches the entry-record budget and the tier
 * thresholds. Each time is the median of `reps` runs after one warm-up, host
 * clock around a stream synchronisation. Every candidate computes the same
 * product (the tiers are exact); settings the library refuses for this shape
 * are skipped. The call allocates and frees the workspace and the outputs of
 * every candidate itself (device memory for the largest one must be free),
 * leaves the operands unchanged and synchronises `stream`. On return *tuning
 * holds the best setting, *best_ms its time and *start_ms (may be NULL) the
 * time of the setting passed in. Errors: INVALID_ARG, and those of the first
 * (starting) run.
 */
sg_status sg_autotune(const sg_semiring *sr, int32_t nprod, const sg_mat *A, const sg_mat *B,
                      const int32_t *group, int32_t ngroup, int32_t out_fmt, int32_t form, int32_t reps,
                      sg_tuning *tuning, double *best_ms, double *start_ms, void *stream);

/*
 * Output mask of one group (Section 6.2.2's breadth-first search removes the
 * vertices already visited from each new frontier). bits is a DEVICE bitmap:
 * bit (i, j) for output vector j (the major id: a column of column-major C)
 * and output id i is bit i % 32 of bits[j * stride_words + i / 32];
 * stride_words >= ceil(minor dimension / 32). complement = 1 keeps only the
 * entries whose bit is 0 (C = (A B) with the set positions removed),
 * complement = 0 only those whose bit is 1. bits == NULL: no mask.
 */
typedef struct {
    const uint32_t *bits;
    int64_t stride_words;
    int32_t complement;
    int32_t pad;
} sg_mask;

/*
 * sg_spgemm_symbolic with an output mask per group (host array masks[ngroup]
 * of descriptors; NULL = no masks). Every phase applies the mask: the exact
 * sizes count only the kept entries, and the numeric phase writes only
 * those. The bitmaps are read by the symbolic call and by every later
 * numeric call of the plan, so they must stay unchanged (and alive) until the
 * last numeric call has completed. The flops and nnz_ub of sg_sym_info stay
 * those of the unmasked product. Errors: as sg_spgemm_symbolic, and
 * INVALID_ARG for a stride below ceil(minor / 32).
 */
sg_status sg_spgemm_symbolic_masked(const sg_semiring *sr, int32_t nprod,
                                    const sg_mat *A, const sg_mat *B,
                                    const int32_t *group, int32_t ngroup,
                                    int32_t out_fmt, const sg_mask *masks,
                                    const sg_tuning *tuning, void *ws,
                                    size_t ws_bytes, sg_plan **plan,
                                    sg_sym_info *info, void *stream);

/*
 * Fused chain products C_p = X_p Y_p Z_p for p in [0, nprod) (host arrays of
 * descriptors of device data, all CSR or all CSC, plain compressed), each
 * into its own output C_p (format out_fmt, the operands' orientation). The
 * intermediate product is never written to memory: for every output vector
 * (a column of C column-major, a row row-major) one wavefront or one
 * workgroup forms that vector of the inner product (Y Z(:, j), or X(i, :) Y)
 * in registers or LDS, merges it, and immediately multiplies the outer
 * operand by it (the triple products of multigrid setup, R A P, which the
 * paper's Section 8 names as the next step). The result equals the two-call
 * product X (Y Z), column-major, or (X Y) Z, row-major: the intermediate
 * vector is merged before the second stage exactly as the two calls would
 * write it.
 *
 * The plan is a normal sg_plan: sg_spgemm_numeric / sg_spgemm_batched
 * recompute every C_p from the current operand VALUES (the structure must
 * stay the same), so the symbolic phase of a setup is reused across repeated
 * setups with new values, and the numeric phase can be captured in a graph.
 * sg_sym_info per product: flops counts the multiplications of both stages,
 * nnz_ub the sum over output vectors of min(unmerged fused multiplications,
 * minor dimension). Errors: as sg_spgemm_symbolic; UNSUPPORTED for doubly
 * compressed operands, and for an output vector whose intermediate or result
 * exceeds the LDS-resident tier (the message gives the limit).
 */
sg_status sg_chain_workspace_size(const sg_semiring *sr, int32_t nprod, const sg_mat *X, const sg_mat *Y,
                                  const sg_mat *Z, int32_t out_fmt, const sg_tuning *tuning, size_t *ws_bytes);
sg_status sg_chain_symbolic(const sg_semiring *sr, int32_t nprod, const sg_mat *X, const sg_mat *Y, const sg_mat *Z,
                            int32_t out_fmt, const sg_tuning *tuning, void *ws, size_t ws_bytes, sg_plan **plan,
                            sg_sym_info *info, void *stream);

/*
 * Mask update (a BFS's "visited |= new frontier"): for each of the n
 * matrices M[k] (host array of descriptors of device data) sets bit (i, j) of
 * masks[k] for every stored entry i of M[k]'s vector j, with atomic ORs on
 * the device. One launch per 16 matrices; asynchronous.
 */
sg_status sg_mask_set(int32_t n, const sg_mat *M, const sg_mask *masks, void *stream);

/*
 * Numeric phase: writes every C_g (host array C[ngroup] of descriptors of
 * caller-allocated device arrays with capacities >= info[g].nnz / .nvec).
 * Stream-ordered and asynchronous, with one kernel launch per tier. Output
 * is canonical (ids ascending inside each vector; doubly compressed output
 * elides empty vectors). Errors: INVALID_ARG, CAPACITY, HIP.
 */
sg_status sg_spgemm_numeric(sg_plan *plan, sg_mat_out *C, void *stream);

/*
 * Batched numeric phase: the same result as sg_spgemm_numeric, computed by
 * ONE persistent launch whose workgroups pull (output vector, tier) work
 * items of every product and group from a device queue, heaviest first. It
 * records no memset, no copy and no host synchronisation, so it can be
 * captured in a hipGraph and replayed; a replay recomputes C (the output
 * arrays given at capture) from the current operand values. Calls on one
 * plan share its workspace and must be ordered on one stream. Errors: as
 * sg_spgemm_numeric.
 */
sg_status sg_spgemm_batched(sg_plan *plan, sg_mat_out *C, void *stream);

/*
 * Kernel timing for measurement. With enable = 1, the following
 * sg_spgemm_numeric / sg_spgemm_batched calls on this plan record HIP events
 * on their stream around every kernel launch (do not enable it for a call
 * that is being captured into a graph). sg_plan_kernel_times waits for the
 * events of the last such call and writes up to n durations in milliseconds:
 * out_ms[0] heavy tier (or the whole persistent launch of a batched call),
 * out_ms[1] mid tier, out_ms[2] tiny tier, out_ms[3] output pointers.
 * A launch that did not run reports 0.
 */
sg_status sg_plan_profile(sg_plan *plan, int32_t enable);
sg_status sg_plan_kernel_times(sg_plan *plan, double *out_ms, int32_t n);

/*
 * Release a plan. Host memory only: it frees the handle and makes no HIP
 * call that waits for the device (kernel-timing events, if any were made,
 * are destroyed), so it may be called while launches of the plan are still
 * in flight. The workspace and the operand and output arrays stay the
 * caller's, and must stay alive until those launches have completed.
 */
sg_status sg_plan_destroy(sg_plan *plan);

/*
 * Invariant counters of the checking build (the library compiled with
 * SG_CHECK=1; sg_build_checked() returns 1 there and 0 in the normal
 * build). Waits for the whole device, then writes up to n counters summed
 * over every launch made with the plan so far: out[0] the work items after
 * which a workgroup's LDS was not back to all-zero bits, out[1] the output
 * vectors or heavy windows whose numeric phase wrote a different number of
 * entries than the symbolic phase counted. Both are zero in a correct run,
 * and always zero in the normal build, which compiles no checks.
 */
sg_status sg_plan_check(sg_plan *plan, int64_t *out, int32_t n);
int32_t sg_build_checked(void);

/*
 * Check that one operand is canonical (see the conventions above) on the
 * device. `ws` needs 64 bytes of device memory. Synchronises the stream.
 * Returns SG_OK or SG_ERR_NOT_CANONICAL.
 */
sg_status sg_validate(const sg_mat *M, void *ws, void *stream);

/*
 * Build the AUX column index of a doubly compressed matrix (Section 2.3):
 * with chunk = ceil(major_dim / nvec) columns, aux[c] is the position in vid
 * of the first stored vector whose id is >= c * chunk, for c in
 * [0, nchunks), and aux[nchunks] = nvec, where nchunks = ceil(major_dim /
 * chunk). `aux` is a device array of nchunks + 1 entries; *nchunks_out
 * (host) receives nchunks. Asynchronous.
 */
sg_status sg_build_aux(const sg_mat *M, int32_t *aux, int64_t *nchunks_out, void *stream);

/*
 * Format utilities on the device (Sections 2.2 and 2.3 define CSR/CSC and the
 * doubly compressed DCSC/DCSR; Section 2.4 transposes an operand so that a
 * row-major product runs column-wise).
 *
 * Triples -> compressed, in two calls that share `ws` (caller-owned device
 * memory of sg_coo_workspace_size bytes; keep it and the triples unchanged
 * between the calls):
 *   sg_coo_compress  sorts the nnz triples (rows[i], cols[i], vals[i]) of an
 *                    nrows x ncols matrix (device arrays; vals NULL for
 *                    SG_OR_AND_BOOL) by (major, minor) of `fmt` with a stable
 *                    radix sort, finds the distinct positions and returns, on
 *                    the host after one stream synchronisation, *nnz_out
 *                    (distinct positions) and *nvec_out (stored vectors of
 *                    `fmt`: the major dimension for CSR/CSC, the non-empty
 *                    vectors for DCSR/DCSC). INVALID_ARG if a triple lies
 *                    outside the matrix.
 *   sg_coo_emit      writes the canonical matrix into `out` (capacities at
 *                    least nnz_out and, doubly compressed, nvec_out; pass the
 *                    values sg_coo_compress returned). A position given
 *                    several times is stored once, with its values combined
 *                    by the semiring's add in list order (a left fold:
 *                    ((v1 + v2) + v3) + ...; min for (min,+), or for bool).
 *                    Asynchronous.
 */
sg_status sg_coo_workspace_size(const sg_semiring *sr, int64_t nrows, int64_t ncols, int64_t nnz, int32_t fmt,
                                size_t *ws_bytes);
sg_status sg_coo_compress(const sg_semiring *sr, int64_t nrows, int64_t ncols, int64_t nnz, const int32_t *rows,
                          const int32_t *cols, const void *vals, int32_t fmt, void *ws, size_t ws_bytes,
                          int64_t *nnz_out, int64_t *nvec_out, void *stream);
sg_status sg_coo_emit(const sg_semiring *sr, int64_t nrows, int64_t ncols, int64_t nnz, int32_t fmt, void *ws,
                      size_t ws_bytes, int64_t nnz_out, int64_t nvec_out, sg_mat_out *out, void *stream);

/*
 * Format change of a canonical matrix M into `fmt` (any of the four, same
 * matrix), written to `out` (capacity: M->nnz entries; doubly compressed
 * output at least the number of non-empty vectors, e.g. min(nnz, major
 * dimension)). Between orientations this is the transpose of the storage
 * (CSC of M holds the arrays of CSR of M^T), by a stable sort on the minor
 * ids, so every new vector comes out with ascending ids. `ws`: device memory
 * of sg_convert_workspace_size bytes. *nvec_out (host, may be NULL) receives
 * the stored vectors of the output; a doubly compressed output needs one
 * stream synchronisation to learn it, otherwise the call is asynchronous.
 * CAPACITY if `out` is too small.
 */
sg_status sg_convert_workspace_size(const sg_semiring *sr, const sg_mat *M, int32_t fmt, size_t *ws_bytes);
sg_status sg_convert(const sg_semiring *sr, const sg_mat *M, int32_t fmt, void *ws, size_t ws_bytes, sg_mat_out *out,
                     int64_t *nvec_out, void *stream);

/*
 * sg_convert for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * the same format change and the same results, with the workspace taken
 * from a fixed device array of this library instead of a caller buffer
 * (sg_convert_static_bytes() bytes, 64 MiB, one array per GPU, held until
 * the process ends; its device address is looked up once per GPU). The call
 * allocates nothing. A matrix whose workspace (sg_convert_workspace_size)
 * exceeds the array is refused with SG_ERR_WORKSPACE and a message in
 * sg_last_error. All calls on one GPU share the array: calls that overlap on
 * one GPU (other streams or threads) race and must be serialised by the
 * caller. Arguments and the other errors as sg_convert.
 */
sg_status sg_convert_static(const sg_semiring *sr, const sg_mat *M, int32_t fmt, sg_mat_out *out,
                            int64_t *nvec_out, void *stream);
size_t sg_convert_static_bytes(void);

#ifdef __cplusplus
}
#endif

#endif /* SG_SPGEMM_H */
