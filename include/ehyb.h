/*
 * ehyb.h - C ABI of the EHYB (explicit-caching hybrid) sparse matrix-vector
 * product for AMD Instinct MI355X (gfx950).
 *
 * Operation (Introduction): y = A x, A a square sparse matrix, x and y dense
 * vectors.  The method (Section 3) prepares A once on the host:
 *   - A is read as an undirected graph whose vertices are the row/column
 *     indices and whose edges are the stored entries (Section 3.1);
 *   - the graph is cut into partitions small enough that each partition's
 *     slice of x fits the on-chip cache of one workgroup (Section 3.3, Eq. 1-2);
 *   - rows are renumbered partition by partition, and inside a partition by
 *     non-increasing count of in-partition entries (Section 3.2, Alg. 1);
 *   - in-partition entries are stored in a sliced-ELL part whose column
 *     indices are 16-bit offsets into the partition's x-slice (Section 3.4);
 *     all other entries go to the residual "extra rows" part with 32-bit
 *     columns (Section 3.2, Alg. 2);
 * and the device kernel (Section 4.2, Alg. 3) stages each x-slice in LDS,
 * sweeps the ELL part against it and adds the residual part read against x
 * in device memory.
 *
 * Conventions for every function below:
 *   - Returns EHYB_OK or a negative ehyb_status; never aborts, never lets a
 *     C++ exception escape.  On failure a message is available from
 *     ehyb_last_error() (thread-local, valid until the next call on the same
 *     thread) and outputs are left unspecified.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *     device allocations on the current device.  The library never allocates
 *     device memory: the caller provides every device buffer.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Device work is enqueued on it and the call returns without waiting,
 *     except where stated.
 *   - Vectors are contiguous, dtype as stated (x, y FP64 for FP64 plans),
 *     each under 4 GiB (the kernels address them with 32-bit byte offsets;
 *     larger ones give EHYB_EUNSUPPORTED).
 *     x and y must not overlap.  x is assumed finite: padding slots multiply
 *     +0.0 by an x element, so an Inf or NaN in x may leak into rows that do
 *     not reference it.
 */
#ifndef EHYB_H
#define EHYB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EHYB_API __attribute__((visibility("default")))

typedef enum {
    EHYB_OK = 0,
    EHYB_EINVAL = -1,        /* malformed argument or input matrix */
    EHYB_ENOMEM = -2,        /* host allocation failed */
    EHYB_EUNSUPPORTED = -3,  /* valid but outside what the format supports */
    EHYB_EDEVICE = -4,       /* a HIP call or kernel launch failed */
    EHYB_ESTATE = -5         /* call out of order (e.g. spmv before upload) */
} ehyb_status;

/* Value type of a plan.  EHYB_F64: FP64 values, FP64 x/y/accumulation.
 * EHYB_F32 / EHYB_BF16: binary32 / bfloat16 values (rounded to nearest even
 * from the FP64 input), binary32 x and y, binary32 accumulation.
 * EHYB_F32_ACC64 / EHYB_BF16_ACC64: the same values and x, binary64
 * accumulation (each product and sum in FP64, y rounded to binary32 once):
 * for long rows, where binary32 accumulation error grows with the row
 * length.  Their residual accumulators take 8 bytes of LDS per row. */
typedef enum { EHYB_F64 = 0, EHYB_F32 = 1, EHYB_BF16 = 2, EHYB_F32_ACC64 = 3, EHYB_BF16_ACC64 = 4 } ehyb_dtype;

/* Which partitioner builds the partitions (Section 3.1 asks for a graph
 * partitioner minimising the entries that fall outside their row's
 * partition). */
typedef enum {
    EHYB_PART_MULTILEVEL = 0, /* multilevel graph partitioner (default) */
    EHYB_PART_NATURAL = 1     /* consecutive blocks of the given row order */
} ehyb_partitioner;

/* How the kernels load the value and column arrays, which every product reads
 * once: AUTO = non-temporal (streaming) loads when the product's bytes exceed
 * 384 MiB (1.5x the 256 MB Infinity Cache), plain loads otherwise, so that
 * repeated products of a smaller plan can hit that cache. */
typedef enum {
    EHYB_LOAD_AUTO = 0,
    EHYB_LOAD_CACHED = 1,
    EHYB_LOAD_STREAM = 2
} ehyb_load_mode;

/* Input matrix in canonical CSR (host memory, borrowed for the call).
 * n_rows == n_cols (the graph reading of Section 3.1 needs a square matrix:
 * otherwise EHYB_EUNSUPPORTED).  row_ptr[0] == 0, row_ptr non-decreasing,
 * row_ptr[n_rows] == nnz, columns strictly increasing within a row and in
 * [0, n_cols) (otherwise EHYB_EINVAL).  Explicit zeros are kept bit for bit. */
typedef struct {
    int64_t n_rows, n_cols, nnz;
    const int64_t *row_ptr;  /* [n_rows + 1] */
    const int32_t *col_idx;  /* [nnz] */
    const double *val;       /* [nnz] */
} ehyb_csr_host;

/* Preprocessing parameters; a zero field takes the stated default. */
typedef struct {
    int32_t slice_rows;     /* target rows per partition (x-slice length).
                               0 = Eq. 1-2: smallest K with n*tau/(K*P) < lds_bytes,
                               VecSize = ceil(n/(K*P)), floored at min(n, 512).
                               At most lds_bytes/tau and 65536 rows. */
    int32_t ell_width_cap;  /* max ELL entries per row: > 0 as given; -1 =
                               unlimited (the paper's split by partition
                               only); 0 = automatic, 128 load steps per lane
                               group (128 * lanes per row * kc entries), which
                               only hub rows reach: their excess entries go
                               to the residual part, where they run on wide
                               slices */
    int32_t rows_per_wave;  /* rows per 64-lane wavefront row-slice, a power of
                               two in [1, 64]; 64/rows_per_wave lanes share a
                               row. 0 = 64 (one lane per row) */
    int32_t value_dtype;    /* ehyb_dtype; 0 = EHYB_F64 */
    int32_t lds_bytes;      /* LDS budget per workgroup; 0 = 160 KiB.  It
                               holds the x-slice, the halo and one residual
                               accumulator per row; Eq. 1 reserves two
                               elements per row (tau = 2 * bytes of an x
                               element) */
    int32_t num_cus;        /* P in Eq. 1; 0 = 256 */
    int32_t n_threads;      /* host threads; 0 = all available */
    int32_t imbalance_pct;  /* allowed overfill of a partition above
                               slice_rows, percent; 0 = 3 */
    int32_t partitioner;    /* ehyb_partitioner; 0 = multilevel */
    int32_t halo_rows;      /* neighbour x entries cached per partition in LDS
                               next to its x-slice (the "halo"): 0 = as many
                               as the LDS budget leaves, > 0 = at most that
                               many, -1 = none, so that every entry outside the
                               partition goes to the residual part (the
                               paper's split) */
    int32_t n_rhs;          /* right-hand sides the plan is sized for: the LDS
                               budget holds n_rhs x elements per row (tau of
                               Eq. 1 grows n_rhs-fold); 0 = 1.  A plan for
                               n_rhs > 1 also runs ehyb_spmv; ehyb_spmm_batched
                               needs plans built for its n_rhs */
    int32_t reserved;       /* must be 0 */
    uint64_t seed;          /* partitioner seed (deterministic for a seed) */
} ehyb_params;

typedef struct {
    int64_t n, nnz;           /* matrix size and stored entries */
    int64_t nnz_ell, nnz_er;  /* entries in the ELL part / residual part */
    int64_t ell_slots;        /* ELL slots including padding */
    int64_t er_slots;         /* residual slots including padding */
    int64_t n_er_rows;        /* rows with at least one residual entry */
    int64_t nnz_halo;         /* ELL entries whose column is in the halo */
    int64_t n_halo;           /* halo entries, all partitions */
    int64_t device_bytes;     /* size of the device blob for ehyb_plan_upload */
    int64_t algorithmic_bytes;/* bytes one permuted-space SpMV must move, each
                                 array element once: ELL and residual slots
                                 (values + columns, padding included), slice
                                 metadata and residual row indices, partition
                                 bounds, x once, y once.  The residual part's
                                 x gathers re-read x and are not counted. */
    int32_t nparts;           /* partitions (one workgroup each) */
    int32_t nslices;          /* ELL row-slices */
    int32_t ner_slices;       /* residual row-slices */
    int32_t slice_rows;       /* target rows per partition actually used */
    int32_t max_part_rows;    /* largest partition */
    int32_t rows_per_slice;   /* C = rows_per_wave */
    int32_t lanes_per_row;    /* L = 64 / C */
    int32_t kc;               /* ELL entries per lane per full load step */
    int32_t value_dtype;      /* ehyb_dtype */
    int32_t eq1_K;            /* K of Eq. 1 for this n (informational) */
    int32_t max_halo;         /* largest halo of one partition */
    int32_t lds_bytes_used;   /* LDS one workgroup of ehyb_spmv uses */
    int32_t n_rhs;            /* right-hand sides the plan is sized for */
    int32_t n_er_wide;        /* wide residual slices (one long row, 64 lanes) */
    int32_t ell_width_cap;    /* ELL width cap in effect, 0 = none */
    int32_t n_er_pieces;      /* pieces of at most 8 steps the wide residual
                                 slices are summed in by ehyb_spmv and
                                 ehyb_spmm_batched (0 = no wide slices) */
    double t_graph_s, t_partition_s, t_reorder_s, t_encode_s; /* host times */
} ehyb_plan_stats;

/* Read-only views of a plan's host arrays (owned by the plan, valid until
 * ehyb_plan_destroy).
 *
 * Rows: partition p owns permuted rows [part_start[p], part_start[p+1]);
 * inside it rows are in non-increasing ELL count.
 *
 * ELL part: partition p's rows are cut into row-slices of C = 64/L rows,
 * slices [slice_start[p], slice_start[p+1]).  They are stored in the order a
 * workgroup takes them: first the ell_free[p] slices none of whose rows has
 * residual entries, then the others, each group by ascending row.  Their slot
 * ranges are placed round by round: queue positions 0..15 of every partition
 * in partition order, then positions 16..31, and so on (any placement is
 * valid; only the offsets say where a slice is).
 * ell_meta[4s..4s+3] = slot offset; width W, the entries each lane loads
 * (low 16 bits), and the slice's index j within its partition (high 16 bits:
 * row r of the slice is local row j*C + r); a 64-bit mask (low word, high
 * word) whose bit r says that row r also has residual entries.  A slice of
 * width W holds 64*W slots: W / KC steps of KC entries per lane, then
 * W % KC single-entry steps, so a row of m ELL entries needs
 * W = (m / (L*KC))*KC + ceil((m mod L*KC) / L), with no padding beyond the
 * slice's longest row.  Columns are 16-bit indices into the
 * partition's LDS vector: c < size of the partition is x-slice element c
 * (permuted row part_start[p] + c); c >= size is halo element
 * halo_idx[halo_start[p] + c - size].
 *
 * Halo: partition p caches the x entries halo_idx[halo_start[p] ..
 * halo_start[p+1]) (permuted global indices, ascending, none inside the
 * partition): entries of the partition's rows whose column is there are
 * stored in the ELL part, the rest of the out-of-partition entries in the
 * residual part.
 *
 * Residual part: the rows of partition p with residual entries, sorted by
 * non-increasing residual count (ties by local row), slices
 * [er_slice_start[p], er_slice_start[p+1]).  When C > 1, each row with more
 * than 32*L residual entries (they come first) has a "wide" slice of its
 * own, processed by all 64 lanes; the other rows are cut into row-slices of
 * C rows.  er_row[e*C + r] is the local row of row r of residual slice e
 * (0xFFFF past the last row; a wide slice names its row at r = 0).
 * er_meta[2e..2e+1] = slot offset, step count (bit 31 set for a wide slice).
 * Columns are permuted global indices.
 *
 * Slots: entry k (ascending permuted column) of row r of a slice with slot
 * offset `off` and F full steps lives, for k < F*L*KC, at
 *   t = k / (L*KC), u = (k / KC) % L, c = k % KC, lane = r*L + u,
 *   slot = off + (t*64 + lane)*KC + c,
 * and otherwise, with k' = k - F*L*KC, in single-entry step t' = k' / L at
 *   slot = off + F*64*KC + t'*64 + r*L + k' % L.
 * In the ELL part KC = kc and F = W / kc; in the residual part KC = 1 and F
 * is the step count; in a wide residual slice, L = 64 and r = 0 (entry k at
 * off + k).  Padding slots hold +0.0 and column 0. */
typedef struct {
    int64_t n;
    int32_t nparts, nslices, ner_slices, lanes_per_row, kc, value_dtype;
    int64_t ell_slots, er_slots, n_halo;
    const int32_t *perm;           /* [n] new index -> original index */
    const int32_t *part_start;     /* [nparts + 1] */
    const int32_t *slice_start;    /* [nparts + 1] first ELL slice of each partition */
    const int32_t *er_slice_start; /* [nparts + 1] first residual slice of each partition */
    const int32_t *ell_free;       /* [nparts] leading ELL slices without residual rows */
    const int32_t *halo_start;     /* [nparts + 1] */
    const int32_t *halo_idx;       /* [n_halo] */
    const uint32_t *ell_meta;      /* [4 * nslices] */
    const uint32_t *er_meta;       /* [2 * ner_slices] */
    const uint16_t *er_row;        /* [C * ner_slices] */
    const void *ell_val;           /* [ell_slots] values, value_dtype */
    const uint16_t *ell_col;       /* [ell_slots] local columns */
    const void *er_val;            /* [er_slots] values, value_dtype */
    const int32_t *er_col;         /* [er_slots] permuted global columns */
    const int32_t *row_ell_len;    /* [n] ELL entries of each permuted row */
    const int32_t *row_er_len;     /* [n] residual entries of each permuted row */
} ehyb_plan_arrays;

typedef struct ehyb_plan ehyb_plan;

/* Flags of ehyb_spmv. */
#define EHYB_VEC_PERMUTED 1u  /* x and y are in the plan's permuted order
                                 (x_perm[i] = x[perm[i]]); otherwise they are in
                                 the original order and the library permutes
                                 through scratch space inside the device blob */

/* Host preprocessing (Alg. 1 and Alg. 2): validate A, build its graph,
 * partition it, reorder rows, and encode both parts.  Host only; `A` is
 * borrowed for the call.  On success *out owns a new plan. */
EHYB_API ehyb_status ehyb_preprocess(const ehyb_csr_host *A, const ehyb_params *params,
                            ehyb_plan **out);

/* Statistics of a plan, all in one struct (sizes, part sizes, bytes per
 * product, preprocessing time by phase), filled by one call. */
EHYB_API ehyb_status ehyb_plan_stats_get(const ehyb_plan *plan, ehyb_plan_stats *out);

/* Views of a plan's host arrays (see ehyb_plan_arrays), valid while the
 * plan lives.  The row permutation is one of them (`perm`: row i of the plan
 * is row perm[i] of A); there is no separate call for it. */
EHYB_API ehyb_status ehyb_plan_arrays_get(const ehyb_plan *plan, ehyb_plan_arrays *out);

/* Decode the plan back to CSR of P A P^T (B[i][j] = A[perm[i]][perm[j]]),
 * columns ascending, values converted exactly to FP64 (bit-identical to A's
 * for FP64 plans).  Host buffers of n+1, nnz and nnz elements. */
EHYB_API ehyb_status ehyb_plan_decode_csr(const ehyb_plan *plan, int64_t *row_ptr, int32_t *col_idx,
                                 double *val);

/* Bytes of device memory the plan needs (metadata, both parts, permutation,
 * two n-vectors of scratch for unpermuted calls and, when the plan has wide
 * residual slices, their piece list and one 8-byte partial sum per piece),
 * 256-byte aligned. */
EHYB_API ehyb_status ehyb_plan_device_bytes(const ehyb_plan *plan, size_t *bytes);

/* Copy the plan into `dev_blob` (device, at least device_bytes bytes,
 * 256-byte aligned; owned by the caller, who keeps it alive and unmodified
 * while any launch on it may run).  Waits for the copies to finish before
 * returning.  Rebinding to another blob is allowed. */
EHYB_API ehyb_status ehyb_plan_upload(ehyb_plan *plan, void *dev_blob, size_t bytes, void *stream);

/* y = A x on the device (Alg. 3).  x, y: device FP64 vectors of length n for
 * FP64 plans.  With EHYB_VEC_PERMUTED they are in permuted order; otherwise in
 * the original order.  A plan with wide residual slices (hub rows, see
 * n_er_pieces) first sums them in pieces over the whole device (the global
 * residual queue of Alg. 3, for these rows only), one more launch on the same
 * stream; each partition then adds its rows' pieces in a fixed order.
 * Launches on one plan blob must not overlap in time when the unpermuted mode
 * is used or the plan has wide residual slices (they share its scratch).
 * Every row of y is overwritten; the result is bitwise deterministic. */
EHYB_API ehyb_status ehyb_spmv(const ehyb_plan *plan, const void *x, void *y, uint32_t flags,
                      void *stream);

/* Launch shape of ehyb_spmv: wavefronts per workgroup (one workgroup per
 * partition), one of 4, 8, 16; 0 = the library's choice.  Applies to later
 * ehyb_spmv calls on this plan; does not change results (each row is summed by
 * one fixed lane group in one fixed order whatever the shape). */
EHYB_API ehyb_status ehyb_plan_set_launch(ehyb_plan *plan, int32_t waves_per_wg);
/* Load mode (ehyb_load_mode) of ehyb_spmv for this plan; results are unchanged. */
EHYB_API ehyb_status ehyb_plan_set_load_mode(ehyb_plan *plan, int32_t mode);

/* x_perm[i] = x[perm[i]] and y[perm[i]] = y_perm[i] on the device (the
 * reordering applied to vectors; FP64 for FP64 plans). */
EHYB_API ehyb_status ehyb_permute_x(const ehyb_plan *plan, const void *x, void *x_perm, void *stream);
EHYB_API ehyb_status ehyb_unpermute_y(const ehyb_plan *plan, const void *y_perm, void *y, void *stream);

/* ---- Batched products (several matrices, several right-hand sides) ----
 *
 * A batch groups uploaded plans of one value type, one rows_per_wave and one
 * n_rhs.  ehyb_spmm_batched computes Y_i = A_i X_i for every matrix i in one
 * persistent kernel launch: workgroups take (matrix, partition) items from
 * queues in the batch's device blob (the global queue of Alg. 3, spread over
 * matrices): the items, by matrix and then partition, are cut into eight runs
 * of about equal bytes, one per XCD, so that neighbouring partitions, which
 * share halo rows of x, run on one XCD's L2; a workgroup whose run is empty
 * takes items from the other runs.  The last workgroup to finish resets the
 * queues, so the launch can be recorded in a HIP graph and replayed.  When
 * plans of the batch have wide residual slices (hub rows, see n_er_pieces),
 * one launch before the product sums the pieces of all of them, n_rhs sums
 * per piece, into the batch's blob, as ehyb_spmv does for one plan; the
 * partitions then add their rows' pieces in a fixed order, so results are
 * bitwise deterministic, and with n_rhs == 1 equal to ehyb_spmv's.  X_i and
 * Y_i are row-major [n_i][n_rhs] in plan i's permuted order (flag
 * EHYB_VEC_PERMUTED required), element type as for ehyb_spmv. */
typedef struct ehyb_batch ehyb_batch;

#define EHYB_BATCH_MAX 128   /* matrices per batch */

/* Group `n_plans` plans (host pointers, borrowed: they must outlive the batch
 * and stay uploaded to the same blobs).  Every plan must have the same value
 * type, rows_per_wave and n_rhs == `n_rhs` (1, 2, 4 or 8). */
EHYB_API ehyb_status ehyb_batch_create(const ehyb_plan *const *plans, int32_t n_plans, int32_t n_rhs,
                                      ehyb_batch **out);
/* Device bytes of the batch descriptor (per-matrix array pointers, work
 * items, queue counters, the piece list and the pieces' sums). */
EHYB_API ehyb_status ehyb_batch_device_bytes(const ehyb_batch *batch, size_t *bytes);
/* Copy the batch descriptor into `dev_blob` (device, caller-owned, 256-byte
 * aligned); the plans must be uploaded first.  Waits for the copy. */
EHYB_API ehyb_status ehyb_batch_upload(ehyb_batch *batch, void *dev_blob, size_t bytes, void *stream);
/* Y_i = A_i X_i for all matrices of the batch, one kernel launch on `stream`.
 * X, Y: host arrays of n_plans device pointers.  Launches on one batch blob
 * must not overlap in time (they share its queue counters and piece sums);
 * a batch with wide residual slices makes two launches on `stream`. */
EHYB_API ehyb_status ehyb_spmm_batched(const ehyb_batch *batch, int32_t n_rhs, const void *const *X,
                                      void *const *Y, uint32_t flags, void *stream);
/* Load mode (ehyb_load_mode) of ehyb_spmm_batched, judged on the batch's
 * total bytes; results are unchanged. */
EHYB_API ehyb_status ehyb_batch_set_load_mode(ehyb_batch *batch, int32_t mode);
EHYB_API void ehyb_batch_destroy(ehyb_batch *batch);

/* Preprocessing with the caller's partition instead of the built-in
 * partitioner (Section 3.1 leaves the partitioner open; the paper uses
 * METIS).  part: host int32 [n_rows], the partition id of each row (and of
 * its column vertex), in [0, n_parts).  Empty ids are dropped and the rest
 * keep their order; every partition must fit the LDS budget of `params`
 * (at most (lds_bytes - 64) / (2 * x bytes * n_rhs) and 65535 rows), else
 * EHYB_EINVAL.  params->slice_rows and params->partitioner are ignored; the
 * plan reports the largest partition as its slice_rows.  A plan from the
 * same partition and other ell_width_cap / rows_per_wave / value_dtype /
 * halo_rows is re-encoded without re-partitioning (the partition vector of a
 * plan follows from its perm and part_start arrays). */
EHYB_API ehyb_status ehyb_preprocess_partitioned(const ehyb_csr_host *A, const ehyb_params *params,
                                                const int32_t *part, int32_t n_parts, ehyb_plan **out);

/* 32 sparsity features of A (square, canonical CSR as for ehyb_preprocess;
 * values unused), the input of the learned parameter predictor, written to
 * out[32] as float.  Row lengths r_i, mean m, population std s; quantiles
 * are lower quantiles r_(floor(q (n-1))) of the sorted lengths:
 *  0 log2 n            1 log2(nnz+1)        2 m          3 s
 *  4 s/m (0 if m = 0)  5 min r              6 max r      7 log2(max r + 1)
 *  8-13 quantiles of r at 0.10 0.25 0.50 0.75 0.90 0.99
 * 14 skewness E[(r-m)^3]/s^3 (0 if s = 0)   15 share of empty rows
 * 16 share of rows with r > 2m
 * 17 mean |i-j| / n over entries            18 max |i-j| / n
 * 19 0.90-quantile of the row bandwidth max_j |i-j| (0 for empty rows), / n
 * 20 share of entries with |i-j| < 4096
 * 21 mean over rows of the distinct 4096-column blocks touched
 * 22 / 23 mean / max over 4096-row blocks of (distinct column blocks touched
 *         / number of column blocks)
 * 24 share of off-diagonal entries (i,j) with (j,i) stored (1 if none)
 * 25 share of rows with a stored diagonal
 * 26 Gini coefficient of r: sum_k (2k - n - 1) r_(k) / (n nnz), k = 1..n
 * 27 share of entries in the ceil(n/100) longest rows
 * 28 m / 64
 * 29 ELL padding at width w = feature 13: sum_i (w - min(r_i, w)) / nnz
 * 30 entries beyond width w: sum_i max(r_i - w, 0) / nnz
 * 31 share of entries with i/512 == j/512
 * (ratios over nnz use max(nnz, 1)).  n_threads: 0 = all. */
EHYB_API ehyb_status ehyb_features(const ehyb_csr_host *A, int32_t n_threads, float *out);

/* Learned parameter predictor: a fully connected network, binary32,
 *   h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = W3 h2 + b3,
 * x: EHYB_MLP_IN features, hidden layers of EHYB_MLP_HIDDEN, y:
 * EHYB_MLP_OUT outputs.  The paper picks the partition size by Eq. 1 and
 * cites learned format selection as related work only; this network
 * predicts (partition size, ELL width, rows per wave) from ehyb_features.
 * params (device, EHYB_MLP_PARAMS floats): W1 [64][32] row-major, b1 [64],
 * W2 [64][64], b2 [64], W3 [3][64], b3 [3].  X: device [batch][32],
 * Y, T: device [batch][3], row-major.  All calls are asynchronous on
 * `stream`; results are bitwise reproducible for a batch size. */
#define EHYB_MLP_IN 32
#define EHYB_MLP_HIDDEN 64
#define EHYB_MLP_OUT 3
#define EHYB_MLP_PARAMS 6467
EHYB_API ehyb_status ehyb_mlp_forward(const float *params, int32_t batch, const float *X, float *Y,
                                      void *stream);
/* Device workspace that ehyb_mlp_grad needs for `batch` samples. */
EHYB_API ehyb_status ehyb_mlp_workspace_bytes(int32_t batch, size_t *bytes);
/* Mean squared error L = sum_{b,o} (y_bo - t_bo)^2 / (batch * 3) and its
 * gradient: grad (device, EHYB_MLP_PARAMS floats, parameter layout) = dL/dparams,
 * *loss (device float, may be NULL) = L.  The ReLU derivative at 0 is 0.
 * workspace: device, >= ehyb_mlp_workspace_bytes(batch), caller-owned. */
EHYB_API ehyb_status ehyb_mlp_grad(const float *params, int32_t batch, const float *X, const float *T,
                                   float *grad, float *loss, void *workspace, size_t workspace_bytes,
                                   void *stream);
/* ehyb_mlp_grad for callers that cannot allocate device memory (code under
 * HIP graph capture, tight training or serving loops, harnesses that forbid
 * hipMalloc): the same computation and results, bit for bit, with the
 * workspace taken from a static device array of the library instead of the
 * caller (256 partial-sum rows of EHYB_MLP_PARAMS + 1 floats: 6.3 MiB on each
 * device it runs on, held until the process ends, enough for any batch; a
 * call that would need more gives EHYB_EUNSUPPORTED).  Calls no allocating
 * routine.  Every call on a device shares that array: calls that overlap in
 * time on one device (other streams, other host threads) race and must not
 * be issued; calls ordered on one stream are safe.  The array's address is
 * looked up on the first call on each device (with that device current). */
EHYB_API ehyb_status ehyb_mlp_grad_noalloc(const float *params, int32_t batch, const float *X, const float *T,
                                           float *grad, float *loss, void *stream);
/* One Adam step (Kingma and Ba) in place: m, v (device, EHYB_MLP_PARAMS,
 * zero before step 1) are the moment estimates, step >= 1 counts updates,
 * bias corrections 1/(1 - beta^step) computed on the host in FP64. */
EHYB_API ehyb_status ehyb_mlp_adam(float *params, const float *grad, float *m, float *v, int32_t step,
                                   float lr, float beta1, float beta2, float eps, void *stream);

/* Save / load a plan (host arrays only) as a versioned binary file with a
 * checksum; a loaded plan must be uploaded before use.  A corrupted or
 * truncated file gives EHYB_EINVAL. */
EHYB_API ehyb_status ehyb_plan_save(const ehyb_plan *plan, const char *path);
EHYB_API ehyb_status ehyb_plan_load(const char *path, ehyb_plan **out);

EHYB_API void ehyb_plan_destroy(ehyb_plan *plan);

/* Baseline: plain CSR y = A x on the device, FP64 (CSR-vector): one group of
 * `lanes_per_row` lanes (power of two in [1, 64]; 0 = the fewest whose first
 * batch of 4 entries per lane covers a row of mean length) per row, each lane
 * loading 4 entries per batch before using any; a wavefront holding a row of
 * more than 1024 entries sums its rows one at a time on all 64 lanes.
 * row_ptr int32 [n_rows+1], col int32 [nnz], val [nnz], x, y device;
 * n_rows and nnz below 2^29 (else EHYB_EUNSUPPORTED).  Each row's sum is a
 * fixed function of lanes_per_row.  The comparator of the method (CSR
 * lineage, Section 2.2). */
EHYB_API ehyb_status ehyb_csr_spmv_f64(int64_t n_rows, int64_t nnz, const int32_t *row_ptr,
                              const int32_t *col_idx, const double *val, const double *x,
                              double *y, int32_t lanes_per_row, void *stream);

/* Bandwidth probes (the denominators of the HBM fraction).  read: streams
 * `bytes` (multiple of 16) from `buf` with 16-byte loads and writes one
 * 8-byte partial per workgroup to `sink` (device, >= 8 * 65536 bytes).
 * copy: copies `bytes` (multiple of 16) from src to dst. */
EHYB_API ehyb_status ehyb_probe_read(const void *buf, size_t bytes, void *sink, void *stream);
/* Cache flush for cold timings: reads `bytes` (multiple of 16) of `buf` with
 * ordinary loads, which allocate in the L2 caches and the 256 MB Infinity
 * Cache, so that a buffer larger than both (1 GiB) evicts what they held
 * (the read probe's non-temporal loads do not).  Nothing is written but one
 * 8-byte partial per workgroup to `sink` (as for ehyb_probe_read), so no
 * dirty lines are left to be written back during the next kernel. */
EHYB_API ehyb_status ehyb_cache_flush(const void *buf, size_t bytes, void *sink, void *stream);
EHYB_API ehyb_status ehyb_probe_copy(const void *src, void *dst, size_t bytes, void *stream);

typedef struct {
    int32_t device, num_cus, lds_per_block, warp_size, clock_khz, mem_clock_khz;
    int32_t mem_bus_width, l2_bytes;
    char arch[64];
} ehyb_device_info;

/* Properties of the current device. */
EHYB_API ehyb_status ehyb_device_info_get(ehyb_device_info *out);

/* Message of the last failing call on this thread ("" if none). */
EHYB_API const char *ehyb_last_error(void);

/* Library version, e.g. "0.1.0". */
EHYB_API const char *ehyb_version(void);

#ifdef __cplusplus
}
#endif

#endif /* EHYB_H */
