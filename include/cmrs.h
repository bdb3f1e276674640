/*
 * cmrs.h -- C ABI of libcmrs.so: Compressed Multi-Row Storage (CMRS) sparse
 * matrices and their matrix-vector product on AMD MI355X (gfx950).
 *
 * Method: Z. Koza, M. Matyka, S. Szkoda, L. Miroslaw, "Compressed Multi-Row
 * Storage Format for Sparse Matrices on Graphics Processing Units",
 * arXiv:1203.2946.
 *
 * Conventions for every call below
 *   - All array pointers are DEVICE pointers (hipMalloc'd or equivalent),
 *     unless marked "host".  Indices are zero-based int32.
 *   - Every call that takes a stream is stream-ordered and asynchronous: it
 *     validates its host-side arguments, enqueues kernels on `stream` and
 *     returns.  Results are visible after the stream is synchronised.
 *   - The library allocates no device memory.  Every buffer, including the
 *     workspaces sized by the *_workspace queries, belongs to the caller and
 *     must stay alive until the enqueued work has finished.
 *   - Every call returns a cmrs_status_t and never throws.  Host-side
 *     argument checks happen before anything is enqueued (nothing is written
 *     on error).  A HIP launch error maps to CMRS_ERR_DEVICE with details in
 *     cmrs_last_error().
 *   - Data-dependent validity of a CSR input (row_ptr[0] == 0, monotone
 *     row_ptr, row_ptr[rows] == nnz, 0 <= col < cols) is NOT checked on the
 *     hot path; cmrs_validate_csr() checks it on the device.  Invalid data
 *     gives unspecified results but never out-of-bounds accesses of the
 *     arrays whose sizes the call was given, except through invalid indices.
 */
#ifndef CMRS_H_
#define CMRS_H_

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CMRS_ABI_VERSION 2

typedef enum {
    CMRS_OK = 0,
    CMRS_ERR_INVALID_VALUE = 1,   /* bad size, height, pointer, dtype or flag   */
    CMRS_ERR_INDEX_OVERFLOW = 2,  /* cols does not fit the packed column field,
                                     or rows / nnz above CMRS_MAX_INDEX         */
    CMRS_ERR_NOT_SUPPORTED = 3,   /* valid request that this build cannot serve */
    CMRS_ERR_DEVICE = 4,          /* HIP error while enqueueing                 */
    CMRS_ERR_WORKSPACE = 5        /* workspace pointer NULL or too small        */
} cmrs_status_t;

typedef enum {
    CMRS_R64F = 0,   /* IEEE binary64 */
    CMRS_R32F = 1,   /* IEEE binary32 */
    CMRS_R16BF = 2   /* bfloat16 (8 significant bits, fp32 exponent range) */
} cmrs_dtype_t;

/* Conversion flag: reorder the entries of every strip by column, ties by
 * RowInStrip, exact duplicates kept in CSR order (Sec. 4, fourth
 * optimisation; the worked height-2 example of that section fixes the tie
 * order). */
#define CMRS_SORT 1u

/* Largest supported strip height. */
#define CMRS_MAX_HEIGHT 32

/* Largest row count and entry count (nnz, padded_nnz) any call accepts,
 * 2^31 - 2^16: the kernels index rows and entries with 32-bit integers and
 * step up to 2^16 past the last one inside their loops.  Larger sizes return
 * CMRS_ERR_INDEX_OVERFLOW before anything is enqueued. */
#define CMRS_MAX_INDEX 2147418112

/* SpMV kernel variants (cmrs_spmv `variant`). */
#define CMRS_SPMV_AUTO 0   /* library's choice for (height, dtype)                  */
#define CMRS_SPMV_LDS 1    /* one wave64 per strip, per-lane partial sums in LDS     */
#define CMRS_SPMV_REG 2    /* one wave64 per strip, per-lane partial sums in VGPRs   */
#define CMRS_SPMV_LDS_NT 3 /* LDS, Val / word streams read with non-temporal loads   */
#define CMRS_SPMV_REG_NT 4 /* REG, Val / word streams read with non-temporal loads   */
#define CMRS_SPMV_GROUP 5  /* 64/G strips per wave, G lanes per strip, LDS partials  */
#define CMRS_SPMV_GROUP_NT 6 /* GROUP with non-temporal Val / word loads             */

/*
 * A CMRS matrix (Sec. 3): `height` rows per strip, strips = ceil(rows/height).
 *   strip_ptr[strips+1]: strip_ptr[j] is the index of the first entry of strip
 *       j, strip_ptr[strips] = nnz; strip j holds rows j*height .. j*height +
 *       height - 1 (the last strip may be partial).
 *   col_word[nnz]: packed (column << bits) | RowInStrip, with RowInStrip = row
 *       mod height (Sec. 4 packs the two into one 32-bit word; bits =
 *       cmrs_bits_for_height(height)).  Unsigned: the column field holds
 *       32 - bits bits.
 *   val[nnz]: the matrix values in `val_dtype`, in the same order.
 * `sorted` records whether the strips were reordered (CMRS_SORT); the SpMV is
 * correct for any order of entries inside a strip.
 * This struct is a host-side, non-owning view; the library keeps no
 * reference to it after a call returns.
 */
typedef struct {
    int32_t rows;
    int32_t cols;
    int32_t nnz;
    int32_t height;
    int32_t bits;
    int32_t sorted;
    cmrs_dtype_t val_dtype;
    const int32_t *strip_ptr;
    const uint32_t *col_word;
    const void *val;
} cmrs_mat_t;

/* ABI version of the loaded library (CMRS_ABI_VERSION it was built with). */
int32_t cmrs_abi_version(void);

/* ceil(rows / height) (Sec. 3); -1 if rows < 0 or height < 1.  Host only. */
int32_t cmrs_num_strips(int32_t rows, int32_t height);

/* Width of the packed RowInStrip field: max(4, ceil(log2(height))).  Sec. 4
 * uses 4 bits (heights up to 16); height 17..32 needs 5.  -1 if height is
 * outside [1, CMRS_MAX_HEIGHT].  Host only. */
int32_t cmrs_bits_for_height(int32_t height);

/* Bytes of workspace cmrs_from_csr needs: 0 without CMRS_SORT; with it,
 * two lists of the strips too long to be sorted inside the conversion kernel
 * and a global sort buffer for strips that do not fit one workgroup's LDS.
 * Host only. */
size_t cmrs_from_csr_workspace(int32_t rows, int32_t nnz, int32_t height, uint32_t flags);

/*
 * CSR -> CMRS (Sec. 3: strip_ptr[j] = row_ptr[j*height], strip_ptr[strips] =
 * nnz, RowInStrip = row mod height; Sec. 4: packed words; with CMRS_SORT the
 * in-strip reorder of Sec. 4).
 *   rows, cols, nnz   matrix sizes (>= 0); cols <= 2^(32 - bits) else
 *                     CMRS_ERR_INDEX_OVERFLOW.
 *   row_ptr[rows+1], col_ind[nnz], val_in[nnz]   CSR input (device).
 *   dtype             element type of val_in / val_out.
 *   height            1 .. CMRS_MAX_HEIGHT.
 *   flags             0 or CMRS_SORT.
 *   strip_ptr_out[strips+1], col_word_out[nnz], val_out[nnz]   CMRS output.
 *   workspace / workspace_bytes  >= cmrs_from_csr_workspace(...) bytes
 *                     (may be NULL when that is 0).
 * Aliasing: without CMRS_SORT, col_word_out may equal col_ind (in-place
 * packing) and val_out may equal val_in (the values are then not touched);
 * the paper's conversion is in place (Sec. 7).  With CMRS_SORT no output may
 * overlap an input.
 */
cmrs_status_t cmrs_from_csr(int32_t rows, int32_t cols, int32_t nnz,
                            const int32_t *row_ptr, const int32_t *col_ind, const void *val_in,
                            cmrs_dtype_t dtype, int32_t height, uint32_t flags,
                            int32_t *strip_ptr_out, uint32_t *col_word_out, void *val_out,
                            void *workspace, size_t workspace_bytes, hipStream_t stream);

/* Bytes of workspace cmrs_to_csr needs (currently always 0).  Host only. */
size_t cmrs_to_csr_workspace(const cmrs_mat_t *A);

/*
 * CMRS -> CSR, the inverse conversion (Sec. 3; Sec. 7 calls it quick and in
 * place).  Row s*height + r of strip s collects, in the order they appear in
 * the strip, the entries whose RowInStrip is r; column = word >> bits.
 *   row_ptr_out[rows+1], col_ind_out[nnz], val_out[nnz]   CSR output (device);
 *   no output may overlap an input.
 * For an unsorted CMRS matrix this reproduces the CSR it came from bit for
 * bit; for a sorted one, columns come out ascending inside each row.  A word
 * whose RowInStrip names no row of its strip is invalid input: it is dropped,
 * nothing is written outside the outputs, and their contents are unspecified.
 */
cmrs_status_t cmrs_to_csr(const cmrs_mat_t *A, int32_t *row_ptr_out, int32_t *col_ind_out,
                          void *val_out, void *workspace, size_t workspace_bytes,
                          hipStream_t stream);

/*
 * y = A x (Sec. 2.1), Algorithm 1 of Sec. 4: every strip is processed by one
 * 64-lane wave; lane l takes entries start+l, start+l+64, ..., adds
 * Val[j] * x[col] into its own partial sum for row RowInStrip; the partials
 * are then reduced across lanes and the wave writes the strip's `height`
 * results.
 *   x[cols], y[rows]  device vectors of xy_dtype; must not overlap.
 *   xy_dtype          R64F with R64F values (fp64 arithmetic), R32F with R32F
 *                     values (fp32 arithmetic), or R32F with R16BF values
 *                     (values widened to fp32, fp32 arithmetic).
 *   variant           CMRS_SPMV_* (AUTO picks per height and dtype).
 * y is overwritten (Algorithm 1 assigns the row sums): rows without entries
 * get +0.0.  rows == 0 is a no-op.  Deterministic: the same inputs give the
 * same bits on every call.
 */
cmrs_status_t cmrs_spmv(const cmrs_mat_t *A, const void *x, void *y, cmrs_dtype_t xy_dtype,
                        int32_t variant, hipStream_t stream);

/*
 * Column-blocked schedule (an MI355X-specific schedule of Algorithm 1, not a
 * format change).  For a sorted matrix (CMRS_SORT: the entries of every strip
 * ascend by column) the columns are cut into col_blocks blocks of width
 * ceil(cols / col_blocks); the entries of a strip that fall in block b are then
 * one contiguous run.  The plan holds, for every strip s and b = 1 ..
 * col_blocks-1, the index of the first entry of strip s in block b:
 *   split[s * (col_blocks - 1) + b - 1]      (int32, device)
 * Every run is processed exactly as cmrs_spmv processes a strip; the gathers
 * of one run touch only 1/col_blocks of x.  Three schedules:
 *   CMRS_COLBLOCK_PASSES      col_blocks launches, pass b adds run b of every
 *                             strip to y (pass 0 overwrites y); no workspace.
 *   CMRS_COLBLOCK_CONCURRENT  one launch; workgroup w takes column block
 *                             w % col_blocks, so with col_blocks = 8 each of
 *                             MI355X's 8 XCDs gathers from one eighth of x,
 *                             which stays in its L2.  Run sums go to a
 *                             workspace of col_blocks * rows partials (fp64
 *                             for fp64 values, fp32 otherwise), then a second
 *                             kernel adds the col_blocks partials of each row
 *                             in block order.
 *   CMRS_COLBLOCK_PHASED      one launch, no workspace: each wave owns whole
 *                             strips (a strip group) and walks block 0 of
 *                             all of them, then block 1, ..., adding into
 *                             the same per-lane partial sums, and writes y
 *                             once; the waves of an XCD move through the
 *                             blocks together, so they gather from about one
 *                             block of x at a time.
 * Results obey the same error bound as cmrs_spmv (the products of a row are
 * summed in a different order) and are deterministic.
 *   col_blocks   1 .. 64; 1 means no blocking (plan of zero bytes).
 *   variant      accumulation variant as for cmrs_spmv (the concurrent
 *                schedule always uses strip groups with non-temporal loads).
 * The plan depends only on A's strip_ptr and col_word; rebuild it when they
 * change.  CMRS_ERR_INVALID_VALUE if A is not sorted.
 */
#define CMRS_COLBLOCK_PASSES 0
#define CMRS_COLBLOCK_CONCURRENT 1
#define CMRS_COLBLOCK_PHASED 2
size_t cmrs_colblock_plan_bytes(const cmrs_mat_t *A, int32_t col_blocks);
cmrs_status_t cmrs_colblock_plan(const cmrs_mat_t *A, int32_t col_blocks, int32_t *split, size_t split_bytes,
                                 hipStream_t stream);
size_t cmrs_spmv_colblock_workspace(const cmrs_mat_t *A, int32_t col_blocks, int32_t schedule);
cmrs_status_t cmrs_spmv_colblock(const cmrs_mat_t *A, const void *x, void *y, cmrs_dtype_t xy_dtype,
                                 int32_t variant, int32_t col_blocks, const int32_t *split, size_t split_bytes,
                                 int32_t schedule, void *workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * Split schedule for strips of very different lengths (skewed rows).  The
 * paper sets matrices with very long rows aside for special algorithms
 * (Sec. 6.2); Algorithm 1 would give each such strip to one wave, which then
 * sets the time of the whole product.  Here every strip with more than
 * long_len stored entries is "heavy": a plan cuts it into chunks of at most
 * chunk_len consecutive entries, chunk waves compute the chunks' row sums
 * (each as Algorithm 1 computes a strip) while all other strips run as
 * strip groups (CMRS_SPMV_GROUP_NT), and a second small launch adds each
 * split strip's chunk sums in chunk order and writes its rows.  y is
 * overwritten, the error bound of cmrs_spmv holds, results are
 * deterministic.
 *
 * cmrs_spmv_split_plan_bytes: device bytes of the plan buffer (0 for an
 *   invalid matrix or negative long_len / chunk_len).  long_len 0 picks
 *   16 entries per lane of the strip-group width, chunk_len 0 picks 1024.
 * cmrs_spmv_split_plan: fills *plan (host struct) and, asynchronously on
 *   `stream`, the caller's device buffer `buf` (16-byte aligned, at least
 *   cmrs_spmv_split_plan_bytes): the heavy-strip and chunk lists and room
 *   for the chunk sums.  It reads only A's
 *   strip_ptr (device) and needs no synchronisation, so it may run in the
 *   same stream before each product; rebuild it when strip_ptr changes.
 * cmrs_spmv_split: y = A x with the plan.  The product writes the chunk
 *   sums into the plan buffer, so products with one plan must not overlap.
 *   Dtypes as cmrs_spmv.
 * Errors: CMRS_ERR_INVALID_VALUE for a bad matrix, negative long_len /
 *   chunk_len, a plan built for another matrix shape or inconsistent fields,
 *   NULL or overlapping x / y; CMRS_ERR_WORKSPACE for a NULL, misaligned or
 *   short buffer; CMRS_ERR_NOT_SUPPORTED for a dtype pair other than
 *   cmrs_spmv's; CMRS_ERR_DEVICE if a launch fails.  *plan is written only on
 *   success.
 */
typedef struct {
    int32_t rows, nnz, height;  /* shape of the matrix the plan was built for     */
    int32_t group;              /* lanes per strip of the strip-group waves       */
    int32_t long_len;           /* strips with more entries are split             */
    int32_t chunk_len;          /* entries per chunk, at most                     */
    int32_t max_heavy;          /* capacity of the heavy-strip list               */
    int32_t max_chunks;         /* capacity of the chunk list                     */
    void *buf;                  /* the caller's device buffer                     */
    size_t bytes;
} cmrs_split_plan_t;
size_t cmrs_spmv_split_plan_bytes(const cmrs_mat_t *A, int32_t long_len, int32_t chunk_len);
cmrs_status_t cmrs_spmv_split_plan(const cmrs_mat_t *A, int32_t long_len, int32_t chunk_len, void *buf,
                                   size_t bytes, cmrs_split_plan_t *plan, hipStream_t stream);
cmrs_status_t cmrs_spmv_split(const cmrs_mat_t *A, const cmrs_split_plan_t *plan, const void *x, void *y,
                              cmrs_dtype_t xy_dtype, hipStream_t stream);

/*
 * The concurrent column-blocked product without a caller workspace, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  Same arguments,
 * kernels and results as cmrs_spmv_colblock(..., CMRS_COLBLOCK_CONCURRENT,
 * ...), bit for bit; the col_blocks * rows partial sums go to a scratch
 * array of CMRS_NOALLOC_SCRATCH_BYTES that the library holds in device
 * memory (one per GPU, alive until the process ends; its address is looked
 * up on the first call on each device, with that device current).  Nothing
 * is allocated and nothing needs clearing: every partial is written before
 * it is read.  All calls on one GPU share that GPU's scratch, so calls that
 * may overlap on one GPU (other streams, other host threads) race and must
 * be ordered by the caller.  Errors as cmrs_spmv_colblock, plus
 * CMRS_ERR_WORKSPACE when cmrs_spmv_colblock_workspace(A, col_blocks,
 * CMRS_COLBLOCK_CONCURRENT) exceeds CMRS_NOALLOC_SCRATCH_BYTES (e.g. fp64
 * values with 4 blocks: rows <= 2^20), and CMRS_ERR_DEVICE if the scratch
 * address cannot be obtained.  col_blocks == 1 runs the plain product.
 */
#define CMRS_NOALLOC_SCRATCH_BYTES (32u << 20)
cmrs_status_t cmrs_spmv_colblock_noalloc(const cmrs_mat_t *A, const void *x, void *y, cmrs_dtype_t xy_dtype,
                                         int32_t variant, int32_t col_blocks, const int32_t *split,
                                         size_t split_bytes, hipStream_t stream);

/*
 * Products with several right-hand sides, Y = A X (the problem statement
 * y = A x of Sec. 2.1 for nrhs vectors at once; each loaded value and packed
 * word serves all of them).
 *
 * Layout: X and Y are row-major with leading dimensions ldx, ldy >= nrhs:
 *   x_k[c] = X[c * ldx + k],  y_k[r] = Y[r * ldy + k],  k < nrhs,
 * so the nrhs gathers of one entry read one contiguous piece of X.  Entries
 * of Y with k >= nrhs are not touched; every row of Y (k < nrhs) is written,
 * empty rows with +0.  nrhs in [1, CMRS_SPMM_MAX_RHS].  Dtypes as for
 * cmrs_spmv (fp64/fp64, fp32/fp32, bf16 values with fp32 X and Y).  Every
 * y_k obeys cmrs_spmv's error bound; results are deterministic for a fixed
 * `group` (and, for batches, fixed tuning).
 *
 * cmrs_spmm: one matrix, one launch.  The lanes of a wave are strips x
 * entry slots: `group` entry slots per strip (a power of two <= 64; 0
 * chooses it from the mean strip length), every lane handling all nrhs
 * right-hand sides of its entries with next_pow2(height) * next_pow2(nrhs)
 * partial sums in LDS.  That LDS (64 lanes x partials x 8 bytes for fp64
 * values, 4 otherwise) must fit 64 KiB per wave: larger height-nrhs
 * combinations return CMRS_ERR_NOT_SUPPORTED.  X and Y must not overlap.
 * Errors (nothing is enqueued): CMRS_ERR_INVALID_VALUE for a bad matrix
 * descriptor, nrhs, leading dimension, group, NULL X/Y (when used) or
 * overlapping X and Y; CMRS_ERR_NOT_SUPPORTED for a dtype pair other than
 * the three above or the LDS limit; CMRS_ERR_DEVICE if the launch fails.
 */
#define CMRS_SPMM_MAX_RHS 8
cmrs_status_t cmrs_spmm(const cmrs_mat_t *A, int32_t nrhs, const void *X, int32_t ldx, void *Y, int32_t ldy,
                        cmrs_dtype_t xy_dtype, int32_t group, hipStream_t stream);

/*
 * Batched products Y_i = A_i X_i for count matrices of any sizes and heights,
 * in ONE persistent launch.  A plan splits every matrix into work tiles of
 * whole strips (about tuning->tile_nnz stored entries each) and writes, into
 * the caller's device buffer `desc` (cmrs_spmm_plan_bytes() bytes), a small
 * queue header, one descriptor per matrix (its arrays, X_i, Y_i, nrhs_i,
 * ldx_i, ldy_i) and the tile list.  cmrs_spmm_batched() then launches
 * plan->grid workgroups that take tiles from the queues until they are
 * empty: one queue per XCD over a contiguous eighth of the tile list, drained
 * first by that XCD's workgroups; the last wave to finish resets the queues,
 * so the same plan can be launched again, one launch at a time per plan, and
 * captured into a HIP graph.  Tile t of matrix i is computed exactly as
 * cmrs_spmm computes those strips with the plan's group width (clamped to
 * 64), so results equal cmrs_spmm's bit for bit.
 *
 * cmrs_spmm_plan is set-up, not hot path: it copies the descriptor image
 * from host memory with hipMemcpyAsync and synchronises `stream` (so do not
 * call it under graph capture).  The plan binds the device pointers it was
 * given; rebuild it when any of them, or a matrix, changes.  Host arrays
 * mats, nrhs, X, ldx, Y, ldy have `count` entries; all matrices share one
 * value dtype, matched with xy_dtype as for cmrs_spmv.  Y_i must not overlap
 * each other or any X_j (X_j may be shared).  tuning may be NULL (defaults).
 * If a batched launch does not run to completion, rebuild the plan.
 * Errors: cmrs_spmm_plan_bytes returns 0 for an invalid batch or tuning.
 * cmrs_spmm_plan returns CMRS_ERR_INVALID_VALUE for a bad matrix, nrhs,
 * leading dimension, tuning field, NULL array or overlapping outputs,
 * CMRS_ERR_NOT_SUPPORTED for mixed value dtypes or the LDS limit of
 * cmrs_spmm, CMRS_ERR_WORKSPACE when `desc` is NULL or smaller than
 * cmrs_spmm_plan_bytes(), CMRS_ERR_DEVICE when the copy fails; `plan` is
 * written only on success, `desc` not at all when a host-side check fails.
 * cmrs_spmm_batched returns
 * CMRS_ERR_INVALID_VALUE for a plan whose fields are inconsistent (not
 * filled by cmrs_spmm_plan) and CMRS_OK without launching for zero tiles.
 */
typedef struct {
    int32_t tile_nnz;       /* stored entries per work tile (rounded to whole
                               strip passes); 0 = 32768                        */
    int32_t group;          /* entry slots per strip, a power of two; 0 = from
                               each matrix's mean strip length                 */
    int32_t blocks_per_cu;  /* resident 256-thread workgroups per compute unit;
                               0 = 4                                           */
    int32_t reserved;       /* must be 0                                       */
} cmrs_spmm_tuning_t;

typedef struct {            /* filled by cmrs_spmm_plan (host struct)          */
    int32_t count, tiles;   /* matrices, work tiles                            */
    int32_t grid, lds_bytes;/* workgroups of the launch, LDS per workgroup     */
    int32_t val_dtype, xy_dtype;
    int32_t max_slots;      /* largest next_pow2(height) * next_pow2(nrhs)     */
    int32_t waves;          /* waves of the launch (1..4 per workgroup)        */
    void *desc;             /* the caller's device buffer                      */
    size_t desc_bytes;
} cmrs_spmm_plan_t;

size_t cmrs_spmm_plan_bytes(int32_t count, const cmrs_mat_t *mats, const int32_t *nrhs,
                            const cmrs_spmm_tuning_t *tuning);
cmrs_status_t cmrs_spmm_plan(int32_t count, const cmrs_mat_t *mats, const int32_t *nrhs, const void *const *X,
                             const int32_t *ldx, void *const *Y, const int32_t *ldy, cmrs_dtype_t xy_dtype,
                             const cmrs_spmm_tuning_t *tuning, void *desc, size_t desc_bytes,
                             cmrs_spmm_plan_t *plan, hipStream_t stream);
cmrs_status_t cmrs_spmm_batched(const cmrs_spmm_plan_t *plan, hipStream_t stream);

/*
 * Modified CMRS of Sec. 6.7 ("padded"): strips padded with explicit zeros to
 * whole chunks of 64 entries, every row contributing at most 8 contiguous
 * entries to a chunk, so that the SpMV needs only 8 copies of a strip's row
 * sums per wave (lane l adds into copy l mod 8) and every load is an aligned
 * 64-lane access.  The paper gives the constraints; the arrangement used
 * here takes, chunk after chunk, min(8, entries left) entries of every row
 * in CSR order, rows with more entries left first (ties: lower row), until
 * the chunk is full; the remaining slots are padding.  A padding entry has
 * RowInStrip = height, column 0 and value +0 and is skipped by the kernel.
 * The packed RowInStrip field is cmrs_padded_bits(height) wide (one more
 * bit than cmrs_bits_for_height when height is a power of two >= 16).
 * Padding can multiply the stored entries (a row of L entries needs at
 * least L/8 chunks); the plan returns the padded size so the caller can
 * weigh the memory overhead.
 *
 * cmrs_padded_plan: counts the chunks of every strip and writes
 *   strip_ptr_out[strips+1] (entry offsets, multiples of 64) and
 *   *padded_nnz_out (host); synchronises `stream` to return the size.
 *   CMRS_ERR_INDEX_OVERFLOW when the padded size exceeds CMRS_MAX_INDEX
 *   (the size is still returned).  Workspace: cmrs_padded_plan_workspace() bytes,
 *   8-byte aligned.
 * cmrs_padded_from_csr: fills col_word_out / val_out (padded_nnz entries)
 *   for canonical or any CSR; entries keep their CSR order within a row.
 *   Outputs may not overlap the inputs.
 * cmrs_padded_spmv: y = A x for a padded matrix: A->strip_ptr from the plan,
 *   A->nnz = padded_nnz, A->bits = cmrs_padded_bits(height), A->sorted
 *   ignored.  Every row of y is written (empty rows +0); error bound and
 *   dtypes as for cmrs_spmv.  Precondition: the entries are arranged as
 *   cmrs_padded_from_csr arranges them (at most 8 entries of a row in any
 *   64-entry chunk, the constraint of Sec. 6.7).  Lanes l, l+8, ... of a
 *   chunk share copy l mod 8 of the row sums; with fp32 or bf16 values that
 *   copy is updated by a plain read-modify-write, so an arrangement that
 *   breaks the constraint gives unspecified fp32/bf16 results (fp64 uses
 *   the LDS atomic add and stays correct).
 */
int32_t cmrs_padded_bits(int32_t height);
size_t cmrs_padded_plan_workspace(int32_t rows, int32_t height);
cmrs_status_t cmrs_padded_plan(int32_t rows, int32_t nnz, const int32_t *row_ptr, int32_t height,
                               int32_t *strip_ptr_out, int64_t *padded_nnz_out, void *workspace,
                               size_t workspace_bytes, hipStream_t stream);
cmrs_status_t cmrs_padded_from_csr(int32_t rows, int32_t cols, int32_t nnz, const int32_t *row_ptr,
                                   const int32_t *col_ind, const void *val_in, cmrs_dtype_t dtype, int32_t height,
                                   const int32_t *strip_ptr, int32_t padded_nnz, uint32_t *col_word_out,
                                   void *val_out, hipStream_t stream);
cmrs_status_t cmrs_padded_spmv(const cmrs_mat_t *A, const void *x, void *y, cmrs_dtype_t xy_dtype,
                               hipStream_t stream);

/*
 * Device check of CSR validity: writes *flag_out = 0 when row_ptr[0] == 0,
 * row_ptr is non-decreasing, row_ptr[rows] == nnz and every column is in
 * [0, cols); otherwise a non-zero bit mask (1: row_ptr[0] or row_ptr[rows]
 * wrong, 2: row_ptr decreasing, 4: column out of range).  flag_out is one
 * device int32.
 */
cmrs_status_t cmrs_validate_csr(int32_t rows, int32_t cols, int32_t nnz, const int32_t *row_ptr,
                                const int32_t *col_ind, int32_t *flag_out, hipStream_t stream);

/*
 * Learned configuration selection.  The paper chooses the strip height and the
 * kernel options by brute-force search over measured times (Sec. 6.3) and
 * reports how much per-matrix tuning can gain (Sec. 6.8).  These calls provide
 * the pieces of a learned replacement: matrix features and a small MLP
 * (CMRS_SEL_FEATURES -> 64 -> 64 -> CMRS_SEL_CLASSES, ReLU, fp32) with forward,
 * backward and Adam kernels, so the network is trained on the GPU from
 * measured times.  Class c = 4 * log2(height) + schedule (schedules: 0 one
 * wave per strip, 1 the same with non-temporal loads, 2 strip groups, 3
 * concurrent column blocks with 4 blocks; heights 1..32).
 *
 * cmrs_features: 40 floats from a CSR structure: [0,20) fractions of rows
 *   by length in half octaves (bin 0 empty; p = floor(log2 len) -> 1 + 2p,
 *   or 2 + 2p when len >= 1.5 * 2^p; >= 512 -> 19); [20,36) fractions of
 *   entries by |col - floor(row * cols / rows)| (0; then [2^(b-1), 2^b);
 *   last bin open); 36..39 log2(rows)/22, log2(nnz+1)/26,
 *   log2(nnz/rows+1)/14, log2(max len+1)/14.  workspace:
 *   CMRS_SEL_FEATURE_WS bytes of device memory (zeroed by the call).
 * Parameters are one packed float array of CMRS_SEL_PARAMS:
 *   W1[40][64], b1[64], W2[64][64], b2[64], W3[64][24], b3[24] (row-major,
 *   out = in W + b).  Activations are [batch][width] row-major device arrays.
 * cmrs_mlp_forward:  H1, H2 (batch x 64) and Y (batch x 24).
 * cmrs_mlp_backward: from dY (batch x 24) and the forward activations, the
 *   parameter gradients `grads` (CMRS_SEL_PARAMS) with scratch dH2, dH1
 *   (batch x 64 each); batch sums in sample order (deterministic).
 * cmrs_mse_grad:     dY = scale * (Y - T), n values.
 * cmrs_adam_step:    one Adam update of n parameters (step >= 1 for the bias
 *   corrections).
 * All arrays are caller-owned device fp32 arrays.  Errors: CMRS_ERR_INVALID_VALUE
 * for a negative size (batch <= 0 for the backward), step < 1 or a NULL
 * array; CMRS_ERR_WORKSPACE for a missing or short feature workspace;
 * CMRS_ERR_DEVICE when a launch fails.  batch = 0 (forward) and n = 0 are
 * no-ops.
 */
#define CMRS_SEL_FEATURES 40
#define CMRS_SEL_CLASSES 24
#define CMRS_SEL_PARAMS 8344
#define CMRS_SEL_FEATURE_WS 256
cmrs_status_t cmrs_features(int32_t rows, int32_t cols, int32_t nnz, const int32_t *row_ptr, const int32_t *col_ind,
                            float *feat_out, void *workspace, size_t workspace_bytes, hipStream_t stream);
cmrs_status_t cmrs_mlp_forward(int32_t batch, const float *X, const float *params, float *H1, float *H2, float *Y,
                               hipStream_t stream);
cmrs_status_t cmrs_mlp_backward(int32_t batch, const float *X, const float *params, const float *H1,
                                const float *H2, const float *dY, float *dH2, float *dH1, float *grads,
                                hipStream_t stream);
cmrs_status_t cmrs_mse_grad(int32_t n, const float *Y, const float *T, float *dY, float scale, hipStream_t stream);
cmrs_status_t cmrs_adam_step(int32_t n, float *params, const float *grads, float *m, float *v, float lr, float beta1,
                             float beta2, float eps, int32_t step, hipStream_t stream);

/*
 * Measurement aids (not part of y = A x).
 *
 * cmrs_calib_stream_read: the read-only kernel of Sec. 6.3 — it reads the
 * packed words (4*nnz bytes) and values (nnz values of `dtype`) of a CMRS
 * matrix with 16-byte non-temporal loads, while every 256-thread workgroup
 * reserves lds_words_per_lane * 256 values of LDS (the per-lane buffer of a
 * strip of that height), so it runs at the SpMV's occupancy.  Both arrays must
 * be 16-byte aligned; a tail shorter than 16 bytes is not read.
 * lds_words_per_lane in [0, 32].
 *
 * cmrs_calib_gather: reads x[idx[i]] for i < n (n up to 2^31 - 1; every idx
 * below the length of x) and sums them; the rate of random single-element
 * reads.  x_dtype R64F or R32F.
 *
 * sink: one device double, never written for real data.
 */
cmrs_status_t cmrs_calib_stream_read(const uint32_t *col_word, const void *val, int32_t nnz, cmrs_dtype_t dtype,
                                     int32_t lds_words_per_lane, double *sink, hipStream_t stream);
cmrs_status_t cmrs_calib_gather(const uint32_t *idx, int64_t n, const void *x, cmrs_dtype_t x_dtype, double *sink,
                                hipStream_t stream);

/* Static string for a status code. */
const char *cmrs_status_string(cmrs_status_t s);

/* Detail of the last error on the calling host thread ("" if none). */
const char *cmrs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CMRS_H_ */
