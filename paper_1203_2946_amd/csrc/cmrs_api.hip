// Host side of the C ABI declared in include/cmrs.h: argument validation,
// error reporting and dispatch to the kernels.  Nothing here allocates.
#include <limits.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "cmrs_ext.hpp"

namespace {

thread_local char g_last_error[512] = {0};

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
}

cmrs_status_t fail(cmrs_status_t st, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
    return st;
}

cmrs_status_t from_hip(hipError_t e, const char* where) {
    if (e == hipSuccess) return CMRS_OK;
    set_error("%s: %s (%s)", where, hipGetErrorName(e), hipGetErrorString(e));
    return CMRS_ERR_DEVICE;
}

bool valid_dtype(cmrs_dtype_t t) { return t == CMRS_R64F || t == CMRS_R32F || t == CMRS_R16BF; }

// Column field width check: cols must fit in 32 - bits bits.
bool cols_fit(int32_t cols, int32_t bits) {
    return static_cast<uint64_t>(cols) <= (static_cast<uint64_t>(1) << (32 - bits));
}

// Sizes the 32-bit row and entry indexing of the kernels can serve.
bool size_fits(int64_t n) { return n <= CMRS_MAX_INDEX; }

bool ranges_overlap(const void* a, size_t an, const void* b, size_t bn) {
    if (!a || !b || an == 0 || bn == 0) return false;
    const char* pa = static_cast<const char*>(a);
    const char* pb = static_cast<const char*>(b);
    return pa < pb + bn && pb < pa + an;
}

cmrs_status_t check_mat(const cmrs_mat_t* A) {
    if (!A) return fail(CMRS_ERR_INVALID_VALUE, "matrix descriptor is NULL");
    if (A->rows < 0 || A->cols < 0 || A->nnz < 0)
        return fail(CMRS_ERR_INVALID_VALUE, "negative size (rows=%d cols=%d nnz=%d)", A->rows, A->cols, A->nnz);
    if (A->height < 1 || A->height > CMRS_MAX_HEIGHT)
        return fail(CMRS_ERR_INVALID_VALUE, "height %d outside [1, %d]", A->height, CMRS_MAX_HEIGHT);
    if (!size_fits(A->rows) || !size_fits(A->nnz))
        return fail(CMRS_ERR_INDEX_OVERFLOW, "rows=%d or nnz=%d above %d", A->rows, A->nnz, CMRS_MAX_INDEX);
    if (A->bits != cmrs_bits_for_height(A->height))
        return fail(CMRS_ERR_INVALID_VALUE, "bits %d != cmrs_bits_for_height(%d) = %d", A->bits, A->height,
                    cmrs_bits_for_height(A->height));
    if (!valid_dtype(A->val_dtype)) return fail(CMRS_ERR_INVALID_VALUE, "unknown value dtype %d", (int)A->val_dtype);
    if (!cols_fit(A->cols, A->bits))
        return fail(CMRS_ERR_INDEX_OVERFLOW, "cols=%d does not fit %d column bits", A->cols, 32 - A->bits);
    if (A->rows > 0 && !A->strip_ptr) return fail(CMRS_ERR_INVALID_VALUE, "strip_ptr is NULL");
    if (A->nnz > 0 && (!A->col_word || !A->val)) return fail(CMRS_ERR_INVALID_VALUE, "col_word or val is NULL");
    return CMRS_OK;
}

}  // namespace

extern "C" {

int32_t cmrs_abi_version(void) { return CMRS_ABI_VERSION; }

int32_t cmrs_num_strips(int32_t rows, int32_t height) {
    if (rows < 0 || height < 1) return -1;
    return static_cast<int32_t>((static_cast<int64_t>(rows) + height - 1) / height);
}

int32_t cmrs_bits_for_height(int32_t height) {
    if (height < 1 || height > CMRS_MAX_HEIGHT) return -1;
    int32_t b = 0;
    while ((1 << b) < height) ++b;
    return b < 4 ? 4 : b;
}

size_t cmrs_from_csr_workspace(int32_t rows, int32_t nnz, int32_t height, uint32_t flags) {
    if (!(flags & CMRS_SORT) || nnz <= 0 || rows < 0 || height < 1) return 0;
    return cmrs::from_csr_workspace_layout(rows, nnz, height).total;
}

cmrs_status_t cmrs_from_csr(int32_t rows, int32_t cols, int32_t nnz, const int32_t* row_ptr, const int32_t* col_ind,
                            const void* val_in, cmrs_dtype_t dtype, int32_t height, uint32_t flags,
                            int32_t* strip_ptr_out, uint32_t* col_word_out, void* val_out, void* workspace,
                            size_t workspace_bytes, hipStream_t stream) {
    g_last_error[0] = 0;
    if (rows < 0 || cols < 0 || nnz < 0)
        return fail(CMRS_ERR_INVALID_VALUE, "negative size (rows=%d cols=%d nnz=%d)", rows, cols, nnz);
    if (height < 1 || height > CMRS_MAX_HEIGHT)
        return fail(CMRS_ERR_INVALID_VALUE, "height %d outside [1, %d]", height, CMRS_MAX_HEIGHT);
    if (flags & ~CMRS_SORT) return fail(CMRS_ERR_INVALID_VALUE, "unknown flags 0x%x", flags);
    if (!valid_dtype(dtype)) return fail(CMRS_ERR_INVALID_VALUE, "unknown dtype %d", (int)dtype);
    if (!size_fits(rows) || !size_fits(nnz))
        return fail(CMRS_ERR_INDEX_OVERFLOW, "rows=%d or nnz=%d above %d", rows, nnz, CMRS_MAX_INDEX);
    const int32_t bits = cmrs_bits_for_height(height);
    if (!cols_fit(cols, bits))
        return fail(CMRS_ERR_INDEX_OVERFLOW, "cols=%d does not fit %d column bits", cols, 32 - bits);
    if (!row_ptr || !strip_ptr_out) return fail(CMRS_ERR_INVALID_VALUE, "row_ptr or strip_ptr_out is NULL");
    if (nnz > 0 && (!col_ind || !val_in || !col_word_out || !val_out))
        return fail(CMRS_ERR_INVALID_VALUE, "an nnz-sized array is NULL");
    const size_t es = cmrs::dtype_bytes(dtype);
    const size_t nz = static_cast<size_t>(nnz);
    if (flags & CMRS_SORT) {
        if (ranges_overlap(col_word_out, 4 * nz, col_ind, 4 * nz) || ranges_overlap(val_out, es * nz, val_in, es * nz) ||
            ranges_overlap(col_word_out, 4 * nz, val_in, es * nz) || ranges_overlap(val_out, es * nz, col_ind, 4 * nz))
            return fail(CMRS_ERR_INVALID_VALUE, "sorted conversion cannot run in place");
        const size_t need = cmrs_from_csr_workspace(rows, nnz, height, flags);
        if (need > 0 && (!workspace || workspace_bytes < need))
            return fail(CMRS_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, workspace_bytes);
    } else {
        // In place is allowed only as exact aliasing.
        if ((ranges_overlap(col_word_out, 4 * nz, col_ind, 4 * nz) && (const void*)col_word_out != (const void*)col_ind) ||
            (ranges_overlap(val_out, es * nz, val_in, es * nz) && val_out != val_in))
            return fail(CMRS_ERR_INVALID_VALUE, "outputs partially overlap inputs");
    }
    return from_hip(cmrs::launch_from_csr(rows, cols, nnz, row_ptr, col_ind, val_in, dtype, height, bits, flags,
                                          strip_ptr_out, col_word_out, val_out, workspace, stream),
                    "cmrs_from_csr");
}

size_t cmrs_to_csr_workspace(const cmrs_mat_t* A) {
    (void)A;
    return 0;
}

cmrs_status_t cmrs_to_csr(const cmrs_mat_t* A, int32_t* row_ptr_out, int32_t* col_ind_out, void* val_out,
                          void* workspace, size_t workspace_bytes, hipStream_t stream) {
    (void)workspace;
    (void)workspace_bytes;
    g_last_error[0] = 0;
    cmrs_status_t st = check_mat(A);
    if (st != CMRS_OK) return st;
    if (!row_ptr_out) return fail(CMRS_ERR_INVALID_VALUE, "row_ptr_out is NULL");
    if (A->nnz > 0 && (!col_ind_out || !val_out)) return fail(CMRS_ERR_INVALID_VALUE, "col_ind_out or val_out is NULL");
    const size_t es = cmrs::dtype_bytes(A->val_dtype);
    const size_t nz = static_cast<size_t>(A->nnz);
    if (ranges_overlap(col_ind_out, 4 * nz, A->col_word, 4 * nz) || ranges_overlap(val_out, es * nz, A->val, es * nz))
        return fail(CMRS_ERR_INVALID_VALUE, "outputs overlap inputs");
    return from_hip(cmrs::launch_to_csr(A, row_ptr_out, col_ind_out, val_out, stream), "cmrs_to_csr");
}

static cmrs_status_t check_spmv_args(const cmrs_mat_t* A, const void* x, void* y, cmrs_dtype_t xy_dtype,
                                     int32_t variant) {
    cmrs_status_t st = check_mat(A);
    if (st != CMRS_OK) return st;
    const bool ok_types = (A->val_dtype == CMRS_R64F && xy_dtype == CMRS_R64F) ||
                          (A->val_dtype == CMRS_R32F && xy_dtype == CMRS_R32F) ||
                          (A->val_dtype == CMRS_R16BF && xy_dtype == CMRS_R32F);
    if (!ok_types)
        return fail(CMRS_ERR_NOT_SUPPORTED, "value dtype %d with x/y dtype %d", (int)A->val_dtype, (int)xy_dtype);
    if (variant < CMRS_SPMV_AUTO || variant > CMRS_SPMV_GROUP_NT)
        return fail(CMRS_ERR_INVALID_VALUE, "unknown variant %d", variant);
    if (A->rows == 0) return CMRS_OK;
    if (!y || (A->cols > 0 && !x)) return fail(CMRS_ERR_INVALID_VALUE, "x or y is NULL");
    const size_t xs = cmrs::dtype_bytes(xy_dtype);
    if (ranges_overlap(x, xs * static_cast<size_t>(A->cols), y, xs * static_cast<size_t>(A->rows)))
        return fail(CMRS_ERR_INVALID_VALUE, "x and y overlap");
    return CMRS_OK;
}

cmrs_status_t cmrs_spmv(const cmrs_mat_t* A, const void* x, void* y, cmrs_dtype_t xy_dtype, int32_t variant,
                        hipStream_t stream) {
    g_last_error[0] = 0;
    cmrs_status_t st = check_spmv_args(A, x, y, xy_dtype, variant);
    if (st != CMRS_OK || A->rows == 0) return st;
    return from_hip(cmrs::launch_spmv(A, x, y, xy_dtype, variant, stream), "cmrs_spmv");
}

size_t cmrs_colblock_plan_bytes(const cmrs_mat_t* A, int32_t col_blocks) {
    if (!A || col_blocks <= 1 || A->rows <= 0 || A->height < 1) return 0;
    const size_t strips = static_cast<size_t>(cmrs_num_strips(A->rows, A->height));
    return strips * static_cast<size_t>(col_blocks - 1) * sizeof(int32_t);
}

static cmrs_status_t check_colblock(const cmrs_mat_t* A, int32_t col_blocks, const int32_t* split,
                                    size_t split_bytes) {
    if (col_blocks < 1 || col_blocks > 64) return fail(CMRS_ERR_INVALID_VALUE, "col_blocks %d outside [1, 64]", col_blocks);
    if (col_blocks > 1 && !A->sorted) return fail(CMRS_ERR_INVALID_VALUE, "column blocking needs a sorted matrix");
    const size_t need = cmrs_colblock_plan_bytes(A, col_blocks);
    if (need > 0 && (!split || split_bytes < need))
        return fail(CMRS_ERR_WORKSPACE, "plan of %zu bytes needed, %zu given", need, split_bytes);
    return CMRS_OK;
}

static inline int colblock_width(const cmrs_mat_t* A, int32_t col_blocks) {
    const int64_t w = (static_cast<int64_t>(A->cols) + col_blocks - 1) / col_blocks;
    return static_cast<int>(w < 1 ? 1 : w);
}

cmrs_status_t cmrs_colblock_plan(const cmrs_mat_t* A, int32_t col_blocks, int32_t* split, size_t split_bytes,
                                 hipStream_t stream) {
    g_last_error[0] = 0;
    cmrs_status_t st = check_mat(A);
    if (st != CMRS_OK) return st;
    st = check_colblock(A, col_blocks, split, split_bytes);
    if (st != CMRS_OK) return st;
    return from_hip(cmrs::launch_colblock_plan(A, col_blocks, colblock_width(A, col_blocks), split, stream),
                    "cmrs_colblock_plan");
}

size_t cmrs_spmv_colblock_workspace(const cmrs_mat_t* A, int32_t col_blocks, int32_t schedule) {
    if (!A || schedule != CMRS_COLBLOCK_CONCURRENT || col_blocks <= 1 || A->rows <= 0) return 0;
    const size_t at = A->val_dtype == CMRS_R64F ? 8 : 4;
    return static_cast<size_t>(col_blocks) * static_cast<size_t>(A->rows) * at;
}

cmrs_status_t cmrs_spmv_colblock(const cmrs_mat_t* A, const void* x, void* y, cmrs_dtype_t xy_dtype, int32_t variant,
                                 int32_t col_blocks, const int32_t* split, size_t split_bytes, int32_t schedule,
                                 void* workspace, size_t workspace_bytes, hipStream_t stream) {
    g_last_error[0] = 0;
    cmrs_status_t st = check_spmv_args(A, x, y, xy_dtype, variant);
    if (st != CMRS_OK || A->rows == 0) return st;
    st = check_colblock(A, col_blocks, split, split_bytes);
    if (st != CMRS_OK) return st;
    if (schedule != CMRS_COLBLOCK_PASSES && schedule != CMRS_COLBLOCK_CONCURRENT && schedule != CMRS_COLBLOCK_PHASED)
        return fail(CMRS_ERR_INVALID_VALUE, "unknown schedule %d", schedule);
    const size_t need = cmrs_spmv_colblock_workspace(A, col_blocks, schedule);
    if (need > 0 && (!workspace || workspace_bytes < need))
        return fail(CMRS_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, workspace_bytes);
    if (need > 0 && (ranges_overlap(workspace, need, y, cmrs::dtype_bytes(xy_dtype) * static_cast<size_t>(A->rows)) ||
                     ranges_overlap(workspace, need, x, cmrs::dtype_bytes(xy_dtype) * static_cast<size_t>(A->cols))))
        return fail(CMRS_ERR_INVALID_VALUE, "workspace overlaps x or y");
    return from_hip(cmrs::launch_spmv_colblock(A, x, y, variant, col_blocks, split, schedule, workspace, stream),
                    "cmrs_spmv_colblock");
}

size_t cmrs_spmv_split_plan_bytes(const cmrs_mat_t* A, int32_t long_len, int32_t chunk_len) {
    if (!A || long_len < 0 || chunk_len < 0) return 0;
    if (check_mat(A) != CMRS_OK) return 0;
    return cmrs::split_shape(A, long_len, chunk_len).total;
}

cmrs_status_t cmrs_spmv_split_plan(const cmrs_mat_t* A, int32_t long_len, int32_t chunk_len, void* buf,
                                   size_t bytes, cmrs_split_plan_t* plan, hipStream_t stream) {
    g_last_error[0] = 0;
    cmrs_status_t st = check_mat(A);
    if (st != CMRS_OK) return st;
    if (long_len < 0 || chunk_len < 0)
        return fail(CMRS_ERR_INVALID_VALUE, "long_len %d / chunk_len %d negative", long_len, chunk_len);
    if (!plan) return fail(CMRS_ERR_INVALID_VALUE, "plan is NULL");
    const cmrs::SplitShape sh = cmrs::split_shape(A, long_len, chunk_len);
    if (!buf || bytes < sh.total || (reinterpret_cast<uintptr_t>(buf) & 15u))
        return fail(CMRS_ERR_WORKSPACE, "plan buffer of %zu bytes (16-byte aligned) needed, %zu given", sh.total,
                    bytes);
    st = from_hip(cmrs::launch_split_plan(A, sh, buf, stream), "cmrs_spmv_split_plan");
    if (st != CMRS_OK) return st;
    plan->rows = A->rows;
    plan->nnz = A->nnz;
    plan->height = A->height;
    plan->group = sh.group;
    plan->long_len = sh.long_len;
    plan->chunk_len = sh.chunk_len;
    plan->max_heavy = sh.max_heavy;
    plan->max_chunks = sh.max_chunks;
    plan->buf = buf;
    plan->bytes = bytes;
    return CMRS_OK;
}

cmrs_status_t cmrs_spmv_split(const cmrs_mat_t* A, const cmrs_split_plan_t* plan, const void* x, void* y,
                              cmrs_dtype_t xy_dtype, hipStream_t stream) {
    g_last_error[0] = 0;
    cmrs_status_t st = check_spmv_args(A, x, y, xy_dtype, CMRS_SPMV_AUTO);
    if (st != CMRS_OK) return st;
    if (!plan) return fail(CMRS_ERR_INVALID_VALUE, "plan is NULL");
    if (plan->rows != A->rows || plan->nnz != A->nnz || plan->height != A->height)
        return fail(CMRS_ERR_INVALID_VALUE, "plan built for rows=%d nnz=%d height=%d, matrix has %d/%d/%d", plan->rows,
                    plan->nnz, plan->height, A->rows, A->nnz, A->height);
    if (plan->long_len < 1 || plan->chunk_len < 1) return fail(CMRS_ERR_INVALID_VALUE, "corrupt plan");
    const cmrs::SplitShape sh = cmrs::split_shape(A, plan->long_len, plan->chunk_len);
    if (sh.group != plan->group || sh.max_heavy != plan->max_heavy || sh.max_chunks != plan->max_chunks)
        return fail(CMRS_ERR_INVALID_VALUE, "corrupt plan");
    if (!plan->buf || plan->bytes < sh.total || (reinterpret_cast<uintptr_t>(plan->buf) & 15u))
        return fail(CMRS_ERR_WORKSPACE, "plan buffer NULL, misaligned or below %zu bytes", sh.total);
    const size_t xs = cmrs::dtype_bytes(xy_dtype);
    if (ranges_overlap(plan->buf, sh.total, y, xs * static_cast<size_t>(A->rows)) ||
        ranges_overlap(plan->buf, sh.total, x, xs * static_cast<size_t>(A->cols)))
        return fail(CMRS_ERR_INVALID_VALUE, "plan buffer overlaps x or y");
    if (A->rows == 0) return CMRS_OK;
    return from_hip(cmrs::launch_spmv_split(A, sh, plan->buf, x, y, stream), "cmrs_spmv_split");
}

cmrs_status_t cmrs_spmv_colblock_noalloc(const cmrs_mat_t* A, const void* x, void* y, cmrs_dtype_t xy_dtype,
                                         int32_t variant, int32_t col_blocks, const int32_t* split,
                                         size_t split_bytes, hipStream_t stream) {
    g_last_error[0] = 0;
    cmrs_status_t st = check_spmv_args(A, x, y, xy_dtype, variant);
    if (st != CMRS_OK || A->rows == 0) return st;
    st = check_colblock(A, col_blocks, split, split_bytes);
    if (st != CMRS_OK) return st;
    const size_t need = cmrs_spmv_colblock_workspace(A, col_blocks, CMRS_COLBLOCK_CONCURRENT);
    if (need > CMRS_NOALLOC_SCRATCH_BYTES)
        return fail(CMRS_ERR_WORKSPACE, "%zu bytes of partial sums needed, the static scratch holds %u", need,
                    CMRS_NOALLOC_SCRATCH_BYTES);
    void* scratch = nullptr;
    if (need > 0) {
        st = from_hip(cmrs::noalloc_scratch(&scratch), "cmrs_spmv_colblock_noalloc (scratch address)");
        if (st != CMRS_OK) return st;
    }
    return from_hip(cmrs::launch_spmv_colblock(A, x, y, variant, col_blocks, split, CMRS_COLBLOCK_CONCURRENT, scratch,
                                               stream),
                    "cmrs_spmv_colblock_noalloc");
}

static bool dtype_pair_ok(cmrs_dtype_t val, cmrs_dtype_t xy) {
    return (val == CMRS_R64F && xy == CMRS_R64F) || (val == CMRS_R32F && xy == CMRS_R32F) ||
           (val == CMRS_R16BF && xy == CMRS_R32F);
}

static bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Bytes from the first to one past the last element of a row-major block of
// n rows, leading dimension ld, k used columns.
static size_t block_bytes(int32_t n, int32_t ld, int32_t k, size_t es) {
    if (n <= 0) return 0;
    return (static_cast<size_t>(n - 1) * static_cast<size_t>(ld) + static_cast<size_t>(k)) * es;
}

static cmrs_status_t check_spmm_one(const cmrs_mat_t* A, int32_t nrhs, const void* X, int32_t ldx, const void* Y,
                                    int32_t ldy, cmrs_dtype_t xy_dtype, int idx) {
    cmrs_status_t st = check_mat(A);
    if (st != CMRS_OK) return st;
    if (!dtype_pair_ok(A->val_dtype, xy_dtype))
        return fail(CMRS_ERR_NOT_SUPPORTED, "matrix %d: value dtype %d with X/Y dtype %d", idx, (int)A->val_dtype,
                    (int)xy_dtype);
    if (nrhs < 1 || nrhs > CMRS_SPMM_MAX_RHS)
        return fail(CMRS_ERR_INVALID_VALUE, "matrix %d: nrhs %d outside [1, %d]", idx, nrhs, CMRS_SPMM_MAX_RHS);
    if (ldx < nrhs || ldy < nrhs)
        return fail(CMRS_ERR_INVALID_VALUE, "matrix %d: ldx %d / ldy %d below nrhs %d", idx, ldx, ldy, nrhs);
    if (A->rows > 0 && !Y) return fail(CMRS_ERR_INVALID_VALUE, "matrix %d: Y is NULL", idx);
    if (A->nnz > 0 && A->cols > 0 && !X) return fail(CMRS_ERR_INVALID_VALUE, "matrix %d: X is NULL", idx);
    const size_t es = cmrs::dtype_bytes(xy_dtype);
    if (ranges_overlap(X, block_bytes(A->cols, ldx, nrhs, es), Y, block_bytes(A->rows, ldy, nrhs, es)))
        return fail(CMRS_ERR_INVALID_VALUE, "matrix %d: X and Y overlap", idx);
    return CMRS_OK;
}

cmrs_status_t cmrs_spmm(const cmrs_mat_t* A, int32_t nrhs, const void* X, int32_t ldx, void* Y, int32_t ldy,
                        cmrs_dtype_t xy_dtype, int32_t group, hipStream_t stream) {
    g_last_error[0] = 0;
    cmrs_status_t st = check_spmm_one(A, nrhs, X, ldx, Y, ldy, xy_dtype, 0);
    if (st != CMRS_OK) return st;
    if (group != 0 && (!is_pow2(group) || group > 64))
        return fail(CMRS_ERR_INVALID_VALUE, "group %d: need 0 or a power of two <= 64", group);
    if (!cmrs::spmm_fits(A->height, nrhs, A->val_dtype))
        return fail(CMRS_ERR_NOT_SUPPORTED, "height %d with %d right-hand sides needs more than 64 KiB of LDS per wave",
                    A->height, nrhs);
    if (A->rows == 0) return CMRS_OK;
    return from_hip(cmrs::launch_spmm(A, nrhs, X, ldx, Y, ldy, group, stream), "cmrs_spmm");
}

static cmrs_status_t check_tuning(const cmrs_spmm_tuning_t* t) {
    if (!t) return CMRS_OK;
    if (t->tile_nnz < 0) return fail(CMRS_ERR_INVALID_VALUE, "tile_nnz %d is negative", t->tile_nnz);
    if (t->group != 0 && (!is_pow2(t->group) || t->group > 64))
        return fail(CMRS_ERR_INVALID_VALUE, "group %d: need 0 or a power of two <= 64", t->group);
    if (t->blocks_per_cu < 0 || t->blocks_per_cu > 64)
        return fail(CMRS_ERR_INVALID_VALUE, "blocks_per_cu %d outside [0, 64]", t->blocks_per_cu);
    if (t->reserved != 0) return fail(CMRS_ERR_INVALID_VALUE, "reserved tuning field must be 0");
    return CMRS_OK;
}

static cmrs_status_t check_batch_shape(int32_t count, const cmrs_mat_t* mats, const int32_t* nrhs) {
    if (count < 0) return fail(CMRS_ERR_INVALID_VALUE, "negative count");
    if (count > 0 && (!mats || !nrhs)) return fail(CMRS_ERR_INVALID_VALUE, "mats or nrhs is NULL");
    for (int32_t i = 0; i < count; ++i) {
        cmrs_status_t st = check_mat(&mats[i]);
        if (st != CMRS_OK) return st;
        if (nrhs[i] < 1 || nrhs[i] > CMRS_SPMM_MAX_RHS)
            return fail(CMRS_ERR_INVALID_VALUE, "matrix %d: nrhs %d outside [1, %d]", i, nrhs[i], CMRS_SPMM_MAX_RHS);
        if (mats[i].val_dtype != mats[0].val_dtype)
            return fail(CMRS_ERR_NOT_SUPPORTED, "matrix %d: value dtype differs from matrix 0", i);
        if (!cmrs::spmm_fits(mats[i].height, nrhs[i], mats[i].val_dtype))
            return fail(CMRS_ERR_NOT_SUPPORTED, "matrix %d: height %d with %d right-hand sides needs more than 64 KiB "
                        "of LDS per wave", i, mats[i].height, nrhs[i]);
    }
    return CMRS_OK;
}

size_t cmrs_spmm_plan_bytes(int32_t count, const cmrs_mat_t* mats, const int32_t* nrhs,
                            const cmrs_spmm_tuning_t* tuning) {
    if (check_batch_shape(count, mats, nrhs) != CMRS_OK || check_tuning(tuning) != CMRS_OK) return 0;
    return cmrs::spmm_plan_shape(count, mats, nrhs, tuning ? tuning->tile_nnz : 0, tuning ? tuning->group : 0,
                                 nullptr)
        .bytes;
}

namespace {
struct Span {
    uintptr_t lo, hi;
    int idx;
};
}  // namespace

cmrs_status_t cmrs_spmm_plan(int32_t count, const cmrs_mat_t* mats, const int32_t* nrhs, const void* const* X,
                             const int32_t* ldx, void* const* Y, const int32_t* ldy, cmrs_dtype_t xy_dtype,
                             const cmrs_spmm_tuning_t* tuning, void* desc, size_t desc_bytes,
                             cmrs_spmm_plan_t* plan, hipStream_t stream) {
    g_last_error[0] = 0;
    cmrs_status_t st = check_batch_shape(count, mats, nrhs);
    if (st != CMRS_OK) return st;
    st = check_tuning(tuning);
    if (st != CMRS_OK) return st;
    if (!plan) return fail(CMRS_ERR_INVALID_VALUE, "plan is NULL");
    if (count > 0 && (!X || !ldx || !Y || !ldy)) return fail(CMRS_ERR_INVALID_VALUE, "X, ldx, Y or ldy is NULL");
    for (int32_t i = 0; i < count; ++i) {
        st = check_spmm_one(&mats[i], nrhs[i], X[i], ldx[i], Y[i], ldy[i], xy_dtype, i);
        if (st != CMRS_OK) return st;
    }
    // No Y may overlap another Y or any X.
    const size_t es = cmrs::dtype_bytes(xy_dtype);
    std::vector<Span> ys;
    for (int32_t i = 0; i < count; ++i) {
        const size_t n = block_bytes(mats[i].rows, ldy[i], nrhs[i], es);
        if (n) ys.push_back({reinterpret_cast<uintptr_t>(Y[i]), reinterpret_cast<uintptr_t>(Y[i]) + n, i});
    }
    std::sort(ys.begin(), ys.end(), [](const Span& a, const Span& b) { return a.lo < b.lo; });
    for (size_t i = 1; i < ys.size(); ++i)
        if (ys[i].lo < ys[i - 1].hi)
            return fail(CMRS_ERR_INVALID_VALUE, "Y of matrices %d and %d overlap", ys[i - 1].idx, ys[i].idx);
    for (int32_t j = 0; j < count && !ys.empty(); ++j) {
        const size_t n = block_bytes(mats[j].cols, ldx[j], nrhs[j], es);
        if (!n || mats[j].nnz == 0) continue;
        const uintptr_t lo = reinterpret_cast<uintptr_t>(X[j]), hi = lo + n;
        // First Y span ending after lo: the only candidate to intersect.
        auto it = std::upper_bound(ys.begin(), ys.end(), lo, [](uintptr_t v, const Span& s) { return v < s.hi; });
        if (it != ys.end() && it->lo < hi)
            return fail(CMRS_ERR_INVALID_VALUE, "X of matrix %d overlaps Y of matrix %d", j, it->idx);
    }
    const size_t need = cmrs_spmm_plan_bytes(count, mats, nrhs, tuning);
    if (!desc || desc_bytes < need)
        return fail(CMRS_ERR_WORKSPACE, "plan buffer of %zu bytes needed, %zu given", need, desc_bytes);
    if (reinterpret_cast<uintptr_t>(desc) & 15u) return fail(CMRS_ERR_INVALID_VALUE, "plan buffer not 16-byte aligned");
    return from_hip(cmrs::build_spmm_plan(count, mats, nrhs, X, ldx, Y, ldy, xy_dtype, tuning ? tuning->tile_nnz : 0,
                                          tuning ? tuning->group : 0, tuning ? tuning->blocks_per_cu : 0, desc, plan,
                                          stream),
                    "cmrs_spmm_plan");
}

cmrs_status_t cmrs_spmm_batched(const cmrs_spmm_plan_t* plan, hipStream_t stream) {
    g_last_error[0] = 0;
    if (!plan) return fail(CMRS_ERR_INVALID_VALUE, "plan is NULL");
    if (plan->tiles < 0 || plan->count < 0) return fail(CMRS_ERR_INVALID_VALUE, "corrupt plan");
    if (plan->tiles == 0) return CMRS_OK;
    const bool waves_ok = plan->grid >= 1 && plan->waves >= plan->grid && plan->waves <= 4 * plan->grid &&
                          plan->waves % plan->grid == 0;
    if (!plan->desc || !waves_ok || !is_pow2(plan->max_slots) || plan->max_slots > CMRS_MAX_HEIGHT * CMRS_SPMM_MAX_RHS ||
        !valid_dtype(static_cast<cmrs_dtype_t>(plan->val_dtype)) || plan->lds_bytes < 1 ||
        plan->lds_bytes > 65536 ||
        static_cast<size_t>(plan->lds_bytes) <
            static_cast<size_t>(plan->waves / plan->grid) * plan->max_slots * 64 * (plan->val_dtype == CMRS_R64F ? 8 : 4))
        return fail(CMRS_ERR_INVALID_VALUE, "corrupt plan");
    return from_hip(cmrs::launch_spmm_batched(plan, stream), "cmrs_spmm_batched");
}

int32_t cmrs_padded_bits(int32_t height) {
    if (height < 1 || height > CMRS_MAX_HEIGHT) return -1;
    int32_t b = 0;
    while ((1 << b) < height + 1) ++b;
    return b < 4 ? 4 : b;
}

size_t cmrs_padded_plan_workspace(int32_t rows, int32_t height) {
    if (rows < 0 || height < 1 || height > CMRS_MAX_HEIGHT) return 0;
    return cmrs::padded_workspace_layout(cmrs_num_strips(rows, height)).total;
}

cmrs_status_t cmrs_padded_plan(int32_t rows, int32_t nnz, const int32_t* row_ptr, int32_t height,
                               int32_t* strip_ptr_out, int64_t* padded_nnz_out, void* workspace,
                               size_t workspace_bytes, hipStream_t stream) {
    g_last_error[0] = 0;
    if (rows < 0 || nnz < 0) return fail(CMRS_ERR_INVALID_VALUE, "negative size");
    if (height < 1 || height > CMRS_MAX_HEIGHT)
        return fail(CMRS_ERR_INVALID_VALUE, "height %d outside [1, %d]", height, CMRS_MAX_HEIGHT);
    if (!size_fits(rows) || !size_fits(nnz))
        return fail(CMRS_ERR_INDEX_OVERFLOW, "rows=%d or nnz=%d above %d", rows, nnz, CMRS_MAX_INDEX);
    if (!row_ptr || !strip_ptr_out || !padded_nnz_out) return fail(CMRS_ERR_INVALID_VALUE, "NULL pointer");
    const size_t need = cmrs_padded_plan_workspace(rows, height);
    if (!workspace || workspace_bytes < need)
        return fail(CMRS_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, workspace_bytes);
    if (reinterpret_cast<uintptr_t>(workspace) & 7u) return fail(CMRS_ERR_INVALID_VALUE, "workspace not 8-byte aligned");
    const int strips = cmrs_num_strips(rows, height);
    cmrs_status_t st = from_hip(cmrs::launch_padded_count(rows, height, row_ptr, workspace, stream), "cmrs_padded_plan");
    if (st != CMRS_OK) return st;
    long long chunks = 0;
    st = from_hip(hipMemcpyAsync(&chunks, cmrs::padded_total_ptr(strips, workspace), sizeof(chunks),
                                 hipMemcpyDeviceToHost, stream),
                  "cmrs_padded_plan");
    if (st == CMRS_OK) st = from_hip(hipStreamSynchronize(stream), "cmrs_padded_plan");
    if (st != CMRS_OK) return st;
    const long long padded = chunks * 64;
    *padded_nnz_out = padded;
    if (!size_fits(padded))
        return fail(CMRS_ERR_INDEX_OVERFLOW, "padded matrix would hold %lld entries, above %d", padded,
                    CMRS_MAX_INDEX);
    return from_hip(cmrs::launch_padded_strip_ptr(strips, workspace, strip_ptr_out, stream), "cmrs_padded_plan");
}

cmrs_status_t cmrs_padded_from_csr(int32_t rows, int32_t cols, int32_t nnz, const int32_t* row_ptr,
                                   const int32_t* col_ind, const void* val_in, cmrs_dtype_t dtype, int32_t height,
                                   const int32_t* strip_ptr, int32_t padded_nnz, uint32_t* col_word_out,
                                   void* val_out, hipStream_t stream) {
    g_last_error[0] = 0;
    if (rows < 0 || cols < 0 || nnz < 0 || padded_nnz < 0) return fail(CMRS_ERR_INVALID_VALUE, "negative size");
    if (height < 1 || height > CMRS_MAX_HEIGHT)
        return fail(CMRS_ERR_INVALID_VALUE, "height %d outside [1, %d]", height, CMRS_MAX_HEIGHT);
    if (!valid_dtype(dtype)) return fail(CMRS_ERR_INVALID_VALUE, "unknown dtype %d", (int)dtype);
    if (!size_fits(rows) || !size_fits(padded_nnz))
        return fail(CMRS_ERR_INDEX_OVERFLOW, "rows=%d or padded_nnz=%d above %d", rows, padded_nnz, CMRS_MAX_INDEX);
    if (padded_nnz < nnz || padded_nnz % 64) return fail(CMRS_ERR_INVALID_VALUE, "padded_nnz %d is not a plan's size", padded_nnz);
    const int32_t bits = cmrs_padded_bits(height);
    if (!cols_fit(cols, bits)) return fail(CMRS_ERR_INDEX_OVERFLOW, "cols=%d does not fit %d column bits", cols, 32 - bits);
    if (!row_ptr || !strip_ptr) return fail(CMRS_ERR_INVALID_VALUE, "row_ptr or strip_ptr is NULL");
    if (padded_nnz > 0 && (!col_ind || !val_in || !col_word_out || !val_out))
        return fail(CMRS_ERR_INVALID_VALUE, "an entry array is NULL");
    const size_t es = cmrs::dtype_bytes(dtype);
    const size_t pz = static_cast<size_t>(padded_nnz), nz = static_cast<size_t>(nnz);
    if (ranges_overlap(col_word_out, 4 * pz, col_ind, 4 * nz) || ranges_overlap(val_out, es * pz, val_in, es * nz) ||
        ranges_overlap(col_word_out, 4 * pz, val_in, es * nz) || ranges_overlap(val_out, es * pz, col_ind, 4 * nz) ||
        ranges_overlap(col_word_out, 4 * pz, val_out, es * pz))
        return fail(CMRS_ERR_INVALID_VALUE, "outputs overlap inputs or each other");
    if (rows == 0 || padded_nnz == 0) return CMRS_OK;
    return from_hip(cmrs::launch_padded_fill(rows, height, bits, row_ptr, col_ind, val_in, dtype, strip_ptr,
                                             col_word_out, val_out, stream),
                    "cmrs_padded_from_csr");
}

cmrs_status_t cmrs_padded_spmv(const cmrs_mat_t* A, const void* x, void* y, cmrs_dtype_t xy_dtype,
                               hipStream_t stream) {
    g_last_error[0] = 0;
    if (!A) return fail(CMRS_ERR_INVALID_VALUE, "matrix descriptor is NULL");
    if (A->height < 1 || A->height > CMRS_MAX_HEIGHT || A->bits != cmrs_padded_bits(A->height))
        return fail(CMRS_ERR_INVALID_VALUE, "height %d / bits %d are not a padded matrix's", A->height, A->bits);
    cmrs_mat_t plain = *A;
    plain.bits = cmrs_bits_for_height(A->height);
    if (!cols_fit(A->cols, A->bits))
        return fail(CMRS_ERR_INDEX_OVERFLOW, "cols=%d does not fit %d column bits", A->cols, 32 - A->bits);
    if (A->nnz % 64) return fail(CMRS_ERR_INVALID_VALUE, "nnz %d of a padded matrix is not a multiple of 64", A->nnz);
    if (A->nnz > 0 && A->cols < 1) return fail(CMRS_ERR_INVALID_VALUE, "entries but no columns");
    cmrs_status_t st = check_spmv_args(&plain, x, y, xy_dtype, CMRS_SPMV_AUTO);
    if (st != CMRS_OK || A->rows == 0) return st;
    return from_hip(cmrs::launch_padded_spmv(A, x, y, stream), "cmrs_padded_spmv");
}

cmrs_status_t cmrs_validate_csr(int32_t rows, int32_t cols, int32_t nnz, const int32_t* row_ptr,
                                const int32_t* col_ind, int32_t* flag_out, hipStream_t stream) {
    g_last_error[0] = 0;
    if (rows < 0 || cols < 0 || nnz < 0) return fail(CMRS_ERR_INVALID_VALUE, "negative size");
    if (!size_fits(rows) || !size_fits(nnz))
        return fail(CMRS_ERR_INDEX_OVERFLOW, "rows=%d or nnz=%d above %d", rows, nnz, CMRS_MAX_INDEX);
    if (!row_ptr || !flag_out || (nnz > 0 && !col_ind)) return fail(CMRS_ERR_INVALID_VALUE, "NULL pointer");
    return from_hip(cmrs::launch_validate_csr(rows, cols, nnz, row_ptr, col_ind, flag_out, stream),
                    "cmrs_validate_csr");
}

cmrs_status_t cmrs_calib_stream_read(const uint32_t* col_word, const void* val, int32_t nnz, cmrs_dtype_t dtype,
                                     int32_t lds_words_per_lane, double* sink, hipStream_t stream) {
    g_last_error[0] = 0;
    if (nnz < 0 || !valid_dtype(dtype) || lds_words_per_lane < 0 || lds_words_per_lane > 32 || !sink)
        return fail(CMRS_ERR_INVALID_VALUE, "bad calibration arguments");
    if (nnz > 0 && (!col_word || !val)) return fail(CMRS_ERR_INVALID_VALUE, "NULL array");
    if ((reinterpret_cast<uintptr_t>(col_word) | reinterpret_cast<uintptr_t>(val)) & 15u)
        return fail(CMRS_ERR_INVALID_VALUE, "arrays must be 16-byte aligned");
    return from_hip(cmrs::launch_calib_stream(col_word, val, nnz, dtype, lds_words_per_lane, sink, stream),
                    "cmrs_calib_stream_read");
}

cmrs_status_t cmrs_calib_gather(const uint32_t* idx, int64_t n, const void* x, cmrs_dtype_t x_dtype, double* sink,
                                hipStream_t stream) {
    g_last_error[0] = 0;
    if (n < 0 || n > 0x7fffffff || (x_dtype != CMRS_R64F && x_dtype != CMRS_R32F) || !sink)
        return fail(CMRS_ERR_INVALID_VALUE, "bad calibration arguments");
    if (n > 0 && (!idx || !x)) return fail(CMRS_ERR_INVALID_VALUE, "NULL array");
    return from_hip(cmrs::launch_calib_gather(idx, n, x, x_dtype, sink, stream), "cmrs_calib_gather");
}

cmrs_status_t cmrs_features(int32_t rows, int32_t cols, int32_t nnz, const int32_t* row_ptr, const int32_t* col_ind,
                            float* feat_out, void* workspace, size_t workspace_bytes, hipStream_t stream) {
    g_last_error[0] = 0;
    if (rows < 0 || cols < 0 || nnz < 0) return fail(CMRS_ERR_INVALID_VALUE, "negative size");
    if (!size_fits(rows) || !size_fits(nnz))
        return fail(CMRS_ERR_INDEX_OVERFLOW, "rows=%d or nnz=%d above %d", rows, nnz, CMRS_MAX_INDEX);
    if (!row_ptr || !feat_out || (nnz > 0 && !col_ind)) return fail(CMRS_ERR_INVALID_VALUE, "NULL pointer");
    if (!workspace || workspace_bytes < CMRS_SEL_FEATURE_WS)
        return fail(CMRS_ERR_WORKSPACE, "workspace of %d bytes needed", CMRS_SEL_FEATURE_WS);
    return from_hip(cmrs::launch_features(rows, cols, nnz, row_ptr, col_ind, feat_out, static_cast<int*>(workspace),
                                          stream),
                    "cmrs_features");
}

cmrs_status_t cmrs_mlp_forward(int32_t batch, const float* X, const float* params, float* H1, float* H2, float* Y,
                               hipStream_t stream) {
    g_last_error[0] = 0;
    if (batch < 0) return fail(CMRS_ERR_INVALID_VALUE, "negative batch");
    if (batch == 0) return CMRS_OK;
    if (!X || !params || !H1 || !H2 || !Y) return fail(CMRS_ERR_INVALID_VALUE, "NULL pointer");
    return from_hip(cmrs::launch_mlp_forward(batch, X, params, H1, H2, Y, stream), "cmrs_mlp_forward");
}

cmrs_status_t cmrs_mlp_backward(int32_t batch, const float* X, const float* params, const float* H1, const float* H2,
                                const float* dY, float* dH2, float* dH1, float* grads, hipStream_t stream) {
    g_last_error[0] = 0;
    if (batch <= 0) return fail(CMRS_ERR_INVALID_VALUE, "batch must be positive");
    if (!X || !params || !H1 || !H2 || !dY || !dH2 || !dH1 || !grads) return fail(CMRS_ERR_INVALID_VALUE, "NULL pointer");
    return from_hip(cmrs::launch_mlp_backward(batch, X, params, H1, H2, dY, dH2, dH1, grads, stream),
                    "cmrs_mlp_backward");
}

cmrs_status_t cmrs_mse_grad(int32_t n, const float* Y, const float* T, float* dY, float scale, hipStream_t stream) {
    g_last_error[0] = 0;
    if (n < 0) return fail(CMRS_ERR_INVALID_VALUE, "negative size");
    if (n == 0) return CMRS_OK;
    if (!Y || !T || !dY) return fail(CMRS_ERR_INVALID_VALUE, "NULL pointer");
    return from_hip(cmrs::launch_mse_grad(n, Y, T, dY, scale, stream), "cmrs_mse_grad");
}

cmrs_status_t cmrs_adam_step(int32_t n, float* params, const float* grads, float* m, float* v, float lr, float beta1,
                             float beta2, float eps, int32_t step, hipStream_t stream) {
    g_last_error[0] = 0;
    if (n < 0 || step < 1) return fail(CMRS_ERR_INVALID_VALUE, "bad size or step");
    if (n == 0) return CMRS_OK;
    if (!params || !grads || !m || !v) return fail(CMRS_ERR_INVALID_VALUE, "NULL pointer");
    return from_hip(cmrs::launch_adam(n, params, grads, m, v, lr, beta1, beta2, eps, step, stream), "cmrs_adam_step");
}

const char* cmrs_status_string(cmrs_status_t s) {
    switch (s) {
        case CMRS_OK: return "CMRS_OK";
        case CMRS_ERR_INVALID_VALUE: return "CMRS_ERR_INVALID_VALUE";
        case CMRS_ERR_INDEX_OVERFLOW: return "CMRS_ERR_INDEX_OVERFLOW";
        case CMRS_ERR_NOT_SUPPORTED: return "CMRS_ERR_NOT_SUPPORTED";
        case CMRS_ERR_DEVICE: return "CMRS_ERR_DEVICE";
        case CMRS_ERR_WORKSPACE: return "CMRS_ERR_WORKSPACE";
    }
    return "CMRS_UNKNOWN_STATUS";
}

const char* cmrs_last_error(void) { return g_last_error; }

}  // extern "C"
