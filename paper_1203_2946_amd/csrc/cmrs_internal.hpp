// Host-side declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "cmrs.h"

namespace cmrs {

inline int next_pow2(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

inline size_t dtype_bytes(cmrs_dtype_t t) {
    switch (t) {
        case CMRS_R64F: return 8;
        case CMRS_R32F: return 4;
        case CMRS_R16BF: return 2;
    }
    return 0;
}

// Strips that one wave sorts in its LDS slice (sorted conversion), and the
// largest strip a 1024-thread workgroup sorts in LDS; longer strips are
// sorted in the global workspace.
constexpr int kWaveSortCap = 1024;
constexpr int kBlockSortCap = 16384;

struct FromCsrWorkspaceLayout {
    size_t small_off;   // int32 counts at offset 0 (short / long list), short-strip list at small_off
    size_t small_cap;
    size_t big_off;     // long-strip list
    size_t big_cap;
    size_t global_off;  // uint64 sort area: 2*nnz entries
    size_t total;
};
FromCsrWorkspaceLayout from_csr_workspace_layout(int32_t rows, int32_t nnz, int32_t height);

// Shape of the conversion group kernels: G lanes per strip and E = 8 entries
// per lane, so that a group holds about 2.5 times the average strip where it
// can (most strips then fit and take the fast path); G at least hb, since the strip's row
// pointers sit one per lane of the group.
struct ConvShape {
    int g, e;
};
inline ConvShape conv_shape(int nnz, int strips, int hb) {
    const double want = strips > 0 ? 2.5 * static_cast<double>(nnz) / strips : 0.0;
    ConvShape s{2, 8};
    while (s.g < 64 && s.g * s.e < want) s.g <<= 1;
    if (s.g < hb) s.g = hb;
    if (s.g < 2) s.g = 2;
    return s;
}

hipError_t launch_from_csr(int32_t rows, int32_t cols, int32_t nnz, const int32_t* row_ptr,
                           const int32_t* col_ind, const void* val_in, cmrs_dtype_t dtype, int32_t height,
                           int32_t bits, uint32_t flags, int32_t* strip_ptr, uint32_t* col_word, void* val_out,
                           void* workspace, hipStream_t stream);

hipError_t launch_to_csr(const cmrs_mat_t* A, int32_t* row_ptr, int32_t* col_ind, void* val_out,
                         hipStream_t stream);

hipError_t launch_spmv(const cmrs_mat_t* A, const void* x, void* y, cmrs_dtype_t xy_dtype, int variant,
                       hipStream_t stream);
int resolve_spmv_variant(const cmrs_mat_t* A, int variant);
hipError_t launch_colblock_plan(const cmrs_mat_t* A, int nb, int bw, int* split, hipStream_t stream);
hipError_t launch_spmv_colblock(const cmrs_mat_t* A, const void* x, void* y, int variant, int nb, const int* split,
                                int schedule, void* workspace, hipStream_t stream);

hipError_t launch_calib_stream(const void* word, const void* val, int32_t nnz, cmrs_dtype_t dtype,
                               int32_t lds_words_per_lane, double* sink, hipStream_t stream);
hipError_t launch_calib_gather(const uint32_t* idx, int64_t n, const void* x, cmrs_dtype_t dtype, double* sink,
                               hipStream_t stream);

hipError_t launch_features(int rows, int cols, int nnz, const int* row_ptr, const int* col_ind, float* feat,
                           int* ws, hipStream_t stream);
hipError_t launch_mlp_forward(int batch, const float* X, const float* params, float* H1, float* H2, float* Y,
                              hipStream_t stream);
hipError_t launch_mlp_backward(int batch, const float* X, const float* params, const float* H1, const float* H2,
                               const float* dY, float* dH2, float* dH1, float* grads, hipStream_t stream);
hipError_t launch_mse_grad(int n, const float* Y, const float* T, float* dY, float scale, hipStream_t stream);
hipError_t launch_adam(int n, float* p, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
                       int step, hipStream_t stream);

// Multi-right-hand-side products: one matrix as the kernels see it, and the
// work tiles (a matrix and a half-open range of its strips) of a batch plan.
struct alignas(16) SpmmMat {
    const int32_t* strip_ptr;
    const uint32_t* word;
    const void* val;
    const void* x;
    void* y;
    int32_t rows, height, bits, nrhs;
    int32_t ldx, ldy, hb, rb_log;     // hb = next_pow2(height), 2^rb_log = next_pow2(nrhs)
    int32_t g_log, pad0, pad1, pad2;  // 2^g_log entry slots per strip
};
struct SpmmTile {
    int32_t mat, s0, s1, pad;
};
struct SpmmPlanShape {
    int tiles;
    int max_slots;  // largest next_pow2(height) * next_pow2(nrhs) of the batch
    size_t bytes;
};
constexpr size_t kSpmmHeaderBytes = 1024;  // 8 per-XCD queue counters + done counter, 64 B apart

size_t spmm_wave_lds_bytes(int slots, size_t acc_bytes);
int spmm_waves_per_block(size_t wave_bytes);
bool spmm_fits(int height, int nrhs, cmrs_dtype_t val_dtype);
SpmmMat spmm_mat(const cmrs_mat_t* A, int nrhs, const void* X, int ldx, void* Y, int ldy, int group);
SpmmPlanShape spmm_plan_shape(int count, const cmrs_mat_t* mats, const int* nrhs, int tile_nnz, int group,
                              std::vector<SpmmTile>* tiles_out);
hipError_t launch_spmm(const cmrs_mat_t* A, int nrhs, const void* X, int ldx, void* Y, int ldy, int group,
                       hipStream_t stream);
hipError_t build_spmm_plan(int count, const cmrs_mat_t* mats, const int* nrhs, const void* const* X, const int* ldx,
                           void* const* Y, const int* ldy, cmrs_dtype_t xy_dtype, int tile_nnz, int group,
                           int blocks_per_cu, void* desc, cmrs_spmm_plan_t* plan, hipStream_t stream);
hipError_t launch_spmm_batched(const cmrs_spmm_plan_t* plan, hipStream_t stream);

// Modified CMRS of Sec. 6.7 (padded strips): conversion workspace, int64
// chunk counts, their prefix sums and the scan's block totals.
struct PaddedWorkspaceLayout {
    int nb;
    size_t chunks_off, prefix_off, bsum_off, total;
};
PaddedWorkspaceLayout padded_workspace_layout(int strips);
hipError_t launch_padded_count(int rows, int height, const int* row_ptr, void* workspace, hipStream_t stream);
const long long* padded_total_ptr(int strips, const void* workspace);
hipError_t launch_padded_strip_ptr(int strips, const void* workspace, int32_t* strip_ptr, hipStream_t stream);
hipError_t launch_padded_fill(int rows, int height, int bits, const int* row_ptr, const int* col_ind,
                              const void* val_in, cmrs_dtype_t dtype, const int* strip_ptr, uint32_t* word_out,
                              void* val_out, hipStream_t stream);
hipError_t launch_padded_spmv(const cmrs_mat_t* A, const void* x, void* y, hipStream_t stream);

hipError_t launch_validate_csr(int32_t rows, int32_t cols, int32_t nnz, const int32_t* row_ptr,
                               const int32_t* col_ind, int32_t* flag, hipStream_t stream);

}  // namespace cmrs
