// Host-side declarations of the extension kernels: several right-hand sides
// and batches, the padded layout of Sec. 6.7 and the learned selector.
#pragma once

#include <algorithm>
#include <vector>

#include "cmrs_internal.hpp"

namespace cmrs {

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
    int32_t g_log;                    // 2^g_log entry slots per strip
    int32_t pad0;
    int32_t nnz;                      // stored entries (strip_ptr[strips])
    int32_t pad;
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

// Split schedule for skewed strips: a heavy strip's entry in the plan, one
// chunk of it, and the plan's sizes and buffer layout.
struct SplitHeavy {
    int32_t strip, first, nchunks, pad;
};
struct SplitChunk {
    int32_t heavy, lo, hi, pad;
};
constexpr int kSplitU = 8;  // entries per lane in flight (stream loads, then gathers)
struct SplitShape {
    int group, long_len, chunk_len, max_heavy, max_chunks;
    size_t block_off, heavy_off, chunk_off, partial_off, total;
};
SplitShape split_shape(const cmrs_mat_t* A, int long_len, int chunk_len);
hipError_t launch_split_plan(const cmrs_mat_t* A, const SplitShape& s, void* buf, hipStream_t stream);
hipError_t launch_spmv_split(const cmrs_mat_t* A, const SplitShape& s, const void* buf, const void* x, void* y,
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

}  // namespace cmrs
