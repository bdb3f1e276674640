// Host-side declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

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
// can (most strips then fit and take the fast path), 1.25 times at heights
// 3-8 (more strips per wave; measured on 2^20 Poisson(16) rows: 154 -> 147 us
// at h = 4, 182 -> 167 us at h = 8, slower at h = 1-2); G at least hb, since
// the strip's row pointers sit one per lane of the group.
struct ConvShape {
    int g, e;
};
inline ConvShape conv_shape(int nnz, int strips, int hb) {
    const double per = (hb >= 4 && hb <= 8) ? 1.25 : 2.5;
    const double want = strips > 0 ? per * static_cast<double>(nnz) / strips : 0.0;
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
// Lanes per strip of the strip-group SpMV: about 8 entries per lane for the
// average strip, at least hb (next_pow2 of the height), a power of two <= 64.
int spmv_group_width(int nnz, int strips, int hb);
int resolve_spmv_variant(const cmrs_mat_t* A, int variant);
hipError_t launch_colblock_plan(const cmrs_mat_t* A, int nb, int bw, int* split, hipStream_t stream);
hipError_t launch_spmv_colblock(const cmrs_mat_t* A, const void* x, void* y, int variant, int nb, const int* split,
                                int schedule, void* workspace, hipStream_t stream);
hipError_t launch_spmv_phased(const cmrs_mat_t* A, const void* x, void* y, int nb, const int* split,
                              hipStream_t stream);
// Device address of this GPU's CMRS_NOALLOC_SCRATCH_BYTES scratch array
// (looked up once per device, with that device current).
hipError_t noalloc_scratch(void** ptr);

hipError_t launch_calib_stream(const void* word, const void* val, int32_t nnz, cmrs_dtype_t dtype,
                               int32_t lds_words_per_lane, double* sink, hipStream_t stream);
hipError_t launch_calib_gather(const uint32_t* idx, int64_t n, const void* x, cmrs_dtype_t dtype, double* sink,
                               hipStream_t stream);

hipError_t launch_validate_csr(int32_t rows, int32_t cols, int32_t nnz, const int32_t* row_ptr,
                               const int32_t* col_ind, int32_t* flag, hipStream_t stream);

}  // namespace cmrs
