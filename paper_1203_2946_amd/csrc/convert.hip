// CSR <-> CMRS conversion kernels and the CSR validity check (gfx950).
//
// CSR -> CMRS follows Sec. 3 and 4 of Koza et al. (arXiv:1203.2946):
//   StripPtr[j] = RowPtr[j*height], StripPtr[strips] = nnz;
//   word[k] = (ColInd[k] << bits) | (row(k) mod height);
//   optionally every strip reordered by (column, RowInStrip), ties in CSR
//   order (Sec. 4, fourth optimisation).
// CMRS -> CSR is the inverse: per-row counts inside a strip give RowPtr (no
// global scan is needed, a strip's entries are exactly its rows' entries), and
// a stable scatter by RowInStrip restores row order.
//
// Work split: one 64-lane wave per strip.  The strip's height+1 row pointers
// sit one per lane; the row of an entry is found with a binary search over
// those lanes (cross-lane reads, no memory traffic).  Reordering sorts 64-bit
// keys (word << 32 | position in strip), which makes the sort stable, with a
// bitonic network: in the wave's LDS slice for strips of up to 1024 entries, in
// a 1024-thread workgroup's LDS for up to 16384, in the workspace beyond that.
#include <limits.h>

#include "cmrs_device.hpp"
#include "cmrs_internal.hpp"

namespace cmrs {

constexpr int kConvWaves = 4;
constexpr int kConvThreads = kConvWaves * kWave;
constexpr int kBlockSortThreads = 1024;

__global__ void set_int_kernel(int32_t* p, int32_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// Sec. 3: StripPtr[j] = RowPtr[j*height] for j < strips, StripPtr[strips] = nnz.
__global__ void strip_ptr_kernel(int strips, int height, int nnz, const int* __restrict__ row_ptr,
                                 int* __restrict__ strip_ptr) {
    const int j = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x);
    if (j < strips)
        strip_ptr[j] = row_ptr[j * height];
    else if (j == strips)
        strip_ptr[j] = nnz;
}

// Lane t (t <= nr) holds rp_t = RowPtr[first row of the strip + t]; lanes
// above nr hold INT_MAX.  Returns the largest t with rp_t <= e, i.e. the
// RowInStrip of entry e (empty rows are skipped because their rp_t repeats).
// All lanes of the wave must be active.
template <int HB>
__device__ inline int row_in_strip(int myrp, int e) {
    int lo = 0;
#pragma unroll
    for (int step = HB / 2; step >= 1; step >>= 1) {
        const int v = __shfl(myrp, lo + step);
        if (v <= e) lo += step;
    }
    return lo;
}

struct StripRows {
    int r0, nr, myrp, s0, s1;
};

// Row pointers of strip `strip` spread over the wave's lanes.
__device__ inline StripRows load_strip_rows(int strip, int rows, int height, const int* __restrict__ row_ptr,
                                            int lane) {
    StripRows s;
    s.r0 = strip * height;
    s.nr = min(height, rows - s.r0);
    s.myrp = lane <= s.nr ? row_ptr[s.r0 + lane] : INT_MAX;
    s.s0 = __shfl(s.myrp, 0);
    s.s1 = __shfl(s.myrp, s.nr);
    return s;
}

// Unsorted conversion.  col_word may alias col_ind (in place); val_out may
// alias val_in, in which case copy_val is 0.
template <int HB, typename ET>
__global__ __launch_bounds__(kConvThreads) void pack_kernel(int rows, int strips, int height, int bits,
                                                            const int* __restrict__ row_ptr, const int* col_ind,
                                                            const ET* val_in, uint32_t* col_word, ET* val_out,
                                                            int copy_val) {
    const int lane = lane_id();
    const int wave = uniform(static_cast<int>(threadIdx.x) / kWave);
    const int strip = xcd_logical_block(blockIdx.x, gridDim.x) * kConvWaves + wave;
    if (strip >= strips) return;
    const StripRows sr = load_strip_rows(strip, rows, height, row_ptr, lane);
    for (int base = sr.s0; base < sr.s1; base += kWave) {
        const int e = base + lane;
        const int r = row_in_strip<HB>(sr.myrp, e);
        if (e < sr.s1) {
            const uint32_t c = static_cast<uint32_t>(col_ind[e]);
            col_word[e] = (c << bits) | static_cast<uint32_t>(r);
            if (copy_val) val_out[e] = val_in[e];
        }
    }
}

__device__ inline int pow2_at_least(int n) {
    int p = 1;
    while (p < n) p <<= 1;
    return n == 0 ? 0 : p;
}

// Ascending bitonic network over keys k[0..P), P a power of two, run by
// `nthreads` threads numbered `tid`; `sync` orders the passes.
template <typename Sync>
__device__ inline void bitonic_sort(uint64_t* k, int P, int tid, int nthreads, Sync sync) {
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = tid; t < P / 2; t += nthreads) {
                const int i = ((t & ~(stride - 1)) << 1) | (t & (stride - 1));
                const int l = i + stride;
                const bool up = (i & size) == 0;
                const uint64_t a = k[i], b = k[l];
                if ((a > b) == up) {
                    k[i] = b;
                    k[l] = a;
                }
            }
            sync();
        }
    }
}

// Sorted conversion, one wave per strip of at most kWaveSortCap entries;
// longer strips are appended to the workspace list for the block kernel.
template <int HB, typename ET>
__global__ __launch_bounds__(kConvThreads) void sort_strips_wave_kernel(
    int rows, int strips, int height, int bits, const int* __restrict__ row_ptr, const int* __restrict__ col_ind,
    const ET* __restrict__ val_in, uint32_t* __restrict__ col_word, ET* __restrict__ val_out,
    int* __restrict__ ws_count, int* __restrict__ ws_list) {
    __shared__ uint64_t keys[kConvWaves][kWaveSortCap];
    const int lane = lane_id();
    const int wave = uniform(static_cast<int>(threadIdx.x) / kWave);
    const int strip = xcd_logical_block(blockIdx.x, gridDim.x) * kConvWaves + wave;
    if (strip >= strips) return;
    const StripRows sr = load_strip_rows(strip, rows, height, row_ptr, lane);
    const int n = sr.s1 - sr.s0;
    if (n > kWaveSortCap) {
        if (lane == 0) ws_list[atomicAdd(ws_count, 1)] = strip;
        return;
    }
    uint64_t* k = keys[wave];
    const int P = pow2_at_least(n);
    for (int base = 0; base < P; base += kWave) {
        const int i = base + lane;
        const int r = row_in_strip<HB>(sr.myrp, sr.s0 + i);
        if (i < n) {
            const uint32_t w = (static_cast<uint32_t>(col_ind[sr.s0 + i]) << bits) | static_cast<uint32_t>(r);
            k[i] = (static_cast<uint64_t>(w) << 32) | static_cast<uint32_t>(i);
        } else if (i < P) {
            k[i] = ~0ull;
        }
    }
    wave_lds_sync();
    bitonic_sort(k, P, lane, kWave, [] { wave_lds_sync(); });
    for (int i = lane; i < n; i += kWave) {
        const uint64_t kk = k[i];
        col_word[sr.s0 + i] = static_cast<uint32_t>(kk >> 32);
        val_out[sr.s0 + i] = val_in[sr.s0 + static_cast<int>(static_cast<uint32_t>(kk))];
    }
}

// Sorted conversion of the long strips listed by the wave kernel: one
// 1024-thread workgroup per strip, strips taken in a grid-stride loop.
template <int HB, typename ET>
__global__ __launch_bounds__(kBlockSortThreads) void sort_strips_block_kernel(
    int rows, int height, int bits, const int* __restrict__ row_ptr, const int* __restrict__ col_ind,
    const ET* __restrict__ val_in, uint32_t* __restrict__ col_word, ET* __restrict__ val_out,
    const int* __restrict__ ws_count, const int* __restrict__ ws_list, uint64_t* __restrict__ gkeys) {
    __shared__ uint64_t skeys[kBlockSortCap];
    const int lane = lane_id();
    const int wave = static_cast<int>(threadIdx.x) / kWave;
    const int count = *ws_count;
    for (int item = blockIdx.x; item < count; item += gridDim.x) {
        const int strip = ws_list[item];
        const StripRows sr = load_strip_rows(strip, rows, height, row_ptr, lane);
        const int n = sr.s1 - sr.s0;
        const int P = pow2_at_least(n);
        const bool in_lds = n <= kBlockSortCap;
        // P <= 2n, so [2*s0, 2*s0 + P) lies inside this strip's own slice [2*s0, 2*s1).
        uint64_t* k = in_lds ? skeys : gkeys + 2 * static_cast<size_t>(sr.s0);
        for (int base = wave * kWave; base < P; base += kBlockSortThreads) {
            const int i = base + lane;
            const int r = row_in_strip<HB>(sr.myrp, sr.s0 + i);
            if (i < n) {
                const uint32_t w = (static_cast<uint32_t>(col_ind[sr.s0 + i]) << bits) | static_cast<uint32_t>(r);
                k[i] = (static_cast<uint64_t>(w) << 32) | static_cast<uint32_t>(i);
            } else if (i < P) {
                k[i] = ~0ull;
            }
        }
        if (in_lds) {
            __syncthreads();
            bitonic_sort(k, P, static_cast<int>(threadIdx.x), kBlockSortThreads, [] { __syncthreads(); });
        } else {
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
            __syncthreads();
            bitonic_sort(k, P, static_cast<int>(threadIdx.x), kBlockSortThreads, [] {
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
                __syncthreads();
            });
        }
        for (int i = static_cast<int>(threadIdx.x); i < n; i += kBlockSortThreads) {
            const uint64_t kk = k[i];
            col_word[sr.s0 + i] = static_cast<uint32_t>(kk >> 32);
            val_out[sr.s0 + i] = val_in[sr.s0 + static_cast<int>(static_cast<uint32_t>(kk))];
        }
        __syncthreads();  // the next item reuses skeys
    }
}

// CMRS -> CSR, one wave per strip.
template <int HB, typename ET>
__global__ __launch_bounds__(kConvThreads) void to_csr_kernel(int rows, int strips, int height, int bits,
                                                              const int* __restrict__ strip_ptr,
                                                              const uint32_t* __restrict__ word,
                                                              const ET* __restrict__ val, int* __restrict__ row_ptr,
                                                              int* __restrict__ col_ind, ET* __restrict__ val_out) {
    const int lane = lane_id();
    const int wave = uniform(static_cast<int>(threadIdx.x) / kWave);
    const int strip = xcd_logical_block(blockIdx.x, gridDim.x) * kConvWaves + wave;
    if (strip >= strips) return;
    const int r0 = strip * height;
    const int nr = min(height, rows - r0);
    const int s0 = strip_ptr[strip], s1 = strip_ptr[strip + 1];
    const uint32_t mask = (1u << bits) - 1u;

    // Pass 1: lane t counts the entries whose RowInStrip is t.
    int cnt = 0;
    for (int base = s0; base < s1; base += kWave) {
        const int e = base + lane;
        const uint32_t r = e < s1 ? (word[e] & mask) : 0xffffffffu;
#pragma unroll
        for (int t = 0; t < HB; ++t) {
            const uint64_t m = ballot(r == static_cast<uint32_t>(t));
            if (lane == t) cnt += __popcll(m);
        }
    }
    // Exclusive prefix over lanes: the CSR position of each row's first entry.
    int incl = cnt;
#pragma unroll
    for (int off = 1; off < HB; off <<= 1) {
        const int v = __shfl_up(incl, off);
        if (lane >= off) incl += v;
    }
    const int start = s0 + incl - cnt;
    if (lane < nr) row_ptr[r0 + lane] = start;
    if (strip == strips - 1 && lane == 0) row_ptr[rows] = s1;

    // Pass 2: stable scatter; lane t tracks the next free slot of row t.
    int next = start;
    for (int base = s0; base < s1; base += kWave) {
        const int e = base + lane;
        const bool act = e < s1;
        const uint32_t w = act ? word[e] : 0u;
        const uint32_t r = act ? (w & mask) : 0xffffffffu;
        int pos = 0;
#pragma unroll
        for (int t = 0; t < HB; ++t) {
            const uint64_t m = ballot(r == static_cast<uint32_t>(t));
            const int base_t = __shfl(next, t);
            if (r == static_cast<uint32_t>(t)) pos = base_t + __popcll(m & lanemask_lt());
            if (lane == t) next += __popcll(m);
        }
        if (act) {
            col_ind[pos] = static_cast<int>(w >> bits);
            val_out[pos] = val[e];
        }
    }
}

__global__ void validate_csr_kernel(int rows, int cols, int nnz, const int* __restrict__ row_ptr,
                                    const int* __restrict__ col_ind, int* __restrict__ flag) {
    const int tid = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x);
    const int nth = static_cast<int>(gridDim.x * blockDim.x);
    int f = 0;
    if (tid == 0 && (row_ptr[0] != 0 || row_ptr[rows] != nnz)) f |= 1;
    for (int i = tid; i < rows; i += nth)
        if (row_ptr[i + 1] < row_ptr[i]) f |= 2;
    for (int k = tid; k < nnz; k += nth) {
        const int c = col_ind[k];
        if (c < 0 || c >= cols) f |= 4;
    }
    if (f) atomicOr(flag, f);
}

namespace {

inline size_t align256(size_t v) { return (v + 255) & ~static_cast<size_t>(255); }

template <typename ET, int HB>
hipError_t from_csr_hb(int rows, int nnz, const int* row_ptr, const int* col_ind, const void* val_in, int height,
                       int bits, uint32_t flags, uint32_t* col_word, void* val_out, void* workspace,
                       hipStream_t stream) {
    const int strips = (rows + height - 1) / height;
    const int blocks = (strips + kConvWaves - 1) / kConvWaves;
    const auto* vin = static_cast<const ET*>(val_in);
    auto* vout = static_cast<ET*>(val_out);
    if (!(flags & CMRS_SORT)) {
        hipLaunchKernelGGL((pack_kernel<HB, ET>), dim3(blocks), dim3(kConvThreads), 0, stream, rows, strips, height,
                           bits, row_ptr, col_ind, vin, col_word, vout, val_out != val_in ? 1 : 0);
        return hipGetLastError();
    }
    const FromCsrWorkspaceLayout L = from_csr_workspace_layout(nnz);
    auto* ws = static_cast<char*>(workspace);
    int* ws_count = reinterpret_cast<int*>(ws);
    int* ws_list = reinterpret_cast<int*>(ws + L.list_off);
    auto* gkeys = reinterpret_cast<uint64_t*>(ws + L.global_off);
    hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(64), 0, stream, ws_count, 0);
    hipLaunchKernelGGL((sort_strips_wave_kernel<HB, ET>), dim3(blocks), dim3(kConvThreads), 0, stream, rows,
                       strips, height, bits, row_ptr, col_ind, vin, col_word, vout, ws_count, ws_list);
    const int grid2 = static_cast<int>(L.list_cap < 512 ? L.list_cap : 512);
    hipLaunchKernelGGL((sort_strips_block_kernel<HB, ET>), dim3(grid2), dim3(kBlockSortThreads), 0, stream, rows,
                       height, bits, row_ptr, col_ind, vin, col_word, vout, ws_count, ws_list, gkeys);
    return hipGetLastError();
}

template <typename ET>
hipError_t from_csr_typed(int rows, int nnz, const int* row_ptr, const int* col_ind, const void* val_in, int height,
                          int bits, uint32_t flags, uint32_t* col_word, void* val_out, void* workspace,
                          hipStream_t stream) {
    switch (next_pow2(height)) {
        case 1: return from_csr_hb<ET, 1>(rows, nnz, row_ptr, col_ind, val_in, height, bits, flags, col_word, val_out, workspace, stream);
        case 2: return from_csr_hb<ET, 2>(rows, nnz, row_ptr, col_ind, val_in, height, bits, flags, col_word, val_out, workspace, stream);
        case 4: return from_csr_hb<ET, 4>(rows, nnz, row_ptr, col_ind, val_in, height, bits, flags, col_word, val_out, workspace, stream);
        case 8: return from_csr_hb<ET, 8>(rows, nnz, row_ptr, col_ind, val_in, height, bits, flags, col_word, val_out, workspace, stream);
        case 16: return from_csr_hb<ET, 16>(rows, nnz, row_ptr, col_ind, val_in, height, bits, flags, col_word, val_out, workspace, stream);
        default: return from_csr_hb<ET, 32>(rows, nnz, row_ptr, col_ind, val_in, height, bits, flags, col_word, val_out, workspace, stream);
    }
}

template <typename ET, int HB>
hipError_t to_csr_hb(const cmrs_mat_t* A, int* row_ptr, int* col_ind, void* val_out, hipStream_t stream) {
    const int strips = (A->rows + A->height - 1) / A->height;
    const int blocks = (strips + kConvWaves - 1) / kConvWaves;
    hipLaunchKernelGGL((to_csr_kernel<HB, ET>), dim3(blocks), dim3(kConvThreads), 0, stream, A->rows, strips,
                       A->height, A->bits, A->strip_ptr, A->col_word, static_cast<const ET*>(A->val), row_ptr,
                       col_ind, static_cast<ET*>(val_out));
    return hipGetLastError();
}

template <typename ET>
hipError_t to_csr_typed(const cmrs_mat_t* A, int* row_ptr, int* col_ind, void* val_out, hipStream_t stream) {
    switch (next_pow2(A->height)) {
        case 1: return to_csr_hb<ET, 1>(A, row_ptr, col_ind, val_out, stream);
        case 2: return to_csr_hb<ET, 2>(A, row_ptr, col_ind, val_out, stream);
        case 4: return to_csr_hb<ET, 4>(A, row_ptr, col_ind, val_out, stream);
        case 8: return to_csr_hb<ET, 8>(A, row_ptr, col_ind, val_out, stream);
        case 16: return to_csr_hb<ET, 16>(A, row_ptr, col_ind, val_out, stream);
        default: return to_csr_hb<ET, 32>(A, row_ptr, col_ind, val_out, stream);
    }
}

}  // namespace

FromCsrWorkspaceLayout from_csr_workspace_layout(int32_t nnz) {
    FromCsrWorkspaceLayout L;
    L.list_off = 256;
    L.list_cap = static_cast<size_t>(nnz) / (kWaveSortCap + 1) + 1;
    L.global_off = align256(L.list_off + 4 * L.list_cap);
    L.total = L.global_off + 16 * static_cast<size_t>(nnz);
    return L;
}

hipError_t launch_from_csr(int32_t rows, int32_t cols, int32_t nnz, const int32_t* row_ptr, const int32_t* col_ind,
                           const void* val_in, cmrs_dtype_t dtype, int32_t height, int32_t bits, uint32_t flags,
                           int32_t* strip_ptr, uint32_t* col_word, void* val_out, void* workspace,
                           hipStream_t stream) {
    (void)cols;
    const int strips = (rows + height - 1) / height;
    const int g = (strips + 1 + 255) / 256;
    hipLaunchKernelGGL(strip_ptr_kernel, dim3(g), dim3(256), 0, stream, strips, height, nnz, row_ptr, strip_ptr);
    hipError_t e = hipGetLastError();
    // No entries: the strip pointers are the whole result (and the sorted
    // path's workspace is then zero bytes, so nothing may touch it).
    if (e != hipSuccess || strips == 0 || nnz == 0) return e;
    switch (dtype_bytes(dtype)) {
        case 8: return from_csr_typed<uint64_t>(rows, nnz, row_ptr, col_ind, val_in, height, bits, flags, col_word, val_out, workspace, stream);
        case 4: return from_csr_typed<uint32_t>(rows, nnz, row_ptr, col_ind, val_in, height, bits, flags, col_word, val_out, workspace, stream);
        default: return from_csr_typed<uint16_t>(rows, nnz, row_ptr, col_ind, val_in, height, bits, flags, col_word, val_out, workspace, stream);
    }
}

hipError_t launch_to_csr(const cmrs_mat_t* A, int32_t* row_ptr, int32_t* col_ind, void* val_out,
                         hipStream_t stream) {
    if (A->rows == 0) {
        hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(64), 0, stream, row_ptr, 0);
        return hipGetLastError();
    }
    switch (dtype_bytes(A->val_dtype)) {
        case 8: return to_csr_typed<uint64_t>(A, row_ptr, col_ind, val_out, stream);
        case 4: return to_csr_typed<uint32_t>(A, row_ptr, col_ind, val_out, stream);
        default: return to_csr_typed<uint16_t>(A, row_ptr, col_ind, val_out, stream);
    }
}

hipError_t launch_validate_csr(int32_t rows, int32_t cols, int32_t nnz, const int32_t* row_ptr,
                               const int32_t* col_ind, int32_t* flag, hipStream_t stream) {
    hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(64), 0, stream, flag, 0);
    int work = rows > nnz ? rows : nnz;
    int g = (work + 255) / 256;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(validate_csr_kernel, dim3(g), dim3(256), 0, stream, rows, cols, nnz, row_ptr, col_ind, flag);
    return hipGetLastError();
}

}  // namespace cmrs
