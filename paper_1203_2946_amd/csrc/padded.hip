// The modified CMRS of Sec. 6.7: padded strips and a small per-wave buffer.
//
// Algorithm 1 gives each lane its own `height` partial sums.  Sec. 6.7
// shrinks the buffer to M copies (lane l uses copy l mod M), which is safe
// when no two lanes of one step (64 consecutive entries here) can hit the
// same (copy, row) pair.  The entries of every strip are therefore arranged
// in chunks of 64 where each row contributes at most M = 8 entries, stored
// contiguously (so lanes l and l + 8 never share a row), and every strip is
// padded with explicit zero entries to a whole number of chunks, which also
// makes every word and value load of the kernel an aligned, fully used
// 64-lane access.
//
// Arrangement (the paper fixes the constraints, not the order; this is the
// reading used here): chunk after chunk, every row with entries left offers
// min(8, remaining) of them, in CSR order; rows with more entries left go
// first (ties: lower row first) until the 64 slots are full; the slots left
// over are padding.  A padding entry has RowInStrip = height (the packed
// field is one bit wider when height is a power of two), column 0 and value
// +0, and the kernel skips it, so y is exactly the product of the stored
// matrix whatever x holds.
//
// Conversion: one wave per strip runs the arrangement twice, first counting
// chunks (a scan of the counts gives the strip pointers), then writing.
#include <limits.h>

#include "cmrs_device.hpp"
#include "cmrs_ext.hpp"

namespace cmrs {

constexpr int kPadM = 8;
constexpr int kPadWaves = 4;
constexpr int kScanThreads = 1024;
constexpr int kScanItems = 4;
constexpr int kScanBlock = kScanThreads * kScanItems;

// One chunk of the arrangement for the strip whose row r < nr sits in lane r
// with `rem` entries left.  Returns this lane's slot offset and entry count.
// All 64 lanes must be active (nr is uniform).
__device__ inline void pad_chunk(int rem, int nr, int lane, int& off, int& take) {
    const int t = lane < nr ? min(kPadM, rem) : 0;
    int before = 0;
    for (int q = 0; q < nr; ++q) {
        const int rq = __shfl(rem, q);
        const int tq = __shfl(t, q);
        if (rq > rem || (rq == rem && q < lane)) before += tq;
    }
    off = min(kWave, before);
    take = min(t, kWave - off);
}

__global__ __launch_bounds__(kPadWaves * kWave) void padded_count_kernel(int rows, int strips, int height,
                                                                         const int* __restrict__ row_ptr,
                                                                         long long* __restrict__ chunks) {
    const int lane = lane_id();
    const int strip = static_cast<int>(blockIdx.x) * kPadWaves + static_cast<int>(threadIdx.x) / kWave;
    if (strip >= strips) return;
    const int r0 = strip * height;
    const int nr = min(height, rows - r0);
    int rem = lane < nr ? row_ptr[r0 + lane + 1] - row_ptr[r0 + lane] : 0;
    long long n = 0;
    while (ballot(rem > 0)) {
        int off, take;
        pad_chunk(rem, nr, lane, off, take);
        rem -= take;
        ++n;
    }
    if (lane == 0) chunks[strip] = n;
}

// Exclusive prefix sums of n int64 counts: block scans, a scan of the block
// totals in one workgroup, then the block offsets added.  out has n + 1
// entries (out[n] = total).
__device__ inline long long block_inclusive_scan(long long v, long long* sh) {
    const int t = static_cast<int>(threadIdx.x);
    const int lane = lane_id(), wave = t / kWave;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const long long u = __shfl_up(v, o);
        if (lane >= o) v += u;
    }
    if (lane == kWave - 1) sh[wave] = v;
    __syncthreads();
    if (wave == 0) {
        long long w = lane < kScanThreads / kWave ? sh[lane] : 0;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const long long u = __shfl_up(w, o);
            if (lane >= o) w += u;
        }
        if (lane < kScanThreads / kWave) sh[lane] = w;
    }
    __syncthreads();
    const long long add = wave > 0 ? sh[wave - 1] : 0;
    __syncthreads();
    return v + add;
}

__global__ __launch_bounds__(kScanThreads) void scan_blocks_kernel(const long long* __restrict__ in, int n,
                                                                   long long* __restrict__ out,
                                                                   long long* __restrict__ bsum) {
    __shared__ long long sh[kScanThreads / kWave];
    const size_t base = static_cast<size_t>(blockIdx.x) * kScanBlock + threadIdx.x * kScanItems;
    long long v[kScanItems];
    long long s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = base + i < static_cast<size_t>(n) ? in[base + i] : 0;
        s += v[i];
    }
    const long long incl = block_inclusive_scan(s, sh);
    long long run = incl - s;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < static_cast<size_t>(n)) out[base + i] = run;
        run += v[i];
    }
    if (threadIdx.x == kScanThreads - 1) bsum[blockIdx.x] = incl;
}

// One workgroup: exclusive scan of nb block totals in place, total at bsum[nb].
__global__ __launch_bounds__(kScanThreads) void scan_top_kernel(long long* __restrict__ bsum, int nb) {
    __shared__ long long sh[kScanThreads / kWave];
    const int per = (nb + kScanThreads - 1) / kScanThreads;
    const int b0 = static_cast<int>(threadIdx.x) * per;
    long long s = 0;
    for (int i = 0; i < per; ++i)
        if (b0 + i < nb) s += bsum[b0 + i];
    const long long incl = block_inclusive_scan(s, sh);
    long long run = incl - s;
    for (int i = 0; i < per; ++i) {
        if (b0 + i < nb) {
            const long long v = bsum[b0 + i];
            bsum[b0 + i] = run;
            run += v;
        }
    }
    if (threadIdx.x == kScanThreads - 1) bsum[nb] = incl;
}

__global__ __launch_bounds__(256) void scan_add_kernel(long long* __restrict__ out, int n,
                                                       const long long* __restrict__ bsum, int nb) {
    const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < static_cast<size_t>(n)) out[i] += bsum[i / kScanBlock];
    if (i == static_cast<size_t>(n)) out[n] = bsum[nb];
}

__global__ __launch_bounds__(256) void padded_strip_ptr_kernel(const long long* __restrict__ prefix, int n,
                                                               int32_t* __restrict__ strip_ptr) {
    const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i <= static_cast<size_t>(n)) strip_ptr[i] = static_cast<int32_t>(prefix[i] * kWave);
}

template <typename ET>
__global__ __launch_bounds__(kPadWaves * kWave) void padded_fill_kernel(
    int rows, int strips, int height, int bits, const int* __restrict__ row_ptr, const int* __restrict__ col_ind,
    const ET* __restrict__ val_in, const int* __restrict__ strip_ptr, uint32_t* __restrict__ word_out,
    ET* __restrict__ val_out) {
    __shared__ int slot_row[kPadWaves][kWave];
    const int lane = lane_id();
    const int wave = static_cast<int>(threadIdx.x) / kWave;
    const int strip = static_cast<int>(blockIdx.x) * kPadWaves + wave;
    if (strip >= strips) return;
    int* map = slot_row[wave];
    const int r0 = strip * height;
    const int nr = min(height, rows - r0);
    const int start = lane < nr ? row_ptr[r0 + lane] : 0;
    int rem = lane < nr ? row_ptr[r0 + lane + 1] - start : 0;
    int consumed = 0;
    int pos = strip_ptr[strip];
    const int end = strip_ptr[strip + 1];
    while (ballot(rem > 0) && pos < end) {
        int off, take;
        pad_chunk(rem, nr, lane, off, take);
        map[lane] = -1;
        wave_lds_sync();
        for (int t = 0; t < take; ++t) map[off + t] = lane;
        wave_lds_sync();
        const int r = map[lane];
        const int src = r < 0 ? 0 : r;
        const int s_off = __shfl(off, src), s_cons = __shfl(consumed, src), s_start = __shfl(start, src);
        if (r >= 0) {
            const int k = s_start + s_cons + (lane - s_off);
            word_out[pos + lane] = (static_cast<uint32_t>(col_ind[k]) << bits) | static_cast<uint32_t>(r);
            val_out[pos + lane] = val_in[k];
        } else {
            word_out[pos + lane] = static_cast<uint32_t>(height);
            val_out[pos + lane] = ET(0);
        }
        wave_lds_sync();
        consumed += take;
        rem -= take;
        pos += kWave;
    }
}

// One wave per strip; U chunks of loads in flight; partials in M copies of
// the strip's rows, b[(lane mod M) * HB + row].
template <int HB, int U, typename VT, typename XT, typename AT>
__global__ __launch_bounds__(kPadWaves * kWave) void padded_spmv_kernel(int rows, int strips, int height, int bits,
                                                                        const int* __restrict__ strip_ptr,
                                                                        const uint32_t* __restrict__ word,
                                                                        const VT* __restrict__ val,
                                                                        const XT* __restrict__ x,
                                                                        XT* __restrict__ y) {
    __shared__ AT buf[kPadWaves][kPadM * HB];
    const int lane = lane_id();
    const int wave = uniform(static_cast<int>(threadIdx.x) / kWave);
    const int strip = xcd_logical_block(blockIdx.x, gridDim.x) * kPadWaves + wave;
    if (strip >= strips) return;
    AT* b = buf[wave];
    for (int i = lane; i < kPadM * HB; i += kWave) b[i] = AT(0);
    wave_lds_sync();
    const int p0 = strip_ptr[strip], p1 = strip_ptr[strip + 1];
    const uint32_t mask = (1u << bits) - 1u;
    AT* mine = b + (lane & (kPadM - 1)) * HB;
    for (int base = p0; base < p1; base += U * kWave) {
        uint32_t w[U];
        VT v[U];
        XT xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            // Chunks past the strip re-read its last chunk (valid addresses).
            const int j = min(base + u * kWave, p1 - kWave) + lane;
            w[u] = __builtin_nontemporal_load(word + j);
            v[u] = val[j];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = x[w[u] >> bits];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = static_cast<int>(w[u] & mask);
            if (base + u * kWave < p1 && r < height)
                lds_add(mine + (r & (HB - 1)),
                        static_cast<AT>(ValTraits<VT>::widen(v[u])) * static_cast<AT>(xv[u]));
        }
    }
    wave_lds_sync();
    if (lane < height) {
        AT s = b[lane];
#pragma unroll
        for (int m = 1; m < kPadM; ++m) s += b[m * HB + lane];
        const long long row = static_cast<long long>(strip) * height + lane;
        if (row < rows) y[row] = static_cast<XT>(s);
    }
}

// ------------------------------------------------------------------ host

PaddedWorkspaceLayout padded_workspace_layout(int strips) {
    PaddedWorkspaceLayout L{};
    const size_t n = static_cast<size_t>(strips);
    L.nb = static_cast<int>((n + kScanBlock - 1) / kScanBlock);
    L.chunks_off = 0;
    L.prefix_off = 8 * n;
    L.bsum_off = L.prefix_off + 8 * (n + 1);
    L.total = L.bsum_off + 8 * (static_cast<size_t>(L.nb) + 1);
    return L;
}

hipError_t launch_padded_count(int rows, int height, const int* row_ptr, void* workspace, hipStream_t stream) {
    const int strips = (rows + height - 1) / height;
    const PaddedWorkspaceLayout L = padded_workspace_layout(strips);
    unsigned char* ws = static_cast<unsigned char*>(workspace);
    long long* chunks = reinterpret_cast<long long*>(ws + L.chunks_off);
    long long* prefix = reinterpret_cast<long long*>(ws + L.prefix_off);
    long long* bsum = reinterpret_cast<long long*>(ws + L.bsum_off);
    if (strips > 0)
        hipLaunchKernelGGL(padded_count_kernel, dim3((strips + kPadWaves - 1) / kPadWaves), dim3(kPadWaves * kWave),
                           0, stream, rows, strips, height, row_ptr, chunks);
    if (L.nb > 0)
        hipLaunchKernelGGL(scan_blocks_kernel, dim3(L.nb), dim3(kScanThreads), 0, stream, chunks, strips, prefix,
                           bsum);
    hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(kScanThreads), 0, stream, bsum, L.nb);
    hipLaunchKernelGGL(scan_add_kernel, dim3((strips + 1 + 255) / 256), dim3(256), 0, stream, prefix, strips, bsum,
                       L.nb);
    return hipGetLastError();
}

hipError_t launch_padded_strip_ptr(int strips, const void* workspace, int32_t* strip_ptr, hipStream_t stream) {
    const PaddedWorkspaceLayout L = padded_workspace_layout(strips);
    const long long* prefix =
        reinterpret_cast<const long long*>(static_cast<const unsigned char*>(workspace) + L.prefix_off);
    hipLaunchKernelGGL(padded_strip_ptr_kernel, dim3((strips + 1 + 255) / 256), dim3(256), 0, stream, prefix, strips,
                       strip_ptr);
    return hipGetLastError();
}

const long long* padded_total_ptr(int strips, const void* workspace) {
    const PaddedWorkspaceLayout L = padded_workspace_layout(strips);
    return reinterpret_cast<const long long*>(static_cast<const unsigned char*>(workspace) + L.prefix_off) + strips;
}

hipError_t launch_padded_fill(int rows, int height, int bits, const int* row_ptr, const int* col_ind,
                              const void* val_in, cmrs_dtype_t dtype, const int* strip_ptr, uint32_t* word_out,
                              void* val_out, hipStream_t stream) {
    const int strips = (rows + height - 1) / height;
    if (strips == 0) return hipSuccess;
    const dim3 grid((strips + kPadWaves - 1) / kPadWaves), block(kPadWaves * kWave);
    switch (dtype_bytes(dtype)) {
        case 8:
            hipLaunchKernelGGL(padded_fill_kernel<uint64_t>, grid, block, 0, stream, rows, strips, height, bits,
                               row_ptr, col_ind, static_cast<const uint64_t*>(val_in), strip_ptr, word_out,
                               static_cast<uint64_t*>(val_out));
            break;
        case 4:
            hipLaunchKernelGGL(padded_fill_kernel<uint32_t>, grid, block, 0, stream, rows, strips, height, bits,
                               row_ptr, col_ind, static_cast<const uint32_t*>(val_in), strip_ptr, word_out,
                               static_cast<uint32_t*>(val_out));
            break;
        default:
            hipLaunchKernelGGL(padded_fill_kernel<uint16_t>, grid, block, 0, stream, rows, strips, height, bits,
                               row_ptr, col_ind, static_cast<const uint16_t*>(val_in), strip_ptr, word_out,
                               static_cast<uint16_t*>(val_out));
            break;
    }
    return hipGetLastError();
}

namespace {

template <typename VT, typename XT, typename AT, int HB>
void launch_padded_spmv_hb(const cmrs_mat_t* A, const void* x, void* y, hipStream_t stream) {
    const int strips = (A->rows + A->height - 1) / A->height;
    const dim3 grid((strips + kPadWaves - 1) / kPadWaves), block(kPadWaves * kWave);
    hipLaunchKernelGGL((padded_spmv_kernel<HB, 4, VT, XT, AT>), grid, block, 0, stream, A->rows, strips, A->height,
                       A->bits, A->strip_ptr, A->col_word, static_cast<const VT*>(A->val),
                       static_cast<const XT*>(x), static_cast<XT*>(y));
}

template <typename VT, typename XT, typename AT>
void launch_padded_spmv_typed(const cmrs_mat_t* A, const void* x, void* y, hipStream_t stream) {
    switch (next_pow2(A->height)) {
        case 1: launch_padded_spmv_hb<VT, XT, AT, 1>(A, x, y, stream); break;
        case 2: launch_padded_spmv_hb<VT, XT, AT, 2>(A, x, y, stream); break;
        case 4: launch_padded_spmv_hb<VT, XT, AT, 4>(A, x, y, stream); break;
        case 8: launch_padded_spmv_hb<VT, XT, AT, 8>(A, x, y, stream); break;
        case 16: launch_padded_spmv_hb<VT, XT, AT, 16>(A, x, y, stream); break;
        default: launch_padded_spmv_hb<VT, XT, AT, 32>(A, x, y, stream); break;
    }
}

}  // namespace

hipError_t launch_padded_spmv(const cmrs_mat_t* A, const void* x, void* y, hipStream_t stream) {
    if (A->rows == 0) return hipSuccess;
    switch (A->val_dtype) {
        case CMRS_R64F: launch_padded_spmv_typed<double, double, double>(A, x, y, stream); break;
        case CMRS_R32F: launch_padded_spmv_typed<float, float, float>(A, x, y, stream); break;
        default: launch_padded_spmv_typed<bf16_t, float, float>(A, x, y, stream); break;
    }
    return hipGetLastError();
}

}  // namespace cmrs
