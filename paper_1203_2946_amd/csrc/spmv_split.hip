// CMRS SpMV for matrices whose strips differ widely in length (skewed rows).
//
// Algorithm 1 of Sec. 4 gives every strip to one wave.  A strip with 10^4
// entries next to strips of a few dozen makes that one wave the critical
// path, and with strip groups it also stalls the other strips of its wave.
// The paper leaves such matrices to special algorithms (Sec. 6.2).  Here a
// plan, built on the device from StripPtr alone, lists every strip longer
// than long_len ("heavy") and cuts it into chunks of at most chunk_len
// consecutive entries.  The SpMV launch then has two kinds of waves:
//   chunk waves  (the first workgroups) take chunks from the list and
//                compute the chunk's height row sums exactly as Algorithm 1
//                does for a whole strip: a strip of one chunk writes its rows
//                of y, the others store the sums in the plan's partial-sum
//                area;
//   group waves  process all other strips as strip groups (G lanes per
//                strip) and leave the heavy strips alone.
// A second small launch adds the chunk sums of every strip of several chunks
// in chunk order and writes its rows.  (Combining in the first launch, by the
// wave that finishes a strip's last chunk, needs agent-scope release and
// acquire fences per chunk; on gfx950 those write back and invalidate the
// XCD's L2, which measured 3-7x slower.)  Results are deterministic: a chunk
// is summed in a fixed order and a strip's chunk sums are added in chunk
// order.
#include "cmrs_ext.hpp"
#include "spmv_device.hpp"

namespace cmrs {

// Workgroups of chunk waves: at most this many, each wave looping over the
// chunk list (the number of chunks is known on the device only).
constexpr int kSplitChunkBlocksMax = 1024;

// The plan, in three launches and in strip order: (1) every block of 256
// strips counts its heavy strips and their chunks; (2) one workgroup turns
// the block counts into offsets (exclusive scan) and writes the totals;
// (3) every block scans its strips again and writes its heavy strips and
// their chunks at those offsets.  A heavy strip has more than long_len
// entries and n = ceil(len / chunk_len) chunks of len / n entries (one more
// for the first len % n).  No atomics, so the lists come out the same on
// every build.
constexpr int kPlanThreads = 256;

struct SplitCount {
    int heavy, chunks;
};

__device__ inline SplitCount split_strip_count(int s, int strips, int long_len, int chunk_len,
                                               const int* __restrict__ strip_ptr, int& lo, int& len) {
    lo = 0;
    len = 0;
    if (s < strips) {
        lo = strip_ptr[s];
        len = strip_ptr[s + 1] - lo;
    }
    if (s >= strips || len <= long_len) return SplitCount{0, 0};
    return SplitCount{1, (len + chunk_len - 1) / chunk_len};
}

// Exclusive scan of v over the block's 256 threads (4 waves); returns the
// block total through *total.
__device__ inline int block_exclusive_scan(int v, int* wave_tot, int* total) {
    const int lane = lane_id();
    const int wave = static_cast<int>(threadIdx.x) / kWave;
    int inc = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int t = __shfl_up(inc, off);
        if (lane >= off) inc += t;
    }
    if (lane == kWave - 1) wave_tot[wave] = inc;
    __syncthreads();
    int before = 0, all = 0;
    for (int w = 0; w < kPlanThreads / kWave; ++w) {
        if (w < wave) before += wave_tot[w];
        all += wave_tot[w];
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

__global__ __launch_bounds__(kPlanThreads) void split_count_kernel(int strips, int long_len, int chunk_len,
                                                                   const int* __restrict__ strip_ptr,
                                                                   int* __restrict__ block_sums) {
    __shared__ int tot[2][kPlanThreads / kWave];
    const int s = static_cast<int>(blockIdx.x) * kPlanThreads + static_cast<int>(threadIdx.x);
    int lo, len;
    const SplitCount c = split_strip_count(s, strips, long_len, chunk_len, strip_ptr, lo, len);
    int th, tc;
    block_exclusive_scan(c.heavy, tot[0], &th);
    block_exclusive_scan(c.chunks, tot[1], &tc);
    if (threadIdx.x == 0) {
        block_sums[2 * blockIdx.x] = th;
        block_sums[2 * blockIdx.x + 1] = tc;
    }
}

// One workgroup: block_sums[2b], [2b+1] become the block's first heavy slot
// and first chunk slot; counts[0], counts[1] the totals.
__global__ __launch_bounds__(kPlanThreads) void split_scan_kernel(int nblocks, int* __restrict__ block_sums,
                                                                  int* __restrict__ counts) {
    __shared__ int tot[2][kPlanThreads / kWave];
    int carry_h = 0, carry_c = 0;
    for (int base = 0; base < nblocks; base += kPlanThreads) {
        const int b = base + static_cast<int>(threadIdx.x);
        const int h = b < nblocks ? block_sums[2 * b] : 0;
        const int c = b < nblocks ? block_sums[2 * b + 1] : 0;
        int th, tc;
        const int oh = block_exclusive_scan(h, tot[0], &th);
        const int oc = block_exclusive_scan(c, tot[1], &tc);
        if (b < nblocks) {
            block_sums[2 * b] = carry_h + oh;
            block_sums[2 * b + 1] = carry_c + oc;
        }
        carry_h += th;
        carry_c += tc;
    }
    if (threadIdx.x == 0) {
        counts[0] = carry_h;
        counts[1] = carry_c;
    }
}

__global__ __launch_bounds__(kPlanThreads) void split_fill_kernel(int strips, int long_len, int chunk_len,
                                                                  const int* __restrict__ strip_ptr,
                                                                  const int* __restrict__ block_sums,
                                                                  SplitHeavy* __restrict__ heavy,
                                                                  SplitChunk* __restrict__ chunks, int max_heavy,
                                                                  int max_chunks) {
    __shared__ int tot[2][kPlanThreads / kWave];
    const int s = static_cast<int>(blockIdx.x) * kPlanThreads + static_cast<int>(threadIdx.x);
    int lo, len;
    const SplitCount c = split_strip_count(s, strips, long_len, chunk_len, strip_ptr, lo, len);
    int th, tc;
    const int h = block_sums[2 * blockIdx.x] + block_exclusive_scan(c.heavy, tot[0], &th);
    const int c0 = block_sums[2 * blockIdx.x + 1] + block_exclusive_scan(c.chunks, tot[1], &tc);
    if (!c.heavy || h >= max_heavy || c0 > max_chunks - c.chunks) return;
    const int n = c.chunks;
    heavy[h] = SplitHeavy{s, c0, n, 0};
    const int q = len / n, rem = len - q * n;
    int a = lo;
    for (int k = 0; k < n; ++k) {
        const int e = a + q + (k < rem ? 1 : 0);
        chunks[c0 + k] = SplitChunk{h, a, e, 0};
        a = e;
    }
}

template <int HB, int G, int U, bool NT, typename VT, typename XT, typename AT>
__global__ __launch_bounds__(kSpmvThreads) void spmv_split_kernel(
    int rows, int strips, int height, int bits, const int* __restrict__ strip_ptr, const uint32_t* __restrict__ word,
    const VT* __restrict__ val, const XT* __restrict__ x, XT* __restrict__ y, int long_len, int chunk_blocks,
    int max_chunks, const int* __restrict__ counts, const SplitHeavy* __restrict__ heavy,
    const SplitChunk* __restrict__ chunks, AT* __restrict__ partial) {
    constexpr int NG = kWave / G;
    constexpr int GW = kWave / HB;
    __shared__ AT buf[kSpmvWaves][HB * kWave];
    const int lane = lane_id();
    const int wave = uniform(static_cast<int>(threadIdx.x) / kWave);
    const int b = static_cast<int>(blockIdx.x);
    if (b < chunk_blocks) {
        const int nchunks = min(uniform(counts[1]), max_chunks);
        for (int c = b * kSpmvWaves + wave; c < nchunks; c += chunk_blocks * kSpmvWaves) {
            const SplitChunk ck = chunks[c];
            const SplitHeavy hv = heavy[ck.heavy];
            LdsAcc<HB, AT> acc{buf[wave]};
            acc.init(lane);
            accumulate_run<U, NT, VT, XT, AT>(acc, ck.lo, ck.hi, bits, word, val, x, lane);
            const AT s = acc.finish(lane);
            const int r = lane / GW;
            if (hv.nchunks == 1) {
                const int row = hv.strip * height + r;
                if ((lane % GW) == 0 && r < height && row < rows) y[row] = static_cast<XT>(s);
            } else if ((lane % GW) == 0) {
                partial[static_cast<size_t>(c) * HB + r] = s;
            }
            wave_lds_sync();
        }
        return;
    }
    const int gb = b - chunk_blocks;
    const int strip0 = (xcd_logical_block(gb, static_cast<int>(gridDim.x) - chunk_blocks) * kSpmvWaves + wave) * NG;
    if (strip0 >= strips) return;
    const int strip = strip0 + lane / G;
    int lo = 0, hi = 0;
    if (strip < strips) {
        lo = strip_ptr[strip];
        hi = strip_ptr[strip + 1];
    }
    auto out = [&](int gg, int rr, AT s) {
        const int st = strip0 + gg;
        const int row = st * height + rr;
        if (st < strips && rr < height && row < rows) y[row] = static_cast<XT>(s);
    };
    group_runs<HB, G, U, NT, VT, XT, AT, decltype(out), true>(lo, hi, long_len, bits, word, val, x, buf[wave], lane,
                                                             out);
}

// Second launch: the rows of every strip cut into several chunks, as the sum
// of its chunk sums in chunk order (one wave per heavy strip, lane r < HB
// takes row r).
template <int HB, typename XT, typename AT>
__global__ __launch_bounds__(256) void split_combine_kernel(int rows, int height, int max_heavy,
                                                            const int* __restrict__ counts,
                                                            const SplitHeavy* __restrict__ heavy,
                                                            const AT* __restrict__ partial, XT* __restrict__ y) {
    const int lane = lane_id();
    const int nheavy = min(uniform(counts[0]), max_heavy);
    const int waves = static_cast<int>(gridDim.x * blockDim.x) / kWave;
    for (int h = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x) / kWave; h < nheavy; h += waves) {
        const SplitHeavy hv = heavy[h];
        if (hv.nchunks < 2 || lane >= HB) continue;
        const AT* p = partial + static_cast<size_t>(hv.first) * HB + lane;
        AT t = p[0];
        for (int k = 1; k < hv.nchunks; ++k) t += p[static_cast<size_t>(k) * HB];
        const int row = hv.strip * height + lane;
        if (lane < height && row < rows) y[row] = static_cast<XT>(t);
    }
}

SplitShape split_shape(const cmrs_mat_t* A, int long_len, int chunk_len) {
    SplitShape s{};
    const int strips = (A->rows + A->height - 1) / A->height;
    const int hb = next_pow2(A->height);
    s.group = spmv_group_width(A->nnz, strips, hb);
    s.long_len = long_len > 0 ? long_len : 2 * kSplitU * s.group;
    s.chunk_len = chunk_len > 0 ? chunk_len : 1024;
    const long long nnz = A->nnz;
    s.max_heavy = static_cast<int>(std::min<long long>(strips, nnz / (static_cast<long long>(s.long_len) + 1)));
    s.max_chunks = static_cast<int>(std::min<long long>(nnz, nnz / s.chunk_len + s.max_heavy));
    auto up = [](size_t v) { return (v + 255) & ~static_cast<size_t>(255); };
    const int nblocks = (strips + kPlanThreads - 1) / kPlanThreads;
    s.block_off = 256;
    s.heavy_off = up(s.block_off + 2 * sizeof(int) * static_cast<size_t>(nblocks));
    s.chunk_off = up(s.heavy_off + sizeof(SplitHeavy) * static_cast<size_t>(s.max_heavy));
    s.partial_off = up(s.chunk_off + sizeof(SplitChunk) * static_cast<size_t>(s.max_chunks));
    s.total = up(s.partial_off + sizeof(double) * static_cast<size_t>(hb) * static_cast<size_t>(s.max_chunks));
    return s;
}

hipError_t launch_split_plan(const cmrs_mat_t* A, const SplitShape& s, void* buf, hipStream_t stream) {
    char* base = static_cast<char*>(buf);
    int* counts = reinterpret_cast<int*>(base);
    const int strips = (A->rows + A->height - 1) / A->height;
    const int nblocks = (strips + kPlanThreads - 1) / kPlanThreads;
    int* block_sums = reinterpret_cast<int*>(base + s.block_off);
    if (nblocks > 0)
        hipLaunchKernelGGL(split_count_kernel, dim3(nblocks), dim3(kPlanThreads), 0, stream, strips, s.long_len,
                           s.chunk_len, A->strip_ptr, block_sums);
    hipLaunchKernelGGL(split_scan_kernel, dim3(1), dim3(kPlanThreads), 0, stream, nblocks, block_sums, counts);
    if (nblocks > 0 && s.max_heavy > 0)
        hipLaunchKernelGGL(split_fill_kernel, dim3(nblocks), dim3(kPlanThreads), 0, stream, strips, s.long_len,
                           s.chunk_len, A->strip_ptr, block_sums, reinterpret_cast<SplitHeavy*>(base + s.heavy_off),
                           reinterpret_cast<SplitChunk*>(base + s.chunk_off), s.max_heavy, s.max_chunks);
    return hipGetLastError();
}

namespace {

template <typename VT, typename XT, typename AT, int HB, int G>
hipError_t launch_split_g(const cmrs_mat_t* A, const SplitShape& s, const void* buf, const void* x, void* y,
                          hipStream_t stream) {
    constexpr int NG = kWave / G;
    const int strips = (A->rows + A->height - 1) / A->height;
    const int waves = (strips + NG - 1) / NG;
    const int group_blocks = (waves + kSpmvWaves - 1) / kSpmvWaves;
    int chunk_blocks = 0;
    if (s.max_chunks > 0) {
        chunk_blocks = std::min((s.max_chunks + kSpmvWaves - 1) / kSpmvWaves, kSplitChunkBlocksMax);
        chunk_blocks = (chunk_blocks + kNumXcd - 1) / kNumXcd * kNumXcd;
    }
    const char* base = static_cast<const char*>(buf);
    char* mbase = const_cast<char*>(base);
    // 6 loads per lane in a step up to height 8 (1.5 times the 4 entries a
    // lane gets there; skewed rows, cold, h = 8: fp64 139 -> 134 us, fp32
    // 103 -> 98 us), kSplitU above (12 was slower at h = 16: 124 -> 131 us).
    constexpr int SU = HB <= 8 ? 6 : kSplitU;
    hipLaunchKernelGGL((spmv_split_kernel<HB, G, SU, true, VT, XT, AT>), dim3(chunk_blocks + group_blocks),
                       dim3(kSpmvThreads), 0, stream, A->rows, strips, A->height, A->bits, A->strip_ptr, A->col_word,
                       static_cast<const VT*>(A->val), static_cast<const XT*>(x), static_cast<XT*>(y), s.long_len,
                       chunk_blocks, s.max_chunks, reinterpret_cast<const int*>(base),
                       reinterpret_cast<const SplitHeavy*>(base + s.heavy_off),
                       reinterpret_cast<const SplitChunk*>(base + s.chunk_off),
                       reinterpret_cast<AT*>(mbase + s.partial_off));
    if (s.max_heavy > 0) {
        const int blocks = std::min((s.max_heavy + 3) / 4, 1024);
        hipLaunchKernelGGL((split_combine_kernel<HB, XT, AT>), dim3(blocks), dim3(256), 0, stream, A->rows, A->height,
                           s.max_heavy, reinterpret_cast<const int*>(base),
                           reinterpret_cast<const SplitHeavy*>(base + s.heavy_off),
                           reinterpret_cast<const AT*>(base + s.partial_off), static_cast<XT*>(y));
    }
    return hipGetLastError();
}

template <typename VT, typename XT, typename AT, int HB>
hipError_t launch_split_hb(const cmrs_mat_t* A, const SplitShape& s, const void* buf, const void* x, void* y,
                           hipStream_t stream) {
    const int g = s.group;
    if constexpr (HB <= 2) {
        if (g <= 2) return launch_split_g<VT, XT, AT, HB, 2>(A, s, buf, x, y, stream);
    }
    if constexpr (HB <= 4) {
        if (g <= 4) return launch_split_g<VT, XT, AT, HB, 4>(A, s, buf, x, y, stream);
    }
    if constexpr (HB <= 8) {
        if (g <= 8) return launch_split_g<VT, XT, AT, HB, 8>(A, s, buf, x, y, stream);
    }
    if constexpr (HB <= 16) {
        if (g <= 16) return launch_split_g<VT, XT, AT, HB, 16>(A, s, buf, x, y, stream);
    }
    if (g <= 32) return launch_split_g<VT, XT, AT, HB, 32>(A, s, buf, x, y, stream);
    return launch_split_g<VT, XT, AT, HB, 64>(A, s, buf, x, y, stream);
}

template <typename VT, typename XT, typename AT>
hipError_t launch_split_typed(const cmrs_mat_t* A, const SplitShape& s, const void* buf, const void* x, void* y,
                              hipStream_t stream) {
    switch (next_pow2(A->height)) {
        case 1: return launch_split_hb<VT, XT, AT, 1>(A, s, buf, x, y, stream);
        case 2: return launch_split_hb<VT, XT, AT, 2>(A, s, buf, x, y, stream);
        case 4: return launch_split_hb<VT, XT, AT, 4>(A, s, buf, x, y, stream);
        case 8: return launch_split_hb<VT, XT, AT, 8>(A, s, buf, x, y, stream);
        case 16: return launch_split_hb<VT, XT, AT, 16>(A, s, buf, x, y, stream);
        default: return launch_split_hb<VT, XT, AT, 32>(A, s, buf, x, y, stream);
    }
}

}  // namespace

hipError_t launch_spmv_split(const cmrs_mat_t* A, const SplitShape& s, const void* buf, const void* x, void* y,
                             hipStream_t stream) {
    if (A->rows == 0) return hipSuccess;
    if (A->val_dtype == CMRS_R64F) return launch_split_typed<double, double, double>(A, s, buf, x, y, stream);
    if (A->val_dtype == CMRS_R32F) return launch_split_typed<float, float, float>(A, s, buf, x, y, stream);
    return launch_split_typed<bf16_t, float, float>(A, s, buf, x, y, stream);
}

}  // namespace cmrs
