// CMRS sparse matrix-vector product y = A x on gfx950.
//
// Algorithm 1 of Sec. 4 (Koza et al., arXiv:1203.2946), laid out for wave64:
// one 64-lane wave per strip; lane l walks entries start+l, start+l+64, ...;
// each entry's packed word gives the column (word >> bits) and RowInStrip
// (word & (2^bits - 1)); the product Val[j] * x[col] goes to lane l's own
// partial sum for that row.  After the strip the partials are reduced over
// the 64 lanes and the wave writes the strip's `height` results.
//
// Two ways to hold the per-lane partials (the buffer of Algorithm 1):
//   LDS  buf[r][lane] in LDS, updated with ds_add (no read-modify-write round
//        trip in the shader; each lane owns its slots, so the order of the
//        additions is fixed and the result deterministic).  Any height.
//   REG  HB accumulators per lane in VGPRs, updated with predicated adds;
//        the reduction is a register reduce-scatter butterfly.  Heights <= 8.
// Either can read the Val / word streams with non-temporal loads (NT), which
// keeps them from displacing x in L2.
//
// Column-blocked schedule: for a sorted matrix (entries of a strip ascending
// by column) the entries of strip s with columns in block b are a contiguous
// run [split(s, b), split(s, b+1)).  Pass b processes run b of every strip and
// adds it to y (pass 0 writes y), so one pass gathers from a 1/nb slice of x,
// small enough to stay resident in one XCD's L2.  The split points are the
// plan built by colblock_plan_kernel.
//
// Workgroups hold 4 waves (4 strips); workgroup ids are renumbered so that each
// XCD processes one contiguous range of strips.
#include <mutex>

#include "cmrs_internal.hpp"
#include "spmv_device.hpp"

namespace cmrs {

// One wave per strip.  split == nullptr: the whole strip, y overwritten.
// Otherwise run `blk` of `nb` column blocks, y overwritten for blk 0 and
// accumulated for later blocks.
template <int HB, int U, bool NT, bool REG, typename VT, typename XT, typename AT>
__global__ __launch_bounds__(kSpmvThreads) void spmv_kernel(
    int rows, int strips, int height, int bits, const int* __restrict__ strip_ptr,
    const uint32_t* __restrict__ word, const VT* __restrict__ val, const XT* __restrict__ x, XT* __restrict__ y,
    const int* __restrict__ split, int nb, int blk) {
    __shared__ AT buf[REG ? 1 : kSpmvWaves][REG ? 1 : HB * kWave];
    const int lane = lane_id();
    const int wave = uniform(static_cast<int>(threadIdx.x) / kWave);
    const int strip = xcd_logical_block(blockIdx.x, gridDim.x) * kSpmvWaves + wave;
    if (strip >= strips) return;
    int lo, hi;
    if (split == nullptr) {
        lo = strip_ptr[strip];
        hi = strip_ptr[strip + 1];
    } else {
        const int* sp = split + static_cast<size_t>(strip) * (nb - 1);
        lo = blk == 0 ? strip_ptr[strip] : sp[blk - 1];
        hi = blk == nb - 1 ? strip_ptr[strip + 1] : sp[blk];
    }
    AT s;
    if constexpr (REG) {
        RegAcc<HB, AT> acc;
        acc.init(lane);
        accumulate_run<U, NT, VT, XT, AT>(acc, lo, hi, bits, word, val, x, lane);
        s = acc.finish(lane);
    } else {
        LdsAcc<HB, AT> acc{buf[wave]};
        acc.init(lane);
        accumulate_run<U, NT, VT, XT, AT>(acc, lo, hi, bits, word, val, x, lane);
        s = acc.finish(lane);
    }
    constexpr int G = kWave / HB;
    const int r = lane / G;
    const int row = strip * height + r;
    if ((lane % G) == 0 && r < height && row < rows) {
        if (split != nullptr && blk > 0)
            y[row] = static_cast<XT>(static_cast<AT>(y[row]) + s);
        else
            y[row] = static_cast<XT>(s);
    }
}

// Whole strips, y overwritten.
template <int HB, int G, int U, bool NT, typename VT, typename XT, typename AT>
__global__ __launch_bounds__(kSpmvThreads) void spmv_group_kernel(
    int rows, int strips, int height, int bits, const int* __restrict__ strip_ptr,
    const uint32_t* __restrict__ word, const VT* __restrict__ val, const XT* __restrict__ x, XT* __restrict__ y,
    int long_len) {
    constexpr int NG = kWave / G;
    __shared__ AT buf[kSpmvWaves][HB * kWave];
    const int lane = lane_id();
    const int wave = uniform(static_cast<int>(threadIdx.x) / kWave);
    const int strip0 = (xcd_logical_block(blockIdx.x, gridDim.x) * kSpmvWaves + wave) * NG;
    if (strip0 >= strips) return;
    const int strip = strip0 + lane / G;
    int lo = 0, hi = 0;
    if (strip < strips) {
        lo = strip_ptr[strip];
        hi = strip_ptr[strip + 1];
    }
    group_runs<HB, G, U, NT, VT, XT, AT>(lo, hi, long_len, bits, word, val, x, buf[wave], lane,
                                         [&](int gg, int rr, AT s) {
                                             const int st = strip0 + gg;
                                             const int row = st * height + rr;
                                             if (st < strips && rr < height && row < rows) y[row] = static_cast<XT>(s);
                                         });
}

// Column-blocked schedule in one launch: workgroup b takes column block
// b % nb (with nb = 8 that is the XCD the workgroup runs on, so each XCD
// gathers from one eighth of x) and strips from (b / nb) onward; run cb of
// each strip goes to partial[cb * rows + row].  colblock_combine_kernel then
// adds the nb partials of every row in block order.
template <int HB, int G, int U, bool NT, typename VT, typename XT, typename AT>
__global__ __launch_bounds__(kSpmvThreads) void spmv_colblock_concurrent_kernel(
    int rows, int strips, int height, int bits, const int* __restrict__ strip_ptr,
    const uint32_t* __restrict__ word, const VT* __restrict__ val, const XT* __restrict__ x,
    AT* __restrict__ partial, const int* __restrict__ split, int nb, int long_len) {
    constexpr int NG = kWave / G;
    __shared__ AT buf[kSpmvWaves][HB * kWave];
    const int lane = lane_id();
    const int wave = uniform(static_cast<int>(threadIdx.x) / kWave);
    const int cb = static_cast<int>(blockIdx.x) % nb;
    const int strip0 = (static_cast<int>(blockIdx.x) / nb * kSpmvWaves + wave) * NG;
    if (strip0 >= strips) return;
    const int strip = strip0 + lane / G;
    int lo = 0, hi = 0;
    if (strip < strips) {
        const int* sp = split + static_cast<size_t>(strip) * (nb - 1);
        lo = cb == 0 ? strip_ptr[strip] : sp[cb - 1];
        hi = cb == nb - 1 ? strip_ptr[strip + 1] : sp[cb];
    }
    AT* part = partial + static_cast<size_t>(cb) * rows;
    group_runs<HB, G, U, NT, VT, XT, AT>(lo, hi, long_len, bits, word, val, x, buf[wave], lane,
                                         [&](int gg, int rr, AT s) {
                                             const int st = strip0 + gg;
                                             const int row = st * height + rr;
                                             if (st < strips && rr < height && row < rows) part[row] = s;
                                         });
}

template <typename XT, typename AT>
__global__ __launch_bounds__(256) void colblock_combine_kernel(int rows, int nb, const AT* __restrict__ partial,
                                                               XT* __restrict__ y) {
    const int i = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= rows) return;
    AT s = partial[i];
    for (int k = 1; k < nb; ++k) s += partial[static_cast<size_t>(k) * rows + i];
    y[i] = static_cast<XT>(s);
}

// Plan of the column-blocked schedule: split[s*(nb-1) + b-1] = first entry of
// strip s whose column is >= b*bw, for b = 1..nb-1 (strip entries ascending by
// column).  One wave per strip; the count of entries below each boundary is
// accumulated with ballots (lane b-1 keeps boundary b).
__global__ __launch_bounds__(256) void colblock_plan_kernel(int strips, int bits, int bw, int nb,
                                                            const int* __restrict__ strip_ptr,
                                                            const uint32_t* __restrict__ word,
                                                            int* __restrict__ split) {
    const int lane = lane_id();
    const int wave = uniform(static_cast<int>(threadIdx.x) / kWave);
    const int strip = xcd_logical_block(blockIdx.x, gridDim.x) * 4 + wave;
    if (strip >= strips) return;
    const int s0 = strip_ptr[strip], s1 = strip_ptr[strip + 1];
    // U rounds of 64 words are loaded before any is counted, so a strip of up
    // to 64*U entries costs one memory round trip, not one per round.
    constexpr int U = 8;
    int below = 0;
    for (int base = s0; base < s1; base += U * kWave) {
        uint32_t w[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = base + u * kWave + lane;
            w[u] = e < s1 ? word[e] : 0u;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (base + u * kWave >= s1) break;  // uniform
            const int e = base + u * kWave + lane;
            const int blk = e < s1 ? static_cast<int>(w[u] >> bits) / bw : nb;
            for (int b = 1; b < nb; ++b) {
                const uint64_t m = ballot(blk < b);
                if (lane == b - 1) below += __popcll(m);
            }
        }
    }
    if (lane < nb - 1) split[static_cast<size_t>(strip) * (nb - 1) + lane] = s0 + below;
}

namespace {

struct Launch {
    const cmrs_mat_t* A;
    int strips;
    const void* x;
    void* y;
    const int* split;
    int nb;
    hipStream_t stream;
    void* partial = nullptr;  // concurrent column-blocked schedule: nb * rows partial sums
};

template <typename VT, typename XT, typename AT, int HB, bool NT, bool REG>
hipError_t launch_one(const Launch& L) {
    const int blocks = (L.strips + kSpmvWaves - 1) / kSpmvWaves;
    constexpr int U = HB >= 16 ? 4 : 2;
    const auto* v = static_cast<const VT*>(L.A->val);
    const auto* xx = static_cast<const XT*>(L.x);
    auto* yy = static_cast<XT*>(L.y);
    const int passes = L.split ? L.nb : 1;
    for (int b = 0; b < passes; ++b) {
        hipLaunchKernelGGL((spmv_kernel<HB, U, NT, REG, VT, XT, AT>), dim3(blocks), dim3(kSpmvThreads), 0, L.stream,
                           L.A->rows, L.strips, L.A->height, L.A->bits, L.A->strip_ptr, L.A->col_word, v, xx, yy,
                           L.split, L.nb, b);
    }
    return hipGetLastError();
}

template <typename VT, typename XT, typename AT, int HB, int G, bool NT>
hipError_t launch_group_g(const Launch& L) {
    constexpr int NG = kWave / G;
    // Loads per lane in one step: about 1.5 times the entries a lane gets
    // from spmv_group_width (4 up to height 8, 8 above), so that most strips
    // take one step while few loads go to the clamped slots past their end:
    // 6 up to height 8, 12 at height 32; 8 at height 16, where 12 was mixed.
    // Cold, against 8 everywhere: 2^20 Poisson(16) rows, fp32, height
    // 2/4/32 179/155/125 -> 164/146/112 us; the skewed rows, fp64, height 32
    // 162 -> 154 us (6 there: 173 us).
    constexpr int U = HB <= 8 ? 6 : (HB <= 16 ? 8 : 12);
    const int waves = (L.strips + NG - 1) / NG;
    const int blocks = (waves + kSpmvWaves - 1) / kSpmvWaves;
    hipLaunchKernelGGL((spmv_group_kernel<HB, G, U, NT, VT, XT, AT>), dim3(blocks), dim3(kSpmvThreads), 0, L.stream,
                       L.A->rows, L.strips, L.A->height, L.A->bits, L.A->strip_ptr, L.A->col_word,
                       static_cast<const VT*>(L.A->val), static_cast<const XT*>(L.x), static_cast<XT*>(L.y),
                       4 * U * G);
    return hipGetLastError();
}


template <typename VT, typename XT, typename AT, int HB, bool NT>
hipError_t launch_group(const Launch& L) {
    const int g = spmv_group_width(L.A->nnz, L.strips, HB);
    if constexpr (HB <= 2) {
        if (g <= 2) return launch_group_g<VT, XT, AT, HB, 2, NT>(L);
    }
    if constexpr (HB <= 4) {
        if (g <= 4) return launch_group_g<VT, XT, AT, HB, 4, NT>(L);
    }
    if constexpr (HB <= 8) {
        if (g <= 8) return launch_group_g<VT, XT, AT, HB, 8, NT>(L);
    }
    if constexpr (HB <= 16) {
        if (g <= 16) return launch_group_g<VT, XT, AT, HB, 16, NT>(L);
    }
    if (g <= 32) return launch_group_g<VT, XT, AT, HB, 32, NT>(L);
    return launch_group_g<VT, XT, AT, HB, 64, NT>(L);
}

template <typename VT, typename XT, typename AT, int HB, int G>
hipError_t launch_concurrent_g(const Launch& L) {
    constexpr int NG = kWave / G;
    // Loads per lane in one step: 1.5 times the ~4 entries a lane gets (the
    // rule below), so nearly every run takes one step while few loads go to
    // the clamped slots past its end (cold, 2^20 Poisson(16) rows, 4 blocks,
    // height 32: fp64 136 -> 130 us, fp32 116 -> 109 us against 8; 4 was
    // slower, 160 us).
    constexpr int U = 6;
    const int waves = (L.strips + NG - 1) / NG;
    const int blocks_per_cb = (waves + kSpmvWaves - 1) / kSpmvWaves;
    auto* part = static_cast<AT*>(L.partial);
    hipLaunchKernelGGL((spmv_colblock_concurrent_kernel<HB, G, U, true, VT, XT, AT>), dim3(blocks_per_cb * L.nb),
                       dim3(kSpmvThreads), 0, L.stream, L.A->rows, L.strips, L.A->height, L.A->bits, L.A->strip_ptr,
                       L.A->col_word, static_cast<const VT*>(L.A->val), static_cast<const XT*>(L.x), part, L.split,
                       L.nb, 4 * U * G);
    hipLaunchKernelGGL((colblock_combine_kernel<XT, AT>), dim3((L.A->rows + 255) / 256), dim3(256), 0, L.stream,
                       L.A->rows, L.nb, static_cast<const AT*>(part), static_cast<XT*>(L.y));
    return hipGetLastError();
}

// Lanes per column-block run: about 4 entries per lane for the average run.
// (Measured with 4 blocks, cold, 2^20-row Poisson(16) rows: fp64 at height
// 8/16/32 204/161/131 us against 244/190/145 us with 8 entries per lane;
// fp32 at height 32 115 against 147 us.)
template <typename VT, typename XT, typename AT, int HB>
hipError_t launch_concurrent(const Launch& L) {
    const double avg = static_cast<double>(L.A->nnz) / (static_cast<double>(L.strips) * L.nb);
    int g = 2;
    while (g < 64 && g * 4 * 1.5 < avg) g <<= 1;
    switch (g) {
        case 2: return launch_concurrent_g<VT, XT, AT, HB, 2>(L);
        case 4: return launch_concurrent_g<VT, XT, AT, HB, 4>(L);
        case 8: return launch_concurrent_g<VT, XT, AT, HB, 8>(L);
        case 16: return launch_concurrent_g<VT, XT, AT, HB, 16>(L);
        case 32: return launch_concurrent_g<VT, XT, AT, HB, 32>(L);
        default: return launch_concurrent_g<VT, XT, AT, HB, 64>(L);
    }
}

template <typename VT, typename XT, typename AT, int HB>
hipError_t launch_hb(int variant, const Launch& L) {
    if (L.partial != nullptr) return launch_concurrent<VT, XT, AT, HB>(L);
    if (variant == CMRS_SPMV_GROUP || variant == CMRS_SPMV_GROUP_NT) {
        if (L.split == nullptr)
            return variant == CMRS_SPMV_GROUP_NT ? launch_group<VT, XT, AT, HB, true>(L)
                                                 : launch_group<VT, XT, AT, HB, false>(L);
        variant = variant == CMRS_SPMV_GROUP_NT ? CMRS_SPMV_LDS_NT : CMRS_SPMV_LDS;
    }
    const bool nt = variant == CMRS_SPMV_LDS_NT || variant == CMRS_SPMV_REG_NT;
    const bool reg = (variant == CMRS_SPMV_REG || variant == CMRS_SPMV_REG_NT) && HB <= 8;
    if constexpr (HB <= 8) {
        if (reg) return nt ? launch_one<VT, XT, AT, HB, true, true>(L) : launch_one<VT, XT, AT, HB, false, true>(L);
    }
    return nt ? launch_one<VT, XT, AT, HB, true, false>(L) : launch_one<VT, XT, AT, HB, false, false>(L);
}

template <typename VT, typename XT, typename AT>
hipError_t launch_typed(int variant, const Launch& L) {
    switch (next_pow2(L.A->height)) {
        case 1: return launch_hb<VT, XT, AT, 1>(variant, L);
        case 2: return launch_hb<VT, XT, AT, 2>(variant, L);
        case 4: return launch_hb<VT, XT, AT, 4>(variant, L);
        case 8: return launch_hb<VT, XT, AT, 8>(variant, L);
        case 16: return launch_hb<VT, XT, AT, 16>(variant, L);
        default: return launch_hb<VT, XT, AT, 32>(variant, L);
    }
}

hipError_t dispatch(int variant, const Launch& L) {
    if (L.A->val_dtype == CMRS_R64F) return launch_typed<double, double, double>(variant, L);
    if (L.A->val_dtype == CMRS_R32F) return launch_typed<float, float, float>(variant, L);
    return launch_typed<bf16_t, float, float>(variant, L);
}

}  // namespace

// Lanes per strip of the strip-group kernels: about `per` entries per lane
// for the average strip, per = 4 up to height 8 and 8 above.  (Measured, cold
// fp64: 2^20-row Poisson(16) rows at height 2/4/8, 268/219/199 us with 8
// entries per lane against 221/198/188 us with 4, and the skewed 2*10^6-row
// workload gains a little there too; at heights 16 and 32 that workload loses
// with 4, e.g. 142 -> 147 us at height 16 and 162 -> 185 us at height 32,
// where one wave then takes each strip.)
int spmv_group_width(int nnz, int strips, int hb) {
    const double avg = strips > 0 ? static_cast<double>(nnz) / strips : 0.0;
    const int per = hb <= 8 ? 4 : 8;
    int g = 2;
    while (g < 64 && g * per * 1.5 < avg) g <<= 1;
    return g < hb ? hb : g;
}

int resolve_spmv_variant(const cmrs_mat_t* A, int variant) {
    (void)A;
    if (variant != CMRS_SPMV_AUTO) return variant;
    return CMRS_SPMV_GROUP_NT;
}

hipError_t launch_spmv(const cmrs_mat_t* A, const void* x, void* y, cmrs_dtype_t xy_dtype, int variant,
                       hipStream_t stream) {
    (void)xy_dtype;
    const int strips = (A->rows + A->height - 1) / A->height;
    if (strips == 0) return hipSuccess;
    return dispatch(resolve_spmv_variant(A, variant), Launch{A, strips, x, y, nullptr, 1, stream});
}

hipError_t launch_colblock_plan(const cmrs_mat_t* A, int nb, int bw, int* split, hipStream_t stream) {
    const int strips = (A->rows + A->height - 1) / A->height;
    if (strips == 0 || nb <= 1) return hipSuccess;
    const int blocks = (strips + 3) / 4;
    hipLaunchKernelGGL(colblock_plan_kernel, dim3(blocks), dim3(256), 0, stream, strips, A->bits, bw, nb,
                       A->strip_ptr, A->col_word, split);
    return hipGetLastError();
}

// Scratch of the allocation-free concurrent column-blocked product
// (cmrs_spmv_colblock_noalloc): the nb * rows partial sums live in this
// file-scope array instead of a caller workspace.  Every GPU the library runs
// on holds its own copy at its own address until the process ends; host code
// must use that address (from hipGetSymbolAddress), never the array's name,
// which on the host is only a stand-in for the symbol.
static __device__ __align__(256) unsigned char scratch[CMRS_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch(void** ptr) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (p == nullptr) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

hipError_t launch_spmv_colblock(const cmrs_mat_t* A, const void* x, void* y, int variant, int nb,
                                const int* split, int schedule, void* workspace, hipStream_t stream) {
    const int strips = (A->rows + A->height - 1) / A->height;
    if (strips == 0) return hipSuccess;
    variant = resolve_spmv_variant(A, variant);
    if (nb <= 1) return dispatch(variant, Launch{A, strips, x, y, nullptr, 1, stream});
    if (schedule == CMRS_COLBLOCK_PHASED) return launch_spmv_phased(A, x, y, nb, split, stream);
    Launch L{A, strips, x, y, split, nb, stream};
    if (schedule == CMRS_COLBLOCK_CONCURRENT) L.partial = workspace;
    return dispatch(variant, L);
}

}  // namespace cmrs
