// Column-phased CMRS SpMV: the column-blocked schedule without partial sums
// in memory.
//
// For a sorted matrix (entries of a strip ascending by column; Sec. 4,
// fourth optimisation) the entries of strip s with columns in block b are a
// contiguous run; the colblock plan holds the run boundaries.  Here every
// wave owns NG = 64/G whole strips (G lanes each, as the strip-group SpMV)
// and walks column block 0 of all of them, then block 1, and so on, adding
// into the same per-lane partial sums of Algorithm 1 (in LDS) across the
// blocks; after the last block it reduces them and writes its rows of y.
// All waves of an XCD start together and do similar work, so at any time
// they gather from one or two blocks of x: with blocks of 1/nb of x, those
// stay in the XCD's L2 instead of coming from the MALL.  Every entry and
// every run boundary is read once; nothing is written but y.  The run
// boundary of the next block is loaded while the current block runs.
#include "cmrs_internal.hpp"
#include "spmv_device.hpp"

namespace cmrs {

template <int HB, int G, int U, typename VT, typename XT, typename AT>
__global__ __launch_bounds__(kSpmvThreads) void spmv_phased_kernel(
    int rows, int strips, int height, int bits, const int* __restrict__ strip_ptr, const uint32_t* __restrict__ word,
    const VT* __restrict__ val, const XT* __restrict__ x, XT* __restrict__ y, const int* __restrict__ split, int nb) {
    constexpr int NG = kWave / G;
    __shared__ AT buf[kSpmvWaves][HB * kWave];
    const int lane = lane_id();
    const int wave = uniform(static_cast<int>(threadIdx.x) / kWave);
    const int strip0 = (xcd_logical_block(blockIdx.x, gridDim.x) * kSpmvWaves + wave) * NG;
    if (strip0 >= strips) return;
    const int g = lane / G, q = lane % G;
    const int strip = strip0 + g;
    AT* b = buf[wave];
#pragma unroll
    for (int r = 0; r < HB; ++r) b[(g * HB + r) * G + q] = AT(0);
    int lo = 0, hi = 0, end = 0;
    const int* sp = split + static_cast<size_t>(strip < strips ? strip : 0) * (nb - 1);
    if (strip < strips) {
        lo = strip_ptr[strip];
        end = strip_ptr[strip + 1];
        hi = nb > 1 ? sp[0] : end;
    }
    for (int blk = 0; blk < nb; ++blk) {
        // Boundary of the next run, loaded while this one is walked.
        int next = end;
        if (strip < strips && blk + 2 < nb) next = sp[blk + 1];
        group_walk<HB, G, U, true, VT, XT, AT>(lo, hi, bits, word, val, x, b, g, q);
        lo = hi;
        hi = next;
    }
    wave_lds_sync();
    group_reduce<HB, G, AT>(b, lane, [&](int gg, int rr, AT s) {
        const int st = strip0 + gg;
        const int row = st * height + rr;
        if (st < strips && rr < height && row < rows) y[row] = static_cast<XT>(s);
    });
}

namespace {

template <typename VT, typename XT, typename AT, int HB, int G>
hipError_t launch_phased_g(const cmrs_mat_t* A, const void* x, void* y, int nb, const int* split, hipStream_t stream) {
    constexpr int NG = kWave / G;
    const int strips = (A->rows + A->height - 1) / A->height;
    const int waves = (strips + NG - 1) / NG;
    const int blocks = (waves + kSpmvWaves - 1) / kSpmvWaves;
    hipLaunchKernelGGL((spmv_phased_kernel<HB, G, 8, VT, XT, AT>), dim3(blocks), dim3(kSpmvThreads), 0, stream,
                       A->rows, strips, A->height, A->bits, A->strip_ptr, A->col_word, static_cast<const VT*>(A->val),
                       static_cast<const XT*>(x), static_cast<XT*>(y), split, nb);
    return hipGetLastError();
}

template <typename VT, typename XT, typename AT, int HB>
hipError_t launch_phased_hb(const cmrs_mat_t* A, const void* x, void* y, int nb, const int* split, hipStream_t stream) {
    const int strips = (A->rows + A->height - 1) / A->height;
    // About 8 entries per lane for the average run (a strip's entries in one block).
    const double avg = strips > 0 ? static_cast<double>(A->nnz) / (static_cast<double>(strips) * nb) : 0.0;
    int g = 2;
    while (g < 64 && g * 8 * 1.5 < avg) g <<= 1;
    switch (g) {
        case 2: return launch_phased_g<VT, XT, AT, HB, 2>(A, x, y, nb, split, stream);
        case 4: return launch_phased_g<VT, XT, AT, HB, 4>(A, x, y, nb, split, stream);
        case 8: return launch_phased_g<VT, XT, AT, HB, 8>(A, x, y, nb, split, stream);
        case 16: return launch_phased_g<VT, XT, AT, HB, 16>(A, x, y, nb, split, stream);
        case 32: return launch_phased_g<VT, XT, AT, HB, 32>(A, x, y, nb, split, stream);
        default: return launch_phased_g<VT, XT, AT, HB, 64>(A, x, y, nb, split, stream);
    }
}

template <typename VT, typename XT, typename AT>
hipError_t launch_phased_typed(const cmrs_mat_t* A, const void* x, void* y, int nb, const int* split,
                               hipStream_t stream) {
    switch (next_pow2(A->height)) {
        case 1: return launch_phased_hb<VT, XT, AT, 1>(A, x, y, nb, split, stream);
        case 2: return launch_phased_hb<VT, XT, AT, 2>(A, x, y, nb, split, stream);
        case 4: return launch_phased_hb<VT, XT, AT, 4>(A, x, y, nb, split, stream);
        case 8: return launch_phased_hb<VT, XT, AT, 8>(A, x, y, nb, split, stream);
        case 16: return launch_phased_hb<VT, XT, AT, 16>(A, x, y, nb, split, stream);
        default: return launch_phased_hb<VT, XT, AT, 32>(A, x, y, nb, split, stream);
    }
}

}  // namespace

hipError_t launch_spmv_phased(const cmrs_mat_t* A, const void* x, void* y, int nb, const int* split,
                              hipStream_t stream) {
    if (A->rows == 0) return hipSuccess;
    if (A->val_dtype == CMRS_R64F) return launch_phased_typed<double, double, double>(A, x, y, nb, split, stream);
    if (A->val_dtype == CMRS_R32F) return launch_phased_typed<float, float, float>(A, x, y, nb, split, stream);
    return launch_phased_typed<bf16_t, float, float>(A, x, y, nb, split, stream);
}

}  // namespace cmrs
