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
//        the reduction is a register reduce-scatter butterfly.  Small heights.
// Workgroups hold 4 waves (4 strips); workgroup ids are renumbered so that each
// XCD processes one contiguous range of strips.
#include "cmrs_device.hpp"
#include "cmrs_internal.hpp"

namespace cmrs {

constexpr int kSpmvWaves = 4;
constexpr int kSpmvThreads = kSpmvWaves * kWave;

// Sum, for each row r < HB, the 64 per-lane partials b[r*64 + l].  Lanes form
// HB groups of G = 64/HB; group r sums row r: each lane adds HB consecutive
// partials, then an xor butterfly inside the group.  Every lane of the group
// ends with the same value.
template <int HB, typename AT>
__device__ inline AT reduce_rows_lds(const AT* b, int lane) {
    constexpr int G = kWave / HB;
    constexpr int PER = kWave / G;
    const int r = lane / G, q = lane % G;
    const AT* p = b + r * kWave + q * PER;
    AT s = p[0];
#pragma unroll
    for (int i = 1; i < PER; ++i) s += p[i];
#pragma unroll
    for (int off = G / 2; off >= 1; off >>= 1) s += __shfl_xor(s, off);
    return s;
}

template <int HB, int U, typename VT, typename XT, typename AT>
__global__ __launch_bounds__(kSpmvThreads) void spmv_lds_kernel(
    int rows, int strips, int height, int bits, const int* __restrict__ strip_ptr,
    const uint32_t* __restrict__ word, const VT* __restrict__ val, const XT* __restrict__ x,
    XT* __restrict__ y) {
    __shared__ AT buf[kSpmvWaves][HB * kWave];
    const int lane = lane_id();
    const int wave = uniform(static_cast<int>(threadIdx.x) / kWave);
    const int strip = xcd_logical_block(blockIdx.x, gridDim.x) * kSpmvWaves + wave;
    if (strip >= strips) return;
    AT* b = buf[wave];
#pragma unroll
    for (int r = 0; r < HB; ++r) b[r * kWave + lane] = AT(0);

    const int s0 = strip_ptr[strip], s1 = strip_ptr[strip + 1];
    const uint32_t mask = (1u << bits) - 1u;
    for (int base = s0; base < s1; base += U * kWave) {
        uint32_t w[U];
        VT v[U];
        XT xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = base + u * kWave + lane;
            if (j < s1) {
                w[u] = word[j];
                v[u] = val[j];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = base + u * kWave + lane;
            if (j < s1) xv[u] = x[w[u] >> bits];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = base + u * kWave + lane;
            if (j < s1) {
                const AT p = static_cast<AT>(ValTraits<VT>::widen(v[u])) * static_cast<AT>(xv[u]);
                const int r = static_cast<int>(w[u] & mask) & (HB - 1);
                atomicAdd(&b[r * kWave + lane], p);
            }
        }
    }
    wave_lds_sync();
    const AT s = reduce_rows_lds<HB>(b, lane);
    constexpr int G = kWave / HB;
    const int r = lane / G;
    const int row = strip * height + r;
    if ((lane % G) == 0 && r < height && row < rows) y[row] = static_cast<XT>(s);
}

template <int HB, int U, typename VT, typename XT, typename AT>
__global__ __launch_bounds__(kSpmvThreads) void spmv_reg_kernel(
    int rows, int strips, int height, int bits, const int* __restrict__ strip_ptr,
    const uint32_t* __restrict__ word, const VT* __restrict__ val, const XT* __restrict__ x,
    XT* __restrict__ y) {
    const int lane = lane_id();
    const int wave = uniform(static_cast<int>(threadIdx.x) / kWave);
    const int strip = xcd_logical_block(blockIdx.x, gridDim.x) * kSpmvWaves + wave;
    if (strip >= strips) return;
    AT acc[HB];
#pragma unroll
    for (int r = 0; r < HB; ++r) acc[r] = AT(0);

    const int s0 = strip_ptr[strip], s1 = strip_ptr[strip + 1];
    const uint32_t mask = (1u << bits) - 1u;
    for (int base = s0; base < s1; base += U * kWave) {
        uint32_t w[U];
        VT v[U];
        XT xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = base + u * kWave + lane;
            if (j < s1) {
                w[u] = word[j];
                v[u] = val[j];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = base + u * kWave + lane;
            if (j < s1) xv[u] = x[w[u] >> bits];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = base + u * kWave + lane;
            if (j < s1) {
                const AT p = static_cast<AT>(ValTraits<VT>::widen(v[u])) * static_cast<AT>(xv[u]);
                const uint32_t r = w[u] & mask;
#pragma unroll
                for (int k = 0; k < HB; ++k) acc[k] += (r == static_cast<uint32_t>(k)) ? p : AT(0);
            }
        }
    }
    // Reduce-scatter butterfly: at the step with xor offset o, a lane whose
    // bit o is set keeps the upper half of its rows and sends the lower half.
    // After log2(HB) steps lane l holds a partial of row l / (64/HB); the
    // remaining offsets sum the group.
    int n = HB;
#pragma unroll
    for (int o = kWave / 2; o >= 1; o >>= 1) {
        if (n > 1) {
            const bool upper = (lane & o) != 0;
#pragma unroll
            for (int i = 0; i < HB / 2; ++i) {
                if (i < n / 2) {
                    const AT send = upper ? acc[i] : acc[i + n / 2];
                    const AT keep = upper ? acc[i + n / 2] : acc[i];
                    acc[i] = keep + __shfl_xor(send, o);
                }
            }
            n >>= 1;
        } else {
            acc[0] += __shfl_xor(acc[0], o);
        }
    }
    constexpr int G = kWave / HB;
    const int r = lane / G;
    const int row = strip * height + r;
    if ((lane % G) == 0 && r < height && row < rows) y[row] = static_cast<XT>(acc[0]);
}

namespace {

template <typename VT, typename XT, typename AT, int HB>
hipError_t launch_hb(int variant, const cmrs_mat_t* A, int strips, const void* x, void* y,
                     hipStream_t stream) {
    const int blocks = (strips + kSpmvWaves - 1) / kSpmvWaves;
    constexpr int U = HB >= 16 ? 4 : 2;
    const auto* sp = A->strip_ptr;
    const auto* w = A->col_word;
    const auto* v = static_cast<const VT*>(A->val);
    const auto* xx = static_cast<const XT*>(x);
    auto* yy = static_cast<XT*>(y);
    if (variant == CMRS_SPMV_REG && HB <= 8) {
        hipLaunchKernelGGL((spmv_reg_kernel<HB, U, VT, XT, AT>), dim3(blocks), dim3(kSpmvThreads), 0, stream,
                           A->rows, strips, A->height, A->bits, sp, w, v, xx, yy);
    } else {
        hipLaunchKernelGGL((spmv_lds_kernel<HB, U, VT, XT, AT>), dim3(blocks), dim3(kSpmvThreads), 0, stream,
                           A->rows, strips, A->height, A->bits, sp, w, v, xx, yy);
    }
    return hipGetLastError();
}

template <typename VT, typename XT, typename AT>
hipError_t launch_typed(int variant, const cmrs_mat_t* A, int strips, const void* x, void* y,
                        hipStream_t stream) {
    switch (next_pow2(A->height)) {
        case 1: return launch_hb<VT, XT, AT, 1>(variant, A, strips, x, y, stream);
        case 2: return launch_hb<VT, XT, AT, 2>(variant, A, strips, x, y, stream);
        case 4: return launch_hb<VT, XT, AT, 4>(variant, A, strips, x, y, stream);
        case 8: return launch_hb<VT, XT, AT, 8>(variant, A, strips, x, y, stream);
        case 16: return launch_hb<VT, XT, AT, 16>(variant, A, strips, x, y, stream);
        default: return launch_hb<VT, XT, AT, 32>(variant, A, strips, x, y, stream);
    }
}

}  // namespace

int resolve_spmv_variant(const cmrs_mat_t* A, int variant) {
    if (variant != CMRS_SPMV_AUTO) return variant;
    return CMRS_SPMV_LDS;
}

hipError_t launch_spmv(const cmrs_mat_t* A, const void* x, void* y, cmrs_dtype_t xy_dtype, int variant,
                       hipStream_t stream) {
    const int strips = (A->rows + A->height - 1) / A->height;
    if (strips == 0) return hipSuccess;
    variant = resolve_spmv_variant(A, variant);
    if (A->val_dtype == CMRS_R64F) return launch_typed<double, double, double>(variant, A, strips, x, y, stream);
    if (A->val_dtype == CMRS_R32F) return launch_typed<float, float, float>(variant, A, strips, x, y, stream);
    return launch_typed<bf16_t, float, float>(variant, A, strips, x, y, stream);
}

}  // namespace cmrs
