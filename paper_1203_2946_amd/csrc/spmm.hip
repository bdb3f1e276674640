// CMRS products with several right-hand sides, single and batched.
//
// The hot loop is Algorithm 1 of Sec. 4 with the wave's 64 lanes split three
// ways: S = 64 / (G * R) strips at a time, G entry slots per strip and R =
// next_pow2(nrhs) right-hand sides per entry.  Lane (s, e, k) walks entries
// e, e + G, ... of its strip, reads each packed word and value (the R lanes
// of an entry read the same address: one request), gathers x_k[col] from the
// row-major X (the R gathers of an entry are one contiguous piece) and adds
// the product to its own partial for (row, k) in LDS.  A strip's results are
// then the sums over its G entry slots, taken in slot order by the lane that
// writes y_k[row].
//
// The batched path runs that body from one persistent kernel: waves take
// work tiles (a matrix and a range of its strips) from a queue counter in the
// plan until the queue is empty; the last wave out resets the counter, so
// the same plan can be launched again and replayed from a HIP graph.  A grid
// stride over strip passes (the listing's loop over strips in the paper's
// appendix) is the special case of one tile per wave.
#include <string.h>

#include <algorithm>
#include <vector>

#include "cmrs_device.hpp"
#include "cmrs_internal.hpp"

namespace cmrs {

constexpr int kSpmmWaves = 4;
constexpr int kSpmmThreads = kSpmmWaves * kWave;
constexpr int kSpmmUnroll = 4;

template <typename T>
__device__ inline T nt_load(const T* p) {
    return __builtin_nontemporal_load(p);
}
__device__ inline bf16_t nt_load(const bf16_t* p) {
    bf16_t v;
    v.bits = __builtin_nontemporal_load(&p->bits);
    return v;
}

// Strips [sb, sb + S) (those below s_end) of matrix m; buf holds HB * 64
// partials of this wave.
template <int HB, typename VT, typename XT, typename AT>
__device__ inline void spmm_pass(const SpmmMat& m, int sb, int s_end, AT* __restrict__ buf, int lane) {
    const int rl_log = m.rl_log, g_log = m.g_log;
    const int R = 1 << rl_log, G = 1 << g_log;
    const int k = lane & (R - 1);
    const int e = (lane >> rl_log) & (G - 1);
    const int ss = lane >> (rl_log + g_log);
    const int s = sb + ss;
    const int bits = m.bits;
    const uint32_t mask = (1u << bits) - 1u;
#pragma unroll
    for (int r = 0; r < HB; ++r) buf[r * kWave + lane] = AT(0);
    if (s < s_end) {
        const int lo = m.strip_ptr[s], hi = m.strip_ptr[s + 1];
        const VT* __restrict__ val = static_cast<const VT*>(m.val);
        const XT* __restrict__ x = static_cast<const XT*>(m.x);
        const bool kact = k < m.nrhs;
        const size_t ldx = static_cast<size_t>(m.ldx);
        for (int base = lo + e; base < hi; base += kSpmmUnroll * G) {
            uint32_t w[kSpmmUnroll];
            VT v[kSpmmUnroll];
            XT xv[kSpmmUnroll];
#pragma unroll
            for (int u = 0; u < kSpmmUnroll; ++u) {
                const int j = base + u * G;
                if (j < hi) {
                    w[u] = nt_load(m.word + j);
                    v[u] = nt_load(val + j);
                }
            }
#pragma unroll
            for (int u = 0; u < kSpmmUnroll; ++u) {
                const int j = base + u * G;
                if (j < hi && kact) xv[u] = x[static_cast<size_t>(w[u] >> bits) * ldx + k];
            }
#pragma unroll
            for (int u = 0; u < kSpmmUnroll; ++u) {
                const int j = base + u * G;
                if (j < hi && kact) {
                    const AT p = static_cast<AT>(ValTraits<VT>::widen(v[u])) * static_cast<AT>(xv[u]);
                    atomicAdd(&buf[static_cast<int>(w[u] & mask & (HB - 1)) * kWave + lane], p);
                }
            }
        }
    }
    wave_lds_sync();
    // Outputs o = (strip slot, row, k) with k fastest; each sums the G entry
    // slots of its strip in slot order.
    const int nout = kWave * HB >> g_log;
    XT* __restrict__ y = static_cast<XT*>(m.y);
    const size_t ldy = static_cast<size_t>(m.ldy);
    for (int o = lane; o < nout; o += kWave) {
        const int kk = o & (R - 1);
        const int rr = (o >> rl_log) & (HB - 1);
        const int so = o >> rl_log >> __builtin_ctz(HB);
        const AT* p = buf + rr * kWave + ((so << g_log) << rl_log) + kk;
        AT sum = p[0];
        for (int q = 1; q < G; ++q) sum += p[q << rl_log];
        const int strip = sb + so;
        const long long row = static_cast<long long>(strip) * m.height + rr;
        if (strip < s_end && rr < m.height && row < m.rows && kk < m.nrhs)
            y[static_cast<size_t>(row) * ldy + kk] = static_cast<XT>(sum);
    }
    wave_lds_sync();
}

template <int HB, typename VT, typename XT, typename AT>
__global__ __launch_bounds__(kSpmmThreads) void spmm_kernel(SpmmMat m, int strips) {
    __shared__ AT buf[kSpmmWaves][HB * kWave];
    const int lane = lane_id();
    const int wave = uniform(static_cast<int>(threadIdx.x) / kWave);
    const int S = kWave >> (m.rl_log + m.g_log);
    const long long sb = (static_cast<long long>(xcd_logical_block(blockIdx.x, gridDim.x)) * kSpmmWaves + wave) * S;
    if (sb >= strips) return;
    spmm_pass<HB, VT, XT, AT>(m, static_cast<int>(sb), strips, buf[wave], lane);
}

template <int HB, typename VT, typename XT, typename AT>
__device__ inline void spmm_tile(const SpmmMat& m, int s0, int s1, AT* buf, int lane) {
    const int S = kWave >> (m.rl_log + m.g_log);
    for (int sb = s0; sb < s1; sb += S) spmm_pass<HB, VT, XT, AT>(m, sb, s1, buf, lane);
}

// queue[0]: next tile; queue[kQueueDone]: waves finished.  Both are zero at
// launch and are zero again when the last wave leaves.
constexpr int kQueueDone = 16;

template <typename VT, typename XT, typename AT>
__global__ __launch_bounds__(kSpmmThreads) void spmm_persistent_kernel(const SpmmMat* __restrict__ mats,
                                                                       const SpmmTile* __restrict__ tiles,
                                                                       int ntiles, unsigned* __restrict__ queue,
                                                                       int waves_total, int wave_slots) {
    extern __shared__ __align__(16) unsigned char spmm_smem[];
    const int lane = lane_id();
    const int wave = uniform(static_cast<int>(threadIdx.x) / kWave);
    AT* buf = reinterpret_cast<AT*>(spmm_smem) + static_cast<size_t>(wave) * wave_slots;
    for (;;) {
        unsigned t = 0;
        if (lane == 0) t = __hip_atomic_fetch_add(&queue[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        t = static_cast<unsigned>(uniform(static_cast<int>(__shfl(t, 0))));
        if (t >= static_cast<unsigned>(ntiles)) break;
        const SpmmTile tile = tiles[t];
        const SpmmMat m = mats[tile.mat];
        switch (m.hb) {
            case 1: spmm_tile<1, VT, XT, AT>(m, tile.s0, tile.s1, buf, lane); break;
            case 2: spmm_tile<2, VT, XT, AT>(m, tile.s0, tile.s1, buf, lane); break;
            case 4: spmm_tile<4, VT, XT, AT>(m, tile.s0, tile.s1, buf, lane); break;
            case 8: spmm_tile<8, VT, XT, AT>(m, tile.s0, tile.s1, buf, lane); break;
            case 16: spmm_tile<16, VT, XT, AT>(m, tile.s0, tile.s1, buf, lane); break;
            default: spmm_tile<32, VT, XT, AT>(m, tile.s0, tile.s1, buf, lane); break;
        }
    }
    // Every wave has taken its last ticket before it counts itself out, so
    // the wave that counts last may reset the queue for the next launch.
    if (lane == 0) {
        const unsigned d =
            __hip_atomic_fetch_add(&queue[kQueueDone], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (d == static_cast<unsigned>(waves_total - 1)) {
            __hip_atomic_store(&queue[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&queue[kQueueDone], 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ------------------------------------------------------------------ host

namespace {

int ilog2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

template <typename VT, typename XT, typename AT>
hipError_t launch_spmm_typed(const SpmmMat& m, int strips, hipStream_t stream) {
    const int S = kWave >> (m.rl_log + m.g_log);
    const long long waves = (static_cast<long long>(strips) + S - 1) / S;
    const int grid = static_cast<int>((waves + kSpmmWaves - 1) / kSpmmWaves);
    switch (m.hb) {
        case 1: hipLaunchKernelGGL((spmm_kernel<1, VT, XT, AT>), dim3(grid), dim3(kSpmmThreads), 0, stream, m, strips); break;
        case 2: hipLaunchKernelGGL((spmm_kernel<2, VT, XT, AT>), dim3(grid), dim3(kSpmmThreads), 0, stream, m, strips); break;
        case 4: hipLaunchKernelGGL((spmm_kernel<4, VT, XT, AT>), dim3(grid), dim3(kSpmmThreads), 0, stream, m, strips); break;
        case 8: hipLaunchKernelGGL((spmm_kernel<8, VT, XT, AT>), dim3(grid), dim3(kSpmmThreads), 0, stream, m, strips); break;
        case 16: hipLaunchKernelGGL((spmm_kernel<16, VT, XT, AT>), dim3(grid), dim3(kSpmmThreads), 0, stream, m, strips); break;
        default: hipLaunchKernelGGL((spmm_kernel<32, VT, XT, AT>), dim3(grid), dim3(kSpmmThreads), 0, stream, m, strips); break;
    }
    return hipGetLastError();
}

}  // namespace

SpmmMat spmm_mat(const cmrs_mat_t* A, int nrhs, const void* X, int ldx, void* Y, int ldy, int group) {
    SpmmMat m{};
    m.strip_ptr = A->strip_ptr;
    m.word = A->col_word;
    m.val = A->val;
    m.x = X;
    m.y = Y;
    m.rows = A->rows;
    m.height = A->height;
    m.bits = A->bits;
    m.nrhs = nrhs;
    m.ldx = ldx;
    m.ldy = ldy;
    m.hb = next_pow2(A->height);
    m.rl_log = ilog2(nrhs);
    const int gmax = kWave >> m.rl_log;
    int g = group;
    if (g <= 0) {
        // Enough entry slots that one unrolled step covers the mean strip.
        const int strips = (A->rows + A->height - 1) / A->height;
        const double mean = strips > 0 ? static_cast<double>(A->nnz) / strips : 0.0;
        g = next_pow2(static_cast<int>(std::min(64.0, std::max(1.0, mean / kSpmmUnroll))));
    }
    if (g > gmax) g = gmax;
    m.g_log = ilog2(g);
    return m;
}

hipError_t launch_spmm(const cmrs_mat_t* A, int nrhs, const void* X, int ldx, void* Y, int ldy, int group,
                       hipStream_t stream) {
    const SpmmMat m = spmm_mat(A, nrhs, X, ldx, Y, ldy, group);
    const int strips = (A->rows + A->height - 1) / A->height;
    if (strips == 0) return hipSuccess;
    switch (A->val_dtype) {
        case CMRS_R64F: return launch_spmm_typed<double, double, double>(m, strips, stream);
        case CMRS_R32F: return launch_spmm_typed<float, float, float>(m, strips, stream);
        default: return launch_spmm_typed<bf16_t, float, float>(m, strips, stream);
    }
}

SpmmPlanShape spmm_plan_shape(int count, const cmrs_mat_t* mats, const int* nrhs, int tile_nnz, int group,
                              std::vector<SpmmTile>* tiles_out) {
    SpmmPlanShape sh{};
    const int target = tile_nnz > 0 ? tile_nnz : 32768;
    for (int i = 0; i < count; ++i) {
        const cmrs_mat_t& A = mats[i];
        const SpmmMat m = spmm_mat(&A, nrhs[i], nullptr, nrhs[i], nullptr, nrhs[i], group);
        sh.max_hb = std::max(sh.max_hb, m.hb);
        const long long strips = (static_cast<long long>(A.rows) + A.height - 1) / A.height;
        if (strips == 0) continue;
        const int S = kWave >> (m.rl_log + m.g_log);
        const double per_strip = std::max(1.0, static_cast<double>(A.nnz) / static_cast<double>(strips));
        long long T = static_cast<long long>(target / per_strip) / S * S;
        if (T < S) T = S;
        for (long long s0 = 0; s0 < strips; s0 += T) {
            if (tiles_out) tiles_out->push_back(SpmmTile{i, static_cast<int>(s0), static_cast<int>(std::min(strips, s0 + T)), 0});
            ++sh.tiles;
        }
    }
    sh.bytes = kSpmmHeaderBytes + sizeof(SpmmMat) * static_cast<size_t>(count) + sizeof(SpmmTile) * sh.tiles;
    return sh;
}

hipError_t build_spmm_plan(int count, const cmrs_mat_t* mats, const int* nrhs, const void* const* X, const int* ldx,
                           void* const* Y, const int* ldy, cmrs_dtype_t xy_dtype, int tile_nnz, int group,
                           int blocks_per_cu, void* desc, cmrs_spmm_plan_t* plan, hipStream_t stream) {
    std::vector<SpmmTile> tiles;
    const SpmmPlanShape sh = spmm_plan_shape(count, mats, nrhs, tile_nnz, group, &tiles);
    std::vector<unsigned char> image(sh.bytes, 0);
    SpmmMat* md = reinterpret_cast<SpmmMat*>(image.data() + kSpmmHeaderBytes);
    for (int i = 0; i < count; ++i) md[i] = spmm_mat(&mats[i], nrhs[i], X[i], ldx[i], Y[i], ldy[i], group);
    if (!tiles.empty())
        memcpy(image.data() + kSpmmHeaderBytes + sizeof(SpmmMat) * count, tiles.data(), sizeof(SpmmTile) * tiles.size());
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const int bpc = blocks_per_cu > 0 ? blocks_per_cu : 4;
    const long long want_blocks = (static_cast<long long>(sh.tiles) + kSpmmWaves - 1) / kSpmmWaves;
    const int grid = static_cast<int>(std::max(1LL, std::min(static_cast<long long>(cus) * bpc, want_blocks)));
    const size_t at = count > 0 && mats[0].val_dtype == CMRS_R64F ? 8 : 4;
    const int wave_slots = std::max(1, sh.max_hb) * kWave;
    plan->count = count;
    plan->tiles = sh.tiles;
    plan->grid = sh.tiles > 0 ? grid : 0;
    plan->lds_bytes = static_cast<int>(at * wave_slots * kSpmmWaves);
    plan->val_dtype = count > 0 ? mats[0].val_dtype : CMRS_R64F;
    plan->xy_dtype = xy_dtype;
    plan->max_height = sh.max_hb;
    plan->waves = plan->grid * kSpmmWaves;
    plan->desc = desc;
    plan->desc_bytes = sh.bytes;
    e = hipMemcpyAsync(desc, image.data(), sh.bytes, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    return e;
}

hipError_t launch_spmm_batched(const cmrs_spmm_plan_t* plan, hipStream_t stream) {
    if (plan->tiles == 0) return hipSuccess;
    unsigned char* base = static_cast<unsigned char*>(plan->desc);
    unsigned* queue = reinterpret_cast<unsigned*>(base);
    const SpmmMat* mats = reinterpret_cast<const SpmmMat*>(base + kSpmmHeaderBytes);
    const SpmmTile* tiles = reinterpret_cast<const SpmmTile*>(base + kSpmmHeaderBytes + sizeof(SpmmMat) * plan->count);
    const int wave_slots = plan->max_height * kWave;
    const dim3 grid(plan->grid), block(kSpmmThreads);
    const size_t lds = static_cast<size_t>(plan->lds_bytes);
    switch (plan->val_dtype) {
        case CMRS_R64F:
            hipLaunchKernelGGL((spmm_persistent_kernel<double, double, double>), grid, block, lds, stream, mats, tiles,
                               plan->tiles, queue, plan->waves, wave_slots);
            break;
        case CMRS_R32F:
            hipLaunchKernelGGL((spmm_persistent_kernel<float, float, float>), grid, block, lds, stream, mats, tiles,
                               plan->tiles, queue, plan->waves, wave_slots);
            break;
        default:
            hipLaunchKernelGGL((spmm_persistent_kernel<bf16_t, float, float>), grid, block, lds, stream, mats, tiles,
                               plan->tiles, queue, plan->waves, wave_slots);
            break;
    }
    return hipGetLastError();
}

}  // namespace cmrs
