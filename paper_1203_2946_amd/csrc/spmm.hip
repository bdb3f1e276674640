// CMRS products with several right-hand sides, single and batched.
//
// The hot loop is Algorithm 1 of Sec. 4, every entry feeding all nrhs
// right-hand sides: the wave's 64 lanes are S = 64 / G strips times G entry
// slots; lane (s, e) walks entries e, e + G, ... of its strip, reads each
// packed word and value once, gathers the nrhs values x_k[col] (one
// contiguous piece of the row-major X) and adds the nrhs products to its own
// partials for (row, k) in LDS, laid out [row * RB + k][lane] (RB =
// next_pow2(nrhs)) so that the additions of one instruction hit 64 distinct
// banks.  A strip's results are the sums over its G entry slots; the lane
// that sums output (s, row, k) starts at slot (row * RB + k) mod G, which
// spreads the reads of one instruction over distinct banks too.
//
// The batched path runs that body from one persistent kernel: waves take
// work tiles (a matrix and a range of its strips) from per-XCD queue counters
// in the plan until every queue is empty; the last wave out resets the
// counters, so the same plan can be launched again and replayed from a HIP
// graph.  A grid
// stride over strip passes (the listing's loop over strips in the paper's
// appendix) is the special case of one tile per wave.
#include <string.h>

#include <algorithm>
#include <vector>

#include "cmrs_device.hpp"
#include "cmrs_ext.hpp"

namespace cmrs {

constexpr int kSpmmMaxWaves = 4;
constexpr size_t kSpmmWaveLdsMax = 65536;

template <typename T>
__device__ inline T nt_load(const T* p) {
    return __builtin_nontemporal_load(p);
}
__device__ inline bf16_t nt_load(const bf16_t* p) {
    bf16_t v;
    v.bits = __builtin_nontemporal_load(&p->bits);
    return v;
}

// Strips [sb, sb + S) (those below s_end) of matrix m; buf holds HB * RB * 64
// partials of this wave.
// 16 bytes of X: XV consecutive values of one row.
template <typename XT>
struct alignas(16) XVec {
    XT v[16 / sizeof(XT)];
};

template <int HB, int RB, typename VT, typename XT, typename AT>
__device__ inline void spmm_pass(const SpmmMat& m, int sb, int s_end, AT* __restrict__ buf, int lane) {
    constexpr int U = RB >= 4 ? 4 : 8;
    constexpr int XV = static_cast<int>(16 / sizeof(XT));
    constexpr int SLOTS = HB * RB;
    const int g_log = m.g_log;
    const int G = 1 << g_log;
    const int s_log = 6 - g_log;
    const int e = lane & (G - 1);
    const int s = sb + (lane >> g_log);
    const int bits = m.bits;
    const int nrhs = m.nrhs;
    const uint32_t mask = (1u << bits) - 1u;
#pragma unroll
    for (int i = 0; i < SLOTS; ++i) buf[i * kWave + lane] = AT(0);
    if (s < s_end) {
        const int lo = m.strip_ptr[s], hi = m.strip_ptr[s + 1];
        const VT* __restrict__ val = static_cast<const VT*>(m.val);
        const XT* __restrict__ x = static_cast<const XT*>(m.x);
        const size_t ldx = static_cast<size_t>(m.ldx);
        for (int base = lo + e; base < hi; base += U * G) {
            // Out-of-range entries are clamped to the last one of the strip
            // (a valid address), so the stream loads of the step issue
            // without a branch; their gathers are masked off.
            uint32_t w[U];
            VT v[U];
            XT xv[U][RB];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = min(base + u * G, hi - 1);
                w[u] = nt_load(m.word + j);
                v[u] = nt_load(val + j);
            }
            // The row piece x[col][0 .. nrhs) of every entry: 16-byte loads
            // where X keeps its rows aligned, single loads otherwise, the slots
            // past nrhs not loaded (nrhs is the same in every lane).  fp64 X
            // with fewer than 4 right-hand-side slots: one load per slot, the
            // slots past nrhs reading x_0 (measured faster there; from 4 slots
            // on the 16-byte loads are faster, e.g. 481 -> 363 us for 8
            // right-hand sides on a 27-point stencil of 2*10^6 rows).
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (base + u * G < hi) {
                    const XT* xr = x + static_cast<size_t>(w[u] >> bits) * ldx;
                    if constexpr (sizeof(XT) == 8 && RB < 4) {
#pragma unroll
                        for (int k = 0; k < RB; ++k) xv[u][k] = xr[k < nrhs ? k : 0];
                    } else if (RB >= XV && m.xvec) {
#pragma unroll
                        for (int k = 0; k < RB; k += XV) {
                            if (k + XV <= nrhs) {
                                const XVec<XT> t = *reinterpret_cast<const XVec<XT>*>(xr + k);
#pragma unroll
                                for (int q = 0; q < XV; ++q) xv[u][k + q] = t.v[q];
                            } else {
#pragma unroll
                                for (int q = 0; q < XV; ++q)
                                    if (k + q < nrhs) xv[u][k + q] = xr[k + q];
                            }
                        }
                    } else {
#pragma unroll
                        for (int k = 0; k < RB; ++k)
                            if (k < nrhs) xv[u][k] = xr[k];
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (base + u * G < hi) {
                    const AT a = static_cast<AT>(ValTraits<VT>::widen(v[u]));
                    AT* slot = buf + static_cast<int>(w[u] & mask & (HB - 1)) * RB * kWave + lane;
#pragma unroll
                    for (int k = 0; k < RB; ++k)
                        if (k < nrhs) lds_add(slot + k * kWave, a * static_cast<AT>(xv[u][k]));
                }
            }
        }
    }
    wave_lds_sync();
    // Output o: strip slot so = o mod S (fastest), partial i = o / S with
    // i = row * RB + k; it sums the G entry slots starting at slot i mod G.
    constexpr int NOUT_PER_S = SLOTS;
    const int nout = NOUT_PER_S << s_log;
    XT* __restrict__ y = static_cast<XT*>(m.y);
    const size_t ldy = static_cast<size_t>(m.ldy);
    for (int o = lane; o < nout; o += kWave) {
        const int so = o & ((1 << s_log) - 1);
        const int i = o >> s_log;
        const int k = i & (RB - 1);
        const int rr = i / RB;
        const AT* p = buf + i * kWave + (so << g_log);
        AT sum = AT(0);
        for (int q = 0; q < G; ++q) sum += p[(q + i) & (G - 1)];
        const int strip = sb + so;
        const long long row = static_cast<long long>(strip) * m.height + rr;
        if (strip < s_end && rr < m.height && row < m.rows && k < nrhs)
            y[static_cast<size_t>(row) * ldy + k] = static_cast<XT>(sum);
    }
    wave_lds_sync();
}

template <int HB, int RB, typename VT, typename XT, typename AT>
__global__ __launch_bounds__(kSpmmMaxWaves * kWave) void spmm_kernel(SpmmMat m, int strips) {
    extern __shared__ __align__(16) unsigned char spmm_lds[];
    AT* buf = reinterpret_cast<AT*>(spmm_lds);
    const int lane = lane_id();
    const int wpb = static_cast<int>(blockDim.x) / kWave;
    const int wave = uniform(static_cast<int>(threadIdx.x) / kWave);
    const int s_log = 6 - m.g_log;
    const long long sb =
        (static_cast<long long>(xcd_logical_block(blockIdx.x, gridDim.x)) * wpb + wave) << s_log;
    if (sb >= strips) return;
    spmm_pass<HB, RB, VT, XT, AT>(m, static_cast<int>(sb), strips, buf + wave * (HB * RB * kWave), lane);
}

template <int HB, int RB, typename VT, typename XT, typename AT>
__device__ inline void spmm_tile(const SpmmMat& m, int s0, int s1, AT* buf, int lane) {
    const int S = kWave >> m.g_log;
    for (int sb = s0; sb < s1; sb += S) spmm_pass<HB, RB, VT, XT, AT>(m, sb, s1, buf, lane);
}

template <int HB, typename VT, typename XT, typename AT>
__device__ inline void spmm_tile_rb(const SpmmMat& m, int s0, int s1, AT* buf, int lane) {
    switch (m.rb_log) {
        case 0: spmm_tile<HB, 1, VT, XT, AT>(m, s0, s1, buf, lane); break;
        case 1: spmm_tile<HB, 2, VT, XT, AT>(m, s0, s1, buf, lane); break;
        case 2: spmm_tile<HB, 4, VT, XT, AT>(m, s0, s1, buf, lane); break;
        default: spmm_tile<HB, 8, VT, XT, AT>(m, s0, s1, buf, lane); break;
    }
}

// Work queues, one per XCD: queue x hands out the tiles [x*n/8, (x+1)*n/8)
// through the counter queue[x * 16] (one 64-byte line each).  Workgroup b
// runs on XCD b mod 8 and drains that XCD's queue first, so neighbouring
// tiles (and the parts of X they gather) stay in one L2; then it takes tiles
// left in the other queues.  queue[kQueueDone] counts finished waves.  All
// counters are zero at launch and again when the last wave leaves.
constexpr int kQueueStride = 16;
constexpr int kQueueDone = kNumXcd * kQueueStride;

template <typename VT, typename XT, typename AT>
__global__ __launch_bounds__(kSpmmMaxWaves * kWave) __attribute__((amdgpu_waves_per_eu(4))) void spmm_persistent_kernel(
    const SpmmMat* __restrict__ mats, const SpmmTile* __restrict__ tiles, int ntiles, unsigned* __restrict__ queue,
    int waves_total, int wave_slots) {
    extern __shared__ __align__(16) unsigned char spmm_lds[];
    const int lane = lane_id();
    const int wave = uniform(static_cast<int>(threadIdx.x) / kWave);
    AT* buf = reinterpret_cast<AT*>(spmm_lds) + static_cast<size_t>(wave) * wave_slots;
    const int home = static_cast<int>(blockIdx.x) % kNumXcd;
    for (int a = 0; a < kNumXcd; ++a) {
        const int qx = (home + a) % kNumXcd;
        const long long lo = static_cast<long long>(qx) * ntiles / kNumXcd;
        const long long hi = static_cast<long long>(qx + 1) * ntiles / kNumXcd;
        for (;;) {
            unsigned c = 0;
            if (lane == 0)
                c = __hip_atomic_fetch_add(&queue[qx * kQueueStride], 1u, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
            c = static_cast<unsigned>(uniform(static_cast<int>(__shfl(c, 0))));
            const long long t = lo + c;
            if (t >= hi) break;
            const SpmmTile tile = tiles[t];
            const SpmmMat m = mats[tile.mat];
            switch (m.hb) {
                case 1: spmm_tile_rb<1, VT, XT, AT>(m, tile.s0, tile.s1, buf, lane); break;
                case 2: spmm_tile_rb<2, VT, XT, AT>(m, tile.s0, tile.s1, buf, lane); break;
                case 4: spmm_tile_rb<4, VT, XT, AT>(m, tile.s0, tile.s1, buf, lane); break;
                case 8: spmm_tile_rb<8, VT, XT, AT>(m, tile.s0, tile.s1, buf, lane); break;
                case 16: spmm_tile_rb<16, VT, XT, AT>(m, tile.s0, tile.s1, buf, lane); break;
                default: spmm_tile_rb<32, VT, XT, AT>(m, tile.s0, tile.s1, buf, lane); break;
            }
        }
    }
    // Every wave has taken its last ticket from every queue before it counts
    // itself out, so the wave that counts last may reset them for the next
    // launch.
    if (lane == 0) {
        const unsigned d =
            __hip_atomic_fetch_add(&queue[kQueueDone], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (d == static_cast<unsigned>(waves_total - 1)) {
            for (int x = 0; x < kNumXcd; ++x)
                __hip_atomic_store(&queue[x * kQueueStride], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

template <int HB, int RB, typename VT, typename XT, typename AT>
void launch_spmm_hb_rb(const SpmmMat& m, int strips, int wpb, size_t lds, hipStream_t stream) {
    const int S = kWave >> m.g_log;
    const long long waves = (static_cast<long long>(strips) + S - 1) / S;
    const int grid = static_cast<int>((waves + wpb - 1) / wpb);
    hipLaunchKernelGGL((spmm_kernel<HB, RB, VT, XT, AT>), dim3(grid), dim3(wpb * kWave), lds, stream, m, strips);
}

template <int HB, typename VT, typename XT, typename AT>
void launch_spmm_hb(const SpmmMat& m, int strips, int wpb, size_t lds, hipStream_t stream) {
    switch (m.rb_log) {
        case 0: launch_spmm_hb_rb<HB, 1, VT, XT, AT>(m, strips, wpb, lds, stream); break;
        case 1: launch_spmm_hb_rb<HB, 2, VT, XT, AT>(m, strips, wpb, lds, stream); break;
        case 2: launch_spmm_hb_rb<HB, 4, VT, XT, AT>(m, strips, wpb, lds, stream); break;
        default: launch_spmm_hb_rb<HB, 8, VT, XT, AT>(m, strips, wpb, lds, stream); break;
    }
}

template <typename VT, typename XT, typename AT>
hipError_t launch_spmm_typed(const SpmmMat& m, int strips, hipStream_t stream) {
    const size_t wave_bytes = spmm_wave_lds_bytes(m.hb << m.rb_log, sizeof(AT));
    const int wpb = spmm_waves_per_block(wave_bytes);
    const size_t lds = wave_bytes * wpb;
    switch (m.hb) {
        case 1: launch_spmm_hb<1, VT, XT, AT>(m, strips, wpb, lds, stream); break;
        case 2: launch_spmm_hb<2, VT, XT, AT>(m, strips, wpb, lds, stream); break;
        case 4: launch_spmm_hb<4, VT, XT, AT>(m, strips, wpb, lds, stream); break;
        case 8: launch_spmm_hb<8, VT, XT, AT>(m, strips, wpb, lds, stream); break;
        case 16: launch_spmm_hb<16, VT, XT, AT>(m, strips, wpb, lds, stream); break;
        default: launch_spmm_hb<32, VT, XT, AT>(m, strips, wpb, lds, stream); break;
    }
    return hipGetLastError();
}

}  // namespace

size_t spmm_wave_lds_bytes(int slots, size_t acc_bytes) {
    return static_cast<size_t>(slots) * kWave * acc_bytes;
}

int spmm_waves_per_block(size_t wave_bytes) {
    if (wave_bytes == 0) return kSpmmMaxWaves;
    const size_t w = kSpmmWaveLdsMax / wave_bytes;
    return static_cast<int>(std::max<size_t>(1, std::min<size_t>(kSpmmMaxWaves, w)));
}

bool spmm_fits(int height, int nrhs, cmrs_dtype_t val_dtype) {
    const size_t at = val_dtype == CMRS_R64F ? 8 : 4;
    return spmm_wave_lds_bytes(next_pow2(height) * next_pow2(nrhs), at) <= kSpmmWaveLdsMax;
}

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
    m.rb_log = ilog2(nrhs);
    int g = group;
    if (g <= 0) {
        // Enough entry slots that one unrolled step covers the mean strip.
        const int unroll = (1 << m.rb_log) >= 4 ? 4 : 8;
        const int strips = (A->rows + A->height - 1) / A->height;
        const double mean = strips > 0 ? static_cast<double>(A->nnz) / strips : 0.0;
        g = next_pow2(static_cast<int>(std::min(64.0, std::max(1.0, mean / unroll))));
    }
    if (g > kWave) g = kWave;
    m.g_log = ilog2(g);
    const size_t xs = A->val_dtype == CMRS_R64F ? 8 : 4;  // X holds doubles with fp64 values, else floats
    m.xvec = (reinterpret_cast<uintptr_t>(X) % 16 == 0 && (static_cast<size_t>(ldx) * xs) % 16 == 0) ? 1 : 0;
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
    // Tiles grouped by (height bucket, right-hand-side bucket), so that waves
    // running at the same time mostly execute the same code.
    std::vector<std::pair<int, int>> order;
    for (int i = 0; i < count; ++i) {
        const SpmmMat m = spmm_mat(&mats[i], nrhs[i], nullptr, nrhs[i], nullptr, nrhs[i], group);
        order.push_back({m.hb * 16 + m.rb_log, i});
        sh.max_slots = std::max(sh.max_slots, m.hb << m.rb_log);
    }
    std::stable_sort(order.begin(), order.end(),
                     [](const std::pair<int, int>& a, const std::pair<int, int>& b) { return a.first < b.first; });
    for (const auto& oi : order) {
        const int i = oi.second;
        const cmrs_mat_t& A = mats[i];
        const SpmmMat m = spmm_mat(&A, nrhs[i], nullptr, nrhs[i], nullptr, nrhs[i], group);
        const long long strips = (static_cast<long long>(A.rows) + A.height - 1) / A.height;
        if (strips == 0) continue;
        const int S = kWave >> m.g_log;
        const double per_strip = std::max(1.0, static_cast<double>(A.nnz) / static_cast<double>(strips));
        long long T = static_cast<long long>(target / per_strip) / S * S;
        if (T < S) T = S;
        for (long long s0 = 0; s0 < strips; s0 += T) {
            if (tiles_out)
                tiles_out->push_back(SpmmTile{i, static_cast<int>(s0), static_cast<int>(std::min(strips, s0 + T)), 0});
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
        memcpy(image.data() + kSpmmHeaderBytes + sizeof(SpmmMat) * count, tiles.data(),
               sizeof(SpmmTile) * tiles.size());
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const size_t at = count > 0 && mats[0].val_dtype == CMRS_R64F ? 8 : 4;
    const size_t wave_bytes = spmm_wave_lds_bytes(std::max(1, sh.max_slots), at);
    const int wpb = spmm_waves_per_block(wave_bytes);
    const int bpc = blocks_per_cu > 0 ? blocks_per_cu : 4;
    const long long want_blocks = (static_cast<long long>(sh.tiles) + wpb - 1) / wpb;
    const int grid = static_cast<int>(std::max(1LL, std::min(static_cast<long long>(cus) * bpc, want_blocks)));
    cmrs_spmm_plan_t P{};
    P.count = count;
    P.tiles = sh.tiles;
    P.grid = sh.tiles > 0 ? grid : 0;
    P.lds_bytes = static_cast<int>(wave_bytes * wpb);
    P.val_dtype = count > 0 ? mats[0].val_dtype : CMRS_R64F;
    P.xy_dtype = xy_dtype;
    P.max_slots = std::max(1, sh.max_slots);
    P.waves = P.grid * wpb;
    P.desc = desc;
    P.desc_bytes = sh.bytes;
    e = hipMemcpyAsync(desc, image.data(), sh.bytes, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e == hipSuccess) *plan = P;
    return e;
}

hipError_t launch_spmm_batched(const cmrs_spmm_plan_t* plan, hipStream_t stream) {
    if (plan->tiles == 0) return hipSuccess;
    unsigned char* base = static_cast<unsigned char*>(plan->desc);
    unsigned* queue = reinterpret_cast<unsigned*>(base);
    const SpmmMat* mats = reinterpret_cast<const SpmmMat*>(base + kSpmmHeaderBytes);
    const SpmmTile* tiles =
        reinterpret_cast<const SpmmTile*>(base + kSpmmHeaderBytes + sizeof(SpmmMat) * plan->count);
    const int wave_slots = plan->max_slots * kWave;
    const int wpb = plan->waves / plan->grid;
    const dim3 grid(plan->grid), block(wpb * kWave);
    const size_t lds = static_cast<size_t>(plan->lds_bytes);
    switch (plan->val_dtype) {
        case CMRS_R64F:
            hipLaunchKernelGGL((spmm_persistent_kernel<double, double, double>), grid, block, lds, stream, mats,
                               tiles, plan->tiles, queue, plan->waves, wave_slots);
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
