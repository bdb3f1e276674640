// CSR <-> CMRS conversion kernels and the CSR validity check (gfx950).
//
// CSR -> CMRS follows Sec. 3 and 4 of Koza et al. (arXiv:1203.2946):
//   StripPtr[j] = RowPtr[j*height], StripPtr[strips] = nnz;
//   word[k] = (ColInd[k] << bits) | (row(k) mod height);
//   optionally every strip reordered by (column, RowInStrip), ties in CSR
//   order (Sec. 4, fourth optimisation).
// CMRS -> CSR is the inverse: per-row counts inside a strip give RowPtr (no
// global scan is needed, a strip's entries are exactly its rows' entries), and
// a stable scatter by RowInStrip restores row order.  One wave takes the
// whole strips of 32 consecutive rows and streams their entries (contiguous)
// with coalesced loads, counting, then scattering; at height 1 the
// conversion is a plain copy.
//
// Work split of CSR -> CMRS.  Without the reorder, entries keep their
// places: one wave takes the whole strips of 32 consecutive rows and streams
// their entries with coalesced loads, stepping through the row pointers to
// find each entry's row.  With the reorder, the main kernel gives each strip a
// group of G lanes (64/G strips per wave) and each lane up to E = 8 entries,
// all loaded before any is used, so a wave keeps 64*E entries of traffic in
// flight.  The row of an entry comes from a binary search over the strip's row
// pointers, which sit one per lane of the group (cross-lane reads, no memory
// traffic).
//
// Reorder: a strip of canonical CSR is `height` runs (its rows) that are
// already sorted by column, and within a strip (column, RowInStrip) order is
// the order of the packed words.  The runs are merged pairwise, log2(height)
// levels, in LDS: each entry counts the keys of the partner run below its own
// (binary search) and moves to its place in the merged run.  Keys are
// (word << 32 | position in strip), unique, so the result is the stable order.
// Strips that are longer than a group holds, or whose rows are not sorted,
// go to a list in the workspace: strips of up to 1024 entries are sorted by
// one wave (run merge, or a bitonic network for unsorted rows); longer ones
// by a 1024-thread workgroup, in LDS up to 16384 entries (each entry ranked
// against the strip's short rows gathered and sorted once, and by a binary
// search over each long row; a bitonic network for unsorted rows), in the
// workspace beyond that.
#include <limits.h>

#include "cmrs_device.hpp"
#include "cmrs_internal.hpp"

namespace cmrs {

constexpr int kConvWaves = 4;
constexpr int kConvThreads = kConvWaves * kWave;
constexpr int kBlockSortThreads = 1024;
// Workgroups of the long-strip sort: its LDS allows one per CU, 256 CUs.
constexpr int kBlockSortGrid = 256;

__global__ void set_ints_kernel(int32_t* p, int32_t n, int32_t v) {
    if (blockIdx.x == 0 && static_cast<int>(threadIdx.x) < n) p[threadIdx.x] = v;
}

// Largest t with rp_t <= e, where lane base+t holds rp_t = RowPtr[first row of
// the strip + t] (INT_MAX for rows the strip does not have): the RowInStrip of
// entry e (empty rows are skipped because their rp_t repeats).  All lanes of
// the wave must be active.
template <int HB>
__device__ inline int row_in_strip(int myrp, int e, int base) {
    int lo = 0;
#pragma unroll
    for (int step = HB / 2; step >= 1; step >>= 1) {
        const int v = __shfl(myrp, base + lo + step);
        if (v <= e) lo += step;
    }
    return lo;
}

struct StripRows {
    int r0, nr, myrp, s0, s1;
};

// Row pointers of strip `strip` spread over the lanes of the whole wave.
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

// ------------------------------------------------------------------ whole-wave paths

// Merge of the row runs of strips held in registers, G lanes per strip, slot u
// of lane q holding entry q + G*u: words (col << bits | RowInStrip) in wd and
// their current place in the strip in pos.  LDS
// buffers A and B (the group's words by place, A filled on entry) alternate
// per level, level k merging the runs of 2^k rows pairwise; the words of
// different runs never tie (their RowInStrip fields differ), so
// an entry's place after a level is its rank in its own run plus the number
// of partner-run words below it.  On return pos holds each entry's place in
// the sorted strip.  The caller has made A and rt visible to the wave.
template <int HB, int G, int E>
__device__ inline void merge_runs_regs(uint32_t* A, uint32_t* B, const int* rt, const uint32_t (&wd)[E],
                                       int (&pos)[E], int umax, bool go, int n, int q) {
#pragma unroll 1
    for (int k = 0; (1 << k) < HB; ++k) {
        if (k > 0) wave_lds_sync();
#pragma unroll
        for (int u = 0; u < E; ++u) {
            if (u >= umax) break;
            const int run = static_cast<int>(wd[u] & static_cast<uint32_t>(HB - 1)) >> k;
            const int partner = run ^ 1;
            const int run_lo = rt[run << k];
            const int merged_lo = rt[(run & ~1) << k];
            const int p_lo = rt[partner << k];
            const int p_hi = rt[(partner + 1) << k];
            if (go && q + G * u < n) {
                int a = p_lo, len = p_hi - p_lo;
                while (len > 0) {
                    const int half = len >> 1;
                    if (A[a + half] < wd[u]) {
                        a += half + 1;
                        len -= half + 1;
                    } else {
                        len = half;
                    }
                }
                pos[u] = merged_lo + (pos[u] - run_lo) + (a - p_lo);
                B[pos[u]] = wd[u];
            }
        }
        uint32_t* tmp = A;
        A = B;
        B = tmp;
    }
}

// Sorted conversion of one strip of at most kWave*E entries by the whole wave,
// words in registers (slot u of lane l: entry l + kWave*u), in its LDS slice
// of kWave*E 64-bit words: rows sorted by column, a merge of the row runs
// (merge_runs_regs), then each entry and its value (read again) to its place;
// otherwise a bitonic network over (word, position) keys.
template <int HB, int E, typename ET>
__device__ inline void sort_strip_mid(int strip, int rows, int height, int bits, const int* __restrict__ row_ptr,
                                      const int* __restrict__ col_ind, const ET* __restrict__ val_in,
                                      uint32_t* __restrict__ col_word, ET* __restrict__ val_out, uint64_t* slice,
                                      int* rt, int lane) {
    const StripRows sr = load_strip_rows(strip, rows, height, row_ptr, lane);
    const int n = sr.s1 - sr.s0;
    const int umax = uniform((n + kWave - 1) / kWave);
    const uint32_t mask = (1u << bits) - 1u;
    uint32_t* A = reinterpret_cast<uint32_t*>(slice);
    uint32_t* B = A + kWave * E;
    uint32_t wd[E];
    int pos[E];
#pragma unroll
    for (int u = 0; u < E; ++u) {
        wd[u] = 0u;
        pos[u] = lane + kWave * u;
        if (u < umax) {
            const int i = lane + kWave * u;
            const int r = row_in_strip<HB>(sr.myrp, sr.s0 + i, 0);
            if (i < n) {
                wd[u] = (static_cast<uint32_t>(col_ind[sr.s0 + i]) << bits) | static_cast<uint32_t>(r);
                A[i] = wd[u];
            }
        }
    }
    if (lane <= HB) rt[lane] = lane < sr.nr ? sr.myrp - sr.s0 : n;
    wave_lds_sync();
    bool bad = false;
#pragma unroll
    for (int u = 0; u < E; ++u) {
        if (u >= umax) break;
        const int i = lane + kWave * u;
        if (i + 1 < n) {
            const uint32_t nw = A[i + 1];
            if ((nw & mask) == (wd[u] & mask) && (nw >> bits) < (wd[u] >> bits)) bad = true;
        }
    }
    if (ballot(bad) == 0ull) {
        merge_runs_regs<HB, kWave, E>(A, B, rt, wd, pos, umax, true, n, lane);
#pragma unroll
        for (int u = 0; u < E; ++u) {
            if (u >= umax) break;
            const int i = lane + kWave * u;
            if (i < n && static_cast<unsigned>(pos[u]) < static_cast<unsigned>(n)) {
                col_word[sr.s0 + pos[u]] = wd[u];
                val_out[sr.s0 + pos[u]] = val_in[sr.s0 + i];
            }
        }
    } else {
        const int P = pow2_at_least(n);
        wave_lds_sync();  // A is read above; the keys overwrite it
#pragma unroll
        for (int u = 0; u < E; ++u) {
            const int i = lane + kWave * u;
            if (i < n)
                slice[i] = (static_cast<uint64_t>(wd[u]) << 32) | static_cast<uint32_t>(i);
            else if (i < P)
                slice[i] = ~0ull;
        }
        wave_lds_sync();
        bitonic_sort(slice, P, lane, kWave, [] { wave_lds_sync(); });
        for (int i = lane; i < n; i += kWave) {
            const uint64_t kk = slice[i];
            col_word[sr.s0 + i] = static_cast<uint32_t>(kk >> 32);
            val_out[sr.s0 + i] = val_in[sr.s0 + static_cast<int>(static_cast<uint32_t>(kk))];
        }
    }
    wave_lds_sync();
}

// ------------------------------------------------------------------ group kernels

__device__ inline uint64_t group_mask(int gbase, int G) {
    return G == kWave ? ~0ull : (((1ull << G) - 1ull) << gbase);
}

// Number of per-lane slots any group of the wave uses: ceil(max n / G)
// (wave-uniform), so the slot loops stop at the longest strip of the wave.
template <int G>
__device__ inline int used_slots(int n) {
    int m = n;
#pragma unroll
    for (int off = kWave / 2; off >= G; off >>= 1) m = max(m, __shfl_xor(m, off));
    return uniform((m + G - 1) / G);
}

// Strips past a group's capacity of at most this many entries are sorted by
// the group kernel's wave itself, longer ones listed for the list kernels.
// (Listing every such strip spreads the work but costs a wave per strip;
// measured on the skewed 2*10^6-row workload, sorted conversion at height
// 2/4/8: 256/275/298 us inline up to 512 entries, 243/257/273 us up to 256,
// 383/289/272 us listing all; the benchmark matrix is unchanged.)
constexpr int kInlineSortMax = 256;

// CSR -> CMRS with the reorder, for strips of at most G*E entries, G lanes
// per strip.  Writes strip_ptr too.  Longer strips of at most kInlineSortMax
// entries (and no more than kWave*E), and strips with unsorted rows as short,
// are sorted by the whole wave afterwards in the wave's LDS slice; longer ones
// go to the workspace lists (ws_count[0] / ws_small: at most kWaveSortCap
// entries; ws_count[1] / ws_big: longer).  No output may alias an input.
template <int HB, int G, int E, typename ET>
__global__ __launch_bounds__(kConvThreads) __attribute__((amdgpu_waves_per_eu(8))) void from_csr_group_kernel(
    int rows, int strips, int height, int bits, int nnz, const int* __restrict__ row_ptr,
    const int* __restrict__ col_ind, const ET* __restrict__ val_in, int* __restrict__ strip_ptr,
    uint32_t* __restrict__ col_word, ET* __restrict__ val_out, int* __restrict__ ws_count,
    int* __restrict__ ws_small, int* __restrict__ ws_big) {
    static_assert(G >= HB && G <= kWave && G >= 2, "group width");
    constexpr int NG = kWave / G;
    constexpr int CAP = G * E;
    __shared__ uint64_t lds[kConvWaves][kWave * E];
    __shared__ int rowtab[kConvWaves][NG * (HB + 1)];
    const int lane = lane_id();
    const int wave = uniform(static_cast<int>(threadIdx.x) / kWave);
    const int strip0 = (xcd_logical_block(blockIdx.x, gridDim.x) * kConvWaves + wave) * NG;
    if (strip0 >= strips) return;
    const int g = lane / G, q = lane % G, gbase = g * G;
    const int strip = strip0 + g;
    const bool valid = strip < strips;
    const int r0 = strip * height;
    const int nr = valid ? min(height, rows - r0) : 0;
    const int myrp = (valid && q < nr) ? row_ptr[r0 + q] : INT_MAX;
    const int s1 = valid ? row_ptr[r0 + nr] : 0;
    const int s0_lane = __shfl(myrp, gbase);
    const int s0 = valid ? s0_lane : 0;
    const int n = s1 - s0;
    if (valid && q == 0) {
        strip_ptr[strip] = s0;
        if (strip == strips - 1) strip_ptr[strips] = nnz;
    }
    bool special = valid && n > CAP;
    const int umax = used_slots<G>(valid && !special ? n : 0);

    int c[E], t[E];
    ET v[E];
#pragma unroll
    for (int u = 0; u < E; ++u) {
        c[u] = 0;
        t[u] = 0;
        v[u] = ET(0);
        if (u < umax) {
            const int j = s0 + q + G * u;
            const bool act = valid && !special && j < s1;
            if (act) {
                c[u] = col_ind[j];
                v[u] = val_in[j];
            }
            t[u] = row_in_strip<HB>(myrp, j, gbase);
        }
    }

    {
        // Words of every strip the group holds in LDS by place, and the
        // strip-relative row pointers of rows 0..HB (rows past the strip: n).
        const bool fits = valid && !special;
        uint32_t* A = reinterpret_cast<uint32_t*>(&lds[wave][0]) + gbase * E;
        uint32_t* B = reinterpret_cast<uint32_t*>(&lds[wave][0]) + kWave * E + gbase * E;
        int* rtab = &rowtab[wave][g * (HB + 1)];
        uint32_t wd[E];
        int pos[E];
#pragma unroll
        for (int u = 0; u < E; ++u) {
            const int p = q + G * u;
            wd[u] = (static_cast<uint32_t>(c[u]) << bits) | static_cast<uint32_t>(t[u]);
            pos[u] = p;
            if (u < umax && fits && p < n) A[p] = wd[u];
        }
        if (q < HB) rtab[q] = q < nr ? myrp - s0 : n;
        if (q == 0) rtab[HB] = n;
        wave_lds_sync();
        // Rows must ascend (non-strictly) by column for the merge: an entry
        // and the next one of the strip, when they share the RowInStrip field
        // (the same row), must not descend.
        const uint32_t mask = (1u << bits) - 1u;
        bool bad = false;
#pragma unroll
        for (int u = 0; u < E; ++u) {
            if (u >= umax) break;
            const int p = q + G * u;
            if (fits && p + 1 < n) {
                const uint32_t nw = A[p + 1];
                if ((nw & mask) == (wd[u] & mask) && (nw >> bits) < (wd[u] >> bits)) bad = true;
            }
        }
        const bool gbad = (ballot(bad) & group_mask(gbase, G)) != 0;
        special = special || (valid && gbad);
        constexpr int WCAP = kWave * E;  // what sort_strip_mid<HB, E> holds
        constexpr int INLINE = kInlineSortMax < WCAP ? kInlineSortMax : WCAP;
        if (valid && special && q == 0 && n > INLINE) {
            if (n <= kWaveSortCap)
                ws_small[atomicAdd(&ws_count[0], 1)] = strip;
            else
                ws_big[atomicAdd(&ws_count[1], 1)] = strip;
        }
        const bool go = valid && !special;
        merge_runs_regs<HB, G, E>(A, B, rtab, wd, pos, umax, go, n, q);
        // Out from registers: each entry to its place in the sorted strip.
        // (Staging through LDS as the tall-strip kernel does was measured
        // slower here: 133 -> 137 us at height 2, 156 -> 164 us at height 4.)
#pragma unroll
        for (int u = 0; u < E; ++u) {
            if (u >= umax) break;
            if (go && q + G * u < n && static_cast<unsigned>(pos[u]) < static_cast<unsigned>(n)) {
                col_word[s0 + pos[u]] = wd[u];
                val_out[s0 + pos[u]] = v[u];
            }
        }
        wave_lds_sync();  // the wave's slice is reused below
        uint64_t mids = ballot(valid && special && q == 0 && n <= INLINE);
        while (mids) {
            const int leader = __ffsll(static_cast<unsigned long long>(mids)) - 1;
            mids &= mids - 1;
            sort_strip_mid<HB, E, ET>(strip0 + leader / G, rows, height, bits, row_ptr, col_ind, val_in, col_word,
                                      val_out, lds[wave], rowtab[wave], lane);
        }
    }
}

// ------------------------------------------------------------------ tall strips

// Sorted CSR -> CMRS for tall strips, one wave per strip of at most
// kWave*E entries (longer strips go to the workspace lists).  The merge of
// the group kernel costs log2(height) levels of binary searches; here an
// entry's place comes from one bucketing pass instead, whatever the height:
// entries fall into NB buckets of about equal width over the strip's column
// range [cmin, cmax] (NB about n/4; the bucket is a multiply and a shift of
// c - cmin, non-decreasing in c), a count per bucket (LDS atomics) and a
// scan give each bucket's start, the
// keys (word << 32 | position in strip) are scattered by bucket, and an
// entry's place is its bucket's start plus the number of keys of its bucket
// below its own.  Keys are unique and ordered as the reorder of Sec. 4
// requires (column, then RowInStrip, then CSR order), so unsorted rows and
// duplicates need no special path.  A strip whose largest bucket holds more
// than kBucketMax keys (columns bunched at a few values far apart) is sorted
// by a bitonic network over the same keys instead.
constexpr int kBucketMax = 64;
// The sorted conversion uses it from this height (next power of two) on, for
// strips of at least kBucketMinMean entries on average: one wave per strip
// costs more than the merge for short strips (measured).
constexpr int kBucketMinHeight = 16;
constexpr double kBucketMinMean = 320.0;

template <int HB, int E, typename ET>
__global__ __launch_bounds__(kConvThreads) void from_csr_bucket_kernel(
    int rows, int strips, int height, int bits, int nnz, const int* __restrict__ row_ptr,
    const int* __restrict__ col_ind, const ET* __restrict__ val_in, int* __restrict__ strip_ptr,
    uint32_t* __restrict__ col_word, ET* __restrict__ val_out, int* __restrict__ ws_count,
    int* __restrict__ ws_small, int* __restrict__ ws_big) {
    constexpr int CAP = kWave * E;
    constexpr int NBMAX = CAP / 4;
    // The bucket count doubles up to NBMAX, so NBMAX must be a power of two
    // (otherwise it would pass NBMAX and overrun bcnt/bstart).
    static_assert((NBMAX & (NBMAX - 1)) == 0, "bucket capacity must be a power of two");
    __shared__ uint64_t keys[kConvWaves][CAP];
    __shared__ int bcnt[kConvWaves][NBMAX];
    __shared__ int bstart[kConvWaves][NBMAX];
    const int lane = lane_id();
    const int wave = uniform(static_cast<int>(threadIdx.x) / kWave);
    const int strip = xcd_logical_block(blockIdx.x, gridDim.x) * kConvWaves + wave;
    if (strip >= strips) return;
    const StripRows sr = load_strip_rows(strip, rows, height, row_ptr, lane);
    const int n = sr.s1 - sr.s0;
    if (lane == 0) {
        strip_ptr[strip] = sr.s0;
        if (strip == strips - 1) strip_ptr[strips] = nnz;
    }
    if (n > CAP) {
        if (lane == 0) {
            if (n <= kWaveSortCap)
                ws_small[atomicAdd(&ws_count[0], 1)] = strip;
            else
                ws_big[atomicAdd(&ws_count[1], 1)] = strip;
        }
        return;
    }
    if (n == 0) return;
    const int umax = uniform((n + kWave - 1) / kWave);
    uint32_t wd[E];
    ET v[E];
    int cmin = INT_MAX, cmax = -1;
#pragma unroll
    for (int u = 0; u < E; ++u) {
        wd[u] = 0u;
        v[u] = ET(0);
        if (u < umax) {
            const int i = lane + kWave * u;
            const int r = row_in_strip<HB>(sr.myrp, sr.s0 + i, 0);
            if (i < n) {
                const int c = col_ind[sr.s0 + i];
                v[u] = val_in[sr.s0 + i];
                wd[u] = (static_cast<uint32_t>(c) << bits) | static_cast<uint32_t>(r);
                cmin = min(cmin, c);
                cmax = max(cmax, c);
            }
        }
    }
#pragma unroll
    for (int off = kWave / 2; off >= 1; off >>= 1) {
        cmin = min(cmin, __shfl_xor(cmin, off));
        cmax = max(cmax, __shfl_xor(cmax, off));
    }
    int nbk = 1;
    while (nbk < NBMAX && nbk * 4 < n) nbk <<= 1;
    // bucket(c) = ((c - cmin) * scale) >> 32 with scale = floor(2^32 nbk /
    // range): non-decreasing in c and below nbk for c <= cmax.
    const uint64_t range = static_cast<uint64_t>(cmax - cmin) + 1u;
    const uint64_t scale = (static_cast<uint64_t>(nbk) << 32) / range;
    int* cnt = bcnt[wave];
    int* start = bstart[wave];
    uint64_t* K = keys[wave];
    for (int b = lane; b < nbk; b += kWave) cnt[b] = 0;
    wave_lds_sync();
    int bs[E];  // bucket << 16 | slot in bucket
#pragma unroll
    for (int u = 0; u < E; ++u) {
        bs[u] = 0;
        if (u < umax && lane + kWave * u < n) {
            const uint32_t c = wd[u] >> bits;
            const int bk = static_cast<int>((static_cast<uint64_t>(c - static_cast<uint32_t>(cmin)) * scale) >> 32);
            bs[u] = (bk << 16) | atomicAdd(&cnt[bk], 1);
        }
    }
    wave_lds_sync();
    // Exclusive scan of the counts: lane l sums buckets [l*per, (l+1)*per).
    const int per = (nbk + kWave - 1) / kWave;
    int mysum = 0, mymax = 0;
    for (int k = 0; k < per; ++k) {
        const int b = lane * per + k;
        if (b < nbk) {
            mysum += cnt[b];
            mymax = max(mymax, cnt[b]);
        }
    }
    int incl = mysum;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int t = __shfl_up(incl, off);
        if (lane >= off) incl += t;
    }
#pragma unroll
    for (int off = kWave / 2; off >= 1; off >>= 1) mymax = max(mymax, __shfl_xor(mymax, off));
    int run = incl - mysum;
    for (int k = 0; k < per; ++k) {
        const int b = lane * per + k;
        if (b < nbk) {
            start[b] = run;
            run += cnt[b];
        }
    }
    wave_lds_sync();
    if (mymax <= kBucketMax) {
#pragma unroll
        for (int u = 0; u < E; ++u) {
            const int i = lane + kWave * u;
            if (u < umax && i < n)
                K[start[bs[u] >> 16] + (bs[u] & 0xffff)] = (static_cast<uint64_t>(wd[u]) << 32) | static_cast<uint32_t>(i);
        }
        wave_lds_sync();
        int pos[E];
#pragma unroll
        for (int u = 0; u < E; ++u) {
            const int i = lane + kWave * u;
            pos[u] = 0;
            if (u < umax && i < n) {
                const int bk = bs[u] >> 16;
                const int b0 = start[bk], b1 = b0 + cnt[bk];
                const uint64_t key = (static_cast<uint64_t>(wd[u]) << 32) | static_cast<uint32_t>(i);
                int p = b0;
                for (int k = b0; k < b1; ++k) p += K[k] < key ? 1 : 0;
                pos[u] = p;
            }
        }
        // The strip's sorted words, then its sorted values, go through the
        // key buffer and out in order: a scatter into the strip's range would
        // leave partly written lines (each reaching HBM more than once).
        wave_lds_sync();
        uint32_t* KW = reinterpret_cast<uint32_t*>(K);
#pragma unroll
        for (int u = 0; u < E; ++u)
            if (u < umax && lane + kWave * u < n) KW[pos[u]] = wd[u];
        wave_lds_sync();
        for (int i = lane; i < n; i += kWave) col_word[sr.s0 + i] = KW[i];
        wave_lds_sync();
        ET* KV = reinterpret_cast<ET*>(K);
#pragma unroll
        for (int u = 0; u < E; ++u)
            if (u < umax && lane + kWave * u < n) KV[pos[u]] = v[u];
        wave_lds_sync();
        for (int i = lane; i < n; i += kWave) val_out[sr.s0 + i] = KV[i];
    } else {
        const int P = pow2_at_least(n);
#pragma unroll
        for (int u = 0; u < E; ++u) {
            const int i = lane + kWave * u;
            if (i < n)
                K[i] = (static_cast<uint64_t>(wd[u]) << 32) | static_cast<uint32_t>(i);
            else if (i < P)
                K[i] = ~0ull;
        }
        wave_lds_sync();
        bitonic_sort(K, P, lane, kWave, [] { wave_lds_sync(); });
        for (int i = lane; i < n; i += kWave) {
            const uint64_t kk = K[i];
            col_word[sr.s0 + i] = static_cast<uint32_t>(kk >> 32);
            val_out[sr.s0 + i] = val_in[sr.s0 + static_cast<int>(static_cast<uint32_t>(kk))];
        }
    }
}

// CMRS -> CSR at height 1: every strip is one row, so RowPtr is StripPtr and
// every entry keeps its place (column = word >> bits); a plain coalesced
// stream.  (A word with a non-zero RowInStrip is invalid input at height 1;
// it is copied like the others.)
template <typename ET>
__global__ __launch_bounds__(256) void to_csr_h1_kernel(int rows, int nnz, int bits, const int* __restrict__ strip_ptr,
                                                        const uint32_t* __restrict__ word, const ET* __restrict__ val,
                                                        int* __restrict__ row_ptr, int* __restrict__ col_ind,
                                                        ET* __restrict__ val_out) {
    constexpr int U = 4;
    const int64_t nthreads = static_cast<int64_t>(gridDim.x) * blockDim.x;
    const int64_t tid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    for (int64_t i = tid; i <= rows; i += nthreads) row_ptr[i] = strip_ptr[i];
    for (int64_t b0 = static_cast<int64_t>(blockIdx.x) * blockDim.x * U; b0 < nnz; b0 += nthreads * U) {
        uint32_t w[U];
        ET v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t j = b0 + u * blockDim.x + threadIdx.x;
            w[u] = j < nnz ? word[j] : 0u;
            v[u] = j < nnz ? val[j] : ET(0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t j = b0 + u * blockDim.x + threadIdx.x;
            if (j < nnz) {
                col_ind[j] = static_cast<int>(w[u] >> bits);
                val_out[j] = v[u];
            }
        }
    }
}

// Strip of every lane's entry in one round of a wave's run of whole strips.
// Lane t <= nsw holds StripPtr[S + t] (INT_MAX past that); `tc` (uniform)
// enters as the last strip whose pointer is <= the round's first entry and
// leaves as that of the round's last entry `lim`, so the rounds of a run step
// through its strip pointers once, whatever the strip lengths.  Empty strips
// are passed over because their pointer repeats.
__device__ inline int round_strip(int myp, int j, int lim, int& tc) {
    int t = tc;
    for (;;) {
        const int nx = __builtin_amdgcn_readlane(myp, tc + 1);
        if (nx > lim) break;
        if (j >= nx) t = tc + 1;
        ++tc;
    }
    return t;
}

// Key of an entry of strip t of the run: t*height + RowInStrip, the row's
// offset from the run's first row; -1 for a word whose RowInStrip names no
// row of its strip (the entry is then neither counted nor written).
__device__ inline int run_row_key(int t, uint32_t r, int height, int nrow) {
    const int key = t * height + static_cast<int>(r);
    return (r < static_cast<uint32_t>(height) && key < nrow) ? key : -1;
}

// Rows per wave of the CMRS -> CSR kernel: lane k < kRunRows owns row k of
// the wave's run, and row keys fit in kRunKeyBits bits.
constexpr int kRunRows = 32;
constexpr int kRunKeyBits = 5;

// Lanes of `valid` whose key (< kRunRows) equals k, from kb[b] = ballot of bit
// b of every lane's key: a match over the wave without a loop over key values.
__device__ inline uint64_t key_match(int k, uint64_t valid, const uint64_t (&kb)[kRunKeyBits]) {
    uint64_t m = valid;
#pragma unroll
    for (int b = 0; b < kRunKeyBits; ++b) m &= ((k >> b) & 1) ? kb[b] : ~kb[b];
    return m;
}

// One round of 64 consecutive entries [b, b + 64) of a run: every lane's row
// key (-1: no entry or an invalid word), its key ballots and the valid mask.
struct RunRound {
    int key;
    uint64_t valid;
    uint64_t kb[kRunKeyBits];
};

__device__ inline RunRound run_round(int myp, int b, int e1, uint32_t w, uint32_t mask, int height, int nrow, int& tc) {
    RunRound rr;
    const int j = b + lane_id();
    const int t = round_strip(myp, j, min(b + kWave, e1) - 1, tc);
    rr.key = j < e1 ? run_row_key(t, w & mask, height, nrow) : -1;
#pragma unroll
    for (int k = 0; k < kRunKeyBits; ++k) rr.kb[k] = ballot(rr.key >= 0 && ((rr.key >> k) & 1));
    rr.valid = ballot(rr.key >= 0);
    return rr;
}

// Waves per workgroup of the CMRS -> CSR kernel, and the run length above
// which the workgroup's waves share a run.  (2 and 8 waves were measured
// slower on both the benchmark and the skewed-row matrices.)
constexpr int kToCsrWaves = 4;
constexpr int kToCsrThreads = kToCsrWaves * kWave;
constexpr int kLongRun = 2048;
constexpr int kToCsrStage = 640;

// One run of the CMRS -> CSR kernel: strips [S, S + nsw), rows [r0, r0 +
// nrow), entries [e0, e1); lane t <= nsw holds StripPtr[S + t] in myp.
struct ToCsrRun {
    int S, nsw, r0, nrow, e0, e1, myp;
};

__device__ inline ToCsrRun to_csr_run(int run, int ns, int strips, int rows, int height,
                                      const int* __restrict__ strip_ptr, int lane) {
    ToCsrRun R;
    R.S = run * ns;
    R.nsw = R.S < strips ? min(ns, strips - R.S) : 0;
    R.myp = (R.nsw > 0 && lane <= R.nsw) ? strip_ptr[R.S + lane] : INT_MAX;
    const int p0 = __shfl(R.myp, 0), p1 = __shfl(R.myp, R.nsw);
    R.e0 = R.nsw > 0 ? uniform(p0) : 0;
    R.e1 = R.nsw > 0 ? uniform(p1) : 0;
    R.r0 = R.S * height;
    R.nrow = R.nsw > 0 ? min(R.nsw * height, rows - R.r0) : 0;
    return R;
}

// CMRS -> CSR with one wave per run of `ns` whole strips (ns*height <=
// kRunRows consecutive rows, lane k owning row k of the run).  The run's
// entries are contiguous, so the wave streams them 64 at a time with
// coalesced loads whatever the strip lengths.  Pass 1 counts the entries of
// every row (the rows' CSR starts are then a prefix sum over the lanes); pass
// 2 scatters each entry to its row's start plus its rank, the number of
// earlier entries of the same row (earlier rounds: a per-row counter; this
// round: lanes below it with the same key).  The scatter keeps strip order
// inside every row, the stable order of the inverse conversion.  A run of at
// most FIT entries is loaded once and both passes work on the registers;
// longer runs are read twice.  A run of more than kLongRun entries is shared
// by the workgroup's waves after they have finished their own runs: each wave
// counts a contiguous slice, the per-row counts of earlier slices (LDS) start
// its ranks, and each wave scatters its slice.  Every wave reads the lengths
// of the workgroup's runs and so takes the same barrier-or-not decision; a
// workgroup without a long run has no barrier.
template <typename ET, bool STAGE>
__global__ __launch_bounds__(kToCsrThreads) __attribute__((amdgpu_waves_per_eu(STAGE ? 5 : 8))) void to_csr_rows_kernel(
    int rows, int strips, int height, int bits, int ns, const int* __restrict__ strip_ptr,
    const uint32_t* __restrict__ word, const ET* __restrict__ val, int* __restrict__ row_ptr,
    int* __restrict__ col_ind, ET* __restrict__ val_out) {
    constexpr int UF = 12, U = 8, FIT = UF * kWave;
    __shared__ int slice_cnt[kToCsrWaves][kRunRows];
    // STAGE: a run of at most kToCsrStage entries is scattered into LDS and
    // then written out in order (the run's CSR range is contiguous): with many
    // rows per strip the 64 lanes of a scatter would otherwise each write into
    // another line.  The LDS lowers the waves per SIMD from 8 to 5, which costs
    // more than it saves at small heights and on runs of very uneven length.
    constexpr int SCAP = STAGE ? kToCsrStage : 1;
    __shared__ int stage_col[kToCsrWaves][SCAP];
    __shared__ ET stage_val[kToCsrWaves][SCAP];
    const int lane = lane_id();
    const int wave = uniform(static_cast<int>(threadIdx.x) / kWave);
    const int run0 = xcd_logical_block(blockIdx.x, gridDim.x) * kToCsrWaves;
    const int nruns = (strips + ns - 1) / ns;
    const uint32_t mask = (1u << bits) - 1u;
    const uint64_t lt = lanemask_lt();

    // This wave's run, loaded before the lengths below so that both loads are
    // in flight together.
    const ToCsrRun Rw = to_csr_run(run0 + wave, ns, strips, rows, height, strip_ptr, lane);
    // Bit r: run run0 + r holds more than kLongRun entries (lanes r <
    // kToCsrWaves read the runs' first strip pointers, the next kToCsrWaves
    // lanes their last).
    uint64_t longs;
    {
        const int run = run0 + (lane & (kToCsrWaves - 1));
        const int sidx = min(run * ns + (lane >= kToCsrWaves ? ns : 0), strips);
        const int p = (lane < 2 * kToCsrWaves && run < nruns) ? strip_ptr[sidx] : 0;
        const int pend = __shfl(p, (lane & (kToCsrWaves - 1)) + kToCsrWaves);
        longs = ballot(lane < kToCsrWaves && run < nruns && pend - p > kLongRun);
    }

    // CSR starts of the run's rows from per-row counts (lane k: row k);
    // `write` stores them.
    auto row_starts = [&](const ToCsrRun& R, int cnt, bool write) {
        int incl = cnt;
#pragma unroll
        for (int off = 1; off < kRunRows; off <<= 1) {
            const int v = __shfl_up(incl, off);
            if (lane >= off) incl += v;
        }
        const int start = R.e0 + incl - cnt;
        if (write && lane < R.nrow) row_ptr[R.r0 + lane] = start;
        if (write && R.S + R.nsw == strips && lane == 0) row_ptr[rows] = R.e1;
        return start;
    };
    // Scatter of one round; `next` (lane k): CSR position of the next entry of row k.
    auto scatter = [&](const ToCsrRun& R, const RunRound& rr, uint32_t w, ET v, int& next) {
        const int src = rr.key >= 0 ? rr.key : 0;
        const int pos = __shfl(next, src) + __popcll(key_match(src, rr.valid, rr.kb) & lt);
        // pos lies in [e0, e1) by construction; the check keeps a corrupt
        // strip from writing outside its run.
        if (rr.key >= 0 && static_cast<unsigned>(pos - R.e0) < static_cast<unsigned>(R.e1 - R.e0)) {
            col_ind[pos] = static_cast<int>(w >> bits);
            val_out[pos] = v;
        }
        next += __popcll(key_match(lane, rr.valid, rr.kb));
    };
    // Per-row counts (lane k: row k) of the run's entries [lo, hi).
    auto count_range = [&](const ToCsrRun& R, int lo, int hi) {
        int cnt = 0, tc = 0;
        for (int b0 = lo; b0 < hi; b0 += U * kWave) {
            uint32_t w[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = b0 + u * kWave + lane;
                w[u] = j < hi ? word[j] : 0u;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (b0 + u * kWave >= hi) break;
                const RunRound rr = run_round(R.myp, b0 + u * kWave, hi, w[u], mask, height, R.nrow, tc);
                cnt += __popcll(key_match(lane, rr.valid, rr.kb));
            }
        }
        return cnt;
    };
    // Scatter of the run's entries [lo, hi).
    auto scatter_range = [&](const ToCsrRun& R, int lo, int hi, int& next) {
        int tc = 0;
        for (int b0 = lo; b0 < hi; b0 += U * kWave) {
            uint32_t w[U];
            ET v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = b0 + u * kWave + lane;
                w[u] = j < hi ? word[j] : 0u;
                v[u] = j < hi ? val[j] : ET(0);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (b0 + u * kWave >= hi) break;
                const RunRound rr = run_round(R.myp, b0 + u * kWave, hi, w[u], mask, height, R.nrow, tc);
                scatter(R, rr, w[u], v[u], next);
            }
        }
    };

    // This wave's own run, unless it is long.
    if (run0 + wave < nruns && !((longs >> wave) & 1)) {
        const ToCsrRun& R = Rw;
        if (R.e1 - R.e0 <= FIT) {
            uint32_t w[UF];
            ET v[UF];
#pragma unroll
            for (int u = 0; u < UF; ++u) {
                const int j = R.e0 + u * kWave + lane;
                w[u] = j < R.e1 ? word[j] : 0u;
                v[u] = j < R.e1 ? val[j] : ET(0);
            }
            int cnt = 0, tc = 0;
#pragma unroll
            for (int u = 0; u < UF; ++u) {
                if (R.e0 + u * kWave >= R.e1) break;
                const RunRound rr = run_round(R.myp, R.e0 + u * kWave, R.e1, w[u], mask, height, R.nrow, tc);
                cnt += __popcll(key_match(lane, rr.valid, rr.kb));
            }
            int next = row_starts(R, cnt, true);
            tc = 0;
            const int n = R.e1 - R.e0;
            if (STAGE && n <= SCAP) {
                int* sc = stage_col[wave];
                ET* sv = stage_val[wave];
#pragma unroll
                for (int u = 0; u < UF; ++u) {
                    if (R.e0 + u * kWave >= R.e1) break;
                    const RunRound rr = run_round(R.myp, R.e0 + u * kWave, R.e1, w[u], mask, height, R.nrow, tc);
                    const int src = rr.key >= 0 ? rr.key : 0;
                    const int pos = __shfl(next, src) + __popcll(key_match(src, rr.valid, rr.kb) & lt) - R.e0;
                    if (rr.key >= 0 && static_cast<unsigned>(pos) < static_cast<unsigned>(n)) {
                        sc[pos] = static_cast<int>(w[u] >> bits);
                        sv[pos] = v[u];
                    }
                    next += __popcll(key_match(lane, rr.valid, rr.kb));
                }
                wave_lds_sync();
                // Every place of the run is written above (the rows' counts
                // add up to n) unless a word names no row of its strip; those
                // places keep what the stage held and are not valid output.
                for (int i = lane; i < n; i += kWave) {
                    col_ind[R.e0 + i] = sc[i];
                    val_out[R.e0 + i] = sv[i];
                }
                wave_lds_sync();
            } else {
#pragma unroll
                for (int u = 0; u < UF; ++u) {
                    if (R.e0 + u * kWave >= R.e1) break;
                    const RunRound rr = run_round(R.myp, R.e0 + u * kWave, R.e1, w[u], mask, height, R.nrow, tc);
                    scatter(R, rr, w[u], v[u], next);
                }
            }
        } else {
            int next = row_starts(R, count_range(R, R.e0, R.e1), true);
            scatter_range(R, R.e0, R.e1, next);
        }
    }

    // The workgroup's long runs, shared by all its waves (`longs` is the same
    // in every wave, so every wave meets the same barriers).
    if (longs) {
        for (int r = 0; r < kToCsrWaves; ++r) {
            if (!((longs >> r) & 1)) continue;
            const ToCsrRun R = to_csr_run(run0 + r, ns, strips, rows, height, strip_ptr, lane);
            const int n = R.e1 - R.e0;
            const int chunk = ((n + kToCsrWaves - 1) / kToCsrWaves + kWave - 1) / kWave * kWave;
            const int lo = min(R.e0 + wave * chunk, R.e1), hi = min(lo + chunk, R.e1);
            const int cnt = count_range(R, lo, hi);
            if (lane < kRunRows) slice_cnt[wave][lane] = cnt;
            __syncthreads();
            int tot = 0, before = 0;
            if (lane < kRunRows) {
                for (int w2 = 0; w2 < kToCsrWaves; ++w2) {
                    const int c = slice_cnt[w2][lane];
                    tot += c;
                    if (w2 < wave) before += c;
                }
            }
            int next = row_starts(R, tot, wave == 0) + before;
            scatter_range(R, lo, hi, next);
            __syncthreads();  // slice_cnt is reused by the next long run
        }
    }
}

// CSR -> CMRS without the reorder, one wave per run of `ns` whole strips
// (ns*height <= kRunRows consecutive rows); lane k <= nrow holds RowPtr of
// row k of the run.  Entries keep their places, so the wave streams the run's
// (contiguous) entries 64 at a time with coalesced loads: the row of every
// entry comes from stepping through the run's row pointers (`round_strip`),
// and word = col << bits | (row mod height).  Writes the strip pointers too.
// col_word may alias col_ind and val_out may alias val_in (each entry is read
// and written by the same lane).
template <typename ET>
__global__ __launch_bounds__(kConvThreads) void from_csr_rows_kernel(
    int rows, int strips, int height, int bits, int nnz, int ns, const int* __restrict__ row_ptr,
    const int* col_ind, const ET* val_in, int* __restrict__ strip_ptr, uint32_t* col_word, ET* val_out,
    int copy_val) {
    constexpr int U = 8;
    const int lane = lane_id();
    const int wave = uniform(static_cast<int>(threadIdx.x) / kWave);
    const int S = (xcd_logical_block(blockIdx.x, gridDim.x) * kConvWaves + wave) * ns;
    if (S >= strips) return;
    const int nsw = min(ns, strips - S);
    const int r0 = S * height;
    const int nrow = min(nsw * height, rows - r0);
    const int myrp = lane <= nrow ? row_ptr[r0 + lane] : INT_MAX;
    const int e0 = uniform(__shfl(myrp, 0)), e1 = uniform(__shfl(myrp, nrow));
    const int sfirst = __shfl(myrp, min(lane * height, kRunRows));  // first entry of strip S + lane
    if (lane < nsw) strip_ptr[S + lane] = sfirst;
    if (S + nsw == strips && lane == 0) strip_ptr[strips] = nnz;
    const bool pow2 = (height & (height - 1)) == 0;
    int tc = 0;
    for (int b0 = e0; b0 < e1; b0 += U * kWave) {
        int c[U];
        ET v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = b0 + u * kWave + lane;
            c[u] = j < e1 ? col_ind[j] : 0;
            v[u] = j < e1 ? val_in[j] : ET(0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (b0 + u * kWave >= e1) break;
            const int j = b0 + u * kWave + lane;
            const int k = round_strip(myrp, j, min(b0 + u * kWave + kWave, e1) - 1, tc);
            const int r = pow2 ? (k & (height - 1)) : k % height;
            if (j < e1) {
                col_word[j] = (static_cast<uint32_t>(c[u]) << bits) | static_cast<uint32_t>(r);
                if (copy_val) val_out[j] = v[u];
            }
        }
    }
}

// ------------------------------------------------------------------ list kernels

// One listed long strip of n entries by the whole 1024-thread workgroup, in K
// (LDS, or the strip's workspace slice of 2n 64-bit words when keys_global;
// passes over global memory then need an agent-scope fence before the
// barrier).  Rows sorted by column: the words sit in K as 32-bit words in
// strip order and each entry's place in the sorted strip is its index in its
// own row plus, for every other row, the number of that row's words below
// its own (binary search; the words of different rows never tie).  No second
// buffer and no passes: one barrier after the words are in.  Otherwise a
// bitonic network over (word, position) keys in K, which needs room for
// pow2(n) <= 2n keys.  Forced inline, so that the LDS call site keeps the LDS
// address space.
template <int HB, typename ET>
__device__ __forceinline__ void sort_strip_block(const StripRows& sr, int n, int bits,
                                                 const int* __restrict__ col_ind, const ET* __restrict__ val_in,
                                                 uint32_t* __restrict__ col_word, ET* __restrict__ val_out, uint64_t* K,
                                                 bool keys_global, int* rt, int tid, int wave, int lane) {
    uint32_t* W = reinterpret_cast<uint32_t*>(K);
    const auto sync = [keys_global] {
        if (keys_global) __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
        __syncthreads();
    };
    // Words in order, with the canonical-row check on the way: entry i and
    // i + 1 of one row must not descend by column.
    bool bad = false;
    for (int base = wave * kWave; base < n; base += kBlockSortThreads) {
        const int i = base + lane;
        const int r = row_in_strip<HB>(sr.myrp, sr.s0 + i, 0);
        const int rn = row_in_strip<HB>(sr.myrp, sr.s0 + i + 1, 0);
        if (i < n) {
            const int c = col_ind[sr.s0 + i];
            W[i] = (static_cast<uint32_t>(c) << bits) | static_cast<uint32_t>(r);
            if (i + 1 < n && rn == r && col_ind[sr.s0 + i + 1] < c) bad = true;
        }
    }
    if (tid <= HB) rt[tid] = tid < sr.nr ? sr.myrp - sr.s0 : n;  // wave 0: lane == tid
    if (keys_global) __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
    if (__syncthreads_or(bad) == 0) {
        for (int i = tid; i < n; i += kBlockSortThreads) {
            const uint32_t w = W[i];
            const int r = static_cast<int>(w & static_cast<uint32_t>(HB - 1));
            int pos = i - rt[r];
            for (int x = 0; x < HB; ++x) {
                if (x == r) continue;
                const int lo = rt[x];
                int a = lo, len = rt[x + 1] - lo;
                while (len > 0) {
                    const int half = len >> 1;
                    if (W[a + half] < w) {
                        a += half + 1;
                        len -= half + 1;
                    } else {
                        len = half;
                    }
                }
                pos += a - lo;
            }
            if (static_cast<unsigned>(pos) < static_cast<unsigned>(n)) {
                col_word[sr.s0 + pos] = w;
                val_out[sr.s0 + pos] = val_in[sr.s0 + i];
            }
        }
    } else {
        const int P = pow2_at_least(n);
        sync();  // W is read above; the keys overwrite it
        // P is a multiple of 64, so every lane of a wave takes each trip of
        // this loop: the row lookup's cross-lane reads see all lanes.
        for (int i = tid; i < P; i += kBlockSortThreads) {
            const int r = row_in_strip<HB>(sr.myrp, sr.s0 + i, 0);
            uint64_t key = ~0ull;
            if (i < n)
                key = (static_cast<uint64_t>((static_cast<uint32_t>(col_ind[sr.s0 + i]) << bits) |
                                             static_cast<uint32_t>(r))
                       << 32) |
                      static_cast<uint32_t>(i);
            K[i] = key;
        }
        sync();
        bitonic_sort(K, P, tid, kBlockSortThreads, sync);
        for (int i = tid; i < n; i += kBlockSortThreads) {
            const uint64_t kk = K[i];
            col_word[sr.s0 + i] = static_cast<uint32_t>(kk >> 32);
            val_out[sr.s0 + i] = val_in[sr.s0 + static_cast<int>(static_cast<uint32_t>(kk))];
        }
    }
}

// Entries [lo, lo + len) of a sorted LDS array below w, for C entries at
// once: the searches step together (binary lifting, as many steps as the
// longest of the C ranges needs) so their LDS reads are in flight together.
template <int C>
__device__ inline void count_below(const uint32_t* S, const uint32_t (&w)[C], const int (&lo)[C],
                                   const int (&len)[C], int (&cnt)[C]) {
    int top = 0;
#pragma unroll
    for (int v = 0; v < C; ++v) {
        top |= len[v];
        cnt[v] = 0;
    }
    top = top > 0 ? 1 << (31 - __clz(top)) : 0;
    for (int step = top; step > 0; step >>= 1) {
#pragma unroll
        for (int v = 0; v < C; ++v) {
            const bool ok = cnt[v] + step <= len[v];
            const uint32_t x = S[ok ? lo[v] + cnt[v] + step - 1 : 0];
            if (ok && x < w[v]) cnt[v] += step;
        }
    }
}

// Rows of at most kLightRow entries are light; the light/heavy ranking below
// is used while a strip's light rows hold at most kLightCap entries in all.
constexpr int kLightRow = 64;
constexpr int kLightCap = 512;

// One listed strip of n <= 16*NT entries by a workgroup of NT threads;
// thread t owns entries t + NT*u.  Rows sorted by column: the words go to
// LDS (A) and each entry's place in the sorted strip is its rank among the
// strip's words (the words of different rows never tie; equal words of one
// row keep CSR order).  Long listed strips are mostly one or a few long rows
// among short ones, and one binary search per (entry, other row) makes the
// entries of a long row search every short row; instead:
//  * the words of the light rows are gathered, in strip order, into LW (m of
//    them); thread t takes light word t and counts the light words below it
//    by reading all m (the same words for every lane: no bank conflicts, no
//    dependent loads); that count is its rank among the light words, kept in
//    LR, and its word goes to that rank in SL (the light words sorted);
//  * an entry of a heavy row adds to its index in its row one binary search
//    over SL, a light entry starts from its rank in LR, and every entry adds
//    one binary search over each other heavy row.
// With more than kLightCap light entries every row counts as heavy (one
// search per other row).  Words and values then go to their places.  Global
// loads (columns and values) are issued together, indices past the strip
// clamped to its last entry, so a thread waits for memory once per strip;
// prefetch() is called while they are in flight.  Rows not sorted: a bitonic
// network over (word, position) keys in K, which holds pow2(n) keys.  K, A,
// LW, LR and SL share the same LDS.
template <int HB, int NT, typename ET, typename Prefetch>
__device__ __forceinline__ void rank_strip_block(const StripRows& sr, int n, int bits,
                                                 const int* __restrict__ col_ind, const ET* __restrict__ val_in,
                                                 uint32_t* __restrict__ col_word, ET* __restrict__ val_out,
                                                 uint64_t* K, int tid, Prefetch prefetch) {
    constexpr int E = 16;
    constexpr int CAP = E * NT;
    constexpr int C = 4;  // slots searched together
    static_assert(CAP + 3 * kLightCap <= 2 * CAP, "light lists must fit beside the words");
    uint32_t* A = reinterpret_cast<uint32_t*>(K);
    uint32_t* LW = A + CAP;
    uint32_t* SL = LW + kLightCap;
    int* LR = reinterpret_cast<int*>(SL + kLightCap);
    const int lane = static_cast<int>(threadIdx.x) % kWave;
    const int umax = (n + NT - 1) / NT;
    int pos[E];
    // Values: those of the first E/2 slots are loaded with the columns (one
    // wait per strip for strips of up to 8*NT entries), the rest at the end.
    ET vv[E / 2];
    // Rows sorted by column: entry i and i + 1 of one row do not descend.
    // Pairs inside a wave are checked before the first barrier, the pairs
    // across waves (lane 63, next wave's lane 0) after it, from A.
    bool bad = false;
    {
        uint32_t c[E];
#pragma unroll
        for (int u = 0; u < E; ++u) {
            pos[u] = tid + NT * u;
            if (u < umax) {
                const int j = sr.s0 + min(pos[u], n - 1);
                c[u] = static_cast<uint32_t>(col_ind[j]);
                if (u < E / 2) vv[u % (E / 2)] = val_in[j];
            }
        }
        prefetch();  // the caller's loads for its next strip, in flight with these
#pragma unroll
        for (int u = 0; u < E; ++u) {
            if (u < umax) {  // uniform: every lane runs the row lookup and the shuffles
                const int i = pos[u];
                const int r = row_in_strip<HB>(sr.myrp, sr.s0 + i, 0);
                const int rend = __shfl(sr.myrp, r + 1) - sr.s0;  // end of the entry's row
                const uint32_t cn = __shfl_down(c[u], 1);
                if (lane < kWave - 1 && i + 1 < n && i + 1 < rend && cn < c[u]) bad = true;
                if (i < n) A[i] = (c[u] << bits) | static_cast<uint32_t>(r);
            }
        }
    }
    bad = __syncthreads_or(bad) != 0;  // uniform from here on
    bool bad_across = false;
    if (!bad && lane == kWave - 1) {
        const uint32_t rmask = (1u << bits) - 1u;
#pragma unroll
        for (int u = 0; u < E; ++u) {
            const int i = tid + NT * u;
            if (u < umax && i + 1 < n) {
                const uint32_t w = A[i], nw = A[i + 1];
                if ((nw & rmask) == (w & rmask) && (nw >> bits) < (w >> bits)) bad_across = true;
            }
        }
    }
    // Row table in the lanes of every wave: lane x < HB holds row x's start
    // and length in the strip (rows past the strip: start n, length 0).
    const int rlo = lane < sr.nr ? sr.myrp - sr.s0 : n;
    const int rnext = __shfl(rlo, min(lane + 1, kWave - 1));
    const int rlen = lane < HB ? rnext - rlo : 0;
    int m = 0;  // entries in light rows
    {
        int v = (lane < HB && rlen <= kLightRow) ? rlen : 0;
#pragma unroll
        for (int off = 1; off < HB; off <<= 1) v += __shfl_xor(v, off);
        m = __shfl(v, 0);
    }
    const int lt = m <= kLightCap ? kLightRow : -1;  // rows of at most lt entries are light
    if (lt < 0) m = 0;
    const bool rlight = lane < HB && rlen <= lt;
    int rls = rlight ? rlen : 0;  // row's first index in LW: exclusive prefix over the lanes
#pragma unroll
    for (int off = 1; off < HB; off <<= 1) {
        const int t = __shfl_up(rls, off);
        if (lane >= off) rls += t;
    }
    rls -= rlight ? rlen : 0;
    const uint64_t heavy = ballot(lane < HB && rlen > lt && rlen > 0);
    if (!bad && m > 0) {  // uniform
#pragma unroll
        for (int u = 0; u < E; ++u) {
            if (u < umax) {  // uniform: every lane runs the shuffles
                const int i = tid + NT * u;
                const uint32_t w = i < n ? A[i] : 0u;
                const int r = static_cast<int>(w & static_cast<uint32_t>(HB - 1));
                const int lo = __shfl(rlo, r), ls = __shfl(rls, r), lg = __shfl(rlight ? 1 : 0, r);
                if (i < n && lg) LW[ls + i - lo] = w;
            }
        }
    }
    if (!bad) bad = __syncthreads_or(bad_across) != 0;
    if (!bad) {
        if (m > 0) {
            // Rank of light word t among the light words; LW is 16-byte aligned
            // and read four words at a time (the same words in every lane).
            const uint4* LW4 = reinterpret_cast<const uint4*>(LW);
            for (int t = tid; t < m; t += NT) {
                const uint32_t w = LW[t];
                int cnt = 0;
                const auto add = [&](uint32_t a, int j) { cnt += (a < w || (a == w && j < t)) ? 1 : 0; };
                int j = 0;
                for (; j + 8 <= m; j += 8) {
                    const uint4 p = LW4[j / 4], q = LW4[j / 4 + 1];
                    add(p.x, j); add(p.y, j + 1); add(p.z, j + 2); add(p.w, j + 3);
                    add(q.x, j + 4); add(q.y, j + 5); add(q.z, j + 6); add(q.w, j + 7);
                }
                for (; j < m; ++j) add(LW[j], j);
                LR[t] = cnt;
                SL[cnt] = w;
            }
            __syncthreads();
        }
        // Places.
#pragma unroll
        for (int u0 = 0; u0 < E; u0 += C) {
            if (u0 >= umax) break;
            uint32_t w[C];
            int r[C], lo[C], len[C], cnt[C];
            bool live[C];
#pragma unroll
            for (int v = 0; v < C; ++v) {
                const int i = tid + NT * (u0 + v);
                live[v] = i < n;
                w[v] = live[v] ? A[i] : 0u;
                r[v] = static_cast<int>(w[v] & static_cast<uint32_t>(HB - 1));
                const int rl = __shfl(rlo, r[v]), ls = __shfl(rls, r[v]), lg = __shfl(rlight ? 1 : 0, r[v]);
                const bool hv = live[v] && !lg;
                if (live[v]) pos[u0 + v] = hv ? i - rl : LR[ls + i - rl];
                lo[v] = 0;
                len[v] = hv ? m : 0;
            }
            count_below<C>(SL, w, lo, len, cnt);
#pragma unroll
            for (int v = 0; v < C; ++v) pos[u0 + v] += cnt[v];
            for (uint64_t hm = heavy; hm; hm &= hm - 1) {  // uniform
                const int x = __ffsll(static_cast<unsigned long long>(hm)) - 1;
                const int xlo = __shfl(rlo, x), xlen = __shfl(rlen, x);
#pragma unroll
                for (int v = 0; v < C; ++v) {
                    lo[v] = xlo;
                    len[v] = (live[v] && x != r[v]) ? xlen : 0;
                }
                count_below<C>(A, w, lo, len, cnt);
#pragma unroll
                for (int v = 0; v < C; ++v) pos[u0 + v] += cnt[v];
            }
        }
        ET vl[E / 2];
#pragma unroll
        for (int u = E / 2; u < E; ++u)
            if (u < umax) vl[u - E / 2] = val_in[sr.s0 + min(tid + NT * u, n - 1)];
#pragma unroll
        for (int u = 0; u < E; ++u) {
            const int i = tid + NT * u;
            if (u < umax && i < n && static_cast<unsigned>(pos[u]) < static_cast<unsigned>(n)) {
                col_word[sr.s0 + pos[u]] = A[i];
                val_out[sr.s0 + pos[u]] = u < E / 2 ? vv[u % (E / 2)] : vl[u % (E / 2)];
            }
        }
    } else {
        const int P = pow2_at_least(n);
        // P is a multiple of 64, so every lane of a wave takes each trip of
        // this loop: the row lookup's cross-lane reads see all lanes.
        for (int i = tid; i < P; i += NT) {
            const int r = row_in_strip<HB>(sr.myrp, sr.s0 + i, 0);
            uint64_t key = ~0ull;
            if (i < n)
                key = (static_cast<uint64_t>((static_cast<uint32_t>(col_ind[sr.s0 + i]) << bits) |
                                             static_cast<uint32_t>(r))
                       << 32) |
                      static_cast<uint32_t>(i);
            K[i] = key;
        }
        __syncthreads();
        bitonic_sort(K, P, tid, NT, [] { __syncthreads(); });
        for (int i = tid; i < n; i += NT) {
            const uint64_t kk = K[i];
            col_word[sr.s0 + i] = static_cast<uint32_t>(kk >> 32);
            val_out[sr.s0 + i] = val_in[sr.s0 + static_cast<int>(static_cast<uint32_t>(kk))];
        }
    }
}

// Row pointers of strip `strip` for lane <= rows of the strip (INT_MAX past
// them), as load_strip_rows reads them.
__device__ inline int strip_row_ptr(int strip, int rows, int height, const int* __restrict__ row_ptr, int lane) {
    const int r0 = strip * height;
    return lane <= min(height, rows - r0) ? row_ptr[r0 + lane] : INT_MAX;
}

// Sorted conversion of the listed strips, both lists in one launch of one
// 1024-thread workgroup per CU.  First the long strips (more than
// kWaveSortCap entries): workgroup b takes list entry b first, then the next
// untaken entry of a shared counter (ws_count[2], zero at launch), so strips
// of very different lengths still spread evenly.  In LDS when the strip fits
// (n <= kBlockSortCap, rank_strip_block), else in the strip's own slice of
// the workspace [2*s0, 2*s1) (sort_strip_block).  A strip costs a chain of
// dependent global loads (list entry, row pointers, then entries); the next
// strip's list entry and row pointers are loaded while the current one is
// sorted.  Then the short listed strips (at most kWaveSortCap entries): each
// of the workgroup's 16 waves takes the next one from a second counter
// (ws_count[3], zero at launch) and sorts it alone in its sixteenth of the
// key buffer.  A workgroup whose long strips are done (or that drew none)
// goes on to the short ones while others still sort long strips: run as two
// launches, the CUs left idle by the last long strips waited for them.
template <int HB, typename ET>
__global__ __launch_bounds__(kBlockSortThreads) void sort_lists_kernel(
    int rows, int height, int bits, const int* __restrict__ row_ptr, const int* __restrict__ col_ind,
    const ET* __restrict__ val_in, uint32_t* __restrict__ col_word, ET* __restrict__ val_out,
    int* __restrict__ ws_count, const int* __restrict__ ws_small, const int* __restrict__ ws_big,
    uint64_t* __restrict__ gkeys) {
    constexpr int NW = kBlockSortThreads / kWave;
    static_assert(kBlockSortCap >= NW * kWaveSortCap, "a short strip's keys per wave");
    __shared__ uint64_t skeys[kBlockSortCap];
    __shared__ int rt[HB + 1];
    __shared__ int taken[2];
    __shared__ int wrt[NW][HB + 1];
    const int tid = static_cast<int>(threadIdx.x);
    const int lane = lane_id();
    const int wave = uniform(tid / kWave);
    const int count = ws_count[1];
    int item = static_cast<int>(blockIdx.x);
    if (item < count) {
        if (tid == 0) taken[0] = static_cast<int>(gridDim.x) + atomicAdd(&ws_count[2], 1);
        int strip = ws_big[item];
        int myrp = strip_row_ptr(strip, rows, height, row_ptr, lane);
        __syncthreads();
        int next = taken[0];
        for (int k = 1; item < count; ++k) {
            // The entry after `next` is taken now and read after this strip's
            // last barrier (taken[] alternates, so it is not overwritten early).
            if (tid == 0 && next < count) taken[k & 1] = static_cast<int>(gridDim.x) + atomicAdd(&ws_count[2], 1);
            StripRows sr;
            sr.r0 = strip * height;
            sr.nr = min(height, rows - sr.r0);
            sr.myrp = myrp;
            sr.s0 = __shfl(myrp, 0);
            sr.s1 = __shfl(myrp, sr.nr);
            const int n = sr.s1 - sr.s0;
            const int nstrip = next < count ? ws_big[next] : 0;
            int nmyrp = INT_MAX;
            const auto prefetch = [&] {
                if (next < count) nmyrp = strip_row_ptr(nstrip, rows, height, row_ptr, lane);
            };
            if (n <= kBlockSortCap) {
                rank_strip_block<HB, kBlockSortThreads, ET>(sr, n, bits, col_ind, val_in, col_word, val_out, skeys,
                                                            tid, prefetch);
            } else {
                prefetch();
                sort_strip_block<HB, ET>(sr, n, bits, col_ind, val_in, col_word, val_out,
                                         gkeys + 2 * static_cast<size_t>(sr.s0), true, rt, tid, wave, lane);
            }
            __syncthreads();  // the next item reuses skeys and rt
            item = next;
            next = next < count ? taken[k & 1] : count;
            strip = nstrip;
            myrp = nmyrp;
        }
    }
    const int scount = ws_count[0];
    uint64_t* slice = skeys + wave * kWaveSortCap;
    const int nwaves = static_cast<int>(gridDim.x) * NW;
    for (int it = static_cast<int>(blockIdx.x) * NW + wave; it < scount; it += nwaves)
        sort_strip_mid<HB, kWaveSortCap / kWave, ET>(ws_small[it], rows, height, bits, row_ptr, col_ind, val_in,
                                                     col_word, val_out, slice, wrt[wave], lane);
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

struct Conv {
    int rows, strips, height, bits, nnz;
};

// Both lists of strips the first kernel could not sort (sort_lists_kernel):
// one workgroup per CU, or fewer when the lists cannot be that long.
template <int HB, typename ET>
void launch_sort_lists(const Conv& cv, const FromCsrWorkspaceLayout& L, const int* row_ptr, const int* col_ind,
                       const ET* vin, uint32_t* col_word, ET* vout, int* ws_count, const int* ws_small,
                       const int* ws_big, uint64_t* gkeys, hipStream_t stream) {
    constexpr size_t NW = kBlockSortThreads / kWave;
    const size_t want = std::max<size_t>(L.big_cap, (L.small_cap + NW - 1) / NW);
    const int g = static_cast<int>(std::max<size_t>(1, std::min<size_t>(want, kBlockSortGrid)));
    hipLaunchKernelGGL((sort_lists_kernel<HB, ET>), dim3(g), dim3(kBlockSortThreads), 0, stream, cv.rows,
                       cv.height, cv.bits, row_ptr, col_ind, vin, col_word, vout, ws_count, ws_small, ws_big, gkeys);
}

template <int G, int E, int HB, typename ET>
hipError_t from_csr_g(const Conv& cv, const int* row_ptr, const int* col_ind, const void* val_in,
                      int* strip_ptr, uint32_t* col_word, void* val_out, void* workspace, hipStream_t stream) {
    constexpr int NG = kWave / G;
    const int waves = (cv.strips + NG - 1) / NG;
    const int blocks = (waves + kConvWaves - 1) / kConvWaves;
    const auto* vin = static_cast<const ET*>(val_in);
    auto* vout = static_cast<ET*>(val_out);
    const FromCsrWorkspaceLayout L = from_csr_workspace_layout(cv.rows, cv.nnz, cv.height);
    auto* ws = static_cast<char*>(workspace);
    int* ws_count = reinterpret_cast<int*>(ws);
    int* ws_small = reinterpret_cast<int*>(ws + L.small_off);
    int* ws_big = reinterpret_cast<int*>(ws + L.big_off);
    auto* gkeys = reinterpret_cast<uint64_t*>(ws + L.global_off);
    hipLaunchKernelGGL(set_ints_kernel, dim3(1), dim3(64), 0, stream, ws_count, 4, 0);
    hipLaunchKernelGGL((from_csr_group_kernel<HB, G, E, ET>), dim3(blocks), dim3(kConvThreads), 0, stream,
                       cv.rows, cv.strips, cv.height, cv.bits, cv.nnz, row_ptr, col_ind, vin, strip_ptr, col_word,
                       vout, ws_count, ws_small, ws_big);
    launch_sort_lists<HB, ET>(cv, L, row_ptr, col_ind, vin, col_word, vout, ws_count, ws_small, ws_big, gkeys,
                              stream);
    return hipGetLastError();
}

// Tall strips: the bucket kernel (one wave per strip of up to kWaveSortCap
// entries), then the same list kernel for longer strips.
template <int HB, typename ET>
hipError_t from_csr_bucket(const Conv& cv, const int* row_ptr, const int* col_ind, const void* val_in,
                           int* strip_ptr, uint32_t* col_word, void* val_out, void* workspace, hipStream_t stream) {
    constexpr int E = kWaveSortCap / kWave;
    const int blocks = (cv.strips + kConvWaves - 1) / kConvWaves;
    const auto* vin = static_cast<const ET*>(val_in);
    auto* vout = static_cast<ET*>(val_out);
    const FromCsrWorkspaceLayout L = from_csr_workspace_layout(cv.rows, cv.nnz, cv.height);
    auto* ws = static_cast<char*>(workspace);
    int* ws_count = reinterpret_cast<int*>(ws);
    int* ws_small = reinterpret_cast<int*>(ws + L.small_off);
    int* ws_big = reinterpret_cast<int*>(ws + L.big_off);
    auto* gkeys = reinterpret_cast<uint64_t*>(ws + L.global_off);
    hipLaunchKernelGGL(set_ints_kernel, dim3(1), dim3(64), 0, stream, ws_count, 4, 0);
    hipLaunchKernelGGL((from_csr_bucket_kernel<HB, E, ET>), dim3(blocks), dim3(kConvThreads), 0, stream, cv.rows,
                       cv.strips, cv.height, cv.bits, cv.nnz, row_ptr, col_ind, vin, strip_ptr, col_word, vout,
                       ws_count, ws_small, ws_big);
    launch_sort_lists<HB, ET>(cv, L, row_ptr, col_ind, vin, col_word, vout, ws_count, ws_small, ws_big, gkeys,
                              stream);
    return hipGetLastError();
}

template <int HB, typename ET>
hipError_t from_csr_hb(const Conv& cv, const int* row_ptr, const int* col_ind, const void* val_in,
                       int* strip_ptr, uint32_t* col_word, void* val_out, void* workspace, hipStream_t stream) {
    if constexpr (HB >= kBucketMinHeight) {
        if (static_cast<double>(cv.nnz) >= kBucketMinMean * static_cast<double>(cv.strips))
            return from_csr_bucket<HB, ET>(cv, row_ptr, col_ind, val_in, strip_ptr, col_word, val_out, workspace,
                                           stream);
    }
    const ConvShape sh = conv_shape(cv.nnz, cv.strips, HB);
#define CMRS_FROM_G(GG, EE)                                                                                      \
    if constexpr (GG >= HB) {                                                                                    \
        if (sh.g == GG && sh.e == EE)                                                                            \
            return from_csr_g<GG, EE, HB, ET>(cv, row_ptr, col_ind, val_in, strip_ptr, col_word, val_out, \
                                              workspace, stream);                                                \
    }
    CMRS_FROM_G(2, 8)
    CMRS_FROM_G(4, 8)
    CMRS_FROM_G(8, 8)
    CMRS_FROM_G(16, 8)
    CMRS_FROM_G(32, 8)
    CMRS_FROM_G(64, 8)
#undef CMRS_FROM_G
    return hipErrorInvalidValue;
}

template <typename ET>
hipError_t from_csr_typed(const Conv& cv, uint32_t flags, const int* row_ptr, const int* col_ind,
                          const void* val_in, int* strip_ptr, uint32_t* col_word, void* val_out, void* workspace,
                          hipStream_t stream) {
    if (!(flags & CMRS_SORT)) {
        const int ns = kRunRows / cv.height;
        const int waves = (cv.strips + ns - 1) / ns;
        const int blocks = (waves + kConvWaves - 1) / kConvWaves;
        hipLaunchKernelGGL((from_csr_rows_kernel<ET>), dim3(blocks), dim3(kConvThreads), 0, stream, cv.rows,
                           cv.strips, cv.height, cv.bits, cv.nnz, ns, row_ptr, col_ind, static_cast<const ET*>(val_in),
                           strip_ptr, col_word, static_cast<ET*>(val_out), val_out != val_in ? 1 : 0);
        return hipGetLastError();
    }
    switch (next_pow2(cv.height)) {
        case 1: return from_csr_hb<1, ET>(cv, row_ptr, col_ind, val_in, strip_ptr, col_word, val_out, workspace, stream);
        case 2: return from_csr_hb<2, ET>(cv, row_ptr, col_ind, val_in, strip_ptr, col_word, val_out, workspace, stream);
        case 4: return from_csr_hb<4, ET>(cv, row_ptr, col_ind, val_in, strip_ptr, col_word, val_out, workspace, stream);
        case 8: return from_csr_hb<8, ET>(cv, row_ptr, col_ind, val_in, strip_ptr, col_word, val_out, workspace, stream);
        case 16: return from_csr_hb<16, ET>(cv, row_ptr, col_ind, val_in, strip_ptr, col_word, val_out, workspace, stream);
        default: return from_csr_hb<32, ET>(cv, row_ptr, col_ind, val_in, strip_ptr, col_word, val_out, workspace, stream);
    }
}

template <typename ET>
hipError_t to_csr_typed(const cmrs_mat_t* A, int* row_ptr, int* col_ind, void* val_out, hipStream_t stream) {
    if (A->height == 1) {
        const int64_t work = static_cast<int64_t>(A->nnz > A->rows + 1 ? A->nnz : A->rows + 1);
        const int64_t want = (work + 1023) / 1024;
        const int blocks = static_cast<int>(want < 4096 ? want : 4096);
        hipLaunchKernelGGL((to_csr_h1_kernel<ET>), dim3(blocks), dim3(256), 0, stream, A->rows, A->nnz, A->bits,
                           A->strip_ptr, A->col_word, static_cast<const ET*>(A->val), row_ptr, col_ind,
                           static_cast<ET*>(val_out));
        return hipGetLastError();
    }
    const int strips = (A->rows + A->height - 1) / A->height;
    // Whole strips per wave: as many as fit in kRunRows rows (height <= 32).
    const int ns = kRunRows / A->height;
    const int runs = (strips + ns - 1) / ns;
    const int blocks = (runs + kToCsrWaves - 1) / kToCsrWaves;
    // Staged output from height 8 on, for runs of at least kToCsrStage/2.5
    // entries on average (measured: 2^20 rows of Poisson(16), height 32: 160
    // -> 107 us; height 2 and the skewed rows of up to 10^4 entries are faster
    // without).
    const bool stage = A->height >= 8 && static_cast<double>(A->nnz) >= kToCsrStage / 2.5 * runs;
    auto kern = stage ? to_csr_rows_kernel<ET, true> : to_csr_rows_kernel<ET, false>;
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(kToCsrThreads), 0, stream, A->rows, strips,
                       A->height, A->bits, ns, A->strip_ptr, A->col_word, static_cast<const ET*>(A->val), row_ptr,
                       col_ind, static_cast<ET*>(val_out));
    return hipGetLastError();
}

}  // namespace

FromCsrWorkspaceLayout from_csr_workspace_layout(int32_t rows, int32_t nnz, int32_t height) {
    FromCsrWorkspaceLayout L;
    const size_t strips = height > 0 ? (static_cast<size_t>(rows) + height - 1) / height : 0;
    L.small_off = 256;
    L.small_cap = strips > 0 ? strips : 1;
    L.big_off = align256(L.small_off + 4 * L.small_cap);
    L.big_cap = static_cast<size_t>(nnz) / (kWaveSortCap + 1) + 1;
    L.global_off = align256(L.big_off + 4 * L.big_cap);
    L.total = L.global_off + 16 * static_cast<size_t>(nnz);
    return L;
}

hipError_t launch_from_csr(int32_t rows, int32_t cols, int32_t nnz, const int32_t* row_ptr, const int32_t* col_ind,
                           const void* val_in, cmrs_dtype_t dtype, int32_t height, int32_t bits, uint32_t flags,
                           int32_t* strip_ptr, uint32_t* col_word, void* val_out, void* workspace,
                           hipStream_t stream) {
    (void)cols;
    const int strips = (rows + height - 1) / height;
    if (strips == 0) {
        hipLaunchKernelGGL(set_ints_kernel, dim3(1), dim3(64), 0, stream, strip_ptr, 1, nnz);
        return hipGetLastError();
    }
    const Conv cv{rows, strips, height, bits, nnz};
    // No entries: nothing to pack or sort (and the sorted path's workspace is
    // then zero bytes); the group kernel only writes the strip pointers.
    if (nnz == 0) flags &= ~CMRS_SORT;
    switch (dtype_bytes(dtype)) {
        case 8: return from_csr_typed<uint64_t>(cv, flags, row_ptr, col_ind, val_in, strip_ptr, col_word, val_out, workspace, stream);
        case 4: return from_csr_typed<uint32_t>(cv, flags, row_ptr, col_ind, val_in, strip_ptr, col_word, val_out, workspace, stream);
        default: return from_csr_typed<uint16_t>(cv, flags, row_ptr, col_ind, val_in, strip_ptr, col_word, val_out, workspace, stream);
    }
}

hipError_t launch_to_csr(const cmrs_mat_t* A, int32_t* row_ptr, int32_t* col_ind, void* val_out,
                         hipStream_t stream) {
    if (A->rows == 0) {
        hipLaunchKernelGGL(set_ints_kernel, dim3(1), dim3(64), 0, stream, row_ptr, 1, 0);
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
    hipLaunchKernelGGL(set_ints_kernel, dim3(1), dim3(64), 0, stream, flag, 1, 0);
    int work = rows > nnz ? rows : nnz;
    int g = (work + 255) / 256;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(validate_csr_kernel, dim3(g), dim3(256), 0, stream, rows, cols, nnz, row_ptr, col_ind, flag);
    return hipGetLastError();
}

}  // namespace cmrs
