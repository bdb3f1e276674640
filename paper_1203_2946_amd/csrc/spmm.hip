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
// spreads the reads of one instruction over distinct banks too.  From 3
// right-hand sides on (and for every bucket of the batched kernel) the steps
// are software-pipelined: each step issues the next step's stream loads
// before adding its own products (spmm_tile).  Where a row piece spans two or
// four 16-byte chunks, groups of adjacent lanes share their entries and each
// lane gathers one chunk of every piece of its group (chunk lanes, below);
// for one or two right-hand sides a lane takes its entries in runs of four
// consecutive ones, read as vectors (BlkStream).
//
// The batched path runs that body from one persistent kernel: waves take
// work tiles (a matrix and a range of its strips) from per-XCD queue counters
// in the plan until every queue is empty; the last wave out resets the
// counters, so the same plan can be launched again and replayed from a HIP
// graph.  A grid stride over strip passes (the listing's loop over strips in
// the paper's appendix) is the special case of one tile per wave.
#include <string.h>

#include <algorithm>
#include <type_traits>
#include <vector>

#include "cmrs_device.hpp"
#include "cmrs_ext.hpp"

namespace cmrs {

constexpr int kSpmmMaxWaves = 4;
constexpr size_t kSpmmWaveLdsMax = 65536;
constexpr int kSpmmMaxPassesPerWave = 8;

template <typename T>
__device__ inline T nt_load(const T* p) {
    return __builtin_nontemporal_load(p);
}
__device__ inline bf16_t nt_load(const bf16_t* p) {
    bf16_t v;
    v.bits = __builtin_nontemporal_load(&p->bits);
    return v;
}

template <int RB>
struct SpmmUnroll {
    static constexpr int U = RB >= 4 ? 4 : 8;  // entries per lane in one step
};

// Chunk lanes (below) for a matrix: log2 of the lanes per group, or 0.  Used
// alike on the host (LDS sizes) and in the kernels (which path runs).  xv:
// X values per 16 bytes; a group needs at least two chunks per row piece, a
// group width of at least C lanes and a whole vector of entries in the
// matrix; bf16 values (2-byte aligned) stay on single loads.
__host__ __device__ inline int spmm_chunk_log(const SpmmMat& m, int xv, bool bf16) {
    const int rb = 1 << m.rb_log;
    if (bf16 || rb < 2 * xv) return 0;
    const int cl = rb >= 4 * xv ? 2 : 1;
    return m.g_log >= cl && m.nnz >= (1 << cl) ? cl : 0;
}

// Partial slots per lane: HB * RB, or HB * XV with chunk lanes in fp64 (a
// lane keeps the slots of its own chunk only: a quarter or half of the LDS,
// so more waves fit; fp32 chunk lanes keep the full layout, measured faster
// there).
__host__ __device__ inline int spmm_lane_slots(const SpmmMat& m, int xv, bool bf16) {
    return m.hb * (xv == 2 && spmm_chunk_log(m, xv, bf16) > 0 ? xv : (1 << m.rb_log));
}

// The stream loads of one step of a lane: the packed words and values of
// entries base, base + G, ..., base + (U - 1) G of its strip.  Entries past
// the strip's end are clamped to its last entry, and a lane with no entry at
// all (past its strip's end, or without a strip) to entry 0, so that every
// lane loads a valid address with no branch: the compiler then keeps these
// loads in flight across the gathers and additions that follow them.  Called
// only for matrices with entries (so entry 0 exists).
template <int U, typename VT>
__device__ inline void spmm_load_step(const SpmmMat& m, int base, int G, int hi, uint32_t (&w)[U], VT (&v)[U]) {
    const VT* __restrict__ val = static_cast<const VT*>(m.val);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int j = max(min(base + u * G, hi - 1), 0);
        w[u] = nt_load(m.word + j);
        v[u] = nt_load(val + j);
    }
}

// The row pieces x[col][0 .. RB) of the step's U entries, in straight-line
// code: the first NV 16-byte chunks of each piece as vector loads (the caller
// picks NV so that they lie below nrhs on 16-byte aligned rows), the rest one
// value at a time at index min(k, nrhs - 1), a valid address whose value is
// not used for k >= nrhs.  Entries past the strip's end gather their clamped
// entry's row and are not added.  With no branch between them, the loads of
// all U entries are in flight together (a branch per entry made the compiler
// wait for each entry's gathers before issuing the next ones).
// 16 bytes of X: XV consecutive values of one row, at an element boundary
// (dword alignment is all the load needs).
template <typename XT>
struct XLoose;
template <>
struct XLoose<double> {
    typedef double type __attribute__((ext_vector_type(2), aligned(8)));
};
template <>
struct XLoose<float> {
    typedef float type __attribute__((ext_vector_type(4), aligned(4)));
};

template <int U, int RB, int NV, typename XT>
__device__ inline void spmm_gather(const SpmmMat& m, const uint32_t (&w)[U], XT (&xv)[U][RB]) {
    constexpr int XV = static_cast<int>(16 / sizeof(XT));
    const XT* __restrict__ x = static_cast<const XT*>(m.x);
    const size_t ldx = static_cast<size_t>(m.ldx);
    const int last = m.nrhs - 1;
    if constexpr (NV < 0) {
        // nrhs between RB/2 and RB, nrhs >= XV: every chunk as one 16-byte
        // load; the chunks below RB/2 lie below nrhs, the others are moved
        // back to end at nrhs (overlapping the chunk before), and slot k takes
        // element k - start of its chunk (slots k >= nrhs take any element:
        // their products are never read).  For 5-7 right-hand sides that is
        // 4 loads per entry in fp64 and 2 in fp32, against up to 8 single
        // loads.
        typedef typename XLoose<XT>::type XL;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const XT* xr = x + static_cast<size_t>(w[u] >> m.bits) * ldx;
#pragma unroll
            for (int c = 0; c < RB / XV; ++c) {
                if (c * XV + XV <= RB / 2) {
                    const XL t = *reinterpret_cast<const XL*>(xr + c * XV);
#pragma unroll
                    for (int q = 0; q < XV; ++q) xv[u][c * XV + q] = t[q];
                } else {
                    const int st = min(c * XV, m.nrhs - XV);
                    const XL t = *reinterpret_cast<const XL*>(xr + st);
#pragma unroll
                    for (int q = 0; q < XV; ++q) {
                        const int p = min(c * XV + q - st, XV - 1);
                        XT vq = t[XV - 1];
#pragma unroll
                        for (int r = XV - 2; r >= 0; --r) vq = p == r ? t[r] : vq;
                        xv[u][c * XV + q] = vq;
                    }
                }
            }
        }
        return;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const XT* xr = x + static_cast<size_t>(w[u] >> m.bits) * ldx;
#pragma unroll
        for (int c = 0; c < NV; ++c) {
            const typename XLoose<XT>::type t = *reinterpret_cast<const typename XLoose<XT>::type*>(xr + c * XV);
#pragma unroll
            for (int q = 0; q < XV; ++q) xv[u][c * XV + q] = t[q];
        }
#pragma unroll
        for (int k = NV * XV; k < RB; ++k) xv[u][k] = xr[min(k, last)];
    }
}

// The step's products added to the lane's partials for (row, k), for every
// entry slot and all RB right-hand-side slots, with no branch: a clamped
// entry adds +0.0 (its product is replaced, so a non-finite x cannot leak
// in), and slots k >= nrhs collect products that are never read.  A partial
// starts at +0.0 and, in round-to-nearest, never becomes -0.0, so adding +0.0
// leaves it bit for bit unchanged.  (A branch here would let the compiler
// sink the gathers into it and then wait for every load in flight, the
// next step's prefetch included, before the first addition.)
template <int HB, int U, int RB, typename VT, typename XT, typename AT>
__device__ inline void spmm_accumulate(const SpmmMat& m, int base, int G, int hi, const uint32_t (&w)[U],
                                       const VT (&v)[U], const XT (&xv)[U][RB], AT* __restrict__ buf, int lane) {
    const uint32_t mask = (1u << m.bits) - 1u;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const bool ok = base + u * G < hi;
        const AT a = static_cast<AT>(ValTraits<VT>::widen(v[u]));
        AT* slot = buf + static_cast<int>(w[u] & mask & (HB - 1)) * RB * kWave + lane;
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            const AT p = a * static_cast<AT>(xv[u][k]);
            lds_add(slot + k * kWave, ok ? p : AT(0));
        }
    }
}

// Chunk lanes.  From two 16-byte chunks per row piece on (4 or 8 fp64
// right-hand-side slots, 8 fp32 ones), each group of C = 2^CL consecutive
// lanes (a pair or a quad) shares the work of its entries: lane c of the
// group gathers chunk c of every one of the group's row pieces and adds the
// products for its own XV slots c * XV .. c * XV + XV - 1.  A gather
// instruction then touches 64 / C row pieces, each read whole by C adjacent
// lanes, instead of 64 pieces read a chunk at a time (with X in L2, 64-byte
// pieces gathered that way ran ~1.45x faster in a probe).  The stream data
// are loaded C entries per lane as vectors (ChunkStream) and exchanged
// within the group with DPP quad permutations (no LDS).  Lane c keeps
// partials for the slots of chunk c only: in fp64 just those (HB * XV per
// lane, spmm_lane_slots), in fp32 within the full layout, the rest +0.0.

// The value of lane `src` of this lane's group of 2^CL lanes (CL = 1: pairs
// (0, 1), (2, 3) of each quad; CL = 2: the quad).  src must fold to a
// constant (the loops calling it are unrolled).
template <int CL>
__device__ inline int group_read(int v, int src) {
    static_assert(CL == 1 || CL == 2, "pairs or quads");
    // quad_perm selectors: [s, s, s, s] for a quad, [s, s, 2 + s, 2 + s] for pairs.
    if constexpr (CL == 2) {
        switch (src) {
            case 0: return __builtin_amdgcn_mov_dpp(v, 0x00, 0xf, 0xf, false);
            case 1: return __builtin_amdgcn_mov_dpp(v, 0x55, 0xf, 0xf, false);
            case 2: return __builtin_amdgcn_mov_dpp(v, 0xaa, 0xf, 0xf, false);
            default: return __builtin_amdgcn_mov_dpp(v, 0xff, 0xf, 0xf, false);
        }
    } else {
        return src == 0 ? __builtin_amdgcn_mov_dpp(v, 0xa0, 0xf, 0xf, false)
                        : __builtin_amdgcn_mov_dpp(v, 0xf5, 0xf, 0xf, false);
    }
}
template <int CL>
__device__ inline uint32_t group_read(uint32_t v, int src) {
    return static_cast<uint32_t>(group_read<CL>(static_cast<int>(v), src));
}
template <int CL>
__device__ inline float group_read(float v, int src) {
    return __int_as_float(group_read<CL>(__float_as_int(v), src));
}
template <int CL>
__device__ inline double group_read(double v, int src) {
    const long long b = __double_as_longlong(v);
    const uint32_t lo = group_read<CL>(static_cast<uint32_t>(b), src);
    const uint32_t hi = group_read<CL>(static_cast<uint32_t>(static_cast<unsigned long long>(b) >> 32), src);
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// C consecutive stream elements at their own alignment (a multi-dword load
// needs dword alignment only).
template <typename T, int C>
struct SVec;
template <int C>
struct SVec<uint32_t, C> {
    typedef uint32_t type __attribute__((ext_vector_type(C), aligned(4)));
};
template <int C>
struct SVec<double, C> {
    typedef double type __attribute__((ext_vector_type(C), aligned(8)));
};
template <int C>
struct SVec<float, C> {
    typedef float type __attribute__((ext_vector_type(C), aligned(4)));
};

// The stream data of one step of a chunk-lane group.  The group's entries at
// step offset u are the C consecutive entries g + u * G + j, j < C (g: the
// group's first entry slot); lane c loads those of the offsets u = k * C + c
// as one vector of words and one of values (the vector-memory address path
// costs about the same per lane whatever the width, so this is C times fewer
// addresses than a word and a value per lane and entry).  A vector that
// would reach past the last entry of the matrix is moved back to end there,
// d[k] places later than wanted; one wholly past its strip is moved to the
// strip's last entry.  Elements are then picked at min(j + d, C - 1): the
// wanted one for every entry inside the strip, a valid one otherwise.
template <int U, int CL, typename VT>
struct ChunkStream {
    static constexpr int C = 1 << CL;
    static constexpr int NV = U >> CL;
    typename SVec<uint32_t, C>::type w[NV];
    typename SVec<VT, C>::type v[NV];
    int d[NV];
};

template <int U, int CL, typename VT>
__device__ inline void spmm_load_chunk(const SpmmMat& m, int g, int G, int hi, int c, ChunkStream<U, CL, VT>& t) {
    typedef ChunkStream<U, CL, VT> CS;
    typedef typename SVec<uint32_t, CS::C>::type WV;
    typedef typename SVec<VT, CS::C>::type VV;
    const VT* __restrict__ val = static_cast<const VT*>(m.val);
#pragma unroll
    for (int k = 0; k < CS::NV; ++k) {
        const int j = g + (k * CS::C + c) * G;
        const int jv = max(min(min(j, hi - 1), m.nnz - CS::C), 0);
        t.d[k] = j - jv;
        t.w[k] = __builtin_nontemporal_load(reinterpret_cast<const WV*>(m.word + jv));
        t.v[k] = __builtin_nontemporal_load(reinterpret_cast<const VV*>(val + jv));
    }
}

// Element j of this lane's vector k, placed as described above.
template <int C, typename V>
__device__ inline auto chunk_pick(const V& vec, int d, int j) -> decltype(vec[0] + vec[0]) {
    const int p = min(j + d, C - 1);
    auto r = vec[C - 1];
#pragma unroll
    for (int q = C - 2; q >= 0; --q) r = p == q ? vec[q] : r;
    return r;
}

// The word of the group's entry (u, j), read from the lane that loaded it.
template <int U, int CL, typename VT>
__device__ inline uint32_t chunk_word(const ChunkStream<U, CL, VT>& t, int u, int j) {
    constexpr int C = 1 << CL;
    return group_read<CL>(chunk_pick<C>(t.w[u >> CL], t.d[u >> CL], j), u & (C - 1));
}

// Stream data of one or two right-hand sides, blocked: lane e of a strip
// takes runs of V = 4 consecutive entries, lo + V e + k V G + i (i < V), and
// loads each run as one vector of words and one of values (a quarter of the
// addresses of one entry per load; the vector-memory address path costs
// about the same per lane whatever the width).  Runs are moved back from
// past the matrix's last entry or to the strip's last entry as in
// ChunkStream; element i is picked at min(i + d, V - 1).  Only matrices of
// at least V entries take this path; bf16 values (2-byte aligned) do not.
constexpr int kBlk = 4;

template <int U, typename VT>
struct BlkStream {
    static constexpr int NV = U / kBlk;
    typename SVec<uint32_t, kBlk>::type w[NV];
    typename SVec<VT, kBlk>::type v[NV];
    int d[NV];
    __device__ uint32_t word(int u) const { return chunk_pick<kBlk>(w[u / kBlk], d[u / kBlk], u % kBlk); }
    __device__ VT value(int u) const { return chunk_pick<kBlk>(v[u / kBlk], d[u / kBlk], u % kBlk); }
};

// Entry u of a lane's step starting at base (base = lo + V e + step U G).
__device__ inline int blk_entry(int base, int G, int u) {
    return base + (u / kBlk) * kBlk * G + u % kBlk;
}

template <int U, typename VT>
__device__ inline void spmm_load_blk(const SpmmMat& m, int base, int G, int hi, BlkStream<U, VT>& t) {
    typedef typename SVec<uint32_t, kBlk>::type WV;
    typedef typename SVec<VT, kBlk>::type VV;
    const VT* __restrict__ val = static_cast<const VT*>(m.val);
#pragma unroll
    for (int k = 0; k < BlkStream<U, VT>::NV; ++k) {
        const int j = base + k * kBlk * G;
        const int jv = max(min(min(j, hi - 1), m.nnz - kBlk), 0);
        t.d[k] = j - jv;
        t.w[k] = __builtin_nontemporal_load(reinterpret_cast<const WV*>(m.word + jv));
        t.v[k] = __builtin_nontemporal_load(reinterpret_cast<const VV*>(val + jv));
    }
}

template <typename VT>
__host__ __device__ constexpr bool spmm_blk_type() {
    return !std::is_same<VT, bf16_t>::value;
}

// Chunk c of the row pieces of the group's U * C entries: one 16-byte load
// each, elements st .. st + XV - 1 with st = c * XV, moved back to st = nrhs
// - XV when the chunk would reach past nrhs.  Entries past their strip's end
// gather the piece of a valid word.  Only the loads are issued here; the
// chunks are used after the next step's stream loads are on their way.
template <int U, int CL, typename VT, typename XT>
__device__ inline void spmm_gather_chunk(const SpmmMat& m, const ChunkStream<U, CL, VT>& t, int st,
                                         XT (&xc)[U << CL][16 / sizeof(XT)]) {
    constexpr int C = 1 << CL;
    constexpr int XV = static_cast<int>(16 / sizeof(XT));
    typedef typename XLoose<XT>::type XL;
    const XT* __restrict__ x = static_cast<const XT*>(m.x) + st;
    const size_t ldx = static_cast<size_t>(m.ldx);
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int j = 0; j < C; ++j) {
            const uint32_t wj = chunk_word<U, CL, VT>(t, u, j);
            const XL v = *reinterpret_cast<const XL*>(x + static_cast<size_t>(wj >> m.bits) * ldx);
#pragma unroll
            for (int q = 0; q < XV; ++q) xc[u * C + j][q] = v[q];
        }
    }
}

// The products of the group's U * C entries with this lane's chunk, added to
// the lane's own partials, with no branch (entries past their strip's end add
// +0.0, as in spmm_accumulate).  Entry (u, j) is entry g + u * G + j of the
// strip.  fp64: a lane keeps the XV slots of its chunk only, partial (row, q)
// at [row * XV + q][lane] for right-hand side c * XV + q; a chunk moved back
// by sh = c * XV - st elements holds right-hand side c * XV + q in element q
// + sh, and its first sh elements (chunk c - 1's) add +0.0 to slot 0.  fp32:
// the full layout [row * RB + k][lane], element q going to k = st + q; the
// slots below c * XV that a moved-back chunk adds to are chunk c - 1's, never
// read from this lane's column (the row sums of slot k read the lanes of
// chunk k / XV only) and cleared with the rest.
template <int HB, int U, int RB, int CL, typename VT, typename XT, typename AT>
__device__ inline void spmm_accumulate_chunk(const SpmmMat& m, int g, int G, int hi, int c, int st,
                                             const ChunkStream<U, CL, VT>& t,
                                             const XT (&xc)[U << CL][16 / sizeof(XT)], AT* __restrict__ buf,
                                             int lane) {
    constexpr int C = 1 << CL;
    constexpr int XV = static_cast<int>(16 / sizeof(XT));
    constexpr bool COMPACT = sizeof(AT) == 8;
    const uint32_t mask = (1u << m.bits) - 1u;
    const int sh = c * XV - st;
    AT* mine = COMPACT ? buf + lane : buf + st * kWave + lane;
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int j = 0; j < C; ++j) {
            const bool ok = g + u * G + j < hi;
            const uint32_t wj = chunk_word<U, CL, VT>(t, u, j);
            const AT aj = group_read<CL>(static_cast<AT>(chunk_pick<C>(t.v[u >> CL], t.d[u >> CL], j)), u & (C - 1));
            AT* slot = mine + static_cast<int>(wj & mask & (HB - 1)) * (COMPACT ? XV : RB) * kWave;
#pragma unroll
            for (int q = 0; q < XV; ++q) {
                const AT p = aj * static_cast<AT>(xc[u * C + j][q]);
                if constexpr (COMPACT)
                    lds_add(slot + max(q - sh, 0) * kWave, ok && q >= sh ? p : AT(0));
                else
                    lds_add(slot + q * kWave, ok ? p : AT(0));
            }
        }
    }
}

// Row sums of the pass over strips [sb, sb + S) (those below s_end), written
// to Y, and the partials cleared for the next pass.  Output o: strip slot
// so = o mod S (fastest), partial i = o / S with i = row * RB + k; it sums
// the G entry slots starting at slot i mod G.
template <int HB, int RB, typename XT, typename AT>
__device__ inline void spmm_finish(const SpmmMat& m, int sb, int s_end, AT* __restrict__ buf, int lane) {
    constexpr int SLOTS = HB * RB;
    const int g_log = m.g_log;
    const int G = 1 << g_log;
    const int s_log = 6 - g_log;
    const int nout = SLOTS << s_log;
    XT* __restrict__ y = static_cast<XT*>(m.y);
    const size_t ldy = static_cast<size_t>(m.ldy);
    wave_lds_sync();
    for (int o = lane; o < nout; o += kWave) {
        const int so = o & ((1 << s_log) - 1);
        const int i = o >> s_log;
        const int k = i & (RB - 1);
        const int rr = i / RB;
        const AT* p = buf + i * kWave + (so << g_log);
        AT sum = AT(0);
        // Eight reads in flight at a time, added in the same order.
        int q = 0;
        for (; q + 8 <= G; q += 8) {
            AT t[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) t[j] = p[(q + j + i) & (G - 1)];
#pragma unroll
            for (int j = 0; j < 8; ++j) sum += t[j];
        }
        for (; q < G; ++q) sum += p[(q + i) & (G - 1)];
        const int strip = sb + so;
        const long long row = static_cast<long long>(strip) * m.height + rr;
        if (strip < s_end && rr < m.height && row < m.rows && k < m.nrhs)
            y[static_cast<size_t>(row) * ldy + k] = static_cast<XT>(sum);
    }
    wave_lds_sync();
#pragma unroll
    for (int i = 0; i < SLOTS; ++i) buf[i * kWave + lane] = AT(0);
}

// spmm_finish for chunk lanes: output (row, k) sums the G / C lanes of chunk
// k / XV (entry slot e = e' * C + k / XV), partial [row * XV + k mod XV] in
// fp64 ([row * RB + k] in fp32), starting at the (i mod G/C)-th; the
// partials are cleared.
template <int HB, int RB, typename XT, typename AT, int CL>
__device__ inline void spmm_finish_chunk(const SpmmMat& m, int sb, int s_end, AT* __restrict__ buf, int lane) {
    constexpr int XV = static_cast<int>(16 / sizeof(XT));
    constexpr bool COMPACT = sizeof(AT) == 8;
    constexpr int SLOTS = HB * RB;
    const int g_log = m.g_log;
    const int G = 1 << (g_log - CL);
    const int s_log = 6 - g_log;
    const int nout = SLOTS << s_log;
    XT* __restrict__ y = static_cast<XT*>(m.y);
    const size_t ldy = static_cast<size_t>(m.ldy);
    wave_lds_sync();
    for (int o = lane; o < nout; o += kWave) {
        const int so = o & ((1 << s_log) - 1);
        const int i = o >> s_log;
        const int k = i & (RB - 1);
        const int rr = i / RB;
        const AT* p = buf + (COMPACT ? rr * XV + k % XV : i) * kWave + (so << g_log) + k / XV;
        AT sum = AT(0);
        int q = 0;
        for (; q + 8 <= G; q += 8) {
            AT t[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) t[j] = p[((q + j + i) & (G - 1)) << CL];
#pragma unroll
            for (int j = 0; j < 8; ++j) sum += t[j];
        }
        for (; q < G; ++q) sum += p[((q + i) & (G - 1)) << CL];
        const int strip = sb + so;
        const long long row = static_cast<long long>(strip) * m.height + rr;
        if (strip < s_end && rr < m.height && row < m.rows && k < m.nrhs)
            y[static_cast<size_t>(row) * ldy + k] = static_cast<XT>(sum);
    }
    wave_lds_sync();
#pragma unroll
    for (int i = 0; i < HB * (COMPACT ? XV : RB); ++i) buf[i * kWave + lane] = AT(0);
}

// Strips [s0, s1) of matrix m in passes of S = 64 / G strips; buf holds the
// HB * RB * 64 partials of this wave.  Lane (s, e) walks entries e, e + G, ...
// of its strip, U per step.  The loads are software-pipelined: a step first
// gathers its X pieces, then issues the stream loads of the next step (of
// this pass, or the first of the next pass, whose strip pointers were read one
// pass ahead), and only then adds its products, so the next step's HBM
// latency overlaps this step's gathers, additions and the pass-end reduction.
// Every load of the step is issued by every lane at a valid address (clamped
// entries and strip indices), with no branch around it: at a branch the
// compiler would have to assume the worst of the loads still in flight and
// wait for the prefetch too.  The additions per lane and the reduction run in
// the same order as without the pipelining.  CL > 0: chunk lanes, groups of
// 2^CL lanes sharing their entries (the group width G is at least 2^CL); the
// stream loads are the same, a lane gathers and adds its chunk of the
// group's entries instead of its own entries' whole pieces.
template <int HB, int RB, int NV, typename VT, typename XT, typename AT>
__device__ inline void spmm_tile(const SpmmMat& m, int s0, int s1, AT* __restrict__ buf, int lane) {
    constexpr int U = SpmmUnroll<RB>::U;
    constexpr int SLOTS = HB * RB;
    const int g_log = m.g_log;
    const int G = 1 << g_log;
    const int S = kWave >> g_log;
    const int e = lane & (G - 1);
    const int32_t* __restrict__ sp = m.strip_ptr;
#pragma unroll
    for (int i = 0; i < SLOTS; ++i) buf[i * kWave + lane] = AT(0);
    if (m.nnz == 0) {
        // No entries to load: every row sum is zero.
        for (int sb = s0; sb < s1; sb += S) spmm_finish<HB, RB, XT, AT>(m, sb, s1, buf, lane);
        return;
    }
    // A lane whose strip is at or past s1 gets the empty range [sp[s1], sp[s1]).
    int s = s0 + (lane >> g_log);
    int lo = sp[min(s, s1)], hi = sp[min(s + 1, s1)];
    int lo_n = sp[min(s + S, s1)], hi_n = sp[min(s + S + 1, s1)];
    int base = lo + e;
    uint32_t w[U];
    VT v[U];
    spmm_load_step<U, VT>(m, base, G, hi, w, v);
    for (int sb = s0;;) {
        XT xv[U][RB];
        spmm_gather<U, RB, NV, XT>(m, w, xv);
        const int nb = base + U * G;
        const bool more = ballot(nb < hi) != 0ull;
        uint32_t w2[U];
        VT v2[U];
        spmm_load_step<U, VT>(m, more ? nb : lo_n + e, G, more ? hi : hi_n, w2, v2);
        spmm_accumulate<HB, U, RB, VT, XT, AT>(m, base, G, hi, w, v, xv, buf, lane);
        if (more) {
            base = nb;
        } else {
            spmm_finish<HB, RB, XT, AT>(m, sb, s1, buf, lane);
            sb += S;
            if (sb >= s1) break;
            s += S;
            lo = lo_n;
            hi = hi_n;
            base = lo + e;
            lo_n = sp[min(s + S, s1)];
            hi_n = sp[min(s + S + 1, s1)];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            w[u] = w2[u];
            v[u] = v2[u];
        }
    }
}

// spmm_tile with chunk lanes: groups of C = 2^CL lanes (G >= C) sharing their
// entries, the stream data loaded C entries per lane and vector
// (ChunkStream), each lane gathering and adding its chunk of the group's
// entries.  Same pipelining, with two scheduling barriers fixing the order of
// a step: the gathers, then the next step's stream loads, then the products
// (without the first the compiler issued one gather at a time; without the
// second it hoisted the multiplications above the stream loads, which then
// waited for every gather).  Lane (s, e) of group g = e - c: the group's
// entries of a step are g + u * G + j.
template <int HB, int RB, typename VT, typename XT, typename AT, int CL>
__device__ inline void spmm_tile_chunk(const SpmmMat& m, int s0, int s1, AT* __restrict__ buf, int lane) {
    constexpr int U = SpmmUnroll<RB>::U;
    constexpr int XV = static_cast<int>(16 / sizeof(XT));
    constexpr int C = 1 << CL;
    static_assert(U % C == 0, "whole vectors per lane");
    const int g_log = m.g_log;
    const int G = 1 << g_log;
    const int S = kWave >> g_log;
    const int e = lane & (G - 1);
    const int c = e & (C - 1);
    const int32_t* __restrict__ sp = m.strip_ptr;
#pragma unroll
    for (int i = 0; i < HB * (sizeof(AT) == 8 ? XV : RB); ++i) buf[i * kWave + lane] = AT(0);
    int s = s0 + (lane >> g_log);
    int lo = sp[min(s, s1)], hi = sp[min(s + 1, s1)];
    int lo_n = sp[min(s + S, s1)], hi_n = sp[min(s + S + 1, s1)];
    int base = lo + e;
    const int st = min(c * XV, m.nrhs - XV);
    ChunkStream<U, CL, VT> t;
    spmm_load_chunk<U, CL, VT>(m, base - c, G, hi, c, t);
    for (int sb = s0;;) {
        XT xv[U << CL][XV];
        spmm_gather_chunk<U, CL, VT, XT>(m, t, st, xv);
        __builtin_amdgcn_sched_barrier(0);
        const int nb = base + U * G;
        const bool more = ballot(nb < hi) != 0ull;
        ChunkStream<U, CL, VT> t2;
        spmm_load_chunk<U, CL, VT>(m, (more ? nb : lo_n + e) - c, G, more ? hi : hi_n, c, t2);
        __builtin_amdgcn_sched_barrier(0);
        spmm_accumulate_chunk<HB, U, RB, CL, VT, XT, AT>(m, base - c, G, hi, c, st, t, xv, buf, lane);
        if (more) {
            base = nb;
        } else {
            spmm_finish_chunk<HB, RB, XT, AT, CL>(m, sb, s1, buf, lane);
            sb += S;
            if (sb >= s1) break;
            s += S;
            lo = lo_n;
            hi = hi_n;
            base = lo + e;
            lo_n = sp[min(s + S, s1)];
            hi_n = sp[min(s + S + 1, s1)];
        }
        t = t2;
    }
}

// spmm_tile for one or two right-hand sides with blocked stream data
// (BlkStream): the same pipelined step, each lane's entries taken in runs of
// kBlk consecutive ones.  Sums the same products in the same order as
// spmm_pass_small_blk, the single-launch form.
template <int HB, int RB, typename VT, typename XT, typename AT>
__device__ inline void spmm_tile_blk(const SpmmMat& m, int s0, int s1, AT* __restrict__ buf, int lane) {
    constexpr int U = SpmmUnroll<RB>::U;
    constexpr int SLOTS = HB * RB;
    const int g_log = m.g_log;
    const int G = 1 << g_log;
    const int S = kWave >> g_log;
    const int e = lane & (G - 1);
    const uint32_t mask = (1u << m.bits) - 1u;
    const XT* __restrict__ x = static_cast<const XT*>(m.x);
    const size_t ldx = static_cast<size_t>(m.ldx);
    const int last = m.nrhs - 1;
    const int32_t* __restrict__ sp = m.strip_ptr;
#pragma unroll
    for (int i = 0; i < SLOTS; ++i) buf[i * kWave + lane] = AT(0);
    int s = s0 + (lane >> g_log);
    int lo = sp[min(s, s1)], hi = sp[min(s + 1, s1)];
    int lo_n = sp[min(s + S, s1)], hi_n = sp[min(s + S + 1, s1)];
    int base = lo + kBlk * e;
    BlkStream<U, VT> t;
    spmm_load_blk<U, VT>(m, base, G, hi, t);
    for (int sb = s0;;) {
        XT xv[U][RB];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const XT* xr = x + static_cast<size_t>(t.word(u) >> m.bits) * ldx;
#pragma unroll
            for (int k = 0; k < RB; ++k) xv[u][k] = xr[min(k, last)];
        }
        const int nb = base + U * G;
        const bool more = ballot(nb < hi) != 0ull;
        BlkStream<U, VT> t2;
        spmm_load_blk<U, VT>(m, more ? nb : lo_n + kBlk * e, G, more ? hi : hi_n, t2);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool ok = blk_entry(base, G, u) < hi;
            const uint32_t w = t.word(u);
            const AT a = static_cast<AT>(t.value(u));
            AT* slot = buf + static_cast<int>(w & mask & (HB - 1)) * RB * kWave + lane;
#pragma unroll
            for (int k = 0; k < RB; ++k) {
                const AT p = a * static_cast<AT>(xv[u][k]);
                lds_add(slot + k * kWave, ok ? p : AT(0));
            }
        }
        if (more) {
            base = nb;
        } else {
            spmm_finish<HB, RB, XT, AT>(m, sb, s1, buf, lane);
            sb += S;
            if (sb >= s1) break;
            s += S;
            lo = lo_n;
            hi = hi_n;
            base = lo + kBlk * e;
            lo_n = sp[min(s + S, s1)];
            hi_n = sp[min(s + S + 1, s1)];
        }
        t = t2;
    }
}

// One pass over strips [sb, sb + S) (those below s_end) for one or two
// right-hand sides, without the pipelining: a lane loads the words and values
// of its U entries, gathers and adds only those inside its strip (branches
// that skip the additions of entries past the end).  As a single launch with
// one pass per wave this is faster than the branch-free pipelined step, which
// adds +0.0 for every clamped entry (measured 11-16 % on 2*10^6-row band and
// stencil matrices).  It sums the same products in the same order.
template <int HB, int RB, typename VT, typename XT, typename AT>
__device__ inline void spmm_pass_small(const SpmmMat& m, int sb, int s_end, AT* __restrict__ buf, int lane) {
    static_assert(RB <= 2, "one or two right-hand-side slots");
    constexpr int U = SpmmUnroll<RB>::U;
    const int g_log = m.g_log;
    const int G = 1 << g_log;
    const int e = lane & (G - 1);
    const int s = sb + (lane >> g_log);
    const uint32_t mask = (1u << m.bits) - 1u;
    if (s < s_end) {
        const int lo = m.strip_ptr[s], hi = m.strip_ptr[s + 1];
        const VT* __restrict__ val = static_cast<const VT*>(m.val);
        const XT* __restrict__ x = static_cast<const XT*>(m.x);
        const size_t ldx = static_cast<size_t>(m.ldx);
        for (int base = lo + e; base < hi; base += U * G) {
            uint32_t w[U];
            VT v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = min(base + u * G, hi - 1);
                w[u] = nt_load(m.word + j);
                v[u] = nt_load(val + j);
            }
            XT xv[U][RB];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (base + u * G < hi) {
                    const XT* xr = x + static_cast<size_t>(w[u] >> m.bits) * ldx;
#pragma unroll
                    for (int k = 0; k < RB; ++k) xv[u][k] = xr[k];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (base + u * G < hi) {
                    const AT a = static_cast<AT>(ValTraits<VT>::widen(v[u]));
                    AT* slot = buf + static_cast<int>(w[u] & mask & (HB - 1)) * RB * kWave + lane;
#pragma unroll
                    for (int k = 0; k < RB; ++k) lds_add(slot + k * kWave, a * static_cast<AT>(xv[u][k]));
                }
            }
        }
    }
    spmm_finish<HB, RB, XT, AT>(m, sb, s_end, buf, lane);
}

// spmm_pass_small with blocked stream data (BlkStream): the products of the
// same entries, added in the same order as spmm_tile_blk.
template <int HB, int RB, typename VT, typename XT, typename AT>
__device__ inline void spmm_pass_small_blk(const SpmmMat& m, int sb, int s_end, AT* __restrict__ buf, int lane) {
    static_assert(RB <= 2, "one or two right-hand-side slots");
    constexpr int U = SpmmUnroll<RB>::U;
    const int g_log = m.g_log;
    const int G = 1 << g_log;
    const int e = lane & (G - 1);
    const int s = sb + (lane >> g_log);
    const uint32_t mask = (1u << m.bits) - 1u;
    if (s < s_end) {
        const int lo = m.strip_ptr[s], hi = m.strip_ptr[s + 1];
        const XT* __restrict__ x = static_cast<const XT*>(m.x);
        const size_t ldx = static_cast<size_t>(m.ldx);
        for (int base = lo + kBlk * e; base < hi; base += U * G) {
            BlkStream<U, VT> t;
            spmm_load_blk<U, VT>(m, base, G, hi, t);
            XT xv[U][RB];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (blk_entry(base, G, u) < hi) {
                    const XT* xr = x + static_cast<size_t>(t.word(u) >> m.bits) * ldx;
#pragma unroll
                    for (int k = 0; k < RB; ++k) xv[u][k] = xr[k];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (blk_entry(base, G, u) < hi) {
                    const AT a = static_cast<AT>(t.value(u));
                    AT* slot = buf + static_cast<int>(t.word(u) & mask & (HB - 1)) * RB * kWave + lane;
#pragma unroll
                    for (int k = 0; k < RB; ++k) lds_add(slot + k * kWave, a * static_cast<AT>(xv[u][k]));
                }
            }
        }
    }
    spmm_finish<HB, RB, XT, AT>(m, sb, s_end, buf, lane);
}

// How many 16-byte chunks of each X piece are read as vector loads: all of
// them (those reaching past nrhs moved back to end at nrhs, NV = -1, when
// nrhs does not fill the bucket; at least one chunk's worth of right-hand
// sides needed).  The loads need the elements' own alignment only (dword
// alignment is what a 16-byte global load requires), so any leading
// dimension takes them: with rows of 5 or 7 doubles (or 3, 5, 6, 7 floats) a
// piece costs 4 (2) loads instead of 6 (5).  fp64 pieces of fewer than 4
// slots are read one value at a time (measured faster there).
// Buckets whose partials exceed a wave's LDS share are never planned
// (spmm_fits) and not compiled.
template <int HB, int RB, typename VT, typename XT, typename AT>
__device__ inline void spmm_tile_nv(const SpmmMat& m, int s0, int s1, AT* buf, int lane) {
    constexpr int XV = static_cast<int>(16 / sizeof(XT));
    constexpr bool VEC = RB >= XV && !(sizeof(XT) == 8 && RB < 4);
    if constexpr (static_cast<size_t>(HB) * RB * kWave * sizeof(AT) > kSpmmWaveLdsMax) {
        return;
    } else if constexpr (!VEC) {
        if constexpr (RB <= 2 && spmm_blk_type<VT>()) {
            if (m.nnz >= kBlk) {
                spmm_tile_blk<HB, RB, VT, XT, AT>(m, s0, s1, buf, lane);
                return;
            }
        }
        spmm_tile<HB, RB, 0, VT, XT, AT>(m, s0, s1, buf, lane);
    } else if constexpr (RB / XV >= 2 && !std::is_same<VT, bf16_t>::value) {
        // Chunk lanes when the group has room for them and the matrix holds a
        // whole vector of entries (nrhs > RB / 2 >= XV here, so every chunk is
        // one 16-byte load; bf16 values, 2-byte aligned, stay on single loads).
        constexpr int CL = RB / XV >= 4 ? 2 : 1;
        if (spmm_chunk_log(m, XV, false) == CL) {
            spmm_tile_chunk<HB, RB, VT, XT, AT, CL>(m, s0, s1, buf, lane);
        } else if (m.nrhs == RB) {
            spmm_tile<HB, RB, RB / XV, VT, XT, AT>(m, s0, s1, buf, lane);
        } else {
            spmm_tile<HB, RB, -1, VT, XT, AT>(m, s0, s1, buf, lane);
        }
    } else {
        if (m.nrhs == RB)
            spmm_tile<HB, RB, RB / XV, VT, XT, AT>(m, s0, s1, buf, lane);
        else if (m.nrhs >= XV)
            spmm_tile<HB, RB, -1, VT, XT, AT>(m, s0, s1, buf, lane);
        else
            spmm_tile<HB, RB, 0, VT, XT, AT>(m, s0, s1, buf, lane);
    }
}

// One launch over one matrix: wave w takes the `passes` consecutive passes
// of strips [w * passes * S, (w + 1) * passes * S), so the next pass's loads
// overlap the current one's work as in the batched kernel.  One or two
// right-hand sides: one pass per wave through spmm_pass_small, measured
// faster there as a single launch (the batched kernel runs those buckets
// through the pipelined loop too, where that was faster).
template <int HB, int RB, typename VT, typename XT, typename AT>
__global__ __launch_bounds__(kSpmmMaxWaves * kWave) void spmm_kernel(SpmmMat m, int strips, int passes) {
    extern __shared__ __align__(16) unsigned char spmm_lds[];
    AT* buf = reinterpret_cast<AT*>(spmm_lds);
    const int lane = lane_id();
    const int wpb = static_cast<int>(blockDim.x) / kWave;
    const int wave = uniform(static_cast<int>(threadIdx.x) / kWave);
    const long long span = static_cast<long long>(passes) << (6 - m.g_log);
    const long long sb = (static_cast<long long>(xcd_logical_block(blockIdx.x, gridDim.x)) * wpb + wave) * span;
    if (sb >= strips) return;
    const int s1 = static_cast<int>(std::min<long long>(strips, sb + span));
    buf += wave * (spmm_lane_slots(m, static_cast<int>(16 / sizeof(XT)), std::is_same<VT, bf16_t>::value) * kWave);
    if constexpr (RB <= 2) {
        // One pass per wave (passes == 1), no pipelining.
#pragma unroll
        for (int i = 0; i < HB * RB; ++i) buf[i * kWave + lane] = AT(0);
        if constexpr (spmm_blk_type<VT>()) {
            if (m.nnz >= kBlk) {
                spmm_pass_small_blk<HB, RB, VT, XT, AT>(m, static_cast<int>(sb), s1, buf, lane);
                return;
            }
        }
        spmm_pass_small<HB, RB, VT, XT, AT>(m, static_cast<int>(sb), s1, buf, lane);
    } else {
        spmm_tile_nv<HB, RB, VT, XT, AT>(m, static_cast<int>(sb), s1, buf, lane);
    }
}

template <int HB, typename VT, typename XT, typename AT>
__device__ inline void spmm_tile_rb(const SpmmMat& m, int s0, int s1, AT* buf, int lane) {
    switch (m.rb_log) {
        case 0: spmm_tile_nv<HB, 1, VT, XT, AT>(m, s0, s1, buf, lane); break;
        case 1: spmm_tile_nv<HB, 2, VT, XT, AT>(m, s0, s1, buf, lane); break;
        case 2: spmm_tile_nv<HB, 4, VT, XT, AT>(m, s0, s1, buf, lane); break;
        default: spmm_tile_nv<HB, 8, VT, XT, AT>(m, s0, s1, buf, lane); break;
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
__global__ __launch_bounds__(kSpmmMaxWaves * kWave) __attribute__((amdgpu_waves_per_eu(sizeof(AT) == 8 ? 4 : 1))) void spmm_persistent_kernel(
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
    const long long npass = (static_cast<long long>(strips) + S - 1) / S;
    // Several passes per wave once there are enough waves to fill the chip
    // twice over (256 CUs x 16 resident waves).
    int passes = 1;
    while (RB > 2 && passes < kSpmmMaxPassesPerWave && npass >= 2LL * passes * 8192) passes *= 2;
    const long long waves = (npass + passes - 1) / passes;
    const int grid = static_cast<int>((waves + wpb - 1) / wpb);
    hipLaunchKernelGGL((spmm_kernel<HB, RB, VT, XT, AT>), dim3(grid), dim3(wpb * kWave), lds, stream, m, strips,
                       passes);
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
    const size_t wave_bytes = spmm_wave_lds_bytes(
        spmm_lane_slots(m, static_cast<int>(16 / sizeof(XT)), std::is_same<VT, bf16_t>::value), sizeof(AT));
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
    m.nnz = A->nnz;
    m.ldx = ldx;
    m.ldy = ldy;
    m.hb = next_pow2(A->height);
    m.rb_log = ilog2(nrhs);
    int g = group;
    if (g <= 0) {
        // Enough entry slots that one unrolled step covers the mean strip,
        // but at most 128 / RB for 4 or more right-hand-side slots: a pass
        // then takes several steps, which spreads its reduction (64 * HB *
        // RB partials whatever G is) over more entries and gives the
        // prefetch of the next step something to overlap (measured on band
        // and stencil matrices of 2*10^6 rows, height 2 and 4: e.g. 1146 ->
        // 574 us for 8 right-hand sides, fp64, height 4).
        const int unroll = (1 << m.rb_log) >= 4 ? 4 : 8;
        const int strips = (A->rows + A->height - 1) / A->height;
        const double mean = strips > 0 ? static_cast<double>(A->nnz) / strips : 0.0;
        const double cap = m.rb_log >= 2 ? 128.0 / (1 << m.rb_log) : 64.0;
        g = next_pow2(static_cast<int>(std::min(cap, std::max(1.0, mean / unroll))));
    }
    if (g > kWave) g = kWave;
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
    // Tiles grouped by (height bucket, right-hand-side bucket), so that waves
    // running at the same time mostly execute the same code.
    std::vector<std::pair<int, int>> order;
    for (int i = 0; i < count; ++i) {
        const SpmmMat m = spmm_mat(&mats[i], nrhs[i], nullptr, nrhs[i], nullptr, nrhs[i], group);
        order.push_back({m.hb * 16 + m.rb_log, i});
        const int xv = mats[i].val_dtype == CMRS_R64F ? 2 : 4;
        sh.max_slots = std::max(sh.max_slots, spmm_lane_slots(m, xv, mats[i].val_dtype == CMRS_R16BF));
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
