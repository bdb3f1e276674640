// Device building blocks of the CMRS SpMV kernels (gfx950, wave64): stream
// loads, the per-lane partial sums of Algorithm 1 (Sec. 4) in LDS or VGPRs,
// their reduction to row sums, and the strip-group walk.  Included by the
// SpMV translation units.
#pragma once

#include "cmrs_device.hpp"

namespace cmrs {

constexpr int kSpmvWaves = 4;
constexpr int kSpmvThreads = kSpmvWaves * kWave;

template <bool NT, typename T>
__device__ inline T stream_load(const T* p) {
    if constexpr (NT) {
        return __builtin_nontemporal_load(p);
    } else {
        return *p;
    }
}

template <bool NT>
__device__ inline bf16_t stream_load(const bf16_t* p) {
    bf16_t v;
    if constexpr (NT) {
        v.bits = __builtin_nontemporal_load(&p->bits);
    } else {
        v.bits = p->bits;
    }
    return v;
}

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
    // Group r starts at partial r mod PER and wraps, so the HB groups, which
    // read at a stride of 64 slots, do not all hit the same LDS banks.
    const int rot = r & (PER - 1);
    AT s = p[rot];
#pragma unroll
    for (int i = 1; i < PER; ++i) s += p[(i + rot) & (PER - 1)];
#pragma unroll
    for (int off = G / 2; off >= 1; off >>= 1) s += __shfl_xor(s, off);
    return s;
}

template <int HB, typename AT>
struct LdsAcc {
    AT* b;
    __device__ inline void init(int lane) {
#pragma unroll
        for (int r = 0; r < HB; ++r) b[r * kWave + lane] = AT(0);
    }
    __device__ inline void add(uint32_t r, int lane, AT p) {
        lds_add(&b[(static_cast<int>(r) & (HB - 1)) * kWave + lane], p);
    }
    // Row sums; lane l holds the sum of row l / (64 / HB).
    __device__ inline AT finish(int lane) {
        wave_lds_sync();
        return reduce_rows_lds<HB>(b, lane);
    }
};

template <int HB, typename AT>
struct RegAcc {
    AT acc[HB];
    __device__ inline void init(int) {
#pragma unroll
        for (int r = 0; r < HB; ++r) acc[r] = AT(0);
    }
    __device__ inline void add(uint32_t r, int, AT p) {
#pragma unroll
        for (int k = 0; k < HB; ++k) acc[k] += (r == static_cast<uint32_t>(k)) ? p : AT(0);
    }
    // Reduce-scatter butterfly: at the step with xor offset o, a lane whose
    // bit o is set keeps the upper half of its rows and sends the lower half.
    // After log2(HB) steps lane l holds a partial of row l / (64/HB); the
    // remaining offsets sum the group.
    __device__ inline AT finish(int lane) {
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
        return acc[0];
    }
};

// Entries [lo, hi) of one strip into `acc`; U batches of 64 entries have all
// their stream loads, then all their gathers, in flight together.
template <int U, bool NT, typename VT, typename XT, typename AT, typename Acc>
__device__ inline void accumulate_run(Acc& acc, int lo, int hi, int bits, const uint32_t* __restrict__ word,
                                      const VT* __restrict__ val, const XT* __restrict__ x, int lane) {
    const uint32_t mask = (1u << bits) - 1u;
    for (int base = lo; base < hi; base += U * kWave) {
        // Entries past the run are clamped to its last entry (a valid
        // address) so the stream loads of the step issue without a branch;
        // their gathers are masked off and their products dropped.
        uint32_t w[U];
        VT v[U];
        XT xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = min(base + u * kWave + lane, hi - 1);
            w[u] = stream_load<NT>(word + j);
            v[u] = stream_load<NT>(val + j);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (base + u * kWave + lane < hi) xv[u] = x[w[u] >> bits];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (base + u * kWave + lane < hi) {
                const AT p = static_cast<AT>(ValTraits<VT>::widen(v[u])) * static_cast<AT>(xv[u]);
                acc.add(w[u] & mask, lane, p);
            }
        }
    }
}

// Sum each (group g, row r) set of G partials held in LDS slots
// ((g*HB + r)*G + q, q < G) and hand the sum to out(g, r, sum).  There are
// S = NG*HB sums: with S <= 64, L = 64/S lanes share one sum (xor butterfly);
// otherwise every lane takes S/64 whole sums.  A lane reading PER consecutive
// slots starts at slot si mod PER of them and wraps: lanes reading at a
// stride of PER slots would otherwise all hit the same LDS banks.  (The
// order of the additions is fixed per sum, so results stay deterministic.)
// out() is called by a subset of the lanes and must not use cross-lane
// operations.
template <int HB, int G, typename AT, typename Out>
__device__ inline void group_reduce(const AT* b, int lane, Out out) {
    constexpr int NG = kWave / G;
    constexpr int S = NG * HB;
    if constexpr (S <= kWave) {
        constexpr int L = kWave / S;
        constexpr int PER = G / L;
        const int si = lane / L, part = lane % L;
        const AT* pp = b + si * G + part * PER;
        const int rot = si & (PER - 1);
        AT s = pp[rot];
#pragma unroll
        for (int i = 1; i < PER; ++i) s += pp[(i + rot) & (PER - 1)];
#pragma unroll
        for (int off = L / 2; off >= 1; off >>= 1) s += __shfl_xor(s, off);
        if (part == 0) out(si / HB, si % HB, s);
    } else {
        constexpr int K = S / kWave;
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const int si = lane + kWave * i;
            const AT* pp = b + si * G;
            const int rot = si & (G - 1);
            AT s = pp[rot];
#pragma unroll
            for (int j = 1; j < G; ++j) s += pp[(j + rot) & (G - 1)];
            out(si / HB, si % HB, s);
        }
    }
}

// Lane q of group g adds the products of entries lo+q, lo+q+G, ... < hi into
// its LDS slots (g*HB + r)*G + q: U stream loads, then U gathers in flight.
template <int HB, int G, int U, bool NT, typename VT, typename XT, typename AT>
__device__ inline void group_walk(int lo, int hi, int bits, const uint32_t* __restrict__ word,
                                  const VT* __restrict__ val, const XT* __restrict__ x, AT* b, int g, int q) {
    const uint32_t mask = (1u << bits) - 1u;
    for (int j0 = lo + q; j0 < hi; j0 += U * G) {
        uint32_t w[U];
        VT v[U];
        XT xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = min(j0 + u * G, hi - 1);
            w[u] = stream_load<NT>(word + j);
            v[u] = stream_load<NT>(val + j);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (j0 + u * G < hi) xv[u] = x[w[u] >> bits];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = j0 + u * G;
            if (j < hi) {
                const AT p = static_cast<AT>(ValTraits<VT>::widen(v[u])) * static_cast<AT>(xv[u]);
                const int r = static_cast<int>(w[u] & mask) & (HB - 1);
                lds_add(&b[(g * HB + r) * G + q], p);
            }
        }
    }
}

// Strip groups: one wave processes NG = 64/G runs at once (a run is a strip,
// or one column block of a strip), G lanes per run, so a wave keeps 64*U
// entries of memory traffic outstanding instead of one strip's.  Partials
// live in LDS slot (g*HB + r)*G + q (each lane owns its slots, as in
// Algorithm 1).  Runs longer than long_len are skipped by their group and
// processed afterwards by the whole wave, one at a time, with the per-lane
// layout of spmv_kernel; with SKIP_LONG they are left alone (another wave
// processes them) and get no out() call.  out(g, r, sum) receives every other
// row sum.
template <int HB, int G, int U, bool NT, typename VT, typename XT, typename AT, typename Out, bool SKIP_LONG = false>
__device__ inline void group_runs(int lo, int hi, int long_len, int bits, const uint32_t* __restrict__ word,
                                  const VT* __restrict__ val, const XT* __restrict__ x, AT* b, int lane, Out out) {
    const int g = lane / G, q = lane % G;
    const bool is_long = hi - lo > long_len;
#pragma unroll
    for (int r = 0; r < HB; ++r) b[(g * HB + r) * G + q] = AT(0);
    if (!is_long) group_walk<HB, G, U, NT, VT, XT, AT>(lo, hi, bits, word, val, x, b, g, q);
    wave_lds_sync();
    const uint64_t longs = ballot(is_long && q == 0);
    group_reduce<HB, G, AT>(b, lane, [&](int gg, int rr, AT s) {
        if (!((longs >> (gg * G)) & 1ull)) out(gg, rr, s);
    });
    if (SKIP_LONG || longs == 0) return;
    wave_lds_sync();
    uint64_t rest = longs;
    while (rest) {
        const int leader = __ffsll(static_cast<unsigned long long>(rest)) - 1;
        rest &= rest - 1;
        const int llo = __shfl(lo, leader), lhi = __shfl(hi, leader);
        LdsAcc<HB, AT> acc{b};
        acc.init(lane);
        accumulate_run<U, NT, VT, XT, AT>(acc, llo, lhi, bits, word, val, x, lane);
        const AT s = acc.finish(lane);
        constexpr int GW = kWave / HB;
        if ((lane % GW) == 0) out(leader / G, lane / GW, s);
        wave_lds_sync();
    }
}

}  // namespace cmrs
