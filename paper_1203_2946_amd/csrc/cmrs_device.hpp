// Device-side helpers shared by the CMRS kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cmrs {

constexpr int kWave = 64;
constexpr int kNumXcd = 8;  // MI355X: 8 XCDs, workgroups are dealt to them round-robin

// bfloat16 stored as its raw 16-bit pattern.
struct bf16_t {
    uint16_t bits;
};

template <typename T>
struct ValTraits;
template <>
struct ValTraits<double> {
    __device__ static inline double widen(double v) { return v; }
};
template <>
struct ValTraits<float> {
    __device__ static inline float widen(float v) { return v; }
};
template <>
struct ValTraits<bf16_t> {
    __device__ static inline float widen(bf16_t v) { return __uint_as_float(static_cast<uint32_t>(v.bits) << 16); }
};

__device__ inline int lane_id() { return static_cast<int>(threadIdx.x) & (kWave - 1); }

__device__ inline int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Workgroup b of n is placed on XCD b % 8.  Renumber workgroups so that each
// XCD owns one contiguous range of logical ids: neighbouring strips then share
// an XCD's L2 (cache lines straddling strip boundaries, clustered x gathers).
__device__ inline int xcd_logical_block(int b, int n) {
    const int xcd = b % kNumXcd, idx = b / kNumXcd;
    const int q = n / kNumXcd, rem = n % kNumXcd;
    return xcd * q + (xcd < rem ? xcd : rem) + idx;
}

__device__ inline uint64_t ballot(bool p) { return __ballot(p); }

__device__ inline uint64_t lanemask_lt() {
    const int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Add v to an LDS partial sum that no other lane of the same instruction
// updates: a lane-owned slot, or (the padded kernel of Sec. 6.7) a copy
// shared by lanes that the padded arrangement keeps from ever holding
// entries of the same row in one 64-entry chunk.  fp64 uses the LDS atomic
// add, one instruction.  The fp32 LDS atomic add runs about 25x below the
// LDS rate on gfx950 (measured with lane-private slots), so fp32 partials
// take a plain read-modify-write, which is exact under that condition and
// would lose additions without it.
template <typename AT>
__device__ inline void lds_add(AT* p, AT v) {
    *p += v;
}
template <>
__device__ inline void lds_add<double>(double* p, double v) {
    atomicAdd(p, v);
}

// Order this wave's LDS accesses: every lane's earlier LDS writes/atomics are
// complete and visible to the wave's later LDS reads.
// (Workgroup-scope fences: they make the compiler wait for outstanding LDS
// operations; the wave barrier keeps it from moving LDS accesses across.)
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

}  // namespace cmrs
