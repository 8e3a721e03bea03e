// Device-side constants and helpers shared by the kernels of the gfx950
// strength-SPH library: neighbour-entry encoding, XCD-aware block order,
// Morton keys, the exact squared separation and lane-group reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sph {

// ------------------------------------------------------------------ limits
constexpr int kWave = 64;
constexpr int kIdxBits = 26;                       // neighbour entry: j index bits
constexpr uint32_t kIdxMask = (1u << kIdxBits) - 1;
constexpr int kCodeShift = kIdxBits;               // 5 bits: stencil cell 0..26
constexpr uint32_t kDensityBit = 1u << 31;         // j is in the density set of i
constexpr int kMaxMortonBits = 10;                 // per axis
constexpr int kNumXcd = 8;                         // MI355X: 8 XCDs, round-robin dispatch

// --------------------------------------------------------- device helpers
__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Block index remapped so that consecutive logical blocks run on the same
// XCD (hardware dispatches block b to XCD b % 8): XCD x gets a contiguous
// range of logical blocks.  Bijective for any grid size.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb) {
    uint32_t q = nb / kNumXcd, r = nb % kNumXcd;
    uint32_t x = b % kNumXcd, k = b / kNumXcd;
    return x * q + (x < r ? x : r) + k;
}

// Interleave cell coordinates into a Morton key with per-axis bit counts.
__device__ __forceinline__ uint32_t morton(uint32_t cx, uint32_t cy, uint32_t cz,
                                           int bx, int by, int bz) {
    uint32_t key = 0;
    int pos = 0;
    int mb = bx > by ? bx : by;
    mb = mb > bz ? mb : bz;
    for (int l = 0; l < mb; ++l) {
        if (l < bx) key |= ((cx >> l) & 1u) << pos++;
        if (l < by) key |= ((cy >> l) & 1u) << pos++;
        if (l < bz) key |= ((cz >> l) & 1u) << pos++;
    }
    return key;
}

// Squared separation ((dx*dx + dy*dy) + dz*dz) in IEEE double with every
// operation rounded separately: contraction into FMA is switched off here,
// so the neighbour criterion r^2 < H^2 is decided exactly as by any other
// implementation that evaluates the same expression without fusion.
__device__ __forceinline__ double sep2_exact(double xi, double yi, double zi, double xj,
                                             double yj, double zj) {
#pragma clang fp contract(off)
    const double dx = xi - xj;
    const double dy = yi - yj;
    const double dz = zi - zj;
    const double a = dx * dx;
    const double b = dy * dy;
    const double c = dz * dz;
    return (a + b) + c;
}

// Sum over groups of L consecutive lanes (L a power of two <= 64); every
// lane of the group receives the group sum.
template <int L>
__device__ __forceinline__ float group_sum(float v) {
#pragma unroll
    for (int o = L / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, L);
    return v;
}
template <int L>
__device__ __forceinline__ int group_sum(int v) {
#pragma unroll
    for (int o = L / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, L);
    return v;
}
template <int L>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
    for (int o = L / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, L);
    return v;
}
template <int L>
__device__ __forceinline__ float group_min(float v) {
#pragma unroll
    for (int o = L / 2; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, L));
    return v;
}
template <int L>
__device__ __forceinline__ double group_max(double v) {
#pragma unroll
    for (int o = L / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, L));
    return v;
}
template <int L>
__device__ __forceinline__ float group_max(float v) {
#pragma unroll
    for (int o = L / 2; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, L));
    return v;
}

}  // namespace sph
