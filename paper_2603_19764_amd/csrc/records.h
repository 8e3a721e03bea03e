// Velocity and mass in the pair-pass records (array of structures; slot =
// one float4 in the FP32 form, one double4 in the FP64 form).
//
// The FP64 form keeps (v, m) in one slot.  The FP32 form keeps v in FP64 as
// well, in two slots (vx, vy, vz as doubles, then m as a float): a pair's
// velocity difference is formed in FP64 and rounded once to FP32, so
// particles that move fast together (a projectile at km/s) keep the digits
// of their small relative velocities, as positions do through the
// cell-relative offsets.  All other pair arithmetic stays FP32.
#pragma once

#include <hip/hip_runtime.h>

namespace sph {

struct VelM32 {
    double x, y, z;
    float m, pad;
};

template <bool F32>
constexpr int kVelSlots = F32 ? 2 : 1;
// gradient pass: (p, 1/H) (v, m) (Kn/(Omega rho), -, -, -)
template <bool F32>
constexpr int kRecGradSlots = 2 + kVelSlots<F32>;
// force pass: (p, 1/H) (v, m) (Kn A: xx yy zz xy) (Kn A: xz yz, rho, c) (Kn, h, -, -)
template <bool F32>
constexpr int kRecForceSlots = 4 + kVelSlots<F32>;
// fused gradient + force sweep: (p, 1/H) (v, m) (m Kn A: xx yy zz xy)
// (m Kn A: xz yz, rho/2, c/2) (-m Kn/(2 Omega rho), m Kn/2, h/2, 1/m)
template <bool F32>
constexpr int kRecBothSlots = 4 + kVelSlots<F32>;
// Slots between consecutive records of the fused sweep in memory (dense:
// padding the 96-byte FP32 record to one aligned 128-byte line made the sweep
// on the 1.1M impact 1.6x slower, its records no longer fitting the caches).
template <bool F32>
constexpr int kRecBothStride = kRecBothSlots<F32>;

template <typename R>
struct VM {
    double x, y, z;
    R m;
};

template <bool F32, typename R4>
__device__ __forceinline__ void store_vm(R4 *slot, double vx, double vy, double vz, double m) {
    if constexpr (F32)
        *reinterpret_cast<VelM32 *>(slot) = VelM32{vx, vy, vz, (float)m, 0.f};
    else
        slot[0] = R4{vx, vy, vz, m};
}

template <bool F32, typename R, typename R4>
__device__ __forceinline__ VM<R> load_vm(const R4 *slot) {
    if constexpr (F32) {
        const VelM32 v = *reinterpret_cast<const VelM32 *>(slot);
        return VM<R>{v.x, v.y, v.z, v.m};
    } else {
        const R4 v = slot[0];
        return VM<R>{v.x, v.y, v.z, v.w};
    }
}

}  // namespace sph
