// Fixed-point P2G contributions shared by the transfer kernels and the
// differentiable rollout's scatter: B-spline weights in 2^-22 units (u32) and
// the APIC affine momentum in 2^-fx_shift units (int64), each rounded to
// nearest by an FP64 sum with 1.5 * 2^52. Integer sums are exact, so LDS
// tiles can be accumulated with the fast integer LDS atomics in any order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mpm_internal.h"

namespace mpm {

constexpr double kMagic = 6755399441055744.0;           // 1.5 * 2^52
constexpr long long kMagicBits = 0x4338000000000000LL;  // its bit pattern
// 2^22 weight units per unit weight: a node's sum over the particles of one
// work item (at most kItemMax, each weight at most 0.75^3) stays below 2^32.
// Finer units would let a crowded node wrap; coarser ones add rounding noise
// to p/m that the affine matrix C amplifies by 4/dx.
constexpr float kWeightUnits = 4194304.0f;             // 2^22
static_assert((double)kItemMax * 0.421875 * 4194304.0 + kItemMax < 4294967296.0,
              "a work item cannot overflow a 32-bit weight sum");

// ------------------------------------------------------------------ P2G values
// Per-particle inputs of the P2G scatter: weights and the affine momentum
// field m v + A (x_I - x_p) = q + A o dx in fixed-point units (q = m v - A f dx,
// A = m C - dt V0 (4/dx^2) tau).
struct P2GIn {
  int base[3];
  float w[3][3];
  double q[3];
  double Adx[9];
};

// o in {0, 1, 2}: base, base + slope, base + 2 slope (o is a constant after
// unrolling, so only the needed operation remains).
__device__ __forceinline__ double affine_step(double base, double slope, int o) {
  return o == 0 ? base : (o == 1 ? base + slope : fma(slope, 2.0, base));
}

__device__ __forceinline__ long long fx_mul(double n, double v) {
  return __double_as_longlong(fma(n, v, kMagic)) - kMagicBits;
}

// The 27 contributions (weight units, 3 momentum values) of one particle, in
// a fixed order and with one fixed sequence of operations, handed to `sink`.
template <class Sink>
__device__ __forceinline__ void p2g_emit(const P2GIn& P, Sink&& sink) {
  // The x offset is a loop variable (not unrolled) to bound register use.
#pragma unroll 1
  for (int ox = 0; ox < 3; ++ox) {
    const float wx = ox == 0 ? P.w[0][0] : (ox == 1 ? P.w[0][1] : P.w[0][2]);
    double qx[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) qx[a] = fma(P.Adx[3 * a], (double)ox, P.q[a]);
#pragma unroll
    for (int oy = 0; oy < 3; ++oy) {
      double qy[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) qy[a] = affine_step(qx[a], P.Adx[3 * a + 1], oy);
      const float wxy = wx * P.w[1][oy];
#pragma unroll
      for (int oz = 0; oz < 3; ++oz) {
        const float N = wxy * P.w[2][oz];
        const double Nd = (double)N;
        const uint32_t wq = (uint32_t)fmaf(N, kWeightUnits, 0.5f);
        const long long p0 = fx_mul(Nd, affine_step(qy[0], P.Adx[2], oz));
        const long long p1 = fx_mul(Nd, affine_step(qy[1], P.Adx[5], oz));
        const long long p2 = fx_mul(Nd, affine_step(qy[2], P.Adx[8], oz));
        sink(ox, oy, oz, wq, p0, p1, p2);
      }
    }
  }
}

}  // namespace mpm
