// Internal declarations of the differentiable rollout (dense-grid substep,
// its reverse kernels and their buffers), shared by diff.hip and api.hip.
#pragma once

#include "mpm_internal.h"

namespace mpm {

// ---------------------------------------------------------------- differentiable rollout
// A particle state in the caller's order: x (N x 3), v (N x 3), C (N x 9),
// F (N x 9), consecutive in one block of kStateFloats * N floats. Adjoint
// states use the same layout.
constexpr int kStateFloats = 24;
constexpr int kToolRedCopies = 16;

struct DState {
  float* x;
  float* v;
  float* C;
  float* F;
};

inline DState dstate(float* base, int64_t N) {
  return {base, base + 3 * N, base + 6 * N, base + 15 * N};
}

// Dense-grid buffers of the differentiable path (n^3 nodes, node (i, j, k)
// at index (i * n + j) * n + k).
struct DiffGrid {
  float* m = nullptr;                       // P2G mass accumulator
  float* p[3] = {nullptr, nullptr, nullptr};  // P2G momentum accumulators
  float4* vel = nullptr;                    // velocity after the grid update when no grid is kept (w unused)
  float* vb[3] = {nullptr, nullptr, nullptr};  // cotangent of vel (accumulated by G2P adjoint)
  float4* pb = nullptr;                     // cotangent of momentum (xyz) and of mass (w)
  uint8_t* skip = nullptr;                  // per particle: left unchanged this substep
};

// A spatial order of the rollout's particles (launch_order): the scatter
// kernels walk `work` (info[0] items of at most kItemRollout sorted positions
// of one block, whose LDS tile takes the block's stencils), then the sorted
// positions from info[1] on, which hold the particles outside the grid.
// Particles that move out of their block's tile after the order was taken
// scatter straight into the global grid, so any order gives the same sums
// up to the order of FP32 additions.
struct DiffOrder {
  const uint32_t* order;    // sorted position -> caller index
  const uint32_t* blk_end;  // per block: end of its sorted positions
  const uint2* work;        // {block, first sorted position}
  const uint32_t* info;     // device: {items, first position outside the grid}
};

// Forward substep on the dense grid: P2G from `in`, grid update (tools,
// walls) into `vel` (and, if `hat` is not null, the pre-contact velocity and
// the mass into `hat`), G2P into `out` (skipped when out.x is null).
// Particles with a non-finite state or a stencil outside the grid are copied
// unchanged (and counted when `count`); g.skip records them.
void launch_diff_substep(const DiffGrid& g, float4* vel, float4* hat, const SimK& s, const ToolSetK& tools,
                         int64_t N, DState in, const float* E, DState out, bool count, Status* st,
                         const DiffOrder& o, hipStream_t stream);
// Reverse of one substep from the state `in` it started from and its grid
// (`vel`, `hat`) as its forward pass left them, in two parts: the head (G2P
// reverse, grid reverse) and the tail (P2G reverse). On entry `adj` is the
// cotangent of the state after the substep, after the tail that of `in`.
// The tail may be deferred: the head of the substep before, given that
// substep's successor state as `pending`, runs it per particle inside its
// G2P reverse (the grid cotangents in g.pb stay valid until the next head's
// grid reverse). The last tail runs on its own. Adds d/d log E to theta_bar
// and the tools' linear-velocity and centre cotangents to
// tool_red[kToolRedCopies][kMaxTools * 6] (FP64): each workgroup adds its
// sums into one of the copies, so that the FP64 atomics of the many
// workgroups that touch a tool do not all meet on one address.
void launch_adjoint_head(const DiffGrid& g, const float4* vel, const float4* hat, const SimK& s,
                         const ToolSetK& tools, int64_t N, DState in, const float* E, DState adj, float* theta_bar,
                         double* tool_red, const DiffOrder& o, const DState* pending, hipStream_t stream);
void launch_adjoint_tail(const DiffGrid& g, const SimK& s, int64_t N, DState in, const float* E, DState adj,
                         float* theta_bar, hipStream_t stream);
// out[j][c] = sum over the copies of parts[j][copy][c] (j < T, c < kMaxTools * 6).
void launch_sum_tool_copies(const double* parts, int T, double* out, hipStream_t st);
// Fill helpers.
void launch_fill_f32(float* p, int64_t n, float v, hipStream_t st);
void launch_fill_f64(double* p, int64_t n, double v, hipStream_t st);
void launch_exp(const float* theta, float* E, int64_t n, hipStream_t st);
// E of the handle's particles in the caller's order (E_default when absent).
void launch_unpermute_E(const Buffers& b, int64_t N, const SimK& s, float* E, hipStream_t st);

}  // namespace mpm
