// Grid update of the explicit MLS-MPM substep (CRESSim-MPM Algorithm 1, second
// loop): for every node with mass, v = (m v)/m + dt g (Sec. III-A, eq.
// mls_mpm_grid), then the SDF contact of each tool in id order (Sec. IV-A,
// eq. v_correction), then sticky walls (Sec. III-A, boundary conditions by
// altering the momentum). Empty nodes get v = 0. The kernel also clears the
// accumulator it has read, which is the grid reset of Algorithm 1 for the next
// substep.
//
// Work list: the active blocks of the current binning, then the overflow
// blocks claimed by particles that drifted out of their tile in this substep.
// The tool poses arrive as kernel arguments (they live in SGPRs).
#include "mpm_device.h"
#include "mpm_internal.h"

namespace mpm {

constexpr int kGridWG = 256;

__global__ __launch_bounds__(kGridWG) void k_grid(void* __restrict__ acc_m, void* __restrict__ acc_p0,
                                                  void* __restrict__ acc_p1, void* __restrict__ acc_p2,
                                                  float4* __restrict__ vel,
                                                  const uint32_t* __restrict__ act_list,
                                                  const uint32_t* __restrict__ ovf_list,
                                                  uint32_t* mark, uint32_t* __restrict__ node_cnt,
                                                  float* __restrict__ imp_slots, Status* st, int parity,
                                                  SimK s, ToolSetK tools) {
  // Momentum given to the material by each tool and by the walls on the nodes
  // this workgroup visits (two-way coupling, Sec. IV-A), summed per
  // workgroup into its own slot at the end: the walls' in registers, the
  // tools' (few nodes touch a tool) with LDS atomics.
  __shared__ float imp_tools[kMaxTools * 3];
  float imp_w[3] = {0.0f, 0.0f, 0.0f};
  if (threadIdx.x < kMaxTools * 3) imp_tools[threadIdx.x] = 0.0f;
  const unsigned n_act = st->n_act;
  const unsigned total = n_act + st->ovf_count[parity];
  __shared__ unsigned blk_cnt;
  const int lo = s.band, hi = s.n - 1 - s.band;
  for (unsigned li = blockIdx.x; li < total; li += gridDim.x) {
    const bool overflow = li >= n_act;
    const unsigned b = overflow ? ovf_list[li - n_act] : act_list[li];
    const int bi = (int)(b % (unsigned)s.nb);
    const int bj = (int)((b / (unsigned)s.nb) % (unsigned)s.nb);
    const int bk = (int)(b / ((unsigned)s.nb * (unsigned)s.nb));
    if (threadIdx.x == 0) blk_cnt = 0u;
    __syncthreads();
    unsigned cnt = 0;
    for (int l = threadIdx.x; l < kBlockNodes; l += kGridWG) {
      const size_t g = ((size_t)b << (3 * kTileLog2)) + (size_t)l;
      // Mass and momentum of the node (P2G result), then the reset.
      float m, p0, p1, p2;
      if (s.fixed) {
        m = (float)((uint32_t*)acc_m)[g] * s.m_unit;
        p0 = (float)((double)((long long*)acc_p0)[g] * s.fx_p_inv);
        p1 = (float)((double)((long long*)acc_p1)[g] * s.fx_p_inv);
        p2 = (float)((double)((long long*)acc_p2)[g] * s.fx_p_inv);
        ((uint32_t*)acc_m)[g] = 0u;
        ((long long*)acc_p0)[g] = 0ll;
        ((long long*)acc_p1)[g] = 0ll;
        ((long long*)acc_p2)[g] = 0ll;
      } else {
        m = ((float*)acc_m)[g];
        p0 = ((float*)acc_p0)[g];
        p1 = ((float*)acc_p1)[g];
        p2 = ((float*)acc_p2)[g];
        ((float*)acc_m)[g] = 0.0f;
        ((float*)acc_p0)[g] = 0.0f;
        ((float*)acc_p1)[g] = 0.0f;
        ((float*)acc_p2)[g] = 0.0f;
      }
      float v[3] = {0.0f, 0.0f, 0.0f};
      if (m > 0.0f) {
        cnt++;
        const float im = 1.0f / m;
        v[0] = p0 * im + s.dt * s.g[0];
        v[1] = p1 * im + s.dt * s.g[1];
        v[2] = p2 * im + s.dt * s.g[2];
        const int i = bi * kTile + (l & (kTile - 1));
        const int j = bj * kTile + ((l >> kTileLog2) & (kTile - 1));
        const int k = bk * kTile + (l >> (2 * kTileLog2));
        const float xI[3] = {(float)i * s.dx, (float)j * s.dx, (float)k * s.dx};
#pragma unroll 1
        for (int q = 0; q < tools.n; ++q) {
          if (tools.t[q].type == TOOL_NONE) continue;
          const float vb[3] = {v[0], v[1], v[2]};
          if (tool_contact(tools.t[q], xI, v)) {
#pragma unroll
            for (int a = 0; a < 3; ++a) atomicAdd(&imp_tools[3 * q + a], m * (v[a] - vb[a]));
          }
        }
        if (i < lo || i > hi || j < lo || j > hi || k < lo || k > hi) {
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            imp_w[a] -= m * v[a];
            v[a] = 0.0f;
          }
        }
      }
      vel[g] = make_float4(v[0], v[1], v[2], 0.0f);
    }
    // Nodes with mass in this block (plain store, summed on demand by the host
    // call that reports it; a shared counter would serialise every workgroup).
    if (cnt) atomicAdd(&blk_cnt, cnt);
    __syncthreads();
    if (threadIdx.x == 0) {
      node_cnt[b] = blk_cnt;
      if (overflow) mark[b] = 0u;
    }
  }
  // Clear the other parity's overflow list for the next substep.
  if (blockIdx.x == 0 && threadIdx.x == 0) st->ovf_count[parity ^ 1] = 0u;
  // Workgroup sum of the impulses into this workgroup's slot (no other
  // workgroup writes it, so a plain read-modify-write accumulates substeps).
  __shared__ float red[kGridWG / 64][3];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float x = imp_w[a];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if (lane == 0) red[wave][a] = x;
  }
  __syncthreads();
  if (threadIdx.x < kImpulseRows * 3) {
    float x;
    if (threadIdx.x < kMaxTools * 3) {
      x = imp_tools[threadIdx.x];
    } else {
      x = 0.0f;
#pragma unroll
      for (int w = 0; w < kGridWG / 64; ++w) x += red[w][threadIdx.x - kMaxTools * 3];
    }
    imp_slots[(size_t)blockIdx.x * (kImpulseRows * 3) + threadIdx.x] += x;
  }
}

void launch_grid(Buffers& b, const SimK& s, const ToolSetK& tools, int parity, int max_act,
                 hipStream_t st) {
  int wgs = max_act < kGridSlots ? max_act : kGridSlots;
  if (wgs < 1) wgs = 1;
  hipLaunchKernelGGL(k_grid, dim3(wgs), dim3(kGridWG), 0, st, b.acc_m, b.acc_p[0], b.acc_p[1],
                     b.acc_p[2], b.vel, b.act_list,
                     b.ovf_list[parity], b.mark, b.node_cnt, b.imp_slots, b.status, parity, s, tools);
}

}  // namespace mpm
