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
                                                  Status* st, int parity, SimK s,
                                                  ToolSetK tools) {
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
        for (int q = 0; q < tools.n; ++q)
          if (tools.t[q].type != TOOL_NONE) tool_contact(tools.t[q], xI, v);
        if (i < lo || i > hi || j < lo || j > hi || k < lo || k > hi) v[0] = v[1] = v[2] = 0.0f;
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
}

void launch_grid(Buffers& b, const SimK& s, const ToolSetK& tools, int parity, int max_act,
                 hipStream_t st) {
  int wgs = max_act < 8192 ? max_act : 8192;
  if (wgs < 1) wgs = 1;
  hipLaunchKernelGGL(k_grid, dim3(wgs), dim3(kGridWG), 0, st, b.acc_m, b.acc_p[0], b.acc_p[1],
                     b.acc_p[2], b.vel, b.act_list,
                     b.ovf_list[parity], b.mark, b.node_cnt, b.status, parity, s, tools);
}

}  // namespace mpm
