// Grid update of the explicit MLS-MPM substep (CRESSim-MPM Algorithm 1, second
// loop): for every node with mass, v = (m v)/m + dt g (Sec. III-A, eq.
// mls_mpm_grid; PB-MPM iterations leave out g, which it adds to the particles
// once per step), then the SDF contact of each tool in id order (Sec. IV-A,
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

constexpr int kGridWG = 128;
static_assert(kBlockNodes % kGridWG == 0, "every lane of the grid kernel must visit the same number of nodes");
constexpr int kNodesPerLane = kBlockNodes / kGridWG;

__global__ __launch_bounds__(kGridWG) void k_grid(void* __restrict__ acc_m, void* __restrict__ acc_p0,
                                                  void* __restrict__ acc_p1, void* __restrict__ acc_p2,
                                                  float4* __restrict__ vel,
                                                  const uint32_t* __restrict__ act_list,
                                                  const uint32_t* __restrict__ ovf0,
                                                  const uint32_t* __restrict__ ovf1,
                                                  uint32_t* mark, uint32_t* __restrict__ node_cnt,
                                                  float* __restrict__ imp_blocks, const ToolDesc* __restrict__ tools,
                                                  Status* st, Clock* clk, int parity, int dsub, int record,
                                                  unsigned long long* drift_host, SimK s) {
  const long long substep = clk[parity].substep;
  const uint32_t* __restrict__ ovf_list = parity ? ovf1 : ovf0;
  // Momentum given to the material by each tool and by the walls on the nodes
  // of one block (two-way coupling, Sec. IV-A), added to the block's own
  // sums. Each wave reduces its contributions with shuffles (a tool's only
  // when one of its lanes touched the tool) and the waves' partial sums are
  // added in a fixed order, so the sums do not depend on timing.
  __shared__ float red_t[kGridWG / 64][kMaxTools * 3];
  __shared__ float red[kGridWG / 64][3];
  __shared__ unsigned blk_cnt;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned n_act = st->n_act;
  const unsigned total = n_act + st->ovf_count[parity];
  const int lo = s.band, hi = s.n - 1 - s.band;
  for (unsigned li = blockIdx.x; li < total; li += gridDim.x) {
    const bool overflow = li >= n_act;
    const unsigned b = overflow ? ovf_list[li - n_act] : act_list[li];
    const unsigned scene = b / s.nb3;
    const unsigned lb = b - scene * s.nb3;
    const int bi = (int)(lb % (unsigned)s.nb);
    const int bj = (int)((lb / (unsigned)s.nb) % (unsigned)s.nb);
    const int bk = (int)(lb / ((unsigned)s.nb * (unsigned)s.nb));
    const ToolDesc* td = tools + (size_t)scene * kMaxTools;
    if (threadIdx.x == 0) blk_cnt = 0u;
    if (lane < kMaxTools * 3) red_t[wave][lane] = 0.0f;
    __syncthreads();
    unsigned cnt = 0;
    float imp_w[3] = {0.0f, 0.0f, 0.0f};
    // Mass and momentum of this lane's nodes (P2G result), all loaded before
    // any is used so that the loads are in flight together, then the reset.
    const size_t g0 = ((size_t)b << (3 * kTileLog2)) + (size_t)threadIdx.x;
    float nm[kNodesPerLane], np0[kNodesPerLane], np1[kNodesPerLane], np2[kNodesPerLane];
    if (s.fixed) {
      uint32_t um[kNodesPerLane];
      long long q0[kNodesPerLane], q1[kNodesPerLane], q2[kNodesPerLane];
#pragma unroll
      for (int r = 0; r < kNodesPerLane; ++r) {
        const size_t g = g0 + (size_t)r * kGridWG;
        um[r] = ((uint32_t*)acc_m)[g];
        q0[r] = ((long long*)acc_p0)[g];
        q1[r] = ((long long*)acc_p1)[g];
        q2[r] = ((long long*)acc_p2)[g];
      }
#pragma unroll
      for (int r = 0; r < kNodesPerLane; ++r) {
        const size_t g = g0 + (size_t)r * kGridWG;
        ((uint32_t*)acc_m)[g] = 0u;
        ((long long*)acc_p0)[g] = 0ll;
        ((long long*)acc_p1)[g] = 0ll;
        ((long long*)acc_p2)[g] = 0ll;
        nm[r] = (float)um[r] * s.m_unit;
        np0[r] = (float)((double)q0[r] * s.fx_p_inv);
        np1[r] = (float)((double)q1[r] * s.fx_p_inv);
        np2[r] = (float)((double)q2[r] * s.fx_p_inv);
      }
    } else {
#pragma unroll
      for (int r = 0; r < kNodesPerLane; ++r) {
        const size_t g = g0 + (size_t)r * kGridWG;
        nm[r] = ((float*)acc_m)[g];
        np0[r] = ((float*)acc_p0)[g];
        np1[r] = ((float*)acc_p1)[g];
        np2[r] = ((float*)acc_p2)[g];
      }
#pragma unroll
      for (int r = 0; r < kNodesPerLane; ++r) {
        const size_t g = g0 + (size_t)r * kGridWG;
        ((float*)acc_m)[g] = 0.0f;
        ((float*)acc_p0)[g] = 0.0f;
        ((float*)acc_p1)[g] = 0.0f;
        ((float*)acc_p2)[g] = 0.0f;
      }
    }
    // Grid velocities of this lane's nodes: v = p/m + dt g where there is
    // mass (Sec. III-A), 0 elsewhere.
    float v[kNodesPerLane][3];
#pragma unroll
    for (int r = 0; r < kNodesPerLane; ++r) {
      v[r][0] = v[r][1] = v[r][2] = 0.0f;
      if (nm[r] > 0.0f) {
        cnt++;
        const float im = 1.0f / nm[r];
        v[r][0] = np0[r] * im + s.dt * s.g[0];
        v[r][1] = np1[r] * im + s.dt * s.g[1];
        v[r][2] = np2[r] * im + s.dt * s.g[2];
      }
    }
    // Tools in id order, each applied to every node of the lane; the pose is
    // computed once per tool. The loop runs on every lane (kBlockNodes is a
    // multiple of the workgroup size), so the wave reductions see full waves.
#pragma unroll 1
    for (int q = 0; q < s.tool_slots; ++q) {
      if (td[q].k.type == TOOL_NONE) continue;
      const ToolK t = tool_at(td[q], substep, (double)s.dt);
      float dm[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int r = 0; r < kNodesPerLane; ++r) {
        if (!(nm[r] > 0.0f)) continue;
        const int l = threadIdx.x + r * kGridWG;
        const float xI[3] = {(float)(bi * kTile + (l & (kTile - 1))) * s.dx,
                             (float)(bj * kTile + ((l >> kTileLog2) & (kTile - 1))) * s.dx,
                             (float)(bk * kTile + (l >> (2 * kTileLog2))) * s.dx};
        const float vb[3] = {v[r][0], v[r][1], v[r][2]};
        if (tool_contact(t, xI, v[r])) {
#pragma unroll
          for (int c = 0; c < 3; ++c) dm[c] += nm[r] * (v[r][c] - vb[c]);
        }
      }
      if (__ballot(dm[0] != 0.0f || dm[1] != 0.0f || dm[2] != 0.0f) != 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          float x = dm[c];
#pragma unroll
          for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
          if (lane == 0) red_t[wave][3 * q + c] = x;
        }
      }
    }
    // Sticky walls, then the velocities out.
#pragma unroll
    for (int r = 0; r < kNodesPerLane; ++r) {
      const int l = threadIdx.x + r * kGridWG;
      const int i = bi * kTile + (l & (kTile - 1));
      const int j = bj * kTile + ((l >> kTileLog2) & (kTile - 1));
      const int k = bk * kTile + (l >> (2 * kTileLog2));
      if (nm[r] > 0.0f && (i < lo || i > hi || j < lo || j > hi || k < lo || k > hi)) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          imp_w[c] -= nm[r] * v[r][c];
          v[r][c] = 0.0f;
        }
      }
      vel[g0 + (size_t)r * kGridWG] = make_float4(v[r][0], v[r][1], v[r][2], 0.0f);
    }
    // Nodes with mass in this block (plain store, summed on demand by the host
    // call that reports it; a shared counter would serialise every workgroup).
    if (cnt) atomicAdd(&blk_cnt, cnt);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      float x = imp_w[a];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
      if (lane == 0) red[wave][a] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      node_cnt[b] = blk_cnt;
      if (overflow) mark[b] = 0u;
    }
    // The block's impulse sums (each block is visited once per substep).
    if (threadIdx.x < kImpulseRows * 3) {
      float x;
      if (threadIdx.x < kMaxTools * 3) {
        x = 0.0f;
#pragma unroll
        for (int w = 0; w < kGridWG / 64; ++w) x += red_t[w][threadIdx.x];
      } else {
        x = 0.0f;
#pragma unroll
        for (int w = 0; w < kGridWG / 64; ++w) x += red[w][threadIdx.x - kMaxTools * 3];
      }
      if (record && x != 0.0f) imp_blocks[(size_t)b * (kImpulseRows * 3) + threadIdx.x] += x;
    }
    __syncthreads();
  }
  // Clear the other parity's overflow list for the next substep, and set the
  // other parity's clock: every workgroup has read this parity's entry, and
  // the kernels of the next grid update's parity read the other one.
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->ovf_count[parity ^ 1] = 0u;
    clk[parity ^ 1].substep = substep + dsub;
    // After a substep's last pass, the fallback count so far (the fused
    // kernel before this one has added its own) for the host to read
    // without waiting; the substep word goes last.
    if (dsub && drift_host) {
      __hip_atomic_store(&drift_host[1], st->n_fallback, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_store(&drift_host[2], st->fb_at_sort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_store(&drift_host[0], (unsigned long long)(substep + dsub), __ATOMIC_RELEASE,
                         __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

__global__ void k_set_clock(Clock* clk, long long substep, int parity) { clk[parity].substep = substep; }

void launch_set_clock(Buffers& b, long long substep, int parity, hipStream_t st) {
  hipLaunchKernelGGL(k_set_clock, dim3(1), dim3(1), 0, st, b.clock, substep, parity & 1);
}

void launch_grid(Buffers& b, const SimK& s, int max_act, int parity, hipStream_t st, bool gravity, bool record,
                 bool last, KernelEvents ev) {
  int wgs = max_act < kGridSlots ? max_act : kGridSlots;
  if (wgs < 1) wgs = 1;
  SimK k = s;
  if (!gravity) k.g[0] = k.g[1] = k.g[2] = 0.0f;
  launch_kernel(k_grid, dim3(wgs), dim3(kGridWG), st, ev, b.acc_m, b.acc_p[0], b.acc_p[1],
                     b.acc_p[2], b.vel, b.act_list, b.ovf_list[0], b.ovf_list[1], b.mark, b.node_cnt, b.imp_blocks,
                     (const ToolDesc*)b.tools, b.status, b.clock, parity & 1, last ? 1 : 0, record ? 1 : 0,
                     b.drift_host, k);
}

}  // namespace mpm
