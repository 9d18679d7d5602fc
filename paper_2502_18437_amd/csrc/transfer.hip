// Particle <-> grid transfers of the explicit MLS-MPM substep (CRESSim-MPM
// Sec. III-B, Algorithm 1), block-tiled for CDNA4.
//
// Particles are binned by the grid block (kTile^3 cells) of their base cell.
// One workgroup owns one block at a time: it stages the grid velocities of the
// block's tile (kSpan^3 nodes: the block's stencils plus kSlack cells of
// drift) in LDS, gathers (G2P) from LDS, scatters (P2G) into an LDS
// accumulator tile with LDS float atomics, then flushes the non-empty tile
// nodes into the global accumulator with one float atomic per value. A
// particle whose stencil has drifted out of the tile since binning takes a
// correct global-memory path and claims the blocks it touches for the grid
// update (overflow list).
//
// k_g2p2g fuses the G2P of substep k-1 with the P2G of substep k: v and C never
// leave registers between the two, so a fused substep streams x, F, E in and
// x, F out (100 B/particle).
#include "mpm_device.h"
#include "mpm_internal.h"

namespace mpm {

constexpr int kXcds = 8;
constexpr int kWG = 256;

// Walk of a block list by a persistent grid whose size is a multiple of 8.
// Workgroups are dealt round-robin to the 8 XCDs, so workgroup w runs on XCD
// w % 8; each XCD takes one contiguous eighth of the spatially ordered list,
// so blocks that share halo nodes share an L2.
__device__ __forceinline__ void xcd_walk(unsigned n_items, unsigned* pos, unsigned* end,
                                         unsigned* stride) {
  const unsigned per = gridDim.x / kXcds;
  const unsigned xcd = blockIdx.x % kXcds, slot = blockIdx.x / kXcds;
  const unsigned chunk = (n_items + kXcds - 1) / kXcds;
  const unsigned s = xcd * chunk;
  *pos = s + slot;
  *end = min(s + chunk, n_items);
  *stride = per;
}

struct Counters {
  unsigned inv = 0, dom = 0, nf = 0, fb = 0;
};

__device__ __forceinline__ void flush_counters(Status* st, const Counters& c) {
  if (c.inv) atomicAdd(&st->n_inverted, (unsigned long long)c.inv);
  if (c.dom) atomicAdd(&st->n_domain, (unsigned long long)c.dom);
  if (c.nf) atomicAdd(&st->n_nonfinite, (unsigned long long)c.nf);
  if (c.fb) atomicAdd(&st->n_fallback, (unsigned long long)c.fb);
}

// Base node and fractional offsets of a particle; false if the 3x3x3
// stencil is not inside [0, n-1]^3 (or x is not finite).
__device__ __forceinline__ bool particle_stencil(const SimK& s, const float* x, int* base, float* f) {
  bool ok = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float r = x[a] * s.inv_dx;
    const float b = floorf(r - 0.5f);
    ok = ok && (b >= 0.0f) && (b + 2.0f <= (float)(s.n - 1));
    base[a] = ok ? (int)b : 0;
    f[a] = r - b;
  }
  return ok;
}

// ------------------------------------------------------------------ fallbacks
// P2G of one particle straight into the global accumulator; claims every
// block its stencil touches that the current binning did not activate.
__device__ __forceinline__ void p2g_global(const SimK& s, const int* base, const float (*w)[3],
                                        const float* q, const float* Adx, float4* acc,
                                        uint32_t* mark, uint32_t* ovf, Status* st, int parity) {
#pragma unroll
  for (int ox = 0; ox < 3; ++ox)
#pragma unroll
    for (int oy = 0; oy < 3; ++oy)
#pragma unroll
      for (int oz = 0; oz < 3; ++oz) {
        const float N = w[0][ox] * w[1][oy] * w[2][oz];
        const float fo[3] = {(float)ox, (float)oy, (float)oz};
        float val[3];
        for (int a = 0; a < 3; ++a)
          val[a] = q[a] + Adx[3 * a] * fo[0] + Adx[3 * a + 1] * fo[1] + Adx[3 * a + 2] * fo[2];
        const int g = grid_index(base[0] + ox, base[1] + oy, base[2] + oz, s.nb);
        unsafeAtomicAdd(&acc[g].x, N * s.mass);
        unsafeAtomicAdd(&acc[g].y, N * val[0]);
        unsafeAtomicAdd(&acc[g].z, N * val[1]);
        unsafeAtomicAdd(&acc[g].w, N * val[2]);
      }
  const int b0[3] = {base[0] >> kTileLog2, base[1] >> kTileLog2, base[2] >> kTileLog2};
  const int b1[3] = {(base[0] + 2) >> kTileLog2, (base[1] + 2) >> kTileLog2, (base[2] + 2) >> kTileLog2};
  for (int bz = b0[2]; bz <= b1[2]; ++bz)
    for (int by = b0[1]; by <= b1[1]; ++by)
      for (int bx = b0[0]; bx <= b1[0]; ++bx) {
        const unsigned b = (unsigned)((bz * s.nb + by) * s.nb + bx);
        if (__hip_atomic_load(&mark[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) continue;
        if (atomicCAS(&mark[b], 0u, 2u) == 0u) {
          const unsigned slot = atomicAdd(&st->ovf_count[parity], 1u);
          ovf[slot] = b;
        }
      }
}

// G2P of one particle from the global velocity grid.
__device__ __forceinline__ void g2p_global(const SimK& s, const int* base, const float (*w)[3],
                                        const float4* vel, float* S, float* T) {
  for (int i = 0; i < 3; ++i) S[i] = 0.0f;
  for (int i = 0; i < 9; ++i) T[i] = 0.0f;
#pragma unroll
  for (int ox = 0; ox < 3; ++ox)
#pragma unroll
    for (int oy = 0; oy < 3; ++oy)
#pragma unroll
      for (int oz = 0; oz < 3; ++oz) {
        const float N = w[0][ox] * w[1][oy] * w[2][oz];
        const float4 vv = vel[grid_index(base[0] + ox, base[1] + oy, base[2] + oz, s.nb)];
        const float nv[3] = {N * vv.x, N * vv.y, N * vv.z};
        for (int a = 0; a < 3; ++a) {
          S[a] += nv[a];
          T[3 * a + 0] += nv[a] * (float)ox;
          T[3 * a + 1] += nv[a] * (float)oy;
          T[3 * a + 2] += nv[a] * (float)oz;
        }
      }
}

// ------------------------------------------------------------------ per particle
struct Lds {
  float4 v[kSpanNodes];     // staged grid velocity
  float m[kSpanNodes];      // accumulated mass
  float p0[kSpanNodes], p1[kSpanNodes], p2[kSpanNodes];  // accumulated momentum
};

__device__ __forceinline__ int lds_index(int lx, int ly, int lz) {
  return (lz * kSpan + ly) * kSpan + lx;
}

// P2G of one particle (Algorithm 1, first loop): mass N m and momentum
// N [m v + (m C - dt V0 (4/dx^2) tau)(x_I - x_p)] to each of the 27 nodes.
__device__ __forceinline__ void p2g_particle(const SimK& s, const float* x, const float* v,
                                             const float* C, const float* F, float E,
                                             const int* to, Lds& L, float4* acc, uint32_t* mark,
                                             uint32_t* ovf, Status* st, int parity, Counters& cnt) {
  int base[3];
  float f[3];
  if (!particle_stencil(s, x, base, f)) {
    if (isfinite(x[0] + x[1] + x[2]))
      cnt.dom++;
    else
      cnt.nf++;
    return;
  }
  float w[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) bspline_w(f[a], w[a]);
  float tau[9];
  bool inv;
  kirchhoff(F, s.c_mu * E, s.c_la * E, tau, &inv);
  float A[9];
  float chk = v[0] + v[1] + v[2];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    A[i] = s.mass * C[i] - s.p2g_stress * tau[i];
    chk += A[i];
  }
  if (!isfinite(chk)) {
    cnt.nf++;
    return;
  }
  if (inv) cnt.inv++;
  // m v + A (x_I - x_p) = q + A o dx with q = m v - A f dx.
  float q[3], Adx[9];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    q[a] = s.mass * v[a] - (A[3 * a] * f[0] + A[3 * a + 1] * f[1] + A[3 * a + 2] * f[2]) * s.dx;
#pragma unroll
    for (int b = 0; b < 3; ++b) Adx[3 * a + b] = A[3 * a + b] * s.dx;
  }
  const int l0 = base[0] - to[0], l1 = base[1] - to[1], l2 = base[2] - to[2];
  const bool in_tile = ((unsigned)l0 <= (unsigned)(kSpan - 3)) && ((unsigned)l1 <= (unsigned)(kSpan - 3)) &&
                       ((unsigned)l2 <= (unsigned)(kSpan - 3));
  if (!in_tile) {
    cnt.fb++;
    p2g_global(s, base, w, q, Adx, acc, mark, ovf, st, parity);
    return;
  }
#pragma unroll
  for (int ox = 0; ox < 3; ++ox) {
    float qx[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) qx[a] = q[a] + Adx[3 * a] * (float)ox;
#pragma unroll
    for (int oy = 0; oy < 3; ++oy) {
      float qy[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) qy[a] = qx[a] + Adx[3 * a + 1] * (float)oy;
      const float wxy = w[0][ox] * w[1][oy];
#pragma unroll
      for (int oz = 0; oz < 3; ++oz) {
        const float N = wxy * w[2][oz];
        const int idx = lds_index(l0 + ox, l1 + oy, l2 + oz);
        atomicAdd(&L.m[idx], N * s.mass);
        atomicAdd(&L.p0[idx], N * (qy[0] + Adx[2] * (float)oz));
        atomicAdd(&L.p1[idx], N * (qy[1] + Adx[5] * (float)oz));
        atomicAdd(&L.p2[idx], N * (qy[2] + Adx[8] * (float)oz));
      }
    }
  }
}

// G2P of one particle (Algorithm 1, third loop): v' = sum N v_I,
// C' = (4/dx^2) sum N v_I (x_I - x_p)^T. Returns false if the stencil is
// outside the grid (the particle is then left unchanged).
__device__ __forceinline__ bool g2p_particle(const SimK& s, const float* x, const int* to,
                                             const Lds& L, const float4* vel, float* vn, float* Cn,
                                             Counters& cnt) {
  int base[3];
  float f[3];
  if (!particle_stencil(s, x, base, f)) return false;
  float w[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) bspline_w(f[a], w[a]);
  float S[3] = {0.0f, 0.0f, 0.0f};
  float T[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};  // T[a][b] = sum N v_a o_b
  const int l0 = base[0] - to[0], l1 = base[1] - to[1], l2 = base[2] - to[2];
  const bool in_tile = ((unsigned)l0 <= (unsigned)(kSpan - 3)) && ((unsigned)l1 <= (unsigned)(kSpan - 3)) &&
                       ((unsigned)l2 <= (unsigned)(kSpan - 3));
  if (in_tile) {
#pragma unroll
    for (int ox = 0; ox < 3; ++ox)
#pragma unroll
      for (int oy = 0; oy < 3; ++oy) {
        const float wxy = w[0][ox] * w[1][oy];
#pragma unroll
        for (int oz = 0; oz < 3; ++oz) {
          const float N = wxy * w[2][oz];
          const float4 vv = L.v[lds_index(l0 + ox, l1 + oy, l2 + oz)];
          const float nv[3] = {N * vv.x, N * vv.y, N * vv.z};
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            S[a] += nv[a];
            if (ox) T[3 * a + 0] += nv[a] * (float)ox;
            if (oy) T[3 * a + 1] += nv[a] * (float)oy;
            if (oz) T[3 * a + 2] += nv[a] * (float)oz;
          }
        }
      }
  } else {
    cnt.fb++;
    g2p_global(s, base, w, vel, S, T);
  }
  const float k = 4.0f * s.inv_dx;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    vn[a] = S[a];
#pragma unroll
    for (int b = 0; b < 3; ++b) Cn[3 * a + b] = k * (T[3 * a + b] - S[a] * f[b]);
  }
  return true;
}

// ------------------------------------------------------------------ tile helpers
__device__ __forceinline__ void block_origin(const SimK& s, unsigned b, int* to) {
  const int bi = (int)(b % (unsigned)s.nb);
  const int bj = (int)((b / (unsigned)s.nb) % (unsigned)s.nb);
  const int bk = (int)(b / ((unsigned)s.nb * (unsigned)s.nb));
  to[0] = bi * kTile - kSlack;
  to[1] = bj * kTile - kSlack;
  to[2] = bk * kTile - kSlack;
}

__device__ __forceinline__ void tile_clear(Lds& L) {
  for (int i = threadIdx.x; i < kSpanNodes; i += blockDim.x) {
    L.m[i] = 0.0f;
    L.p0[i] = 0.0f;
    L.p1[i] = 0.0f;
    L.p2[i] = 0.0f;
  }
}

__device__ __forceinline__ void tile_stage_velocity(const SimK& s, const int* to, const float4* vel,
                                                    Lds& L) {
  for (int i = threadIdx.x; i < kSpanNodes; i += blockDim.x) {
    const int lx = i % kSpan, ly = (i / kSpan) % kSpan, lz = i / (kSpan * kSpan);
    const int gx = to[0] + lx, gy = to[1] + ly, gz = to[2] + lz;
    float4 val = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if ((unsigned)gx < (unsigned)s.n && (unsigned)gy < (unsigned)s.n && (unsigned)gz < (unsigned)s.n)
      val = vel[grid_index(gx, gy, gz, s.nb)];
    L.v[i] = val;
  }
}

// Non-empty tile nodes -> global accumulator.
__device__ __forceinline__ void tile_flush(const SimK& s, const int* to, const Lds& L, float4* acc) {
  for (int i = threadIdx.x; i < kSpanNodes; i += blockDim.x) {
    const float m = L.m[i];
    if (m == 0.0f) continue;
    const int lx = i % kSpan, ly = (i / kSpan) % kSpan, lz = i / (kSpan * kSpan);
    const int gx = to[0] + lx, gy = to[1] + ly, gz = to[2] + lz;
    // Only in-grid nodes can carry mass (stencils are checked against the
    // grid); the test keeps the index in range regardless.
    if ((unsigned)gx >= (unsigned)s.n || (unsigned)gy >= (unsigned)s.n || (unsigned)gz >= (unsigned)s.n) continue;
    const int g = grid_index(gx, gy, gz, s.nb);
    unsafeAtomicAdd(&acc[g].x, m);
    unsafeAtomicAdd(&acc[g].y, L.p0[i]);
    unsafeAtomicAdd(&acc[g].z, L.p1[i]);
    unsafeAtomicAdd(&acc[g].w, L.p2[i]);
  }
}

__device__ __forceinline__ float particle_E(const SimK& s, const float* __restrict__ part, int64_t cap,
                                            unsigned p) {
  return s.has_E ? part[FE * cap + p] : s.E_default;
}

// ------------------------------------------------------------------ kernels
// P2G from the materialised particle state (first substep after binning).
__global__ __launch_bounds__(kWG) void k_p2g(const float* __restrict__ part, int64_t cap,
                                             const uint32_t* __restrict__ blk_begin,
                                             const uint32_t* __restrict__ blk_end,
                                             const uint32_t* __restrict__ occ_list, Status* st,
                                             float4* acc, uint32_t* mark, uint32_t* ovf, int parity,
                                             SimK s) {
  __shared__ Lds L;
  Counters cnt;
  unsigned pos, end, stride;
  xcd_walk(st->n_occ, &pos, &end, &stride);
  for (; pos < end; pos += stride) {
    const unsigned b = occ_list[pos];
    int to[3];
    block_origin(s, b, to);
    tile_clear(L);
    __syncthreads();
    const unsigned pe = blk_end[b];
    for (unsigned p = blk_begin[b] + threadIdx.x; p < pe; p += kWG) {
      float x[3], v[3], C[9], F[9];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        x[a] = part[(FX + a) * cap + p];
        v[a] = part[(FV + a) * cap + p];
      }
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        C[i] = part[(FC + i) * cap + p];
        F[i] = part[(FF + i) * cap + p];
      }
      p2g_particle(s, x, v, C, F, particle_E(s, part, cap, p), to, L, acc, mark, ovf, st, parity, cnt);
    }
    __syncthreads();
    tile_flush(s, to, L, acc);
    __syncthreads();
  }
  flush_counters(st, cnt);
}

// Fused G2P (substep k-1) -> F, x update -> stress -> P2G (substep k).
__global__ __launch_bounds__(kWG) void k_g2p2g(float* __restrict__ part, int64_t cap,
                                               const uint32_t* __restrict__ blk_begin,
                                               const uint32_t* __restrict__ blk_end,
                                               const uint32_t* __restrict__ occ_list, Status* st,
                                               float4* acc, const float4* __restrict__ vel,
                                               uint32_t* mark, uint32_t* ovf, int parity, SimK s) {
  __shared__ Lds L;
  Counters cnt;
  unsigned pos, end, stride;
  xcd_walk(st->n_occ, &pos, &end, &stride);
  for (; pos < end; pos += stride) {
    const unsigned b = occ_list[pos];
    int to[3];
    block_origin(s, b, to);
    tile_stage_velocity(s, to, vel, L);
    tile_clear(L);
    __syncthreads();
    const unsigned pe = blk_end[b];
    for (unsigned p = blk_begin[b] + threadIdx.x; p < pe; p += kWG) {
      float x[3], F[9];
#pragma unroll
      for (int a = 0; a < 3; ++a) x[a] = part[(FX + a) * cap + p];
#pragma unroll
      for (int i = 0; i < 9; ++i) F[i] = part[(FF + i) * cap + p];
      float vn[3], Cn[9];
      if (!g2p_particle(s, x, to, L, vel, vn, Cn, cnt)) continue;  // frozen (out of grid)
      float Fn[9];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b2 = 0; b2 < 3; ++b2)
          Fn[3 * a + b2] = F[3 * a + b2] + s.dt * (Cn[3 * a] * F[b2] + Cn[3 * a + 1] * F[3 + b2] +
                                                   Cn[3 * a + 2] * F[6 + b2]);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        x[a] += s.dt * vn[a];
        part[(FX + a) * cap + p] = x[a];
      }
#pragma unroll
      for (int i = 0; i < 9; ++i) part[(FF + i) * cap + p] = Fn[i];
      p2g_particle(s, x, vn, Cn, Fn, particle_E(s, part, cap, p), to, L, acc, mark, ovf, st, parity,
                   cnt);
    }
    __syncthreads();
    tile_flush(s, to, L, acc);
    __syncthreads();
  }
  flush_counters(st, cnt);
}

// G2P that materialises the full state (x, v, C, F) in memory.
__global__ __launch_bounds__(kWG) void k_g2p(float* __restrict__ part, int64_t cap,
                                             const uint32_t* __restrict__ blk_begin,
                                             const uint32_t* __restrict__ blk_end,
                                             const uint32_t* __restrict__ occ_list, Status* st,
                                             const float4* __restrict__ vel, SimK s) {
  __shared__ Lds L;
  Counters cnt;
  unsigned pos, end, stride;
  xcd_walk(st->n_occ, &pos, &end, &stride);
  for (; pos < end; pos += stride) {
    const unsigned b = occ_list[pos];
    int to[3];
    block_origin(s, b, to);
    tile_stage_velocity(s, to, vel, L);
    __syncthreads();
    const unsigned pe = blk_end[b];
    for (unsigned p = blk_begin[b] + threadIdx.x; p < pe; p += kWG) {
      float x[3], F[9];
#pragma unroll
      for (int a = 0; a < 3; ++a) x[a] = part[(FX + a) * cap + p];
#pragma unroll
      for (int i = 0; i < 9; ++i) F[i] = part[(FF + i) * cap + p];
      float vn[3], Cn[9];
      if (!g2p_particle(s, x, to, L, vel, vn, Cn, cnt)) continue;
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b2 = 0; b2 < 3; ++b2)
          part[(FF + 3 * a + b2) * cap + p] =
              F[3 * a + b2] +
              s.dt * (Cn[3 * a] * F[b2] + Cn[3 * a + 1] * F[3 + b2] + Cn[3 * a + 2] * F[6 + b2]);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        part[(FX + a) * cap + p] = x[a] + s.dt * vn[a];
        part[(FV + a) * cap + p] = vn[a];
      }
#pragma unroll
      for (int i = 0; i < 9; ++i) part[(FC + i) * cap + p] = Cn[i];
    }
    __syncthreads();
  }
  flush_counters(st, cnt);
}

// ------------------------------------------------------------------ launchers
void launch_p2g(Buffers& b, int64_t N, const SimK& s, int parity, int grid_wgs, hipStream_t st) {
  (void)N;
  hipLaunchKernelGGL(k_p2g, dim3(grid_wgs), dim3(kWG), 0, st, b.part[b.cur], b.cap, b.blk_begin,
                     b.blk_end, b.occ_list, b.status, b.acc, b.mark, b.ovf_list[parity], parity, s);
}

void launch_g2p2g(Buffers& b, int64_t N, const SimK& s, int parity, int grid_wgs, hipStream_t st) {
  (void)N;
  hipLaunchKernelGGL(k_g2p2g, dim3(grid_wgs), dim3(kWG), 0, st, b.part[b.cur], b.cap, b.blk_begin,
                     b.blk_end, b.occ_list, b.status, b.acc, b.vel, b.mark, b.ovf_list[parity],
                     parity, s);
}

void launch_g2p(Buffers& b, int64_t N, const SimK& s, int grid_wgs, hipStream_t st) {
  (void)N;
  hipLaunchKernelGGL(k_g2p, dim3(grid_wgs), dim3(kWG), 0, st, b.part[b.cur], b.cap, b.blk_begin,
                     b.blk_end, b.occ_list, b.status, b.vel, s);
}

}  // namespace mpm
