// Particle <-> grid transfers of the MPM substep (CRESSim-MPM Sec. III-B,
// Algorithm 1, and the solver variants of Sec. III-A and III-C), tiled for
// CDNA4.
//
// Particles are binned by the work tile of their base cell: a cube of T = 8
// cells (one grid block) or T = 4 cells (one of its eight sub-blocks). The
// kernels are templates on T; a 4-cell tile is worked by 128-thread
// workgroups with a 6^3-node LDS tile, an 8-cell tile by 512-thread
// workgroups with a 10^3-node tile. One workgroup owns one work item at a
// time (a tile's particles, or a run of s.item_particles of them when the
// tile is dense): it stages the grid velocities of the tile's (T + 2)^3 nodes
// (the stencils of its cells) in LDS, gathers (G2P) from LDS, scatters (P2G)
// into an LDS accumulator tile with integer LDS atomics, then flushes the
// non-empty tile nodes into the global accumulator (FP32 or integer atomics,
// one per value). A particle whose stencil has drifted out of the tile since
// binning takes a global-memory path with the same integer contributions
// and claims the grid blocks it touches for the grid update (overflow list).
//
// P2G accumulates integers because LDS float atomics are slow on gfx950 while
// ds_add_u32 / ds_add_u64 run near LDS bandwidth; integer sums are also exact,
// so the result does not depend on the order of the atomics (nor on the tile
// edge). Weights are u32 in 2^-22 units: one work item (at most kItemMax
// particles, each adding at most 0.75^3 to a node) cannot carry a node's sum
// past 2^32 - 1. Momentum is int64 in fixed units, except in the FP32 mode of
// MLS-MPM, whose tile packs each node into two 64-bit words of 32-bit fields
// at a unit chosen per work item (the packed P2G below): 2 LDS atomics per
// node instead of 4.
//
// k_g2p2g fuses the G2P of substep k-1 with the P2G of substep k: v and C never
// leave registers between the two, so a fused substep streams x, F, E in and
// x, F out (100 B/particle). When a tool pushes particles out, an
// instantiation with the push-out after the position update runs instead. A
// dense tile's work items deal their particles to a wave's lanes kWG / 64
// apart (item_lane), so that one wave's atomics spread over different cells.

#include "mpm_device.h"
#include "mpm_internal.h"
#include "p2g_fixed.h"

namespace mpm {

// Work distribution of the persistent transfer kernels (a grid size that is
// a multiple of kXcds). XCD x owns the x-th contiguous eighth of the
// spatially ordered work list, so tiles that share halo nodes share an L2.
// Workgroup w starts at item w / kXcds of its XCD's range; after that, the
// XCD's workgroups claim the range's next unclaimed item from a counter, so
// a workgroup that drew items of sparse tiles (tens of particles against up
// to a few thousand in a dense one) takes more of them. Thread 0 claims and
// hands the item to its workgroup through LDS; every workgroup calls finish
// once, after its last claim.
struct WorkWalk {
  unsigned begin, end, xcd, per;
  __device__ __forceinline__ explicit WorkWalk(unsigned n_items) {
    per = gridDim.x / kXcds;
    xcd = blockIdx.x % kXcds;
    const unsigned chunk = (n_items + kXcds - 1) / kXcds;
    begin = min(xcd * chunk, n_items);
    end = min(begin + chunk, n_items);
  }
  __device__ __forceinline__ unsigned first() const { return begin + blockIdx.x / kXcds; }
  __device__ __forceinline__ unsigned claim(Status* st) const {
    return begin + per + atomicAdd(&st->claim[xcd], 1u);
  }
  // The last workgroup of the XCD to finish puts the counters back to zero
  // for the next launch (all claims of the others are done by then).
  __device__ __forceinline__ void finish(Status* st) const {
    if (atomicAdd(&st->claim_done[xcd], 1u) == per - 1u) {
      atomicExch(&st->claim[xcd], 0u);
      atomicExch(&st->claim_done[xcd], 0u);
    }
  }
};

// This thread's position in each run of kWG particles of a work item: its
// own index, or for a dense tile's items (kDenseFlag) lane l of wave w takes
// position l * (kWG / 64) + w, so one wave's 64 particles lie kWG / 64 apart
// in the tile's order (different cells) instead of side by side.
template <int T>
__device__ __forceinline__ unsigned item_lane(unsigned tagged_unit) {
  constexpr unsigned kWG = TileShape<T>::kWG;
  return (tagged_unit & kDenseFlag) ? (threadIdx.x & 63u) * (kWG / 64) + (threadIdx.x >> 6) : threadIdx.x;
}

struct Counters {
  unsigned inv = 0, dom = 0, nf = 0, fb = 0, rng = 0;
};

// Events of one particle as bits of one word, added to the thread's Counters
// once per particle. The per-particle code sets bits of a single scalar: had
// it incremented different Counters fields on different paths, the compiler
// could merge those increments into one store through a computed field
// offset, leaving Counters as a per-thread array that it then places in LDS
// (indexed by the flat work-item id, read from the dispatch packet).
enum : unsigned { kEvInv = 1u, kEvDom = 2u, kEvNf = 4u, kEvRng = 8u, kEvFbG2P = 16u, kEvFbP2G = 32u };

__device__ __forceinline__ void count_events(Counters& c, unsigned ev) {
  c.inv += ev & 1u;
  c.dom += (ev >> 1) & 1u;
  c.nf += (ev >> 2) & 1u;
  c.rng += (ev >> 3) & 1u;
  c.fb += ((ev >> 4) & 1u) + ((ev >> 5) & 1u);
}

__device__ __forceinline__ void flush_counters(Status* st, const Counters& c) {
  if (c.inv) atomicAdd(&st->n_inverted, (unsigned long long)c.inv);
  if (c.dom) atomicAdd(&st->n_domain, (unsigned long long)c.dom);
  if (c.nf) atomicAdd(&st->n_nonfinite, (unsigned long long)c.nf);
  if (c.fb) atomicAdd(&st->n_fallback, (unsigned long long)c.fb);
  if (c.rng) atomicAdd(&st->n_range, (unsigned long long)c.rng);
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

// Per-particle inputs of the standard-MPM scatter (Sec. III-A): weights,
// their derivatives, m v and the internal-force impulse coefficients
// tk = (dt V0 / dx) tau, so that node I receives N m v - tk (grad N dx) with
// grad N dx = (w'_x w_y w_z, w_x w'_y w_z, w_x w_y w'_z).
struct PICIn {
  int base[3];
  float w[3][3], dw[3][3];
  float mv[3];
  float tk[9];
  double fx_p;
};

template <class Sink>
__device__ __forceinline__ void p2g_emit(const PICIn& P, Sink&& sink) {
  // The x weights of the current offset move down a register queue, so the
  // non-unrolled loop indexes no array.
  float wx = P.w[0][0], wx1 = P.w[0][1], wx2 = P.w[0][2];
  float dwx = P.dw[0][0], dwx1 = P.dw[0][1], dwx2 = P.dw[0][2];
#pragma unroll 1
  for (int ox = 0; ox < 3; ++ox) {
#pragma unroll
    for (int oy = 0; oy < 3; ++oy) {
      const float wxy = wx * P.w[1][oy], dxy = dwx * P.w[1][oy], xdy = wx * P.dw[1][oy];
#pragma unroll
      for (int oz = 0; oz < 3; ++oz) {
        const float N = wxy * P.w[2][oz];
        const float g0 = dxy * P.w[2][oz], g1 = xdy * P.w[2][oz], g2 = wxy * P.dw[2][oz];
        const uint32_t wq = (uint32_t)fmaf(N, kWeightUnits, 0.5f);
        long long q[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const float val = N * P.mv[a] - (P.tk[3 * a] * g0 + P.tk[3 * a + 1] * g1 + P.tk[3 * a + 2] * g2);
          q[a] = fx_mul((double)val, P.fx_p);
        }
        sink(ox, oy, oz, wq, q[0], q[1], q[2]);
      }
    }
    wx = wx1;
    wx1 = wx2;
    dwx = dwx1;
    dwx1 = dwx2;
  }
}

// ------------------------------------------------------------------ global accumulator
// Channel types of the global accumulator: FP32 sums, or exact integer sums
// (weights in 2^-22 units as u32, momentum in 2^-fx_shift units as int64).
template <bool FIXED> struct AccT;
template <> struct AccT<false> {
  using M = float;
  using P = float;
};
template <> struct AccT<true> {
  using M = uint32_t;
  using P = long long;
};

template <bool FIXED>
__device__ __forceinline__ void acc_add(const SimK& s, typename AccT<FIXED>::M* am, typename AccT<FIXED>::P* ap0,
                                        typename AccT<FIXED>::P* ap1, typename AccT<FIXED>::P* ap2, int g,
                                        uint32_t wq, long long p0, long long p1, long long p2) {
  if constexpr (FIXED) {
    atomicAdd(am + g, wq);
    atomicAdd((unsigned long long*)ap0 + g, (unsigned long long)p0);
    atomicAdd((unsigned long long*)ap1 + g, (unsigned long long)p1);
    atomicAdd((unsigned long long*)ap2 + g, (unsigned long long)p2);
  } else {
    unsafeAtomicAdd(am + g, (float)wq * s.m_unit);
    unsafeAtomicAdd(ap0 + g, (float)((double)p0 * s.fx_p_inv));
    unsafeAtomicAdd(ap1 + g, (float)((double)p1 * s.fx_p_inv));
    unsafeAtomicAdd(ap2 + g, (float)((double)p2 * s.fx_p_inv));
  }
}

#define ACC_PARAMS typename AccT<FIXED>::M *__restrict__ am, typename AccT<FIXED>::P *__restrict__ ap0, \
                   typename AccT<FIXED>::P *__restrict__ ap1, typename AccT<FIXED>::P *__restrict__ ap2
#define ACC_ARGS am, ap0, ap1, ap2

// P2G of one particle straight into the global accumulator; claims every
// block its stencil touches that the current binning did not activate.
// Claims every block that the stencil with base node `base` touches and the
// current binning did not activate, for the grid update (overflow list).
__device__ __forceinline__ void claim_stencil_blocks(const SimK& s, const int* base, uint32_t* mark, uint32_t* ovf,
                                                     Status* st, int parity, int scene) {
  // The stencil spans one or two blocks per axis. All their marks are loaded
  // before any is tested, so that the loads overlap instead of each waiting
  // on the previous test.
  const int b0[3] = {base[0] >> kTileLog2, base[1] >> kTileLog2, base[2] >> kTileLog2};
  const int b1[3] = {(base[0] + 2) >> kTileLog2, (base[1] + 2) >> kTileLog2, (base[2] + 2) >> kTileLog2};
  unsigned blk[8], seen[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int bx = b0[0] + (k & 1), by = b0[1] + ((k >> 1) & 1), bz = b0[2] + (k >> 2);
    const bool spans = bx <= b1[0] && by <= b1[1] && bz <= b1[2];
    blk[k] = (unsigned)scene * s.nb3 + (unsigned)((bz * s.nb + by) * s.nb + bx);
    seen[k] = spans ? __hip_atomic_load(&mark[blk[k]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 1u;
  }
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (seen[k] == 0u && atomicCAS(&mark[blk[k]], 0u, 2u) == 0u) {
      const unsigned slot = atomicAdd(&st->ovf_count[parity], 1u);
      ovf[slot] = blk[k];
    }
}

template <bool FIXED, class In>
__device__ __forceinline__ void p2g_global(const SimK& s, const In& P, ACC_PARAMS, uint32_t* mark,
                                        uint32_t* ovf, Status* st, int parity, int scene) {
  const int node_base = scene * s.n3;
  p2g_emit(P, [&](int ox, int oy, int oz, uint32_t wq, long long p0, long long p1, long long p2) {
    const int g = node_base + grid_index(P.base[0] + ox, P.base[1] + oy, P.base[2] + oz, s.nb);
    acc_add<FIXED>(s, ACC_ARGS, g, wq, p0, p1, p2);
  });
  claim_stencil_blocks(s, P.base, mark, ovf, st, parity, scene);
}

// G2P sums of one particle, S = sum N v_I and T[a][b] = sum N v_I[a] o_b, with
// the sum over oz done first for each (ox, oy) (separable weights). `node`
// returns the velocity of stencil node (ox, oy, oz); the LDS and the global
// path share this arithmetic, so both give the same bits.
template <class Node>
__device__ __forceinline__ void g2p_sums(const float (*w)[3], Node&& node, float* S, float* T) {
#pragma unroll
  for (int i = 0; i < 3; ++i) S[i] = 0.0f;
#pragma unroll
  for (int i = 0; i < 9; ++i) T[i] = 0.0f;
  const float wz1 = w[2][1], wz2 = 2.0f * w[2][2];
  // The x offset is a loop variable (not unrolled) to bound the LDS loads in
  // flight and the register use.
#pragma unroll 1
  for (int ox = 0; ox < 3; ++ox) {
    const float wx = ox == 0 ? w[0][0] : (ox == 1 ? w[0][1] : w[0][2]);
    const float fox = (float)ox;
#pragma unroll
    for (int oy = 0; oy < 3; ++oy) {
      const float4 v0 = node(ox, oy, 0), v1 = node(ox, oy, 1), v2 = node(ox, oy, 2);
      float Z0[3], Z1[3];
      Z0[0] = w[2][0] * v0.x + w[2][1] * v1.x + w[2][2] * v2.x;
      Z0[1] = w[2][0] * v0.y + w[2][1] * v1.y + w[2][2] * v2.y;
      Z0[2] = w[2][0] * v0.z + w[2][1] * v1.z + w[2][2] * v2.z;
      Z1[0] = wz1 * v1.x + wz2 * v2.x;
      Z1[1] = wz1 * v1.y + wz2 * v2.y;
      Z1[2] = wz1 * v1.z + wz2 * v2.z;
      const float wxy = wx * w[1][oy];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        S[a] += wxy * Z0[a];
        T[3 * a + 2] += wxy * Z1[a];
        T[3 * a + 0] += (fox * wxy) * Z0[a];
        if (oy) T[3 * a + 1] += ((float)oy * wxy) * Z0[a];
      }
    }
  }
}

// Standard-MPM gather of one particle: S = sum N v_I and
// T[a][b] = sum v_I[a] (grad N dx)[b], with the same separable order as
// g2p_sums (w' are the weight derivatives).
template <class Node>
__device__ __forceinline__ void g2p_sums_pic(const float (*w)[3], const float (*dw)[3], Node&& node, float* S,
                                             float* T) {
#pragma unroll
  for (int i = 0; i < 3; ++i) S[i] = 0.0f;
#pragma unroll
  for (int i = 0; i < 9; ++i) T[i] = 0.0f;
  float wx = w[0][0], wx1 = w[0][1], wx2 = w[0][2];
  float dwx = dw[0][0], dwx1 = dw[0][1], dwx2 = dw[0][2];
#pragma unroll 1
  for (int ox = 0; ox < 3; ++ox) {
#pragma unroll
    for (int oy = 0; oy < 3; ++oy) {
      const float4 v0 = node(ox, oy, 0), v1 = node(ox, oy, 1), v2 = node(ox, oy, 2);
      float Z0[3], Zd[3];
      Z0[0] = w[2][0] * v0.x + w[2][1] * v1.x + w[2][2] * v2.x;
      Z0[1] = w[2][0] * v0.y + w[2][1] * v1.y + w[2][2] * v2.y;
      Z0[2] = w[2][0] * v0.z + w[2][1] * v1.z + w[2][2] * v2.z;
      Zd[0] = dw[2][0] * v0.x + dw[2][1] * v1.x + dw[2][2] * v2.x;
      Zd[1] = dw[2][0] * v0.y + dw[2][1] * v1.y + dw[2][2] * v2.y;
      Zd[2] = dw[2][0] * v0.z + dw[2][1] * v1.z + dw[2][2] * v2.z;
      const float wxy = wx * w[1][oy], dxy = dwx * w[1][oy], xdy = wx * dw[1][oy];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        S[a] += wxy * Z0[a];
        T[3 * a + 0] += dxy * Z0[a];
        T[3 * a + 1] += xdy * Z0[a];
        T[3 * a + 2] += wxy * Zd[a];
      }
    }
    wx = wx1;
    wx1 = wx2;
    dwx = dwx1;
    dwx1 = dwx2;
  }
}

// G2P of one particle from the global velocity grid.
__device__ __forceinline__ void g2p_global(const SimK& s, const int* base, const float (*w)[3],
                                        const float4* vel, float* S, float* T, int scene) {
  const int node_base = scene * s.n3;
  g2p_sums(w, [&](int ox, int oy, int oz) {
    return vel[node_base + grid_index(base[0] + ox, base[1] + oy, base[2] + oz, s.nb)];
  }, S, T);
}

// ------------------------------------------------------------------ per particle
// The LDS tile of a work tile of edge T: (T + 2)^3 nodes, the span of the
// stencils whose base cell lies in the tile. Scatters also have a shell one
// node thick around the span: a particle whose base cell has moved at most
// one cell out of the tile since the binning (base -1 .. T per axis) still
// scatters into LDS instead of global memory. Such particles come in waves
// (a layer of a lattice crossing a block boundary), and their global
// atomics pile up on the same nodes.
template <int T>
struct Lds {
  static constexpr int kNodes = TileShape<T>::kSpanNodes;
  static constexpr int kSpan = TileShape<T>::kSpan;
  static constexpr int kOuter = kSpan + 2;
  static constexpr int kShell = kOuter * kOuter * kOuter - kNodes;
  float4 v[kNodes];                             // staged grid velocity
  // Weight sums (2^-22 units) and momentum (fixed point). The packed tile of
  // the FP32 MLS-MPM kernel holds a node in p0 and p1 (and its shell in sp0
  // and sp1) and keeps the 8-cell tiles' slot table in p2; m, sm and sp2 are
  // then unused.
  uint32_t m[kNodes];
  long long p0[kNodes], p1[kNodes], p2[kNodes];
  uint32_t sm[kShell];                          // the shell's sums
  long long sp0[kShell], sp1[kShell], sp2[kShell];
  // A scatter into the shell copies item_tag (set per work item) into
  // shell_mark, so the flush can tell whether this item used the shell.
  uint32_t item_tag, shell_mark;
  uint32_t claimed[2];  // work items claimed by thread 0 (WorkWalk)
  // Per velocity buffer, per wave: the largest |velocity component| of the
  // nodes the wave staged (the packed scatter's capacity).
  float vw[2][TileShape<T>::kWG / 64];
  unsigned long long pbe[2];  // per velocity buffer: its item's tile bound entry (Buffers::pbound)
};

// Shell node index of tile node (x, y, z), each in [-1, kSpan], at least
// one of them outside [0, kSpan): the two z faces (kOuter^2 nodes each),
// then the two y faces without the z faces (kSpan x kOuter), then the two x
// faces (kSpan^2).
template <int T>
__device__ __forceinline__ int shell_index(int x, int y, int z) {
  constexpr int S = Lds<T>::kSpan, A = Lds<T>::kOuter;
  if (z < 0) return (y + 1) * A + (x + 1);
  if (z >= S) return A * A + (y + 1) * A + (x + 1);
  if (y < 0) return 2 * A * A + z * A + (x + 1);
  if (y >= S) return 2 * A * A + S * A + z * A + (x + 1);
  if (x < 0) return 2 * A * A + 2 * S * A + z * S + y;
  return 2 * A * A + 2 * S * A + S * S + z * S + y;
}

// Tile node (x, y, z) of shell node j (the inverse of shell_index).
template <int T>
__device__ __forceinline__ void shell_node(int j, int* x, int* y, int* z) {
  constexpr int S = Lds<T>::kSpan, A = Lds<T>::kOuter;
  if (j < 2 * A * A) {
    *z = j < A * A ? -1 : S;
    j %= A * A;
    *y = j / A - 1;
    *x = j % A - 1;
  } else if ((j -= 2 * A * A) < 2 * S * A) {
    *y = j < S * A ? -1 : S;
    j %= S * A;
    *z = j / A;
    *x = j % A - 1;
  } else {
    j -= 2 * S * A;
    *x = j < S * S ? -1 : S;
    j %= S * S;
    *z = j / S;
    *y = j % S;
  }
}

template <int T>
__device__ __forceinline__ int lds_index(int lx, int ly, int lz) {
  constexpr int S = TileShape<T>::kSpan;
  return (lz * S + ly) * S + lx;
}

// Whether a stencil with base node `l` (tile coordinates) lies in the tile.
template <int T>
__device__ __forceinline__ bool in_tile(int l0, int l1, int l2) {
  constexpr unsigned kMax = TileShape<T>::kSpan - 3;
  return ((unsigned)l0 <= kMax) && ((unsigned)l1 <= kMax) && ((unsigned)l2 <= kMax);
}

// Commit one particle's scatter: into the LDS tile when its stencil lies in
// the block's tile, else straight into the global accumulator.
template <bool FIXED, int T, bool SHELL, class In>
__device__ __forceinline__ void p2g_commit(const SimK& s, const In& P, const int* to, Lds<T>& L, ACC_PARAMS,
                                           uint32_t* mark, uint32_t* ovf, Status* st, int parity, unsigned& ev) {
  const int l0 = P.base[0] - to[0], l1 = P.base[1] - to[1], l2 = P.base[2] - to[2];
  if (!in_tile<T>(l0, l1, l2)) {
    constexpr unsigned kMarginMax = T + 1;  // base -1 .. T, shifted by one
    if (!SHELL || (unsigned)(l0 + 1) > kMarginMax || (unsigned)(l1 + 1) > kMarginMax ||
        (unsigned)(l2 + 1) > kMarginMax) {
      ev |= kEvFbP2G;
      p2g_global<FIXED>(s, P, ACC_ARGS, mark, ovf, st, parity, to[3]);
      return;
    }
    // One cell out: the nodes in the span go to the tile, the others to the
    // shell. (The PB-MPM and push-out variants leave this to the global path:
    // the shell's code does not fit their registers at 4 waves per SIMD.)
    constexpr int S = TileShape<T>::kSpan;
    L.shell_mark = L.item_tag;
    p2g_emit(P, [&](int ox, int oy, int oz, uint32_t wq, long long p0, long long p1, long long p2) {
      const int x = l0 + ox, y = l1 + oy, z = l2 + oz;
      uint32_t* m;
      unsigned long long *a0, *a1, *a2;
      if ((unsigned)x < (unsigned)S && (unsigned)y < (unsigned)S && (unsigned)z < (unsigned)S) {
        const int idx = lds_index<T>(x, y, z);
        m = &L.m[idx];
        a0 = (unsigned long long*)&L.p0[idx];
        a1 = (unsigned long long*)&L.p1[idx];
        a2 = (unsigned long long*)&L.p2[idx];
      } else {
        const int j = shell_index<T>(x, y, z);
        m = &L.sm[j];
        a0 = (unsigned long long*)&L.sp0[j];
        a1 = (unsigned long long*)&L.sp1[j];
        a2 = (unsigned long long*)&L.sp2[j];
      }
      atomicAdd(m, wq);
      atomicAdd(a0, (unsigned long long)p0);
      atomicAdd(a1, (unsigned long long)p1);
      atomicAdd(a2, (unsigned long long)p2);
    });
    return;
  }
  const int l = lds_index<T>(l0, l1, l2);
  p2g_emit(P, [&](int ox, int oy, int oz, uint32_t wq, long long p0, long long p1, long long p2) {
    const int idx = l + lds_index<T>(ox, oy, oz);
    atomicAdd(&L.m[idx], wq);
    atomicAdd((unsigned long long*)&L.p0[idx], (unsigned long long)p0);
    atomicAdd((unsigned long long*)&L.p1[idx], (unsigned long long)p1);
    atomicAdd((unsigned long long*)&L.p2[idx], (unsigned long long)p2);
  });
}

// P2G of one particle with the APIC affine momentum (Algorithm 1, first
// loop): weight N and momentum N [m v + A (x_I - x_p)] to each of the 27
// nodes, where
//   MLS-MPM: A = m C - dt V0 (4/dx^2) tau (fixed-corotated tau);
//   PB-MPM:  A = m C' with C' the constraint projection of C (Sec. III-C);
//            on the first pass of a step v also receives dt g.
// The PB-MPM iterations after the first count no errors (the first pass of
// the step has counted them).
// `bmax` takes the largest contribution bound of the particles scattered.
template <bool FIXED, int SOL, int PASS, int T, bool SHELL>
__device__ __forceinline__ void p2g_particle(const SimK& s, const float* x, const float* v, const float* C,
                                             const float* F, float E, const int* to, Lds<T>& L, ACC_PARAMS,
                                             uint32_t* mark, uint32_t* ovf, Status* st, int parity, unsigned& ev,
                                             float& bmax) {
  constexpr bool kCount = !(SOL == SOLVER_PB && PASS == PB_ITER);
  P2GIn P;
  float f[3];
  if (!particle_stencil(s, x, P.base, f)) {
    if (kCount) {
      if (isfinite(x[0] + x[1] + x[2]))
        ev |= kEvDom;
      else
        ev |= kEvNf;
    }
    return;
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) bspline_w(f[a], P.w[a]);
  float Af[9];
  float vp[3];
  bool inv;
  if constexpr (SOL == SOLVER_MLS) {
    float tau[9];
    kirchhoff(F, s.c_mu * E, s.c_la * E, tau, &inv);
#pragma unroll
    for (int i = 0; i < 9; ++i) Af[i] = s.mass * C[i] - s.p2g_stress * tau[i];
#pragma unroll
    for (int a = 0; a < 3; ++a) vp[a] = v[a];
  } else {
    float Cc[9];
    const float J = pb_constraint(F, C, s.dt, s.pb_beta, Cc);
    inv = !(J > 0.0f);
#pragma unroll
    for (int i = 0; i < 9; ++i) Af[i] = s.mass * Cc[i];
#pragma unroll
    for (int a = 0; a < 3; ++a) vp[a] = PASS == PB_FIRST ? v[a] + s.dt * s.g[a] : v[a];
  }
  float chk = vp[0] + vp[1] + vp[2];
#pragma unroll
  for (int i = 0; i < 9; ++i) chk += Af[i];
  if (!isfinite(chk)) {
    if (kCount) ev |= kEvNf;
    return;
  }
  if (kCount && inv) ev |= kEvInv;
  // Bound of |m v + A (x_I - x_p)| over the stencil (|x_I - x_p| <= 1.5 dx
  // per axis): contributions beyond the fixed-point range are refused.
  float bound = 0.0f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float row = fabsf(Af[3 * a]) + fabsf(Af[3 * a + 1]) + fabsf(Af[3 * a + 2]);
    bound = fmaxf(bound, fabsf(s.mass * vp[a]) + 1.5f * s.dx * row);
  }
  if (!(bound < s.p_limit)) {
    ev |= kEvRng;
    return;
  }
  bmax = fmaxf(bmax, bound);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float qa = s.mass * vp[a] - (Af[3 * a] * f[0] + Af[3 * a + 1] * f[1] + Af[3 * a + 2] * f[2]) * s.dx;
    P.q[a] = (double)qa * s.fx_p;
#pragma unroll
    for (int b = 0; b < 3; ++b) P.Adx[3 * a + b] = (double)(Af[3 * a + b] * s.dx) * s.fx_p;
  }
  p2g_commit<FIXED, T, SHELL>(s, P, to, L, ACC_ARGS, mark, ovf, st, parity, ev);
}

// ------------------------------------------------------------------ packed P2G
// FP32 accumulation, MLS-MPM: the LDS tile holds each node as two 64-bit
// words, (p1, p0) and (p2, weight), every field a 32-bit integer, so that a
// node takes 2 LDS atomics instead of 4. The momentum fields count units of
// 2^e kg m/s, with e chosen per work item (item_scale) so that no node sum of
// the item can leave 32 bits. The scale comes from a capacity: 1.25 times the
// larger of the tile's largest contribution bound in the previous substep
// (Buffers::pbound) and the particle mass times the largest staged grid
// velocity. A particle whose own bound exceeds the capacity scatters into the
// global accumulator instead, so no sum can wrap whatever the estimate said.
// A contribution is rounded to an integer by one FP32 fma with 1.5 * 2^23. Two such biased words, less the doubled bias in one 64-bit
// subtraction, give hi 2^32 + lo with lo signed; 64-bit sums of such words
// decode into the exact sums of both fields while each stays within 32 bits.
// The weight field is unsigned and needs no bias.
constexpr float kMagicF = 12582912.0f;  // 1.5 * 2^23
constexpr uint32_t kMagicFBits = 0x4B400000u;
constexpr unsigned long long kMagicPair = ((unsigned long long)kMagicFBits << 32) | kMagicFBits;

// Per work item: the largest particle bound (kg m/s) its LDS sums take
// (cap < 0: none, every particle takes the global path), and 2^-e. Both are
// the same in every lane and are kept in scalar registers.
struct ItemScale {
  float cap, in;
  // 2^e, from the exponent bits of 2^-e
  __device__ __forceinline__ float out() const { return __int_as_float((254 << 23) - __float_as_int(in)); }
};

// Scale of a work item of n particles from its tile's bound entry (valid if
// stamped with substep `prev`) and vmax, the largest velocity component of
// the tile's staged nodes: the item takes particles whose bound is at most
// 1.25 times the larger of the recorded bound and m vmax. The recorded bound
// follows the stress; m vmax bounds |m v| of every particle that gathers from
// the tile, and covers the first substeps from rest, where the bounds grow by
// large factors from one substep to the next. A node sum of the item has at
// most n terms, each at most 0.421875 (the largest weight) times that
// capacity, so X below
// bounds every |sum|; with X 2^-e < 2^31 / (1 + 2^-10) every sum decodes from
// its 32 bits with room for the FP32 rounding of the terms (and, n counted as
// at least 512, every term stays under the 2^22 range of the rounding fma).
__device__ __forceinline__ ItemScale item_scale(unsigned long long entry, unsigned prev, unsigned n, float mvmax) {
  float cap = -1.0f;
  int e = 0;
  {
    const float recorded = (unsigned)(entry >> 32) == prev ? __uint_as_float((uint32_t)entry) : 0.0f;
    const float c = 1.25f * fmaxf(recorded, mvmax);
    if (c > 0.0f && c < 1e30f) {
      cap = c;
      const float X = (float)max(n, 512u) * 0.421875f * c * (1.0f + 0x1p-10f);
      e = max(ilogbf(X) - 30, -100);
    }
  }
  ItemScale sc;
  sc.cap = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(cap)));
  sc.in = __int_as_float(__builtin_amdgcn_readfirstlane((127 - e) << 23));
  return sc;
}

// Merge the largest bound of a wave's particles into the tile's entry for
// this substep (all lanes of the wave call it).
__device__ __forceinline__ void record_bound(unsigned long long* pb, unsigned unit, unsigned stamp, float bmax) {
  float m = bmax;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63u) == 0u && m > 0.0f)
    atomicMax(pb + unit, ((unsigned long long)stamp << 32) | __float_as_uint(m));
}

// Per-particle inputs of the packed scatter: the affine momentum field
// q + A o dx in units of 2^e as FP32 (q = m v - A f dx).
struct P2GPk {
  float w[3][3];
  float q[3];
  float Adx[9];
};

__device__ __forceinline__ float affine_step_f(float base, float slope, int o) {
  return o == 0 ? base : (o == 1 ? base + slope : fmaf(slope, 2.0f, base));
}

// The 27 contributions of one particle as FP32 (weight N and the affine
// field q + A o dx at the node, not yet times N), handed to `sink`.
template <class Sink>
__device__ __forceinline__ void p2g_emit_f32(const P2GPk& P, Sink&& sink) {
#pragma unroll 1
  for (int ox = 0; ox < 3; ++ox) {
    const float wx = ox == 0 ? P.w[0][0] : (ox == 1 ? P.w[0][1] : P.w[0][2]);
    float qx[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) qx[a] = fmaf(P.Adx[3 * a], (float)ox, P.q[a]);
#pragma unroll
    for (int oy = 0; oy < 3; ++oy) {
      float qy[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) qy[a] = affine_step_f(qx[a], P.Adx[3 * a + 1], oy);
      const float wxy = wx * P.w[1][oy];
#pragma unroll
      for (int oz = 0; oz < 3; ++oz)
        sink(ox, oy, oz, wxy * P.w[2][oz], affine_step_f(qy[0], P.Adx[2], oz), affine_step_f(qy[1], P.Adx[5], oz),
             affine_step_f(qy[2], P.Adx[8], oz));
    }
  }
}

// The 27 packed contributions of one particle (q, A dx in units of 2^e),
// handed to `sink`.
template <class Sink>
__device__ __forceinline__ void p2g_emit_pk(const P2GPk& P, Sink&& sink) {
  p2g_emit_f32(P, [&](int ox, int oy, int oz, float N, float c0, float c1, float c2) {
    const uint32_t wq = (uint32_t)fmaf(N, kWeightUnits, 0.5f);
    const uint32_t b0 = __float_as_uint(fmaf(N, c0, kMagicF));
    const uint32_t b1 = __float_as_uint(fmaf(N, c1, kMagicF));
    const uint32_t b2 = __float_as_uint(fmaf(N, c2, kMagicF));
    const unsigned long long w01 = (((unsigned long long)b1 << 32) | b0) - kMagicPair;
    const unsigned long long w2m = ((unsigned long long)(b2 - kMagicFBits) << 32) | wq;
    sink(ox, oy, oz, w01, w2m);
  });
}

// The sums of a packed node: weight units and momentum in units of 2^e.
__device__ __forceinline__ void unpack_node(unsigned long long w01, unsigned long long w2m, uint32_t& wq, int& p0,
                                            int& p1, int& p2) {
  p0 = (int)(uint32_t)w01;
  p1 = (int)(uint32_t)((w01 - (unsigned long long)(long long)p0) >> 32);
  wq = (uint32_t)w2m;
  p2 = (int)(uint32_t)(w2m >> 32);
}

__device__ __forceinline__ void acc_add_pk(const SimK& s, float* am, float* ap0, float* ap1, float* ap2, int g,
                                           uint32_t wq, int p0, int p1, int p2, float out) {
  unsafeAtomicAdd(am + g, (float)wq * s.m_unit);
  unsafeAtomicAdd(ap0 + g, (float)p0 * out);
  unsafeAtomicAdd(ap1 + g, (float)p1 * out);
  unsafeAtomicAdd(ap2 + g, (float)p2 * out);
}

// MLS-MPM P2G of one particle into the packed tile (the arithmetic of
// p2g_particle up to the contribution bound); particles outside the tile and
// its shell, or beyond the item's capacity, add their FP32 contributions
// straight into the FP32 accumulator. Uses L.p0 / L.p1 (L.sp0 / L.sp1 for
// the shell) as the two packed words of a node.
template <bool FIXED, int T>
__device__ __forceinline__ void p2g_particle_pk(const SimK& s, const float* x, const float* v, const float* C,
                                                const float* F, float E, const int* to, Lds<T>& L,
                                                const ItemScale& sc, ACC_PARAMS, uint32_t* mark, uint32_t* ovf,
                                                Status* st, int parity, unsigned& ev, float& bmax) {
  static_assert(!FIXED, "the packed tile feeds the FP32 accumulator");
  int base[3];
  float f[3];
  if (!particle_stencil(s, x, base, f)) {
    if (isfinite(x[0] + x[1] + x[2]))
      ev |= kEvDom;
    else
      ev |= kEvNf;
    return;
  }
  float tau[9];
  bool inv;
  kirchhoff(F, s.c_mu * E, s.c_la * E, tau, &inv);
  float Af[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) Af[i] = s.mass * C[i] - s.p2g_stress * tau[i];
  float chk = v[0] + v[1] + v[2];
#pragma unroll
  for (int i = 0; i < 9; ++i) chk += Af[i];
  if (!isfinite(chk)) {
    ev |= kEvNf;
    return;
  }
  if (inv) ev |= kEvInv;
  float bound = 0.0f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float row = fabsf(Af[3 * a]) + fabsf(Af[3 * a + 1]) + fabsf(Af[3 * a + 2]);
    bound = fmaxf(bound, fabsf(s.mass * v[a]) + 1.5f * s.dx * row);
  }
  if (!(bound < s.p_limit)) {
    ev |= kEvRng;
    return;
  }
  bmax = fmaxf(bmax, bound);
  const int l0 = base[0] - to[0], l1 = base[1] - to[1], l2 = base[2] - to[2];
  constexpr unsigned kMarginMax = T + 1;  // base -1 .. T, shifted by one
  const bool in = in_tile<T>(l0, l1, l2);
  const bool shell = !in && (unsigned)(l0 + 1) <= kMarginMax && (unsigned)(l1 + 1) <= kMarginMax &&
                     (unsigned)(l2 + 1) <= kMarginMax;
  const bool lds = (in || shell) && bound <= sc.cap;
  const float scale = lds ? sc.in : 1.0f;
  P2GPk P;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    bspline_w(f[a], P.w[a]);
    const float qa = s.mass * v[a] - (Af[3 * a] * f[0] + Af[3 * a + 1] * f[1] + Af[3 * a + 2] * f[2]) * s.dx;
    P.q[a] = qa * scale;
#pragma unroll
    for (int b = 0; b < 3; ++b) P.Adx[3 * a + b] = (Af[3 * a + b] * s.dx) * scale;
  }
  if (!lds) {
    // FP32 contributions straight into the FP32 accumulator.
    if (!(in || shell)) ev |= kEvFbP2G;
    const int node_base = to[3] * s.n3;
    p2g_emit_f32(P, [&](int ox, int oy, int oz, float N, float c0, float c1, float c2) {
      const int g = node_base + grid_index(base[0] + ox, base[1] + oy, base[2] + oz, s.nb);
      unsafeAtomicAdd(am + g, N * s.mass);
      unsafeAtomicAdd(ap0 + g, N * c0);
      unsafeAtomicAdd(ap1 + g, N * c1);
      unsafeAtomicAdd(ap2 + g, N * c2);
    });
    claim_stencil_blocks(s, base, mark, ovf, st, parity, to[3]);
    return;
  }
  if (shell) {
    // One cell out: the nodes in the span go to the tile, the others to the shell.
    constexpr int S = TileShape<T>::kSpan;
    L.shell_mark = L.item_tag;
    p2g_emit_pk(P, [&](int ox, int oy, int oz, unsigned long long w01, unsigned long long w2m) {
      const int x = l0 + ox, y = l1 + oy, z = l2 + oz;
      unsigned long long *a0, *a1;
      if ((unsigned)x < (unsigned)S && (unsigned)y < (unsigned)S && (unsigned)z < (unsigned)S) {
        const int idx = lds_index<T>(x, y, z);
        a0 = (unsigned long long*)&L.p0[idx];
        a1 = (unsigned long long*)&L.p1[idx];
      } else {
        const int j = shell_index<T>(x, y, z);
        a0 = (unsigned long long*)&L.sp0[j];
        a1 = (unsigned long long*)&L.sp1[j];
      }
      atomicAdd(a0, w01);
      atomicAdd(a1, w2m);
    });
    return;
  }
  const int l = lds_index<T>(l0, l1, l2);
  p2g_emit_pk(P, [&](int ox, int oy, int oz, unsigned long long w01, unsigned long long w2m) {
    const int idx = l + lds_index<T>(ox, oy, oz);
    atomicAdd((unsigned long long*)&L.p0[idx], w01);
    atomicAdd((unsigned long long*)&L.p1[idx], w2m);
  });
}

// P2G of one particle for standard MPM (Sec. III-A): mass N m and momentum
// N m v + dt f_I with the internal force f_I = -V0 tau grad N of the
// Neo-Hookean stress (gravity is added by the grid update). C is not
// transferred; it holds the velocity gradient and is only checked for being
// finite.
template <bool FIXED, int T, bool SHELL>
__device__ __forceinline__ void p2g_particle_pic(const SimK& s, const float* x, const float* v, const float* C,
                                                 const float* F, float E, const int* to, Lds<T>& L, ACC_PARAMS,
                                                 uint32_t* mark, uint32_t* ovf, Status* st, int parity,
                                                 unsigned& ev) {
  PICIn P;
  float f[3];
  if (!particle_stencil(s, x, P.base, f)) {
    if (isfinite(x[0] + x[1] + x[2]))
      ev |= kEvDom;
    else
      ev |= kEvNf;
    return;
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    bspline_w(f[a], P.w[a]);
    bspline_dw(f[a], P.dw[a]);
  }
  float tau[9];
  const float J = neo_hookean_tau(F, s.c_mu * E, s.c_la * E, tau);
  float chk = v[0] + v[1] + v[2];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    P.tk[i] = s.pic_force * tau[i];
    chk += P.tk[i] + C[i];
  }
  if (!isfinite(chk)) {
    ev |= kEvNf;
    return;
  }
  if (!(J > 0.0f)) ev |= kEvInv;
  // |grad N dx| <= 9/16 per component, so |m v| + sum_b |tk[a][b]| bounds
  // every contribution.
  float bound = 0.0f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    P.mv[a] = s.mass * v[a];
    bound = fmaxf(bound, fabsf(P.mv[a]) + fabsf(P.tk[3 * a]) + fabsf(P.tk[3 * a + 1]) + fabsf(P.tk[3 * a + 2]));
  }
  if (!(bound < s.p_limit)) {
    ev |= kEvRng;
    return;
  }
  P.fx_p = s.fx_p;
  p2g_commit<FIXED, T, SHELL>(s, P, to, L, ACC_ARGS, mark, ovf, st, parity, ev);
}

// G2P of one particle (Algorithm 1, third loop). APIC (MLS-MPM, PB-MPM):
// v' = sum N v_I, C' = (4/dx^2) sum N v_I (x_I - x_p)^T. Standard MPM:
// v' = sum N v_I and the velocity gradient L = sum v_I grad N^T in Cn.
// Returns false if the stencil is outside the grid (the particle is then
// left unchanged).
template <int SOL, int T>
__device__ __forceinline__ bool g2p_particle(const SimK& s, const float* x, const int* to,
                                             const float4* Lv, const float4* vel, float* vn, float* Cn,
                                             unsigned& ev) {
  int base[3];
  float f[3];
  if (!particle_stencil(s, x, base, f)) return false;
  float w[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) bspline_w(f[a], w[a]);
  float S[3], Tm[9];
  const int l0 = base[0] - to[0], l1 = base[1] - to[1], l2 = base[2] - to[2];
  const bool in_tile_ = in_tile<T>(l0, l1, l2);
  if constexpr (SOL == SOLVER_PIC) {
    float dw[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) bspline_dw(f[a], dw[a]);
    if (in_tile_) {
      const int l = lds_index<T>(l0, l1, l2);
      g2p_sums_pic(w, dw, [&](int ox, int oy, int oz) { return Lv[l + lds_index<T>(ox, oy, oz)]; }, S, Tm);
    } else {
      ev |= kEvFbG2P;
      const int node_base = to[3] * s.n3;
      g2p_sums_pic(w, dw, [&](int ox, int oy, int oz) {
        return vel[node_base + grid_index(base[0] + ox, base[1] + oy, base[2] + oz, s.nb)];
      }, S, Tm);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      vn[a] = S[a];
#pragma unroll
      for (int b = 0; b < 3; ++b) Cn[3 * a + b] = s.inv_dx * Tm[3 * a + b];
    }
  } else {
    // Tm[a][b] = sum N v_a o_b
    if (in_tile_) {
      const int l = lds_index<T>(l0, l1, l2);
      g2p_sums(w, [&](int ox, int oy, int oz) { return Lv[l + lds_index<T>(ox, oy, oz)]; }, S, Tm);
    } else {
      ev |= kEvFbG2P;
      g2p_global(s, base, w, vel, S, Tm, to[3]);
    }
    const float k = 4.0f * s.inv_dx;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      vn[a] = S[a];
#pragma unroll
      for (int b = 0; b < 3; ++b) Cn[3 * a + b] = k * (Tm[3 * a + b] - S[a] * f[b]);
    }
  }
  return true;
}

// ------------------------------------------------------------------ tile helpers
// Tile origin of work tile u (node coordinates within its scene) in to[0..2]
// and its scene in to[3]. For T = 4, u = block * 8 + (sx + 2 sy + 4 sz).
template <int T>
__device__ __forceinline__ void unit_origin(const SimK& s, unsigned u, int* to) {
  constexpr int kShift = TileShape<T>::kUnitShift;
  const unsigned b = u >> kShift;
  const unsigned scene = b / s.nb3;
  const unsigned lb = b - scene * s.nb3;
  const int bi = (int)(lb % (unsigned)s.nb);
  const int bj = (int)((lb / (unsigned)s.nb) % (unsigned)s.nb);
  const int bk = (int)(lb / ((unsigned)s.nb * (unsigned)s.nb));
  to[0] = bi * kTile;
  to[1] = bj * kTile;
  to[2] = bk * kTile;
  if constexpr (kShift != 0) {
    to[0] += (int)(u & 1u) * T;
    to[1] += (int)((u >> 1) & 1u) * T;
    to[2] += (int)((u >> 2) & 1u) * T;
  }
  to[3] = (int)scene;
}

// Clears the span and the shell, and starts work item `tag` (nonzero, new
// for each item of a workgroup); a barrier must follow.
// (KEEP_P2: the packed tile uses p0 and p1 only and keeps its slot table in
// p2.)
template <int T, bool KEEP_P2 = false>
__device__ __forceinline__ void tile_clear(Lds<T>& L, uint32_t tag) {
  for (int i = threadIdx.x; i < Lds<T>::kNodes; i += blockDim.x) {
    L.m[i] = 0u;
    L.p0[i] = 0ll;
    L.p1[i] = 0ll;
    if constexpr (!KEEP_P2) L.p2[i] = 0ll;
  }
  for (int j = threadIdx.x; j < Lds<T>::kShell; j += blockDim.x) {
    L.sm[j] = 0u;
    L.sp0[j] = 0ll;
    L.sp1[j] = 0ll;
    L.sp2[j] = 0ll;
  }
  if (threadIdx.x == 0) {
    L.item_tag = tag;
    L.shell_mark = 0u;
  }
}

// The shell's non-empty nodes -> global accumulator, if work item `tag`
// scattered into it, clearing them on the way. A shell node one cell below
// the tile can lie in a block that the binning did not activate: it is
// claimed for the grid update as the global path does.
template <bool FIXED, int T>
__device__ __forceinline__ void shell_flush_clear(const SimK& s, const int* to, Lds<T>& L, ACC_PARAMS, uint32_t tag,
                                                  uint32_t* mark, uint32_t* ovf, Status* st, int parity) {
  if (L.shell_mark != tag) return;  // the same in every thread: no scatter of this item reached the shell
  for (int j = threadIdx.x; j < Lds<T>::kShell; j += blockDim.x) {
    const uint32_t wq = L.sm[j];
    const long long p0 = L.sp0[j], p1 = L.sp1[j], p2 = L.sp2[j];
    if ((wq | p0 | p1 | p2) == 0) continue;
    L.sm[j] = 0u;
    L.sp0[j] = 0ll;
    L.sp1[j] = 0ll;
    L.sp2[j] = 0ll;
    int x, y, z;
    shell_node<T>(j, &x, &y, &z);
    const int gx = to[0] + x, gy = to[1] + y, gz = to[2] + z;
    if ((unsigned)gx >= (unsigned)s.n || (unsigned)gy >= (unsigned)s.n || (unsigned)gz >= (unsigned)s.n) continue;
    acc_add<FIXED>(s, ACC_ARGS, to[3] * s.n3 + grid_index(gx, gy, gz, s.nb), wq, p0, p1, p2);
    const unsigned b = (unsigned)to[3] * s.nb3 +
                       (unsigned)((((gz >> kTileLog2) * s.nb) + (gy >> kTileLog2)) * s.nb + (gx >> kTileLog2));
    if (__hip_atomic_load(&mark[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u &&
        atomicCAS(&mark[b], 0u, 2u) == 0u) {
      const unsigned slot = atomicAdd(&st->ovf_count[parity], 1u);
      ovf[slot] = b;
    }
  }
}

template <int T>
__device__ __forceinline__ void tile_stage_velocity(const SimK& s, const int* to, const float4* vel,
                                                    float4* Lv) {
  constexpr int S = TileShape<T>::kSpan;
  for (int i = threadIdx.x; i < Lds<T>::kNodes; i += blockDim.x) {
    const int lx = i % S, ly = (i / S) % S, lz = i / (S * S);
    const int gx = to[0] + lx, gy = to[1] + ly, gz = to[2] + lz;
    float4 val = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if ((unsigned)gx < (unsigned)s.n && (unsigned)gy < (unsigned)s.n && (unsigned)gz < (unsigned)s.n)
      val = vel[to[3] * s.n3 + grid_index(gx, gy, gz, s.nb)];
    Lv[i] = val;
  }
}

// Hides a value from the optimiser, so that index arithmetic that only
// depends on the thread is recomputed where it is used instead of being
// hoisted out of the work-item loop and held in registers across it.
__device__ __forceinline__ void opaque(int& v) { asm volatile("" : "+v"(v)); }

// tile_stage_velocity that also leaves, per wave, the largest |velocity
// component| of the staged nodes in vw (one slot per wave).
template <int T>
__device__ __forceinline__ void tile_stage_velocity_max(const SimK& s, const int* to, const float4* vel, float4* Lv,
                                                        float* vw) {
  constexpr int S = TileShape<T>::kSpan;
  float m = 0.0f;
  for (int i = threadIdx.x; i < Lds<T>::kNodes; i += blockDim.x) {
    const int lx = i % S, ly = (i / S) % S, lz = i / (S * S);
    const int gx = to[0] + lx, gy = to[1] + ly, gz = to[2] + lz;
    float4 val = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if ((unsigned)gx < (unsigned)s.n && (unsigned)gy < (unsigned)s.n && (unsigned)gz < (unsigned)s.n)
      val = vel[to[3] * s.n3 + grid_index(gx, gy, gz, s.nb)];
    Lv[i] = val;
    m = fmaxf(m, fmaxf(fabsf(val.x), fmaxf(fabsf(val.y), fabsf(val.z))));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
  int w = (int)(threadIdx.x >> 6);
  opaque(w);  // recomputed here rather than held across the work-item loop
  if ((threadIdx.x & 63u) == 0u) vw[w] = m;
}

// Slot table of a block-aligned (8-cell) tile, in the packed kernel's free
// weight-sum array: per tile node, its offset from the tile's first node in
// the block-major grid layout (low 32 bits) and its tile coordinates (4 bits
// each from bit 32). A thread fills and reads only the slots it stages and
// flushes (node i of thread threadIdx.x + k * blockDim.x), so no barrier
// orders them.
__device__ __forceinline__ void fill_slot_table(const SimK& s, long long* tab) {
  constexpr int S = TileShape<8>::kSpan;
  for (int i = threadIdx.x; i < Lds<8>::kNodes; i += blockDim.x) {
    const int lx = i % S, ly = (i / S) % S, lz = i / (S * S);
    const unsigned blk = (unsigned)((((lz >> 3) * s.nb + (ly >> 3)) * s.nb) + (lx >> 3));
    const unsigned off = (blk << (3 * kTileLog2)) + (unsigned)((((lz & 7) << 3) + (ly & 7)) << 3) + (unsigned)(lx & 7);
    tab[i] = (long long)((unsigned long long)off | ((unsigned long long)(lx | (ly << 4) | (lz << 8)) << 32));
  }
}

// Grid index of the node in slot entry e of the tile at `to`, or -1 outside
// the grid (tile coordinates at or beyond lim = n - to per axis).
__device__ __forceinline__ int slot_node(long long e, int base, int limx, int limy, int limz) {
  const unsigned c = (unsigned)((unsigned long long)e >> 32);
  const bool in = (int)(c & 15u) < limx && (int)((c >> 4) & 15u) < limy && (int)(c >> 8) < limz;
  return in ? base + (int)(unsigned)e : -1;
}

// tile_stage_velocity_max through the slot table (8-cell tiles).
__device__ __forceinline__ void tile_stage_velocity_tab(const SimK& s, const int* to, const float4* vel, float4* Lv,
                                                        float* vw, const long long* tab) {
  const int base = to[3] * s.n3 + grid_index(to[0], to[1], to[2], s.nb);
  const int limx = s.n - to[0], limy = s.n - to[1], limz = s.n - to[2];
  float m = 0.0f;
  for (int i = threadIdx.x; i < Lds<8>::kNodes; i += blockDim.x) {
    const int g = slot_node(tab[i], base, limx, limy, limz);
    float4 val = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (g >= 0) val = vel[g];
    Lv[i] = val;
    m = fmaxf(m, fmaxf(fabsf(val.x), fmaxf(fabsf(val.y), fabsf(val.z))));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
  int w = (int)(threadIdx.x >> 6);
  opaque(w);
  if ((threadIdx.x & 63u) == 0u) vw[w] = m;
}

// Non-empty tile nodes -> global accumulator, clearing the tile for the next
// work item on the way (each thread clears the nodes it flushed).
template <bool FIXED, int T>
__device__ __forceinline__ void tile_flush_clear(const SimK& s, const int* to, Lds<T>& L, ACC_PARAMS) {
  constexpr int S = TileShape<T>::kSpan;
  constexpr int kSlots = (Lds<T>::kNodes + TileShape<T>::kWG - 1) / TileShape<T>::kWG;
#pragma unroll
  for (int k = 0; k < kSlots; ++k) {
    int i = threadIdx.x + k * TileShape<T>::kWG;
    if (i >= Lds<T>::kNodes) break;
    opaque(i);
    const uint32_t wq = L.m[i];
    const long long p0 = L.p0[i], p1 = L.p1[i], p2 = L.p2[i];
    L.m[i] = 0u;
    L.p0[i] = 0ll;
    L.p1[i] = 0ll;
    L.p2[i] = 0ll;
    if ((wq | p0 | p1 | p2) == 0) continue;
    const int lx = i % S, ly = (i / S) % S, lz = i / (S * S);
    const int gx = to[0] + lx, gy = to[1] + ly, gz = to[2] + lz;
    if ((unsigned)gx >= (unsigned)s.n || (unsigned)gy >= (unsigned)s.n || (unsigned)gz >= (unsigned)s.n) continue;
    acc_add<FIXED>(s, ACC_ARGS, to[3] * s.n3 + grid_index(gx, gy, gz, s.nb), wq, p0, p1, p2);
  }
}

// Non-empty tile nodes -> global accumulator.
template <bool FIXED, int T>
__device__ __forceinline__ void tile_flush(const SimK& s, const int* to, const Lds<T>& L, ACC_PARAMS) {
  constexpr int S = TileShape<T>::kSpan;
  for (int i = threadIdx.x; i < Lds<T>::kNodes; i += blockDim.x) {
    const uint32_t wq = L.m[i];
    const long long p0 = L.p0[i], p1 = L.p1[i], p2 = L.p2[i];
    if ((wq | p0 | p1 | p2) == 0) continue;
    const int lx = i % S, ly = (i / S) % S, lz = i / (S * S);
    const int gx = to[0] + lx, gy = to[1] + ly, gz = to[2] + lz;
    // Only in-grid nodes can receive contributions (stencils are checked
    // against the grid); the test keeps the index in range regardless.
    if ((unsigned)gx >= (unsigned)s.n || (unsigned)gy >= (unsigned)s.n || (unsigned)gz >= (unsigned)s.n) continue;
    acc_add<FIXED>(s, ACC_ARGS, to[3] * s.n3 + grid_index(gx, gy, gz, s.nb), wq, p0, p1, p2);
  }
}

// The packed tile's non-empty nodes -> FP32 accumulator (momentum sums
// times `out` = 2^e), clearing them on the way.
template <int T>
__device__ __forceinline__ void tile_flush_clear_pk(const SimK& s, const int* to, Lds<T>& L, float* am, float* ap0,
                                                    float* ap1, float* ap2, float out) {
  constexpr int S = TileShape<T>::kSpan;
  constexpr int kSlots = (Lds<T>::kNodes + TileShape<T>::kWG - 1) / TileShape<T>::kWG;
#pragma unroll
  for (int k = 0; k < kSlots; ++k) {
    int i = threadIdx.x + k * TileShape<T>::kWG;
    if (i >= Lds<T>::kNodes) break;
    opaque(i);
    const unsigned long long w01 = (unsigned long long)L.p0[i], w2m = (unsigned long long)L.p1[i];
    L.p0[i] = 0ll;
    L.p1[i] = 0ll;
    if ((w01 | w2m) == 0ull) continue;
    int g;
    if constexpr (T == 8) {
      // the slot table in the free p2 array (fill_slot_table)
      g = slot_node(L.p2[i], to[3] * s.n3 + grid_index(to[0], to[1], to[2], s.nb), s.n - to[0], s.n - to[1],
                    s.n - to[2]);
      if (g < 0) continue;
    } else {
      const int lx = i % S, ly = (i / S) % S, lz = i / (S * S);
      const int gx = to[0] + lx, gy = to[1] + ly, gz = to[2] + lz;
      if ((unsigned)gx >= (unsigned)s.n || (unsigned)gy >= (unsigned)s.n || (unsigned)gz >= (unsigned)s.n) continue;
      g = to[3] * s.n3 + grid_index(gx, gy, gz, s.nb);
    }
    uint32_t wq;
    int p0, p1, p2;
    unpack_node(w01, w2m, wq, p0, p1, p2);
    acc_add_pk(s, am, ap0, ap1, ap2, g, wq, p0, p1, p2, out);
  }
}

// The packed shell, as shell_flush_clear.
template <int T>
__device__ __forceinline__ void shell_flush_clear_pk(const SimK& s, const int* to, Lds<T>& L, float* am, float* ap0,
                                                     float* ap1, float* ap2, float out, uint32_t tag, uint32_t* mark,
                                                     uint32_t* ovf, Status* st, int parity) {
  if (L.shell_mark != tag) return;  // the same in every thread
  for (int j = threadIdx.x; j < Lds<T>::kShell; j += blockDim.x) {
    const unsigned long long w01 = (unsigned long long)L.sp0[j], w2m = (unsigned long long)L.sp1[j];
    if ((w01 | w2m) == 0ull) continue;
    L.sp0[j] = 0ll;
    L.sp1[j] = 0ll;
    int x, y, z;
    shell_node<T>(j, &x, &y, &z);
    const int gx = to[0] + x, gy = to[1] + y, gz = to[2] + z;
    if ((unsigned)gx >= (unsigned)s.n || (unsigned)gy >= (unsigned)s.n || (unsigned)gz >= (unsigned)s.n) continue;
    uint32_t wq;
    int p0, p1, p2;
    unpack_node(w01, w2m, wq, p0, p1, p2);
    acc_add_pk(s, am, ap0, ap1, ap2, to[3] * s.n3 + grid_index(gx, gy, gz, s.nb), wq, p0, p1, p2, out);
    const unsigned b = (unsigned)to[3] * s.nb3 +
                       (unsigned)((((gz >> kTileLog2) * s.nb) + (gy >> kTileLog2)) * s.nb + (gx >> kTileLog2));
    if (__hip_atomic_load(&mark[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u &&
        atomicCAS(&mark[b], 0u, 2u) == 0u) {
      const unsigned slot = atomicAdd(&st->ovf_count[parity], 1u);
      ovf[slot] = b;
    }
  }
}

__device__ __forceinline__ float particle_E(const SimK& s, const float* __restrict__ part, int64_t cap,
                                            unsigned p) {
  return s.has_E ? part[FE * cap + p] : s.E_default;
}

// ------------------------------------------------------------------ kernels
// Scatter of one particle by the solver's rule (SHELL: one-cell-out
// particles scatter into the tile's shell).
template <bool FIXED, int SOL, int PASS, int T, bool SHELL = true>
__device__ __forceinline__ void p2g_any(const SimK& s, const float* x, const float* v, const float* C,
                                        const float* F, float E, const int* to, Lds<T>& L, ACC_PARAMS,
                                        uint32_t* mark, uint32_t* ovf, Status* st, int parity, unsigned& ev,
                                        float& bmax) {
  if constexpr (SOL == SOLVER_PIC)
    p2g_particle_pic<FIXED, T, SHELL>(s, x, v, C, F, E, to, L, ACC_ARGS, mark, ovf, st, parity, ev);
  else
    p2g_particle<FIXED, SOL, PASS, T, SHELL>(s, x, v, C, F, E, to, L, ACC_ARGS, mark, ovf, st, parity, ev, bmax);
}

// P2G from the materialised particle state (first substep after binning; for
// PB-MPM the first pass of a step).
template <bool FIXED, int SOL, int T>
__global__ __launch_bounds__(TileShape<T>::kWG, 4) void k_p2g(const float* __restrict__ part, int64_t cap,
                                             const uint32_t* __restrict__ blk_end,
                                             const uint2* __restrict__ work, Status* st,
                                             ACC_PARAMS, uint32_t* mark, uint32_t* ovf0, uint32_t* ovf1,
                                             const Clock* __restrict__ clk, unsigned long long* pb_wr,
                                             int parity, SimK s) {
  // The bounds of this substep set the scale of the next (packed) one.
  constexpr bool kTrack = !FIXED && SOL == SOLVER_MLS;
  uint32_t* ovf = parity ? ovf1 : ovf0;
  __shared__ Lds<T> L;
  Counters cnt;
  unsigned stamp = 0u;
  if constexpr (kTrack) stamp = (unsigned)clk[parity].substep;
  const WorkWalk walk(st->n_work);
  unsigned pos = walk.first();
  while (pos < walk.end) {
    const uint2 item = work[pos];
    const unsigned b = item.x & ~kDenseFlag;
    const unsigned q = item_lane<T>(item.x);
    int to[4];
    unit_origin<T>(s, b, to);
    unsigned next = 0u;
    if (threadIdx.x == 0) next = walk.claim(st);
    tile_clear(L, pos + 1u);
    __syncthreads();
    const unsigned pe = min(item.y + s.item_particles, blk_end[b]);
    float bmax = 0.0f;
    for (unsigned p = item.y + q; p < pe; p += TileShape<T>::kWG) {
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
      const float E = SOL == SOLVER_PB ? 0.0f : particle_E(s, part, cap, p);
      unsigned ev = 0u;
      p2g_any<FIXED, SOL, PB_FIRST, T>(s, x, v, C, F, E, to, L, ACC_ARGS, mark, ovf, st, parity, ev, bmax);
      count_events(cnt, ev);
    }
    if constexpr (kTrack) record_bound(pb_wr, b, stamp, bmax);
    if (threadIdx.x == 0) L.claimed[1] = next;
    __syncthreads();
    next = L.claimed[1];
    tile_flush<FIXED, T>(s, to, L, ACC_ARGS);
    shell_flush_clear<FIXED, T>(s, to, L, ACC_ARGS, pos + 1u, mark, ovf, st, parity);
    __syncthreads();
    pos = next;
  }
  if (threadIdx.x == 0) walk.finish(st);
  flush_counters(st, cnt);
}

// Fused G2P (substep k-1) -> F, x update -> stress -> P2G (substep k).
// PB-MPM: PB_FIRST is the same fusion across a step boundary (the G2P of the
// previous step's last iteration, its F and x update, then the first pass of
// the new step); PB_ITER is G2P -> constraint -> P2G within a step, where x
// and F do not change and nothing is written back.
// With PUSH, particles that the position update leaves inside a tool with
// push-out on are moved to its surface (push_out) before the P2G.
template <bool FIXED, int SOL, int PASS, bool PUSH, int T>
__global__ __launch_bounds__(TileShape<T>::kWG, 4) void k_g2p2g(float* __restrict__ part, int64_t cap,
                                               const uint32_t* __restrict__ blk_end,
                                               const uint2* __restrict__ work, Status* st,
                                               ACC_PARAMS, const float4* __restrict__ vel,
                                               uint32_t* mark, uint32_t* ovf0, uint32_t* ovf1,
                                               const Clock* __restrict__ clk,
                                               const unsigned long long* __restrict__ pb_rd,
                                               unsigned long long* pb_wr, int parity,
                                               const ToolDesc* __restrict__ tools, SimK s) {
  constexpr bool kIntegrate = !(SOL == SOLVER_PB && PASS == PB_ITER);
  static_assert(!PUSH || kIntegrate, "push-out follows a position update");
  constexpr bool kShell = SOL != SOLVER_PB && !PUSH;
  // FP32 MLS-MPM scatters into the packed tile (the push-out variant keeps
  // the int64 tile: the packed path does not fit its registers).
  constexpr bool kPack = !FIXED && SOL == SOLVER_MLS && !PUSH;
  long long substep = 0;
  if constexpr (PUSH || kPack) substep = clk[parity].substep;
  uint32_t* ovf = parity ? ovf1 : ovf0;
  __shared__ Lds<T> L;
  __shared__ float4 Vb[Lds<T>::kNodes];  // second velocity buffer
  Counters cnt;
  const WorkWalk walk(st->n_work);
  unsigned pos = walk.first(), npos = walk.end;
  uint2 item = make_uint2(0u, 0u);
  bool flip = false;  // which of the two velocity buffers holds this item's tile
  // The packed tile leaves the p2 array free: 8-cell tiles keep their slot
  // table there (staging and flush address the grid through it).
  constexpr bool kTable = kPack && T == 8;
  if constexpr (kTable) fill_slot_table(s, L.p2);
  if (pos < walk.end) {
    if (threadIdx.x == 0) L.claimed[0] = walk.claim(st);
    item = work[pos];
    if constexpr (kPack)
      if (threadIdx.x == 0) L.pbe[0] = pb_rd[item.x & ~kDenseFlag];
    int to[4];
    unit_origin<T>(s, item.x & ~kDenseFlag, to);
    if constexpr (kTable)
      tile_stage_velocity_tab(s, to, vel, L.v, L.vw[0], L.p2);
    else if constexpr (kPack)
      tile_stage_velocity_max<T>(s, to, vel, L.v, L.vw[0]);
    else
      tile_stage_velocity<T>(s, to, vel, L.v);
    tile_clear<T, kTable>(L, pos + 1u);
    __syncthreads();
    npos = L.claimed[0];
  }
  // Each pass: the particles of one work item, after which each thread
  // stages its share of the next item's velocities into the other buffer
  // (nothing reads it during this item); then, after one barrier, the flush
  // of the tile and its shell, which also clears them.
  while (pos < walk.end) {
    const float4* Lv = flip ? Vb : L.v;
    const unsigned b = item.x & ~kDenseFlag;
    const unsigned q = item_lane<T>(item.x);
    int to[4];
    unit_origin<T>(s, b, to);
    const unsigned pe = min(item.y + s.item_particles, blk_end[b]);
    ItemScale sc{-1.0f, 1.0f};
    if constexpr (kPack) {
      float vmax = 0.0f;
#pragma unroll
      for (int w = 0; w < TileShape<T>::kWG / 64; ++w) vmax = fmaxf(vmax, L.vw[flip ? 1 : 0][w]);
      sc = item_scale(L.pbe[flip ? 1 : 0], (unsigned)(substep - 1), pe - item.y, s.mass * vmax);
    }
    float bmax = 0.0f;
    for (unsigned p = item.y + q; p < pe; p += TileShape<T>::kWG) {
      float x[3], F[9];
#pragma unroll
      for (int a = 0; a < 3; ++a) x[a] = part[(FX + a) * cap + p];
#pragma unroll
      for (int i = 0; i < 9; ++i) F[i] = part[(FF + i) * cap + p];
      float vn[3], Cn[9];
      unsigned ev = 0u;
      if (!g2p_particle<SOL, T>(s, x, to, Lv, vel, vn, Cn, ev)) continue;  // frozen (out of grid), no events
      if constexpr (kIntegrate) {
        float Fn[9];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int b2 = 0; b2 < 3; ++b2)
            Fn[3 * a + b2] = F[3 * a + b2] + s.dt * (Cn[3 * a] * F[b2] + Cn[3 * a + 1] * F[3 + b2] +
                                                     Cn[3 * a + 2] * F[6 + b2]);
#pragma unroll
        for (int a = 0; a < 3; ++a) x[a] += s.dt * vn[a];
        if constexpr (PUSH) push_out(s, tools + (size_t)to[3] * kMaxTools, substep, x);
#pragma unroll
        for (int a = 0; a < 3; ++a) part[(FX + a) * cap + p] = x[a];
#pragma unroll
        for (int i = 0; i < 9; ++i) part[(FF + i) * cap + p] = Fn[i];
        const float E = SOL == SOLVER_PB ? 0.0f : particle_E(s, part, cap, p);
        if constexpr (kPack)
          p2g_particle_pk<FIXED, T>(s, x, vn, Cn, Fn, E, to, L, sc, ACC_ARGS, mark, ovf, st, parity, ev, bmax);
        else
          p2g_any<FIXED, SOL, PASS, T, kShell>(s, x, vn, Cn, Fn, E, to, L, ACC_ARGS, mark, ovf, st, parity, ev,
                                               bmax);
        // An update that moved the particle out of the grid (or left its
        // state not finite) is its last: the particle is left unchanged from
        // then on, so its v and C of this update are kept in memory with it.
        if (ev & (kEvDom | kEvNf)) {
#pragma unroll
          for (int a = 0; a < 3; ++a) part[(FV + a) * cap + p] = vn[a];
#pragma unroll
          for (int i = 0; i < 9; ++i) part[(FC + i) * cap + p] = Cn[i];
        }
      } else {
        p2g_any<FIXED, SOL, PASS, T, kShell>(s, x, vn, Cn, F, 0.0f, to, L, ACC_ARGS, mark, ovf, st, parity, ev,
                                             bmax);
      }
      count_events(cnt, ev);
    }
    if constexpr (kPack) record_bound(pb_wr, b, (unsigned)substep, bmax);
    const bool more = npos < walk.end;  // the same for the whole workgroup
    uint2 nitem = item;
    unsigned claim = 0u;
    if (more) {
      if (threadIdx.x == 0) claim = walk.claim(st);  // the item after the next one
      nitem = work[npos];
      if constexpr (kPack)
        if (threadIdx.x == 0) L.pbe[flip ? 0 : 1] = pb_rd[nitem.x & ~kDenseFlag];
      int nto[4];
      unit_origin<T>(s, nitem.x & ~kDenseFlag, nto);
      if constexpr (kTable)
        tile_stage_velocity_tab(s, nto, vel, flip ? L.v : Vb, L.vw[flip ? 0 : 1], L.p2);
      else if constexpr (kPack)
        tile_stage_velocity_max<T>(s, nto, vel, flip ? L.v : Vb, L.vw[flip ? 0 : 1]);
      else
        tile_stage_velocity<T>(s, nto, vel, flip ? L.v : Vb);
      if (threadIdx.x == 0) L.claimed[1] = claim;
    }
    __syncthreads();  // every P2G atomic into this tile is done; the next velocities are staged
    const unsigned nnpos = more ? L.claimed[1] : walk.end;
    if constexpr (kPack) {
      tile_flush_clear_pk<T>(s, to, L, am, ap0, ap1, ap2, sc.out());
      shell_flush_clear_pk<T>(s, to, L, am, ap0, ap1, ap2, sc.out(), pos + 1u, mark, ovf, st, parity);
    } else {
      tile_flush_clear<FIXED, T>(s, to, L, ACC_ARGS);
      shell_flush_clear<FIXED, T>(s, to, L, ACC_ARGS, pos + 1u, mark, ovf, st, parity);
    }
    if (threadIdx.x == 0) L.item_tag = npos + 1u;  // nothing reads it before the next barrier
    pos = npos;
    npos = nnpos;
    item = nitem;
    flip = !flip;
    if (more) __syncthreads();  // the tile is cleared; L.claimed[1] is read
  }
  if (threadIdx.x == 0) walk.finish(st);
  flush_counters(st, cnt);
}

// G2P that materialises the full state (x, v, C, F) in memory (the C slot
// holds the velocity gradient for standard MPM).
template <int SOL, bool PUSH, int T>
__global__ __launch_bounds__(TileShape<T>::kWG, 4) void k_g2p(float* __restrict__ part, int64_t cap,
                                             const uint32_t* __restrict__ blk_end,
                                             const uint2* __restrict__ work, Status* st,
                                             const float4* __restrict__ vel, const Clock* __restrict__ clk,
                                             int parity, const ToolDesc* __restrict__ tools, SimK s) {
  __shared__ Lds<T> L;
  long long substep = 0;
  if constexpr (PUSH) substep = clk[parity].substep;
  Counters cnt;
  const WorkWalk walk(st->n_work);
  unsigned pos = walk.first();
  while (pos < walk.end) {
    const uint2 item = work[pos];
    const unsigned b = item.x & ~kDenseFlag;
    const unsigned q = item_lane<T>(item.x);
    int to[4];
    unit_origin<T>(s, b, to);
    unsigned next = 0u;
    if (threadIdx.x == 0) next = walk.claim(st);
    tile_stage_velocity<T>(s, to, vel, L.v);
    __syncthreads();
    const unsigned pe = min(item.y + s.item_particles, blk_end[b]);
    for (unsigned p = item.y + q; p < pe; p += TileShape<T>::kWG) {
      float x[3], F[9];
#pragma unroll
      for (int a = 0; a < 3; ++a) x[a] = part[(FX + a) * cap + p];
#pragma unroll
      for (int i = 0; i < 9; ++i) F[i] = part[(FF + i) * cap + p];
      float vn[3], Cn[9];
      unsigned ev = 0u;
      if (!g2p_particle<SOL, T>(s, x, to, L.v, vel, vn, Cn, ev)) continue;  // no events
      count_events(cnt, ev);
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b2 = 0; b2 < 3; ++b2)
          part[(FF + 3 * a + b2) * cap + p] =
              F[3 * a + b2] +
              s.dt * (Cn[3 * a] * F[b2] + Cn[3 * a + 1] * F[3 + b2] + Cn[3 * a + 2] * F[6 + b2]);
#pragma unroll
      for (int a = 0; a < 3; ++a) x[a] += s.dt * vn[a];
      if constexpr (PUSH) push_out(s, tools + (size_t)to[3] * kMaxTools, substep, x);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        part[(FX + a) * cap + p] = x[a];
        part[(FV + a) * cap + p] = vn[a];
      }
#pragma unroll
      for (int i = 0; i < 9; ++i) part[(FC + i) * cap + p] = Cn[i];
    }
    if (threadIdx.x == 0) L.claimed[1] = next;
    __syncthreads();
    pos = L.claimed[1];
  }
  if (threadIdx.x == 0) walk.finish(st);
  flush_counters(st, cnt);
}

// ------------------------------------------------------------------ launchers
template <bool FIXED, int SOL, int T>
static void launch_p2g_t(Buffers& b, const SimK& s, int grid_wgs, int parity, hipStream_t st, KernelEvents ev) {
  using M = typename AccT<FIXED>::M;
  using P = typename AccT<FIXED>::P;
  launch_kernel(k_p2g<FIXED, SOL, T>, dim3(grid_wgs), dim3(TileShape<T>::kWG), st, ev, (const float*)b.part[b.cur], b.cap,
                     b.blk_end, b.work, b.status, (M*)b.acc_m, (P*)b.acc_p[0], (P*)b.acc_p[1],
                     (P*)b.acc_p[2], b.mark, b.ovf_list[0], b.ovf_list[1], (const Clock*)b.clock,
                     b.pbound[parity & 1], parity, s);
}

template <bool FIXED, int SOL, int PASS, bool PUSH, int T>
static void launch_g2p2g_t(Buffers& b, const SimK& s, int grid_wgs, int parity, hipStream_t st, KernelEvents ev) {
  using M = typename AccT<FIXED>::M;
  using P = typename AccT<FIXED>::P;
  launch_kernel(k_g2p2g<FIXED, SOL, PASS, PUSH, T>, dim3(grid_wgs), dim3(TileShape<T>::kWG), st, ev,
                     b.part[b.cur], b.cap, b.blk_end, b.work, b.status, (M*)b.acc_m, (P*)b.acc_p[0],
                     (P*)b.acc_p[1], (P*)b.acc_p[2], b.vel, b.mark, b.ovf_list[0], b.ovf_list[1],
                     (const Clock*)b.clock, (const unsigned long long*)b.pbound[(parity & 1) ^ 1],
                     b.pbound[parity & 1], parity, (const ToolDesc*)b.tools, s);
}

// The integrating passes with or without push-out.
template <bool FIXED, int SOL, int T>
static void launch_g2p2g_p(Buffers& b, const SimK& s, int grid_wgs, int parity, hipStream_t st, KernelEvents ev) {
  if (s.push_out)
    launch_g2p2g_t<FIXED, SOL, PB_FIRST, true, T>(b, s, grid_wgs, parity, st, ev);
  else
    launch_g2p2g_t<FIXED, SOL, PB_FIRST, false, T>(b, s, grid_wgs, parity, st, ev);
}

template <bool FIXED, int T>
static void launch_p2g_s(Buffers& b, const SimK& s, int grid_wgs, int parity, hipStream_t st, KernelEvents ev) {
  if (s.solver == SOLVER_PIC)
    launch_p2g_t<FIXED, SOLVER_PIC, T>(b, s, grid_wgs, parity, st, ev);
  else if (s.solver == SOLVER_PB)
    launch_p2g_t<FIXED, SOLVER_PB, T>(b, s, grid_wgs, parity, st, ev);
  else
    launch_p2g_t<FIXED, SOLVER_MLS, T>(b, s, grid_wgs, parity, st, ev);
}

template <bool FIXED, int T>
static void launch_g2p2g_s(Buffers& b, const SimK& s, int grid_wgs, int parity, hipStream_t st, int pass, KernelEvents ev) {
  if (s.solver == SOLVER_PIC)
    launch_g2p2g_p<FIXED, SOLVER_PIC, T>(b, s, grid_wgs, parity, st, ev);
  else if (s.solver == SOLVER_PB && pass == PB_ITER)
    launch_g2p2g_t<FIXED, SOLVER_PB, PB_ITER, false, T>(b, s, grid_wgs, parity, st, ev);
  else if (s.solver == SOLVER_PB)
    launch_g2p2g_p<FIXED, SOLVER_PB, T>(b, s, grid_wgs, parity, st, ev);
  else
    launch_g2p2g_p<FIXED, SOLVER_MLS, T>(b, s, grid_wgs, parity, st, ev);
}

void launch_p2g(Buffers& b, int64_t N, const SimK& s, int grid_wgs, int parity, hipStream_t st, KernelEvents ev) {
  (void)N;
  if (s.tile == 4) {
    if (s.fixed)
      launch_p2g_s<true, 4>(b, s, grid_wgs, parity, st, ev);
    else
      launch_p2g_s<false, 4>(b, s, grid_wgs, parity, st, ev);
  } else {
    if (s.fixed)
      launch_p2g_s<true, 8>(b, s, grid_wgs, parity, st, ev);
    else
      launch_p2g_s<false, 8>(b, s, grid_wgs, parity, st, ev);
  }
}

void launch_g2p2g(Buffers& b, int64_t N, const SimK& s, int grid_wgs, int parity, hipStream_t st, int pass, KernelEvents ev) {
  (void)N;
  if (s.tile == 4) {
    if (s.fixed)
      launch_g2p2g_s<true, 4>(b, s, grid_wgs, parity, st, pass, ev);
    else
      launch_g2p2g_s<false, 4>(b, s, grid_wgs, parity, st, pass, ev);
  } else {
    if (s.fixed)
      launch_g2p2g_s<true, 8>(b, s, grid_wgs, parity, st, pass, ev);
    else
      launch_g2p2g_s<false, 8>(b, s, grid_wgs, parity, st, pass, ev);
  }
}

template <int SOL, int T>
static void launch_g2p_t(Buffers& b, const SimK& s, int grid_wgs, int parity, hipStream_t st, KernelEvents ev) {
  const Clock* clk = (const Clock*)b.clock;
  const ToolDesc* tools = (const ToolDesc*)b.tools;
  if (s.push_out)
    launch_kernel(k_g2p<SOL, true, T>, dim3(grid_wgs), dim3(TileShape<T>::kWG), st, ev, b.part[b.cur], b.cap,
                       b.blk_end, b.work, b.status, b.vel, clk, parity, tools, s);
  else
    launch_kernel(k_g2p<SOL, false, T>, dim3(grid_wgs), dim3(TileShape<T>::kWG), st, ev, b.part[b.cur], b.cap,
                       b.blk_end, b.work, b.status, b.vel, clk, parity, tools, s);
}

template <int T>
static void launch_g2p_s(Buffers& b, const SimK& s, int grid_wgs, int parity, hipStream_t st, KernelEvents ev) {
  if (s.solver == SOLVER_PIC)
    launch_g2p_t<SOLVER_PIC, T>(b, s, grid_wgs, parity, st, ev);
  else
    launch_g2p_t<SOLVER_MLS, T>(b, s, grid_wgs, parity, st, ev);
}

void launch_g2p(Buffers& b, int64_t N, const SimK& s, int grid_wgs, int parity, hipStream_t st, KernelEvents ev) {
  (void)N;
  if (s.tile == 4)
    launch_g2p_s<4>(b, s, grid_wgs, parity, st, ev);
  else
    launch_g2p_s<8>(b, s, grid_wgs, parity, st, ev);
}

}  // namespace mpm
