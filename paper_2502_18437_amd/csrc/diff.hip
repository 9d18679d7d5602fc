// Differentiable rollout: the MLS-MPM substep on a dense grid in the caller's
// particle order, and its hand-written reverse-mode adjoint.
//
// The paper builds CRESSim-MPM for robot learning and names differentiable
// simulation as a direction (Sec. I, Sec. V); this path provides gradients of
// a loss on the final state with respect to each particle's stiffness
// (theta_p = log E_p), the tools' per-substep linear velocities and the
// starting state, for the substep of Algorithm 1 with the contact law of
// Sec. IV-A-C. Each stage is differentiated as written and the stages run in
// reverse order:
//   G2P:  x' = x + dt v', F' = (I + dt C') F, C' = (4/dx^2) sum N v_I d^T,
//         v' = sum N v_I (d = x_I - x_p): a scatter of the grid-velocity
//         cotangent plus the particle terms.
//   grid: walls zero the cotangent; the tools are reversed in the opposite
//         order through the contact law (including how the normal and the
//         curve tangent move with the node's position relative to the tool);
//         v_hat = p/m + dt g gives the momentum and mass cotangents.
//   P2G:  a gather of those cotangents; the stress term goes through the
//         fixed-corotated Kirchhoff stress and the polar-decomposition
//         derivative (dR = R [w]x with (tr(S) I - S) w = k(R^T dF)).
// Contact sets, stencil bases and clamps are held fixed: the derivative is
// that of the smooth piece the forward pass is on.
//
// Grid: n^3 nodes, node (i, j, k) at index (i n + j) n + k. Particle state
// blocks: x, v, C, F as AoS arrays (N x 3, N x 3, N x 9, N x 9).
//
// The two scatters (P2G forward, G2P reverse) walk the particles in a
// spatial order (DiffOrder): each workgroup takes a run of one grid block's
// particles, adds their contributions into an LDS tile of the block's
// stencil nodes with integer LDS atomics (the forward P2G in the fixed-point
// units of the main path, the cotangent scatter in int64 units chosen per
// run) and then adds the tile's non-empty nodes into the dense grid. A particle that has left its block's
// tile since the order was taken scatters straight into the dense grid.
#include <hip/hip_runtime.h>

#include "mpm_device.h"
#include "mpm_internal.h"
#include "diff_internal.h"
#include "p2g_fixed.h"

namespace mpm {

namespace {

constexpr int kDWG = 256;

unsigned blocks_for(int64_t n) {
  int64_t b = (n + kDWG - 1) / kDWG;
  if (b < 1) b = 1;
  if (b > (1 << 20)) b = 1 << 20;
  return (unsigned)b;
}

__device__ __forceinline__ bool finite_n(const float* a, int n) {
  float s = 0.0f;
  for (int i = 0; i < n; ++i) s += a[i] * 0.0f;
  return s == 0.0f;  // any inf or nan makes the sum nan
}

// Stencil base and fractional offsets; false if it leaves [0, n-1]^3.
__device__ __forceinline__ bool dense_stencil(const SimK& s, const float* x, int* base, float* f) {
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

// A particle takes part in a substep iff its state is finite and its stencil
// lies in the grid (otherwise the substep leaves it unchanged); 1 = non-finite,
// 2 = outside, 0 = live.
__device__ __forceinline__ int particle_state(const SimK& s, const float* x, const float* v, const float* C,
                                              const float* F, float e, int* base, float* f) {
  if (!(finite_n(x, 3) && finite_n(v, 3) && finite_n(C, 9) && finite_n(F, 9) && finite_n(&e, 1))) return 1;
  return dense_stencil(s, x, base, f) ? 0 : 2;
}

__device__ __forceinline__ int dense_index(const SimK& s, int i, int j, int k) {
  return (i * s.n + j) * s.n + k;
}

__device__ __forceinline__ void load_state(DState S, int64_t p, float* x, float* v, float* C, float* F) {
#pragma unroll
  for (int a = 0; a < 3; ++a) x[a] = S.x[3 * p + a], v[a] = S.v[3 * p + a];
#pragma unroll
  for (int i = 0; i < 9; ++i) C[i] = S.C[9 * p + i], F[i] = S.F[9 * p + i];
}

constexpr int kXcd = 8;

// ---------------------------------------------------------------- tiles
// Tile node (lx, ly, lz) of a block's kSpan^3 stencil tile, z fastest like
// the dense grid, so that a tile row flushes to consecutive addresses.
__device__ __forceinline__ int tile_index(int lx, int ly, int lz) { return (lx * kSpan + ly) * kSpan + lz; }

// Origin node of block b's tile (one scene; blocks x fastest).
__device__ __forceinline__ void tile_origin(const SimK& s, unsigned b, int* o) {
  o[0] = (int)(b % (unsigned)s.nb) * kTile;
  o[1] = (int)((b / (unsigned)s.nb) % (unsigned)s.nb) * kTile;
  o[2] = (int)(b / ((unsigned)s.nb * (unsigned)s.nb)) * kTile;
}

// Persistent walk of the work items: each XCD (workgroup w runs on XCD
// w % 8) takes one contiguous eighth of the spatially ordered list.
__device__ __forceinline__ void item_walk(unsigned n_items, unsigned* pos, unsigned* end, unsigned* stride) {
  const unsigned per = gridDim.x / kXcd;
  const unsigned xcd = blockIdx.x % kXcd, slot = blockIdx.x / kXcd;
  const unsigned chunk = (n_items + kXcd - 1) / kXcd;
  *pos = xcd * chunk + slot;
  *end = min(xcd * chunk + chunk, n_items);
  *stride = per;
}

// Stencil base relative to a tile origin; true if the whole stencil is in
// the tile.
__device__ __forceinline__ bool in_tile(const int* base, const int* org, int* l) {
#pragma unroll
  for (int a = 0; a < 3; ++a) l[a] = base[a] - org[a];
  return ((unsigned)l[0] <= (unsigned)(kSpan - 3)) && ((unsigned)l[1] <= (unsigned)(kSpan - 3)) &&
         ((unsigned)l[2] <= (unsigned)(kSpan - 3));
}

constexpr unsigned kScatterWGs = 1024;  // persistent scatter grid (a multiple of 8)

__device__ __forceinline__ void flush_status(Status* st, unsigned inv, unsigned dom, unsigned nf) {
  if (inv) atomicAdd(&st->n_inverted, (unsigned long long)inv);
  if (dom) atomicAdd(&st->n_domain, (unsigned long long)dom);
  if (nf) atomicAdd(&st->n_nonfinite, (unsigned long long)nf);
}

// ---------------------------------------------------------------- forward
// P2G of one particle straight into the dense grid (FP32 atomics).
__device__ __forceinline__ void p2g_direct(const SimK& s, const int* base, const float (*w)[3], const float* f,
                                           const float* v, const float* A, float* gm, float* gp0, float* gp1,
                                           float* gp2) {
  // x weights move down a register queue (no array indexed by ox)
  float wx = w[0][0], wx1 = w[0][1], wx2 = w[0][2];
#pragma unroll 1
  for (int ox = 0; ox < 3; ++ox) {
#pragma unroll
    for (int oy = 0; oy < 3; ++oy)
#pragma unroll
      for (int oz = 0; oz < 3; ++oz) {
        const float Nw = wx * w[1][oy] * w[2][oz];
        const float d[3] = {((float)ox - f[0]) * s.dx, ((float)oy - f[1]) * s.dx, ((float)oz - f[2]) * s.dx};
        const int I = dense_index(s, base[0] + ox, base[1] + oy, base[2] + oz);
        unsafeAtomicAdd(gm + I, Nw * s.mass);
        float* gp[3] = {gp0, gp1, gp2};
#pragma unroll
        for (int a = 0; a < 3; ++a)
          unsafeAtomicAdd(gp[a] + I, Nw * (s.mass * v[a] + A[3 * a] * d[0] + A[3 * a + 1] * d[1] + A[3 * a + 2] * d[2]));
      }
    wx = wx1;
    wx1 = wx2;
  }
}

struct P2GTile {
  uint32_t m[kSpanNodes];  // weight sums (2^-22 units)
  long long p0[kSpanNodes], p1[kSpanNodes], p2[kSpanNodes];  // momentum (fixed point)
};

__global__ __launch_bounds__(kDWG) void k_dp2g(SimK s, int64_t N, DState in, const float* __restrict__ E,
                                               DiffOrder o, float* gm, float* gp0, float* gp1, float* gp2,
                                               uint8_t* __restrict__ skip, Status* st, int count) {
  __shared__ P2GTile T;
  unsigned c_inv = 0, c_dom = 0, c_nf = 0;
  unsigned pos, end, stride;
  item_walk(o.info[0], &pos, &end, &stride);
  for (; pos < end; pos += stride) {
    const uint2 item = o.work[pos];
    const unsigned pe = min(item.y + (unsigned)kItemRollout, o.blk_end[item.x]);
    int org[3];
    tile_origin(s, item.x, org);
    for (int t = threadIdx.x; t < kSpanNodes; t += kDWG) {
      T.m[t] = 0u;
      T.p0[t] = 0ll;
      T.p1[t] = 0ll;
      T.p2[t] = 0ll;
    }
    __syncthreads();
    for (unsigned i = item.y + threadIdx.x; i < pe; i += kDWG) {
      const int64_t p = o.order[i];
      float x[3], v[3], C[9], F[9];
      load_state(in, p, x, v, C, F);
      const float e = E[p];
      int base[3];
      float f[3];
      const int ps = particle_state(s, x, v, C, F, e, base, f);
      skip[p] = ps != 0;
      if (ps == 1) {
        c_nf++;
        continue;
      }
      if (ps == 2) {
        c_dom++;
        continue;
      }
      P2GIn P;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        P.base[a] = base[a];
        bspline_w(f[a], P.w[a]);
      }
      float tau[9];
      bool inv;
      kirchhoff(F, s.c_mu * e, s.c_la * e, tau, &inv);
      if (inv) c_inv++;
      float A[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) A[k] = s.mass * C[k] - s.p2g_stress * tau[k];
      // |m v + A (x_I - x_p)| over the stencil must fit the fixed-point range
      float bound = 0.0f;
#pragma unroll
      for (int a = 0; a < 3; ++a)
        bound = fmaxf(bound, fabsf(s.mass * v[a]) + 1.5f * s.dx * (fabsf(A[3 * a]) + fabsf(A[3 * a + 1]) + fabsf(A[3 * a + 2])));
      int l[3];
      if (in_tile(base, org, l) && bound < s.p_limit) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const float qa = s.mass * v[a] - (A[3 * a] * f[0] + A[3 * a + 1] * f[1] + A[3 * a + 2] * f[2]) * s.dx;
          P.q[a] = (double)qa * s.fx_p;
#pragma unroll
          for (int b2 = 0; b2 < 3; ++b2) P.Adx[3 * a + b2] = (double)(A[3 * a + b2] * s.dx) * s.fx_p;
        }
        const int l0 = tile_index(l[0], l[1], l[2]);
        p2g_emit(P, [&](int ox, int oy, int oz, uint32_t wq, long long q0, long long q1, long long q2) {
          const int idx = l0 + tile_index(ox, oy, oz);
          atomicAdd(&T.m[idx], wq);
          atomicAdd((unsigned long long*)&T.p0[idx], (unsigned long long)q0);
          atomicAdd((unsigned long long*)&T.p1[idx], (unsigned long long)q1);
          atomicAdd((unsigned long long*)&T.p2[idx], (unsigned long long)q2);
        });
      } else {
        p2g_direct(s, base, P.w, f, v, A, gm, gp0, gp1, gp2);
      }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kSpanNodes; t += kDWG) {
      const uint32_t wq = T.m[t];
      const long long q0 = T.p0[t], q1 = T.p1[t], q2 = T.p2[t];
      if ((wq | q0 | q1 | q2) == 0) continue;
      const int gx = org[0] + t / (kSpan * kSpan), gy = org[1] + (t / kSpan) % kSpan, gz = org[2] + t % kSpan;
      if (gx >= s.n || gy >= s.n || gz >= s.n) continue;  // no stencil reaches past the grid
      const int I = dense_index(s, gx, gy, gz);
      unsafeAtomicAdd(gm + I, (float)wq * s.m_unit);
      unsafeAtomicAdd(gp0 + I, (float)((double)q0 * s.fx_p_inv));
      unsafeAtomicAdd(gp1 + I, (float)((double)q1 * s.fx_p_inv));
      unsafeAtomicAdd(gp2 + I, (float)((double)q2 * s.fx_p_inv));
    }
    __syncthreads();
  }
  // Particles outside the grid (or with a non-finite x) when the order was
  // taken: a skipped particle does not move, so they still are.
  for (int64_t i = o.info[1] + blockIdx.x * (int64_t)kDWG + threadIdx.x; i < N; i += (int64_t)gridDim.x * kDWG) {
    const int64_t p = o.order[i];
    float x[3], v[3], C[9], F[9];
    load_state(in, p, x, v, C, F);
    int base[3];
    float f[3];
    const int ps = particle_state(s, x, v, C, F, E[p], base, f);
    skip[p] = 1;
    if (ps == 1)
      c_nf++;
    else
      c_dom++;
  }
  if (count) flush_status(st, c_inv, c_dom, c_nf);
}

__device__ __forceinline__ bool wall_node(const SimK& s, int i, int j, int k) {
  const int lo = s.band, hi = s.n - 1 - s.band;
  return i < lo || i > hi || j < lo || j > hi || k < lo || k > hi;
}

__global__ __launch_bounds__(kDWG) void k_dgrid(SimK s, ToolSetK ts, float* gm, float* gp0, float* gp1, float* gp2,
                                                float4* __restrict__ vel, float4* __restrict__ hat) {
  const int64_t nn = (int64_t)s.n * s.n * s.n;
  for (int64_t I = blockIdx.x * (int64_t)kDWG + threadIdx.x; I < nn; I += (int64_t)gridDim.x * kDWG) {
    const int I32 = (int)I;  // n^3 < 2^31
    const int i = I32 / (s.n * s.n), j = (I32 / s.n) % s.n, k = I32 % s.n;
    const float m = gm[I];
    float v[3] = {0.0f, 0.0f, 0.0f};
    if (m > 0.0f) {
      v[0] = gp0[I] / m + s.dt * s.g[0];
      v[1] = gp1[I] / m + s.dt * s.g[1];
      v[2] = gp2[I] / m + s.dt * s.g[2];
      if (hat) hat[I] = make_float4(v[0], v[1], v[2], m);
      const float xI[3] = {(float)i * s.dx, (float)j * s.dx, (float)k * s.dx};
#pragma unroll 1
      for (int q = 0; q < ts.n; ++q)
        if (ts.t[q].type != TOOL_NONE) tool_contact(ts.t[q], xI, v);
      if (wall_node(s, i, j, k)) v[0] = v[1] = v[2] = 0.0f;
    } else if (hat) {
      hat[I] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    vel[I] = make_float4(v[0], v[1], v[2], 0.0f);
    gm[I] = 0.0f, gp0[I] = 0.0f, gp1[I] = 0.0f, gp2[I] = 0.0f;
  }
}

__global__ __launch_bounds__(kDWG) void k_dg2p(SimK s, int64_t N, DState in, const float4* __restrict__ vel,
                                               const uint8_t* __restrict__ skip, DState out) {
  const float Minv = 4.0f * s.inv_dx * s.inv_dx;
  for (int64_t p = blockIdx.x * (int64_t)kDWG + threadIdx.x; p < N; p += (int64_t)gridDim.x * kDWG) {
    float x[3], v[3], C[9], F[9];
    load_state(in, p, x, v, C, F);
    if (!skip[p]) {
      int base[3];
      float f[3];
      dense_stencil(s, x, base, f);
      float w[3][3];
#pragma unroll
      for (int a = 0; a < 3; ++a) bspline_w(f[a], w[a]);
      float vn[3] = {0.0f, 0.0f, 0.0f}, B[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll 1
      for (int ox = 0; ox < 3; ++ox)
#pragma unroll
        for (int oy = 0; oy < 3; ++oy)
#pragma unroll
          for (int oz = 0; oz < 3; ++oz) {
            const float Nw = w[0][ox] * w[1][oy] * w[2][oz];
            const float d[3] = {((float)ox - f[0]) * s.dx, ((float)oy - f[1]) * s.dx, ((float)oz - f[2]) * s.dx};
            const float4 g = vel[dense_index(s, base[0] + ox, base[1] + oy, base[2] + oz)];
            const float vI[3] = {g.x, g.y, g.z};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              vn[a] += Nw * vI[a];
#pragma unroll
              for (int b = 0; b < 3; ++b) B[3 * a + b] += Nw * vI[a] * d[b];
            }
          }
      float Fn[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) C[i] = Minv * B[i];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
          Fn[3 * a + b] = F[3 * a + b] + s.dt * (C[3 * a] * F[b] + C[3 * a + 1] * F[3 + b] + C[3 * a + 2] * F[6 + b]);
#pragma unroll
      for (int i = 0; i < 9; ++i) F[i] = Fn[i];
#pragma unroll
      for (int a = 0; a < 3; ++a) x[a] += s.dt * vn[a], v[a] = vn[a];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) out.x[3 * p + a] = x[a], out.v[3 * p + a] = v[a];
#pragma unroll
    for (int i = 0; i < 9; ++i) out.C[9 * p + i] = C[i], out.F[9 * p + i] = F[i];
  }
}

// ---------------------------------------------------------------- adjoint helpers
__device__ __forceinline__ void mm3(const float* A, const float* B, float* O) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) O[3 * r + c] = A[3 * r] * B[c] + A[3 * r + 1] * B[3 + c] + A[3 * r + 2] * B[6 + c];
}

// A^T B
__device__ __forceinline__ void mtm3(const float* A, const float* B, float* O) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) O[3 * r + c] = A[r] * B[c] + A[3 + r] * B[3 + c] + A[6 + r] * B[6 + c];
}

__device__ __forceinline__ void cof3(const float* F, float* o) {
  o[0] = F[4] * F[8] - F[5] * F[7];
  o[1] = F[5] * F[6] - F[3] * F[8];
  o[2] = F[3] * F[7] - F[4] * F[6];
  o[3] = F[2] * F[7] - F[1] * F[8];
  o[4] = F[0] * F[8] - F[2] * F[6];
  o[5] = F[1] * F[6] - F[0] * F[7];
  o[6] = F[1] * F[5] - F[2] * F[4];
  o[7] = F[2] * F[3] - F[0] * F[5];
  o[8] = F[0] * F[4] - F[1] * F[3];
}

// Fb += R [y]x with (tr(S) I - sym S) y = k(R^T Rb), S = R^T F.
__device__ __forceinline__ void polar_adjoint_dev(const float* F, const float* R, const float* Rb, float* Fb) {
  float S[9], M[9];
  mtm3(R, F, S);
  mtm3(R, Rb, M);
  const float m0 = M[7] - M[5], m1 = M[2] - M[6], m2 = M[3] - M[1];
  const float tr = S[0] + S[4] + S[8];
  float G[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) G[3 * r + c] = (r == c ? tr : 0.0f) - 0.5f * (S[3 * r + c] + S[3 * c + r]);
  float cg[9];
  cof3(G, cg);  // G symmetric: G^-1 = cof(G) / det G
  const float id = 1.0f / (G[0] * cg[0] + G[1] * cg[1] + G[2] * cg[2]);
  const float y0 = (cg[0] * m0 + cg[1] * m1 + cg[2] * m2) * id;
  const float y1 = (cg[3] * m0 + cg[4] * m1 + cg[5] * m2) * id;
  const float y2 = (cg[6] * m0 + cg[7] * m1 + cg[8] * m2) * id;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    // (R [y]x)_{r,:} = R_r x-product form: columns c0 = R_r1 y2 - R_r2 y1, ...
    Fb[3 * r + 0] += R[3 * r + 1] * y2 - R[3 * r + 2] * y1;
    Fb[3 * r + 1] += R[3 * r + 2] * y0 - R[3 * r + 0] * y2;
    Fb[3 * r + 2] += R[3 * r + 0] * y1 - R[3 * r + 1] * y0;
  }
}

enum { LAW_NONE = 0, LAW_CORRECT = 1, LAW_TANGENT = 2, LAW_STICKY = 3 };

// Frame of the contact of node xI with tool t (the geometry tool_contact
// evaluates), with the derivatives of the normal and the curve tangent with
// respect to xI (world frame, row-major).
__device__ __forceinline__ int contact_frame_dev(const ToolK& t, const float* xI, float* n, float* tg, float* Jn,
                                                 float* Jt) {
  const float r0 = xI[0] - t.c[0], r1 = xI[1] - t.c[1], r2 = xI[2] - t.c[2];
  float pl[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) pl[i] = t.R[i] * r0 + t.R[3 + i] * r1 + t.R[6 + i] * r2;
  float nl[3] = {0.0f, 1.0f, 0.0f}, tl[3] = {0.0f, 0.0f, 0.0f};
  float Jl[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, Jtl[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  float e[3] = {0.0f, 0.0f, 0.0f}, De[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  float L = 0.0f;
  bool use_e = false;
  int law;
  if (t.type == TOOL_CAPSULE || t.type == TOOL_SEGMENT) {
    const float h = t.size[0];
    e[0] = pl[0] - fminf(fmaxf(pl[0], -h), h), e[1] = pl[1], e[2] = pl[2];
    L = sqrtf(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    if (t.type == TOOL_CAPSULE) {
      if (!(L - t.size[1] < t.margin)) return LAW_NONE;
      law = LAW_CORRECT;
    } else {
      if (!(L < t.size[1])) return LAW_NONE;
      law = LAW_TANGENT;
      tl[0] = 1.0f;
    }
    if (pl[0] > -h && pl[0] < h) De[0] = 0.0f;
    use_e = L > 0.0f;
  } else if (t.type == TOOL_BOX) {
    float q[3], o[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) q[i] = fabsf(pl[i]) - t.size[i], o[i] = fmaxf(q[i], 0.0f);
    L = sqrtf(o[0] * o[0] + o[1] * o[1] + o[2] * o[2]);
    int k = 0;
    float qm = q[0];
    if (q[1] > qm) qm = q[1], k = 1;
    if (q[2] > qm) qm = q[2], k = 2;
    if (!(L + fminf(qm, 0.0f) < t.margin)) return LAW_NONE;
    law = LAW_CORRECT;
    if (L > 0.0f) {
#pragma unroll
      for (int i = 0; i < 3; ++i) e[i] = copysignf(o[i], pl[i]), De[4 * i] = q[i] > 0.0f ? 1.0f : 0.0f;
      use_e = true;
    } else {
      // face normal of axis k (selects rather than nl[k], pl[k], so that
      // the arrays stay in registers)
      const float pk = k == 0 ? pl[0] : (k == 1 ? pl[1] : pl[2]);
      const float sg = (pk < 0.0f) ? -1.0f : 1.0f;
      nl[0] = k == 0 ? sg : 0.0f;
      nl[1] = k == 1 ? sg : 0.0f;
      nl[2] = k == 2 ? sg : 0.0f;
    }
  } else if (t.type == TOOL_PLANE) {
    if (!(pl[1] < t.margin)) return LAW_NONE;
    law = LAW_CORRECT;
  } else if (t.type == TOOL_SLICER) {
    const float qx = fmaxf(fabsf(pl[0]) - t.size[0], 0.0f);
    const float qy = fmaxf(fabsf(pl[1]) - t.size[1], 0.0f);
    if (!(sqrtf(qx * qx + qy * qy + pl[2] * pl[2]) < t.margin)) return LAW_NONE;
    if (pl[1] > t.size[1]) {
      law = LAW_STICKY;
    } else {
      law = LAW_CORRECT;
      nl[0] = 0.0f, nl[1] = 0.0f, nl[2] = (pl[2] < 0.0f) ? -1.0f : 1.0f;
    }
  } else if (t.type == TOOL_ARC) {
    const float ra = t.size[0], ha = t.size[1];
    float ang = atan2f(pl[1], pl[0]);
    const bool interior = !(ang > ha || ang < -ha);
    if (!interior) {
      float sh, ch;
      sincosf(ha, &sh, &ch);
      const float dp = (pl[0] - ra * ch) * (pl[0] - ra * ch) + (pl[1] - ra * sh) * (pl[1] - ra * sh);
      const float dm = (pl[0] - ra * ch) * (pl[0] - ra * ch) + (pl[1] + ra * sh) * (pl[1] + ra * sh);
      ang = (dm < dp) ? -ha : ha;
    }
    float sa, ca;
    sincosf(ang, &sa, &ca);
    e[0] = pl[0] - ra * ca, e[1] = pl[1] - ra * sa, e[2] = pl[2];
    L = sqrtf(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    if (!(L < t.size[2])) return LAW_NONE;
    law = LAW_TANGENT;
    tl[0] = -sa, tl[1] = ca;
    float ga[3] = {0.0f, 0.0f, 0.0f};  // d ang / d pl on the open arc
    if (interior) {
      const float irho2 = 1.0f / (pl[0] * pl[0] + pl[1] * pl[1]);
      ga[0] = -pl[1] * irho2, ga[1] = pl[0] * irho2;
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      Jtl[j] = -ca * ga[j];
      Jtl[3 + j] = -sa * ga[j];
#pragma unroll
      for (int i = 0; i < 3; ++i) De[3 * i + j] = (i == j ? 1.0f : 0.0f) - ra * tl[i] * ga[j];
    }
    use_e = L > 0.0f;
    if (!use_e) nl[0] = -tl[1], nl[1] = tl[0], nl[2] = 0.0f;
  } else {
    return LAW_NONE;
  }
  if (use_e) {
    // n = e / |e|: dn/dpl = (I - n n^T) De / L
    const float il = 1.0f / L;
#pragma unroll
    for (int i = 0; i < 3; ++i) nl[i] = e[i] * il;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        float acc = 0.0f;
#pragma unroll
        for (int k = 0; k < 3; ++k) acc += ((i == k ? 1.0f : 0.0f) - nl[i] * nl[k]) * De[3 * k + j];
        Jl[3 * i + j] = acc * il;
      }
  } else if (t.type == TOOL_CAPSULE || t.type == TOOL_SEGMENT) {
    nl[0] = 0.0f, nl[1] = 1.0f, nl[2] = 0.0f;
  }
  // world frame: n = R nl, dn/dxI = R Jl R^T
  float T1[9];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    n[i] = t.R[3 * i] * nl[0] + t.R[3 * i + 1] * nl[1] + t.R[3 * i + 2] * nl[2];
    tg[i] = t.R[3 * i] * tl[0] + t.R[3 * i + 1] * tl[1] + t.R[3 * i + 2] * tl[2];
  }
  mm3(t.R, Jl, T1);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Jn[3 * i + j] = T1[3 * i] * t.R[3 * j] + T1[3 * i + 1] * t.R[3 * j + 1] + T1[3 * i + 2] * t.R[3 * j + 2];
  mm3(t.R, Jtl, T1);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Jt[3 * i + j] = T1[3 * i] * t.R[3 * j] + T1[3 * i + 1] * t.R[3 * j + 1] + T1[3 * i + 2] * t.R[3 * j + 2];
  return law;
}

// Reverse of v_out = v_r + law(v_in - v_r) for one node and one tool: vb
// holds the cotangent of v_out on entry and that of v_in on exit; the tool
// centre and linear-velocity cotangents are added to cb and lvb.
__device__ __forceinline__ void contact_adjoint_dev(const ToolK& t, const float* xI, const float* vin, float* vb,
                                                    float* cb, float* lvb) {
  const float r0 = xI[0] - t.c[0], r1 = xI[1] - t.c[1], r2 = xI[2] - t.c[2];
  if (t.reach2 >= 0.0f && r0 * r0 + r1 * r1 + r2 * r2 > t.reach2) return;  // far from the tool
  float n[3], tg[3], Jn[9], Jt[9];
  const int law = contact_frame_dev(t, xI, n, tg, Jn, Jt);
  if (law == LAW_NONE) return;
  const float* w = t.av;
  const float vr[3] = {t.lv[0] + w[1] * r2 - w[2] * r1, t.lv[1] + w[2] * r0 - w[0] * r2,
                       t.lv[2] + w[0] * r1 - w[1] * r0};
  const float u[3] = {vin[0] - vr[0], vin[1] - vr[1], vin[2] - vr[2]};
  float ub[3] = {0.0f, 0.0f, 0.0f}, nb[3] = {0.0f, 0.0f, 0.0f}, tb[3] = {0.0f, 0.0f, 0.0f};
  const float un = n[0] * u[0] + n[1] * u[1] + n[2] * u[2];
  if (law == LAW_STICKY) {
    // u' = 0
  } else if (!(un < 0.0f)) {
#pragma unroll
    for (int a = 0; a < 3; ++a) ub[a] = vb[a];
  } else {
    float unb = 0.0f;
    bool live = false;
    if (law == LAW_CORRECT) {
      const float t0 = u[0] - un * n[0], t1 = u[1] - un * n[1], t2 = u[2] - un * n[2];
      const float s = sqrtf(t0 * t0 + t1 * t1 + t2 * t2);
      if (s > 0.0f && 1.0f + t.mu * un / s > 0.0f) {
        live = true;
        const float is = 1.0f / s;
        const float th[3] = {t0 * is, t1 * is, t2 * is};
        const float tob = th[0] * vb[0] + th[1] * vb[1] + th[2] * vb[2];
        float tbar[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) tbar[a] = t.drag * (vb[a] + t.mu * un * (vb[a] - th[a] * tob) * is);
        unb = t.drag * t.mu * tob - (n[0] * tbar[0] + n[1] * tbar[1] + n[2] * tbar[2]);
#pragma unroll
        for (int a = 0; a < 3; ++a) ub[a] = tbar[a], nb[a] = -un * tbar[a];
      }
    } else {  // LAW_TANGENT
      const float ut = tg[0] * u[0] + tg[1] * u[1] + tg[2] * u[2];
      const float s = fabsf(ut);
      if (s > 0.0f && 1.0f + t.mu * un / s > 0.0f) {
        live = true;
        const float sg = ut < 0.0f ? -1.0f : 1.0f;
        const float amp = t.drag * (ut + t.mu * un * sg);
        const float ab = tg[0] * vb[0] + tg[1] * vb[1] + tg[2] * vb[2];
        const float utb = t.drag * ab;
        unb = t.drag * t.mu * sg * ab;
#pragma unroll
        for (int a = 0; a < 3; ++a) tb[a] = amp * vb[a] + utb * u[a], ub[a] = utb * tg[a];
      }
    }
    if (live) {
#pragma unroll
      for (int a = 0; a < 3; ++a) ub[a] += unb * n[a], nb[a] += unb * u[a];
    }
  }
  float vrb[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) vrb[a] = vb[a] - ub[a], vb[a] = ub[a], lvb[a] += vrb[a];
  cb[0] += w[1] * vrb[2] - w[2] * vrb[1];
  cb[1] += w[2] * vrb[0] - w[0] * vrb[2];
  cb[2] += w[0] * vrb[1] - w[1] * vrb[0];
#pragma unroll
  for (int j = 0; j < 3; ++j)
    cb[j] -= Jn[j] * nb[0] + Jn[3 + j] * nb[1] + Jn[6 + j] * nb[2] + Jt[j] * tb[0] + Jt[3 + j] * tb[1] + Jt[6 + j] * tb[2];
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// ---------------------------------------------------------------- adjoint kernels
// P2G reverse of one particle: gather of the momentum and mass cotangents,
// then the stress adjoint. Writes its v and C cotangents, adds to those of x
// and F and to d/d log E, and returns the resulting x, v, C, F cotangents in
// xb, vb, Cb, Fb; returns false (nothing changed) for a particle the
// substep skipped.
__device__ __forceinline__ bool bp2g_particle(const SimK& s, int64_t p, const DState& in,
                                              const float* __restrict__ E, const float4* __restrict__ pb,
                                              const DState& adj, float* __restrict__ theta_bar, float* xb,
                                              float* vb, float* Cb, float* Fb) {
  float x[3], v[3], C[9], F[9];
  load_state(in, p, x, v, C, F);
  const float e = E[p];
  int base[3];
  float f[3];
  if (particle_state(s, x, v, C, F, e, base, f) != 0) return false;
  float w[3][3], dw[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) bspline_w(f[a], w[a]), bspline_dw(f[a], dw[a]);
  const float mu = s.c_mu * e, la = s.c_la * e;
  float tau[9], R[9];
  bool inv;
  const float J = kirchhoff_r(F, mu, la, tau, R, &inv);
  float A[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) A[i] = s.mass * C[i] - s.p2g_stress * tau[i];
  float vbar[3] = {0.0f, 0.0f, 0.0f}, Ab[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, xg[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll 1
  for (int ox = 0; ox < 3; ++ox)
#pragma unroll
    for (int oy = 0; oy < 3; ++oy)
#pragma unroll
      for (int oz = 0; oz < 3; ++oz) {
        const float Nw = w[0][ox] * w[1][oy] * w[2][oz];
        const float dN[3] = {dw[0][ox] * w[1][oy] * w[2][oz] * s.inv_dx, w[0][ox] * dw[1][oy] * w[2][oz] * s.inv_dx,
                             w[0][ox] * w[1][oy] * dw[2][oz] * s.inv_dx};
        const float d[3] = {((float)ox - f[0]) * s.dx, ((float)oy - f[1]) * s.dx, ((float)oz - f[2]) * s.dx};
        const float4 g = pb[dense_index(s, base[0] + ox, base[1] + oy, base[2] + oz)];
        const float P[3] = {g.x, g.y, g.z};
        float contrib = s.mass * g.w;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          contrib += P[a] * (s.mass * v[a] + A[3 * a] * d[0] + A[3 * a + 1] * d[1] + A[3 * a + 2] * d[2]);
          vbar[a] += Nw * s.mass * P[a];
#pragma unroll
          for (int b = 0; b < 3; ++b) Ab[3 * a + b] += Nw * P[a] * d[b];
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) xg[j] += dN[j] * contrib - Nw * (A[j] * P[0] + A[3 + j] * P[1] + A[6 + j] * P[2]);
      }
#pragma unroll
  for (int i = 0; i < 9; ++i) Fb[i] = adj.F[9 * p + i];
  // tau cotangent: A = m C - p2g_stress tau
  float tb[9];
  float th = 0.0f;
#pragma unroll
  for (int i = 0; i < 9; ++i) tb[i] = -s.p2g_stress * Ab[i], th += tb[i] * tau[i];
  // tau1 = 2 mu (F - R) F^T: Fb += 2 mu (tb F + tb^T (F - R)), Rb = -2 mu tb F
  float tbF[9], Rb[9], D[9], tbtD[9];
  mm3(tb, F, tbF);
#pragma unroll
  for (int i = 0; i < 9; ++i) D[i] = F[i] - R[i];
  mtm3(tb, D, tbtD);
#pragma unroll
  for (int i = 0; i < 9; ++i) Fb[i] += 2.0f * mu * (tbF[i] + tbtD[i]), Rb[i] = -2.0f * mu * tbF[i];
  polar_adjoint_dev(F, R, Rb, Fb);
  // tau2 = la (J^2 - J) I: Fb += la (2J - 1) tr(tb) cof(F)
  float cf[9];
  cof3(F, cf);
  const float kv = la * (2.0f * J - 1.0f) * (tb[0] + tb[4] + tb[8]);
#pragma unroll
  for (int i = 0; i < 9; ++i) Fb[i] += kv * cf[i], adj.F[9 * p + i] = Fb[i];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    xb[a] = adj.x[3 * p + a] + xg[a];
    adj.x[3 * p + a] = xb[a];
    vb[a] = vbar[a];
    adj.v[3 * p + a] = vb[a];
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) Cb[i] = s.mass * Ab[i], adj.C[9 * p + i] = Cb[i];
  theta_bar[p] += th;
  return true;
}

// G2P reverse: scatter of the grid-velocity cotangent, x and F cotangents.
//
// A work item has at most one particle per thread. The cotangent
// contributions N q (q = v'_bar + B_bar (x_I - x_p)) go into the LDS tile as
// int64 in units of 2^-e, with e chosen per item so that the largest
// contribution bound of the item is about 2^40 units (a workgroup max over
// |v'_bar_a| + 1.5 dx sum_b |B_bar_ab|); the flush converts back. Integer LDS
// atomics run about 25 times faster than FP32 ones on this GPU. An item whose
// bound is zero or not finite, and particles outside their block's tile, add
// FP32 values straight into the dense grid.
static_assert(kItemRollout == kDWG, "one particle per thread in a rollout work item");

struct BG2PTile {
  float4 v[kSpanNodes];                                          // staged grid velocity
  long long g0[kSpanNodes], g1[kSpanNodes], g2[kSpanNodes];      // cotangent sums (2^-e units)
  float wmax[kDWG / 64];
};

// With FUSED, the P2G reverse of the substep that follows (state `next`,
// momentum and mass cotangents `pb`) runs first for each particle, in the
// same thread: it reads only that particle's data, and a particle this
// substep skips was skipped by the next one too (it did not move).
template <bool FUSED>
__global__ __launch_bounds__(kDWG) void k_bg2p(SimK s, int64_t N, DState in, const float* __restrict__ E,
                                               const float4* __restrict__ vel, DiffOrder o, DState adj,
                                               float* gvb0, float* gvb1, float* gvb2, DState next,
                                               const float4* __restrict__ pb, float* __restrict__ theta_bar) {
  __shared__ BG2PTile T;
  const float Minv = 4.0f * s.inv_dx * s.inv_dx;
  unsigned pos, end, stride;
  item_walk(o.info[0], &pos, &end, &stride);
  for (; pos < end; pos += stride) {
    const uint2 item = o.work[pos];
    const unsigned pe = min(item.y + (unsigned)kItemRollout, o.blk_end[item.x]);
    int org[3];
    tile_origin(s, item.x, org);
    for (int t = threadIdx.x; t < kSpanNodes; t += kDWG) {
      const int gx = org[0] + t / (kSpan * kSpan), gy = org[1] + (t / kSpan) % kSpan, gz = org[2] + t % kSpan;
      T.v[t] = (gx < s.n && gy < s.n && gz < s.n) ? vel[dense_index(s, gx, gy, gz)] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      T.g0[t] = 0ll;
      T.g1[t] = 0ll;
      T.g2[t] = 0ll;
    }
    __syncthreads();
    // Phase 1: this thread's particle up to the cotangents of v' and C'.
    const unsigned i = item.y + threadIdx.x;
    int64_t p = -1;
    int base[3] = {0, 0, 0}, l[3] = {0, 0, 0};
    float f[3] = {0.0f, 0.0f, 0.0f}, xb[3] = {0.0f, 0.0f, 0.0f}, vnb[3] = {0.0f, 0.0f, 0.0f};
    float Bb[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    bool live = false, tiled = false;
    float bound = 0.0f;
    if (i < pe) {
      p = o.order[i];
      float x[3], v[3], C[9], F[9];
      load_state(in, p, x, v, C, F);
      // a skipped particle is unchanged by the substep: its cotangent passes through
      live = particle_state(s, x, v, C, F, E[p], base, f) == 0;
      if (live) {
        tiled = in_tile(base, org, l);
        const int l0 = tile_index(l[0], l[1], l[2]);
        float w[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a) bspline_w(f[a], w[a]);
        float B[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        float wx = w[0][0], wx1 = w[0][1], wx2 = w[0][2];
#pragma unroll 1
        for (int ox = 0; ox < 3; ++ox) {
#pragma unroll
          for (int oy = 0; oy < 3; ++oy)
#pragma unroll
            for (int oz = 0; oz < 3; ++oz) {
              const float Nw = wx * w[1][oy] * w[2][oz];
              const float d[3] = {((float)ox - f[0]) * s.dx, ((float)oy - f[1]) * s.dx, ((float)oz - f[2]) * s.dx};
              const float4 g = tiled ? T.v[l0 + tile_index(ox, oy, oz)]
                                     : vel[dense_index(s, base[0] + ox, base[1] + oy, base[2] + oz)];
              const float vI[3] = {g.x, g.y, g.z};
#pragma unroll
              for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b2 = 0; b2 < 3; ++b2) B[3 * a + b2] += Nw * vI[a] * d[b2];
            }
          wx = wx1;
          wx1 = wx2;
        }
        float vb[3], Cb[9], Fb[9];
        if (!(FUSED && bp2g_particle(s, p, next, E, pb, adj, theta_bar, xb, vb, Cb, Fb)))
          load_state(adj, p, xb, vb, Cb, Fb);
        // x' = x + dt v', F' = G F (G = I + dt C'), C' = Minv B, v' = sum N v_I.
#pragma unroll
        for (int a = 0; a < 3; ++a) vnb[a] = vb[a] + s.dt * xb[a];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            // Cb' + dt Fb F^T, then the Minv of C' = Minv B
            const float FbFt = Fb[3 * r] * F[3 * c] + Fb[3 * r + 1] * F[3 * c + 1] + Fb[3 * r + 2] * F[3 * c + 2];
            Bb[3 * r + c] = Minv * (Cb[3 * r + c] + s.dt * FbFt);
          }
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            // G^T Fb with G_kr = delta_kr + dt Minv B_kr
            float acc = Fb[3 * r + c];
#pragma unroll
            for (int k = 0; k < 3; ++k) acc += s.dt * Minv * B[3 * k + r] * Fb[3 * k + c];
            adj.F[9 * p + 3 * r + c] = acc;
          }
        if (tiled) {
#pragma unroll
          for (int a = 0; a < 3; ++a)
            bound = fmaxf(bound, fabsf(vnb[a]) + 1.5f * s.dx * (fabsf(Bb[3 * a]) + fabsf(Bb[3 * a + 1]) + fabsf(Bb[3 * a + 2])));
        }
      }
    }
    // Item scale: the largest bound over the workgroup (NaN propagates).
    float m = bound;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const float other = __shfl_xor(m, off, 64);
      m = (m != m || other != other) ? __int_as_float(0x7fc00000) : fmaxf(m, other);
    }
    if ((threadIdx.x & 63) == 0) T.wmax[threadIdx.x >> 6] = m;
    __syncthreads();
    float mx = T.wmax[0];
#pragma unroll
    for (int w2 = 1; w2 < kDWG / 64; ++w2) mx = (mx != mx || T.wmax[w2] != T.wmax[w2]) ? mx + T.wmax[w2] : fmaxf(mx, T.wmax[w2]);
    const bool fixed = isfinite(mx) && mx > 0.0f;
    const int e = fixed ? 40 - ilogbf(mx) : 0;
    const double unit = ldexp(1.0, e), unit_inv = ldexp(1.0, -e);
    // Phase 2: scatter and the x cotangent.
    if (live) {
      float w[3][3], dw[3][3];
#pragma unroll
      for (int a = 0; a < 3; ++a) bspline_w(f[a], w[a]), bspline_dw(f[a], dw[a]);
      const bool lds = tiled && fixed;
      const int l0 = tile_index(l[0], l[1], l[2]);
      float xg[3] = {0.0f, 0.0f, 0.0f};
      float wx = w[0][0], wx1 = w[0][1], wx2 = w[0][2], dwx = dw[0][0], dwx1 = dw[0][1], dwx2 = dw[0][2];
#pragma unroll 1
      for (int ox = 0; ox < 3; ++ox) {
#pragma unroll
        for (int oy = 0; oy < 3; ++oy)
#pragma unroll
          for (int oz = 0; oz < 3; ++oz) {
            const float Nw = wx * w[1][oy] * w[2][oz];
            const float dN[3] = {dwx * w[1][oy] * w[2][oz] * s.inv_dx, wx * dw[1][oy] * w[2][oz] * s.inv_dx,
                                 wx * w[1][oy] * dw[2][oz] * s.inv_dx};
            const float d[3] = {((float)ox - f[0]) * s.dx, ((float)oy - f[1]) * s.dx, ((float)oz - f[2]) * s.dx};
            const float4 g = tiled ? T.v[l0 + tile_index(ox, oy, oz)]
                                   : vel[dense_index(s, base[0] + ox, base[1] + oy, base[2] + oz)];
            const float vI[3] = {g.x, g.y, g.z};
            float q[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) q[a] = vnb[a] + Bb[3 * a] * d[0] + Bb[3 * a + 1] * d[1] + Bb[3 * a + 2] * d[2];
            if (lds) {
              const int idx = l0 + tile_index(ox, oy, oz);
              atomicAdd((unsigned long long*)&T.g0[idx], (unsigned long long)fx_mul((double)(Nw * q[0]), unit));
              atomicAdd((unsigned long long*)&T.g1[idx], (unsigned long long)fx_mul((double)(Nw * q[1]), unit));
              atomicAdd((unsigned long long*)&T.g2[idx], (unsigned long long)fx_mul((double)(Nw * q[2]), unit));
            } else {
              const int I = dense_index(s, base[0] + ox, base[1] + oy, base[2] + oz);
              unsafeAtomicAdd(gvb0 + I, Nw * q[0]);
              unsafeAtomicAdd(gvb1 + I, Nw * q[1]);
              unsafeAtomicAdd(gvb2 + I, Nw * q[2]);
            }
            const float sc = vI[0] * q[0] + vI[1] * q[1] + vI[2] * q[2];
#pragma unroll
            for (int j = 0; j < 3; ++j)
              xg[j] += dN[j] * sc - Nw * (Bb[j] * vI[0] + Bb[3 + j] * vI[1] + Bb[6 + j] * vI[2]);
          }
        wx = wx1;
        wx1 = wx2;
        dwx = dwx1;
        dwx1 = dwx2;
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) adj.x[3 * p + a] = xb[a] + xg[a];
    }
    __syncthreads();
    if (fixed) {
      for (int t = threadIdx.x; t < kSpanNodes; t += kDWG) {
        const long long a0 = T.g0[t], a1 = T.g1[t], a2 = T.g2[t];
        if ((a0 | a1 | a2) == 0) continue;
        const int gx = org[0] + t / (kSpan * kSpan), gy = org[1] + (t / kSpan) % kSpan, gz = org[2] + t % kSpan;
        if (gx >= s.n || gy >= s.n || gz >= s.n) continue;
        const int I = dense_index(s, gx, gy, gz);
        unsafeAtomicAdd(gvb0 + I, (float)((double)a0 * unit_inv));
        unsafeAtomicAdd(gvb1 + I, (float)((double)a1 * unit_inv));
        unsafeAtomicAdd(gvb2 + I, (float)((double)a2 * unit_inv));
      }
    }
    __syncthreads();
  }
}

// Grid reverse: walls, tools in reverse order, v_hat = p/m + dt g. Writes the
// momentum and mass cotangents (pb) and clears the velocity cotangent.
__global__ __launch_bounds__(kDWG) void k_bgrid(SimK s, ToolSetK ts, const float4* __restrict__ hat, float* gvb0,
                                                float* gvb1, float* gvb2, float4* __restrict__ pb,
                                                double* __restrict__ tool_red) {
  const int64_t nn = (int64_t)s.n * s.n * s.n;
  // Per-wave tool sums, accumulated over the trips and then added into this
  // workgroup's copy of the substep's sums.
  __shared__ double red[kDWG / 64][kMaxTools * 6];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int c = lane; c < kMaxTools * 6; c += 64) red[wave][c] = 0.0;
  __syncthreads();
  // Every lane runs the same trip count so that the wave reductions below
  // see full waves.
  const int64_t stride = (int64_t)gridDim.x * kDWG;
  const int64_t first = blockIdx.x * (int64_t)kDWG + threadIdx.x;
  const int64_t trips = (nn + stride - 1) / stride;
  for (int64_t it = 0; it < trips; ++it) {
    const int64_t I = first + it * stride;
    const bool inside = I < nn;
    float4 h = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    float vb[3] = {0.0f, 0.0f, 0.0f};
    int i = 0, j = 0, k = 0;
    if (inside) {
      h = hat[I];
      vb[0] = gvb0[I], vb[1] = gvb1[I], vb[2] = gvb2[I];
      gvb0[I] = 0.0f, gvb1[I] = 0.0f, gvb2[I] = 0.0f;
      const int I32 = (int)I;  // n^3 < 2^31
      i = I32 / (s.n * s.n), j = (I32 / s.n) % s.n, k = I32 % s.n;
    }
    const float m = h.w;
    const bool live = inside && m > 0.0f && !wall_node(s, i, j, k);
    if (!live) vb[0] = vb[1] = vb[2] = 0.0f;
    const float xI[3] = {(float)i * s.dx, (float)j * s.dx, (float)k * s.dx};
#pragma unroll 1
    for (int q = ts.n - 1; q >= 0; --q) {
      const ToolK& t = ts.t[q];
      if (t.type == TOOL_NONE) continue;  // uniform across the wave
      float cb[3] = {0.0f, 0.0f, 0.0f}, lvb[3] = {0.0f, 0.0f, 0.0f};
      if (live) {
        // velocity entering tool q: replay tools 0..q-1 from v_hat
        float vin[3] = {h.x, h.y, h.z};
#pragma unroll 1
        for (int r = 0; r < q; ++r)
          if (ts.t[r].type != TOOL_NONE) tool_contact(ts.t[r], xI, vin);
        contact_adjoint_dev(t, xI, vin, vb, cb, lvb);
      }
      const bool any = (cb[0] != 0.0f) || (cb[1] != 0.0f) || (cb[2] != 0.0f) || (lvb[0] != 0.0f) ||
                       (lvb[1] != 0.0f) || (lvb[2] != 0.0f);
      if (__ballot(any) != 0) {
        const float r6[6] = {lvb[0], lvb[1], lvb[2], cb[0], cb[1], cb[2]};
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          const float sum = wave_sum(r6[c]);
          if (lane == 0) red[wave][6 * q + c] += (double)sum;
        }
      }
    }
    if (inside) {
      float4 o = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if (live) {
        const float im = 1.0f / m;
        o.x = vb[0] * im, o.y = vb[1] * im, o.z = vb[2] * im;
        o.w = -(vb[0] * (h.x - s.dt * s.g[0]) + vb[1] * (h.y - s.dt * s.g[1]) + vb[2] * (h.z - s.dt * s.g[2])) * im;
      }
      pb[I] = o;
    }
  }
  __syncthreads();
  double* mine = tool_red + (size_t)(blockIdx.x % kToolRedCopies) * (kMaxTools * 6);
  for (int c = threadIdx.x; c < kMaxTools * 6; c += kDWG) {
    double v = 0.0;
#pragma unroll
    for (int w2 = 0; w2 < kDWG / 64; ++w2) v += red[w2][c];
    if (v != 0.0) atomicAdd(mine + c, v);
  }
}

// P2G reverse of every particle (the last step of a substep's reverse when
// no G2P reverse of the substep before follows it).
__global__ __launch_bounds__(kDWG) void k_bp2g(SimK s, int64_t N, DState in, const float* __restrict__ E,
                                               const float4* __restrict__ pb, DState adj,
                                               float* __restrict__ theta_bar) {
  for (int64_t p = blockIdx.x * (int64_t)kDWG + threadIdx.x; p < N; p += (int64_t)gridDim.x * kDWG) {
    float xb[3], vb[3], Cb[9], Fb[9];
    (void)bp2g_particle(s, p, in, E, pb, adj, theta_bar, xb, vb, Cb, Fb);
  }
}

// ---------------------------------------------------------------- small kernels
__global__ void k_fill_f32(float* p, int64_t n, float v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_f64(double* p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_sum_tool_copies(const double* __restrict__ parts, int T, double* __restrict__ out) {
  constexpr int kRow = kMaxTools * 6;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < T * kRow; i += gridDim.x * blockDim.x) {
    const int j = i / kRow, c = i % kRow;
    double v = 0.0;
    for (int k = 0; k < kToolRedCopies; ++k) v += parts[((size_t)j * kToolRedCopies + k) * kRow + c];
    out[i] = v;
  }
}

__global__ void k_exp(const float* theta, float* E, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    E[i] = expf(theta[i]);
}

__global__ void k_unpermute_E(const float* __restrict__ part, const uint32_t* __restrict__ id, int64_t cap,
                              int64_t N, int has_E, float E_default, float* __restrict__ E) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
    E[id[i]] = has_E ? part[FE * cap + i] : E_default;
}

}  // namespace

void launch_diff_substep(const DiffGrid& g, float4* vel, float4* hat, const SimK& s, const ToolSetK& tools,
                         int64_t N, DState in, const float* E, DState out, bool count, Status* st,
                         const DiffOrder& o, hipStream_t stream) {
  const int64_t nn = (int64_t)s.n * s.n * s.n;
  hipLaunchKernelGGL(k_dp2g, dim3(kScatterWGs), dim3(kDWG), 0, stream, s, N, in, E, o, g.m, g.p[0], g.p[1],
                     g.p[2], g.skip, st, count ? 1 : 0);
  hipLaunchKernelGGL(k_dgrid, dim3(blocks_for(nn)), dim3(kDWG), 0, stream, s, tools, g.m, g.p[0], g.p[1], g.p[2],
                     vel, hat);
  if (out.x)
    hipLaunchKernelGGL(k_dg2p, dim3(blocks_for(N)), dim3(kDWG), 0, stream, s, N, in, (const float4*)vel,
                       (const uint8_t*)g.skip, out);
}

void launch_adjoint_head(const DiffGrid& g, const float4* vel, const float4* hat, const SimK& s,
                         const ToolSetK& tools, int64_t N, DState in, const float* E, DState adj, float* theta_bar,
                         double* tool_red, const DiffOrder& o, const DState* pending, hipStream_t stream) {
  const int64_t nn = (int64_t)s.n * s.n * s.n;
  if (pending)
    hipLaunchKernelGGL(k_bg2p<true>, dim3(kScatterWGs), dim3(kDWG), 0, stream, s, N, in, E, vel, o, adj, g.vb[0],
                       g.vb[1], g.vb[2], *pending, (const float4*)g.pb, theta_bar);
  else
    hipLaunchKernelGGL(k_bg2p<false>, dim3(kScatterWGs), dim3(kDWG), 0, stream, s, N, in, E, vel, o, adj, g.vb[0],
                       g.vb[1], g.vb[2], in, (const float4*)g.pb, theta_bar);
  hipLaunchKernelGGL(k_bgrid, dim3(blocks_for(nn)), dim3(kDWG), 0, stream, s, tools, hat, g.vb[0],
                     g.vb[1], g.vb[2], g.pb, tool_red);
}

void launch_adjoint_tail(const DiffGrid& g, const SimK& s, int64_t N, DState in, const float* E, DState adj,
                         float* theta_bar, hipStream_t stream) {
  hipLaunchKernelGGL(k_bp2g, dim3(blocks_for(N)), dim3(kDWG), 0, stream, s, N, in, E, (const float4*)g.pb, adj,
                     theta_bar);
}

void launch_sum_tool_copies(const double* parts, int T, double* out, hipStream_t st) {
  if (T <= 0) return;
  hipLaunchKernelGGL(k_sum_tool_copies, dim3(blocks_for((int64_t)T * kMaxTools * 6)), dim3(kDWG), 0, st, parts, T,
                     out);
}

void launch_fill_f32(float* p, int64_t n, float v, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_f32, dim3(blocks_for(n)), dim3(kDWG), 0, st, p, n, v);
}

void launch_fill_f64(double* p, int64_t n, double v, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_f64, dim3(blocks_for(n)), dim3(kDWG), 0, st, p, n, v);
}

void launch_exp(const float* theta, float* E, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_exp, dim3(blocks_for(n)), dim3(kDWG), 0, st, theta, E, n);
}

void launch_unpermute_E(const Buffers& b, int64_t N, const SimK& s, float* E, hipStream_t st) {
  if (N <= 0) return;
  hipLaunchKernelGGL(k_unpermute_E, dim3(blocks_for(N)), dim3(kDWG), 0, st, (const float*)b.part[b.cur],
                     (const uint32_t*)b.id[b.cur], b.cap, N, s.has_E, s.E_default, E);
}

}  // namespace mpm
