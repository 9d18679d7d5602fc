// Device-side per-particle and per-node arithmetic of the MPM substep
// (FP32): quadratic B-spline weights and their derivatives, polar
// decomposition, the fixed-corotated and Neo-Hookean Kirchhoff stresses, the
// PB-MPM constraint projection, tool SDFs and the contact law.
#pragma once

#include <hip/hip_runtime.h>

#include "mpm_internal.h"

namespace mpm {

// Quadratic B-spline weights of the nodes base, base+1, base+2 along one
// axis, f = x/dx - base in [0.5, 1.5) (Sec. III-A: 3 nodes per dimension).
__device__ __forceinline__ void bspline_w(float f, float w[3]) {
  const float a = 1.5f - f, b = f - 1.0f, c = f - 0.5f;
  w[0] = 0.5f * a * a;
  w[1] = 0.75f - b * b;
  w[2] = 0.5f * c * c;
}

__device__ __forceinline__ float det3(const float* X) {
  return X[0] * (X[4] * X[8] - X[5] * X[7]) - X[1] * (X[3] * X[8] - X[5] * X[6]) +
         X[2] * (X[3] * X[7] - X[4] * X[6]);
}

// Rotation factor of F (det F > 0) by Newton's iteration for the polar
// decomposition, X <- (z X + X^-T / z) / 2 (Higham 1986, "Computing the polar
// decomposition -- with applications"), with the determinant scaling
// z = |det X|^(-1/3) (Byers & Xu 2008) on the first two iterations when det X
// is far from 1. Near convergence the distance of the stretch from I is
// squared every step, so the loop stops once an update is below 1e-4: the
// next error is then below FP32 round-off. X^-T = cof(X) / det X uses the
// hardware reciprocal; the fixed point is still orthogonal to within its
// rounding. Returns false if it did not converge.
__device__ inline bool polar_newton(const float* F, float* R) {
  float X[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) X[i] = F[i];
  for (int it = 0; it < 16; ++it) {
    float c[9];
    c[0] = X[4] * X[8] - X[5] * X[7];
    c[1] = X[5] * X[6] - X[3] * X[8];
    c[2] = X[3] * X[7] - X[4] * X[6];
    c[3] = X[2] * X[7] - X[1] * X[8];
    c[4] = X[0] * X[8] - X[2] * X[6];
    c[5] = X[1] * X[6] - X[0] * X[7];
    c[6] = X[1] * X[5] - X[2] * X[4];
    c[7] = X[2] * X[3] - X[0] * X[5];
    c[8] = X[0] * X[4] - X[1] * X[3];
    const float det = X[0] * c[0] + X[1] * c[1] + X[2] * c[2];
    if (!(det > 0.0f)) return false;
    float z = 1.0f;
    if (it < 2 && fabsf(det - 1.0f) > 0.05f) z = rcbrtf(det);
    const float a = 0.5f * z;
    const float b = 0.5f * __builtin_amdgcn_rcpf(z * det);
    float delta = 0.0f;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const float xn = a * X[i] + b * c[i];
      delta = fmaxf(delta, fabsf(xn - X[i]));
      X[i] = xn;
    }
    if (delta < 1e-4f) {
#pragma unroll
      for (int i = 0; i < 9; ++i) R[i] = X[i];
      return true;
    }
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) R[i] = X[i];
  return false;
}

// Givens-type rotation of the symmetric eigenproblem: the cosine and sine
// that zero the (p, q) entry of a symmetric matrix with diagonal app, aqq and
// off-diagonal apq (the classical Jacobi angle, |theta| <= pi/4).
__device__ __forceinline__ void jacobi_angle(float app, float aqq, float apq, float* c, float* s) {
  if (fabsf(apq) < 1e-30f) {
    *c = 1.0f;
    *s = 0.0f;
    return;
  }
  const float tau = (aqq - app) / (2.0f * apq);
  const float t = copysignf(1.0f, tau) / (fabsf(tau) + sqrtf(1.0f + tau * tau));
  *c = rsqrtf(1.0f + t * t);
  *s = t * *c;
}

// q <- q * (cos(phi/2), sin(phi/2) e_axis): composes a rotation by phi about
// a coordinate axis on the right of the rotation held as unit quaternion q
// (w, x, y, z), given cos(phi) = c and sin(phi) = s with |phi| <= pi/4.
__device__ __forceinline__ void quat_turn(float* q, int axis, float c, float s) {
  const float ch = sqrtf(0.5f * (1.0f + c));
  const float sh = 0.5f * s / ch;
  float e[3] = {0.0f, 0.0f, 0.0f};
  e[axis] = sh;
  const float w = q[0] * ch - (q[1] * e[0] + q[2] * e[1] + q[3] * e[2]);
  const float x = q[0] * e[0] + ch * q[1] + (q[2] * e[2] - q[3] * e[1]);
  const float y = q[0] * e[1] + ch * q[2] + (q[3] * e[0] - q[1] * e[2]);
  const float z = q[0] * e[2] + ch * q[3] + (q[1] * e[1] - q[2] * e[0]);
  q[0] = w, q[1] = x, q[2] = y, q[3] = z;
}

// Rotation U V^T of the sign-fixed SVD F = U diag(s0, s1, s2) V^T, with U
// and V rotations, s0 >= s1 >= |s2| and s2 < 0 when det F < 0 (the sign
// convention of Irving et al. 2004). The steps follow McAdams et al. 2011
// ("Computing the singular value decomposition of 3x3 matrices with minimal
// branching and elementary floating point operations"): a fixed number of
// cyclic Jacobi sweeps on the symmetric F^T F with V kept as a unit
// quaternion; B = F V with its columns sorted by decreasing norm (a swap
// negates one column so V stays a rotation); then the QR decomposition of B
// by Givens rotations, whose orthogonal factor is U and whose triangular
// factor carries the singular values, the last with the sign of det F. Used
// where Newton's polar iteration does not apply (det F <= 0).
__device__ __forceinline__ void polar_svd_signfix(const float* F, float* R) {
  // symmetric S = F^T F
  float S[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) S[r][c] = F[r] * F[c] + F[3 + r] * F[3 + c] + F[6 + r] * F[6 + c];
  float q[4] = {1.0f, 0.0f, 0.0f, 0.0f};
  // Jacobi rotation J in the (p, q) plane (J_pp = J_qq = c, J_pq = s,
  // J_qp = -s): S <- J^T S J, V <- V J. J is the turn by -theta about the
  // third axis for the cyclic pairs (0, 1) and (1, 2), by +theta about y for
  // the pair (0, 2).
  for (int sweep = 0; sweep < 5; ++sweep) {
#pragma unroll
    for (int pair = 0; pair < 3; ++pair) {
      const int p = pair == 2 ? 1 : 0, qq = pair == 0 ? 1 : 2, r = 3 - p - qq;
      float c, s;
      jacobi_angle(S[p][p], S[qq][qq], S[p][qq], &c, &s);
      const float t = s / c;
      const float apq = S[p][qq];
      S[p][p] -= t * apq;
      S[qq][qq] += t * apq;
      S[p][qq] = S[qq][p] = 0.0f;
      const float arp = S[r][p], arq = S[r][qq];
      S[r][p] = S[p][r] = c * arp - s * arq;
      S[r][qq] = S[qq][r] = s * arp + c * arq;
      quat_turn(q, r, c, pair == 1 ? s : -s);
    }
  }
  // V from the quaternion (renormalised)
  const float qn = rsqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  const float w = q[0] * qn, x = q[1] * qn, y = q[2] * qn, z = q[3] * qn;
  float V[3][3] = {{1.0f - 2.0f * (y * y + z * z), 2.0f * (x * y - w * z), 2.0f * (x * z + w * y)},
                   {2.0f * (x * y + w * z), 1.0f - 2.0f * (x * x + z * z), 2.0f * (y * z - w * x)},
                   {2.0f * (x * z - w * y), 2.0f * (y * z + w * x), 1.0f - 2.0f * (x * x + y * y)}};
  // B = F V, columns sorted by decreasing norm
  float B[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) B[r][c] = F[3 * r] * V[0][c] + F[3 * r + 1] * V[1][c] + F[3 * r + 2] * V[2][c];
  float n2[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) n2[c] = B[0][c] * B[0][c] + B[1][c] * B[1][c] + B[2][c] * B[2][c];
  auto swap_cols = [&](int a, int b) {  // exchange columns a, b; negate the new b
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const float tb = B[r][a], tv = V[r][a];
      B[r][a] = B[r][b], V[r][a] = V[r][b];
      B[r][b] = -tb, V[r][b] = -tv;
    }
    const float tn = n2[a];
    n2[a] = n2[b], n2[b] = tn;
  };
  if (n2[1] > n2[0]) swap_cols(0, 1);
  if (n2[2] > n2[0]) swap_cols(0, 2);
  if (n2[2] > n2[1]) swap_cols(1, 2);
  // QR of B by Givens rotations on rows (0,1), (0,2), (1,2): B = U T with T
  // upper triangular, U = G1^T G2^T G3^T accumulated as a matrix.
  float U[3][3] = {{1.0f, 0.0f, 0.0f}, {0.0f, 1.0f, 0.0f}, {0.0f, 0.0f, 1.0f}};
#pragma unroll
  for (int step = 0; step < 3; ++step) {
    const int i = step == 2 ? 1 : 0, k = step == 0 ? 1 : 2;  // zero B[k][i] against B[i][i]
    const float a = B[i][i], b = B[k][i];
    const float rho2 = a * a + b * b;
    float c = 1.0f, s = 0.0f;
    if (rho2 > 1e-36f) {
      const float ir = rsqrtf(rho2);
      c = a * ir;
      s = b * ir;
    }
#pragma unroll
    for (int col = 0; col < 3; ++col) {  // rows i, k of B
      const float bi = B[i][col], bk = B[k][col];
      B[i][col] = c * bi + s * bk;
      B[k][col] = c * bk - s * bi;
    }
#pragma unroll
    for (int row = 0; row < 3; ++row) {  // columns i, k of U (U <- U G^T)
      const float ui = U[row][i], uk = U[row][k];
      U[row][i] = c * ui + s * uk;
      U[row][k] = c * uk - s * ui;
    }
  }
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) R[3 * r + c] = U[r][0] * V[c][0] + U[r][1] * V[c][1] + U[r][2] * V[c][2];
}

// Derivatives of the weights above with respect to f.
__device__ __forceinline__ void bspline_dw(float f, float dw[3]) {
  dw[0] = f - 1.5f;
  dw[1] = 2.0f * (1.0f - f);
  dw[2] = f - 0.5f;
}

// Fixed-corotated Kirchhoff stress tau = 2 mu (F - R) F^T + la (J - 1) J I
// (Stomakhin et al. 2012; the paper leaves the MLS-MPM constitutive law
// open, Algorithm 1), also returning the rotation factor R of F. Returns
// J = det F; *inverted is set when J <= 0.
__device__ __forceinline__ float kirchhoff_r(const float* F, float mu, float la, float* tau, float* R,
                                             bool* inverted) {
  const float J = det3(F);
  bool ok = (J > 0.0f) && polar_newton(F, R);
  if (!ok) polar_svd_signfix(F, R);
  *inverted = !(J > 0.0f);
  float D[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) D[i] = 2.0f * mu * (F[i] - R[i]);
  const float vol = la * (J - 1.0f) * J;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      tau[3 * r + c] = D[3 * r] * F[3 * c] + D[3 * r + 1] * F[3 * c + 1] + D[3 * r + 2] * F[3 * c + 2] +
                       (r == c ? vol : 0.0f);
  return J;
}

__device__ __forceinline__ float kirchhoff(const float* F, float mu, float la, float* tau,
                                           bool* inverted) {
  float R[9];
  return kirchhoff_r(F, mu, la, tau, R, inverted);
}

// Neo-Hookean Kirchhoff stress of standard MPM (Sec. III-A, eq.
// neo_hookean: sigma = (mu (F F^T - I) + lambda ln J I) / J, so tau = J sigma
// drops the 1/J), with J clamped to >= 1e-6 inside the logarithm so that an
// inverted or collapsed element still has a finite stress. Returns J.
__device__ __forceinline__ float neo_hookean_tau(const float* F, float mu, float la, float* tau) {
  const float J = det3(F);
  const float vol = la * logf(fmaxf(J, 1e-6f));
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      tau[3 * r + c] = mu * (F[3 * r] * F[3 * c] + F[3 * r + 1] * F[3 * c + 1] + F[3 * r + 2] * F[3 * c + 2] -
                             (r == c ? 1.0f : 0.0f)) +
                       (r == c ? vol : 0.0f);
  return J;
}

// Co-rotational constraint of PB-MPM (Sec. III-C) on one particle: with
// F* = (I + dt C) F and R its rotation factor, the target shape is
// T = beta R + (1 - beta) F* / det(F*)^(1/3) (a rotation blended with the
// volume-preserving part of F*), and the returned C' satisfies
// (I + dt C') F = T, i.e. C' = (T - F) F^-1 / dt. Returns det F.
__device__ __forceinline__ float pb_constraint(const float* F, const float* C, float dt, float beta, float* Cn) {
  float Fs[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      Fs[3 * r + c] = F[3 * r + c] + dt * (C[3 * r] * F[c] + C[3 * r + 1] * F[3 + c] + C[3 * r + 2] * F[6 + c]);
  const float Js = det3(Fs);
  float R[9];
  if (!((Js > 0.0f) && polar_newton(Fs, R))) polar_svd_signfix(Fs, R);
  const float sv = (1.0f - beta) / cbrtf(Js);
  float D[9];  // T - F
#pragma unroll
  for (int i = 0; i < 9; ++i) D[i] = beta * R[i] + sv * Fs[i] - F[i];
  float cof[9];
  cof[0] = F[4] * F[8] - F[5] * F[7];
  cof[1] = F[5] * F[6] - F[3] * F[8];
  cof[2] = F[3] * F[7] - F[4] * F[6];
  cof[3] = F[2] * F[7] - F[1] * F[8];
  cof[4] = F[0] * F[8] - F[2] * F[6];
  cof[5] = F[1] * F[6] - F[0] * F[7];
  cof[6] = F[1] * F[5] - F[2] * F[4];
  cof[7] = F[2] * F[3] - F[0] * F[5];
  cof[8] = F[0] * F[4] - F[1] * F[3];
  const float J = F[0] * cof[0] + F[1] * cof[1] + F[2] * cof[2];
  const float k = 1.0f / (J * dt);
  // F^-1 = cof(F)^T / J, so (D F^-1)[r][c] = sum_m D[r][m] cof[c][m] / J.
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      Cn[3 * r + c] = k * (D[3 * r] * cof[3 * c] + D[3 * r + 1] * cof[3 * c + 1] + D[3 * r + 2] * cof[3 * c + 2]);
  return J;
}

// Signed distance of a tool at world point p and its unit outward normal.
// Capsule: segment along body x, size {half_length, radius}. Box: half
// extents; inside, the normal of the nearest face (lowest axis on ties,
// sign(0) = +1). Plane: body +y through the centre.
__device__ __forceinline__ float tool_sdf(const ToolK& t, const float* p, float* n) {
  const float d0 = p[0] - t.c[0], d1 = p[1] - t.c[1], d2 = p[2] - t.c[2];
  float pl[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) pl[i] = t.R[i] * d0 + t.R[3 + i] * d1 + t.R[6 + i] * d2;
  float g[3] = {0.0f, 1.0f, 0.0f};
  float phi = 0.0f;
  if (t.type == TOOL_CAPSULE) {
    const float h = t.size[0], r = t.size[1];
    const float e0 = pl[0] - fminf(fmaxf(pl[0], -h), h);
    const float L = sqrtf(e0 * e0 + pl[1] * pl[1] + pl[2] * pl[2]);
    phi = L - r;
    if (L > 0.0f) {
      const float il = 1.0f / L;
      g[0] = e0 * il, g[1] = pl[1] * il, g[2] = pl[2] * il;
    }
  } else if (t.type == TOOL_BOX) {
    float q[3], o[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      q[i] = fabsf(pl[i]) - t.size[i];
      o[i] = fmaxf(q[i], 0.0f);
    }
    const float L = sqrtf(o[0] * o[0] + o[1] * o[1] + o[2] * o[2]);
    int k = 0;
    float qm = q[0];
    if (q[1] > qm) qm = q[1], k = 1;
    if (q[2] > qm) qm = q[2], k = 2;
    phi = L + fminf(qm, 0.0f);
    if (L > 0.0f) {
      const float il = 1.0f / L;
#pragma unroll
      for (int i = 0; i < 3; ++i) g[i] = copysignf(o[i], pl[i]) * il;
    } else {
      g[0] = g[1] = g[2] = 0.0f;
      g[k] = (pl[k] < 0.0f) ? -1.0f : 1.0f;
    }
  } else {  // plane
    phi = pl[1];
  }
  float nw[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) nw[i] = t.R[3 * i] * g[0] + t.R[3 * i + 1] * g[1] + t.R[3 * i + 2] * g[2];
  const float inv = rsqrtf(nw[0] * nw[0] + nw[1] * nw[1] + nw[2] * nw[2]);
  n[0] = nw[0] * inv, n[1] = nw[1] * inv, n[2] = nw[2] * inv;
  return phi;
}

// Tool `d` at its pose of global substep k: the centre follows the constant
// velocity from set_at, or the prefix sums of the velocity table and then the
// constant velocity (FP64, each operation rounded as written).
__device__ __forceinline__ ToolK tool_at(const ToolDesc& d, long long k, double dt) {
  ToolK t = d.k;
  const long long rel = k - d.set_at;
  if (d.rows == 0) {
    const double el = __dmul_rn((double)rel, dt);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      t.c[a] = (float)__dadd_rn(d.c0[a], __dmul_rn(el, d.lv[a]));
      t.lv[a] = (float)d.lv[a];
    }
  } else {
    const long long m = rel < d.rows ? rel : d.rows;
    const double tail = __dmul_rn((double)(rel - m), dt);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double c = __dadd_rn(__dadd_rn(d.c0[a], __dmul_rn(dt, d.vpre[3 * m + a])), __dmul_rn(tail, d.lv[a]));
      t.c[a] = (float)c;
      t.lv[a] = (float)(rel < d.rows ? d.vtab[3 * rel + a] : d.lv[a]);
    }
  }
  return t;
}

// Particle push-out (Sec. IV-A: particles left inside a rigid shape are
// pushed out, after the particle collision step of Stomakhin et al. 2013):
// a particle whose new position is inside a solid tool with push-out on,
// phi(x) < 0 with the tool at its pose of substep k (the substep that the
// new position starts), moves to the surface along the unit outward normal,
// x <- x - phi n. Tools in id order.
__device__ __forceinline__ void push_out(const SimK& s, const ToolDesc* td, long long k, float* x) {
  for (int q = 0; q < s.tool_slots; ++q) {
    if (!td[q].k.push) continue;
    const ToolK t = tool_at(td[q], k, (double)s.dt);
    float n[3];
    const float phi = tool_sdf(t, x, n);
    if (phi < 0.0f) {
#pragma unroll
      for (int a = 0; a < 3; ++a) x[a] -= phi * n[a];
    }
  }
}

// Friction and drag of eq. v_correction on a kept tangential vector t of
// length s, for an approaching node (u_n < 0): c_d max(1 + mu u_n / s, 0) t.
__device__ __forceinline__ float friction_scale(const ToolK& t, float un, float s) {
  return s > 0.0f ? t.drag * fmaxf(1.0f + t.mu * un / s, 0.0f) : 0.0f;
}

// Contact of one node with one tool. Regular geometries (Sec. IV-A, eq.
// v_correction): the relative velocity u = v - v_r is left alone when
// separating (u.n >= 0); otherwise its normal part is removed and its
// tangential part t is scaled by c_d max(1 + mu u.n / |t|, 0).
// Slicer (Sec. IV-B): a rectangle in the body x-y plane; within the fattened
// distance `margin` the normal is +-body z on the node's side (material is
// parted, not pushed), and beyond the spine edge (body y > half height) the
// contact is sticky. Segment and arc (Sec. IV-C): within the thickness only
// the part of u along the curve tangent is kept (then friction and drag),
// unless the node separates. Returns true if the node was in contact.
__device__ __forceinline__ bool tool_contact(const ToolK& t, const float* xI, float* v) {
  const float r0 = xI[0] - t.c[0], r1 = xI[1] - t.c[1], r2 = xI[2] - t.c[2];
  if (t.reach2 >= 0.0f && r0 * r0 + r1 * r1 + r2 * r2 > t.reach2) return false;  // far from the tool
  float n[3];
  float tl[3] = {0.0f, 0.0f, 0.0f};  // curve tangent (body frame), 1D geometries only
  bool sticky = false, curve = false;
  if (t.type == TOOL_CAPSULE || t.type == TOOL_BOX || t.type == TOOL_PLANE) {
    const float phi = tool_sdf(t, xI, n);
    if (!(phi < t.margin)) return false;
  } else {
    float pl[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) pl[i] = t.R[i] * r0 + t.R[3 + i] * r1 + t.R[6 + i] * r2;
    float nl[3];
    if (t.type == TOOL_SLICER) {
      const float qx = fmaxf(fabsf(pl[0]) - t.size[0], 0.0f);
      const float qy = fmaxf(fabsf(pl[1]) - t.size[1], 0.0f);
      const float d = sqrtf(qx * qx + qy * qy + pl[2] * pl[2]);
      if (!(d < t.margin)) return false;
      sticky = pl[1] > t.size[1];
      nl[0] = 0.0f, nl[1] = 0.0f, nl[2] = (pl[2] < 0.0f) ? -1.0f : 1.0f;
    } else {  // segment or arc
      float proj[3], thick;
      if (t.type == TOOL_SEGMENT) {
        thick = t.size[1];
        proj[0] = fminf(fmaxf(pl[0], -t.size[0]), t.size[0]), proj[1] = 0.0f, proj[2] = 0.0f;
        tl[0] = 1.0f;
      } else {
        const float ra = t.size[0], ha = t.size[1];
        thick = t.size[2];
        float ang = atan2f(pl[1], pl[0]);
        if (ang > ha || ang < -ha) {  // nearer end point
          float sh, ch;
          sincosf(ha, &sh, &ch);
          const float dp = (pl[0] - ra * ch) * (pl[0] - ra * ch) + (pl[1] - ra * sh) * (pl[1] - ra * sh);
          const float dm = (pl[0] - ra * ch) * (pl[0] - ra * ch) + (pl[1] + ra * sh) * (pl[1] + ra * sh);
          ang = (dm < dp) ? -ha : ha;
        }
        float sa, ca;
        sincosf(ang, &sa, &ca);
        proj[0] = ra * ca, proj[1] = ra * sa, proj[2] = 0.0f;
        tl[0] = -sa, tl[1] = ca;
      }
      const float e0 = pl[0] - proj[0], e1 = pl[1] - proj[1], e2 = pl[2] - proj[2];
      const float L = sqrtf(e0 * e0 + e1 * e1 + e2 * e2);
      if (!(L < thick)) return false;
      if (L > 0.0f) {
        nl[0] = e0 / L, nl[1] = e1 / L, nl[2] = e2 / L;
      } else {
        nl[0] = -tl[1], nl[1] = tl[0], nl[2] = 0.0f;
      }
      curve = true;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) n[i] = t.R[3 * i] * nl[0] + t.R[3 * i + 1] * nl[1] + t.R[3 * i + 2] * nl[2];
  }
  const float vr0 = t.lv[0] + t.av[1] * r2 - t.av[2] * r1;
  const float vr1 = t.lv[1] + t.av[2] * r0 - t.av[0] * r2;
  const float vr2 = t.lv[2] + t.av[0] * r1 - t.av[1] * r0;
  if (sticky) {
    v[0] = vr0, v[1] = vr1, v[2] = vr2;
    return true;
  }
  const float u0 = v[0] - vr0, u1 = v[1] - vr1, u2 = v[2] - vr2;
  const float un = n[0] * u0 + n[1] * u1 + n[2] * u2;
  if (!(un < 0.0f)) return true;  // separating or tangential: unchanged
  float t0, t1, t2, s;
  if (curve) {
    float tg[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) tg[i] = t.R[3 * i] * tl[0] + t.R[3 * i + 1] * tl[1] + t.R[3 * i + 2] * tl[2];
    const float ut = tg[0] * u0 + tg[1] * u1 + tg[2] * u2;
    t0 = ut * tg[0], t1 = ut * tg[1], t2 = ut * tg[2];
    s = fabsf(ut);
  } else {
    t0 = u0 - un * n[0], t1 = u1 - un * n[1], t2 = u2 - un * n[2];
    s = sqrtf(t0 * t0 + t1 * t1 + t2 * t2);
  }
  const float k = friction_scale(t, un, s);
  v[0] = vr0 + k * t0;
  v[1] = vr1 + k * t1;
  v[2] = vr2 + k * t2;
  return true;
}

// Node (i, j, k) -> index in the blocked grid layout.
__device__ __forceinline__ int grid_index(int i, int j, int k, int nb) {
  const int b = ((k >> kTileLog2) * nb + (j >> kTileLog2)) * nb + (i >> kTileLog2);
  const int l = (((k & (kTile - 1)) * kTile) + (j & (kTile - 1))) * kTile + (i & (kTile - 1));
  return (b << (3 * kTileLog2)) + l;
}

}  // namespace mpm
