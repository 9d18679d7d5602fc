// FP64 CPU oracle for one explicit MLS-MPM substep.
//
// TEST INFRASTRUCTURE ONLY. This file is the slow, plain reference that the
// GPU library is checked against. Only the test suite, the smoke check and the
// benchmark's CPU-baseline leg may load it. It shares no code, header, table
// or helper with the HIP library under paper_2502_18437_amd/csrc, and the
// library never calls it.
//
// What it computes (CRESSim-MPM, arXiv 2502.18437):
//   * Sec. III-A, the four stages of an MPM step: P2G, grid update, G2P,
//     grid reset; the quadratic B-spline basis with 3 nodes per axis; the grid
//     momentum update with external force (eq. mls_mpm_grid).
//   * Sec. III-B, MLS-MPM with APIC transfers: the fused P2G
//     momentum/force transfer (eq. mls_mpm_p2g_momentum_force), the affine
//     update (eq. mls_mpm_g2p_momentum) with D = dx^2/4 I, the F update
//     (eq. mls_mpm_g2p_f), the position update (eq.
//     mls_mpm_g2p_integration), in the order of Algorithm 1 (alg:mls_mpm).
//   * Sec. IV-A, grid-level SDF contact with friction and drag
//     (eq. v_correction).
//
// Readings taken where the paper is garbled or silent (all listed in the
// design notes of the repository):
//   * The fused P2G equation is printed without the particle momentum term;
//     the APIC/MLS form it cites is used: (mv)_I = sum N [m v + (m C -
//     dt V0 M^-1 tau)(x_I - x_p)], M^-1 = 4/dx^2.
//   * The affine matrix is C = B D^-1 = (4/dx^2) sum N v_I (x_I - x_p)^T
//     with grid velocities after the grid update and positions before G2P.
//   * Stress: fixed-corotated elasticity (Stomakhin et al. 2012),
//     Kirchhoff tau = 2 mu (F - R) F^T + lambda (J - 1) J I, and
//     V^t sigma = V0 tau.
//   * Polar decomposition: R = U V^T from an eigen-decomposition of F^T F by
//     cyclic Jacobi rotations (Golub & Van Loan, Matrix Computations,
//     Sec. 8.5), with the sign convention of Irving et al. 2004 (the
//     smallest singular value carries the sign of det F, so R is a rotation).
//   * Contact: outward SDF normal n, u = v_I - v_r, u_n = n.u; approaching
//     iff u_n < 0; then u' = c_d max(1 + mu u_n/|t|, 0) t with t the
//     tangential part (u' = 0 if |t| = 0); otherwise unchanged. Tools are
//     applied in id order at their pose at the start of the substep, then
//     sticky walls (band of B nodes per face). Empty nodes get v = 0.
//   * Cutting and suturing geometries (Sec. IV-B, IV-C): a slicer is a
//     rectangle in its body x-y plane whose side is the sign of body z; a node
//     within the fattened distance `margin` of it gets the contact law with
//     normal +-body z on its own side, except beyond the spine edge (body
//     y > half height), where the field is the distance to the spine and the
//     contact is sticky (relative velocity 0). A line segment (body x axis)
//     and an arc (body x-y plane, centred on the tool) have the unsigned
//     distance to the curve; a node within the thickness keeps only the
//     part of its relative velocity along the curve tangent, corrected by
//     friction and drag, unless it separates.
//   * Errors: a particle whose stencil leaves the grid (EDOMAIN) or whose
//     state is not finite (ENONFINITE) is left unchanged for that substep;
//     det F <= 0 is counted (EINVERTED). Status precedence:
//     ENONFINITE, then EDOMAIN, then EINVERTED.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

namespace {

enum {
  ST_OK = 0,
  ST_EINVAL = -1,
  ST_ENOMEM = -2,
  ST_EDOMAIN = -4,
  ST_ENONFINITE = -5,
  ST_EINVERTED = -6,
};

enum { TOOL_NONE = 0, TOOL_CAPSULE = 1, TOOL_BOX = 2, TOOL_PLANE = 3, TOOL_SLICER = 4, TOOL_SEGMENT = 5, TOOL_ARC = 6 };
constexpr int kMaxTools = 8;

// ---------------------------------------------------------------- 3x3 algebra
// Row-major 3x3 matrices as double[9].
void mat_mul(const double* A, const double* B, double* out) {
  double t[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += A[3 * r + k] * B[3 * k + c];
      t[3 * r + c] = s;
    }
  std::memcpy(out, t, sizeof(t));
}

void mat_transpose(const double* A, double* out) {
  double t[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) t[3 * r + c] = A[3 * c + r];
  std::memcpy(out, t, sizeof(t));
}

double mat_det(const double* A) {
  return A[0] * (A[4] * A[8] - A[5] * A[7]) -
         A[1] * (A[3] * A[8] - A[5] * A[6]) +
         A[2] * (A[3] * A[7] - A[4] * A[6]);
}

// Cyclic Jacobi eigen-decomposition of a symmetric 3x3 matrix S
// (Golub & Van Loan, Sec. 8.5): S = V diag(lam) V^T, V orthogonal.
void jacobi_eigen(const double* S, double* lam, double* V) {
  double A[9];
  std::memcpy(A, S, sizeof(A));
  for (int i = 0; i < 9; ++i) V[i] = (i % 4 == 0) ? 1.0 : 0.0;
  const int pairs[3][2] = {{0, 1}, {0, 2}, {1, 2}};
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = A[1] * A[1] + A[2] * A[2] + A[5] * A[5];
    double diag = A[0] * A[0] + A[4] * A[4] + A[8] * A[8];
    if (off == 0.0 || off <= 1e-36 * diag) break;
    for (const auto& pq : pairs) {
      const int p = pq[0], q = pq[1];
      const double apq = A[3 * p + q];
      if (apq == 0.0) continue;
      const double app = A[3 * p + p], aqq = A[3 * q + q];
      const double theta = (aqq - app) / (2.0 * apq);
      const double t = (theta >= 0.0 ? 1.0 : -1.0) /
                       (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
      const double c = 1.0 / std::sqrt(t * t + 1.0);
      const double s = t * c;
      // Rotation J equals I except J_pp = J_qq = c, J_pq = s, J_qp = -s.
      // A <- J^T A J, V <- V J.
      double J[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
      J[3 * p + p] = c;
      J[3 * q + q] = c;
      J[3 * p + q] = s;
      J[3 * q + p] = -s;
      double Jt[9];
      mat_transpose(J, Jt);
      mat_mul(A, J, A);
      mat_mul(Jt, A, A);
      A[3 * p + q] = 0.0;
      A[3 * q + p] = 0.0;
      mat_mul(V, J, V);
    }
  }
  lam[0] = A[0];
  lam[1] = A[4];
  lam[2] = A[8];
}

// Rotation part of F from its sign-fixed SVD F = U diag(s0, s1, +-s2) V^T,
// U and V rotations, s0 >= s1 >= s2 >= 0. R = U V^T. Returns det F.
double polar_rotation(const double* F, double* R) {
  double Ft[9], S[9], lam[3], V[9];
  mat_transpose(F, Ft);
  mat_mul(Ft, F, S);
  jacobi_eigen(S, lam, V);
  // Sort eigenpairs in descending order of eigenvalue.
  int order[3] = {0, 1, 2};
  for (int i = 0; i < 3; ++i)
    for (int j = i + 1; j < 3; ++j)
      if (lam[order[j]] > lam[order[i]]) {
        int tmp = order[i];
        order[i] = order[j];
        order[j] = tmp;
      }
  double v[3][3];  // v[i] = i-th right singular vector
  double sig[3];
  for (int i = 0; i < 3; ++i) {
    for (int k = 0; k < 3; ++k) v[i][k] = V[3 * k + order[i]];
    sig[i] = std::sqrt(lam[order[i]] > 0.0 ? lam[order[i]] : 0.0);
  }
  // Make V a rotation.
  double detV = v[0][0] * (v[1][1] * v[2][2] - v[1][2] * v[2][1]) -
                v[0][1] * (v[1][0] * v[2][2] - v[1][2] * v[2][0]) +
                v[0][2] * (v[1][0] * v[2][1] - v[1][1] * v[2][0]);
  if (detV < 0.0)
    for (int k = 0; k < 3; ++k) v[2][k] = -v[2][k];
  // Left singular vectors of the two largest singular values.
  double u[3][3];
  for (int i = 0; i < 2; ++i) {
    for (int r = 0; r < 3; ++r) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += F[3 * r + k] * v[i][k];
      u[i][r] = s;
    }
  }
  // Normalise u0, then orthonormalise u1 against it (Gram-Schmidt).
  double n0 = std::sqrt(u[0][0] * u[0][0] + u[0][1] * u[0][1] + u[0][2] * u[0][2]);
  if (n0 > 0.0) {
    for (int r = 0; r < 3; ++r) u[0][r] /= n0;
  } else {
    u[0][0] = 1.0, u[0][1] = 0.0, u[0][2] = 0.0;
  }
  double d01 = u[0][0] * u[1][0] + u[0][1] * u[1][1] + u[0][2] * u[1][2];
  for (int r = 0; r < 3; ++r) u[1][r] -= d01 * u[0][r];
  double n1 = std::sqrt(u[1][0] * u[1][0] + u[1][1] * u[1][1] + u[1][2] * u[1][2]);
  if (n1 > 1e-300 && sig[1] > 0.0) {
    for (int r = 0; r < 3; ++r) u[1][r] /= n1;
  } else {
    // Rank <= 1: any unit vector orthogonal to u0.
    double a[3] = {0.0, 0.0, 0.0};
    int m = (std::fabs(u[0][0]) < 0.9) ? 0 : 1;
    a[m] = 1.0;
    double d = a[0] * u[0][0] + a[1] * u[0][1] + a[2] * u[0][2];
    for (int r = 0; r < 3; ++r) a[r] -= d * u[0][r];
    double na = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    for (int r = 0; r < 3; ++r) u[1][r] = a[r] / na;
  }
  // u2 = u0 x u1 makes U a rotation; F v2 = (sign det F) s2 u2.
  u[2][0] = u[0][1] * u[1][2] - u[0][2] * u[1][1];
  u[2][1] = u[0][2] * u[1][0] - u[0][0] * u[1][2];
  u[2][2] = u[0][0] * u[1][1] - u[0][1] * u[1][0];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double s = 0.0;
      for (int i = 0; i < 3; ++i) s += u[i][r] * v[i][c];
      R[3 * r + c] = s;
    }
  return mat_det(F);
}

// Lame parameters from Young's modulus and Poisson ratio.
void lame(double E, double nu, double* mu, double* la) {
  *mu = E / (2.0 * (1.0 + nu));
  *la = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
}

// Kirchhoff stress of fixed-corotated elasticity:
// tau = 2 mu (F - R) F^T + lambda (J - 1) J I. Returns J.
double kirchhoff(const double* F, double E, double nu, double* tau) {
  double mu, la, R[9];
  lame(E, nu, &mu, &la);
  const double J = polar_rotation(F, R);
  double D[9], Ft[9];
  for (int i = 0; i < 9; ++i) D[i] = F[i] - R[i];
  mat_transpose(F, Ft);
  mat_mul(D, Ft, tau);
  for (int i = 0; i < 9; ++i) tau[i] *= 2.0 * mu;
  const double vol = la * (J - 1.0) * J;
  tau[0] += vol;
  tau[4] += vol;
  tau[8] += vol;
  return J;
}

// Strain energy density Psi = mu |F - R|_F^2 + lambda/2 (J - 1)^2.
double energy(const double* F, double E, double nu) {
  double mu, la, R[9];
  lame(E, nu, &mu, &la);
  const double J = polar_rotation(F, R);
  double s = 0.0;
  for (int i = 0; i < 9; ++i) s += (F[i] - R[i]) * (F[i] - R[i]);
  return mu * s + 0.5 * la * (J - 1.0) * (J - 1.0);
}

// Quadratic B-spline weights for the 3 nodes base, base+1, base+2 of one
// axis, with f = x/dx - base in [0.5, 1.5) (Sec. III-A).
void bspline_weights(double f, double* w) {
  w[0] = 0.5 * (1.5 - f) * (1.5 - f);
  w[1] = 0.75 - (f - 1.0) * (f - 1.0);
  w[2] = 0.5 * (f - 0.5) * (f - 0.5);
}

// -------------------------------------------------------------------- tools
struct Tool {
  int type = TOOL_NONE;
  double c0[3] = {0, 0, 0};   // centre when set
  double R[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};  // body-to-world rotation
  double size[3] = {0, 0, 0};
  double lv[3] = {0, 0, 0};   // linear velocity
  double av[3] = {0, 0, 0};   // angular velocity (enters v_r only)
  double mu = 0.0, drag = 1.0, margin = 0.0;
  long long set_at = 0;       // substep counter when the tool was set
};

void quat_to_matrix(const double* q, double* R) {
  double w = q[0], x = q[1], y = q[2], z = q[3];
  const double nrm = std::sqrt(w * w + x * x + y * y + z * z);
  w /= nrm, x /= nrm, y /= nrm, z /= nrm;
  R[0] = 1 - 2 * (y * y + z * z);
  R[1] = 2 * (x * y - w * z);
  R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);
  R[4] = 1 - 2 * (x * x + z * z);
  R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);
  R[7] = 2 * (y * z + w * x);
  R[8] = 1 - 2 * (x * x + y * y);
}

// Signed distance and (unnormalised) gradient of a tool at world point p,
// with the tool centred at c. Capsule: segment along the body x axis,
// size = {half_length, radius}. Box: size = half extents. Plane: body +y is
// the outward normal through c.
double tool_sdf(int type, const double* c, const double* R, const double* size,
                const double* p, double* grad) {
  double d[3] = {p[0] - c[0], p[1] - c[1], p[2] - c[2]};
  double pl[3];  // body coordinates: R^T (p - c)
  for (int i = 0; i < 3; ++i) pl[i] = R[0 * 3 + i] * d[0] + R[1 * 3 + i] * d[1] + R[2 * 3 + i] * d[2];
  double gl[3] = {0.0, 1.0, 0.0};
  double phi = 0.0;
  if (type == TOOL_CAPSULE) {
    const double h = size[0], r = size[1];
    double t = pl[0];
    if (t < -h) t = -h;
    if (t > h) t = h;
    double e[3] = {pl[0] - t, pl[1], pl[2]};
    double L = std::sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    phi = L - r;
    if (L > 0.0) {
      gl[0] = e[0] / L, gl[1] = e[1] / L, gl[2] = e[2] / L;
    }  // on the axis: body +y
  } else if (type == TOOL_BOX) {
    double q[3], o[3];
    for (int i = 0; i < 3; ++i) {
      q[i] = std::fabs(pl[i]) - size[i];
      o[i] = q[i] > 0.0 ? q[i] : 0.0;
    }
    double L = std::sqrt(o[0] * o[0] + o[1] * o[1] + o[2] * o[2]);
    double qmax = q[0];
    int k = 0;
    for (int i = 1; i < 3; ++i)
      if (q[i] > qmax) qmax = q[i], k = i;  // ties keep the lowest axis
    phi = L + (qmax < 0.0 ? qmax : 0.0);
    if (L > 0.0) {
      for (int i = 0; i < 3; ++i) gl[i] = (pl[i] < 0.0 ? -o[i] : o[i]) / L;
    } else {
      gl[0] = gl[1] = gl[2] = 0.0;
      gl[k] = (pl[k] < 0.0) ? -1.0 : 1.0;  // sign(0) = +1
    }
  } else if (type == TOOL_PLANE) {
    phi = pl[1];
  }
  for (int i = 0; i < 3; ++i) grad[i] = R[3 * i + 0] * gl[0] + R[3 * i + 1] * gl[1] + R[3 * i + 2] * gl[2];
  return phi;
}

// Contact law of Sec. IV-A (eq. v_correction) on the relative velocity u
// with unit outward normal n. Writes the corrected relative velocity.
void contact_correct(const double* n, const double* u, double mu, double drag, double* out) {
  const double un = n[0] * u[0] + n[1] * u[1] + n[2] * u[2];
  if (!(un < 0.0)) {  // separating or tangential: unchanged
    out[0] = u[0], out[1] = u[1], out[2] = u[2];
    return;
  }
  double t[3] = {u[0] - un * n[0], u[1] - un * n[1], u[2] - un * n[2]};
  const double s = std::sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
  if (!(s > 0.0)) {
    out[0] = out[1] = out[2] = 0.0;
    return;
  }
  double k = 1.0 + mu * un / s;
  if (k < 0.0) k = 0.0;
  k *= drag;
  out[0] = k * t[0], out[1] = k * t[1], out[2] = k * t[2];
}

// Contact law of the 1D geometries (Sec. IV-C): the tangential part of eq.
// v_correction is replaced by the part along the curve tangent tg; the
// cross-section and normal parts are dropped unless the node separates.
void contact_tangent(const double* n, const double* tg, const double* u, double mu, double drag,
                     double* out) {
  const double un = n[0] * u[0] + n[1] * u[1] + n[2] * u[2];
  if (!(un < 0.0)) {
    out[0] = u[0], out[1] = u[1], out[2] = u[2];
    return;
  }
  const double ut = tg[0] * u[0] + tg[1] * u[1] + tg[2] * u[2];
  const double s = std::fabs(ut);
  if (!(s > 0.0)) {
    out[0] = out[1] = out[2] = 0.0;
    return;
  }
  double k = 1.0 + mu * un / s;
  if (k < 0.0) k = 0.0;
  k *= drag * ut;
  out[0] = k * tg[0], out[1] = k * tg[1], out[2] = k * tg[2];
}

void rotate(const double* R, const double* a, double* out) {
  for (int i = 0; i < 3; ++i) out[i] = R[3 * i] * a[0] + R[3 * i + 1] * a[1] + R[3 * i + 2] * a[2];
}

// Contact of one node (position xI, velocity vI) with one tool centred at c.
// Returns true when the tool changed the velocity field (node in contact).
bool tool_node_contact(int type, const double* c, const double* R, const double* size, const double* lv,
                       const double* av, double mu, double drag, double margin, const double* xI,
                       double* vI) {
  const double r[3] = {xI[0] - c[0], xI[1] - c[1], xI[2] - c[2]};
  double pl[3];
  for (int i = 0; i < 3; ++i) pl[i] = R[0 * 3 + i] * r[0] + R[1 * 3 + i] * r[1] + R[2 * 3 + i] * r[2];
  const double vr[3] = {lv[0] + av[1] * r[2] - av[2] * r[1], lv[1] + av[2] * r[0] - av[0] * r[2],
                        lv[2] + av[0] * r[1] - av[1] * r[0]};
  const double u[3] = {vI[0] - vr[0], vI[1] - vr[1], vI[2] - vr[2]};
  double un[3];
  if (type == TOOL_CAPSULE || type == TOOL_BOX || type == TOOL_PLANE) {
    double grad[3];
    const double phi = tool_sdf(type, c, R, size, xI, grad);
    if (!(phi < margin)) return false;
    const double gn = std::sqrt(grad[0] * grad[0] + grad[1] * grad[1] + grad[2] * grad[2]);
    const double nrm[3] = {grad[0] / gn, grad[1] / gn, grad[2] / gn};
    contact_correct(nrm, u, mu, drag, un);
  } else if (type == TOOL_SLICER) {
    const double hx = size[0], hy = size[1];
    const double qx = std::fabs(pl[0]) - hx > 0.0 ? std::fabs(pl[0]) - hx : 0.0;
    const double qy = std::fabs(pl[1]) - hy > 0.0 ? std::fabs(pl[1]) - hy : 0.0;
    const double d = std::sqrt(qx * qx + qy * qy + pl[2] * pl[2]);
    if (!(d < margin)) return false;
    if (pl[1] > hy) {
      un[0] = un[1] = un[2] = 0.0;  // spine side: sticky
    } else {
      const double nl[3] = {0.0, 0.0, pl[2] < 0.0 ? -1.0 : 1.0};
      double nrm[3];
      rotate(R, nl, nrm);
      contact_correct(nrm, u, mu, drag, un);
    }
  } else if (type == TOOL_SEGMENT || type == TOOL_ARC) {
    double proj[3], tl[3];
    double thick;
    if (type == TOOL_SEGMENT) {
      const double h = size[0];
      thick = size[1];
      double t = pl[0];
      if (t < -h) t = -h;
      if (t > h) t = h;
      proj[0] = t, proj[1] = 0.0, proj[2] = 0.0;
      tl[0] = 1.0, tl[1] = 0.0, tl[2] = 0.0;
    } else {
      const double ra = size[0], ha = size[1];
      thick = size[2];
      double ang = std::atan2(pl[1], pl[0]);
      if (ang > ha || ang < -ha) {  // nearest end point
        const double e0[2] = {ra * std::cos(ha), ra * std::sin(ha)};
        const double e1[2] = {ra * std::cos(-ha), ra * std::sin(-ha)};
        const double d0 = (pl[0] - e0[0]) * (pl[0] - e0[0]) + (pl[1] - e0[1]) * (pl[1] - e0[1]);
        const double d1 = (pl[0] - e1[0]) * (pl[0] - e1[0]) + (pl[1] - e1[1]) * (pl[1] - e1[1]);
        ang = (d1 < d0) ? -ha : ha;
      }
      proj[0] = ra * std::cos(ang), proj[1] = ra * std::sin(ang), proj[2] = 0.0;
      tl[0] = -std::sin(ang), tl[1] = std::cos(ang), tl[2] = 0.0;
    }
    double e[3] = {pl[0] - proj[0], pl[1] - proj[1], pl[2] - proj[2]};
    const double L = std::sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    if (!(L < thick)) return false;
    double nl[3];
    if (L > 0.0) {
      nl[0] = e[0] / L, nl[1] = e[1] / L, nl[2] = e[2] / L;
    } else {  // on the curve: the body direction orthogonal to the tangent in the x-y plane
      nl[0] = -tl[1], nl[1] = tl[0], nl[2] = 0.0;
    }
    double nrm[3], tg[3];
    rotate(R, nl, nrm);
    rotate(R, tl, tg);
    contact_tangent(nrm, tg, u, mu, drag, un);
  } else {
    return false;
  }
  for (int a = 0; a < 3; ++a) vI[a] = vr[a] + un[a];
  return true;
}

// -------------------------------------------------------------------- scene
struct Scene {
  int n = 0;
  double dx = 0, inv_dx = 0, dt = 0, g[3] = {0, 0, 0};
  int band = 0;
  double nu = 0, E_default = 0;
  long long N = 0;
  double mass = 0, vol0 = 0;
  std::vector<double> x, v, C, F, E;  // per particle: 3, 3, 9, 9, 1 values
  Tool tools[kMaxTools];
  long long substep = 0;
  std::vector<double> gm, gp, gv;     // grid of the last substep: n^3, 3n^3, 3n^3
  double impulse[kMaxTools + 1][3];   // per tool, then walls; last oracle_step
  long long n_inverted = 0, n_domain = 0, n_nonfinite = 0;
};

inline size_t node_index(const Scene& s, int i, int j, int k) {
  return (static_cast<size_t>(i) * s.n + j) * s.n + k;
}

bool all_finite(const double* a, int m) {
  for (int i = 0; i < m; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

// Per-particle stencil: base node and fractional offsets; false if the
// 3x3x3 stencil leaves the grid.
bool stencil(const Scene& s, const double* xp, int* base, double* f) {
  for (int a = 0; a < 3; ++a) {
    const double r = xp[a] * s.inv_dx;
    const double b = std::floor(r - 0.5);
    if (!(b >= 0.0) || !(b + 2.0 <= s.n - 1)) return false;
    base[a] = static_cast<int>(b);
    f[a] = r - b;
  }
  return true;
}

void substep(Scene& s) {
  const double dx = s.dx, dt = s.dt;
  const double Minv = 4.0 / (dx * dx);
  const size_t nn = static_cast<size_t>(s.n) * s.n * s.n;
  // Stage 4 of the previous step, done first (Algorithm 1, reset grid).
  std::fill(s.gm.begin(), s.gm.end(), 0.0);
  std::fill(s.gp.begin(), s.gp.end(), 0.0);
  std::fill(s.gv.begin(), s.gv.end(), 0.0);
  std::vector<char> skip(static_cast<size_t>(s.N), 0);

  // ---- P2G: mass and fused momentum/force transfer (Algorithm 1, first loop)
  for (long long p = 0; p < s.N; ++p) {
    const double* xp = &s.x[3 * p];
    const double* vp = &s.v[3 * p];
    const double* Cp = &s.C[9 * p];
    const double* Fp = &s.F[9 * p];
    const double Ep = s.E.empty() ? s.E_default : s.E[p];
    if (!all_finite(xp, 3) || !all_finite(vp, 3) || !all_finite(Cp, 9) ||
        !all_finite(Fp, 9) || !std::isfinite(Ep)) {
      s.n_nonfinite++;
      skip[p] = 1;
      continue;
    }
    int base[3];
    double f[3];
    if (!stencil(s, xp, base, f)) {
      s.n_domain++;
      skip[p] = 1;
      continue;
    }
    double w[3][3];
    for (int a = 0; a < 3; ++a) bspline_weights(f[a], w[a]);
    double tau[9];
    const double J = kirchhoff(Fp, Ep, s.nu, tau);
    if (!(J > 0.0)) s.n_inverted++;
    // Affine momentum minus the MLS stress term.
    double A[9];
    for (int i = 0; i < 9; ++i) A[i] = s.mass * Cp[i] - dt * s.vol0 * Minv * tau[i];
    for (int ox = 0; ox < 3; ++ox)
      for (int oy = 0; oy < 3; ++oy)
        for (int oz = 0; oz < 3; ++oz) {
          const double N = w[0][ox] * w[1][oy] * w[2][oz];
          const double d[3] = {(ox - f[0]) * dx, (oy - f[1]) * dx, (oz - f[2]) * dx};
          const size_t I = node_index(s, base[0] + ox, base[1] + oy, base[2] + oz);
          s.gm[I] += N * s.mass;
          for (int a = 0; a < 3; ++a) {
            const double Ad = A[3 * a + 0] * d[0] + A[3 * a + 1] * d[1] + A[3 * a + 2] * d[2];
            s.gp[3 * I + a] += N * (s.mass * vp[a] + Ad);
          }
        }
  }

  // ---- Grid update: velocity, gravity, contact, walls (Algorithm 1, second loop)
  double poses[kMaxTools][3];
  for (int k = 0; k < kMaxTools; ++k) {
    const Tool& t = s.tools[k];
    const double el = static_cast<double>(s.substep - t.set_at) * dt;
    for (int a = 0; a < 3; ++a) poses[k][a] = t.c0[a] + el * t.lv[a];
  }
  for (int i = 0; i < s.n; ++i)
    for (int j = 0; j < s.n; ++j)
      for (int k = 0; k < s.n; ++k) {
        const size_t I = node_index(s, i, j, k);
        const double m = s.gm[I];
        double vI[3] = {0.0, 0.0, 0.0};
        if (!(m > 0.0)) continue;  // empty node: v = 0
        for (int a = 0; a < 3; ++a) vI[a] = s.gp[3 * I + a] / m + dt * s.g[a];
        const double xI[3] = {i * dx, j * dx, k * dx};
        for (int q = 0; q < kMaxTools; ++q) {
          const Tool& t = s.tools[q];
          if (t.type == TOOL_NONE) continue;
          double vnew[3] = {vI[0], vI[1], vI[2]};
          if (!tool_node_contact(t.type, poses[q], t.R, t.size, t.lv, t.av, t.mu, t.drag, t.margin, xI,
                                 vnew))
            continue;
          for (int a = 0; a < 3; ++a) {
            s.impulse[q][a] += m * (vnew[a] - vI[a]);
            vI[a] = vnew[a];
          }
        }
        const int lo = s.band, hi = s.n - 1 - s.band;
        if (i < lo || i > hi || j < lo || j > hi || k < lo || k > hi) {
          for (int a = 0; a < 3; ++a) {
            s.impulse[kMaxTools][a] += m * (0.0 - vI[a]);
            vI[a] = 0.0;
          }
        }
        for (int a = 0; a < 3; ++a) s.gv[3 * I + a] = vI[a];
      }

  // ---- G2P: velocity, affine matrix, F, position (Algorithm 1, third loop)
  for (long long p = 0; p < s.N; ++p) {
    if (skip[p]) continue;
    double* xp = &s.x[3 * p];
    int base[3];
    double f[3];
    stencil(s, xp, base, f);
    double w[3][3];
    for (int a = 0; a < 3; ++a) bspline_weights(f[a], w[a]);
    double vn[3] = {0.0, 0.0, 0.0};
    double B[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int ox = 0; ox < 3; ++ox)
      for (int oy = 0; oy < 3; ++oy)
        for (int oz = 0; oz < 3; ++oz) {
          const double N = w[0][ox] * w[1][oy] * w[2][oz];
          const double d[3] = {(ox - f[0]) * dx, (oy - f[1]) * dx, (oz - f[2]) * dx};
          const size_t I = node_index(s, base[0] + ox, base[1] + oy, base[2] + oz);
          for (int a = 0; a < 3; ++a) {
            const double va = s.gv[3 * I + a];
            vn[a] += N * va;
            for (int b = 0; b < 3; ++b) B[3 * a + b] += N * va * d[b];
          }
        }
    double* Cp = &s.C[9 * p];
    double* Fp = &s.F[9 * p];
    for (int i = 0; i < 9; ++i) Cp[i] = Minv * B[i];
    double G[9];
    for (int i = 0; i < 9; ++i) G[i] = dt * Cp[i] + ((i % 4 == 0) ? 1.0 : 0.0);
    mat_mul(G, Fp, Fp);
    for (int a = 0; a < 3; ++a) {
      s.v[3 * p + a] = vn[a];
      xp[a] += dt * vn[a];
    }
  }
  s.substep++;
  (void)nn;
}

int status_of(const Scene& s) {
  if (s.n_nonfinite) return ST_ENONFINITE;
  if (s.n_domain) return ST_EDOMAIN;
  if (s.n_inverted) return ST_EINVERTED;
  return ST_OK;
}

}  // namespace

extern "C" {

void* oracle_create(int n_grid, double dt, const double* gravity, int wall_band,
                    double nu, double E_default) {
  if (n_grid < 3 || !(dt > 0.0) || wall_band < 0 || !gravity) return nullptr;
  Scene* s = new (std::nothrow) Scene();
  if (!s) return nullptr;
  s->n = n_grid;
  s->dx = 1.0 / n_grid;
  s->inv_dx = static_cast<double>(n_grid);
  s->dt = dt;
  for (int a = 0; a < 3; ++a) s->g[a] = gravity[a];
  s->band = wall_band;
  s->nu = nu;
  s->E_default = E_default;
  const size_t nn = static_cast<size_t>(n_grid) * n_grid * n_grid;
  try {
    s->gm.assign(nn, 0.0);
    s->gp.assign(3 * nn, 0.0);
    s->gv.assign(3 * nn, 0.0);
  } catch (...) {
    delete s;
    return nullptr;
  }
  std::memset(s->impulse, 0, sizeof(s->impulse));
  return s;
}

void oracle_destroy(void* h) { delete static_cast<Scene*>(h); }

// Particle arrays are FP32 as handed to the GPU library; they are widened to
// FP64 here. v, C, F, E may be NULL (zero, zero, identity, E_default).
int oracle_set_particles(void* h, long long n, const float* x, const float* v,
                         const float* C, const float* F, const float* E,
                         double mass, double vol0) {
  Scene* s = static_cast<Scene*>(h);
  if (!s || n < 0 || (n > 0 && !x)) return ST_EINVAL;
  s->N = n;
  s->mass = mass;
  s->vol0 = vol0;
  s->x.assign(3 * n, 0.0);
  s->v.assign(3 * n, 0.0);
  s->C.assign(9 * n, 0.0);
  s->F.assign(9 * n, 0.0);
  s->E.clear();
  if (E) s->E.assign(n, 0.0);
  for (long long p = 0; p < n; ++p) {
    for (int a = 0; a < 3; ++a) {
      s->x[3 * p + a] = x[3 * p + a];
      s->v[3 * p + a] = v ? v[3 * p + a] : 0.0;
    }
    for (int i = 0; i < 9; ++i) {
      s->C[9 * p + i] = C ? C[9 * p + i] : 0.0;
      s->F[9 * p + i] = F ? F[9 * p + i] : ((i % 4 == 0) ? 1.0 : 0.0);
    }
    if (E) s->E[p] = E[p];
  }
  s->n_inverted = s->n_domain = s->n_nonfinite = 0;
  return ST_OK;
}

int oracle_set_tool(void* h, int id, int type, const double* center, const double* quat,
                    const double* size, const double* lin_vel, const double* ang_vel,
                    double mu, double drag, double margin) {
  Scene* s = static_cast<Scene*>(h);
  if (!s || id < 0 || id >= kMaxTools || type < TOOL_NONE || type > TOOL_ARC) return ST_EINVAL;
  Tool& t = s->tools[id];
  t = Tool();
  t.type = type;
  if (type == TOOL_NONE) return ST_OK;
  for (int a = 0; a < 3; ++a) {
    t.c0[a] = center[a];
    t.size[a] = size[a];
    t.lv[a] = lin_vel ? lin_vel[a] : 0.0;
    t.av[a] = ang_vel ? ang_vel[a] : 0.0;
  }
  quat_to_matrix(quat, t.R);
  t.mu = mu;
  t.drag = drag;
  t.margin = margin;
  t.set_at = s->substep;
  return ST_OK;
}

// Advance n substeps. Returns the sticky status (see status precedence).
int oracle_step(void* h, int n) {
  Scene* s = static_cast<Scene*>(h);
  if (!s || n < 0) return ST_EINVAL;
  std::memset(s->impulse, 0, sizeof(s->impulse));
  for (int k = 0; k < n; ++k) substep(*s);
  return status_of(*s);
}

// FP64 state in the caller's particle order. NULL outputs are skipped.
int oracle_read(void* h, double* x, double* v, double* C, double* F) {
  Scene* s = static_cast<Scene*>(h);
  if (!s) return ST_EINVAL;
  if (x) std::memcpy(x, s->x.data(), sizeof(double) * 3 * s->N);
  if (v) std::memcpy(v, s->v.data(), sizeof(double) * 3 * s->N);
  if (C) std::memcpy(C, s->C.data(), sizeof(double) * 9 * s->N);
  if (F) std::memcpy(F, s->F.data(), sizeof(double) * 9 * s->N);
  return status_of(*s);
}

// Dense grid of the most recent substep, indexed [(i*n + j)*n + k] for node
// (i, j, k) at (i, j, k) dx: mass and momentum after P2G, velocity after the
// grid update. NULL outputs are skipped.
int oracle_last_grid(void* h, double* mass, double* mom, double* vel) {
  Scene* s = static_cast<Scene*>(h);
  if (!s) return ST_EINVAL;
  const size_t nn = static_cast<size_t>(s->n) * s->n * s->n;
  if (mass) std::memcpy(mass, s->gm.data(), sizeof(double) * nn);
  if (mom) std::memcpy(mom, s->gp.data(), sizeof(double) * 3 * nn);
  if (vel) std::memcpy(vel, s->gv.data(), sizeof(double) * 3 * nn);
  return ST_OK;
}

// Momentum change applied to the grid by each tool (rows 0..7) and by the
// walls (row 8), summed over the substeps of the last oracle_step call.
int oracle_impulses(void* h, double* out) {
  Scene* s = static_cast<Scene*>(h);
  if (!s || !out) return ST_EINVAL;
  std::memcpy(out, s->impulse, sizeof(s->impulse));
  return ST_OK;
}

// Error counters: inverted, out-of-domain, non-finite particle-substeps.
int oracle_counters(void* h, long long* out) {
  Scene* s = static_cast<Scene*>(h);
  if (!s || !out) return ST_EINVAL;
  out[0] = s->n_inverted;
  out[1] = s->n_domain;
  out[2] = s->n_nonfinite;
  return ST_OK;
}

// ---- unit entry points used by the invariant tests
void oracle_weights(double f, double* w) { bspline_weights(f, w); }
double oracle_polar(const double* F, double* R) { return polar_rotation(F, R); }
double oracle_kirchhoff(const double* F, double E, double nu, double* tau) {
  return kirchhoff(F, E, nu, tau);
}
double oracle_energy(const double* F, double E, double nu) { return energy(F, E, nu); }
double oracle_sdf(int type, const double* center, const double* quat, const double* size,
                  const double* p, double* grad) {
  double R[9];
  quat_to_matrix(quat, R);
  return tool_sdf(type, center, R, size, p, grad);
}
void oracle_contact(const double* n, const double* u, double mu, double drag, double* out) {
  contact_correct(n, u, mu, drag, out);
}
// Velocity of a node at xI after contact with one tool (all geometries);
// returns 1 if the node was in contact.
int oracle_node_contact(int type, const double* center, const double* quat, const double* size,
                        const double* lin_vel, const double* ang_vel, double mu, double drag, double margin,
                        const double* xI, double* vI) {
  double R[9];
  quat_to_matrix(quat, R);
  return tool_node_contact(type, center, R, size, lin_vel, ang_vel, mu, drag, margin, xI, vI) ? 1 : 0;
}

}  // extern "C"
