// Per-structure superposition math shared by the HIP kernels: the 4x4
// quaternion eigenproblem whose top eigenpair gives the optimal rotation of a
// reference onto the current structure (Section 3 of arXiv:1801.02362: the
// rotation comes from diagonalising a quaternion matrix), the exact distance
// of Eq. 3 written as Gx + Ga - 2*lambda_max, and the derivative of the
// rotation with respect to the correlation matrix that Eq. 6 needs for the
// close-structure rotation.
//
// Everything here is FP64.  Functions are __host__ __device__ so that the same
// code is exercised by a host-side unit test library.
//
// Conventions: M is the 3x3 correlation matrix M[a][b] = sum_j w_j a_j[a] x_j[b]
// (row index from the reference a, column index from x), stored row-major.
// The quaternion matrix F(M) is stored packed as the 10 upper-triangle entries
// F00 F01 F02 F03 F11 F12 F13 F22 F23 F33.  R(q) maps a onto x.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#define PCV_HD __host__ __device__ __forceinline__
// Rarely taken paths are kept out of line so their registers do not count
// against the streaming loops that call them.
#define PCV_COLD __host__ __device__ inline __attribute__((noinline))

namespace pcv {

// ---------------------------------------------------------------- basics
PCV_HD double det3(double a, double b, double c, double d, double e, double f,
                   double g, double h, double i) {
  return a * (e * i - f * h) - b * (d * i - f * g) + c * (d * h - e * g);
}

// Packed upper triangle of the 4x4 quaternion matrix.
PCV_HD void horn_matrix(const double M[9], double F[10]) {
  const double xx = M[0], xy = M[1], xz = M[2];
  const double yx = M[3], yy = M[4], yz = M[5];
  const double zx = M[6], zy = M[7], zz = M[8];
  F[0] = xx + yy + zz;   // F00
  F[1] = yz - zy;        // F01
  F[2] = zx - xz;        // F02
  F[3] = xy - yx;        // F03
  F[4] = xx - yy - zz;   // F11
  F[5] = xy + yx;        // F12
  F[6] = zx + xz;        // F13
  F[7] = -xx + yy - zz;  // F22
  F[8] = yz + zy;        // F23
  F[9] = -xx - yy + zz;  // F33
}

PCV_HD void unpack4(const double F[10], double A[4][4]) {
  A[0][0] = F[0]; A[0][1] = F[1]; A[0][2] = F[2]; A[0][3] = F[3];
  A[1][1] = F[4]; A[1][2] = F[5]; A[1][3] = F[6];
  A[2][2] = F[7]; A[2][3] = F[8]; A[3][3] = F[9];
  A[1][0] = F[1]; A[2][0] = F[2]; A[3][0] = F[3];
  A[2][1] = F[5]; A[3][1] = F[6]; A[3][2] = F[8];
}

// det of a 4x4 matrix by the 2x2-minor (Laplace) expansion over rows {0,1}.
PCV_HD double det4(const double A[4][4]) {
  const double s0 = A[0][0] * A[1][1] - A[0][1] * A[1][0];
  const double s1 = A[0][0] * A[1][2] - A[0][2] * A[1][0];
  const double s2 = A[0][0] * A[1][3] - A[0][3] * A[1][0];
  const double s3 = A[0][1] * A[1][2] - A[0][2] * A[1][1];
  const double s4 = A[0][1] * A[1][3] - A[0][3] * A[1][1];
  const double s5 = A[0][2] * A[1][3] - A[0][3] * A[1][2];
  const double c5 = A[2][2] * A[3][3] - A[2][3] * A[3][2];
  const double c4 = A[2][1] * A[3][3] - A[2][3] * A[3][1];
  const double c3 = A[2][1] * A[3][2] - A[2][2] * A[3][1];
  const double c2 = A[2][0] * A[3][3] - A[2][3] * A[3][0];
  const double c1 = A[2][0] * A[3][2] - A[2][2] * A[3][0];
  const double c0 = A[2][0] * A[3][1] - A[2][1] * A[3][0];
  return s0 * c5 - s1 * c4 + s2 * c3 + s3 * c2 - s4 * c1 + s5 * c0;
}

// Characteristic polynomial det(F - l I) = l^4 + c2 l^2 + c1 l + c0 of the
// (trace-free) quaternion matrix: c2 = -2 |M|_F^2, c1 = -8 det M, c0 = det F.
PCV_HD void char_poly(const double M[9], const double F[10], double& c2, double& c1, double& c0) {
  double ss = 0.0;
  for (int k = 0; k < 9; ++k) ss = fma(M[k], M[k], ss);
  c2 = -2.0 * ss;
  c1 = -8.0 * det3(M[0], M[1], M[2], M[3], M[4], M[5], M[6], M[7], M[8]);
  double A[4][4];
  unpack4(F, A);
  c0 = det4(A);
}

// Largest root by Newton from an upper bound.  Right of the largest root the
// polynomial is increasing and convex, so Newton decreases monotonically; it
// stops when the step no longer decreases the iterate.  Returns the root and
// the derivative there (the product of the gaps to the other eigenvalues).
PCV_HD double newton_top_root(double c2, double c1, double c0, double lam, double& dp_out) {
  double dp = 0.0;
  for (int it = 0; it < 100; ++it) {
    const double l2 = lam * lam;
    const double p = ((l2 + c2) * lam + c1) * lam + c0;
    dp = (4.0 * l2 + 2.0 * c2) * lam + c1;
    if (!(dp > 0.0)) break;
    const double step = p / dp;
    if (!(step > 0.0)) break;
    const double nl = lam - step;
    if (!(nl < lam)) break;
    lam = nl;
  }
  const double l2 = lam * lam;
  dp_out = (4.0 * l2 + 2.0 * c2) * lam + c1;
  return lam;
}

// Cofactor (r, c) of a 4x4 matrix, compile-time indices.
template <int r, int c>
PCV_HD double cofactor4(const double A[4][4]) {
  constexpr int r0 = (r == 0) ? 1 : 0, r1 = (r <= 1) ? 2 : 1, r2 = (r <= 2) ? 3 : 2;
  constexpr int c0 = (c == 0) ? 1 : 0, c1 = (c <= 1) ? 2 : 1, c2 = (c <= 2) ? 3 : 2;
  const double d = det3(A[r0][c0], A[r0][c1], A[r0][c2], A[r1][c0], A[r1][c1], A[r1][c2],
                        A[r2][c0], A[r2][c1], A[r2][c2]);
  return ((r + c) & 1) ? -d : d;
}

template <int j>
PCV_HD void adj_column(const double B[4][4], double v[4]) {
  v[0] = cofactor4<j, 0>(B);
  v[1] = cofactor4<j, 1>(B);
  v[2] = cofactor4<j, 2>(B);
  v[3] = cofactor4<j, 3>(B);
}

// Eigenvector of the simple eigenvalue lam: a column of adj(F - lam I), which
// is proportional to q q^T.  The column with the largest diagonal cofactor is
// taken.  Returns the unnormalised squared length of that column's diagonal
// entry, so the caller can judge conditioning.
PCV_HD double adjugate_eigvec(const double F[10], double lam, double q[4]) {
  double B[4][4];
  unpack4(F, B);
  for (int k = 0; k < 4; ++k) B[k][k] -= lam;
  const double d0 = fabs(cofactor4<0, 0>(B));
  const double d1 = fabs(cofactor4<1, 1>(B));
  const double d2 = fabs(cofactor4<2, 2>(B));
  const double d3 = fabs(cofactor4<3, 3>(B));
  double v[4];
  double best;
  if (d0 >= d1 && d0 >= d2 && d0 >= d3) { adj_column<0>(B, v); best = d0; }
  else if (d1 >= d2 && d1 >= d3) { adj_column<1>(B, v); best = d1; }
  else if (d2 >= d3) { adj_column<2>(B, v); best = d2; }
  else { adj_column<3>(B, v); best = d3; }
  const double nn = v[0] * v[0] + v[1] * v[1] + v[2] * v[2] + v[3] * v[3];
  const double inv = (nn > 0.0) ? 1.0 / sqrt(nn) : 0.0;
  for (int k = 0; k < 4; ++k) q[k] = v[k] * inv;
  return best;
}

// One Jacobi rotation annihilating A[p][qq]; V accumulates eigenvectors (columns).
template <int p, int qq>
PCV_HD void jacobi_rot(double A[4][4], double V[4][4]) {
  const double apq = A[p][qq];
  if (apq == 0.0) return;
  const double theta = (A[qq][qq] - A[p][p]) / (2.0 * apq);
  const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
  const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double akp = A[k][p], akq = A[k][qq];
    A[k][p] = c * akp - s * akq;
    A[k][qq] = s * akp + c * akq;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double apk = A[p][k], aqk = A[qq][k];
    A[p][k] = c * apk - s * aqk;
    A[qq][k] = s * apk + c * aqk;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double vkp = V[k][p], vkq = V[k][qq];
    V[k][p] = c * vkp - s * vkq;
    V[k][qq] = s * vkp + c * vkq;
  }
}

// Cyclic Jacobi eigen-decomposition (fallback for (near-)degenerate top
// eigenvalues, where Newton on the characteristic polynomial and the
// adjugate lose accuracy).  Returns the largest eigenvalue and its vector.
PCV_HD double jacobi_top_body(const double F[10], double q[4]) {
  double A[4][4], V[4][4];
  unpack4(F, A);
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) V[r][c] = (r == c) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 16; ++sweep) {
    const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[0][3] * A[0][3] +
                       A[1][2] * A[1][2] + A[1][3] * A[1][3] + A[2][3] * A[2][3];
    const double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2] + A[3][3] * A[3][3];
    if (off <= 1e-34 * dia || off == 0.0) break;
    jacobi_rot<0, 1>(A, V); jacobi_rot<0, 2>(A, V); jacobi_rot<0, 3>(A, V);
    jacobi_rot<1, 2>(A, V); jacobi_rot<1, 3>(A, V); jacobi_rot<2, 3>(A, V);
  }
  double best = A[0][0];
  for (int k = 0; k < 4; ++k) q[k] = V[k][0];
  if (A[1][1] > best) { best = A[1][1]; for (int k = 0; k < 4; ++k) q[k] = V[k][1]; }
  if (A[2][2] > best) { best = A[2][2]; for (int k = 0; k < 4; ++k) q[k] = V[k][2]; }
  if (A[3][3] > best) { best = A[3][3]; for (int k = 0; k < 4; ++k) q[k] = V[k][3]; }
  return best;
}

struct TopPair {
  double lam, q0, q1, q2, q3;
};

// Out-of-line copy for the streaming kernels: arguments and result travel in
// registers, so nothing is stored to scratch memory unless it is called.
PCV_COLD TopPair jacobi_top_v(double f0, double f1, double f2, double f3, double f4, double f5, double f6,
                              double f7, double f8, double f9) {
  const double F[10] = {f0, f1, f2, f3, f4, f5, f6, f7, f8, f9};
  double q[4];
  const double lam = jacobi_top_body(F, q);
  return TopPair{lam, q[0], q[1], q[2], q[3]};
}

PCV_HD double jacobi_top(const double F[10], double q[4]) {
  const TopPair t = jacobi_top_v(F[0], F[1], F[2], F[3], F[4], F[5], F[6], F[7], F[8], F[9]);
  q[0] = t.q0;
  q[1] = t.q1;
  q[2] = t.q2;
  q[3] = t.q3;
  return t.lam;
}

PCV_HD void quat_to_rot(const double q[4], double R[9]) {
  const double q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3];
  R[0] = q0 * q0 + q1 * q1 - q2 * q2 - q3 * q3;
  R[1] = 2.0 * (q1 * q2 - q0 * q3);
  R[2] = 2.0 * (q1 * q3 + q0 * q2);
  R[3] = 2.0 * (q1 * q2 + q0 * q3);
  R[4] = q0 * q0 - q1 * q1 + q2 * q2 - q3 * q3;
  R[5] = 2.0 * (q2 * q3 - q0 * q1);
  R[6] = 2.0 * (q1 * q3 - q0 * q2);
  R[7] = 2.0 * (q2 * q3 + q0 * q1);
  R[8] = q0 * q0 - q1 * q1 - q2 * q2 + q3 * q3;
}

// Relative gap below which the top eigenpair is taken from Jacobi.
constexpr double kDegenerateGap = 1e-6;

// Optimal superposition from the correlation matrix.  lam_up = (Gx + Ga)/2 is
// an upper bound of lambda_max (Cauchy-Schwarz), so D = Gx + Ga - 2 lambda_max
// is the Eq. 3 distance at the optimal rotation.  Outputs the top eigenvalue,
// the unit quaternion and R (reference onto x).  Returns 1 if the Jacobi
// fallback was used.
PCV_HD int top_eigenpair(const double M[9], double lam_up, double F[10], double& lam, double q[4]) {
  horn_matrix(M, F);
  double c2, c1, c0;
  char_poly(M, F, c2, c1, c0);
  const double scale = lam_up > 1e-300 ? lam_up : 1e-300;
  double dp;
  lam = newton_top_root(c2, c1, c0, lam_up, dp);
  int fb = 0;
  bool fallback = !(dp > kDegenerateGap * scale * scale * scale);
  if (!fallback) {
    const double diag = adjugate_eigvec(F, lam, q);
    fallback = !(diag > 0.1 * dp);     // adj(F - lam I) = -dp q q^T: max |diag| >= dp/4
  }
  if (fallback) {
    lam = jacobi_top(F, q);
    fb = 1;
  }
  return fb;
}

// dR/dq_m contracted with G:  g_q[m] = sum_ab G_ab dR_ab/dq_m.
PCV_HD void rot_grad_q(const double q[4], const double G[9], double g[4]) {
  const double q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3];
  g[0] = 2.0 * (G[0] * q0 - G[1] * q3 + G[2] * q2 + G[3] * q3 + G[4] * q0 - G[5] * q1 - G[6] * q2 + G[7] * q1 + G[8] * q0);
  g[1] = 2.0 * (G[0] * q1 + G[1] * q2 + G[2] * q3 + G[3] * q2 - G[4] * q1 - G[5] * q0 + G[6] * q3 + G[7] * q0 - G[8] * q1);
  g[2] = 2.0 * (-G[0] * q2 + G[1] * q1 + G[2] * q0 + G[3] * q1 + G[4] * q2 + G[5] * q3 - G[6] * q0 + G[7] * q3 - G[8] * q2);
  g[3] = 2.0 * (-G[0] * q3 - G[1] * q0 + G[2] * q1 + G[3] * q0 - G[4] * q3 + G[5] * q2 + G[6] * q1 + G[7] * q2 + G[8] * q3);
}

// The part of the rotation adjoint that does not depend on G: the Cholesky
// factor of K = lam I - F + q q^T (lower triangle) and the reciprocals of its
// diagonal, so that the solve for any G takes multiplications only.
struct AdjointFactor {
  double L[4][4];
  double inv[4];
};

PCV_HD void adjoint_factor(const double F[10], double lam, const double q[4], AdjointFactor& af) {
  double A[4][4], K[4][4];
  unpack4(F, A);
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) K[r][c] = ((r == c) ? lam : 0.0) - A[r][c] + q[r] * q[c];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) af.L[i][j] = 0.0;
  for (int i = 0; i < 4; ++i) {
    for (int j = 0; j <= i; ++j) {
      double s = K[i][j];
      for (int k = 0; k < j; ++k) s -= af.L[i][k] * af.L[j][k];
      if (i == j) {
        af.L[i][i] = sqrt(s > 1e-300 ? s : 1e-300);
        af.inv[i] = 1.0 / af.L[i][i];
      } else {
        af.L[i][j] = s * af.inv[j];
      }
    }
  }
}

// Gamma = d(sum_ab G_ab R_ab)/dM through the top eigenvector of F(M):
// mu = (lam I - F)^+ (g_q projected off q), Gamma_ab = mu^T F(E_ab) q, with
// the factor of K from adjoint_factor.
PCV_HD void adjoint_apply(const AdjointFactor& af, const double q[4], const double G[9], double Gamma[9]) {
  double g[4];
  rot_grad_q(q, G, g);
  const double gq = g[0] * q[0] + g[1] * q[1] + g[2] * q[2] + g[3] * q[3];
  double b[4];
  for (int k = 0; k < 4; ++k) b[k] = g[k] - gq * q[k];
  double y[4], mu[4];
  for (int i = 0; i < 4; ++i) {
    double s = b[i];
    for (int k = 0; k < i; ++k) s -= af.L[i][k] * y[k];
    y[i] = s * af.inv[i];
  }
  for (int i = 3; i >= 0; --i) {
    double s = y[i];
    for (int k = i + 1; k < 4; ++k) s -= af.L[k][i] * mu[k];
    mu[i] = s * af.inv[i];
  }
  double P[4][4];
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) P[r][c] = mu[r] * q[c] + mu[c] * q[r];
  for (int k = 0; k < 4; ++k) P[k][k] *= 0.5;
  // d(mu^T F(M) q)/dM_ab from the entries of F(M).
  Gamma[0] = P[0][0] + P[1][1] - P[2][2] - P[3][3];   // xx
  Gamma[4] = P[0][0] - P[1][1] + P[2][2] - P[3][3];   // yy
  Gamma[8] = P[0][0] - P[1][1] - P[2][2] + P[3][3];   // zz
  Gamma[1] = P[0][3] + P[1][2];                       // xy
  Gamma[3] = -P[0][3] + P[1][2];                      // yx
  Gamma[2] = -P[0][2] + P[1][3];                      // xz
  Gamma[6] = P[0][2] + P[1][3];                       // zx
  Gamma[5] = P[0][1] + P[2][3];                       // yz
  Gamma[7] = -P[0][1] + P[2][3];                      // zy
}

PCV_HD void rotation_adjoint(const double F[10], double lam, const double q[4], const double G[9],
                             double Gamma[9]) {
  AdjointFactor af;
  adjoint_factor(F, lam, q, af);
  adjoint_apply(af, q, G, Gamma);
}

}  // namespace pcv
