// Per-pair FP64 solver wavefront: merges the reduction partials in a fixed
// order, then advances Algorithm 1 (robust point-to-point, and Fast ICP as its
// L2 case) or Algorithm 2 (robust point-to-plane) by one step. Every step ends
// with a request "evaluate at transform T with parameter nu" that the next
// closest-point + reduction pass serves, so control never leaves the device.
//
// Readings of the paper (where it is silent, ambiguous or garbled):
//  - F^(k) = G(x^(k)) - x^(k); the Anderson sums run over m_k columns.
//  - Stage convergence ||T^(k) - T'||_F < eps (point-to-point, 4x4) and
//    ||xi*^(k+1) - xi^(k)|| < eps (point-to-plane); not squared.
//  - Anderson metric: Frobenius of the 4x4 logarithm (rotation part x2) for
//    point-to-point, Euclidean for point-to-plane; Algorithm 2 applies no
//    exponential to the mixed vector.
//  - Gauss-Newton: xi* = xi - A^{-1} sum g B J (the sign that decreases the
//    linearised objective of eq. GNSystem).
//  - Line search: tau halves after each trial, at most l_max trials, the
//    lowest-energy trial is kept.
//  - A safeguard rejection keeps the Anderson history.
//  - Zero total weight or a singular 6x6 system ends the registration with a
//    flag and the current transform.
#include "icp_internal.h"
#include "wave_sum.h"

namespace icp {

// ------------------------------------------------------------------ FP64 math

__device__ inline void skew(const double a[3], double W[9]) {
  W[0] = 0.0;   W[1] = -a[2]; W[2] = a[1];
  W[3] = a[2];  W[4] = 0.0;   W[5] = -a[0];
  W[6] = -a[1]; W[7] = a[0];  W[8] = 0.0;
}

__device__ inline void mm3(const double A[9], const double B[9], double C[9]) {
  double t[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      t[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
  for (int i = 0; i < 9; ++i) C[i] = t[i];
}

__device__ inline void mv3(const double A[9], const double x[3], double y[3]) {
  const double a = A[0] * x[0] + A[1] * x[1] + A[2] * x[2];
  const double b = A[3] * x[0] + A[4] * x[1] + A[5] * x[2];
  const double c = A[6] * x[0] + A[7] * x[1] + A[8] * x[2];
  y[0] = a; y[1] = b; y[2] = c;
}

// Coefficients of the Rodrigues-type series and their theta-derivatives over
// theta:  A = sin/t, B = (1-cos)/t^2, C = (t-sin)/t^3, Ad = A'/t, Bd = B'/t,
// Cd = C'/t. Closed forms for t >= 0.3, Taylor series below.
struct Coef { double A, B, C, Ad, Bd, Cd; };

__device__ inline Coef coeffs(double t) {
  Coef k;
  const double t2 = t * t;
  if (t < 0.3) {
    const double t4 = t2 * t2, t6 = t4 * t2, t8 = t4 * t4, t10 = t8 * t2;
    k.A = 1.0 - t2 / 6.0 + t4 / 120.0 - t6 / 5040.0 + t8 / 362880.0 - t10 / 39916800.0;
    k.B = 0.5 - t2 / 24.0 + t4 / 720.0 - t6 / 40320.0 + t8 / 3628800.0 - t10 / 479001600.0;
    k.C = 1.0 / 6.0 - t2 / 120.0 + t4 / 5040.0 - t6 / 362880.0 + t8 / 39916800.0 - t10 / 6227020800.0;
    // derivative series sum_k (-1)^k 2k t^(2k-2) / (2k+1)!, (2k+2)!, (2k+3)!
    // through k = 6 (the first omitted term is below 1e-17 relative at 0.3)
    k.Ad = -1.0 / 3.0 + t2 / 30.0 - t4 / 840.0 + t6 / 45360.0 - t8 / 3991680.0 + t10 / 518918400.0;
    k.Bd = -1.0 / 12.0 + t2 / 180.0 - t4 / 6720.0 + t6 / 453600.0 - t8 / 47900160.0 + t10 / 7264857600.0;
    k.Cd = -1.0 / 60.0 + t2 / 1260.0 - t4 / 60480.0 + t6 / 4989600.0 - t8 / 622702080.0 +
           t10 / 108972864000.0;
  } else {
    double s, c;
    sincos(t, &s, &c);
    const double h = sin(0.5 * t);
    const double omc = 2.0 * h * h;  // 1 - cos t
    k.A = s / t;
    k.B = omc / t2;
    k.C = (t - s) / (t2 * t);
    k.Ad = (t * c - s) / (t2 * t);
    k.Bd = (t * s - 2.0 * omc) / (t2 * t2);
    k.Cd = (omc * t - 3.0 * (t - s)) / (t2 * t2 * t);
  }
  return k;
}

// exp of the twist xi = (delta, u): R = I + A W + B W^2, t = (I + B W + C W^2) u.
__device__ __forceinline__ void twist_exp(const double xi[6], double T[16]) {
  const double th = sqrt(xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]);
  const Coef k = coeffs(th);
  double W[9], W2[9];
  skew(xi, W);
  mm3(W, W, W2);
  double V[9];
  for (int i = 0; i < 9; ++i) {
    const double I = (i % 4 == 0) ? 1.0 : 0.0;
    const double r = I + k.A * W[i] + k.B * W2[i];
    T[4 * (i / 3) + (i % 3)] = r;
    V[i] = I + k.B * W[i] + k.C * W2[i];
  }
  double t[3];
  mv3(V, xi + 3, t);
  T[3] = t[0]; T[7] = t[1]; T[11] = t[2];
  T[12] = 0.0; T[13] = 0.0; T[14] = 0.0; T[15] = 1.0;
}

// Principal logarithm (angle in [0, pi], Appendix A): the rotation vector from
// the skew part (or, near pi, from the symmetric part), u = V^{-1} t.
__device__ __forceinline__ void twist_log(const double T[16], double xi[6]) {
  const double R[9] = {T[0], T[1], T[2], T[4], T[5], T[6], T[8], T[9], T[10]};
  const double v[3] = {R[7] - R[5], R[2] - R[6], R[3] - R[1]};
  const double sn = 0.5 * sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  const double cs = fmin(1.0, fmax(-1.0, 0.5 * (R[0] + R[4] + R[8] - 1.0)));
  const double th = atan2(sn, cs);
  double d[3];
  if (th < 3.0) {
    // theta / (2 sin theta): the quotient itself is accurate down to tiny
    // angles (no cancellation); below 1e-4 its series, whose first omitted
    // term 7 theta^4 / 720 is below 1e-18
    // sn is sin(theta) (the norm of the skew part's axial vector)
    double f;
    if (th < 1e-4) {
      f = 0.5 + th * th / 12.0;
    } else {
      f = th / (2.0 * sn);
    }
    d[0] = f * v[0]; d[1] = f * v[1]; d[2] = f * v[2];
  } else {
    const double oc = 1.0 - cs;
    double S[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        S[3 * i + j] = (0.5 * (R[3 * i + j] + R[3 * j + i]) - (i == j ? cs : 0.0)) / oc;
    // row kk of the largest diagonal entry (first on ties), gathered by
    // selects so that S stays in registers
    const bool k1 = S[4] > S[0];
    const bool k2 = S[8] > (k1 ? S[4] : S[0]);
    double a[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) a[j] = k2 ? S[6 + j] : (k1 ? S[3 + j] : S[j]);
    const double na = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    a[0] /= na; a[1] /= na; a[2] /= na;
    const double akk = k2 ? a[2] : (k1 ? a[1] : a[0]);
    const double sg = a[0] * v[0] + a[1] * v[1] + a[2] * v[2];
    if (sg < 0.0 || (sg == 0.0 && akk < 0.0)) { a[0] = -a[0]; a[1] = -a[1]; a[2] = -a[2]; }
    d[0] = th * a[0]; d[1] = th * a[1]; d[2] = th * a[2];
  }
  double g;
  if (th < 0.2) {
    const double t2 = th * th;
    g = 1.0 / 12.0 + t2 / 720.0 + t2 * t2 / 30240.0 + t2 * t2 * t2 / 1209600.0 +
        t2 * t2 * t2 * t2 / 47900160.0;
  } else {
    const double h = sin(0.5 * th);
    g = (1.0 - th * sn / (4.0 * h * h)) / (th * th);
  }
  double W[9], W2[9];
  skew(d, W);
  mm3(W, W, W2);
  const double t[3] = {T[3], T[7], T[11]};
  double Vi[9];
  for (int i = 0; i < 9; ++i) Vi[i] = ((i % 4 == 0) ? 1.0 : 0.0) - 0.5 * W[i] + g * W2[i];
  double u[3];
  mv3(Vi, t, u);
  xi[0] = d[0]; xi[1] = d[1]; xi[2] = d[2];
  xi[3] = u[0]; xi[4] = u[1]; xi[5] = u[2];
}

// Derivatives of R(delta) and t = V(delta) u at xi (the gradient of App. D):
// K[0..26]  dR/d delta_j = A E_j + B (E_j W + W E_j) + Ad d_j W + Bd d_j W^2
// K[27..35] dt/d delta (column j) = [B E_j + C (E_j W + W E_j) + Bd d_j W + Cd d_j W^2] u
// K[36..44] dt/du = I + B W + C W^2
__device__ __forceinline__ void twist_derivs(const double xi[6], double K[45]) {
  const double* d = xi;
  const double* u = xi + 3;
  const double th = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  const Coef k = coeffs(th);
  double W[9], W2[9];
  skew(d, W);
  mm3(W, W, W2);
  double Wu[3], W2u[3];
  mv3(W, u, Wu);
  mv3(W2, u, W2u);
  for (int j = 0; j < 3; ++j) {
    double e[3] = {0.0, 0.0, 0.0};
    e[j] = 1.0;
    double E[9], EW[9], WE[9];
    skew(e, E);
    mm3(E, W, EW);
    mm3(W, E, WE);
    for (int i = 0; i < 9; ++i)
      K[9 * j + i] = k.A * E[i] + k.B * (EW[i] + WE[i]) + k.Ad * d[j] * W[i] + k.Bd * d[j] * W2[i];
    double S[9];
    for (int i = 0; i < 9; ++i) S[i] = k.B * E[i] + k.C * (EW[i] + WE[i]);
    double Su[3];
    mv3(S, u, Su);
    for (int a = 0; a < 3; ++a) K[27 + 3 * a + j] = Su[a] + k.Bd * d[j] * Wu[a] + k.Cd * d[j] * W2u[a];
  }
  for (int i = 0; i < 9; ++i) K[36 + i] = ((i % 4 == 0) ? 1.0 : 0.0) + k.B * W[i] + k.C * W2[i];
}

// Symmetric 4x4 eigen-decomposition by cyclic Jacobi rotations; returns the
// unit eigenvector of the largest eigenvalue and the two largest eigenvalues.
// One Jacobi rotation in the (p, r) plane of the symmetric 4x4 A, zeroing
// A[p][r], accumulated onto the columns of V. A rotation by a negligible
// angle is skipped (its square is far below the stopping threshold on the
// off-diagonal mass).
__device__ __forceinline__ void jacobi_rot(double A[16], double V[16], int p, int r) {
  const double apr = A[4 * p + r];
  if (!(fabs(apr) > 1e-18 * (fabs(A[5 * p]) + fabs(A[5 * r])))) return;
  const double theta = (A[4 * r + r] - A[4 * p + p]) / (2.0 * apr);
  const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
  const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const double akp = A[4 * kk + p], akr = A[4 * kk + r];
    A[4 * kk + p] = c * akp - s * akr;
    A[4 * kk + r] = s * akp + c * akr;
  }
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const double apk = A[4 * p + kk], ark = A[4 * r + kk];
    A[4 * p + kk] = c * apk - s * ark;
    A[4 * r + kk] = s * apk + c * ark;
  }
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const double vkp = V[4 * kk + p], vkr = V[4 * kk + r];
    V[4 * kk + p] = c * vkp - s * vkr;
    V[4 * kk + r] = s * vkp + c * vkr;
  }
}

// Solves M y = b for a 4x4 M by Gaussian elimination with partial pivoting
// (row exchanges by selects, so that everything stays in registers); an exact
// zero pivot is replaced by a tiny one (M is then an exactly singular shifted
// matrix and any large solution along its null space is what is wanted).
__device__ __forceinline__ void solve4(double M[16], double b[4], double tiny) {
  double inv[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    int p = k;
    double best = fabs(M[5 * k]);
#pragma unroll
    for (int i = k + 1; i < 4; ++i)
      if (fabs(M[4 * i + k]) > best) { best = fabs(M[4 * i + k]); p = i; }
#pragma unroll
    for (int i = k + 1; i < 4; ++i) {
      const bool sw = i == p;
#pragma unroll
      for (int j = k; j < 4; ++j) {
        const double a = M[4 * k + j], c = M[4 * i + j];
        M[4 * k + j] = sw ? c : a;
        M[4 * i + j] = sw ? a : c;
      }
      const double a = b[k], c = b[i];
      b[k] = sw ? c : a;
      b[i] = sw ? a : c;
    }
    if (M[5 * k] == 0.0) M[5 * k] = tiny;
    inv[k] = 1.0 / M[5 * k];
#pragma unroll
    for (int i = k + 1; i < 4; ++i) {
      const double f = M[4 * i + k] * inv[k];
#pragma unroll
      for (int j = k + 1; j < 4; ++j) M[4 * i + j] -= f * M[4 * k + j];
      b[i] -= f * b[k];
    }
  }
#pragma unroll
  for (int k = 3; k >= 0; --k) {
    double v = b[k];
#pragma unroll
    for (int j = k + 1; j < 4; ++j) v -= M[4 * k + j] * b[j];
    b[k] = v * inv[k];
  }
}

// Top eigenpair of a symmetric 4x4 A by Rayleigh-quotient iteration from the
// previous top eigenvector x (unit). Returns false unless the iteration
// settles and the result is certified as the top eigenvector: with an
// orthonormal basis of its complement (a Householder reflection), b I - B is
// positive definite (Cholesky) for the complement block B and
// b = l0 - 2e-12 |l0| - |residual|, so every other eigenvalue is below b,
// which then stands in for l1 (the gap test is decided).
__device__ bool top_eig_rqi(const double A[16], const double x0[4], double q[4], double& l0,
                            double& l1) {
  double nA = 0.0;
#pragma unroll
  for (int i = 0; i < 16; ++i) nA += A[i] * A[i];
  nA = sqrt(nA);
  if (!(nA > 0.0)) return false;
  double x[4] = {x0[0], x0[1], x0[2], x0[3]};
  double mu = 0.0, rn = 0.0, rn_prev = __builtin_inf();
  bool settled = false;
  for (int it = 0; it < 6; ++it) {
    double Ax[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) Ax[i] = A[4 * i] * x[0] + A[4 * i + 1] * x[1] + A[4 * i + 2] * x[2] + A[4 * i + 3] * x[3];
    mu = x[0] * Ax[0] + x[1] * Ax[1] + x[2] * Ax[2] + x[3] * Ax[3];
    double r2 = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) r2 += (Ax[i] - mu * x[i]) * (Ax[i] - mu * x[i]);
    rn = sqrt(r2);
    // settled: at the rounding level, or no longer shrinking (the noise floor)
    if (rn <= 1e-15 * nA || (rn <= 1e-12 * nA && rn > 0.25 * rn_prev)) { settled = true; break; }
    rn_prev = rn;
    double M[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) M[i] = A[i] - ((i % 5 == 0) ? mu : 0.0);
    double y[4] = {x[0], x[1], x[2], x[3]};
    solve4(M, y, 1e-300 * nA);
    const double ny = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2] + y[3] * y[3]);
    if (!(ny > 0.0) || !(ny < __builtin_inf())) return false;
    const double iny = 1.0 / ny;
#pragma unroll
    for (int i = 0; i < 4; ++i) x[i] = y[i] * iny;
  }
  if (!settled || !(rn <= 1e-12 * nA)) return false;
  // Householder reflection H = I - 2 v v^T / (v^T v), v = x + sign(x_0) e_0
  // (v^T v = 2 (1 + |x_0|) >= 2 for any unit x, so the reflection is well
  // conditioned whichever component carries it)
  double v[4] = {x[0], x[1], x[2], x[3]};
  const double sg = x[0] >= 0.0 ? 1.0 : -1.0;
  v[0] += sg;
  const double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2] + v[3] * v[3];
  const double s2 = 2.0 / vv;
  double H[16];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) H[4 * i + j] = ((i == j) ? 1.0 : 0.0) - s2 * v[i] * v[j];
  // H A H; column 0 of H is -sg x, columns 1..3 span its complement
  double AH[16];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 1; j < 4; ++j)
      AH[4 * i + j] = A[4 * i] * H[j] + A[4 * i + 1] * H[4 + j] + A[4 * i + 2] * H[8 + j] + A[4 * i + 3] * H[12 + j];
  // complement block: rows and columns 1..3 of H A H
  double B[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      B[3 * a + c] = H[a + 1] * AH[c + 1] + H[4 + a + 1] * AH[4 + c + 1] + H[8 + a + 1] * AH[8 + c + 1] +
                     H[12 + a + 1] * AH[12 + c + 1];
  l0 = mu;
  const double b = mu - 2e-12 * fabs(mu) - rn;
  const double c11 = b - B[0], c21 = -0.5 * (B[3] + B[1]), c31 = -0.5 * (B[6] + B[2]);
  const double c22 = b - B[4], c32 = -0.5 * (B[7] + B[5]), c33 = b - B[8];
  if (!(c11 > 0.0)) return false;
  const double l11 = sqrt(c11), il11 = 1.0 / l11;
  const double l21 = c21 * il11, l31 = c31 * il11;
  const double d22 = c22 - l21 * l21;
  if (!(d22 > 0.0)) return false;
  const double l22 = sqrt(d22);
  const double l32 = (c32 - l31 * l21) / l22;
  if (!(c33 - l31 * l31 - l32 * l32 > 0.0)) return false;
  l1 = b;
#pragma unroll
  for (int i = 0; i < 4; ++i) q[i] = x[i];
  return true;
}

// Largest eigenpair of a symmetric 4x4 matrix (l1: second largest, or a
// certified upper bound on it). Warm start: Rayleigh-quotient iteration from
// the previous top eigenvector (column 0 of V); otherwise (first call,
// uncertified) cyclic Jacobi rotations from the identity. Column 0 of V
// keeps the top eigenvector for the next call.
__device__ void sym4_top(double A[16], double V[16], double q[4], double& l0, double& l1) {
  const double x0[4] = {V[0], V[4], V[8], V[12]};
  const double n0 = x0[0] * x0[0] + x0[1] * x0[1] + x0[2] * x0[2] + x0[3] * x0[3];
  if (n0 > 0.5 && top_eig_rqi(A, x0, q, l0, l1)) {
#pragma unroll
    for (int i = 0; i < 4; ++i) V[4 * i] = q[i];
    return;
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) V[i] = (i % 5 == 0) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        tot += A[4 * i + j] * A[4 * i + j];
        if (i != j) off += A[4 * i + j] * A[4 * i + j];
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    // fixed (p, r) order, unrolled so that A and V stay in registers
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int r = p + 1; r < 4; ++r) jacobi_rot(A, V, p, r);
  }
  // largest and second largest diagonal entries (first index on ties), by
  // selects so that A and V stay in registers
  int b0 = 0;
  double v0 = A[0];
#pragma unroll
  for (int i = 1; i < 4; ++i) {
    const bool g = A[5 * i] > v0;
    v0 = g ? A[5 * i] : v0;
    b0 = g ? i : b0;
  }
  double v1 = b0 == 0 ? A[5] : A[0];
#pragma unroll
  for (int i = 0; i < 4; ++i) v1 = (i != b0 && A[5 * i] > v1) ? A[5 * i] : v1;
  l0 = v0;
  l1 = v1;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    q[i] = b0 == 0 ? V[4 * i] : b0 == 1 ? V[4 * i + 1] : b0 == 2 ? V[4 * i + 2] : V[4 * i + 3];
#pragma unroll
  for (int i = 0; i < 4; ++i) V[4 * i] = q[i];
}

// Weighted absolute orientation from the merged moments by Horn's unit-
// quaternion method (the optimum of eq. WelschAlignment over rotations):
// S = sum w (p - pb)(q - qb)^T, the quaternion is the top eigenvector of the
// symmetric 4x4 matrix built from S; t = qb - R pb.
__device__ unsigned align_p2p(const double* mom, const double cP[3], const double cQ[3],
                              double V[16], double T[16]) {
  const double W = mom[1];
  if (!(W > 1e-300)) return F_ZERO_WEIGHT;
  const double iW = 1.0 / W;
  const double pb[3] = {mom[2] * iW, mom[3] * iW, mom[4] * iW};
  const double qb[3] = {mom[5] * iW, mom[6] * iW, mom[7] * iW};
  double S[9];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) S[3 * a + b] = mom[8 + 3 * a + b] - pb[a] * mom[5 + b];
  const double Sxx = S[0], Sxy = S[1], Sxz = S[2], Syx = S[3], Syy = S[4], Syz = S[5],
               Szx = S[6], Szy = S[7], Szz = S[8];
  double N[16] = {Sxx + Syy + Szz, Syz - Szy,        Szx - Sxz,        Sxy - Syx,
                  Syz - Szy,       Sxx - Syy - Szz,  Sxy + Syx,        Szx + Sxz,
                  Szx - Sxz,       Sxy + Syx,        -Sxx + Syy - Szz, Syz + Szy,
                  Sxy - Syx,       Szx + Sxz,        Syz + Szy,        -Sxx - Syy + Szz};
  double q[4], l0, l1;
  sym4_top(N, V, q, l0, l1);
  // rank test: for a proper optimum the two largest eigenvalues of the
  // quaternion matrix differ by 2 (s1 + s2) (singular values of S), so a
  // vanishing gap means rank(S) <= 1 and the rotation is not determined
  unsigned flags = 0;
  if (!(l0 - l1 > 1e-12 * fabs(l0))) flags |= F_DEGENERATE;
  const double q0 = q[0], qx = q[1], qy = q[2], qz = q[3];
  double R[9] = {q0 * q0 + qx * qx - qy * qy - qz * qz, 2.0 * (qx * qy - q0 * qz), 2.0 * (qx * qz + q0 * qy),
                 2.0 * (qy * qx + q0 * qz), q0 * q0 - qx * qx + qy * qy - qz * qz, 2.0 * (qy * qz - q0 * qx),
                 2.0 * (qz * qx - q0 * qy), 2.0 * (qz * qy + q0 * qx), q0 * q0 - qx * qx - qy * qy + qz * qz};
  const double pbar[3] = {cP[0] + pb[0], cP[1] + pb[1], cP[2] + pb[2]};
  const double qbar[3] = {cQ[0] + qb[0], cQ[1] + qb[1], cQ[2] + qb[2]};
  double Rp[3];
  mv3(R, pbar, Rp);
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) T[4 * i + j] = R[3 * i + j];
    T[4 * i + 3] = qbar[i] - Rp[i];
  }
  T[12] = 0.0; T[13] = 0.0; T[14] = 0.0; T[15] = 1.0;
  return flags;
}

// Gauss-Newton candidate xi* = xi - A^{-1} c by Cholesky (eq. GNSystem).
__device__ unsigned gn_p2pl(const double* mom, const double xi[6], double out[6]) {
  for (int a = 0; a < 6; ++a) out[a] = xi[a];
  if (!(mom[1] > 1e-300)) return F_ZERO_WEIGHT;
  // every loop is unrolled, so that the small matrices stay in registers
  double A[36];
#pragma unroll
  for (int a = 0; a < 6; ++a)
#pragma unroll
    for (int b = a; b < 6; ++b) {
      const int t = 2 + 6 * a - a * (a - 1) / 2 + (b - a);  // upper triangle, row-major
      A[6 * a + b] = mom[t];
      A[6 * b + a] = mom[t];
    }
  double dmax = 0.0;
#pragma unroll
  for (int a = 0; a < 6; ++a) dmax = fmax(dmax, A[7 * a]);
  if (!(dmax > 0.0)) return F_DEGENERATE;
  double L[36];
#pragma unroll
  for (int i = 0; i < 36; ++i) L[i] = 0.0;
  bool deg = false;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    double s = A[7 * j];
#pragma unroll
    for (int k = 0; k < j; ++k) s -= L[6 * j + k] * L[6 * j + k];
    if (!(s > 1e-14 * dmax)) deg = true;
    L[7 * j] = deg ? 1.0 : sqrt(s);
#pragma unroll
    for (int i = j + 1; i < 6; ++i) {
      double v = A[6 * i + j];
#pragma unroll
      for (int k = 0; k < j; ++k) v -= L[6 * i + k] * L[6 * j + k];
      L[6 * i + j] = v / L[7 * j];
    }
  }
  if (deg) return F_DEGENERATE;
  double y[6], x[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    double v = mom[23 + i];
#pragma unroll
    for (int k = 0; k < i; ++k) v -= L[6 * i + k] * y[k];
    y[i] = v / L[7 * i];
  }
#pragma unroll
  for (int i = 5; i >= 0; --i) {
    double v = y[i];
#pragma unroll
    for (int k = i + 1; k < 6; ++k) v -= L[6 * k + i] * x[k];
    x[i] = v / L[7 * i];
  }
#pragma unroll
  for (int a = 0; a < 6; ++a) out[a] = xi[a] - x[a];
  return 0;
}

// Anderson mixing: theta = argmin || F^k - sum_j theta_j dF_j ||^2 in the given
// metric by normal equations (Cholesky, pivot <= 1e-10 max diag = singular,
// theta = 0); returns G^k - sum_j theta_j dG_j.
// The history length is a template parameter so that every loop unrolls and
// the small matrices live in registers.
template <int mk>
__device__ bool anderson_mk(const SlotState& S, int k, int metric, double out[6]) {
  double dF[6][6], dG[6][6];
#pragma unroll
  for (int j = 1; j <= mk; ++j)
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      dF[j - 1][a] = S.F[(k - j + 1) % kHist][a] - S.F[(k - j) % kHist][a];
      dG[j - 1][a] = S.G[(k - j + 1) % kHist][a] - S.G[(k - j) % kHist][a];
    }
  const double* Fk = S.F[k % kHist];
  const double wr = metric == 0 ? 2.0 : 1.0;
  double N[36], r[6], dmax = 0.0;
#pragma unroll
  for (int i = 0; i < mk; ++i) {
    r[i] = wr * (dF[i][0] * Fk[0] + dF[i][1] * Fk[1] + dF[i][2] * Fk[2]) + dF[i][3] * Fk[3] +
           dF[i][4] * Fk[4] + dF[i][5] * Fk[5];
#pragma unroll
    for (int j = 0; j < mk; ++j)
      N[6 * i + j] = wr * (dF[i][0] * dF[j][0] + dF[i][1] * dF[j][1] + dF[i][2] * dF[j][2]) +
                     dF[i][3] * dF[j][3] + dF[i][4] * dF[j][4] + dF[i][5] * dF[j][5];
    dmax = fmax(dmax, N[7 * i]);
  }
  double L[36], iL[6], th[6];
#pragma unroll
  for (int i = 0; i < 36; ++i) L[i] = 0.0;
  bool sing = !(dmax > 0.0);
#pragma unroll
  for (int j = 0; j < mk; ++j) {
    double s = N[7 * j];
#pragma unroll
    for (int kk = 0; kk < j; ++kk) s -= L[6 * j + kk] * L[6 * j + kk];
    if (!(s > 1e-10 * dmax)) sing = true;
    L[7 * j] = sing ? 1.0 : sqrt(s);
    iL[j] = 1.0 / L[7 * j];
#pragma unroll
    for (int i = j + 1; i < mk; ++i) {
      double v = N[6 * i + j];
#pragma unroll
      for (int kk = 0; kk < j; ++kk) v -= L[6 * i + kk] * L[6 * j + kk];
      L[6 * i + j] = v * iL[j];
    }
  }
  if (sing) {
#pragma unroll
    for (int i = 0; i < mk; ++i) th[i] = 0.0;
  } else {
    double y[6];
#pragma unroll
    for (int i = 0; i < mk; ++i) {
      double v = r[i];
#pragma unroll
      for (int kk = 0; kk < i; ++kk) v -= L[6 * i + kk] * y[kk];
      y[i] = v * iL[i];
    }
#pragma unroll
    for (int i = mk - 1; i >= 0; --i) {
      double v = y[i];
#pragma unroll
      for (int kk = i + 1; kk < mk; ++kk) v -= L[6 * kk + i] * th[kk];
      th[i] = v * iL[i];
    }
  }
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    double v = S.G[k % kHist][a];
#pragma unroll
    for (int j = 1; j <= mk; ++j) v -= th[j - 1] * dG[j - 1][a];
    out[a] = v;
  }
  return sing;
}

__device__ bool anderson(const SlotState& S, int k, int mk, int metric, double out[6]) {
  switch (mk) {
    case 0: return anderson_mk<0>(S, k, metric, out);
    case 1: return anderson_mk<1>(S, k, metric, out);
    case 2: return anderson_mk<2>(S, k, metric, out);
    case 3: return anderson_mk<3>(S, k, metric, out);
    case 4: return anderson_mk<4>(S, k, metric, out);
    case 5: return anderson_mk<5>(S, k, metric, out);
    default: return anderson_mk<6>(S, k, metric, out);  // m <= 6 is validated at submission
  }
}

// ------------------------------------------------------------------ requests

__device__ inline bool same_bits(const double* a, const double* b, int n) {
  for (int i = 0; i < n; ++i)
    if (__double_as_longlong(a[i]) != __double_as_longlong(b[i])) return false;
  return true;
}

__device__ inline void set_nu(SlotState& S, double nu) {
  S.inv2nu2 = mode_l2(S.mode) ? 0.0 : 1.0 / (2.0 * nu * nu);
  S.nu_eval = mode_l2(S.mode) ? 0.0 : nu;
}

// Candidate lists are rebuilt on the first two passes (the first has no warm
// bounds) and whenever some source may have moved farther than the margin
// since the last build: |T p - Tref p| <= ||dR||_F r + |dR c + dt| with c, r
// the centre and half-diagonal of the source box, plus an allowance for the
// FP32 rounding of both transformed points.
__device__ void plan_lists(SlotState& S) {
  if (S.reuse) return;
  bool rebuild = S.nn_passes <= 2 || !(S.verlet > 0.0);
  if (!rebuild) {
    double fro = 0.0, v2 = 0.0, r2 = 0.0, c2 = 0.0, tt = 0.0;
    for (int k = 0; k < 3; ++k) {
      const double e = 0.5 * ((double)S.bbP[3 + k] - (double)S.bbP[k]);
      r2 += e * e;
      c2 += S.cP[k] * S.cP[k];
      double v = S.Teval[4 * k + 3] - S.Tref[4 * k + 3];
      for (int j = 0; j < 3; ++j) {
        const double d = S.Teval[4 * k + j] - S.Tref[4 * k + j];
        fro += d * d;
        v += d * S.cP[j];
      }
      v2 += v * v;
      tt += fabs(S.Teval[4 * k + 3]) + fabs(S.Tref[4 * k + 3]);
    }
    const double r = sqrt(r2);
    const double disp = sqrt(fro) * r + sqrt(v2);
    const double slack = 1e-6 * (sqrt(c2) + r + tt);
    rebuild = !(disp + slack <= S.verlet);
  }
  S.cull = rebuild ? 1 : 0;
  if (rebuild)
    for (int i = 0; i < 16; ++i) S.Tref[i] = S.Teval[i];
}

__device__ __forceinline__ void request_T(SlotState& S, const double T[16], double nu) {
  S.evaluations++;
  const bool same = S.have_last && same_bits(S.last_key, T, 16);
  S.reuse = same ? 1 : 0;
  if (!same) {
    for (int i = 0; i < 16; ++i) S.last_key[i] = T[i];
    S.have_last = 1;
    S.nn_passes++;
  }
  for (int i = 0; i < 16; ++i) S.Teval[i] = T[i];
  plan_lists(S);
  set_nu(S, nu);
}

__device__ __forceinline__ void request_xi(SlotState& S, const double xi[6], double nu) {
  S.evaluations++;
  const bool same = S.have_last && same_bits(S.last_key, xi, 6);
  S.reuse = same ? 1 : 0;
  if (!same) {
    for (int i = 0; i < 6; ++i) S.last_key[i] = xi[i];
    S.have_last = 1;
    S.nn_passes++;
  }
  twist_exp(xi, S.Teval);
  twist_derivs(xi, S.K);
  plan_lists(S);
  set_nu(S, nu);
}

__device__ void finish(SlotState& S, const double T[16], double E) {
  for (int i = 0; i < 16; ++i) S.Tres[i] = T[i];
  S.energy = E;
  S.nu_final = mode_l2(S.mode) ? 0.0 : S.nu;
  S.status = ST_DONE;
}

__device__ inline int stage_cap(const SlotState& S) {
  long v = (long)S.iter_first + (long)S.stage * S.iter_inc;
  if (S.iter_cap > 0 && v > S.iter_cap) v = S.iter_cap;
  return (int)v;
}

__device__ inline double frob16(const double* a, const double* b) {
  double s = 0.0;
  for (int i = 0; i < 16; ++i) s += (a[i] - b[i]) * (a[i] - b[i]);
  return sqrt(s);
}

__device__ inline void cpy(double* d, const double* s, int n) {
  for (int i = 0; i < n; ++i) d[i] = s[i];
}

// ------------------------------------------------------------------ Algorithm 1

__device__ void step_p2p(SlotState& S, const double* mom, double* trace_prop) {
  const double E = mom[0];
  double Tprop[16];
  const unsigned pf = align_p2p(mom, S.cP, S.cQ, S.Vq, Tprop);
  if (trace_prop) cpy(trace_prop, (pf & F_ZERO_WEIGHT) ? S.Teval : Tprop, 16);
  const int m = S.m;
  int sm = S.sm;
  if (sm == SM_INIT) {
    if (S.mode != P2P_L2 && S.nu_auto) {
      S.nu = 3.0 * sqrt(S.median);
      S.want_median = 0;
      request_T(S, S.Tkm1, S.nu);
      S.sm = SM_STAGE_EVAL;
      return;
    }
    S.nu = S.mode == P2P_L2 ? 0.0 : S.nu_max;
    S.want_median = 0;
    sm = SM_STAGE_EVAL;
  }
  if (sm == SM_STAGE_EVAL) {
    // stage start: T' = align(Q^(k-1), T^(k-1), nu)
    S.stages++;
    S.Inu = stage_cap(S);
    S.kstart = S.k - 1;
    S.Eprev = __builtin_inf();
    if (pf & F_ZERO_WEIGHT) {
      S.flags |= F_ZERO_WEIGHT;
      cpy(S.Tk, S.Tkm1, 16);
      finish(S, S.Tk, E);
      return;
    }
    S.flags |= pf & F_DEGENERATE;
    cpy(S.Tp, Tprop, 16);
    cpy(S.Tk, Tprop, 16);
    double lp[6], lq[6];
    twist_log(S.Tp, lp);
    twist_log(S.Tkm1, lq);
    for (int a = 0; a < 6; ++a) {
      S.G[(S.k - 1) % kHist][a] = lp[a];
      S.F[(S.k - 1) % kHist][a] = lp[a] - lq[a];
      S.lk[a] = lp[a];
    }
    S.is_aa = 0;
    request_T(S, S.Tk, S.nu);
    S.sm = SM_ITER_EVAL;
    return;
  }
  bool post = false;
  if (sm == SM_ITER_EVAL) {
    if (!(S.k - S.kstart <= S.Inu)) {
      // iteration cap of the stage reached
      S.flags = (S.flags & ~F_CONVERGED) | F_MAX_ITER;
      goto stage_end;
    }
    if (S.max_total > 0 && S.total >= S.max_total) {
      S.flags |= F_MAX_ITER;
      finish(S, S.Tk, E);
      return;
    }
    S.iterations++;
    S.total++;
    if (m > 0 && E >= S.Eprev) {
      // safeguard: revert to the un-accelerated iterate (whose log is the
      // newest G entry)
      cpy(S.Tk, S.Tp, 16);
      cpy(S.lk, S.G[(S.k - 1) % kHist], 6);
      S.aa_rejected++;
      request_T(S, S.Tk, S.nu);
      S.sm = SM_REVERT_EVAL;
      return;
    }
    if (S.is_aa) S.aa_accepted++;
    post = true;
  } else if (sm == SM_REVERT_EVAL) {
    post = true;
  }
  if (post) {
    S.Eprev = E;
    S.Eit = E;
    if (pf & F_ZERO_WEIGHT) {
      S.flags |= F_ZERO_WEIGHT;
      finish(S, S.Tk, E);
      return;
    }
    S.flags |= pf & F_DEGENERATE;
    cpy(S.Tp, Tprop, 16);
    if (frob16(S.Tk, S.Tp) < S.eps) {
      S.flags = (S.flags & ~F_MAX_ITER) | F_CONVERGED;
      goto stage_end;
    }
    double Tn[16];
    if (m == 0) {
      cpy(Tn, S.Tp, 16);
      S.is_aa = 0;
    } else {
      // F^(k) = G^(k) - log T^(k) with log T^(k) taken from the transform
      // itself (Algorithm 1): the logarithm of the iterate is re-taken after
      // the exponential of the mixed parameters, not carried over from them
      double lp[6], xa[6];
      twist_log(S.Tp, lp);
      for (int a = 0; a < 6; ++a) {
        S.G[S.k % kHist][a] = lp[a];
        S.F[S.k % kHist][a] = lp[a] - S.lk[a];
      }
      const int mk = (S.k - S.kstart) < m ? (S.k - S.kstart) : m;
      if (anderson(S, S.k, mk, 0, xa)) S.flags |= F_AA_SINGULAR;
      twist_exp(xa, Tn);
      twist_log(Tn, S.lk);
      S.is_aa = 1;
    }
    cpy(S.Tk, Tn, 16);
    S.k++;
    request_T(S, S.Tk, S.nu);
    S.sm = SM_ITER_EVAL;
    return;
  }
  return;
stage_end:
  if (S.mode == P2P_L2 || S.nu == S.nu_min) {
    finish(S, S.Tk, E);
    return;
  }
  S.nu = fmax(S.nu / 2.0, S.nu_min);
  S.k++;
  S.stage++;
  cpy(S.Tkm1, S.Tk, 16);
  request_T(S, S.Tkm1, S.nu);
  S.sm = SM_STAGE_EVAL;
}

// ------------------------------------------------------------------ Algorithm 2

__device__ void step_p2pl(SlotState& S, const double* mom, double* trace_prop) {
  const double E = mom[0];
  double xprop[6];
  const double* xeval = S.last_key;  // parameters of this evaluation
  const unsigned pf = gn_p2pl(mom, xeval, xprop);
  if (trace_prop) {
    cpy(trace_prop, xprop, 6);
    cpy(trace_prop + 6, xeval, 6);
    for (int i = 12; i < 16; ++i) trace_prop[i] = 0.0;
  }
  int sm = S.sm;
  if (sm == SM_INIT) {
    if (S.nu_auto) {
      S.nu = 3.0 * S.median;
      S.want_median = 0;
      request_xi(S, S.xkm1, S.nu);
      S.sm = SM_STAGE_EVAL;
      return;
    }
    S.nu = mode_l2(S.mode) ? 0.0 : S.nu_max;
    S.want_median = 0;
    sm = SM_STAGE_EVAL;
  }
  if (sm == SM_STAGE_EVAL) {
    S.stages++;
    S.Inu = stage_cap(S);
    S.kstart = S.k - 1;
    S.Eprev = __builtin_inf();
    if (pf & (F_ZERO_WEIGHT | F_DEGENERATE)) {
      S.flags |= pf;
      cpy(S.xk, S.xkm1, 6);
      double T[16];
      twist_exp(S.xk, T);
      finish(S, T, E);
      return;
    }
    cpy(S.xstar, xprop, 6);
    for (int a = 0; a < 6; ++a) {
      S.G[(S.k - 1) % kHist][a] = S.xstar[a];
      S.F[(S.k - 1) % kHist][a] = S.xstar[a] - S.xkm1[a];
    }
    cpy(S.xk, S.xstar, 6);
    S.is_aa = 0;
    request_xi(S, S.xk, S.nu);
    S.sm = SM_ITER_EVAL;
    return;
  }
  bool post = false;
  if (sm == SM_ITER_EVAL) {
    S.Eit = E;  // energy of the current iterate (used at stage end)
    if (!(S.k - S.kstart <= S.Inu)) {
      S.flags = (S.flags & ~F_CONVERGED) | F_MAX_ITER;
      goto stage_end;
    }
    if (S.max_total > 0 && S.total >= S.max_total) {
      S.flags |= F_MAX_ITER;
      double T[16];
      twist_exp(S.xk, T);
      finish(S, T, E);
      return;
    }
    S.iterations++;
    S.total++;
    cpy(S.best_prop, xprop, 6);
    S.best_flags = pf;
    if (E >= S.Eprev) {
      // line search from xi^(k-1) toward xi*^(k)
      S.tau = 1.0;
      S.ls_l = 1;
      if (S.lmax >= 1) {
        for (int a = 0; a < 6; ++a) S.xt[a] = S.xkm1[a] + S.tau * (S.xstar[a] - S.xkm1[a]);
        request_xi(S, S.xt, S.nu);
        S.sm = SM_LS_EVAL;
        return;
      }
      if (S.is_aa) S.aa_rejected++;
    } else if (S.is_aa) {
      S.aa_accepted++;
    }
    post = true;
  } else if (sm == SM_LS_EVAL) {
    S.ls_trials++;
    if (E < S.Eit) {
      S.Eit = E;
      cpy(S.xk, S.xt, 6);
      cpy(S.best_prop, xprop, 6);
      S.best_flags = pf;
    }
    if (!(E < S.Eprev)) {
      S.tau *= 0.5;
      S.ls_l++;
      if (S.ls_l <= S.lmax) {
        for (int a = 0; a < 6; ++a) S.xt[a] = S.xkm1[a] + S.tau * (S.xstar[a] - S.xkm1[a]);
        request_xi(S, S.xt, S.nu);
        S.sm = SM_LS_EVAL;
        return;
      }
    }
    if (S.is_aa) S.aa_rejected++;
    post = true;
  }
  if (post) {
    S.Eprev = S.Eit;
    if (S.best_flags & (F_ZERO_WEIGHT | F_DEGENERATE)) {
      S.flags |= S.best_flags;
      double T[16];
      twist_exp(S.xk, T);
      finish(S, T, S.Eit);
      return;
    }
    // Algorithm 2 tests the parameter change; classical point-to-plane ICP
    // the change of transform, as the comparison methods do (App. E)
    double dn = 0.0;
    if (mode_l2(S.mode)) {
      double Tn[16], Tc[16];
      twist_exp(S.best_prop, Tn);
      twist_exp(S.xk, Tc);
      dn = frob16(Tn, Tc);
    } else {
      for (int a = 0; a < 6; ++a) dn += (S.best_prop[a] - S.xk[a]) * (S.best_prop[a] - S.xk[a]);
      dn = sqrt(dn);
    }
    if (dn < S.eps) {
      S.flags = (S.flags & ~F_MAX_ITER) | F_CONVERGED;
      goto stage_end;
    }
    for (int a = 0; a < 6; ++a) {
      S.G[S.k % kHist][a] = S.best_prop[a];
      S.F[S.k % kHist][a] = S.best_prop[a] - S.xk[a];
    }
    double xn[6];
    if (S.m == 0) {
      cpy(xn, S.best_prop, 6);
      S.is_aa = 0;
    } else {
      const int mk = (S.k - S.kstart) < S.m ? (S.k - S.kstart) : S.m;
      if (anderson(S, S.k, mk, 1, xn)) S.flags |= F_AA_SINGULAR;
      S.is_aa = 1;
    }
    cpy(S.xkm1, S.xk, 6);
    cpy(S.xstar, S.best_prop, 6);
    cpy(S.xk, xn, 6);
    S.k++;
    request_xi(S, S.xk, S.nu);
    S.sm = SM_ITER_EVAL;
    return;
  }
  return;
stage_end:
  if (mode_l2(S.mode) || S.nu == S.nu_min) {
    double T[16];
    twist_exp(S.xk, T);
    finish(S, T, S.Eit);
    return;
  }
  S.nu = fmax(S.nu / 2.0, S.nu_min);
  S.k++;
  S.stage++;
  cpy(S.xkm1, S.xk, 6);
  request_xi(S, S.xkm1, S.nu);
  S.sm = SM_STAGE_EVAL;
}

// ------------------------------------------------------------------ kernels

// Median of the slot's median keys (the element of rank M/2 of non-negative
// FP64 values, ordered by their bit patterns) by an 8-bit radix select.
__global__ __launch_bounds__(1024) void median_kernel(const SlotDesc* __restrict__ descs,
                                                      SlotState* __restrict__ states, int capacity,
                                                      int branch, int nbranch) {
  const int slot = (int)blockIdx.x * nbranch + branch;
  if (slot >= capacity) return;
  SlotState& S = states[slot];
  if (S.status != ST_RUNNING || !S.want_median) return;
  const SlotDesc& D = descs[slot];
  const int t = threadIdx.x;
  __shared__ unsigned hist[256];
  __shared__ unsigned s_inc[256];
  __shared__ unsigned long long s_prefix, s_mask;
  __shared__ long long s_k;
  if (t == 0) {
    s_prefix = 0ull;
    s_mask = 0ull;
    s_k = D.M / 2;
  }
  __syncthreads();
  for (int shift = 56; shift >= 0; shift -= 8) {
    if (t < 256) hist[t] = 0u;
    __syncthreads();
    const unsigned long long pre = s_prefix, msk = s_mask;
    const long long k = s_k;
    // eight keys per thread in flight at once
    for (int i0 = t; i0 < D.M; i0 += 8 * 1024) {
      unsigned long long key[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = i0 + 1024 * u;
        key[u] = i < D.M ? (unsigned long long)__double_as_longlong(ldg(D.medkey, i)) : 0ull;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (i0 + 1024 * u < D.M && (key[u] & msk) == pre) atomicAdd(&hist[(key[u] >> shift) & 255ull], 1u);
    }
    __syncthreads();
    // the digit holding rank k: inclusive prefix counts over the 256 digits
    if (t < 256) s_inc[t] = hist[t];
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
      const unsigned v = (t < 256 && t >= o) ? s_inc[t - o] : 0u;
      __syncthreads();
      if (t < 256) s_inc[t] += v;
      __syncthreads();
    }
    if (t < 256) {
      const long long lo = t > 0 ? (long long)s_inc[t - 1] : 0ll, hi = (long long)s_inc[t];
      if (lo <= k && k < hi) {
        s_k = k - lo;
        s_prefix = pre | ((unsigned long long)t << shift);
        s_mask = msk | (255ull << shift);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) S.median = __longlong_as_double((long long)s_prefix);
}

// Work list of the next pass for the one-slot engine (written by the solver
// and by the boot kernel, so that no planning kernels run between passes).
__device__ void plan_single(const SlotDesc& D, const SlotState& S, WorkList* wl, int slot) {
  const bool run = S.status == ST_RUNNING;
  const int nn = (run && !S.reuse && S.cull) ? D.ntile : 0;
  if (nn) {
    D.scount[0] = 0;
    D.scount[1] = 0;
  }
  wl->single = 1;
  wl->n_active = run ? 1 : 0;
  wl->slot[0] = slot;
  wl->nn_total = nn;
  wl->nn_base[0] = 0;
  wl->nn_base[1] = nn;
  const int ep = run ? D.nepi : 0;
  wl->epi_total = ep;
  wl->epi_base[0] = 0;
  wl->epi_base[1] = ep;
  wl->s_from_scount = (run && !S.reuse) ? 1 : 0;
  wl->s_total = 0;
  wl->s_base[0] = 0;
  wl->s_base[1] = 0;
  for (int q = 0; q < kQueues; ++q) {
    wl->q_nn[q * kQueueStride] = 0;
    wl->q_epi[q * kQueueStride] = 0;
  }
  for (int q = 0; q < kSliceQueues; ++q) wl->q_s[q * kQueueStride] = 0;
}

// Sum of the per-item partial moments in a fixed order: lane l adds items
// l, l + 64, ... in turn, then the wavefront sums the lanes by recursive
// halving (wave_sum32); every lane receives the totals. The value count is a
// template parameter so that the accumulators stay in registers.
template <int NV>
__device__ __forceinline__ void merge_partials(const SlotDesc& D, double* acc) {
  const int lane = threadIdx.x;
  double a[32];
#pragma unroll
  for (int v = 0; v < 32; ++v) a[v] = 0.0;
  // four items' loads in flight per lane; the sums stay in item order
#pragma unroll 4
  for (int e = lane; e < D.nepi; e += 64) {
    const double* p = D.part + (size_t)e * kPartStride;
#pragma unroll
    for (int v = 0; v < NV; ++v) a[v] += ldg(p, v);
  }
  const double t = wave_sum32(a);
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = readlane_f64(t, 2 * v);
#pragma unroll
  for (int v = NV; v < kP2PLVals; ++v) acc[v] = 0.0;
}

__device__ void solver_step(const SlotDesc& D, SlotState& S, const double* acc);

// One solver step of a slot, run by one wavefront (threads 0..63 of its
// block). The state machine runs on an LDS copy of the slot state: its many
// dependent reads and writes then cost LDS latency instead of a memory round
// trip each. The wavefront copies it in and out cooperatively. The state
// words (status included) and, for the one-slot engine, whose slot stays
// admitted for the whole replay, the partial moments are loaded in the same
// round trip.
__device__ __forceinline__ void solver_run(const SlotDesc* __restrict__ descs,
                                           SlotState* __restrict__ states,
                           int* __restrict__ done, WorkList* __restrict__ wl, int slot,
                           int single) {
  static_assert(sizeof(SlotState) % 8 == 0, "slot state is copied in 8-byte words");
  constexpr int kWords = (int)(sizeof(SlotState) / 8);
  constexpr int kPer = (kWords + 63) / 64;
  __shared__ unsigned long long s_state[kWords];
  const int lane = threadIdx.x;
  const unsigned long long* src = reinterpret_cast<const unsigned long long*>(states + slot);
  unsigned long long w[kPer];
#pragma unroll
  for (int t = 0; t < kPer; ++t) {
    const int i = lane + 64 * t;
    w[t] = ldg(src, i < kWords ? i : 0);
  }
  const SlotDesc& D = descs[slot];
  const bool plane = mode_plane(D.mode);
  double acc[kP2PLVals];
  if (single) {
    if (plane) merge_partials<kP2PLVals>(D, acc);
    else merge_partials<kP2PVals>(D, acc);
  }
#pragma unroll
  for (int t = 0; t < kPer; ++t) {
    const int i = lane + 64 * t;
    if (i < kWords) s_state[i] = w[t];
  }
  wave_lds_sync();
  SlotState& S = *reinterpret_cast<SlotState*>(s_state);
  if (S.status != ST_RUNNING) return;
  if (!single) {
    if (plane) merge_partials<kP2PLVals>(D, acc);
    else merge_partials<kP2PVals>(D, acc);
  }
  if (lane == 0) solver_step(D, S, acc);
  wave_lds_sync();
  {
    unsigned long long* dst = reinterpret_cast<unsigned long long*>(states + slot);
    for (int i = lane; i < kWords; i += 64) dst[i] = s_state[i];
  }
  if (lane == 0 && S.status == ST_DONE) done[slot] = 1;
  if (lane == 0 && single) plan_single(D, S, wl, slot);
}

__global__ __launch_bounds__(64) void solver_kernel(const SlotDesc* __restrict__ descs,
                                                    SlotState* __restrict__ states, int capacity,
                                                    int* __restrict__ done, WorkList* __restrict__ wl,
                                                    int single, int branch, int nbranch) {
  const int slot = (int)blockIdx.x * nbranch + branch;
  if (slot >= capacity) return;
  solver_run(descs, states, done, wl, slot, single);
}

// One pass of the state machine for a slot (lane 0 of the solver wavefront).
__device__ void solver_step(const SlotDesc& D, SlotState& S, const double* acc) {
  S.phases++;
  double* prop = nullptr;  // the trace row's un-accelerated update, written by the step
  if (D.trace && S.trace_len < D.trace_cap) {
    double* row = D.trace + (size_t)S.trace_len * kTraceRow;
    row[0] = acc[0];
    row[1] = S.nu_eval;
    row[2] = S.sm;
    row[3] = S.reuse;
    for (int i = 0; i < 16; ++i) row[4 + i] = S.Teval[i];
    prop = row + 20;
    for (int i = 0; i < 16; ++i) prop[i] = 0.0;
    S.trace_len++;
  }
  if (S.sm == SM_QUERY) {
    S.status = ST_DONE;
  } else if (S.sm == SM_EVAL) {
    // energy at the requested transform and the MM update from it
    double T[16];
    unsigned f;
    if (mode_plane(D.mode)) {
      double xp[6];
      f = gn_p2pl(acc, S.last_key, xp);
      twist_exp(xp, T);
    } else {
      f = align_p2p(acc, S.cP, S.cQ, S.Vq, T);
    }
    S.flags = f;
    S.nu = S.nu_eval;
    finish(S, T, acc[0]);
  } else if (mode_plane(D.mode)) {
    step_p2pl(S, acc, prop);
  } else {
    step_p2p(S, acc, prop);
  }
}

// First request of a freshly admitted slot: evaluation at T0 (point-to-plane:
// at exp(log T0)), then the slot becomes RUNNING.
__global__ void boot_kernel(const SlotDesc* __restrict__ descs, SlotState* __restrict__ states,
                            int slot, WorkList* __restrict__ wl, int single) {
  if (threadIdx.x != 0) return;
  SlotState& S = states[slot];
  S.verlet = descs[slot].method == NN_CLUSTER ? (double)descs[slot].verlet : 0.0;
  S.evaluations = 0;
  S.nn_passes = 0;
  S.have_last = 0;
  if (S.sm == SM_QUERY) {
    request_T(S, S.Tkm1, 1.0);
  } else if (S.sm == SM_EVAL) {
    if (mode_plane(S.mode)) {
      twist_log(S.Tkm1, S.xkm1);
      request_xi(S, S.xkm1, S.nu_max);
    } else {
      request_T(S, S.Tkm1, S.nu_max);
    }
  } else if (mode_plane(S.mode)) {
    twist_log(S.Tkm1, S.xkm1);
    request_xi(S, S.xkm1, S.nu_auto ? 1.0 : S.nu_max);
  } else {
    request_T(S, S.Tkm1, (S.mode == P2P_L2 || S.nu_auto) ? 1.0 : S.nu_max);
  }
  S.status = ST_RUNNING;
  if (single) plan_single(descs[slot], S, wl, slot);
}

// Exact median (element of rank floor(M/2)) of the non-negative FP64 keys of
// one slot by 8-bit radix selection on the bit patterns.

// The slots of branch b of nbranch are b, b + nbranch, ... (one branch: all).
void launch_solver(const SlotDesc* descs, SlotState* states, int capacity, int* done,
                   WorkList* wl, bool single, hipStream_t st, int branch, int nbranch) {
  const int grid = (capacity - branch + nbranch - 1) / nbranch;
  if (grid <= 0) return;
  hipLaunchKernelGGL(solver_kernel, dim3(grid), dim3(64), 0, st, descs, states, capacity, done,
                     wl, single ? 1 : 0, branch, nbranch);
}

void launch_median(const SlotDesc* descs, SlotState* states, int capacity, hipStream_t st,
                   int branch, int nbranch) {
  const int grid = (capacity - branch + nbranch - 1) / nbranch;
  if (grid <= 0) return;
  hipLaunchKernelGGL(median_kernel, dim3(grid), dim3(1024), 0, st, descs, states, capacity, branch,
                     nbranch);
}

void launch_boot(const SlotDesc* descs, SlotState* states, int slot, WorkList* wl, bool single,
                 hipStream_t st) {
  hipLaunchKernelGGL(boot_kernel, dim3(1), dim3(64), 0, st, descs, states, slot, wl, single ? 1 : 0);
}

}  // namespace icp
