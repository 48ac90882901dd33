/*
 * Oracle for Fast and Robust ICP (Zhang, Yao, Deng, arXiv 2007.07627).
 *
 * TEST INFRASTRUCTURE ONLY: plain, slow FP64 C that the GPU path is checked
 * against. Only the tests, the smoke check and the benchmark's CPU-baseline
 * leg may load it; the product path never does. It shares no code with the
 * GPU library.
 *
 * Build: gcc -O2 -std=c11 -fPIC -shared -fopenmp -mfma -ffp-contract=off
 *        (no fast-math; fma/fmaf are called explicitly where a fused operation
 *        is part of a definition).
 *
 * Readings of the paper used here (where it is silent, ambiguous or garbled):
 *   R1  Anderson residual: F^(k) = G(x^(k)) - x^(k) as Algorithm 1 uses it (the
 *       text of Sec. 4.1 also writes F^(k) = G(x^(k))).
 *   R2  The Anderson sums run over the m_k columns of the least-squares problem.
 *   R3  Algorithm 2 takes no exponential of the accelerated se(3) vector: it is
 *       already the parameter vector.
 *   R4  Stage convergence: ||T^(k) - T'||_F < eps (not squared) for point-to-
 *       point; ||xi*^(k+1) - xi^(k)||_2 < eps for point-to-plane.
 *   R5  Least-squares metric: Frobenius norm of the 4x4 logarithm (rotation
 *       part counted twice) for point-to-point, Euclidean for point-to-plane.
 *   R6  Gauss-Newton right-hand side (eq. GNSystem): the solution that
 *       minimises the linearised objective is xi* = xi^(k) - A^{-1} sum g B J;
 *       the printed sign would increase it.
 *   R7  Line search: tau halves and l grows after each trial; l_max = 10; the
 *       lowest-energy trial is kept.
 *   R8  App. D: the term -(2/|d|^4) M d^T d is the outer product (M d) d^T.
 *   R9  App. D at delta = 0: exact small-angle series (dt/ddelta = -u^/2).
 *   R10 App. A eq. calc_V holds with the unit generator; V^-1 below is the
 *       standard closed form.
 *   R11 Median of n values: the element of rank floor(n/2) in ascending order.
 *   R12 Nearest-neighbour ties: lowest target index.
 *   R13 Zero total weight (all Welsch weights underflow) or a singular 6x6
 *       system: no update, the current transform is returned with a flag.
 *   R14 A safeguard rejection does not reset the Anderson history.
 *   R15 Residuals, weights and energies are evaluated in FP64 from the FP64
 *       transform; only the closest-point search uses the FP32 transform.
 */
#include "oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Small dense helpers (FP64)                                                */
/* ------------------------------------------------------------------------ */

static void m3_mul(const double A[9], const double B[9], double C[9]) {
  double t[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      t[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
  memcpy(C, t, sizeof t);
}

static void m3_transpose(const double A[9], double B[9]) {
  double t[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) t[3 * j + i] = A[3 * i + j];
  memcpy(B, t, sizeof t);
}

static double m3_det(const double A[9]) {
  return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
         A[2] * (A[3] * A[7] - A[4] * A[6]);
}

/* a^ : the skew matrix with a^ b = a x b (App. D). */
static void hat3(const double a[3], double A[9]) {
  A[0] = 0;     A[1] = -a[2]; A[2] = a[1];
  A[3] = a[2];  A[4] = 0;     A[5] = -a[0];
  A[6] = -a[1]; A[7] = a[0];  A[8] = 0;
}

static void cross3(const double a[3], const double b[3], double c[3]) {
  double t0 = a[1] * b[2] - a[2] * b[1];
  double t1 = a[2] * b[0] - a[0] * b[2];
  double t2 = a[0] * b[1] - a[1] * b[0];
  c[0] = t0; c[1] = t1; c[2] = t2;
}

static void m3_vec(const double A[9], const double x[3], double y[3]) {
  double t[3];
  for (int i = 0; i < 3; ++i) t[i] = A[3 * i] * x[0] + A[3 * i + 1] * x[1] + A[3 * i + 2] * x[2];
  y[0] = t[0]; y[1] = t[1]; y[2] = t[2];
}

static void T_to_Rt(const double T[16], double R[9], double t[3]) {
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) R[3 * i + j] = T[4 * i + j];
    t[i] = T[4 * i + 3];
  }
}

static void Rt_to_T(const double R[9], const double t[3], double T[16]) {
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) T[4 * i + j] = R[3 * i + j];
    T[4 * i + 3] = t[i];
  }
  T[12] = 0; T[13] = 0; T[14] = 0; T[15] = 1;
}

/* ------------------------------------------------------------------------ */
/* Correspondence step, eq. CorresponcePoint (Sec. 3).                        */
/* ------------------------------------------------------------------------ */

/* The transformed point is evaluated in FP64 with one fixed fused order,
 * x_a = fma(R_a2, p_z, fma(R_a1, p_y, fma(R_a0, p_x, t_a))), and rounded to
 * FP32 once; the search then runs on FP32 coordinates. */
static void xform_f64(const double T[16], const float p[3], double x[3]) {
  for (int a = 0; a < 3; ++a)
    x[a] = fma(T[4 * a + 2], (double)p[2],
               fma(T[4 * a + 1], (double)p[1], fma(T[4 * a + 0], (double)p[0], T[4 * a + 3])));
}

void orc_transform_f32(const double T[16], const float *P, int64_t M, float *out) {
  for (int64_t i = 0; i < M; ++i) {
    double x[3];
    xform_f64(T, P + 3 * i, x);
    out[3 * i] = (float)x[0];
    out[3 * i + 1] = (float)x[1];
    out[3 * i + 2] = (float)x[2];
  }
}

/* Closest point by exhaustive scan: d^2 = fmaf(dz,dz, fmaf(dy,dy, dx*dx)) with
 * FP32 differences; the first (lowest) index attaining the minimum wins. */
void orc_nn_brute(const float *Pt, int64_t M, const float *Q, int64_t N, int32_t *idx,
                  float *d2) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < M; ++i) {
    const float px = Pt[3 * i], py = Pt[3 * i + 1], pz = Pt[3 * i + 2];
    float best = 0.0f;
    int64_t bi = 0;
    for (int64_t j = 0; j < N; ++j) {
      const float dx = px - Q[3 * j], dy = py - Q[3 * j + 1], dz = pz - Q[3 * j + 2];
      const float d = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
      if (j == 0 || d < best) {
        best = d;
        bi = j;
      }
    }
    idx[i] = (int32_t)bi;
    d2[i] = best;
  }
}

void orc_nn_query(const float *P, int64_t M, const float *Q, int64_t N, const double T[16],
                  int32_t *idx, float *d2) {
  float *Pt = (float *)malloc(sizeof(float) * 3 * (size_t)(M > 0 ? M : 1));
  orc_transform_f32(T, P, M, Pt);
  orc_nn_brute(Pt, M, Q, N, idx, d2);
  free(Pt);
}

/* ------------------------------------------------------------------------ */
/* se(3) exponential and logarithm (eq. MatrixExp; Appendix A).               */
/* ------------------------------------------------------------------------ */

/* Coefficients of Rodrigues' formula: A = sin t / t, B = (1 - cos t)/t^2,
 * C = (t - sin t)/t^3, with Taylor series for small t. */
static void rodrigues_coeffs(double th, double *A, double *B, double *C) {
  const double t2 = th * th;
  if (th < 0.1) {
    *A = 1.0 - t2 / 6.0 * (1.0 - t2 / 20.0 * (1.0 - t2 / 42.0 * (1.0 - t2 / 72.0)));
    *B = 0.5 * (1.0 - t2 / 12.0 * (1.0 - t2 / 30.0 * (1.0 - t2 / 56.0 * (1.0 - t2 / 90.0))));
    *C = (1.0 - t2 / 20.0 * (1.0 - t2 / 42.0 * (1.0 - t2 / 72.0 * (1.0 - t2 / 110.0)))) / 6.0;
  } else {
    const double h = sin(0.5 * th);
    *A = sin(th) / th;
    *B = 2.0 * h * h / t2;
    *C = (th - sin(th)) / (t2 * th);
  }
}

/* T = exp([delta^ u; 0 0]): R = I + A W + B W^2, t = (I + B W + C W^2) u. */
void orc_se3_exp(const double xi[6], double T[16]) {
  const double *d = xi, *u = xi + 3;
  const double th = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  double A, B, C, W[9], W2[9], R[9], V[9], t[3];
  rodrigues_coeffs(th, &A, &B, &C);
  hat3(d, W);
  m3_mul(W, W, W2);
  for (int i = 0; i < 9; ++i) {
    const double I = (i % 4 == 0) ? 1.0 : 0.0;
    R[i] = I + A * W[i] + B * W2[i];
    V[i] = I + B * W[i] + C * W2[i];
  }
  m3_vec(V, u, t);
  Rt_to_T(R, t, T);
}

/* Principal logarithm. For d = 3 the real Schur form of Appendix A has one
 * 2x2 rotation block of angle theta in [0, pi]; the plane of that block is
 * the one orthogonal to the rotation axis, so log(R) = theta * axis^ and the
 * translation part is V^{-1} t with
 * V^{-1} = I - W/2 + (1/th^2)(1 - th sin th / (2 (1 - cos th))) W^2. */
void orc_se3_log(const double T[16], double xi[6]) {
  double R[9], t[3];
  T_to_Rt(T, R, t);
  const double tr = R[0] + R[4] + R[8];
  double v[3] = {R[7] - R[5], R[2] - R[6], R[3] - R[1]}; /* vee(R - R^T) */
  const double s = 0.5 * sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  double c = 0.5 * (tr - 1.0);
  if (c > 1.0) c = 1.0;
  if (c < -1.0) c = -1.0;
  const double th = atan2(s, c);
  double d[3];
  if (th < 1e-3) {
    /* theta / (2 sin theta) = 1/2 + theta^2/12 + 7 theta^4/720 */
    const double f = 0.5 + th * th / 12.0 + 7.0 * th * th * th * th / 720.0;
    d[0] = f * v[0]; d[1] = f * v[1]; d[2] = f * v[2];
  } else if (th < 3.14159265358979323846 - 1e-3) {
    const double f = th / (2.0 * sin(th));
    d[0] = f * v[0]; d[1] = f * v[1]; d[2] = f * v[2];
  } else {
    /* Near pi: axis from the symmetric part (R + R^T)/2 = cos th I + (1 - cos th) a a^T. */
    double S[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) S[3 * i + j] = 0.5 * (R[3 * i + j] + R[3 * j + i]) - (i == j ? c : 0.0);
    int k = 0;
    if (S[4] > S[0]) k = 1;
    if (S[8] > S[3 * k + k]) k = 2;
    double a[3] = {S[3 * k], S[3 * k + 1], S[3 * k + 2]};
    double na = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    a[0] /= na; a[1] /= na; a[2] /= na;
    const double sg = a[0] * v[0] + a[1] * v[1] + a[2] * v[2];
    if (sg < 0.0 || (sg == 0.0 && a[k] < 0.0)) { a[0] = -a[0]; a[1] = -a[1]; a[2] = -a[2]; }
    d[0] = th * a[0]; d[1] = th * a[1]; d[2] = th * a[2];
  }
  double W[9], W2[9], Vi[9];
  hat3(d, W);
  m3_mul(W, W, W2);
  double g;
  if (th < 0.1) {
    const double t2 = th * th;
    g = 1.0 / 12.0 + t2 / 720.0 + t2 * t2 / 30240.0 + t2 * t2 * t2 / 1209600.0;
  } else {
    g = (1.0 - th * sin(th) / (2.0 * (1.0 - cos(th)))) / (th * th);
  }
  for (int i = 0; i < 9; ++i) Vi[i] = ((i % 4 == 0) ? 1.0 : 0.0) - 0.5 * W[i] + g * W2[i];
  double u[3];
  m3_vec(Vi, t, u);
  xi[0] = d[0]; xi[1] = d[1]; xi[2] = d[2];
  xi[3] = u[0]; xi[4] = u[1]; xi[5] = u[2];
}

/* ------------------------------------------------------------------------ */
/* 3x3 SVD by one-sided Jacobi rotations (used by the alignment step).        */
/* ------------------------------------------------------------------------ */

int orc_svd3(const double A[9], double U[9], double S[3], double V[9]) {
  double W[9];
  memcpy(W, A, sizeof W);
  for (int i = 0; i < 9; ++i) V[i] = (i % 4 == 0) ? 1.0 : 0.0;
  static const int PQ[3][2] = {{0, 1}, {0, 2}, {1, 2}};
  for (int sweep = 0; sweep < 64; ++sweep) {
    int rotated = 0;
    for (int r = 0; r < 3; ++r) {
      const int p = PQ[r][0], q = PQ[r][1];
      double al = 0, be = 0, ga = 0;
      for (int i = 0; i < 3; ++i) {
        al += W[3 * i + p] * W[3 * i + p];
        be += W[3 * i + q] * W[3 * i + q];
        ga += W[3 * i + p] * W[3 * i + q];
      }
      if (ga == 0.0 || fabs(ga) <= 1e-17 * sqrt(al * be)) continue;
      rotated = 1;
      const double zeta = (be - al) / (2.0 * ga);
      const double tt = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
      const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
      for (int i = 0; i < 3; ++i) {
        const double wp = W[3 * i + p], wq = W[3 * i + q];
        W[3 * i + p] = cs * wp - sn * wq;
        W[3 * i + q] = sn * wp + cs * wq;
        const double vp = V[3 * i + p], vq = V[3 * i + q];
        V[3 * i + p] = cs * vp - sn * vq;
        V[3 * i + q] = sn * vp + cs * vq;
      }
    }
    if (!rotated) break;
  }
  /* Singular values are the column norms; sort descending. */
  double sv[3];
  for (int j = 0; j < 3; ++j)
    sv[j] = sqrt(W[j] * W[j] + W[3 + j] * W[3 + j] + W[6 + j] * W[6 + j]);
  int ord[3] = {0, 1, 2};
  for (int a = 0; a < 3; ++a)
    for (int b = a + 1; b < 3; ++b)
      if (sv[ord[b]] > sv[ord[a]]) { int tmp = ord[a]; ord[a] = ord[b]; ord[b] = tmp; }
  double Vs[9], Ws[9];
  for (int j = 0; j < 3; ++j) {
    S[j] = sv[ord[j]];
    for (int i = 0; i < 3; ++i) {
      Vs[3 * i + j] = V[3 * i + ord[j]];
      Ws[3 * i + j] = W[3 * i + ord[j]];
    }
  }
  memcpy(V, Vs, sizeof Vs);
  /* U columns: normalised W columns; complete an orthonormal basis where a
   * singular value vanishes. */
  const double tiny = 1e-300;
  double u0[3], u1[3], u2[3];
  if (S[0] > tiny) {
    for (int i = 0; i < 3; ++i) u0[i] = Ws[3 * i] / S[0];
  } else {
    u0[0] = 1; u0[1] = 0; u0[2] = 0;
  }
  if (S[1] > 1e-14 * S[0] && S[1] > tiny) {
    for (int i = 0; i < 3; ++i) u1[i] = Ws[3 * i + 1] / S[1];
  } else {
    /* any unit vector orthogonal to u0 */
    double e[3] = {0, 0, 0};
    int k = (fabs(u0[0]) <= fabs(u0[1]) && fabs(u0[0]) <= fabs(u0[2])) ? 0 : (fabs(u0[1]) <= fabs(u0[2]) ? 1 : 2);
    e[k] = 1.0;
    cross3(u0, e, u1);
    double n = sqrt(u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2]);
    u1[0] /= n; u1[1] /= n; u1[2] /= n;
  }
  if (S[2] > 1e-14 * S[0] && S[2] > tiny) {
    for (int i = 0; i < 3; ++i) u2[i] = Ws[3 * i + 2] / S[2];
  } else {
    cross3(u0, u1, u2);
  }
  for (int i = 0; i < 3; ++i) {
    U[3 * i] = u0[i];
    U[3 * i + 1] = u1[i];
    U[3 * i + 2] = u2[i];
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Alignment step: weighted SVD Procrustes (eq. Alignment, eq. WelschAlignment)*/
/* ------------------------------------------------------------------------ */

/* argmin_{R,t} sum_i w_i |R p_i + t - q_i|^2 over rotations: with weighted
 * centroids pb, qb and H = sum_i w_i (p_i - pb)(q_i - qb)^T = U S V^T,
 * R = V diag(1, 1, sign det(V U^T)) U^T and t = qb - R pb. */
unsigned orc_procrustes(const float *P, const float *Qh, const double *w, int64_t M,
                        double T[16]) {
  double W = 0, pb[3] = {0, 0, 0}, qb[3] = {0, 0, 0};
  for (int64_t i = 0; i < M; ++i) {
    const double wi = w ? w[i] : 1.0;
    W += wi;
    for (int a = 0; a < 3; ++a) {
      pb[a] += wi * (double)P[3 * i + a];
      qb[a] += wi * (double)Qh[3 * i + a];
    }
  }
  if (!(W > 1e-300)) return ORC_FLAG_ZERO_WEIGHT;
  for (int a = 0; a < 3; ++a) { pb[a] /= W; qb[a] /= W; }
  double H[9] = {0};
  for (int64_t i = 0; i < M; ++i) {
    const double wi = w ? w[i] : 1.0;
    double dp[3], dq[3];
    for (int a = 0; a < 3; ++a) {
      dp[a] = (double)P[3 * i + a] - pb[a];
      dq[a] = (double)Qh[3 * i + a] - qb[a];
    }
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) H[3 * a + b] += wi * dp[a] * dq[b];
  }
  double U[9], S[3], V[9], Ut[9], R[9], t[3];
  unsigned flags = 0;
  orc_svd3(H, U, S, V);
  if (!(S[1] > 1e-12 * S[0])) flags |= ORC_FLAG_DEGENERATE;
  m3_transpose(U, Ut);
  double VUt[9];
  m3_mul(V, Ut, VUt);
  const double sg = m3_det(VUt) < 0 ? -1.0 : 1.0;
  double VS[9];
  memcpy(VS, V, sizeof VS);
  for (int i = 0; i < 3; ++i) VS[3 * i + 2] *= sg;
  m3_mul(VS, Ut, R);
  double Rp[3];
  m3_vec(R, pb, Rp);
  for (int a = 0; a < 3; ++a) t[a] = qb[a] - Rp[a];
  Rt_to_T(R, t, T);
  return flags;
}

/* ------------------------------------------------------------------------ */
/* Point-to-plane residual and gradient (eq. LieAlgebraPointToPlaneAlignment, */
/* eq. Linearization, Appendix D).                                           */
/* ------------------------------------------------------------------------ */

double orc_plane_residual(const double xi[6], const float p[3], const float q[3],
                          const float n[3]) {
  double T[16], x[3];
  orc_se3_exp(xi, T);
  xform_f64(T, p, x);
  const double dx = x[0] - (double)q[0], dy = x[1] - (double)q[1], dz = x[2] - (double)q[2];
  return fma(dz, (double)n[2], fma(dy, (double)n[1], dx * (double)n[0]));
}

/* Derivatives of R(delta) and t(delta, u) = V(delta) u with respect to the
 * parameters. For |delta| >= 1e-3 the formulas of Appendix D are used as
 * printed (with reading R8); below, the exact small-angle series (R9) of the
 * same derivatives. dR[j] = dR/d delta_j (3x3), Dt = dt/d delta (3x3, column
 * j = dt/d delta_j), Du = dt/du (3x3). */
static void se3_derivs(const double xi[6], double dR[3][9], double Dt[9], double Du[9]) {
  const double *d = xi, *u = xi + 3;
  const double th2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  const double th = sqrt(th2);
  double T[16], R[9], t[3];
  orc_se3_exp(xi, T);
  T_to_Rt(T, R, t);
  double W[9], Uh[9];
  hat3(d, W);
  hat3(u, Uh);
  if (th >= 1e-3) {
    /* dR/d delta_j = (delta_j delta^ + (delta x (I - R) e_j)^) R / |delta|^2 */
    for (int j = 0; j < 3; ++j) {
      double col[3] = {-R[j], -R[3 + j], -R[6 + j]};
      col[j] += 1.0;
      double cr[3], Cx[9], Mj[9];
      cross3(d, col, cr);
      hat3(cr, Cx);
      for (int i = 0; i < 9; ++i) Mj[i] = (d[j] * W[i] + Cx[i]) / th2;
      m3_mul(Mj, R, dR[j]);
    }
    /* M = (R - I) u^ + (delta . u) I;  t = M delta / |delta|^2 */
    double RmI[9], Mm[9];
    for (int i = 0; i < 9; ++i) RmI[i] = R[i] - ((i % 4 == 0) ? 1.0 : 0.0);
    m3_mul(RmI, Uh, Mm);
    const double du = d[0] * u[0] + d[1] * u[1] + d[2] * u[2];
    Mm[0] += du; Mm[4] += du; Mm[8] += du;
    double Md[3];
    m3_vec(Mm, d, Md);
    /* D_j = dR_j u^ delta */
    double ud[3];
    cross3(u, d, ud);
    for (int j = 0; j < 3; ++j) {
      double Dj[3];
      m3_vec(dR[j], ud, Dj);
      for (int i = 0; i < 3; ++i)
        Dt[3 * i + j] = (Mm[3 * i + j] + d[i] * u[j] + Dj[i]) / th2 -
                        2.0 / (th2 * th2) * Md[i] * d[j];
    }
    /* dt/du = ((I - R) delta^ + delta delta^T) / |delta|^2 */
    double ImR[9], ImRW[9];
    for (int i = 0; i < 9; ++i) ImR[i] = -RmI[i];
    m3_mul(ImR, W, ImRW);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Du[3 * i + j] = (ImRW[3 * i + j] + d[i] * d[j]) / th2;
  } else {
    /* R = I + A W + B W^2, V = I + B W + C W^2 with the series of A, B, C and
     * of their derivatives divided by theta (dA/dth / th etc.). */
    const double A = 1.0 - th2 / 6.0 + th2 * th2 / 120.0;
    const double B = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
    const double C = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0;
    const double Ad = -1.0 / 3.0 + th2 / 30.0 - th2 * th2 / 840.0;
    const double Bd = -1.0 / 12.0 + th2 / 180.0 - th2 * th2 / 6720.0;
    const double Cd = -1.0 / 60.0 + th2 / 1260.0 - th2 * th2 / 60480.0;
    double W2[9];
    m3_mul(W, W, W2);
    for (int j = 0; j < 3; ++j) {
      double e[3] = {0, 0, 0}, Ej[9], EW[9], WE[9];
      e[j] = 1.0;
      hat3(e, Ej);
      m3_mul(Ej, W, EW);
      m3_mul(W, Ej, WE);
      for (int i = 0; i < 9; ++i)
        dR[j][i] = A * Ej[i] + B * (EW[i] + WE[i]) + Ad * d[j] * W[i] + Bd * d[j] * W2[i];
      /* dt/d delta_j = B E_j u + C (E_j W + W E_j) u + Bd d_j W u + Cd d_j W^2 u */
      double a1[3], a2[3], a3[3], a4[3], tmp[9];
      m3_vec(Ej, u, a1);
      for (int i = 0; i < 9; ++i) tmp[i] = EW[i] + WE[i];
      m3_vec(tmp, u, a2);
      m3_vec(W, u, a3);
      m3_vec(W2, u, a4);
      for (int i = 0; i < 3; ++i)
        Dt[3 * i + j] = B * a1[i] + C * a2[i] + Bd * d[j] * a3[i] + Cd * d[j] * a4[i];
    }
    for (int i = 0; i < 9; ++i) Du[i] = ((i % 4 == 0) ? 1.0 : 0.0) + B * W[i] + C * W2[i];
  }
}

/* J = [n^T dR_j p + n^T Dt[:, j]]_j ; [Du^T n] */
static void plane_gradient_from(const double dR[3][9], const double Dt[9], const double Du[9],
                                const float p[3], const float n[3], double J[6]) {
  const double pd[3] = {p[0], p[1], p[2]}, nd[3] = {n[0], n[1], n[2]};
  for (int j = 0; j < 3; ++j) {
    double v[3];
    m3_vec(dR[j], pd, v);
    J[j] = nd[0] * (v[0] + Dt[j]) + nd[1] * (v[1] + Dt[3 + j]) + nd[2] * (v[2] + Dt[6 + j]);
    J[3 + j] = Du[j] * nd[0] + Du[3 + j] * nd[1] + Du[6 + j] * nd[2];
  }
}

void orc_plane_gradient(const double xi[6], const float p[3], const float n[3], double J[6]) {
  double dR[3][9], Dt[9], Du[9];
  se3_derivs(xi, dR, Dt, Du);
  plane_gradient_from(dR, Dt, Du, p, n, J);
}

/* ------------------------------------------------------------------------ */
/* Anderson acceleration least squares (Sec. 4.1, Algorithms 1 and 2).        */
/* ------------------------------------------------------------------------ */

static double aa_dot(const double *a, const double *b, int metric) {
  const double wr = metric == 0 ? 2.0 : 1.0;
  return wr * (a[0] * b[0] + a[1] * b[1] + a[2] * b[2]) + a[3] * b[3] + a[4] * b[4] + a[5] * b[5];
}

/* Normal equations N theta = r, N_ij = <dF_i, dF_j>, r_i = <dF_i, F^k>, by
 * Cholesky; a pivot at or below 1e-10 x max diag is treated as singular. */
int orc_anderson_solve(const double *dF, const double *Fk, int m, int metric, double *theta) {
  double N[36], r[6], L[36];
  double dmax = 0;
  for (int i = 0; i < m; ++i) {
    r[i] = aa_dot(dF + 6 * i, Fk, metric);
    for (int j = 0; j < m; ++j) N[6 * i + j] = aa_dot(dF + 6 * i, dF + 6 * j, metric);
    if (N[6 * i + i] > dmax) dmax = N[6 * i + i];
  }
  memset(L, 0, sizeof L);
  int singular = !(dmax > 0);
  for (int j = 0; j < m && !singular; ++j) {
    double s = N[6 * j + j];
    for (int k = 0; k < j; ++k) s -= L[6 * j + k] * L[6 * j + k];
    if (!(s > 1e-10 * dmax)) { singular = 1; break; }
    L[6 * j + j] = sqrt(s);
    for (int i = j + 1; i < m; ++i) {
      double v = N[6 * i + j];
      for (int k = 0; k < j; ++k) v -= L[6 * i + k] * L[6 * j + k];
      L[6 * i + j] = v / L[6 * j + j];
    }
  }
  if (singular) {
    for (int i = 0; i < m; ++i) theta[i] = 0.0;
    return 1;
  }
  double y[6];
  for (int i = 0; i < m; ++i) {
    double v = r[i];
    for (int k = 0; k < i; ++k) v -= L[6 * i + k] * y[k];
    y[i] = v / L[6 * i + i];
  }
  for (int i = m - 1; i >= 0; --i) {
    double v = y[i];
    for (int k = i + 1; k < m; ++k) v -= L[6 * k + i] * theta[k];
    theta[i] = v / L[6 * i + i];
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Median (nu_max rule, Sec. 4.3 and Sec. 5)                                  */
/* ------------------------------------------------------------------------ */

static int cmp_double(const void *a, const void *b) {
  const double x = *(const double *)a, y = *(const double *)b;
  return (x > y) - (x < y);
}

double orc_median(const double *v, int64_t n) {
  double *c = (double *)malloc(sizeof(double) * (size_t)n);
  memcpy(c, v, sizeof(double) * (size_t)n);
  qsort(c, (size_t)n, sizeof(double), cmp_double);
  const double r = c[n / 2];
  free(c);
  return r;
}

/* ------------------------------------------------------------------------ */
/* Automatic nu_min (Sec. 4.3, Sec. 5, App. C)                                */
/* ------------------------------------------------------------------------ */

/* The six nearest other targets of q_i by exhaustive scan: candidates are
 * ordered by (exact FP32 squared distance of q_i - q_j, index j). */
static void six_nearest(const float *Q, int64_t N, int64_t i, int64_t nb[6]) {
  float bd[6];
  int cnt = 0;
  const float qx = Q[3 * i], qy = Q[3 * i + 1], qz = Q[3 * i + 2];
  for (int64_t j = 0; j < N; ++j) {
    if (j == i) continue;
    const float dx = qx - Q[3 * j], dy = qy - Q[3 * j + 1], dz = qz - Q[3 * j + 2];
    const float d = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    /* scanning j upwards, a later equal distance never displaces an earlier one */
    int pos = cnt < 6 ? cnt : 6;
    while (pos > 0 && d < bd[pos - 1]) --pos;
    if (pos >= 6) continue;
    const int last = cnt < 6 ? cnt : 5;
    for (int k = last; k > pos; --k) {
      bd[k] = bd[k - 1];
      nb[k] = nb[k - 1];
    }
    bd[pos] = d;
    nb[pos] = j;
    if (cnt < 6) ++cnt;
  }
}

int orc_nu_min_auto(const float *Q, const float *Qn, int64_t N, int mode, double *nu_min,
                    double *per_point) {
  if (N < 7 || !nu_min || (mode != ORC_P2P_WELSCH && mode != ORC_P2PL_WELSCH)) return -1;
  if (mode == ORC_P2PL_WELSCH && !Qn) return -1;
  double *v = (double *)malloc(sizeof(double) * (size_t)N);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    int64_t nb[6];
    six_nearest(Q, N, i, nb);
    double e[6];
    for (int k = 0; k < 6; ++k) {
      const int64_t j = nb[k];
      if (mode == ORC_P2PL_WELSCH) {
        /* distance of q_j to the tangent plane at q_i (normal n_i as given) */
        const double dx = (double)Q[3 * j] - (double)Q[3 * i];
        const double dy = (double)Q[3 * j + 1] - (double)Q[3 * i + 1];
        const double dz = (double)Q[3 * j + 2] - (double)Q[3 * i + 2];
        e[k] = fabs(fma((double)Qn[3 * i + 2], dz, fma((double)Qn[3 * i + 1], dy, (double)Qn[3 * i] * dx)));
      } else {
        /* squared distance (the median is taken on squares, sqrt at the end) */
        const float dx = Q[3 * i] - Q[3 * j], dy = Q[3 * i + 1] - Q[3 * j + 1], dz = Q[3 * i + 2] - Q[3 * j + 2];
        e[k] = (double)fmaf(dz, dz, fmaf(dy, dy, dx * dx));
      }
    }
    v[i] = orc_median(e, 6);
  }
  const double med = orc_median(v, N);
  if (per_point) memcpy(per_point, v, sizeof(double) * (size_t)N);
  free(v);
  *nu_min = (mode == ORC_P2PL_WELSCH) ? med / 6.0 : sqrt(med) / (3.0 * sqrt(3.0));
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Normal estimation from 30 nearest neighbours                               */
/* ------------------------------------------------------------------------ */

#define ORC_NORMAL_K 30

int orc_estimate_normals(const float *Q, int64_t N, float *normals) {
  if (N < ORC_NORMAL_K || !normals) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    const float qx = Q[3 * i], qy = Q[3 * i + 1], qz = Q[3 * i + 2];
    float bd[ORC_NORMAL_K];
    int64_t nb[ORC_NORMAL_K];
    int cnt = 0;
    for (int64_t j = 0; j < N; ++j) {
      const float dx = qx - Q[3 * j], dy = qy - Q[3 * j + 1], dz = qz - Q[3 * j + 2];
      const float d = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
      int pos = cnt;
      while (pos > 0 && d < bd[pos - 1]) --pos;  /* later equal distances stay behind */
      if (pos >= ORC_NORMAL_K) continue;
      const int last = cnt < ORC_NORMAL_K ? cnt : ORC_NORMAL_K - 1;
      for (int k = last; k > pos; --k) {
        bd[k] = bd[k - 1];
        nb[k] = nb[k - 1];
      }
      bd[pos] = d;
      nb[pos] = j;
      if (cnt < ORC_NORMAL_K) ++cnt;
    }
    double m[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < ORC_NORMAL_K; ++k)
      for (int a = 0; a < 3; ++a) m[a] += (double)Q[3 * nb[k] + a];
    for (int a = 0; a < 3; ++a) m[a] /= ORC_NORMAL_K;
    double C[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = 0; k < ORC_NORMAL_K; ++k) {
      double e[3];
      for (int a = 0; a < 3; ++a) e[a] = (double)Q[3 * nb[k] + a] - m[a];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) C[3 * a + b] += e[a] * e[b];
    }
    for (int a = 0; a < 9; ++a) C[a] /= ORC_NORMAL_K;
    /* symmetric PSD: the SVD is the eigen-decomposition, singular values descending */
    double U[9], S[3], V[9];
    orc_svd3(C, U, S, V);
    double n[3] = {V[2], V[5], V[8]};
    const double l = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    for (int a = 0; a < 3; ++a) n[a] /= l;
    if (n[0] * qx + n[1] * qy + n[2] * qz > 0.0)
      for (int a = 0; a < 3; ++a) n[a] = -n[a];
    for (int a = 0; a < 3; ++a) normals[3 * i + a] = (float)n[a];
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Registration (Algorithm 1 with L2 or Welsch metric; Algorithm 2)           */
/* ------------------------------------------------------------------------ */

typedef struct {
  const float *P, *Q, *Qn;
  int64_t M, N;
  int mode;
  float *Pt;
  int32_t *idx;
  float *d2f;
  float *Qh;       /* gathered closest points, M x 3 */
  double *res;     /* FP64 residual per point: d^2 (point-to-point) or B (point-to-plane) */
  double *w;       /* weights */
  double last[16]; /* the transform (p2p) or parameter vector (p2pl) of the last pass */
  int have_last;
  int nn_passes, evaluations;
  double *trace;
  int trace_cap, trace_len;
  int reason;      /* ORC_ROW_* of the next evaluation (recorded in the trace) */
  double *etrace;
  int etrace_cap, etrace_len;
} orc_ctx;

static void ctx_log_energy(orc_ctx *c, int stage, double E) {
  if (c->etrace && c->etrace_len < c->etrace_cap) {
    c->etrace[2 * c->etrace_len] = stage;
    c->etrace[2 * c->etrace_len + 1] = E;
    c->etrace_len++;
  }
}

typedef struct {
  double E;        /* energy at the evaluated transform for the given nu */
  double prop[16]; /* alignment result T' (p2p) or Gauss-Newton candidate xi* (p2pl) */
  unsigned flags;
} orc_evalres;

/* Correspondences at T (new pass only when T differs bitwise from the last
 * evaluated one), then FP64 residuals. */
static void ctx_record(orc_ctx *c, double E, double nu, int reused, const double T[16]) {
  if (c->trace && c->trace_len < c->trace_cap) {
    double *row = c->trace + 20 * c->trace_len;
    row[0] = E;
    row[1] = nu;
    row[2] = c->reason;
    row[3] = reused;
    memcpy(row + 4, T, sizeof(double) * 16);
    c->trace_len++;
  }
}

/* Returns 1 when the correspondences of the previous pass were reused. */
static int ctx_corr(orc_ctx *c, const double T[16], const double *key, int keylen) {
  c->evaluations++;
  if (c->have_last && memcmp(c->last, key, sizeof(double) * (size_t)keylen) == 0) return 1;
  memcpy(c->last, key, sizeof(double) * (size_t)keylen);
  c->have_last = 1;
  c->nn_passes++;
  orc_transform_f32(T, c->P, c->M, c->Pt);
  orc_nn_brute(c->Pt, c->M, c->Q, c->N, c->idx, c->d2f);
  for (int64_t i = 0; i < c->M; ++i) {
    const int64_t j = c->idx[i];
    c->Qh[3 * i] = c->Q[3 * j];
    c->Qh[3 * i + 1] = c->Q[3 * j + 1];
    c->Qh[3 * i + 2] = c->Q[3 * j + 2];
  }
  return 0;
}

static int mode_plane(int mode) { return mode == ORC_P2PL_WELSCH || mode == ORC_P2PL_L2; }
static int mode_l2(int mode) { return mode == ORC_P2P_L2 || mode == ORC_P2PL_L2; }

static void ctx_residuals(orc_ctx *c, const double T[16]) {
  for (int64_t i = 0; i < c->M; ++i) {
    double x[3];
    xform_f64(T, c->P + 3 * i, x);
    const double dx = x[0] - (double)c->Qh[3 * i], dy = x[1] - (double)c->Qh[3 * i + 1],
                 dz = x[2] - (double)c->Qh[3 * i + 2];
    if (mode_plane(c->mode)) {
      const float *n = c->Qn + 3 * (int64_t)c->idx[i];
      c->res[i] = fma(dz, (double)n[2], fma(dy, (double)n[1], dx * (double)n[0]));
    } else {
      c->res[i] = fma(dz, dz, fma(dy, dy, dx * dx));
    }
  }
}

/* Point-to-point evaluation: E_nu and T' = align(Q^, T, nu). */
static orc_evalres eval_p2p(orc_ctx *c, const double T[16], double nu) {
  orc_evalres ev;
  memset(&ev, 0, sizeof ev);
  const int reused = ctx_corr(c, T, T, 16);
  ctx_residuals(c, T);
  double E = 0;
  if (c->mode == ORC_P2P_L2) {
    for (int64_t i = 0; i < c->M; ++i) E += c->res[i];
    ev.flags = orc_procrustes(c->P, c->Qh, NULL, c->M, ev.prop);
  } else {
    const double s = 1.0 / (2.0 * nu * nu);
    for (int64_t i = 0; i < c->M; ++i) {
      E += -expm1(-c->res[i] * s); /* psi_nu, eq. welsch */
      c->w[i] = exp(-c->res[i] * s);
    }
    ev.flags = orc_procrustes(c->P, c->Qh, c->w, c->M, ev.prop);
  }
  ev.E = E;
  ctx_record(c, E, c->mode == ORC_P2P_L2 ? 0.0 : nu, reused, T);
  return ev;
}

static int chol6_solve(const double A[36], const double b[6], double x[6]) {
  double L[36] = {0}, dmax = 0;
  for (int i = 0; i < 6; ++i) if (A[7 * i] > dmax) dmax = A[7 * i];
  if (!(dmax > 0)) return 1;
  for (int j = 0; j < 6; ++j) {
    double s = A[7 * j];
    for (int k = 0; k < j; ++k) s -= L[6 * j + k] * L[6 * j + k];
    if (!(s > 1e-14 * dmax)) return 1;
    L[7 * j] = sqrt(s);
    for (int i = j + 1; i < 6; ++i) {
      double v = A[6 * i + j];
      for (int k = 0; k < j; ++k) v -= L[6 * i + k] * L[6 * j + k];
      L[6 * i + j] = v / L[7 * j];
    }
  }
  double y[6];
  for (int i = 0; i < 6; ++i) {
    double v = b[i];
    for (int k = 0; k < i; ++k) v -= L[6 * i + k] * y[k];
    y[i] = v / L[7 * i];
  }
  for (int i = 5; i >= 0; --i) {
    double v = y[i];
    for (int k = i + 1; k < 6; ++k) v -= L[6 * k + i] * x[k];
    x[i] = v / L[7 * i];
  }
  return 0;
}

/* Point-to-plane evaluation at xi: E~_nu(xi) and xi* = G_ppl(xi) (eq. GNMapping):
 * A = sum g J J^T, c = sum g B J, xi* = xi - A^{-1} c (reading R6). Classical
 * point-to-plane ICP takes g = 1 and the energy sum B^2 (the limit of the
 * Welsch weights as nu grows). */
static orc_evalres eval_p2pl(orc_ctx *c, const double xi[6], double nu) {
  orc_evalres ev;
  memset(&ev, 0, sizeof ev);
  double T[16];
  orc_se3_exp(xi, T);
  const int reused = ctx_corr(c, T, xi, 6);
  ctx_residuals(c, T);
  double dR[3][9], Dt[9], Du[9];
  se3_derivs(xi, dR, Dt, Du);
  const double s = 1.0 / (2.0 * nu * nu);
  double A[36] = {0}, cv[6] = {0}, E = 0, W = 0;
  const int L2 = mode_l2(c->mode);
  for (int64_t i = 0; i < c->M; ++i) {
    const double B = c->res[i];
    E += L2 ? B * B : -expm1(-B * B * s);
    const double g = L2 ? 1.0 : exp(-B * B * s);
    W += g;
    double J[6];
    plane_gradient_from(dR, Dt, Du, c->P + 3 * i, c->Qn + 3 * (int64_t)c->idx[i], J);
    for (int a = 0; a < 6; ++a) {
      cv[a] += g * B * J[a];
      for (int b = 0; b < 6; ++b) A[6 * a + b] += g * J[a] * J[b];
    }
  }
  ev.E = E;
  ctx_record(c, E, L2 ? 0.0 : nu, reused, T);
  for (int a = 0; a < 6; ++a) ev.prop[a] = xi[a];
  if (!(W > 1e-300)) {
    ev.flags = ORC_FLAG_ZERO_WEIGHT;
    return ev;
  }
  double step[6];
  if (chol6_solve(A, cv, step)) {
    ev.flags = ORC_FLAG_DEGENERATE;
    return ev;
  }
  for (int a = 0; a < 6; ++a) ev.prop[a] = xi[a] - step[a];
  return ev;
}

void orc_params_default(int mode, orc_params *out) {
  memset(out, 0, sizeof *out);
  out->mode = mode;
  out->anderson_m = 5;       /* Sec. 4.2 */
  out->nu_max = -1.0;        /* 3 x median rule */
  out->nu_min = -1.0;
  out->max_line_search = 10; /* reading R7 */
  out->max_total_iter = 0;
  if (mode == ORC_P2PL_WELSCH) {
    out->eps = 1e-5;         /* Sec. 5 */
    out->iter_first = 6;
    out->iter_inc = 1;
    out->iter_cap = 10;
  } else {
    out->eps = 1e-5;         /* Sec. 4.3 */
    out->iter_first = 1000;
    out->iter_inc = 0;
    out->iter_cap = 1000;
  }
  for (int i = 0; i < 16; ++i) out->T0[i] = (i % 5 == 0) ? 1.0 : 0.0;
  if (mode == ORC_P2PL_L2) orc_params_classical(mode, out);
}

/* App. E: the comparison methods stop after 1000 iterations or when the
 * squared Frobenius norm of the change of transform falls below 1e-5. */
int orc_params_classical(int mode, orc_params *out) {
  if (mode != ORC_P2P_L2 && mode != ORC_P2PL_L2) return -1;
  memset(out, 0, sizeof *out);
  out->mode = mode;
  out->anderson_m = 0;
  out->nu_max = -1.0;
  out->nu_min = -1.0;
  out->eps = sqrt(1e-5);
  out->iter_first = 1000;
  out->iter_inc = 0;
  out->iter_cap = 1000;
  out->max_total_iter = 0;
  out->max_line_search = 0;
  for (int i = 0; i < 16; ++i) out->T0[i] = (i % 5 == 0) ? 1.0 : 0.0;
  return 0;
}

#define HIST 8 /* ring capacity (m <= 6, needs m + 1 entries) */

static double frob_diff(const double A[16], const double B[16]) {
  double s = 0;
  for (int i = 0; i < 16; ++i) s += (A[i] - B[i]) * (A[i] - B[i]);
  return sqrt(s);
}

/* Anderson step: hist arrays hold G and F for indices k-m_k .. k (ring by
 * index mod HIST). Returns x_AA = G^k - sum theta_j (G^{k-j+1} - G^{k-j}). */
static int anderson_step(double G[HIST][6], double F[HIST][6], int k, int mk, int metric,
                         double out[6]) {
  double dF[6 * 6], theta[6];
  for (int j = 1; j <= mk; ++j)
    for (int a = 0; a < 6; ++a)
      dF[6 * (j - 1) + a] = F[(k - j + 1) % HIST][a] - F[(k - j) % HIST][a];
  const int sing = orc_anderson_solve(dF, F[k % HIST], mk, metric, theta);
  for (int a = 0; a < 6; ++a) {
    double v = G[k % HIST][a];
    for (int j = 1; j <= mk; ++j) v -= theta[j - 1] * (G[(k - j + 1) % HIST][a] - G[(k - j) % HIST][a]);
    out[a] = v;
  }
  return sing;
}

static int stage_cap(const orc_params *p, int stage) {
  long v = (long)p->iter_first + (long)stage * p->iter_inc;
  if (p->iter_cap > 0 && v > p->iter_cap) v = p->iter_cap;
  return (int)v;
}

static int valid_rigid(const double T[16]) {
  for (int i = 0; i < 16; ++i) if (!isfinite(T[i])) return 0;
  if (T[12] != 0 || T[13] != 0 || T[14] != 0 || T[15] != 1) return 0;
  double R[9], t[3], Rt[9], RtR[9];
  T_to_Rt(T, R, t);
  m3_transpose(R, Rt);
  m3_mul(Rt, R, RtR);
  for (int i = 0; i < 9; ++i)
    if (fabs(RtR[i] - ((i % 4 == 0) ? 1.0 : 0.0)) > 1e-9) return 0;
  return m3_det(R) > 0;
}

/* Algorithm 1 (and Fast ICP = Algorithm 1 with the L2 metric and one stage). */
static void register_p2p(orc_ctx *c, const orc_params *prm, double nu0, orc_result *res) {
  const int m = prm->anderson_m;
  const int L2 = c->mode == ORC_P2P_L2;
  double nu = nu0;
  double Tkm1[16], Tk[16], Tp[16];
  memcpy(Tkm1, prm->T0, sizeof Tkm1);
  double G[HIST][6], F[HIST][6];
  int k = 1, stage = 0, total = 0, stop_all = 0;
  orc_evalres ev;
  for (;;) {
    const int Inu = stage_cap(prm, stage);
    const int kstart = k - 1;
    double Eprev = INFINITY;
    res->stages++;
    c->reason = ORC_ROW_STAGE;
    ev = eval_p2p(c, Tkm1, nu); /* re-weighting at the current transform */
    if (ev.flags & ORC_FLAG_ZERO_WEIGHT) {
      res->flags |= ORC_FLAG_ZERO_WEIGHT;
      memcpy(Tk, Tkm1, sizeof Tk);
      break;
    }
    res->flags |= ev.flags & ORC_FLAG_DEGENERATE;
    memcpy(Tp, ev.prop, sizeof Tp);
    memcpy(Tk, Tp, sizeof Tk);
    {
      double lp[6], lq[6];
      orc_se3_log(Tp, lp);
      orc_se3_log(Tkm1, lq);
      for (int a = 0; a < 6; ++a) {
        G[(k - 1) % HIST][a] = lp[a];
        F[(k - 1) % HIST][a] = lp[a] - lq[a];
      }
    }
    c->reason = ORC_ROW_ITER;
    ev = eval_p2p(c, Tk, nu);
    int is_aa = 0, converged = 0;
    while (k - kstart <= Inu) {
      if (prm->max_total_iter > 0 && total >= prm->max_total_iter) { stop_all = 1; break; }
      res->iterations++;
      total++;
      double E = ev.E;
      if (m > 0 && E >= Eprev) { /* safeguard: revert to the un-accelerated iterate */
        memcpy(Tk, Tp, sizeof Tk);
        c->reason = ORC_ROW_REVERT;
        ev = eval_p2p(c, Tk, nu);
        E = ev.E;
        res->aa_rejected++;
      } else if (is_aa) {
        res->aa_accepted++;
      }
      Eprev = E;
      ctx_log_energy(c, stage, E);
      if (ev.flags & ORC_FLAG_ZERO_WEIGHT) { res->flags |= ORC_FLAG_ZERO_WEIGHT; stop_all = 1; break; }
      res->flags |= ev.flags & ORC_FLAG_DEGENERATE;
      memcpy(Tp, ev.prop, sizeof Tp);
      if (frob_diff(Tk, Tp) < prm->eps) { converged = 1; break; }
      double Tn[16];
      if (m == 0) {
        memcpy(Tn, Tp, sizeof Tn);
        is_aa = 0;
      } else {
        double lp[6], lk[6], xaa[6];
        orc_se3_log(Tp, lp);
        orc_se3_log(Tk, lk);
        for (int a = 0; a < 6; ++a) {
          G[k % HIST][a] = lp[a];
          F[k % HIST][a] = lp[a] - lk[a];
        }
        const int mk = (k - kstart) < m ? (k - kstart) : m;
        if (anderson_step(G, F, k, mk, 0, xaa)) res->flags |= ORC_FLAG_AA_SINGULAR;
        orc_se3_exp(xaa, Tn);
        is_aa = 1;
      }
      memcpy(Tk, Tn, sizeof Tk);
      c->reason = ORC_ROW_ITER;
      ev = eval_p2p(c, Tk, nu);
      k++;
    }
    if (stop_all) {
      if (!(res->flags & ORC_FLAG_ZERO_WEIGHT)) res->flags |= ORC_FLAG_MAX_ITER;
      break;
    }
    if (converged) res->flags = (res->flags & ~(unsigned)ORC_FLAG_MAX_ITER) | ORC_FLAG_CONVERGED;
    else res->flags = (res->flags & ~(unsigned)ORC_FLAG_CONVERGED) | ORC_FLAG_MAX_ITER;
    if (L2 || nu == prm->nu_min) break;
    nu = fmax(nu / 2.0, prm->nu_min);
    k++;
    stage++;
    memcpy(Tkm1, Tk, sizeof Tkm1);
  }
  memcpy(res->T, Tk, sizeof res->T);
  res->energy = ev.E;
  res->nu_final = L2 ? 0.0 : nu;
}

/* Algorithm 2: robust point-to-plane with line search and Anderson mixing.
 * Classical point-to-plane ICP runs the same loop with unit weights, a single
 * stage, and the convergence test on the change of transform (App. E). */
static void register_p2pl(orc_ctx *c, const orc_params *prm, double nu0, orc_result *res) {
  const int m = prm->anderson_m;
  const int L2 = mode_l2(c->mode);
  double nu = nu0;
  double xkm1[6], xk[6], xstar[6];
  orc_se3_log(prm->T0, xkm1);
  double G[HIST][6], F[HIST][6];
  int k = 1, stage = 0, total = 0, stop_all = 0;
  double Ecur = 0;
  for (;;) {
    const int Inu = stage_cap(prm, stage);
    const int kstart = k - 1;
    double Eprev = INFINITY;
    res->stages++;
    c->reason = ORC_ROW_STAGE;
    orc_evalres ev = eval_p2pl(c, xkm1, nu);
    if (ev.flags & (ORC_FLAG_ZERO_WEIGHT | ORC_FLAG_DEGENERATE)) {
      res->flags |= ev.flags;
      memcpy(xk, xkm1, sizeof xk);
      Ecur = ev.E;
      break;
    }
    memcpy(xstar, ev.prop, sizeof xstar);
    for (int a = 0; a < 6; ++a) {
      G[(k - 1) % HIST][a] = xstar[a];
      F[(k - 1) % HIST][a] = xstar[a] - xkm1[a];
    }
    memcpy(xk, xstar, sizeof xk);
    c->reason = ORC_ROW_ITER;
    ev = eval_p2pl(c, xk, nu);
    Ecur = ev.E;
    int converged = 0, is_aa = 0;
    while (k - kstart <= Inu) {
      if (prm->max_total_iter > 0 && total >= prm->max_total_iter) { stop_all = 1; break; }
      res->iterations++;
      total++;
      double E = ev.E;
      orc_evalres best = ev;
      if (E >= Eprev) {
        double tau = 1.0;
        for (int l = 1; l <= prm->max_line_search; ++l) {
          double xt[6];
          for (int a = 0; a < 6; ++a) xt[a] = xkm1[a] + tau * (xstar[a] - xkm1[a]);
          c->reason = ORC_ROW_TRIAL;
          orc_evalres et = eval_p2pl(c, xt, nu);
          res->line_search_trials++;
          if (et.E < E) {
            E = et.E;
            memcpy(xk, xt, sizeof xk);
            best = et;
          }
          if (et.E < Eprev) break;
          tau *= 0.5;
        }
        if (is_aa) res->aa_rejected++;
      } else if (is_aa) {
        res->aa_accepted++;
      }
      Eprev = E;
      Ecur = E;
      ctx_log_energy(c, stage, E);
      if (best.flags & (ORC_FLAG_ZERO_WEIGHT | ORC_FLAG_DEGENERATE)) {
        res->flags |= best.flags;
        stop_all = 1;
        break;
      }
      double xs_next[6];
      memcpy(xs_next, best.prop, sizeof xs_next);
      double dn = 0;
      if (L2) {
        double Tn[16], Tc[16];
        orc_se3_exp(xs_next, Tn);
        orc_se3_exp(xk, Tc);
        dn = frob_diff(Tn, Tc);
      } else {
        for (int a = 0; a < 6; ++a) dn += (xs_next[a] - xk[a]) * (xs_next[a] - xk[a]);
        dn = sqrt(dn);
      }
      if (dn < prm->eps) { converged = 1; break; }
      double xn[6];
      for (int a = 0; a < 6; ++a) {
        G[k % HIST][a] = xs_next[a];
        F[k % HIST][a] = xs_next[a] - xk[a];
      }
      if (m == 0) {
        memcpy(xn, xs_next, sizeof xn);
        is_aa = 0;
      } else {
        const int mk = (k - kstart) < m ? (k - kstart) : m;
        if (anderson_step(G, F, k, mk, 1, xn)) res->flags |= ORC_FLAG_AA_SINGULAR;
        is_aa = 1;
      }
      memcpy(xkm1, xk, sizeof xkm1);
      memcpy(xstar, xs_next, sizeof xstar);
      memcpy(xk, xn, sizeof xk);
      c->reason = ORC_ROW_ITER;
      ev = eval_p2pl(c, xk, nu);
      Ecur = ev.E;
      k++;
    }
    if (stop_all) {
      if (!(res->flags & (ORC_FLAG_ZERO_WEIGHT | ORC_FLAG_DEGENERATE))) res->flags |= ORC_FLAG_MAX_ITER;
      break;
    }
    if (converged) res->flags = (res->flags & ~(unsigned)ORC_FLAG_MAX_ITER) | ORC_FLAG_CONVERGED;
    else res->flags = (res->flags & ~(unsigned)ORC_FLAG_CONVERGED) | ORC_FLAG_MAX_ITER;
    if (L2 || nu == prm->nu_min) break;
    nu = fmax(nu / 2.0, prm->nu_min);
    k++;
    stage++;
    memcpy(xkm1, xk, sizeof xkm1);
  }
  orc_se3_exp(xk, res->T);
  res->energy = Ecur;
  res->nu_final = L2 ? 0.0 : nu;
}

/* Scratch of one map application; freed by eval_ctx_free. */
static int eval_ctx_init(orc_ctx *c, const float *P, int64_t M, const float *Q, const float *Qn,
                         int64_t N, int mode, double nu) {
  if (!P || !Q || M <= 0 || N <= 0 || mode < 0 || mode > 3) return -1;
  if (mode_plane(mode) && !Qn) return -1;
  if (!mode_l2(mode) && !(nu > 0)) return -1;
  memset(c, 0, sizeof *c);
  c->P = P; c->Q = Q; c->Qn = Qn; c->M = M; c->N = N; c->mode = mode;
  c->Pt = (float *)malloc(sizeof(float) * 3 * (size_t)M);
  c->idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)M);
  c->d2f = (float *)malloc(sizeof(float) * (size_t)M);
  c->Qh = (float *)malloc(sizeof(float) * 3 * (size_t)M);
  c->res = (double *)malloc(sizeof(double) * (size_t)M);
  c->w = (double *)malloc(sizeof(double) * (size_t)M);
  return 0;
}

static void eval_ctx_free(orc_ctx *c) {
  free(c->Pt); free(c->idx); free(c->d2f); free(c->Qh); free(c->res); free(c->w);
}

/* One un-accelerated map application at T (see the header). */
int orc_eval(const float *P, int64_t M, const float *Q, const float *Qn, int64_t N, int mode,
             const double T[16], double nu, double *E, double Tout[16], unsigned *flags) {
  orc_ctx c;
  if (eval_ctx_init(&c, P, M, Q, Qn, N, mode, nu)) return -1;
  orc_evalres ev;
  if (mode_plane(mode)) {
    double xi[6];
    orc_se3_log(T, xi);
    ev = eval_p2pl(&c, xi, nu);
    orc_se3_exp(ev.prop, Tout);
  } else {
    ev = eval_p2p(&c, T, nu);
    if (ev.flags & ORC_FLAG_ZERO_WEIGHT) memcpy(Tout, T, sizeof(double) * 16);
    else memcpy(Tout, ev.prop, sizeof(double) * 16);
  }
  *E = ev.E;
  *flags = ev.flags;
  eval_ctx_free(&c);
  return 0;
}

/* Algorithm 2's map at the parameters themselves (see the header). */
int orc_eval_xi(const float *P, int64_t M, const float *Q, const float *Qn, int64_t N, int mode,
                const double xi[6], double nu, double *E, double xi_out[6], unsigned *flags) {
  if (!mode_plane(mode)) return -1;
  orc_ctx c;
  if (eval_ctx_init(&c, P, M, Q, Qn, N, mode, nu)) return -1;
  orc_evalres ev = eval_p2pl(&c, xi, nu);
  memcpy(xi_out, ev.prop, sizeof(double) * 6);
  *E = ev.E;
  *flags = ev.flags;
  eval_ctx_free(&c);
  return 0;
}

int orc_register(const float *P, int64_t M, const float *Q, const float *Qn, int64_t N,
                 const orc_params *prm, orc_result *res, double *trace, int trace_cap,
                 int *trace_len, double *etrace, int etrace_cap, int *etrace_len) {
  if (!P || !Q || !prm || !res || M <= 0 || N <= 0) return -1;
  if (prm->mode < 0 || prm->mode > 3) return -1;
  if (mode_plane(prm->mode) && !Qn) return -1;
  if (prm->anderson_m < 0 || prm->anderson_m > 6) return -1;
  if (!mode_l2(prm->mode) && !(prm->nu_min > 0)) return -1;
  if (!(prm->eps > 0) || prm->iter_first <= 0) return -1;
  if (!valid_rigid(prm->T0)) return -1;
  memset(res, 0, sizeof *res);
  orc_ctx c;
  memset(&c, 0, sizeof c);
  c.P = P; c.Q = Q; c.Qn = Qn; c.M = M; c.N = N; c.mode = prm->mode;
  c.Pt = (float *)malloc(sizeof(float) * 3 * (size_t)M);
  c.idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)M);
  c.d2f = (float *)malloc(sizeof(float) * (size_t)M);
  c.Qh = (float *)malloc(sizeof(float) * 3 * (size_t)M);
  c.res = (double *)malloc(sizeof(double) * (size_t)M);
  c.w = (double *)malloc(sizeof(double) * (size_t)M);
  c.trace = trace; c.trace_cap = trace ? trace_cap : 0;
  c.etrace = etrace; c.etrace_cap = etrace ? etrace_cap : 0;

  /* nu_max = 3 x median of the initial residuals (Sec. 4.3; Sec. 5). */
  double nu0 = prm->nu_max;
  if (!mode_l2(prm->mode) && !(nu0 > 0)) {
    if (prm->mode == ORC_P2PL_WELSCH) {
      double x0[6];
      orc_se3_log(prm->T0, x0);
      double T[16];
      orc_se3_exp(x0, T);
      ctx_corr(&c, T, x0, 6);
      ctx_residuals(&c, T);
      for (int64_t i = 0; i < M; ++i) c.res[i] = fabs(c.res[i]);
      nu0 = 3.0 * orc_median(c.res, M);
    } else {
      ctx_corr(&c, prm->T0, prm->T0, 16);
      ctx_residuals(&c, prm->T0);
      nu0 = 3.0 * sqrt(orc_median(c.res, M));
    }
  }
  if (mode_plane(prm->mode)) register_p2pl(&c, prm, nu0, res);
  else register_p2p(&c, prm, nu0, res);
  res->nn_passes = c.nn_passes;
  res->evaluations = c.evaluations;
  if (trace_len) *trace_len = c.trace_len;
  if (etrace_len) *etrace_len = c.etrace_len;
  free(c.Pt); free(c.idx); free(c.d2f); free(c.Qh); free(c.res); free(c.w);
  return 0;
}
