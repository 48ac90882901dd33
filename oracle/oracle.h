/*
 * Oracle for Fast and Robust ICP (Zhang, Yao, Deng, arXiv 2007.07627).
 *
 * TEST INFRASTRUCTURE ONLY. This is a plain, slow, FP64 CPU implementation of
 * what the GPU path computes. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it. It shares no code, header, table
 * or helper with the GPU library; the GPU library never includes or links it.
 *
 * Conventions
 *   - Point sets are host AoS, row-major n x 3, float32.
 *   - A rigid transform T is FP64 row-major 4x4 [R t; 0 0 0 1].
 *   - An se(3) parameter vector xi is FP64 [delta_1..3, u_1..3] (Sec. 4.2,
 *     eq. Matrixsed: S = delta^, translation part u).
 */
#ifndef ICP_ORACLE_H
#define ICP_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ORC_P2PL_L2 is classical point-to-plane ICP (Chen and Medioni), the
 * "ICP-l" comparison of Sec. 6: energy sum B_i^2, Gauss-Newton map of
 * eq. GNMapping with unit weights, one stage. */
enum { ORC_P2P_L2 = 0, ORC_P2P_WELSCH = 1, ORC_P2PL_WELSCH = 2, ORC_P2PL_L2 = 3 };

/* why the registration evaluated a transform (trace rows) */
enum { ORC_ROW_STAGE = 1, ORC_ROW_ITER = 2, ORC_ROW_REVERT = 3, ORC_ROW_TRIAL = 4 };

enum {
  ORC_FLAG_CONVERGED = 1u,
  ORC_FLAG_MAX_ITER = 2u,
  ORC_FLAG_ZERO_WEIGHT = 4u,
  ORC_FLAG_DEGENERATE = 8u,
  ORC_FLAG_AA_SINGULAR = 16u
};

typedef struct {
  int mode;              /* ORC_P2P_L2 / ORC_P2P_WELSCH / ORC_P2PL_WELSCH / ORC_P2PL_L2 */
  int anderson_m;        /* Anderson depth m; 0 = plain MM iteration */
  double nu_max;         /* <= 0: 3 x median rule at T0 */
  double nu_min;         /* must be > 0 for the Welsch modes */
  double eps;            /* per-stage convergence threshold */
  int iter_first;        /* I_nu for the first stage */
  int iter_inc;          /* I_nu increment per stage */
  int iter_cap;          /* I_nu upper bound */
  int max_total_iter;    /* <= 0: unlimited */
  int max_line_search;   /* l_max of the point-to-plane line search */
  double T0[16];
} orc_params;

typedef struct {
  double T[16];
  double energy;         /* E_nu (or sum of squares for L2) at the returned T */
  double nu_final;
  int iterations;        /* inner-loop iterations over all stages */
  int nn_passes;         /* correspondence computations at a new transform */
  int evaluations;       /* passes incl. re-weighting at an unchanged transform */
  int aa_accepted, aa_rejected, line_search_trials, stages;
  unsigned flags;
} orc_result;

/* Eq. CorresponcePoint with the transform rounded once to FP32 (see .c). */
void orc_transform_f32(const double T[16], const float *P, int64_t M, float *out);
void orc_nn_brute(const float *Pt, int64_t M, const float *Q, int64_t N,
                  int32_t *idx, float *d2);
void orc_nn_query(const float *P, int64_t M, const float *Q, int64_t N,
                  const double T[16], int32_t *idx, float *d2);

/* se(3) exponential and logarithm (eq. MatrixExp, Appendix A). */
void orc_se3_exp(const double xi[6], double T[16]);
void orc_se3_log(const double T[16], double xi[6]);

/* 3x3 SVD A = U diag(S) V^T, S descending; returns 0. */
int orc_svd3(const double A[9], double U[9], double S[3], double V[9]);

/* Weighted rigid Procrustes (eq. WelschAlignment). P, Qh: M x 3 float;
 * w: M weights or NULL for all ones. Returns flags (ZERO_WEIGHT/DEGENERATE). */
unsigned orc_procrustes(const float *P, const float *Qh, const double *w,
                        int64_t M, double T[16]);

/* Signed point-to-plane distance B_i(xi) and its gradient (Appendix D). */
double orc_plane_residual(const double xi[6], const float p[3], const float q[3],
                          const float n[3]);
void orc_plane_gradient(const double xi[6], const float p[3], const float n[3],
                        double J[6]);

/* Anderson least squares (Sec. 4.1). dF: m x 6 rows (F^{k-j+1}-F^{k-j}),
 * Fk: 6, metric 0 = Frobenius on the 4x4 log (rotation part weighted 2),
 * 1 = Euclidean. theta: m. Returns 1 if the system was singular (theta=0). */
int orc_anderson_solve(const double *dF, const double *Fk, int m, int metric,
                       double *theta);

/* Element of rank floor(n/2) in ascending order (copy is sorted). */
double orc_median(const double *v, int64_t n);

/* Automatic nu_min (Sec. 4.3 for point-to-point, Sec. 5 for point-to-plane,
 * rationale in App. C). For every target q_i: its six nearest other targets
 * (exact FP32 squared distances of q_i - q_j, ties to the lower index, j != i);
 * point-to-point: the median of their distances, Ebar = median over i,
 * nu_min = Ebar / (3 sqrt 3); point-to-plane: the median of their distances
 * |n_i . (q_j - q_i)| to the tangent plane at q_i, Hbar = median over i,
 * nu_min = Hbar / 6. Medians are elements of rank floor(n/2). Needs N >= 7
 * (returns -1 otherwise, or for point-to-plane without normals). The
 * per-point values (FP64) go to per_point when it is not NULL. */
int orc_nu_min_auto(const float *Q, const float *Qn, int64_t N, int mode, double *nu_min,
                    double *per_point);

/* Normals of a point set for point-to-plane registration without given
 * normals (the paper estimates them from 30 nearest neighbours): for every
 * point q_i its k = 30 nearest points of the set, q_i itself included (exact
 * FP32 squared distances of q_i - q_j, ties to the lower index); their mean
 * and covariance in FP64 (sums in that order); the unit eigenvector of the
 * smallest eigenvalue, oriented so that n . q_i <= 0 (towards a viewpoint at
 * the origin). Needs N >= 30; returns -1 otherwise. */
int orc_estimate_normals(const float *Q, int64_t N, float *normals);

/* Full registration: Fast ICP (L2 + AA), Algorithm 1, Algorithm 2, and
 * classical point-to-plane ICP. Qn may be NULL except for the point-to-plane
 * modes. trace (optional) receives one
 * row of 20 doubles per evaluation [E, nu, reason, reused, T(16)], up to
 * trace_cap rows (the setup pass that only feeds the median is not a row);
 * reason is ORC_ROW_STAGE (the stage's first evaluation, at T^(k-1)),
 * ORC_ROW_ITER (an iterate T^(k)), ORC_ROW_REVERT (Algorithm 1's safeguard:
 * the un-accelerated T') or ORC_ROW_TRIAL (an Algorithm 2 line-search trial);
 * etrace (optional) receives (stage, accepted energy)
 * for every inner iteration, up to etrace_cap pairs.
 * Returns 0 on success, -1 on invalid arguments. */
int orc_register(const float *P, int64_t M, const float *Q, const float *Qn,
                 int64_t N, const orc_params *prm, orc_result *res,
                 double *trace, int trace_cap, int *trace_len,
                 double *etrace, int etrace_cap, int *etrace_len);

/* One application of the un-accelerated map at T with parameter nu: the
 * energy at T and the alignment update (point-to-point) or exp of the
 * Gauss-Newton candidate at log T (point-to-plane). Returns 0 / -1. */
int orc_eval(const float *P, int64_t M, const float *Q, const float *Qn, int64_t N, int mode,
             const double T[16], double nu, double *E, double Tout[16], unsigned *flags);

/* Algorithm 2's map evaluated at the parameters xi themselves (point-to-plane
 * modes only): the energy at exp(xi) and the Gauss-Newton candidate xi* of
 * eq. GNMapping, linearised at xi. The iterate of Algorithm 2 lives in R^6
 * and may rotate by more than pi, where log(exp(xi)) is another point of R^6
 * with another linearisation; orc_eval goes through log T. Returns 0 / -1. */
int orc_eval_xi(const float *P, int64_t M, const float *Q, const float *Qn, int64_t N, int mode,
                const double xi[6], double nu, double *E, double xi_out[6], unsigned *flags);

void orc_params_default(int mode, orc_params *out);

/* The comparison methods of Sec. 6 with the termination the paper gives them
 * (App. on the experiment settings): ICP (mode ORC_P2P_L2) and ICP-l (mode
 * ORC_P2PL_L2), no Anderson mixing, no line search, one stage of at most
 * 1000 iterations, stop when ||T_{k+1} - T_k||_F^2 < 1e-5 (eps = sqrt(1e-5)
 * on the Frobenius norm). Returns -1 for the other modes. */
int orc_params_classical(int mode, orc_params *out);

#ifdef __cplusplus
}
#endif
#endif
