/*
 * libicp -- Fast and Robust Iterative Closest Point (Zhang, Yao, Deng,
 * arXiv 2007.07627) on AMD Instinct MI355X (gfx950).
 *
 * C ABI. Every call returns icp_status; nothing aborts or throws across the
 * ABI. Plain pointers and sizes only. Unless a function says otherwise,
 * pointers are HOST pointers; the *_dev functions take DEVICE pointers (HBM of
 * the context's GPU) and an optional hipStream_t passed as void*.
 *
 * Problem (Sec. 3, eq. ICPOptimization; Sec. 4.3, eq. WelschRegistration;
 * Sec. 5, eq. WelschPointToPlaneOptimization): find the rigid T = [R t; 0 1]
 * that aligns the source P (M x 3) to the target Q (N x 3, optional unit
 * normals Qn) under the L2, robust point-to-point or robust point-to-plane
 * metric.
 *
 * Layouts: point sets are row-major n x 3 float32 (x, y, z per point).
 * Transforms are float64 row-major 4 x 4, mapping source to target; they must
 * be rigid: |R^T R - I| <= 1e-9 entrywise, det R > 0, last row (0, 0, 0, 1).
 * Coordinates must be finite with magnitude <= 1e15.
 *
 * Threading: one icp_ctx may be used from several threads; calls are
 * serialised internally per engine (synchronous calls vs. the batch engine).
 */
#ifndef ICP_H
#define ICP_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct icp_ctx icp_ctx;

typedef enum {
  ICP_OK = 0,
  ICP_ERR_INVALID_ARG = 1,   /* bad shape, pointer, parameter or transform */
  ICP_ERR_NONFINITE = 2,     /* NaN / Inf (or |x| > 1e15) in an input coordinate */
  ICP_ERR_NO_NORMALS = 3,    /* point-to-plane mode without target normals */
  ICP_ERR_OOM = 4,           /* the request does not fit the context's HBM budget */
  ICP_ERR_DEVICE = 5,        /* a HIP runtime call failed */
  ICP_ERR_NOT_READY = 6,     /* icp_poll: the ticket is still queued or running */
  ICP_ERR_UNKNOWN_TICKET = 7,/* icp_poll: never issued, or its result was already taken */
  ICP_ERR_QUEUE_FULL = 8     /* icp_batch_submit: host queue limit reached */
} icp_status;

typedef enum {
  ICP_P2P_L2 = 0,        /* Fast ICP: L2 point-to-point + Anderson (Sec. 4.2) */
  ICP_P2P_WELSCH = 1,    /* Algorithm 1: Welsch point-to-point + Anderson (Sec. 4.3) */
  ICP_P2PL_WELSCH = 2,   /* Algorithm 2: Welsch point-to-plane + Anderson (Sec. 5) */
  ICP_P2PL_L2 = 3        /* classical point-to-plane ICP ("ICP-l", Sec. 6): energy sum B_i^2,
                            the Gauss-Newton map of Algorithm 2 with unit weights, one stage */
} icp_mode;

/* Closest-point search (eq. CorresponcePoint). All methods return the same
 * bit-exact result: the FP32 transformed point p' = fl32(T p) (FP64 fused
 * order), d2 = fma(dz,dz, fma(dy,dy, dx*dx)) with FP32 differences, minimum
 * d2, ties to the lowest target index. BRUTE scans every target; CLUSTER
 * prunes with a Hilbert-ordered cluster index (Hilbert keys of a 1024^3 cell
 * grid over the target's bounding box, 128 targets per cluster); AUTO picks
 * by size. The batch engine searches a BRUTE pair above about 2^37 source x
 * target pairs per pass with CLUSTER instead (the result is the same). */
typedef enum { ICP_NN_AUTO = 0, ICP_NN_BRUTE = 1, ICP_NN_CLUSTER = 2 } icp_nn_method;

/* How icp_register drives the iterations: GRAPH keeps the per-pair state on
 * the device and replays a captured hipGraph of several passes between host
 * polls; PLAIN launches every pass and synchronises the host after each one
 * (the one-pair-at-a-time comparator). Both give bit-identical results. */
typedef enum { ICP_ENGINE_GRAPH = 0, ICP_ENGINE_PLAIN = 1 } icp_engine;

typedef struct {
  icp_mode mode;
  int anderson_m;        /* Anderson depth m in [0, 6]; 0 disables mixing (plain MM); paper: 5 (Sec. 4.2) */
  double nu_max;         /* <= 0: 3 x median of the initial residuals (Sec. 4.3, Sec. 5) */
  double nu_min;         /* > 0; <= 0: the paper's automatic rule (icp_nu_min_auto, N >= 7) */
  double eps;            /* stage threshold on ||T - T'||_F (point-to-point and ICP_P2PL_L2) /
                            ||xi* - xi|| (ICP_P2PL_WELSCH); paper 1e-5 */
  int iter_first;        /* I_nu of the first stage; paper: 1000 (p2p), 6 (p2pl) */
  int iter_inc;          /* I_nu increment per stage; paper: 0 (p2p), 1 (p2pl) */
  int iter_cap;          /* I_nu upper bound; paper: 1000 (p2p), 10 (p2pl); <= 0 none */
  int max_total_iter;    /* cap on inner iterations over all stages; <= 0 unlimited */
  int max_line_search;   /* l_max of Algorithm 2 (unspecified in the paper): 10 */
  icp_nn_method nn;
  icp_engine engine;
  double T0[16];         /* initial transform, default identity */
} icp_params;

enum {
  ICP_FLAG_CONVERGED = 1u,      /* the last stage ended by the eps test */
  ICP_FLAG_MAX_ITER = 2u,       /* the last stage ended by its iteration cap */
  ICP_FLAG_ZERO_WEIGHT = 4u,    /* every Welsch weight underflowed: no update possible */
  ICP_FLAG_DEGENERATE = 8u,     /* rank-deficient alignment / singular 6x6 system */
  ICP_FLAG_AA_SINGULAR = 16u    /* an Anderson least-squares system was singular (theta = 0 used) */
};

typedef struct {
  double T[16];          /* final transform (source -> target) */
  double energy;         /* target energy at T for the final nu (sum d^2 for L2) */
  double nu_final;
  int iterations;        /* inner iterations over all stages */
  int nn_passes;         /* closest-point passes at a new transform */
  int evaluations;       /* passes including re-weighting at an unchanged transform */
  int aa_accepted, aa_rejected, line_search_trials, stages;
  unsigned status_flags; /* ICP_FLAG_* */
  double latency_ms;     /* batch engine: submit -> done; synchronous calls: wall time */
  double nn_pairs;       /* (source, target) pairs run through the search's filter */
  double nn_exact_pairs; /* pairs evaluated with the exact FP32 definition */
} icp_result;

/* Accumulated device time of the pass kernels since icp_profile(ctx, 1),
 * measured with HIP events recorded around the kernels on the library's own
 * stream: the closest-point search (cull + slice kernels), the
 * weight-and-reduce pass, and the median + solver kernels; passes counted.
 * While profiling, the graph engine launches the same passes directly on its
 * stream (same kernels and host synchronisation cadence) instead of replaying
 * the captured graph; the batch engine's two slot branches, whose passes run
 * side by side in a replay, then run one after the other and a pass's times
 * are the sums over both. */
typedef struct {
  double nn_ms, reduce_ms, solve_ms;
  long long passes;
} icp_profile_stats;

typedef struct {
  const float *P;        /* M x 3 host source */
  int64_t M;
  const float *Q;        /* N x 3 host target */
  const float *Qn;       /* N x 3 host normals or NULL */
  int64_t N;
  icp_params params;
} icp_request;

/* Context on HIP device `device` with an HBM arena of hbm_budget_bytes
 * (0 = 8 GiB). Owns its streams, graphs and memory. */
icp_status icp_create(int device, size_t hbm_budget_bytes, icp_ctx **out);
icp_status icp_destroy(icp_ctx *ctx);

/* The paper's defaults for a mode (Sec. 4.2, Sec. 4.3, Sec. 5); for
 * ICP_P2PL_L2 the classical settings below. */
icp_status icp_params_default(icp_mode mode, icp_params *out);

/* Settings of the comparison methods ICP (mode ICP_P2P_L2) and ICP-l (mode
 * ICP_P2PL_L2) as App. E runs them: no Anderson mixing (anderson_m = 0), no
 * line search (max_line_search = 0), one stage of at most 1000 iterations,
 * stop once ||T_{k+1} - T_k||_F^2 < 1e-5 (eps = sqrt(1e-5)). Other modes:
 * ICP_ERR_INVALID_ARG. */
icp_status icp_params_classical(icp_mode mode, icp_params *out);

/* Synchronous registration (Algorithm 1 / Algorithm 2 / Fast ICP). Inputs are
 * copied before the call returns; `out` is written by the call. */
icp_status icp_register(icp_ctx *ctx, const float *P, int64_t M, const float *Q, const float *Qn,
                        int64_t N, const icp_params *params, icp_result *out);

/* One application of the un-accelerated iteration map at transform T with
 * Welsch parameter nu (ignored for ICP_P2P_L2): correspondences at T
 * (eq. CorresponcePoint), the energy E_nu(T) (eq. WelschRegistration; sum of
 * squared distances for L2; eq. WelschPointToPlaneOptimization for
 * point-to-plane) into *energy_out, and the updated transform into T_out: the
 * weighted Procrustes solution of eq. WelschAlignment (the map G_ICP of
 * eq. FixedPointICP) for point-to-point, or exp of the Gauss-Newton candidate
 * G_ppl(log T) of eq. GNMapping for point-to-plane. *flags_out receives
 * ICP_FLAG_ZERO_WEIGHT / ICP_FLAG_DEGENERATE when no update exists (T_out is
 * then T). Synchronous; host pointers. */
icp_status icp_eval(icp_ctx *ctx, const float *P, int64_t M, const float *Q, const float *Qn,
                    int64_t N, icp_mode mode, const double T[16], double nu,
                    double *energy_out, double T_out[16], unsigned *flags_out);

/* icp_register that also records one row of ICP_TRACE_ROW (36) doubles per
 * pass into the caller's host array trace_out (capacity trace_cap rows):
 * [0] the pass's energy (sum of psi_nu, eq. welsch, or sum of squares for L2),
 * [1] its nu (0 for L2), [2] the solver position that requested it (0 first
 * pass, 1 stage start at T^(k-1), 2 iterate T^(k), 3 safeguard revert to T',
 * 4 line-search trial), [3] 1 if the closest-point search was reused at an
 * unchanged transform, [4..19] the evaluated transform (row-major 4 x 4),
 * [20..35] the un-accelerated update computed from this evaluation: T' of
 * eq. WelschAlignment (point-to-point; T itself when every weight is zero)
 * or the Gauss-Newton parameters xi* of eq. GNMapping in [20..25]
 * (point-to-plane), followed there by the parameters xi of the evaluation
 * itself in [26..31] (exp xi is the transform in [4..19]; the iterate of
 * Algorithm 2 lives in R^6 and may rotate by more than pi, where log T is
 * another point of R^6) and zeros. *trace_len receives the number of rows written (passes
 * beyond the capacity are not recorded). For convergence plots (energy
 * against iteration, Sec. 4.2) and for replaying a registration step by step. */
#define ICP_TRACE_ROW 36
icp_status icp_register_trace(icp_ctx *ctx, const float *P, int64_t M, const float *Q,
                              const float *Qn, int64_t N, const icp_params *params,
                              icp_result *out, double *trace_out, int trace_cap,
                              int *trace_len);

/* Diagnostics of the last icp_register_trace call: for every closest-point
 * work item of its last pass, 8 ints [device cycles, clusters run through the
 * filter, candidate clusters, flags (1 warm start, 2 candidate list, 4 exact
 * re-pass), cycles of: warm start, candidate search, list refinement, filter]
 * into out (capacity cap items); *len = number of items. */
icp_status icp_trace_items(icp_ctx *ctx, int *out, int cap, int *len);

/* Same with device-resident AoS inputs (no host copy); `stream` is ordered
 * before and after the work (NULL = the null stream). Synchronous. */
icp_status icp_register_dev(icp_ctx *ctx, const float *P_dev, int64_t M, const float *Q_dev,
                            const float *Qn_dev, int64_t N, const icp_params *params,
                            icp_result *out, void *stream);

/* Closest target point of every source point under T (eq. CorresponcePoint):
 * idx_out[i] (int32, 0-based target index) and d2_out[i] (FP32 squared
 * distance), both caller-allocated host arrays of M entries. M = 0 is a no-op;
 * N = 0 is ICP_ERR_INVALID_ARG. Synchronous. */
icp_status icp_nn_query(icp_ctx *ctx, const float *P, int64_t M, const float *Q, int64_t N,
                        const double T[16], icp_nn_method method, int32_t *idx_out,
                        float *d2_out);

/* Same with device pointers for inputs and outputs. Synchronous. */
icp_status icp_nn_query_dev(icp_ctx *ctx, const float *P_dev, int64_t M, const float *Q_dev,
                            int64_t N, const double T[16], icp_nn_method method,
                            int32_t *idx_out_dev, float *d2_out_dev, void *stream);

/* For callers that cannot allocate device memory or synchronise with the
 * host -- code under HIP graph capture, serving loops that forbid allocation
 * -- the closest-point query of icp_nn_query_dev without a context: no
 * allocation of any kind, no host synchronisation, no memset or host-copy
 * nodes; every step (setup of the cluster index, search, outputs) is a kernel
 * launched on `stream` (NULL = the null stream), and the call returns once
 * they are enqueued, so the outputs are ready when the stream reaches that
 * point. Same result as icp_nn_query_dev, bit for bit.
 * Working memory: one fixed device array of ICP_NOALLOC_SCRATCH_BYTES (64 MiB)
 * per GPU, held until the process ends; about 100 bytes per source plus 60
 * per target (plus the sort buffers) must fit it, which holds M = N up to
 * about 400000; larger requests return ICP_ERR_OOM without launching
 * anything. Every call on a GPU uses that GPU's one array: calls that overlap
 * on one GPU (other streams, other threads) race and must be serialised by
 * the caller; consecutive calls on one stream are ordered. The array keeps
 * the last call's contents; everything a call reads is rewritten by it first.
 * Device: the current HIP device. Inputs/outputs: device pointers as in
 * icp_nn_query_dev. Errors: ICP_ERR_INVALID_ARG as icp_nn_query_dev,
 * ICP_ERR_OOM beyond the array, ICP_ERR_DEVICE on a launch failure. */
icp_status icp_nn_query_dev_noalloc(const float *P_dev, int64_t M, const float *Q_dev, int64_t N,
                                    const double T[16], icp_nn_method method,
                                    int32_t *idx_out_dev, float *d2_out_dev, void *stream);
#define ICP_NOALLOC_SCRATCH_BYTES (64u << 20)

/* Automatic nu_min of a target set (Sec. 4.3 for point-to-point, Sec. 5 for
 * point-to-plane; rationale in App. C), the value a registration uses when
 * its params.nu_min <= 0: for every target its six nearest other targets
 * (exact FP32 squared distances, ties to the lower index); point-to-point
 * (mode ICP_P2P_WELSCH): the median over targets of the median of their
 * distances, Ebar, and nu_min = Ebar / (3 sqrt 3); point-to-plane (mode
 * ICP_P2PL_WELSCH, normals Qn required, used as given): the same with the
 * distances |n_i . (q_j - q_i)| to the tangent plane, Hbar, and
 * nu_min = Hbar / 6. Medians of n values are the element of rank n / 2.
 * Q, Qn: host AoS N x 3 FP32, N >= 7 (else ICP_ERR_INVALID_ARG). Synchronous. */
icp_status icp_nu_min_auto(icp_ctx *ctx, const float *Q, const float *Qn, int64_t N,
                           icp_mode mode, double *nu_min_out);

/* Normals of a point set for point-to-plane registration of targets given
 * without normals (the paper estimates them from 30 nearest neighbours): for
 * every point its 30 nearest points of the set, the point itself included
 * (exact FP32 squared distances, ties to the lower index); the FP64 mean and
 * covariance of the 30 (summed in that order); the unit eigenvector of the
 * smallest eigenvalue, oriented so that n . q <= 0 (towards a viewpoint at
 * the origin; the registration does not depend on the orientation).
 * Q: host AoS N x 3 FP32, N >= 30; normals_out: host N x 3 FP32. Synchronous. */
icp_status icp_estimate_normals(icp_ctx *ctx, const float *Q, int64_t N, float *normals_out);

/* Batched / served registration. Every request is validated first; on the
 * first invalid one nothing is queued and its status is returned. Then the
 * tickets are issued (tickets_out[i] receives a unique ticket) and each
 * request's arrays are copied into host memory the library owns and queued in
 * turn, all before the call returns (the caller may free its arrays at once).
 * A background scheduler admits queued requests when a slot and enough HBM
 * are free, advances all admitted pairs together (one pass per captured graph
 * node group) and retires them as they finish, so requests that arrive while
 * others run join in flight, and the first requests of a large submission
 * start while the later ones are being copied. */
icp_status icp_batch_submit(icp_ctx *ctx, const icp_request *reqs, int n, uint64_t *tickets_out);

/* icp_batch_submit with device-resident inputs: every request's P, Q (and Qn
 * for point-to-plane) are DEVICE pointers (AoS x,y,z FP32 in HBM of the
 * context's device), read in place by the request's setup; nothing is copied
 * through the host. The arrays must stay valid and unchanged until the
 * request's result has been handed out by icp_poll (or icp_batch_wait_all has
 * returned). `stream` (NULL = the null stream): the setups of these requests
 * wait for the work enqueued on it before this call, so a caller may submit
 * arrays its own kernels are still writing. Sizes and parameters are checked
 * as for icp_batch_submit (ICP_ERR_INVALID_ARG, ICP_ERR_NO_NORMALS; nothing is
 * queued then); coordinates are not read on the host, so non-finite values
 * are not detected. Results are bit-identical to the same requests submitted
 * with host arrays. */
icp_status icp_batch_submit_dev(icp_ctx *ctx, const icp_request *reqs, int n, uint64_t *tickets_out,
                                void *stream);

/* ICP_OK and the result (handed out exactly once), ICP_ERR_NOT_READY while
 * pending, ICP_ERR_OOM (once) for a request that can never fit the HBM budget
 * or whose host copy could not be allocated, ICP_ERR_DEVICE after a HIP
 * failure of the scheduler, ICP_ERR_UNKNOWN_TICKET otherwise. */
icp_status icp_poll(icp_ctx *ctx, uint64_t ticket, icp_result *out);

/* Block until every submitted request has finished (results stay pollable). */
icp_status icp_batch_wait_all(icp_ctx *ctx);

/* Scheduler knobs: passes per graph replay (>= 1) and the maximum number of
 * concurrently resident pairs (1..1024). */
icp_status icp_batch_config(icp_ctx *ctx, int passes_per_replay, int max_slots);

/* Work partition of the closest-point search, chosen per size bucket by the
 * autotuner. No value changes a result: the closest points (and so every
 * registration) are the same bit for bit under any valid setting; only the
 * time differs. */
typedef struct {
  int slice_min;        /* cluster search: candidate clusters per work slice at least, 1..64 (6) */
  float list_margin;    /* cluster search: margin of the reusable candidate lists as a fraction
                           of the median cluster radius, 0..1 (0.08) */
  int brute_clusters;   /* exhaustive search in the batch engine: clusters per work item,
                           1..4096 (8) */
  int brute_items;      /* exhaustive search of a single pair: work items per pass, 64..2^20 (8192) */
  int grid_per_cu;      /* synchronous calls: workgroups per compute unit of the persistent
                           search kernels, 1..64 (16) */
} icp_tuning;

/* One entry of the tuning table: requests with floor(log2 M) == m_bucket and
 * floor(log2 N) == n_bucket of this mode family (ICP_P2P_WELSCH stands for
 * the point-to-point modes, ICP_P2PL_WELSCH for the point-to-plane ones) and
 * search method (ICP_NN_BRUTE or ICP_NN_CLUSTER; AUTO resolves to BRUTE up to
 * 64e6 source x target pairs), run by the engine kind `batch` (0: the
 * synchronous calls, one pair on the GPU; 1: icp_batch_submit, pairs sharing
 * the GPU -- a partition that shortens one pair's latency can cost
 * throughput there). ms: the tuner's time for its test run (0 for an entry
 * set by hand). */
typedef struct {
  int m_bucket, n_bucket, mode, method, batch;
  icp_tuning tuning;
  double ms;
} icp_tuning_entry;

/* The built-in partition (the values in parentheses above). */
icp_status icp_tuning_default(icp_tuning *out);

/* The partition a request of this shape uses in the given engine kind (0
 * synchronous, 1 batch): the entry of its bucket, else the nearest tuned
 * bucket of the same family, method and engine kind within two octaves
 * (|dm| + |dn| <= 2), else the defaults. *found (may be NULL): 2 exact
 * bucket, 1 nearby bucket, 0 defaults. */
icp_status icp_tuning_lookup(icp_ctx *ctx, int64_t M, int64_t N, icp_mode mode,
                             icp_nn_method method, int batch, icp_tuning *out, int *found);

/* Add or replace the entry of a bucket (INVALID_ARG for values out of range). */
icp_status icp_tuning_set(icp_ctx *ctx, const icp_tuning_entry *entry);

/* Copy the table (up to cap entries) into out; *n receives its size. */
icp_status icp_tuning_entries(icp_ctx *ctx, icp_tuning_entry *out, int cap, int *n);

/* Search the partition for one bucket on the context's GPU: a synthetic
 * bumpy-sphere pair of M sources and N targets (70% overlap, 10% outliers;
 * radial normals for point-to-plane) is registered (at most 40 inner
 * iterations) under each candidate setting, each timed as the best of two
 * runs. batch = 0 (synchronous calls, the pair alone): cluster search
 * slice_min {4, 6, 8, 12} x list_margin {0.04, 0.08, 0.16} x grid_per_cu
 * {8, 16, 32}; exhaustive: brute_items {2048, 4096, 8192, 12288, 16384,
 * 24576, 32768} x grid_per_cu {8, 16, 32}. batch = 1 (16 copies of the pair at once through the batch
 * engine, fewer for large pairs: about 4e6 points in flight): cluster
 * search slice_min x list_margin as above; exhaustive:
 * brute_clusters {4, 8, 16, 32}. Every candidate must return the defaults'
 * transform bit for bit (ICP_ERR_DEVICE otherwise: a library fault). The
 * fastest is stored in the table and written to *best (may be NULL). Uses
 * the engines for its duration (a few seconds at 100k points); do not run it
 * while batch requests are being served. */
icp_status icp_autotune(icp_ctx *ctx, int64_t M, int64_t N, icp_mode mode, icp_nn_method method,
                        int batch, icp_tuning_entry *best);

/* Architecture name of a HIP device (gcnArchName up to the first ':', e.g.
 * "gfx950") into out (capacity cap bytes, NUL-terminated). */
icp_status icp_device_arch(int device, char *out, int cap);

/* Tuning cache files (JSON: {"arch": "...", "entries": [{"m_bucket": ..,
 * "n_bucket": .., "mode": .., "method": .., "batch": .., "slice_min": .., "list_margin":
 * .., "brute_clusters": .., "brute_items": .., "grid_per_cu": .., "ms": ..},
 * ...]}). Host-only: no device is needed. Write stores n entries under arch.
 * Read fills out (capacity cap) with the entries of a file whose arch equals
 * `arch` (*n = 0 for another arch; arch NULL accepts any);
 * ICP_ERR_INVALID_ARG for a missing or malformed file or an entry out of
 * range. icp_create loads the file named by the environment variable
 * ICP_TUNING_CACHE, else tuning_<arch>.json beside the library, when it
 * exists and holds this device's arch. */
icp_status icp_tuning_file_write(const char *path, const char *arch, const icp_tuning_entry *entries,
                                 int n);
icp_status icp_tuning_file_read(const char *path, const char *arch, icp_tuning_entry *out, int cap,
                                int *n);

/* Enable (1) or disable (0) per-pass kernel timing; resets the counters.
 * Applies to passes launched afterwards. */
icp_status icp_profile(icp_ctx *ctx, int enable);
icp_status icp_profile_read(icp_ctx *ctx, icp_profile_stats *out);

const char *icp_status_str(icp_status s);

#ifdef __cplusplus
}
#endif
#endif /* ICP_H */
