// Internal layout shared by the HIP translation units of libicp (never by the
// oracle). One "slot" is one registration (or one nearest-neighbour query)
// resident in HBM: its point sets, the cluster index over the target, the
// per-tile partial sums and the per-pair solver state.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace icp {

constexpr int kTile = 64;        // sources per NN work item (one wavefront)
constexpr int kCluster = 128;    // targets per cluster of the Hilbert-ordered index
constexpr int kChunk = 16;       // targets per deferred-argmin chunk
constexpr int kChunksPerCluster = kCluster / kChunk;
constexpr int kSuper = 16;       // clusters per super-cluster (coarse culling level)
constexpr int kEpiRows = 2;      // sources per thread of a reduction work item
constexpr int kEpiTile = 256 * kEpiRows;  // sources per reduction work item
constexpr int kPartStride = 32;  // doubles per reduction partial
constexpr int kHist = 8;         // Anderson ring capacity (m <= 6 needs m + 1)
constexpr int kCandCap = 1024;   // LDS candidate list capacity per NN work item
constexpr int kSupCap = 512;     // LDS candidate super-cluster capacity per NN work item
constexpr int kListCap = 512;    // candidate clusters stored per tile
constexpr int kMaxSlices = 64;   // slices per tile in cluster mode
// Long candidate sequences (lists whose length forced slices longer than
// kSliceMin under the kMaxSlices cap, and ranges over every cluster for tiles
// whose list would overflow) may be cut into up to kMaxLongSlices slices,
// drawing the slices beyond kMaxSlices from a per-pair budget of kExtraSlices.
constexpr int kMaxLongSlices = 1024;
constexpr int kExtraSlices = 8192;
// Defaults of the tunable work partition (each slot carries its own values,
// chosen per size bucket by the autotuner; none of them changes a result).
constexpr int kSliceMinDefault = 6;      // clusters per slice at least (cluster mode)
constexpr float kVerletFracDefault = 0.08f;  // candidate-list margin / median cluster radius
constexpr int kBruteClustersDefault = 8;     // clusters per exhaustive item (multi-slot engine)
constexpr int kBruteItemsDefault = 8192;     // exhaustive items per pass (one-slot engine)
constexpr int kGridPerCuDefault = 16;        // workgroups per CU of the persistent search kernels

// tile record flags (cull kernel -> slice kernel)
enum TileFlags { TI_WARM = 1, TI_LIST = 2, TI_RANGE = 4, TI_LANETEST = 8 };

enum Mode { P2P_L2 = 0, P2P_WELSCH = 1, P2PL_WELSCH = 2, P2PL_L2 = 3 };
// point-to-plane residuals (normals needed) / unit weights (no nu)
__host__ __device__ constexpr bool mode_plane(int m) { return m == P2PL_WELSCH || m == P2PL_L2; }
__host__ __device__ constexpr bool mode_l2(int m) { return m == P2P_L2 || m == P2PL_L2; }
enum NNMethod { NN_AUTO = 0, NN_BRUTE = 1, NN_CLUSTER = 2 };
enum SlotStatus { ST_FREE = 0, ST_SETUP = 1, ST_RUNNING = 2, ST_DONE = 3 };

// Solver state-machine positions.
enum SmPos {
  SM_INIT = 0,         // evaluation at T0 done (setup pass)
  SM_STAGE_EVAL = 1,   // evaluation at T^(k-1) with the stage's nu
  SM_ITER_EVAL = 2,    // evaluation at T^(k)
  SM_REVERT_EVAL = 3,  // point-to-point: evaluation at the un-accelerated T'
  SM_LS_EVAL = 4,      // point-to-plane: line-search trial
  SM_QUERY = 5,        // plain nearest-neighbour query: one pass, then done
  SM_EVAL = 6          // one application of the un-accelerated map, then done
};

enum Flags : unsigned {
  F_CONVERGED = 1u, F_MAX_ITER = 2u, F_ZERO_WEIGHT = 4u, F_DEGENERATE = 8u, F_AA_SINGULAR = 16u
};

// Partial-sum layout (doubles) written per reduction tile.
// point-to-point: [0]=E [1]=W [2..4]=sum w p~ [5..7]=sum w q~ [8..16]=sum w p~ q~^T
// point-to-plane: [0]=E [1]=W [2..22]=A upper (row-major i<=j) [23..28]=c
constexpr int kP2PVals = 17;
constexpr int kP2PLVals = 29;

// Static description of a slot (written once at admission).
struct SlotDesc {
  // sources, Hilbert-ordered SoA (original FP32 values)
  const float* px;
  const float* py;
  const float* pz;
  const int* perm;            // sorted position -> original source index
  const double4* tsph;        // per tile: centre (x,y,z) and radius
  // targets, original order SoA (+ normals)
  const float* qx;
  const float* qy;
  const float* qz;
  const float* nx;
  const float* ny;
  const float* nz;
  // cluster index (Hilbert order, kCluster targets per cluster, padded)
  const float4* qloc;         // (x - cc, y - cc, z - cc, |q - cc|^2 / 2), padding h = +inf
  const float4* qorg;         // (x, y, z, bits(original index)), padding index = -1
  const float4* ccen;         // cluster centre (x, y, z) and radius
  const float4* clo;          // cluster AABB min
  const float4* chi;          // cluster AABB max
  const float4* kbox;         // per chunk of kChunk targets: AABB min, AABB max (2 entries)
  const float4* slo;          // super-cluster AABB min
  const float4* shi;          // super-cluster AABB max
  unsigned long long* keys;   // per sorted source: (bits(d2) << 32) | index, merged by atomic min
  int* clist;                 // per tile: kListCap candidate cluster ids
  int4* squeue;               // slices queued by the cull kernel: (tile, first list
                              // position, end position, flags | (nearest cluster + 1) << 4)
  int* scount;                // [0] queued slices, [1] extra slices granted (reset by the planner)
  int32_t* nnidx;             // per sorted source: closest original target index
  float* nnd2;                // per sorted source: its FP32 squared distance
  double* part;               // nepi x kPartStride
  double* medkey;             // per sorted source (setup pass only)
  int32_t* idx_out;           // optional: original-order outputs (queries)
  float* d2_out;
  unsigned long long* stats;  // kQueues lines of kStatStride: [0] pairs through the
                              // filter, [1] pairs scanned exactly (summed on the host)
  double* trace;              // optional per-pass rows [E, nu, sm, reuse, T(16), prop(16)]
  int* item_stats;            // optional, last pass: per NN work item
                              // [cycles, clusters filtered, candidates, flags]
  int trace_cap;
  int M, N, ntile, ncl, nsup, nepi;
  int method;                 // NN_BRUTE or NN_CLUSTER
  int mode;
  int slice_min;              // clusters per slice at least (cluster search)
  int brute_clusters;         // clusters per exhaustive item (multi-slot engine)
  int brute_items;            // exhaustive items per pass (one-slot engine)
  float rho_max;              // max cluster radius (upper bound)
  float verlet;               // candidate-list margin: lists built with this
                              // slack stay valid while no source moves farther
};

// Per-slot mutable state (device resident; the solver wave owns it).
struct SlotState {
  // ---- evaluation request, read by the NN and reduction kernels
  double Teval[16];
  double K[27 + 9 + 9];       // point-to-plane: dR/d delta_j (3x3 x3), dt/d delta, dt/du
  double inv2nu2;             // 1 / (2 nu^2) of the evaluation (0 for L2)
  double nu_eval;             // nu of the evaluation (0 for L2)
  int reuse;                  // 1: same transform as the previous pass, skip the NN search
  int want_median;            // 1: this pass also writes median keys
  int status;                 // SlotStatus
  int sm;                     // SmPos
  // ---- parameters
  int mode, m, lmax, iter_first, iter_inc, iter_cap, max_total;
  int nu_auto;
  double eps, nu_min, nu_max;
  // ---- algorithm state
  int k, kstart, stage, total, Inu, is_aa, ls_l;
  double nu, Eprev, Eit, tau;
  double Tk[16], Tp[16], Tkm1[16];
  double xk[6], xkm1[6], xstar[6], xt[6];
  double best_prop[6];
  unsigned best_flags;
  double G[kHist][6], F[kHist][6];
  double last_key[16];
  int have_last;
  double median;              // written by the median kernel
  double cP[3], cQ[3];        // fixed centring of the moments (bbox centres)
  double Tref[16];            // transform of the last candidate-list build
  double Vq[16];              // eigenbasis of the last quaternion alignment (warm start)
  double lk[6];               // point-to-point with mixing: log of the current iterate Tk
  double verlet;              // list margin (copied from the descriptor at boot)
  int cull;                   // 1: this pass rebuilds the candidate lists
  int cull_pad;
  float bbP[6], bbQ[6];       // bounding boxes (min xyz, max xyz)
  // ---- results
  double Tres[16];
  double energy, nu_final;
  int iterations, nn_passes, evaluations, aa_accepted, aa_rejected, ls_trials, stages;
  unsigned flags;
  int phases;
  int trace_len;
};

constexpr int kQueues = 8;
// sub-queues of the slice queue: a multiple of kQueues, so that sub-queue x
// is served by the workgroups of die x mod kQueues only
constexpr int kSliceQueues = 8;
constexpr int kQueueStride = 64;  // ints between sub-queue counters
constexpr int kStatStride = 32;  // u64 between per-die statistics lines

// Closest-point key: the FP32 squared distance's bits above the target
// index, so that the integer minimum is the lexicographic (d2, index) minimum.
__device__ __forceinline__ unsigned long long make_key(float d2, int idx) {
  return ((unsigned long long)__float_as_uint(d2) << 32) | (unsigned)idx;
}

// Squared distance from a point to an axis-aligned box (0 inside); every
// member of the box is at exact squared distance at least this (up to the
// rounding of this expression, which callers allow for).
__device__ __forceinline__ float box_lb2(float px, float py, float pz, float4 lo, float4 hi) {
  const float dx = fmaxf(fmaxf(lo.x - px, px - hi.x), 0.0f);
  const float dy = fmaxf(fmaxf(lo.y - py, py - hi.y), 0.0f);
  const float dz = fmaxf(fmaxf(lo.z - pz, pz - hi.z), 0.0f);
  return dx * dx + dy * dy + dz * dz;
}

// Active-slot work lists rebuilt before every phase.
struct WorkList {
  int n_active;
  int nn_total;
  int epi_total;
  int s_total;                // closest-point slices queued this pass
  int single;                 // 1: one-slot engine, planned by the solver itself
  int s_from_scount;          // 1: the slice total is the slot's slice count
  int slot[1024];             // compacted active slot ids
  int nn_base[1025];          // prefix of NN items over the compacted list
  int epi_base[1025];
  int s_base[1025];           // prefix of queued slices over the compacted list
  int b_total;                // exhaustive-method items this pass (multi-slot engine)
  int b_base[1025];           // prefix of exhaustive-method items over the compacted list
  // dynamic work counters (reset by the planners): kQueues sub-queues each
  int q_nn[kQueues * kQueueStride];
  int q_epi[kQueues * kQueueStride];
  int q_s[kSliceQueues * kQueueStride];
  int q_b[kQueues * kQueueStride];  // exhaustive-method items (multi-slot engine)
};

// Exhaustive method in the multi-slot engine: one item = a pair of 64-source
// tiles against a range of about cpi clusters (the slot's brute_clusters).
__host__ __device__ inline int brute_split(int ncl, int cpi) {
  return ncl > 0 ? (ncl + cpi - 1) / cpi : 1;
}
__host__ __device__ inline long long brute_items64(int ntile, int ncl, int cpi) {
  return (long long)((ntile + 1) / 2) * (long long)brute_split(ncl, cpi);
}
// Items of one pair in the multi-slot engine are capped so that the planner's
// int prefix over kMaxSlots pairs cannot overflow (1024 x 2^20 < 2^31); a pair
// beyond the cap is searched with the cluster method, whose result is the same.
constexpr long long kMaxBruteItemsPerPair = 1ll << 20;
__host__ __device__ inline int brute_items(int ntile, int ncl, int cpi) {
  return (int)brute_items64(ntile, ncl, cpi);
}

// Element i of a device array through a global-address-space pointer. The
// descriptor's pointers are generic, and generic loads also hold the LDS
// counter, so that waiting for LDS data would wait for them too; global loads
// count only against the vector memory counter.
template <class T>
__device__ __forceinline__ T ldg(const T* p, size_t i) {
  return ((const __attribute__((address_space(1))) T*)p)[i];
}

// LDS written by some lanes of a wavefront and read by others: a wavefront's
// LDS operations complete in order, so a compiler fence is all it needs.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Work distribution of the persistent kernels. Workgroup b takes item b first
// without an atomic; later items come from kQueues sub-queues, sub-queue
// b mod kQueues serving the items gridDim + x + kQueues k. The hardware deals
// workgroups to its dies in this order, and each counter sits on its own
// 256-byte line, so the counters' atomics do not serialise on one address.
__device__ __forceinline__ int queue_item(int* q, int round) {
  if (round == 0) return (int)blockIdx.x;
  const int x = (int)(blockIdx.x % kQueues);
  return (int)gridDim.x + x + kQueues * atomicAdd(&q[x * kQueueStride], 1);
}

// Slice queue of the closest-point search. Items are queued tile by tile and
// tiles follow the Hilbert order of the sources, so consecutive items need
// nearby clusters. Sub-queue x (the workgroups on die x, blockIdx mod
// kQueues == x) serves runs of kSliceRun consecutive items, runs x, x +
// kQueues, x + 2 kQueues, ...: each die's L2 then sees a run's clusters
// several times instead of every die fetching them for interleaved single
// items, while the fine interleave of runs keeps the dies' shares of work
// equal. Workgroup b takes position b / kQueues of its sub-queue without an
// atomic, later positions come from counter x; positions map to items in
// increasing order, so a sub-queue is used up at its first item >= total.
constexpr int kSliceRun = 16;

__device__ __forceinline__ int slice_queue_item(int* q, int total, int round) {
  static_assert(kSliceQueues % kQueues == 0, "every slice sub-queue belongs to one die");
  const int x = (int)(blockIdx.x % kSliceQueues);
  const int nb = ((int)gridDim.x - x + kSliceQueues - 1) / kSliceQueues;  // workgroups of sub-queue x
  const int k = round == 0 ? (int)(blockIdx.x / kSliceQueues) : nb + atomicAdd(&q[x * kQueueStride], 1);
  const long long item = ((long long)(k / kSliceRun) * kSliceQueues + x) * kSliceRun + (k % kSliceRun);
  return item < total ? (int)item : total;
}

constexpr int kMaxSlots = 1024;

// Compacted-list index of work item g: the largest a < n with base[a] <= g
// (base is a nondecreasing prefix with base[0] = 0 <= g). The wavefront
// probes 64 evenly spaced entries, then the entries between the last probe
// that qualifies and the next: two memory round trips for n <= 4096, where a
// bisection takes one per step. Called by all 64 lanes of a wavefront with
// uniform arguments; returns a uniform value.
__device__ __forceinline__ int wave_find_slot(const int* __restrict__ base, int n, int g) {
  static_assert(kMaxSlots <= 64 * 64, "two probe levels cover the compacted list");
  if (n <= 1) return 0;
  const int lane = (int)(threadIdx.x & 63);
  const int step = (n + 63) >> 6;
  int i = lane * step;
  unsigned long long m = __builtin_amdgcn_ballot_w64(i < n && ldg(base, i) <= g);
  int lo = (63 - __builtin_clzll(m)) * step;  // lane 0 probes base[0] <= g
  if (step > 1) {
    i = lo + lane;
    m = __builtin_amdgcn_ballot_w64(lane < step && i < n && ldg(base, i) <= g);
    lo += 63 - __builtin_clzll(m);
  }
  return __builtin_amdgcn_readfirstlane(lo);
}
// trace row: [E, nu, solver position, reuse, T_eval (16), proposal (16)]
constexpr int kTraceRow = 36;

}  // namespace icp
