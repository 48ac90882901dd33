// Host runtime of libicp: HBM arena, slot admission (device-side setup on a
// side stream), the per-pass launch sequence, the plain host-synchronised loop,
// the hipGraph replay loop and the background scheduler that serves batched
// requests with continuous admission. Exposes the C ABI of include/icp.h.
#include <hip/hip_runtime.h>

#include <dlfcn.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "icp.h"
#include "icp_internal.h"

namespace icp {

// kernels launched from the other translation units
void launch_nn(const SlotDesc*, const SlotState*, WorkList*, int, bool, hipStream_t);
void launch_brute(const SlotDesc*, const SlotState*, int, hipStream_t);
void launch_epi(const SlotDesc*, const SlotState*, WorkList*, int, bool, hipStream_t);
void launch_solver(const SlotDesc*, SlotState*, int, int*, WorkList*, bool, hipStream_t, int, int);
void launch_boot(const SlotDesc*, SlotState*, int, WorkList*, bool, hipStream_t);
void launch_median(const SlotDesc*, SlotState*, int, hipStream_t, int, int);
void launch_estimate_normals(const float4*, const float4*, const float4*, const float4*, const float4*,
                             int, int, const float*, const float*, const float*, float*, hipStream_t);
void launch_nu_min_auto(const float4*, const float4*, const float4*, const float4*, const float4*, int,
                        int, const float*, const float*, const float*, const float*, const float*,
                        const float*, int, bool, double*, double*, hipStream_t);
void launch_plan(const SlotDesc*, const SlotState*, WorkList*, int, hipStream_t, int, int);
void launch_aos_to_soa(const float*, int, float*, float*, float*, hipStream_t);
void launch_bbox(const float*, const float*, const float*, int, float*, double*, hipStream_t);
size_t sort_scratch_words(int);
void launch_hilbert_order(const float*, const float*, const float*, int, const float*, unsigned*,
                          unsigned**, hipStream_t);
void launch_build_clusters(const float*, const float*, const float*, const unsigned*, int, int,
                           float4*, float4*, float4*, float4*, float4*, float4*, hipStream_t);
void launch_build_super(const float4*, const float4*, const float4*, int, int, float4*, float4*,
                        float*, float, hipStream_t);
void launch_build_tiles(const float*, const float*, const float*, const unsigned*, int, int, float*,
                        float*, float*, int*, double4*, hipStream_t);
void launch_fill_u64(unsigned long long*, int, unsigned long long, hipStream_t);

using Clock = std::chrono::steady_clock;

#define HIP_OK(x)                         \
  do {                                    \
    if ((x) != hipSuccess) return false;  \
  } while (0)

// ------------------------------------------------------------------ arena

// First-fit allocator over one hipMalloc'd region (256-byte granules).
class Arena {
 public:
  bool init(size_t bytes) {
    size_ = bytes;
    if (hipMalloc(&base_, bytes) != hipSuccess) { base_ = nullptr; return false; }
    free_[0] = bytes;
    return true;
  }
  ~Arena() { if (base_) (void)hipFree(base_); }
  // returns nullptr when no block is large enough
  char* alloc(size_t bytes) {
    std::lock_guard<std::mutex> g(mu_);
    bytes = (bytes + 255) & ~size_t(255);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const size_t off = it->first, sz = it->second;
        free_.erase(it);
        if (sz > bytes) free_[off + bytes] = sz - bytes;
        used_[off] = bytes;
        in_use_ += bytes;
        return base_ + off;
      }
    }
    return nullptr;
  }
  void release(char* p) {
    std::lock_guard<std::mutex> g(mu_);
    const size_t off = p - base_;
    auto u = used_.find(off);
    if (u == used_.end()) return;
    size_t sz = u->second;
    const size_t orig = sz;
    used_.erase(u);
    in_use_ -= sz;
    size_t start = off;
    auto nx = free_.lower_bound(off);
    if (nx != free_.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == off) { start = pv->first; sz += pv->second; free_.erase(pv); }
    }
    nx = free_.lower_bound(off);
    if (nx != free_.end() && nx->first == off + orig) { sz += nx->second; free_.erase(nx); }
    free_[start] = sz;
  }
  size_t capacity() const { return size_; }

 private:
  char* base_ = nullptr;
  size_t size_ = 0, in_use_ = 0;
  std::map<size_t, size_t> free_, used_;
  std::mutex mu_;
};

// ------------------------------------------------------------------ slot memory

static inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

struct Layout {
  int M, N, ntile, ncl, nsup, nepi;
  bool normals, outputs;
  size_t total = 0;
  // byte offsets
  size_t o_px, o_py, o_pz, o_perm, o_tsph, o_pox, o_poy, o_poz;
  size_t o_qx, o_qy, o_qz, o_nx, o_ny, o_nz;
  size_t o_qloc, o_qorg, o_ccen, o_clo, o_chi, o_kbox, o_slo, o_shi;
  size_t o_clist, o_squeue, o_scount;
  size_t o_keys, o_nnidx, o_nnd2, o_part, o_med, o_idx, o_d2, o_scratch, o_trace, o_stats, o_items;
  int trace_cap = 0;
  size_t add(size_t bytes) {
    const size_t o = total;
    total += (bytes + 255) & ~size_t(255);
    return o;
  }
  void plan(int64_t m, int64_t n, bool nrm, bool outs, int tcap = 0) {
    M = (int)m; N = (int)n;
    trace_cap = tcap;
    normals = nrm; outputs = outs;
    ntile = cdiv(M, kTile);
    ncl = cdiv(N, kCluster);
    nsup = cdiv(ncl, kSuper);
    nepi = cdiv(M, kEpiTile);
    total = 0;
    o_px = add(4ull * M); o_py = add(4ull * M); o_pz = add(4ull * M);
    o_perm = add(4ull * M);
    o_tsph = add(32ull * ntile);
    o_pox = add(4ull * M); o_poy = add(4ull * M); o_poz = add(4ull * M);
    o_qx = add(4ull * N); o_qy = add(4ull * N); o_qz = add(4ull * N);
    o_nx = add(nrm ? 4ull * N : 0); o_ny = add(nrm ? 4ull * N : 0); o_nz = add(nrm ? 4ull * N : 0);
    o_qloc = add(16ull * ncl * kCluster);
    o_qorg = add(16ull * ncl * kCluster);
    o_ccen = add(16ull * ncl); o_clo = add(16ull * ncl); o_chi = add(16ull * ncl);
    o_kbox = add(32ull * ncl * kChunksPerCluster);
    o_slo = add(16ull * nsup); o_shi = add(16ull * nsup);
    o_keys = add(8ull * M);
    o_clist = add(4ull * kListCap * ntile);
    o_squeue = add(16ull * ((size_t)kMaxSlices * ntile + kExtraSlices));
    o_scount = add(16);
    o_nnidx = add(4ull * M);
    o_nnd2 = add(4ull * M);
    o_part = add(8ull * kPartStride * nepi);
    o_med = add(8ull * M);
    o_idx = add(outs ? 4ull * M : 0);
    o_d2 = add(outs ? 4ull * M : 0);
    const size_t sw = std::max(sort_scratch_words(std::max(M, N)) * 4, (size_t)12 * std::max(M, N));
    o_scratch = add(sw);
    o_trace = add(8ull * kTraceRow * tcap);
    o_stats = add(8ull * kQueues * kStatStride);
    o_items = add(tcap > 0 ? 32ull * ntile * kMaxSlices : 0);
  }
};

struct HostSlot {
  bool used = false;
  bool want_median = false;   // the first pass computes the median
  char* mem = nullptr;
  Layout L;
  uint64_t ticket = 0;
  Clock::time_point t_submit;
  int32_t* user_idx = nullptr;  // host outputs of a query (copied at harvest)
  float* user_d2 = nullptr;
  // host sources of the admission's asynchronous uploads (they must outlive
  // the copies, which may still be in flight when admit returns)
  SlotState S0;
  SlotDesc D0;
  int zero = 0;
};

// ------------------------------------------------------------------ requests

// An event recorded on a caller's stream, shared by the requests of one
// submission and destroyed with the last of them.
struct ReadyEvent {
  hipEvent_t ev = nullptr;
  ~ReadyEvent() {
    if (ev) (void)hipEventDestroy(ev);
  }
};

struct OwnedRequest {
  std::vector<float> P, Q, Qn;  // host copies (batch path)
  const float* P_dev = nullptr;  // device AoS inputs (dev path)
  const float* Q_dev = nullptr;
  const float* Qn_dev = nullptr;
  int64_t M = 0, N = 0;
  icp_params prm{};
  bool query = false;
  bool eval = false;   // one application of the MM map (icp_eval)
  bool numin_only = false;  // only the automatic nu_min of the targets (icp_nu_min_auto)
  double Tq[16];
  icp_nn_method qmethod = ICP_NN_AUTO;
  int32_t* idx_dev_out = nullptr;  // device outputs for a dev query
  float* d2_dev_out = nullptr;
  int trace_cap = 0;               // per-pass trace rows kept on the device
  icp_tuning tune{kSliceMinDefault, kVerletFracDefault, kBruteClustersDefault, kBruteItemsDefault,
                  kGridPerCuDefault};    // work partition of this request (no effect on results)
  bool tune_fixed = false;         // tune set by the caller (autotuner), not looked up
  // device inputs of a batch submission: the caller's stream position at the
  // submission, which the setup waits for before reading the arrays
  std::shared_ptr<struct ReadyEvent> ready;
  uint64_t ticket = 0;
  Clock::time_point t_submit;
};

// The search method a request runs: AUTO takes the exhaustive scan up to
// 64e6 source x target pairs.
static icp_nn_method resolve_method(int64_t M, int64_t N, icp_nn_method m) {
  if (m == ICP_NN_AUTO) return ((double)M * (double)N <= 64.0e6) ? ICP_NN_BRUTE : ICP_NN_CLUSTER;
  return m;
}

// nu_min <= 0 selects the automatic rule for the Welsch modes.
static bool auto_nu_min(const icp_params* p) { return !mode_l2(p->mode) && !(p->nu_min > 0.0); }

// Closest-point work counters of a slot (per-die statistics lines).
static void stats_from(const unsigned long long* v, icp_result* r) {
  double a = 0.0, b = 0.0;
  for (int q = 0; q < kQueues; ++q) {
    a += (double)v[q * kStatStride];
    b += (double)v[q * kStatStride + 1];
  }
  r->nn_pairs = a;
  r->nn_exact_pairs = b;
}

// Setup streams of the batch engine (HIP maps streams onto a few hardware
// queues; a handful suffices to overlap the short setup kernels of many
// requests).
constexpr int kSetupStreams = 4;

static void fill_stats(const HostSlot& h, hipStream_t st, icp_result* r) {
  unsigned long long v[kQueues * kStatStride] = {};
  if (h.mem && hipMemcpyAsync(v, h.mem + h.L.o_stats, sizeof v, hipMemcpyDeviceToHost, st) == hipSuccess &&
      hipStreamSynchronize(st) == hipSuccess)
    stats_from(v, r);
}

static void fill_result(const SlotState& S, icp_result* r) {
  std::memcpy(r->T, S.Tres, sizeof r->T);
  r->energy = S.energy;
  r->nu_final = S.nu_final;
  r->iterations = S.iterations;
  r->nn_passes = S.nn_passes;
  r->evaluations = S.evaluations;
  r->aa_accepted = S.aa_accepted;
  r->aa_rejected = S.aa_rejected;
  r->line_search_trials = S.ls_trials;
  r->stages = S.stages;
  r->status_flags = S.flags;
}

// ------------------------------------------------------------------ engine

// Branches of the multi-slot engine: slot s belongs to branch s mod
// kBranches, each branch with its own work list, and a replay runs the
// branches' passes as parallel chains (the second on its own stream), so that
// one branch's reduction, solver and planning overlap the other's search.
constexpr int kBranches = 2;

struct Engine {
  int dev = 0;
  int capacity = 1;
  bool single = false;       // one slot at a time, planned by its own solver
  int nbr = 1;               // branches (kBranches for the multi-slot engine)
  hipStream_t st2 = nullptr;  // the second branch's passes inside a replay
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool brute = false;        // one-slot engine: the resident pair uses the exhaustive method
  hipStream_t st = nullptr;  // passes
  hipStream_t side = nullptr;  // admission / setup (the first of `sides`)
  // Setup streams: slot s is set up on sides[s % sides.size()], so that the
  // setups of a large admission (a few hundred short kernels per request)
  // run side by side instead of one request after another.
  std::vector<hipStream_t> sides;
  hipStream_t setup_stream(int s) const { return sides[(size_t)s % sides.size()]; }
  // Uploads of the admission. Host arrays are pageable, and a pageable copy
  // returns only once it has run, so on their own stream the host waits for
  // the copy itself, not for the setup kernels queued before it on `side`.
  hipStream_t up = nullptr;
  hipEvent_t up_done = nullptr;
  SlotDesc* d_desc = nullptr;
  SlotState* d_state = nullptr;
  WorkList* d_wl = nullptr;
  int* d_done = nullptr;
  int* h_done = nullptr;
  // pinned landing buffers of the batch retirement (all finished slots of a
  // round are read back with one synchronisation) and its reset values
  SlotState* h_fin_state = nullptr;
  unsigned long long* h_fin_stats = nullptr;  // kQueues * kStatStride per slot
  int* h_reset = nullptr;                     // {0, ST_FREE}
  std::vector<HostSlot> hs;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  int gphases = 0;
  int gcap = 0;
  bool gprof = false;
  bool gbrute = false;
  int nn_grid = 4096, epi_grid = 1024;
  int cus = 256;
  int gnn_grid = 0;          // search grid the captured graph was built with
  Arena* arena = nullptr;
  // profiling: timing events around the kernels of every pass. `prof` is
  // read and written only by the thread that enqueues this engine's passes
  // (the caller under the context's sync lock for the one-slot engine; the
  // scheduler, which copies `prof_req` at the start of each round under the
  // context lock, for the batch engine), so that a round's passes and their
  // collection agree even when profiling is switched meanwhile.
  bool prof = false;
  bool prof_req = false;
  std::vector<hipEvent_t> pev;  // 4 per pass
  double prof_ms[3] = {0.0, 0.0, 0.0};  // closest point, reduction, median + solver
  long long prof_passes = 0;

  bool init(int device, int cap, Arena* a) {
    dev = device;
    capacity = cap;
    arena = a;
    HIP_OK(hipSetDevice(dev));
    HIP_OK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    nbr = single ? 1 : kBranches;
    if (nbr > 1) {
      HIP_OK(hipStreamCreateWithFlags(&st2, hipStreamNonBlocking));
      HIP_OK(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming));
      HIP_OK(hipEventCreateWithFlags(&ev_join, hipEventDisableTiming));
    }
    sides.assign(single ? 1 : kSetupStreams, nullptr);
    for (auto& x : sides) HIP_OK(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
    side = sides[0];
    HIP_OK(hipStreamCreateWithFlags(&up, hipStreamNonBlocking));
    HIP_OK(hipEventCreateWithFlags(&up_done, hipEventDisableTiming));
    HIP_OK(hipMalloc(&d_desc, sizeof(SlotDesc) * kMaxSlots));
    HIP_OK(hipMalloc(&d_state, sizeof(SlotState) * kMaxSlots));
    HIP_OK(hipMalloc(&d_wl, sizeof(WorkList) * nbr));
    HIP_OK(hipMalloc(&d_done, sizeof(int) * kMaxSlots));
    HIP_OK(hipHostMalloc((void**)&h_done, sizeof(int) * kMaxSlots, hipHostMallocDefault));
    HIP_OK(hipHostMalloc((void**)&h_fin_state, sizeof(SlotState) * kMaxSlots, hipHostMallocDefault));
    HIP_OK(hipHostMalloc((void**)&h_fin_stats, 8ull * kQueues * kStatStride * kMaxSlots, hipHostMallocDefault));
    HIP_OK(hipHostMalloc((void**)&h_reset, 2 * sizeof(int), hipHostMallocDefault));
    h_reset[0] = 0;
    h_reset[1] = ST_FREE;
    HIP_OK(hipMemset(d_desc, 0, sizeof(SlotDesc) * kMaxSlots));
    HIP_OK(hipMemset(d_state, 0, sizeof(SlotState) * kMaxSlots));
    HIP_OK(hipMemset(d_done, 0, sizeof(int) * kMaxSlots));
    HIP_OK(hipMemset(d_wl, 0, sizeof(WorkList) * nbr));
    std::memset(h_done, 0, sizeof(int) * kMaxSlots);
    hs.assign(kMaxSlots, HostSlot());
    int cus = 256;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
      cus = prop.multiProcessorCount;
    nn_grid = cus * kGridPerCuDefault;
    epi_grid = cus * 4;
    this->cus = cus;
    return true;
  }

  void destroy() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr; graph = nullptr;
    for (auto& h : hs)
      if (h.used && h.mem) arena->release(h.mem);
    for (auto e : pev) (void)hipEventDestroy(e);
    pev.clear();
    if (d_desc) (void)hipFree(d_desc);
    if (d_state) (void)hipFree(d_state);
    if (d_wl) (void)hipFree(d_wl);
    if (d_done) (void)hipFree(d_done);
    if (h_done) (void)hipHostFree(h_done);
    if (h_fin_state) (void)hipHostFree(h_fin_state);
    if (h_fin_stats) (void)hipHostFree(h_fin_stats);
    if (h_reset) (void)hipHostFree(h_reset);
    h_fin_state = nullptr; h_fin_stats = nullptr; h_reset = nullptr;
    if (st) (void)hipStreamDestroy(st);
    if (st2) (void)hipStreamDestroy(st2);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    st2 = nullptr; ev_fork = nullptr; ev_join = nullptr;
    for (auto& x : sides)
      if (x) (void)hipStreamDestroy(x);
    sides.clear();
    if (up) (void)hipStreamDestroy(up);
    if (up_done) (void)hipEventDestroy(up_done);
    d_desc = nullptr; d_state = nullptr; d_wl = nullptr; d_done = nullptr; h_done = nullptr;
    st = nullptr; side = nullptr; up = nullptr; up_done = nullptr;
  }

  bool ensure_events(int passes) {
    while ((int)pev.size() < 4 * passes * nbr) {
      hipEvent_t e;
      HIP_OK(hipEventCreate(&e));
      pev.push_back(e);
    }
    return true;
  }

  // capturing: the events become event-record nodes of the graph
  void mark(int k, hipStream_t s, bool capturing) {
    if (!prof) return;
    if (capturing) (void)hipEventRecordWithFlags(pev[k], s, hipEventRecordExternal);
    else (void)hipEventRecord(pev[k], s);
  }

  // One pass of branch b (the one-slot engine: its single slot). The one-slot
  // engine is planned by its solver (and boot) kernel, so a pass is cull,
  // slices, reduction, solver, with the median only on the pass that needs it
  // (the first); the multi-slot engine plans the branch's work lists on the
  // device and runs the median kernel every pass (it returns at once for
  // slots that do not need it). Timing events 4 k .. 4 k + 3.
  void enqueue_branch(hipStream_t s, int b, int k, bool capturing, bool median) {
    if (!single) launch_plan(d_desc, d_state, d_wl + b, capacity, s, b, nbr);
    mark(4 * k, s, capturing);
    // the one-slot engine's exhaustive method needs no cull pass
    if (single && brute) launch_brute(d_desc, d_state, nn_grid, s);
    else launch_nn(d_desc, d_state, d_wl + b, nn_grid, single, s);
    mark(4 * k + 1, s, capturing);
    launch_epi(d_desc, d_state, d_wl + b, epi_grid, single, s);
    mark(4 * k + 2, s, capturing);
    if (!single || median) launch_median(d_desc, d_state, capacity, s, b, nbr);
    launch_solver(d_desc, d_state, capacity, d_done, d_wl + b, single, s, b, nbr);
    mark(4 * k + 3, s, capturing);
  }

  // One pass of every branch, the branches one after another on stream s
  // (the form with timing events).
  void enqueue_pass(hipStream_t s, int i = 0, bool capturing = false, bool median = false) {
    for (int b = 0; b < nbr; ++b) enqueue_branch(s, b, i * nbr + b, capturing, median);
  }

  // after the stream has been synchronised
  // Per pass, the sums over its branches.
  void collect_profile(int passes) {
    if (!prof) return;
    for (int i = 0; i < passes; ++i) {
      double sum[3] = {0.0, 0.0, 0.0};
      bool ok = true;
      for (int br = 0; br < nbr && ok; ++br) {
        const int k = i * nbr + br;
        float a = 0.f, b = 0.f, c = 0.f;
        ok = hipEventElapsedTime(&a, pev[4 * k], pev[4 * k + 1]) == hipSuccess &&
             hipEventElapsedTime(&b, pev[4 * k + 1], pev[4 * k + 2]) == hipSuccess &&
             hipEventElapsedTime(&c, pev[4 * k + 2], pev[4 * k + 3]) == hipSuccess;
        sum[0] += a;
        sum[1] += b;
        sum[2] += c;
      }
      if (ok) {
        for (int j = 0; j < 3; ++j) prof_ms[j] += sum[j];
        prof_passes++;
      } else {
        (void)hipGetLastError();  // do not leave a timing failure as the sticky error
      }
    }
  }

  bool build_graph(int phases) {
    if (gexec && gphases == phases && gcap == capacity && gprof == prof && gbrute == brute &&
        gnn_grid == nn_grid)
      return true;
    if (prof && !ensure_events(phases)) return false;
    if (gexec) { (void)hipGraphExecDestroy(gexec); gexec = nullptr; }
    if (graph) { (void)hipGraphDestroy(graph); graph = nullptr; }
    HIP_OK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    if (nbr == 1) {
      for (int i = 0; i < phases; ++i) enqueue_pass(st, i, true);
    } else {
      // the two branches' passes as parallel chains of the graph
      static_assert(kBranches == 2, "one extra stream per branch beyond the first");
      HIP_OK(hipEventRecord(ev_fork, st));
      HIP_OK(hipStreamWaitEvent(st2, ev_fork, 0));
      for (int i = 0; i < phases; ++i) enqueue_branch(st, 0, 2 * i, true, false);
      for (int i = 0; i < phases; ++i) enqueue_branch(st2, 1, 2 * i + 1, true, false);
      HIP_OK(hipEventRecord(ev_join, st2));
      HIP_OK(hipStreamWaitEvent(st, ev_join, 0));
    }
    HIP_OK(hipStreamEndCapture(st, &graph));
    HIP_OK(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
    gphases = phases;
    gcap = capacity;
    gprof = prof;
    gbrute = brute;
    gnn_grid = nn_grid;
    return true;
  }

  // A free slot of the branch with the fewest resident slots (then the next
  // fewest), lowest index first.
  int free_slot() const {
    int cnt[kBranches] = {};
    for (int i = 0; i < capacity; ++i)
      if (hs[i].used) cnt[i % nbr]++;
    bool tried[kBranches] = {};
    for (int t = 0; t < nbr; ++t) {
      int b = -1;
      for (int c = 0; c < nbr; ++c)
        if (!tried[c] && (b < 0 || cnt[c] < cnt[b])) b = c;
      tried[b] = true;
      for (int i = b; i < capacity; i += nbr)
        if (!hs[i].used) return i;
    }
    return -1;
  }

  static size_t footprint(const OwnedRequest& r) {
    Layout L;
    L.plan(r.M, r.N, mode_plane(r.prm.mode), r.query && !r.idx_dev_out);
    return L.total;
  }

  // Device-side setup of slot `s` for request r on the side stream. Returns
  // false on a HIP error; OOM is reported through *oom. Without `sync` the
  // setup may still be running on return: r's host arrays must then stay
  // alive until the side stream (or a stream waiting on it) has drained.
  bool admit(int s, const OwnedRequest& r, bool* oom, bool sync = true) {
    *oom = false;
    (void)hipGetLastError();  // launch errors below are checked against a clean slate
    HostSlot& h = hs[s];
    const bool p2pl = !r.query && mode_plane(r.prm.mode);
    h.L.plan(r.M, r.N, p2pl, r.query && !r.idx_dev_out, r.trace_cap);
    h.mem = arena->alloc(h.L.total);
    if (!h.mem) { *oom = true; return true; }
    h.used = true;
    h.ticket = r.ticket;
    h.t_submit = r.t_submit;
    const Layout& L = h.L;
    char* b = h.mem;
    auto F = [&](size_t o) { return reinterpret_cast<float*>(b + o); };
    auto F4 = [&](size_t o) { return reinterpret_cast<float4*>(b + o); };
    unsigned* scratch = reinterpret_cast<unsigned*>(b + L.o_scratch);
    hipStream_t ss = setup_stream(s);
    char* st_base = reinterpret_cast<char*>(d_state + s);
    float* bbQ = reinterpret_cast<float*>(st_base + offsetof(SlotState, bbQ));
    float* bbP = reinterpret_cast<float*>(st_base + offsetof(SlotState, bbP));
    double* cQ = reinterpret_cast<double*>(st_base + offsetof(SlotState, cQ));
    double* cP = reinterpret_cast<double*>(st_base + offsetof(SlotState, cP));
    float* rho = reinterpret_cast<float*>(reinterpret_cast<char*>(d_desc + s) + offsetof(SlotDesc, rho_max));
    // state first (kernels below write some of its fields)
    SlotState& S = h.S0;
    std::memset(&S, 0, sizeof S);
    S.status = ST_SETUP;
    S.mode = r.query ? P2P_L2 : (int)r.prm.mode;
    S.sm = r.query ? SM_QUERY : (r.eval ? SM_EVAL : SM_INIT);
    S.m = r.prm.anderson_m;
    S.lmax = r.prm.max_line_search;
    S.iter_first = r.prm.iter_first;
    S.iter_inc = r.prm.iter_inc;
    S.iter_cap = r.prm.iter_cap;
    S.max_total = r.prm.max_total_iter;
    S.eps = r.prm.eps;
    S.nu_min = r.prm.nu_min;
    S.nu_max = r.prm.nu_max;
    S.nu_auto = (!r.query && !r.eval && !mode_l2(r.prm.mode) && !(r.prm.nu_max > 0)) ? 1 : 0;
    S.want_median = S.nu_auto;
    hs[s].want_median = S.want_median != 0;
    S.k = 1;
    std::memcpy(S.Tkm1, (r.query || r.eval) ? r.Tq : r.prm.T0, sizeof S.Tkm1);
    // Uploads on their own stream, each AoS array into a region of the slot
    // that is free until the setup below overwrites it: Q into the sort
    // scratch (12 N <= its size), the normals into the centred cluster
    // coordinates (16 N), P into the candidate lists (32 B per source).
    HIP_OK(hipMemcpyAsync(d_state + s, &S, sizeof S, hipMemcpyHostToDevice, up));
    const float* srcQ = r.Q_dev ? r.Q_dev : F(L.o_scratch);
    const float* srcN = r.Qn_dev ? r.Qn_dev : F(L.o_qorg);
    const float* srcP = r.P_dev ? r.P_dev : F(L.o_clist);
    if (!r.Q_dev) HIP_OK(hipMemcpyAsync(F(L.o_scratch), r.Q.data(), 12ull * L.N, hipMemcpyHostToDevice, up));
    if (p2pl && !r.Qn_dev)
      HIP_OK(hipMemcpyAsync(F(L.o_qorg), r.Qn.data(), 12ull * L.N, hipMemcpyHostToDevice, up));
    if (!r.P_dev) HIP_OK(hipMemcpyAsync(F(L.o_clist), r.P.data(), 12ull * L.M, hipMemcpyHostToDevice, up));
    HIP_OK(hipEventRecord(up_done, up));
    HIP_OK(hipStreamWaitEvent(ss, up_done, 0));
    if (r.ready) HIP_OK(hipStreamWaitEvent(ss, r.ready->ev, 0));
    // inputs -> SoA
    launch_aos_to_soa(srcQ, L.N, F(L.o_qx), F(L.o_qy), F(L.o_qz), ss);
    if (p2pl) launch_aos_to_soa(srcN, L.N, F(L.o_nx), F(L.o_ny), F(L.o_nz), ss);
    launch_aos_to_soa(srcP, L.M, F(L.o_pox), F(L.o_poy), F(L.o_poz), ss);
    // target cluster index
    launch_bbox(F(L.o_qx), F(L.o_qy), F(L.o_qz), L.N, bbQ, cQ, ss);
    unsigned* order = nullptr;
    launch_hilbert_order(F(L.o_qx), F(L.o_qy), F(L.o_qz), L.N, bbQ, scratch, &order, ss);
    launch_build_clusters(F(L.o_qx), F(L.o_qy), F(L.o_qz), order, L.N, L.ncl, F4(L.o_qloc),
                          F4(L.o_qorg), F4(L.o_ccen), F4(L.o_clo), F4(L.o_chi), F4(L.o_kbox), ss);
    launch_build_super(F4(L.o_clo), F4(L.o_chi), F4(L.o_ccen), L.ncl, L.nsup, F4(L.o_slo),
                       F4(L.o_shi), rho, r.tune.list_margin, ss);
    // automatic nu_min from the targets' six nearest neighbours, into the
    // state (scratch holds the per-target values until the source sort)
    if (r.numin_only || (!r.query && !r.eval && auto_nu_min(&r.prm))) {
      const bool plane = mode_plane(r.prm.mode);
      launch_nu_min_auto(F4(L.o_qorg), F4(L.o_clo), F4(L.o_chi), F4(L.o_slo), F4(L.o_shi), L.ncl,
                         L.nsup, F(L.o_qx), F(L.o_qy), F(L.o_qz), plane ? F(L.o_nx) : nullptr,
                         plane ? F(L.o_ny) : nullptr, plane ? F(L.o_nz) : nullptr, L.N, plane,
                         reinterpret_cast<double*>(b + L.o_scratch),
                         reinterpret_cast<double*>(st_base + offsetof(SlotState, nu_min)), ss);
    }
    // source tiles
    launch_bbox(F(L.o_pox), F(L.o_poy), F(L.o_poz), L.M, bbP, cP, ss);
    launch_hilbert_order(F(L.o_pox), F(L.o_poy), F(L.o_poz), L.M, bbP, scratch, &order, ss);
    launch_build_tiles(F(L.o_pox), F(L.o_poy), F(L.o_poz), order, L.M, L.ntile, F(L.o_px),
                       F(L.o_py), F(L.o_pz), reinterpret_cast<int*>(b + L.o_perm),
                       reinterpret_cast<double4*>(b + L.o_tsph), ss);
    launch_fill_u64(reinterpret_cast<unsigned long long*>(b + L.o_keys), L.M, ~0ull, ss);
    launch_fill_u64(reinterpret_cast<unsigned long long*>(b + L.o_stats), kQueues * kStatStride, 0ull, ss);
    // no previous closest point yet (int32 -1 everywhere)
    launch_fill_u64(reinterpret_cast<unsigned long long*>(b + L.o_nnidx), (L.M + 1) / 2, ~0ull, ss);
    // descriptor (rho_max is written by build_super above, so copy the rest around it)
    SlotDesc& D = h.D0;
    std::memset(&D, 0, sizeof D);
    D.px = F(L.o_px); D.py = F(L.o_py); D.pz = F(L.o_pz);
    D.perm = reinterpret_cast<int*>(b + L.o_perm);
    D.tsph = reinterpret_cast<double4*>(b + L.o_tsph);
    D.qx = F(L.o_qx); D.qy = F(L.o_qy); D.qz = F(L.o_qz);
    D.nx = p2pl ? F(L.o_nx) : nullptr;
    D.ny = p2pl ? F(L.o_ny) : nullptr;
    D.nz = p2pl ? F(L.o_nz) : nullptr;
    D.qloc = F4(L.o_qloc); D.qorg = F4(L.o_qorg); D.ccen = F4(L.o_ccen);
    D.clo = F4(L.o_clo); D.chi = F4(L.o_chi); D.slo = F4(L.o_slo); D.shi = F4(L.o_shi);
    D.kbox = F4(L.o_kbox);
    D.keys = reinterpret_cast<unsigned long long*>(b + L.o_keys);
    D.clist = reinterpret_cast<int*>(b + L.o_clist);
    D.squeue = reinterpret_cast<int4*>(b + L.o_squeue);
    D.scount = reinterpret_cast<int*>(b + L.o_scount);
    D.nnidx = reinterpret_cast<int32_t*>(b + L.o_nnidx);
    D.nnd2 = F(L.o_nnd2);
    D.part = reinterpret_cast<double*>(b + L.o_part);
    D.medkey = reinterpret_cast<double*>(b + L.o_med);
    if (r.query) {
      D.idx_out = r.idx_dev_out ? r.idx_dev_out : reinterpret_cast<int32_t*>(b + L.o_idx);
      D.d2_out = r.d2_dev_out ? r.d2_dev_out : F(L.o_d2);
    }
    D.stats = reinterpret_cast<unsigned long long*>(b + L.o_stats);
    D.item_stats = L.trace_cap > 0 ? reinterpret_cast<int*>(b + L.o_items) : nullptr;
    D.trace = L.trace_cap > 0 ? reinterpret_cast<double*>(b + L.o_trace) : nullptr;
    D.trace_cap = L.trace_cap;
    D.M = L.M; D.N = L.N; D.ntile = L.ntile; D.ncl = L.ncl; D.nsup = L.nsup; D.nepi = L.nepi;
    icp_nn_method meth = r.query ? r.qmethod : r.prm.nn;
    if (meth == ICP_NN_AUTO) meth = ((double)L.M * L.N <= 64.0e6) ? ICP_NN_BRUTE : ICP_NN_CLUSTER;
    D.method = meth == ICP_NN_BRUTE ? NN_BRUTE : NN_CLUSTER;
    D.slice_min = r.tune.slice_min;
    D.brute_clusters = r.tune.brute_clusters;
    D.brute_items = r.tune.brute_items;
    if (!single && D.method == NN_BRUTE &&
        brute_items64(L.ntile, L.ncl, D.brute_clusters) > kMaxBruteItemsPerPair)
      D.method = NN_CLUSTER;
    if (single) {
      brute = D.method == NN_BRUTE;
      nn_grid = cus * r.tune.grid_per_cu;  // the one-slot engine's launch shape follows its pair
    }
    D.mode = S.mode;
    HIP_OK(hipMemcpyAsync(d_desc + s, &D, offsetof(SlotDesc, rho_max), hipMemcpyHostToDevice, up));
    h.zero = 0;
    HIP_OK(hipMemcpyAsync(d_done + s, &h.zero, sizeof(int), hipMemcpyHostToDevice, up));
    HIP_OK(hipEventRecord(up_done, up));
    HIP_OK(hipStreamWaitEvent(ss, up_done, 0));  // the activation on the setup stream covers the uploads
    h_done[s] = 0;
    if (sync) HIP_OK(hipStreamSynchronize(ss));
    return hipGetLastError() == hipSuccess;
  }

  // Wait for the admission streams: after a failed admission, before the
  // host sources of its uploads may be freed.
  void drain() {
    (void)hipStreamSynchronize(up);
    for (auto x : sides) (void)hipStreamSynchronize(x);
  }

  // Make the slot RUNNING on the pass stream once its setup has completed.
  bool activate(int s) {
    hipEvent_t ev;
    HIP_OK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HIP_OK(hipEventRecord(ev, setup_stream(s)));
    HIP_OK(hipStreamWaitEvent(st, ev, 0));
    launch_boot(d_desc, d_state, s, d_wl, single, st);
    (void)hipEventDestroy(ev);
    return hipGetLastError() == hipSuccess;
  }

  bool read_state(int s, SlotState* S) {
    HIP_OK(hipMemcpyAsync(S, d_state + s, sizeof(SlotState), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    return true;
  }

  void release(int s) {
    HostSlot& h = hs[s];
    if (h.mem) arena->release(h.mem);
    h = HostSlot();
    h_done[s] = 0;
  }
};

// ------------------------------------------------------------------ allocation-free query

// Working memory of icp_nn_query_dev_noalloc: one query slot (descriptor,
// state, work list, completion flag and the slot's arrays) in a fixed device
// array, one copy per GPU, held until the process ends. Host code reaches it
// only through the address hipGetSymbolAddress returns for the current device.
constexpr size_t kNoAllocBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr size_t round256(size_t b) { return (b + 255) & ~size_t(255); }
constexpr size_t kNoAllocDesc = 0;
constexpr size_t kNoAllocState = kNoAllocDesc + round256(sizeof(SlotDesc));
constexpr size_t kNoAllocWl = kNoAllocState + round256(sizeof(SlotState));
constexpr size_t kNoAllocDone = kNoAllocWl + round256(sizeof(WorkList));
constexpr size_t kNoAllocSlot = kNoAllocDone + 256;

struct NoAllocDevice {
  bool ready = false;
  unsigned char* ptr = nullptr;  // device address of `scratch` on this GPU
  int nn_grid = 4096, epi_grid = 1024;
};
constexpr int kNoAllocMaxDevices = 64;
static std::mutex g_noalloc_mu;
static NoAllocDevice g_noalloc[kNoAllocMaxDevices];

// Address of the scratch array on the current device (looked up once per
// device with that device current), or nullptr.
static NoAllocDevice* noalloc_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNoAllocMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_noalloc_mu);
  NoAllocDevice& d = g_noalloc[dev];
  if (!d.ready) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    int cus = 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 256;
    d.ptr = static_cast<unsigned char*>(p);
    d.nn_grid = cus * 16;
    d.epi_grid = cus * 4;
    d.ready = true;
  }
  return &d;
}

struct QueryT { double T[16]; };

// Descriptor, state and work list of a fresh query slot, written on the
// device (no host copy, so the sequence can be captured into a graph and
// replayed with other inputs). The descriptor's rho_max and verlet are
// written afterwards by the cluster build.
__global__ __launch_bounds__(256) void noalloc_init_kernel(SlotDesc* __restrict__ desc,
                                                           SlotState* __restrict__ state,
                                                           WorkList* __restrict__ wl,
                                                           int* __restrict__ done, SlotDesc D,
                                                           QueryT T) {
  unsigned long long* sw = reinterpret_cast<unsigned long long*>(state);
  for (size_t i = threadIdx.x; i < sizeof(SlotState) / 8; i += blockDim.x) sw[i] = 0ull;
  int* ww = reinterpret_cast<int*>(wl);
  for (size_t i = threadIdx.x; i < sizeof(WorkList) / 4; i += blockDim.x) ww[i] = 0;
  __syncthreads();
  if (threadIdx.x == 0) {
    D.rho_max = 0.0f;
    D.verlet = 0.0f;
    *desc = D;
    state->status = ST_SETUP;
    state->mode = P2P_L2;
    state->sm = SM_QUERY;
    state->k = 1;
    for (int i = 0; i < 16; ++i) state->Tkm1[i] = T.T[i];
    done[0] = 0;
  }
}

}  // namespace icp

using namespace icp;

// ------------------------------------------------------------------ context

struct icp_ctx {
  int device = 0;
  Arena arena;
  Engine sync_eng;       // icp_register / icp_nn_query
  Engine batch_eng;      // icp_batch_submit / icp_poll
  std::mutex sync_mu;
  // batch scheduler
  std::mutex mu;
  std::condition_variable cv, cv_done;
  std::deque<std::unique_ptr<OwnedRequest>> queue;
  std::unordered_map<uint64_t, int> state;   // 0 queued, 1 running, 2 done
  std::unordered_map<uint64_t, icp_result> results;
  std::thread worker;
  bool stop = false;
  bool started = false;
  bool failed = false;
  uint64_t next_ticket = 1;
  size_t reserved = 0;  // tickets handed out whose requests are still being copied
  int passes_per_replay = 4;
  int max_slots = 256;
  int running = 0;
  int admitting = 0;    // popped from the queue, not yet running or finished
  // work-partition table of the autotuner, per size bucket (tune_mu)
  std::mutex tune_mu;
  std::vector<icp_tuning_entry> tuning;
  std::string arch;     // gcnArchName up to the first ':' (e.g. gfx950)
  std::vector<int> last_items;  // per NN work item of the last traced registration's last pass
};

static const size_t kQueueCap = 1 << 20;
static const unsigned kSubmitThreads = 8;  // host threads of a large icp_batch_submit

// Every coordinate finite with |v| <= 1e15. On the bit patterns: |v| > 1e15f,
// Inf and NaN are exactly the magnitudes above that of 1e15f (0x58635fa9),
// tested branch-free over blocks so that the loop vectorises.
static bool finite_coords(const float* p, int64_t n) {
  const int64_t m = 3 * n;
  for (int64_t i0 = 0; i0 < m; i0 += 4096) {
    const int64_t e = std::min<int64_t>(i0 + 4096, m);
    unsigned bad = 0;
    for (int64_t i = i0; i < e; ++i) {
      uint32_t b;
      std::memcpy(&b, p + i, 4);
      bad |= (b & 0x7fffffffu) > 0x58635fa9u;
    }
    if (bad) return false;
  }
  return true;
}

// fn(i) for i in [0, n) on up to `threads` threads (thread k takes k, k + T, ...).
template <class Fn>
static void parallel_items(int n, int threads, Fn fn) {
  const int T = std::max(1, std::min(threads, n));
  if (T == 1) {
    for (int i = 0; i < n; ++i) fn(i);
    return;
  }
  std::vector<std::thread> th;
  int started = 1;
  try {
    th.reserve(T - 1);
    for (int k = 1; k < T; ++k, ++started)
      th.emplace_back([&fn, n, T, k] { for (int i = k; i < n; i += T) fn(i); });
  } catch (...) {
  }
  // the calling thread takes its own share and that of any thread that did not start
  for (int k = 0; k < T; ++k)
    if (k == 0 || k >= started)
      for (int i = k; i < n; i += T) fn(i);
  for (auto& t : th) t.join();
}

static bool rigid_ok(const double* T) {
  for (int i = 0; i < 16; ++i)
    if (!std::isfinite(T[i])) return false;
  if (T[12] != 0.0 || T[13] != 0.0 || T[14] != 0.0 || T[15] != 1.0) return false;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += T[4 * k + i] * T[4 * k + j];
      if (std::fabs(s - (i == j ? 1.0 : 0.0)) > 1e-9) return false;
    }
  const double det = T[0] * (T[5] * T[10] - T[6] * T[9]) - T[1] * (T[4] * T[10] - T[6] * T[8]) +
                     T[2] * (T[4] * T[9] - T[5] * T[8]);
  return det > 0.0;
}

static icp_status check_params(const icp_params* p) {
  if (!p) return ICP_ERR_INVALID_ARG;
  if (p->mode < ICP_P2P_L2 || p->mode > ICP_P2PL_L2) return ICP_ERR_INVALID_ARG;
  if (p->anderson_m < 0 || p->anderson_m > 6) return ICP_ERR_INVALID_ARG;
  // nu_min <= 0: the automatic rule (six nearest targets), which needs N >= 7
  if (!mode_l2(p->mode) && !std::isfinite(p->nu_min)) return ICP_ERR_INVALID_ARG;
  if (!(p->eps > 0.0) || p->iter_first <= 0 || p->max_line_search < 0) return ICP_ERR_INVALID_ARG;
  if (p->nn < ICP_NN_AUTO || p->nn > ICP_NN_CLUSTER) return ICP_ERR_INVALID_ARG;
  if (p->engine != ICP_ENGINE_GRAPH && p->engine != ICP_ENGINE_PLAIN) return ICP_ERR_INVALID_ARG;
  if (!std::isfinite(p->nu_max)) return ICP_ERR_INVALID_ARG;
  if (!rigid_ok(p->T0)) return ICP_ERR_INVALID_ARG;
  return ICP_OK;
}

static icp_status check_sizes(int64_t M, int64_t N) {
  if (M <= 0 || N <= 0 || M > (1 << 28) || N > (1 << 28)) return ICP_ERR_INVALID_ARG;
  return ICP_OK;
}

static icp_status check_params_sized(const icp_params* p, int64_t N) {
  const icp_status s = check_params(p);
  if (s != ICP_OK) return s;
  if (auto_nu_min(p) && N < 7) return ICP_ERR_INVALID_ARG;  // six other targets needed
  return ICP_OK;
}

// ------------------------------------------------------------------ tuning table

static int size_bucket(int64_t n) {
  int b = 0;
  while (b < 62 && (int64_t(1) << (b + 1)) <= n) ++b;
  return b;
}

// Tuning entries are kept per mode family (point-to-point / point-to-plane)
// and search method.
static int mode_family(int mode) { return mode_plane(mode) ? ICP_P2PL_WELSCH : ICP_P2P_WELSCH; }

static bool tuning_valid(const icp_tuning& t) {
  return t.slice_min >= 1 && t.slice_min <= 64 && t.list_margin >= 0.0f && t.list_margin <= 1.0f &&
         t.brute_clusters >= 1 && t.brute_clusters <= 4096 && t.brute_items >= 64 &&
         t.brute_items <= (1 << 20) && t.grid_per_cu >= 1 && t.grid_per_cu <= 64;
}

static icp_tuning default_tuning() {
  return icp_tuning{kSliceMinDefault, kVerletFracDefault, kBruteClustersDefault, kBruteItemsDefault,
                    kGridPerCuDefault};
}

// The entry of the request's bucket; else the nearest tuned bucket of the same
// family and method within two octaves (sum over M and N); else the defaults.
// *found: 2 exact, 1 nearby, 0 default.
static icp_tuning lookup_tuning(icp_ctx* ctx, int64_t M, int64_t N, int mode, icp_nn_method method,
                                int batch, int* found) {
  const int mb = size_bucket(M), nb = size_bucket(N), fam = mode_family(mode);
  method = resolve_method(M, N, method);
  std::lock_guard<std::mutex> g(ctx->tune_mu);
  int best = -1, bestd = 3;
  for (size_t i = 0; i < ctx->tuning.size(); ++i) {
    const icp_tuning_entry& e = ctx->tuning[i];
    if (e.mode != fam || e.method != (int)method || e.batch != batch) continue;
    const int dd = std::abs(e.m_bucket - mb) + std::abs(e.n_bucket - nb);
    if (dd < bestd) { bestd = dd; best = (int)i; }
  }
  if (found) *found = best < 0 ? 0 : (bestd == 0 ? 2 : 1);
  return best < 0 ? default_tuning() : ctx->tuning[best].tuning;
}

static void put_tuning(icp_ctx* ctx, icp_tuning_entry e) {
  e.mode = mode_family(e.mode);
  std::lock_guard<std::mutex> g(ctx->tune_mu);
  for (auto& x : ctx->tuning)
    if (x.m_bucket == e.m_bucket && x.n_bucket == e.n_bucket && x.mode == e.mode && x.method == e.method &&
        x.batch == e.batch) {
      x = e;
      return;
    }
  ctx->tuning.push_back(e);
}

static void tune_request(icp_ctx* ctx, OwnedRequest& r, int batch) {
  const int mode = r.query ? (int)ICP_P2P_L2 : (int)r.prm.mode;
  r.tune = lookup_tuning(ctx, r.M, r.N, mode, r.query ? r.qmethod : r.prm.nn, batch, nullptr);
}

// Run one slot of the synchronous engine to completion.
static icp_status run_sync(icp_ctx* ctx, OwnedRequest& r, icp_result* out, void* ustream,
                           int32_t* host_idx, float* host_d2, double* host_trace = nullptr,
                           int* trace_len = nullptr, std::vector<int>* item_stats_out = nullptr) {
  Engine& E = ctx->sync_eng;
  const auto t0 = Clock::now();
  if (!r.tune_fixed) tune_request(ctx, r, 0);
  hipStream_t us = reinterpret_cast<hipStream_t>(ustream);
  if (hipSetDevice(ctx->device) != hipSuccess) return ICP_ERR_DEVICE;
  // order after the caller's stream
  if (r.P_dev) {
    hipEvent_t ev;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return ICP_ERR_DEVICE;
    if (hipEventRecord(ev, us) != hipSuccess || hipStreamWaitEvent(E.side, ev, 0) != hipSuccess) {
      (void)hipEventDestroy(ev);
      return ICP_ERR_DEVICE;
    }
    (void)hipEventDestroy(ev);
  }
  bool oom = false;
  if (!E.admit(0, r, &oom)) { E.drain(); E.release(0); return ICP_ERR_DEVICE; }
  if (oom) return ICP_ERR_OOM;
  if (!E.activate(0)) { E.release(0); return ICP_ERR_DEVICE; }
  const bool plain = !r.query && !r.eval && r.prm.engine == ICP_ENGINE_PLAIN;
  icp_status rc = ICP_OK;
  const long kMaxPasses = 200000;  // host guard against a runaway state machine
  long passes = 0;
  E.h_done[0] = 0;
  if (E.hs[0].want_median) {
    // the first pass computes the median for the initial nu: launched
    // directly with the median kernel, the later passes without it
    if (E.prof && !E.ensure_events(1)) rc = ICP_ERR_DEVICE;
    if (rc == ICP_OK) {
      E.enqueue_pass(E.st, 0, false, true);
      if (hipMemcpyAsync(E.h_done, E.d_done, sizeof(int), hipMemcpyDeviceToHost, E.st) != hipSuccess ||
          hipStreamSynchronize(E.st) != hipSuccess)
        rc = ICP_ERR_DEVICE;
      else
        E.collect_profile(1);
    }
    passes = 1;
    if (rc != ICP_OK) { E.release(0); return rc; }
  }
  if (E.h_done[0]) {
    // finished in the first pass
  } else if (plain) {
    for (;; ++passes) {
      if (passes > kMaxPasses) { rc = ICP_ERR_DEVICE; break; }
      if (E.prof && !E.ensure_events(1)) { rc = ICP_ERR_DEVICE; break; }
      E.enqueue_pass(E.st, 0);
      if (hipMemcpyAsync(E.h_done, E.d_done, sizeof(int), hipMemcpyDeviceToHost, E.st) != hipSuccess ||
          hipStreamSynchronize(E.st) != hipSuccess) { rc = ICP_ERR_DEVICE; break; }
      E.collect_profile(1);
      if (E.h_done[0]) break;
    }
  } else {
    const int R = (r.query || r.eval) ? 1 : 16;
    // profiling: the same passes launched directly (timing events around each
    // kernel); otherwise replays of the captured graph
    if (!E.prof && !E.build_graph(R)) { E.release(0); return ICP_ERR_DEVICE; }
    if (E.prof && !E.ensure_events(R)) { E.release(0); return ICP_ERR_DEVICE; }
    for (;; passes += R) {
      if (passes > kMaxPasses) { rc = ICP_ERR_DEVICE; break; }
      if (E.prof)
        for (int i = 0; i < R; ++i) E.enqueue_pass(E.st, i, false);
      if ((!E.prof && hipGraphLaunch(E.gexec, E.st) != hipSuccess) ||
          hipMemcpyAsync(E.h_done, E.d_done, sizeof(int), hipMemcpyDeviceToHost, E.st) != hipSuccess ||
          hipStreamSynchronize(E.st) != hipSuccess) { rc = ICP_ERR_DEVICE; break; }
      E.collect_profile(R);
      if (E.h_done[0]) break;
    }
  }
  if (rc == ICP_OK) {
    SlotState S;
    if (!E.read_state(0, &S)) rc = ICP_ERR_DEVICE;
    else if (out) {
      fill_result(S, out);
      fill_stats(E.hs[0], E.st, out);
      out->latency_ms = std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
    }
    if (rc == ICP_OK && host_trace && trace_len) {
      const Layout& L = E.hs[0].L;
      *trace_len = std::min(S.trace_len, L.trace_cap);
      if (item_stats_out) {
        const SlotDesc* dd = nullptr;
        (void)dd;
        item_stats_out->resize(8ull * L.ntile * kMaxSlices);
        (void)hipMemcpy(item_stats_out->data(), E.hs[0].mem + L.o_items, 32ull * L.ntile * kMaxSlices,
                        hipMemcpyDeviceToHost);
      }
      if (*trace_len > 0 &&
          hipMemcpy(host_trace, E.hs[0].mem + L.o_trace, 8ull * kTraceRow * *trace_len,
                    hipMemcpyDeviceToHost) != hipSuccess)
        rc = ICP_ERR_DEVICE;
    }
    if (rc == ICP_OK && r.query && host_idx) {
      const Layout& L = E.hs[0].L;
      if (hipMemcpy(host_idx, E.hs[0].mem + L.o_idx, 4ull * r.M, hipMemcpyDeviceToHost) != hipSuccess ||
          hipMemcpy(host_d2, E.hs[0].mem + L.o_d2, 4ull * r.M, hipMemcpyDeviceToHost) != hipSuccess)
        rc = ICP_ERR_DEVICE;
    }
  }
  // the caller's stream waits for our work
  if (r.P_dev) {
    hipEvent_t ev;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess) {
      (void)hipEventRecord(ev, E.st);
      (void)hipStreamWaitEvent(us, ev, 0);
      (void)hipEventDestroy(ev);
    }
  }
  (void)hipStreamSynchronize(E.st);
  E.release(0);
  return rc;
}

// ------------------------------------------------------------------ scheduler

static void scheduler(icp_ctx* ctx) {
  Engine& E = ctx->batch_eng;
  (void)hipSetDevice(ctx->device);
  // requests admitted in this round whose host arrays may still be read by
  // uploads in flight; released once the pass stream (which waits on every
  // activation) has been synchronised
  std::vector<std::unique_ptr<OwnedRequest>> held;
  for (;;) {
    int R, running;
    {
      std::unique_lock<std::mutex> lk(ctx->mu);
      ctx->cv.wait(lk, [&] { return ctx->stop || !ctx->queue.empty() || ctx->running > 0; });
      if (ctx->stop) return;
      R = ctx->passes_per_replay;
      running = ctx->running;
      E.prof = E.prof_req;
      if (running == 0) E.capacity = ctx->max_slots;
    }
    bool ok = true;
    // 1) advance every resident pair by R passes (asynchronous)
    if (running > 0) {
      if (E.prof) {
        ok = E.ensure_events(R);
        for (int i = 0; ok && i < R; ++i) E.enqueue_pass(E.st, i, false);
      } else {
        ok = E.build_graph(R) && hipGraphLaunch(E.gexec, E.st) == hipSuccess;
      }
    }
    // 2) meanwhile set up queued requests on the side stream (FIFO; a request
    //    that does not fit waits for memory unless nothing else is resident).
    //    The uploads and setup kernels are only enqueued here; the
    //    synchronisation in 3) covers them, since the pass stream waits on
    //    every activation.
    for (; ok;) {
      std::unique_ptr<OwnedRequest> req;
      int s;
      {
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (ctx->queue.empty()) break;
        s = E.free_slot();
        if (s < 0) break;
        req = std::move(ctx->queue.front());
        ctx->queue.pop_front();
        ctx->admitting++;
      }
      bool oom = false;
      const bool adm = E.admit(s, *req, &oom, false);
      if (adm && oom) {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->admitting--;
        if (ctx->running == 0) {
          ctx->state[req->ticket] = 3;  // can never fit the budget
        } else {
          ctx->queue.push_front(std::move(req));
        }
        break;
      }
      if (!adm || !E.activate(s)) {
        E.drain();
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->admitting--;
        ctx->state[req->ticket] = 4;
        E.release(s);
        ok = false;
        break;
      }
      held.push_back(std::move(req));
      std::lock_guard<std::mutex> lk(ctx->mu);
      ctx->state[held.back()->ticket] = 1;
      ctx->admitting--;
      ctx->running++;
    }
    // 3) completion flags after the replay (and after the boots of new slots)
    if (ok)
      ok = hipMemcpyAsync(E.h_done, E.d_done, sizeof(int) * E.capacity, hipMemcpyDeviceToHost, E.st) ==
               hipSuccess &&
           hipStreamSynchronize(E.st) == hipSuccess;
    if (ok) held.clear();
    if (ok && running > 0 && E.prof) {
      // the sums are read and reset by other threads under the context lock
      std::lock_guard<std::mutex> lk(ctx->mu);
      E.collect_profile(R);
    }
    if (!ok) {
      E.drain();
      std::lock_guard<std::mutex> lk(ctx->mu);
      ctx->failed = true;
      ctx->stop = true;
      ctx->cv_done.notify_all();
      return;
    }
    // 4) retire finished pairs: read back their states and counters and free
    //    their slots on the device, all with one synchronisation
    constexpr int kStatWords = kQueues * kStatStride;
    std::vector<int> fin;
    for (int s = 0; s < E.capacity; ++s)
      if (E.hs[s].used && E.h_done[s]) fin.push_back(s);
    bool got = true;
    for (int s : fin) {
      got = got &&
            hipMemcpyAsync(E.h_fin_state + s, E.d_state + s, sizeof(SlotState), hipMemcpyDeviceToHost, E.st) ==
                hipSuccess &&
            hipMemcpyAsync(E.h_fin_stats + (size_t)s * kStatWords, E.hs[s].mem + E.hs[s].L.o_stats,
                           8ull * kStatWords, hipMemcpyDeviceToHost, E.st) == hipSuccess;
      (void)hipMemcpyAsync(E.d_done + s, E.h_reset, sizeof(int), hipMemcpyHostToDevice, E.st);
      (void)hipMemcpyAsync(reinterpret_cast<char*>(E.d_state + s) + offsetof(SlotState, status), E.h_reset + 1,
                           sizeof(int), hipMemcpyHostToDevice, E.st);
    }
    if (!fin.empty()) got = hipStreamSynchronize(E.st) == hipSuccess && got;
    for (int s : fin) {
      icp_result res;
      std::memset(&res, 0, sizeof res);
      if (got) {
        fill_result(E.h_fin_state[s], &res);
        stats_from(E.h_fin_stats + (size_t)s * kStatWords, &res);
      }
      res.latency_ms = std::chrono::duration<double, std::milli>(Clock::now() - E.hs[s].t_submit).count();
      const uint64_t t = E.hs[s].ticket;
      E.release(s);
      std::lock_guard<std::mutex> lk(ctx->mu);
      ctx->results[t] = res;
      ctx->state[t] = 2;
      ctx->running--;
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->cv_done.notify_all();
  }
}

// ------------------------------------------------------------------ C ABI

extern "C" {

const char* icp_status_str(icp_status s) {
  switch (s) {
    case ICP_OK: return "ok";
    case ICP_ERR_INVALID_ARG: return "invalid argument";
    case ICP_ERR_NONFINITE: return "non-finite or out-of-range coordinate";
    case ICP_ERR_NO_NORMALS: return "point-to-plane mode needs target normals";
    case ICP_ERR_OOM: return "out of device memory budget";
    case ICP_ERR_DEVICE: return "HIP device error";
    case ICP_ERR_NOT_READY: return "not ready";
    case ICP_ERR_UNKNOWN_TICKET: return "unknown ticket";
    case ICP_ERR_QUEUE_FULL: return "queue full";
  }
  return "unknown status";
}

icp_status icp_params_default(icp_mode mode, icp_params* out) {
  if (!out || mode < ICP_P2P_L2 || mode > ICP_P2PL_L2) return ICP_ERR_INVALID_ARG;
  if (mode == ICP_P2PL_L2) return icp_params_classical(mode, out);
  std::memset(out, 0, sizeof *out);
  out->mode = mode;
  out->anderson_m = 5;
  out->nu_max = -1.0;
  out->nu_min = -1.0;
  out->eps = 1e-5;
  out->max_total_iter = 0;
  out->max_line_search = 10;
  if (mode == ICP_P2PL_WELSCH) {
    out->iter_first = 6; out->iter_inc = 1; out->iter_cap = 10;
  } else {
    out->iter_first = 1000; out->iter_inc = 0; out->iter_cap = 1000;
  }
  out->nn = ICP_NN_AUTO;
  out->engine = ICP_ENGINE_GRAPH;
  for (int i = 0; i < 16; ++i) out->T0[i] = (i % 5 == 0) ? 1.0 : 0.0;
  return ICP_OK;
}

// App. E: the comparison methods run to 1000 iterations or until the squared
// Frobenius norm of the change of transform is below 1e-5.
icp_status icp_params_classical(icp_mode mode, icp_params* out) {
  if (!out || (mode != ICP_P2P_L2 && mode != ICP_P2PL_L2)) return ICP_ERR_INVALID_ARG;
  std::memset(out, 0, sizeof *out);
  out->mode = mode;
  out->anderson_m = 0;
  out->nu_max = -1.0;
  out->nu_min = -1.0;
  out->eps = std::sqrt(1e-5);
  out->iter_first = 1000;
  out->iter_inc = 0;
  out->iter_cap = 1000;
  out->max_total_iter = 0;
  out->max_line_search = 0;
  out->nn = ICP_NN_AUTO;
  out->engine = ICP_ENGINE_GRAPH;
  for (int i = 0; i < 16; ++i) out->T0[i] = (i % 5 == 0) ? 1.0 : 0.0;
  return ICP_OK;
}

// The tuning cache of icp_create: $ICP_TUNING_CACHE, else tuning_<arch>.json
// in the directory of this library. A missing or unreadable file leaves the
// defaults.
static void load_tuning_cache(icp_ctx* c) {
  if (c->arch.empty()) return;
  std::string path;
  if (const char* env = std::getenv("ICP_TUNING_CACHE")) {
    path = env;
  } else {
    Dl_info info;
    if (dladdr(reinterpret_cast<void*>(&load_tuning_cache), &info) && info.dli_fname) {
      path = info.dli_fname;
      const size_t sl = path.find_last_of('/');
      path = (sl == std::string::npos ? std::string(".") : path.substr(0, sl)) + "/tuning_" + c->arch + ".json";
    }
  }
  if (path.empty()) return;
  std::vector<icp_tuning_entry> e(4096);
  int n = 0;
  if (icp_tuning_file_read(path.c_str(), c->arch.c_str(), e.data(), (int)e.size(), &n) != ICP_OK) return;
  for (int i = 0; i < n; ++i) put_tuning(c, e[i]);
}

icp_status icp_create(int device, size_t hbm_budget_bytes, icp_ctx** out) {
  if (!out) return ICP_ERR_INVALID_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return ICP_ERR_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return ICP_ERR_DEVICE;
  auto* c = new (std::nothrow) icp_ctx();
  if (!c) return ICP_ERR_OOM;
  c->device = device;
  if (hbm_budget_bytes == 0) hbm_budget_bytes = size_t(8) << 30;
  if (!c->arena.init(hbm_budget_bytes)) { delete c; return ICP_ERR_OOM; }
  c->sync_eng.single = true;
  if (!c->sync_eng.init(device, 1, &c->arena) || !c->batch_eng.init(device, c->max_slots, &c->arena)) {
    c->sync_eng.destroy();
    c->batch_eng.destroy();
    delete c;
    return ICP_ERR_DEVICE;
  }
  char arch[64];
  if (icp_device_arch(device, arch, sizeof arch) == ICP_OK) c->arch = arch;
  load_tuning_cache(c);
  *out = c;
  return ICP_OK;
}

icp_status icp_destroy(icp_ctx* ctx) {
  if (!ctx) return ICP_ERR_INVALID_ARG;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->stop = true;
  }
  ctx->cv.notify_all();
  if (ctx->worker.joinable()) ctx->worker.join();
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  ctx->sync_eng.destroy();
  ctx->batch_eng.destroy();
  delete ctx;
  return ICP_OK;
}

static icp_status validate_host(const float* P, int64_t M, const float* Q, const float* Qn, int64_t N,
                                const icp_params* prm) {
  if (!P || !Q) return ICP_ERR_INVALID_ARG;
  icp_status s = check_sizes(M, N);
  if (s != ICP_OK) return s;
  s = check_params_sized(prm, N);
  if (s != ICP_OK) return s;
  if (mode_plane(prm->mode) && !Qn) return ICP_ERR_NO_NORMALS;
  if (!finite_coords(P, M) || !finite_coords(Q, N)) return ICP_ERR_NONFINITE;
  if (mode_plane(prm->mode)) {
    if (!finite_coords(Qn, N)) return ICP_ERR_NONFINITE;
    for (int64_t i = 0; i < N; ++i) {
      const double l = (double)Qn[3 * i] * Qn[3 * i] + (double)Qn[3 * i + 1] * Qn[3 * i + 1] +
                       (double)Qn[3 * i + 2] * Qn[3 * i + 2];
      if (!(l > 0.25 && l < 4.0)) return ICP_ERR_INVALID_ARG;  // zero or far-from-unit normals
    }
  }
  return ICP_OK;
}

icp_status icp_register(icp_ctx* ctx, const float* P, int64_t M, const float* Q, const float* Qn,
                        int64_t N, const icp_params* params, icp_result* out) {
  if (!ctx || !out) return ICP_ERR_INVALID_ARG;
  const icp_status v = validate_host(P, M, Q, Qn, N, params);
  if (v != ICP_OK) return v;
  OwnedRequest r;
  r.P.assign(P, P + 3 * M);
  r.Q.assign(Q, Q + 3 * N);
  if (mode_plane(params->mode)) r.Qn.assign(Qn, Qn + 3 * N);
  r.M = M; r.N = N; r.prm = *params;
  std::lock_guard<std::mutex> g(ctx->sync_mu);
  return run_sync(ctx, r, out, nullptr, nullptr, nullptr);
}

icp_status icp_eval(icp_ctx* ctx, const float* P, int64_t M, const float* Q, const float* Qn,
                    int64_t N, icp_mode mode, const double T[16], double nu, double* energy_out,
                    double T_out[16], unsigned* flags_out) {
  if (!ctx || !T || !energy_out || !T_out || !flags_out) return ICP_ERR_INVALID_ARG;
  icp_params prm;
  if (icp_params_default(mode, &prm) != ICP_OK) return ICP_ERR_INVALID_ARG;
  if (!mode_l2(mode) && !(nu > 0.0 && std::isfinite(nu))) return ICP_ERR_INVALID_ARG;
  prm.nu_min = mode_l2(mode) ? 0.0 : nu;
  prm.nu_max = mode_l2(mode) ? 1.0 : nu;
  std::memcpy(prm.T0, T, sizeof prm.T0);
  const icp_status v = validate_host(P, M, Q, Qn, N, &prm);
  if (v != ICP_OK) return v;
  OwnedRequest r;
  r.P.assign(P, P + 3 * M);
  r.Q.assign(Q, Q + 3 * N);
  if (mode_plane(mode)) r.Qn.assign(Qn, Qn + 3 * N);
  r.M = M; r.N = N; r.prm = prm;
  r.eval = true;
  std::memcpy(r.Tq, T, sizeof r.Tq);
  icp_result res;
  std::lock_guard<std::mutex> g(ctx->sync_mu);
  const icp_status rc = run_sync(ctx, r, &res, nullptr, nullptr, nullptr);
  if (rc != ICP_OK) return rc;
  *energy_out = res.energy;
  std::memcpy(T_out, res.T, sizeof res.T);
  *flags_out = res.status_flags;
  return ICP_OK;
}

icp_status icp_register_trace(icp_ctx* ctx, const float* P, int64_t M, const float* Q,
                              const float* Qn, int64_t N, const icp_params* params, icp_result* out,
                              double* trace_out, int trace_cap, int* trace_len) {
  if (!ctx || !out || !trace_len || trace_cap < 0 || (trace_cap > 0 && !trace_out))
    return ICP_ERR_INVALID_ARG;
  *trace_len = 0;
  const icp_status v = validate_host(P, M, Q, Qn, N, params);
  if (v != ICP_OK) return v;
  OwnedRequest r;
  r.P.assign(P, P + 3 * M);
  r.Q.assign(Q, Q + 3 * N);
  if (mode_plane(params->mode)) r.Qn.assign(Qn, Qn + 3 * N);
  r.M = M; r.N = N; r.prm = *params;
  r.trace_cap = trace_cap;
  std::lock_guard<std::mutex> g(ctx->sync_mu);
  return run_sync(ctx, r, out, nullptr, nullptr, nullptr, trace_out, trace_len, &ctx->last_items);
}

icp_status icp_trace_items(icp_ctx* ctx, int* out, int cap, int* len) {
  if (!ctx || !len || cap < 0 || (cap > 0 && !out)) return ICP_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(ctx->sync_mu);
  const int n = (int)(ctx->last_items.size() / 8);
  *len = n;
  std::memcpy(out, ctx->last_items.data(), sizeof(int) * 8 * (size_t)std::min(n, cap));
  return ICP_OK;
}

icp_status icp_register_dev(icp_ctx* ctx, const float* P_dev, int64_t M, const float* Q_dev,
                            const float* Qn_dev, int64_t N, const icp_params* params,
                            icp_result* out, void* stream) {
  if (!ctx || !out || !P_dev || !Q_dev) return ICP_ERR_INVALID_ARG;
  icp_status s = check_sizes(M, N);
  if (s != ICP_OK) return s;
  s = check_params_sized(params, N);
  if (s != ICP_OK) return s;
  if (mode_plane(params->mode) && !Qn_dev) return ICP_ERR_NO_NORMALS;
  OwnedRequest r;
  r.P_dev = P_dev; r.Q_dev = Q_dev; r.Qn_dev = Qn_dev;
  r.M = M; r.N = N; r.prm = *params;
  std::lock_guard<std::mutex> g(ctx->sync_mu);
  return run_sync(ctx, r, out, stream, nullptr, nullptr);
}

icp_status icp_nn_query(icp_ctx* ctx, const float* P, int64_t M, const float* Q, int64_t N,
                        const double T[16], icp_nn_method method, int32_t* idx_out, float* d2_out) {
  if (!ctx || !T || method < ICP_NN_AUTO || method > ICP_NN_CLUSTER) return ICP_ERR_INVALID_ARG;
  if (M < 0 || N <= 0 || M > (1 << 28) || N > (1 << 28) || !Q) return ICP_ERR_INVALID_ARG;
  if (M == 0) return ICP_OK;
  if (!P || !idx_out || !d2_out) return ICP_ERR_INVALID_ARG;
  if (!rigid_ok(T)) return ICP_ERR_INVALID_ARG;
  if (!finite_coords(P, M) || !finite_coords(Q, N)) return ICP_ERR_NONFINITE;
  OwnedRequest r;
  r.P.assign(P, P + 3 * M);
  r.Q.assign(Q, Q + 3 * N);
  r.M = M; r.N = N;
  icp_params_default(ICP_P2P_L2, &r.prm);
  r.query = true;
  std::memcpy(r.Tq, T, sizeof r.Tq);
  r.qmethod = method;
  std::lock_guard<std::mutex> g(ctx->sync_mu);
  icp_result res;
  return run_sync(ctx, r, &res, nullptr, idx_out, d2_out);
}

icp_status icp_nu_min_auto(icp_ctx* ctx, const float* Q, const float* Qn, int64_t N, icp_mode mode,
                           double* nu_min_out) {
  if (!ctx || !Q || !nu_min_out) return ICP_ERR_INVALID_ARG;
  if (mode != ICP_P2P_WELSCH && mode != ICP_P2PL_WELSCH) return ICP_ERR_INVALID_ARG;
  if (N < 7 || N > (1 << 28)) return ICP_ERR_INVALID_ARG;
  icp_params prm;
  icp_params_default(mode, &prm);
  prm.nu_min = 0.0;
  // the targets stand in for the sources: the setup needs both sets
  const icp_status v = validate_host(Q, N, Q, Qn, N, &prm);
  if (v != ICP_OK) return v;
  OwnedRequest r;
  r.P.assign(Q, Q + 3 * N);
  r.Q.assign(Q, Q + 3 * N);
  if (mode == ICP_P2PL_WELSCH) r.Qn.assign(Qn, Qn + 3 * N);
  r.M = N; r.N = N; r.prm = prm;
  r.numin_only = true;
  std::lock_guard<std::mutex> g(ctx->sync_mu);
  Engine& E = ctx->sync_eng;
  if (hipSetDevice(ctx->device) != hipSuccess) return ICP_ERR_DEVICE;
  bool oom = false;
  if (!E.admit(0, r, &oom)) { E.drain(); E.release(0); return ICP_ERR_DEVICE; }
  if (oom) return ICP_ERR_OOM;
  SlotState S;
  const bool ok = E.read_state(0, &S);
  E.release(0);
  if (!ok) return ICP_ERR_DEVICE;
  *nu_min_out = S.nu_min;
  return ICP_OK;
}

icp_status icp_estimate_normals(icp_ctx* ctx, const float* Q, int64_t N, float* normals_out) {
  if (!ctx || !Q || !normals_out) return ICP_ERR_INVALID_ARG;
  if (N < 30 || N > (1 << 28)) return ICP_ERR_INVALID_ARG;
  if (!finite_coords(Q, N)) return ICP_ERR_NONFINITE;
  OwnedRequest r;
  // the points stand in for both sets: the setup builds the cluster index
  r.P.assign(Q, Q + 3 * N);
  r.Q.assign(Q, Q + 3 * N);
  r.M = N; r.N = N;
  icp_params_default(ICP_P2P_L2, &r.prm);
  std::lock_guard<std::mutex> g(ctx->sync_mu);
  Engine& E = ctx->sync_eng;
  if (hipSetDevice(ctx->device) != hipSuccess) return ICP_ERR_DEVICE;
  bool oom = false;
  if (!E.admit(0, r, &oom)) { E.drain(); E.release(0); return ICP_ERR_DEVICE; }
  if (oom) return ICP_ERR_OOM;
  const Layout& L = E.hs[0].L;
  char* b = E.hs[0].mem;
  auto F4 = [&](size_t o) { return reinterpret_cast<const float4*>(b + o); };
  auto F = [&](size_t o) { return reinterpret_cast<float*>(b + o); };
  float* out = F(L.o_scratch);  // 12 N bytes, free once the setup is done
  launch_estimate_normals(F4(L.o_qorg), F4(L.o_clo), F4(L.o_chi), F4(L.o_slo), F4(L.o_shi), L.ncl,
                          L.nsup, F(L.o_qx), F(L.o_qy), F(L.o_qz), out, E.side);
  const bool ok = hipGetLastError() == hipSuccess &&
                  hipMemcpyAsync(normals_out, out, 12ull * N, hipMemcpyDeviceToHost, E.side) == hipSuccess &&
                  hipStreamSynchronize(E.side) == hipSuccess;
  E.release(0);
  return ok ? ICP_OK : ICP_ERR_DEVICE;
}

icp_status icp_nn_query_dev(icp_ctx* ctx, const float* P_dev, int64_t M, const float* Q_dev,
                            int64_t N, const double T[16], icp_nn_method method,
                            int32_t* idx_out_dev, float* d2_out_dev, void* stream) {
  if (!ctx || !T || method < ICP_NN_AUTO || method > ICP_NN_CLUSTER) return ICP_ERR_INVALID_ARG;
  if (M < 0 || N <= 0 || M > (1 << 28) || N > (1 << 28) || !Q_dev) return ICP_ERR_INVALID_ARG;
  if (M == 0) return ICP_OK;
  if (!P_dev || !idx_out_dev || !d2_out_dev) return ICP_ERR_INVALID_ARG;
  if (!rigid_ok(T)) return ICP_ERR_INVALID_ARG;
  OwnedRequest r;
  r.P_dev = P_dev; r.Q_dev = Q_dev;
  r.M = M; r.N = N;
  icp_params_default(ICP_P2P_L2, &r.prm);
  r.query = true;
  std::memcpy(r.Tq, T, sizeof r.Tq);
  r.qmethod = method;
  r.idx_dev_out = idx_out_dev;
  r.d2_dev_out = d2_out_dev;
  std::lock_guard<std::mutex> g(ctx->sync_mu);
  icp_result res;
  return run_sync(ctx, r, &res, stream, nullptr, nullptr);
}

icp_status icp_nn_query_dev_noalloc(const float* P_dev, int64_t M, const float* Q_dev, int64_t N,
                                    const double T[16], icp_nn_method method, int32_t* idx_out_dev,
                                    float* d2_out_dev, void* stream) {
  if (!T || method < ICP_NN_AUTO || method > ICP_NN_CLUSTER) return ICP_ERR_INVALID_ARG;
  if (M < 0 || N <= 0 || M > (1 << 28) || N > (1 << 28) || !Q_dev) return ICP_ERR_INVALID_ARG;
  if (M == 0) return ICP_OK;
  if (!P_dev || !idx_out_dev || !d2_out_dev) return ICP_ERR_INVALID_ARG;
  if (!rigid_ok(T)) return ICP_ERR_INVALID_ARG;
  Layout L;
  L.plan(M, N, false, false, 0);
  if (kNoAllocSlot + L.total > kNoAllocBytes) return ICP_ERR_OOM;
  NoAllocDevice* nd = noalloc_device();
  if (!nd) return ICP_ERR_DEVICE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  unsigned char* base = nd->ptr;
  SlotDesc* desc = reinterpret_cast<SlotDesc*>(base + kNoAllocDesc);
  SlotState* state = reinterpret_cast<SlotState*>(base + kNoAllocState);
  WorkList* wl = reinterpret_cast<WorkList*>(base + kNoAllocWl);
  int* done = reinterpret_cast<int*>(base + kNoAllocDone);
  char* b = reinterpret_cast<char*>(base + kNoAllocSlot);
  auto F = [&](size_t o) { return reinterpret_cast<float*>(b + o); };
  auto F4 = [&](size_t o) { return reinterpret_cast<float4*>(b + o); };
  unsigned* sort_scratch = reinterpret_cast<unsigned*>(b + L.o_scratch);
  char* st_base = reinterpret_cast<char*>(state);
  float* bbQ = reinterpret_cast<float*>(st_base + offsetof(SlotState, bbQ));
  float* bbP = reinterpret_cast<float*>(st_base + offsetof(SlotState, bbP));
  double* cQ = reinterpret_cast<double*>(st_base + offsetof(SlotState, cQ));
  double* cP = reinterpret_cast<double*>(st_base + offsetof(SlotState, cP));
  float* rho = reinterpret_cast<float*>(reinterpret_cast<char*>(desc) + offsetof(SlotDesc, rho_max));
  SlotDesc D;
  std::memset(&D, 0, sizeof D);
  D.px = F(L.o_px); D.py = F(L.o_py); D.pz = F(L.o_pz);
  D.perm = reinterpret_cast<int*>(b + L.o_perm);
  D.tsph = reinterpret_cast<double4*>(b + L.o_tsph);
  D.qx = F(L.o_qx); D.qy = F(L.o_qy); D.qz = F(L.o_qz);
  D.qloc = F4(L.o_qloc); D.qorg = F4(L.o_qorg); D.ccen = F4(L.o_ccen);
  D.clo = F4(L.o_clo); D.chi = F4(L.o_chi); D.slo = F4(L.o_slo); D.shi = F4(L.o_shi);
  D.kbox = F4(L.o_kbox);
  D.keys = reinterpret_cast<unsigned long long*>(b + L.o_keys);
  D.clist = reinterpret_cast<int*>(b + L.o_clist);
  D.squeue = reinterpret_cast<int4*>(b + L.o_squeue);
  D.scount = reinterpret_cast<int*>(b + L.o_scount);
  D.nnidx = reinterpret_cast<int32_t*>(b + L.o_nnidx);
  D.nnd2 = F(L.o_nnd2);
  D.part = reinterpret_cast<double*>(b + L.o_part);
  D.medkey = reinterpret_cast<double*>(b + L.o_med);
  D.idx_out = idx_out_dev;
  D.d2_out = d2_out_dev;
  D.stats = reinterpret_cast<unsigned long long*>(b + L.o_stats);
  D.M = L.M; D.N = L.N; D.ntile = L.ntile; D.ncl = L.ncl; D.nsup = L.nsup; D.nepi = L.nepi;
  if (method == ICP_NN_AUTO) method = ((double)L.M * L.N <= 64.0e6) ? ICP_NN_BRUTE : ICP_NN_CLUSTER;
  D.method = method == ICP_NN_BRUTE ? NN_BRUTE : NN_CLUSTER;
  D.mode = P2P_L2;
  D.slice_min = kSliceMinDefault;
  D.brute_clusters = kBruteClustersDefault;
  D.brute_items = kBruteItemsDefault;
  QueryT qt;
  std::memcpy(qt.T, T, sizeof qt.T);
  (void)hipGetLastError();
  hipLaunchKernelGGL(noalloc_init_kernel, dim3(1), dim3(256), 0, st, desc, state, wl, done, D, qt);
  // the setup of icp_nn_query_dev (Engine::admit) with device inputs, on the caller's stream
  launch_aos_to_soa(Q_dev, L.N, F(L.o_qx), F(L.o_qy), F(L.o_qz), st);
  launch_aos_to_soa(P_dev, L.M, F(L.o_pox), F(L.o_poy), F(L.o_poz), st);
  launch_bbox(F(L.o_qx), F(L.o_qy), F(L.o_qz), L.N, bbQ, cQ, st);
  unsigned* order = nullptr;
  launch_hilbert_order(F(L.o_qx), F(L.o_qy), F(L.o_qz), L.N, bbQ, sort_scratch, &order, st);
  launch_build_clusters(F(L.o_qx), F(L.o_qy), F(L.o_qz), order, L.N, L.ncl, F4(L.o_qloc), F4(L.o_qorg),
                        F4(L.o_ccen), F4(L.o_clo), F4(L.o_chi), F4(L.o_kbox), st);
  launch_build_super(F4(L.o_clo), F4(L.o_chi), F4(L.o_ccen), L.ncl, L.nsup, F4(L.o_slo), F4(L.o_shi),
                     rho, kVerletFracDefault, st);
  launch_bbox(F(L.o_pox), F(L.o_poy), F(L.o_poz), L.M, bbP, cP, st);
  launch_hilbert_order(F(L.o_pox), F(L.o_poy), F(L.o_poz), L.M, bbP, sort_scratch, &order, st);
  launch_build_tiles(F(L.o_pox), F(L.o_poy), F(L.o_poz), order, L.M, L.ntile, F(L.o_px), F(L.o_py),
                     F(L.o_pz), reinterpret_cast<int*>(b + L.o_perm), reinterpret_cast<double4*>(b + L.o_tsph),
                     st);
  launch_fill_u64(reinterpret_cast<unsigned long long*>(b + L.o_keys), L.M, ~0ull, st);
  launch_fill_u64(reinterpret_cast<unsigned long long*>(b + L.o_stats), kQueues * kStatStride, 0ull, st);
  launch_fill_u64(reinterpret_cast<unsigned long long*>(b + L.o_nnidx), (L.M + 1) / 2, ~0ull, st);
  // one pass of the one-slot engine: search, output epilogue, solver (marks the query done)
  launch_boot(desc, state, 0, wl, true, st);
  if (D.method == NN_BRUTE) launch_brute(desc, state, nd->nn_grid, st);
  else launch_nn(desc, state, wl, nd->nn_grid, true, st);
  launch_epi(desc, state, wl, nd->epi_grid, true, st);
  launch_solver(desc, state, 1, done, wl, true, st, 0, 1);
  return hipGetLastError() == hipSuccess ? ICP_OK : ICP_ERR_DEVICE;
}

icp_status icp_batch_config(icp_ctx* ctx, int passes_per_replay, int max_slots) {
  if (!ctx || passes_per_replay < 1 || passes_per_replay > 64 || max_slots < 1 || max_slots > kMaxSlots)
    return ICP_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (ctx->running > 0) {
    // shrinking below resident slots is not allowed while pairs run
    if (max_slots < ctx->max_slots) return ICP_ERR_INVALID_ARG;
  }
  ctx->passes_per_replay = passes_per_replay;
  ctx->max_slots = max_slots;
  return ICP_OK;
}

icp_status icp_batch_submit(icp_ctx* ctx, const icp_request* reqs, int n, uint64_t* tickets_out) {
  if (!ctx || n < 0 || (n > 0 && (!reqs || !tickets_out))) return ICP_ERR_INVALID_ARG;
  // host threads for validating and copying a large submission
  int64_t points = 0;
  for (int i = 0; i < n; ++i) points += std::max<int64_t>(reqs[i].M, 0) + std::max<int64_t>(reqs[i].N, 0);
  const int threads = points >= (int64_t)1 << 20
                          ? (int)std::min<unsigned>(kSubmitThreads, std::max(1u, std::thread::hardware_concurrency()))
                          : 1;
  {
    std::vector<icp_status> v(n, ICP_OK);
    parallel_items(n, threads, [&](int i) {
      const icp_request& q = reqs[i];
      v[i] = validate_host(q.P, q.M, q.Q, q.Qn, q.N, &q.params);
    });
    for (int i = 0; i < n; ++i)
      if (v[i] != ICP_OK) return v[i];
  }
  const auto now = Clock::now();
  uint64_t first;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->failed) return ICP_ERR_DEVICE;
    if (ctx->queue.size() + ctx->reserved + n > kQueueCap) return ICP_ERR_QUEUE_FULL;
    first = ctx->next_ticket;
    ctx->next_ticket += (uint64_t)n;
    ctx->reserved += (size_t)n;
    for (int i = 0; i < n; ++i) {
      tickets_out[i] = first + (uint64_t)i;
      ctx->state[tickets_out[i]] = 0;
    }
    if (!ctx->started && n > 0) {
      ctx->started = true;
      ctx->worker = std::thread(scheduler, ctx);
    }
  }
  // Copy and queue one request at a time: the scheduler sets up and advances
  // the first requests while the later ones are still being copied. A
  // request whose host copy cannot be allocated is reported as ICP_ERR_OOM
  // by icp_poll.
  parallel_items(n, threads, [&](int i) {
    const icp_request& q = reqs[i];
    std::unique_ptr<OwnedRequest> r;
    try {
      r = std::make_unique<OwnedRequest>();
      r->P.assign(q.P, q.P + 3 * q.M);
      r->Q.assign(q.Q, q.Q + 3 * q.N);
      if (mode_plane(q.params.mode)) r->Qn.assign(q.Qn, q.Qn + 3 * q.N);
    } catch (const std::bad_alloc&) {
      r.reset();
    }
    {
      std::lock_guard<std::mutex> lk(ctx->mu);
      ctx->reserved--;
      if (!r) {
        ctx->state[tickets_out[i]] = 3;
        ctx->cv_done.notify_all();
        return;
      }
      r->M = q.M; r->N = q.N; r->prm = q.params;
      tune_request(ctx, *r, 1);
      r->t_submit = now;
      r->ticket = tickets_out[i];
      ctx->queue.push_back(std::move(r));
    }
    ctx->cv.notify_all();
  });
  return ICP_OK;
}

icp_status icp_batch_submit_dev(icp_ctx* ctx, const icp_request* reqs, int n, uint64_t* tickets_out,
                                void* stream) {
  if (!ctx || n < 0 || (n > 0 && (!reqs || !tickets_out))) return ICP_ERR_INVALID_ARG;
  for (int i = 0; i < n; ++i) {
    const icp_request& q = reqs[i];
    if (!q.P || !q.Q) return ICP_ERR_INVALID_ARG;
    icp_status st = check_sizes(q.M, q.N);
    if (st == ICP_OK) st = check_params_sized(&q.params, q.N);
    if (st == ICP_OK && mode_plane(q.params.mode) && !q.Qn) st = ICP_ERR_NO_NORMALS;
    if (st != ICP_OK) return st;
  }
  if (n == 0) return ICP_OK;
  if (hipSetDevice(ctx->device) != hipSuccess) return ICP_ERR_DEVICE;
  auto ready = std::make_shared<ReadyEvent>();
  if (hipEventCreateWithFlags(&ready->ev, hipEventDisableTiming) != hipSuccess) {
    ready->ev = nullptr;
    return ICP_ERR_DEVICE;
  }
  if (hipEventRecord(ready->ev, reinterpret_cast<hipStream_t>(stream)) != hipSuccess) return ICP_ERR_DEVICE;
  const auto now = Clock::now();
  std::vector<std::unique_ptr<OwnedRequest>> rs(n);
  for (int i = 0; i < n; ++i) {
    const icp_request& q = reqs[i];
    auto r = std::make_unique<OwnedRequest>();
    r->P_dev = q.P; r->Q_dev = q.Q;
    r->Qn_dev = mode_plane(q.params.mode) ? q.Qn : nullptr;
    r->M = q.M; r->N = q.N; r->prm = q.params;
    r->ready = ready;
    r->t_submit = now;
    rs[i] = std::move(r);
  }
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->failed) return ICP_ERR_DEVICE;
    if (ctx->queue.size() + ctx->reserved + n > kQueueCap) return ICP_ERR_QUEUE_FULL;
    const uint64_t first = ctx->next_ticket;
    ctx->next_ticket += (uint64_t)n;
    for (int i = 0; i < n; ++i) {
      tickets_out[i] = first + (uint64_t)i;
      ctx->state[tickets_out[i]] = 0;
      tune_request(ctx, *rs[i], 1);
      rs[i]->ticket = tickets_out[i];
      ctx->queue.push_back(std::move(rs[i]));
    }
    if (!ctx->started) {
      ctx->started = true;
      ctx->worker = std::thread(scheduler, ctx);
    }
  }
  ctx->cv.notify_all();
  return ICP_OK;
}

icp_status icp_poll(icp_ctx* ctx, uint64_t ticket, icp_result* out) {
  if (!ctx) return ICP_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(ctx->mu);
  auto it = ctx->state.find(ticket);
  if (it == ctx->state.end()) return ICP_ERR_UNKNOWN_TICKET;
  if (it->second == 0 || it->second == 1) return ctx->failed ? ICP_ERR_DEVICE : ICP_ERR_NOT_READY;
  const int st = it->second;
  ctx->state.erase(it);
  auto r = ctx->results.find(ticket);
  if (st == 3) { if (r != ctx->results.end()) ctx->results.erase(r); return ICP_ERR_OOM; }
  if (st == 4) { if (r != ctx->results.end()) ctx->results.erase(r); return ICP_ERR_DEVICE; }
  if (out && r != ctx->results.end()) *out = r->second;
  if (r != ctx->results.end()) ctx->results.erase(r);
  return ICP_OK;
}

icp_status icp_profile(icp_ctx* ctx, int enable) {
  if (!ctx) return ICP_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(ctx->sync_mu);
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->sync_eng.prof = enable != 0;
  ctx->batch_eng.prof_req = enable != 0;  // taken up by the scheduler's next round
  for (Engine* E : {&ctx->sync_eng, &ctx->batch_eng}) {
    E->prof_ms[0] = E->prof_ms[1] = E->prof_ms[2] = 0.0;
    E->prof_passes = 0;
  }
  return ICP_OK;
}

icp_status icp_profile_read(icp_ctx* ctx, icp_profile_stats* out) {
  if (!ctx || !out) return ICP_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(ctx->sync_mu);
  std::lock_guard<std::mutex> lk(ctx->mu);
  std::memset(out, 0, sizeof *out);
  for (Engine* E : {&ctx->sync_eng, &ctx->batch_eng}) {
    out->nn_ms += E->prof_ms[0];
    out->reduce_ms += E->prof_ms[1];
    out->solve_ms += E->prof_ms[2];
    out->passes += E->prof_passes;
  }
  return ICP_OK;
}

icp_status icp_tuning_default(icp_tuning* out) {
  if (!out) return ICP_ERR_INVALID_ARG;
  *out = default_tuning();
  return ICP_OK;
}

icp_status icp_tuning_lookup(icp_ctx* ctx, int64_t M, int64_t N, icp_mode mode, icp_nn_method method,
                             int batch, icp_tuning* out, int* found) {
  if (!ctx || !out || M <= 0 || N <= 0 || mode < ICP_P2P_L2 || mode > ICP_P2PL_L2 ||
      method < ICP_NN_AUTO || method > ICP_NN_CLUSTER || (batch != 0 && batch != 1))
    return ICP_ERR_INVALID_ARG;
  *out = lookup_tuning(ctx, M, N, mode, method, batch, found);
  return ICP_OK;
}

icp_status icp_tuning_set(icp_ctx* ctx, const icp_tuning_entry* e) {
  if (!ctx || !e || e->m_bucket < 0 || e->m_bucket > 62 || e->n_bucket < 0 || e->n_bucket > 62 ||
      e->mode < ICP_P2P_L2 || e->mode > ICP_P2PL_L2 ||
      (e->method != ICP_NN_BRUTE && e->method != ICP_NN_CLUSTER) || (e->batch != 0 && e->batch != 1) ||
      !tuning_valid(e->tuning))
    return ICP_ERR_INVALID_ARG;
  put_tuning(ctx, *e);
  return ICP_OK;
}

icp_status icp_tuning_entries(icp_ctx* ctx, icp_tuning_entry* out, int cap, int* n) {
  if (!ctx || !n || cap < 0 || (cap > 0 && !out)) return ICP_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(ctx->tune_mu);
  *n = (int)ctx->tuning.size();
  for (int i = 0; i < std::min(cap, *n); ++i) out[i] = ctx->tuning[i];
  return ICP_OK;
}

icp_status icp_device_arch(int device, char* out, int cap) {
  if (!out || cap < 2) return ICP_ERR_INVALID_ARG;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return ICP_ERR_DEVICE;
  std::string a(prop.gcnArchName);
  a = a.substr(0, a.find(':'));
  if ((int)a.size() + 1 > cap) return ICP_ERR_INVALID_ARG;
  std::memcpy(out, a.c_str(), a.size() + 1);
  return ICP_OK;
}

icp_status icp_tuning_file_write(const char* path, const char* arch, const icp_tuning_entry* e, int n) {
  if (!path || !arch || n < 0 || (n > 0 && !e)) return ICP_ERR_INVALID_ARG;
  for (const char* p = arch; *p; ++p)
    if (*p == '"' || *p == '\\' || (unsigned char)*p < 32) return ICP_ERR_INVALID_ARG;
  FILE* f = std::fopen(path, "w");
  if (!f) return ICP_ERR_INVALID_ARG;
  std::fprintf(f, "{\"arch\": \"%s\", \"entries\": [", arch);
  for (int i = 0; i < n; ++i) {
    const icp_tuning_entry& x = e[i];
    std::fprintf(f,
                 "%s\n  {\"m_bucket\": %d, \"n_bucket\": %d, \"mode\": %d, \"method\": %d, \"batch\": %d, "
                 "\"slice_min\": %d, \"list_margin\": %.9g, \"brute_clusters\": %d, "
                 "\"brute_items\": %d, \"grid_per_cu\": %d, \"ms\": %.6g}",
                 i ? "," : "", x.m_bucket, x.n_bucket, x.mode, x.method, x.batch, x.tuning.slice_min,
                 (double)x.tuning.list_margin, x.tuning.brute_clusters, x.tuning.brute_items,
                 x.tuning.grid_per_cu, x.ms);
  }
  std::fprintf(f, "\n]}\n");
  return std::fclose(f) == 0 ? ICP_OK : ICP_ERR_INVALID_ARG;
}

// A small reader for the format above: the "arch" string, then every object
// of the "entries" array as "key": number pairs.
icp_status icp_tuning_file_read(const char* path, const char* arch, icp_tuning_entry* out, int cap,
                                int* n) {
  if (!path || !n || cap < 0 || (cap > 0 && !out)) return ICP_ERR_INVALID_ARG;
  *n = 0;
  FILE* f = std::fopen(path, "r");
  if (!f) return ICP_ERR_INVALID_ARG;
  std::string txt;
  char buf[4096];
  for (size_t k; (k = std::fread(buf, 1, sizeof buf, f)) > 0;) txt.append(buf, k);
  std::fclose(f);
  size_t p = txt.find("\"arch\"");
  if (p == std::string::npos) return ICP_ERR_INVALID_ARG;
  p = txt.find('"', txt.find(':', p));
  const size_t q = p == std::string::npos ? p : txt.find('"', p + 1);
  if (q == std::string::npos) return ICP_ERR_INVALID_ARG;
  const std::string farch = txt.substr(p + 1, q - p - 1);
  size_t at = txt.find("\"entries\"");
  if (at == std::string::npos || (at = txt.find('[', at)) == std::string::npos) return ICP_ERR_INVALID_ARG;
  const size_t end = txt.find(']', at);
  if (end == std::string::npos) return ICP_ERR_INVALID_ARG;
  std::vector<icp_tuning_entry> got;
  for (size_t o = txt.find('{', at); o != std::string::npos && o < end; o = txt.find('{', o + 1)) {
    const size_t c = txt.find('}', o);
    if (c == std::string::npos || c > end) return ICP_ERR_INVALID_ARG;
    const std::string obj = txt.substr(o + 1, c - o - 1);
    auto num = [&](const char* key, double* v) -> bool {
      const std::string k = std::string("\"") + key + "\"";
      const size_t kp = obj.find(k);
      if (kp == std::string::npos) return false;
      const size_t cp = obj.find(':', kp + k.size());
      if (cp == std::string::npos) return false;
      const char* s0 = obj.c_str() + cp + 1;
      char* e0 = nullptr;
      *v = std::strtod(s0, &e0);
      return e0 != s0 && std::isfinite(*v);
    };
    double v[11];
    const char* keys[11] = {"m_bucket", "n_bucket", "mode", "method", "batch", "slice_min", "list_margin",
                            "brute_clusters", "brute_items", "grid_per_cu", "ms"};
    for (int k = 0; k < 11; ++k)
      if (!num(keys[k], &v[k])) return ICP_ERR_INVALID_ARG;
    icp_tuning_entry x;
    x.m_bucket = (int)v[0]; x.n_bucket = (int)v[1]; x.mode = (int)v[2]; x.method = (int)v[3];
    x.batch = (int)v[4];
    x.tuning.slice_min = (int)v[5];
    x.tuning.list_margin = (float)v[6];
    x.tuning.brute_clusters = (int)v[7];
    x.tuning.brute_items = (int)v[8];
    x.tuning.grid_per_cu = (int)v[9];
    x.ms = v[10];
    if (x.m_bucket < 0 || x.m_bucket > 62 || x.n_bucket < 0 || x.n_bucket > 62 || x.mode < 0 || x.mode > 3 ||
        (x.method != ICP_NN_BRUTE && x.method != ICP_NN_CLUSTER) || (x.batch != 0 && x.batch != 1) ||
        !tuning_valid(x.tuning))
      return ICP_ERR_INVALID_ARG;
    got.push_back(x);
    o = c;
  }
  if (arch && farch != arch) return ICP_OK;  // another architecture's table: nothing for this one
  *n = (int)got.size();
  for (int i = 0; i < std::min(cap, *n); ++i) out[i] = got[i];
  return ICP_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ autotuner

// Test pair of the tuner: a bumpy sphere r = 1 + 0.1 sin(3 theta) sin(4 phi),
// targets on u_z >= -7/13, sources independently on u_z <= 7/13 moved by 20
// degrees and a small translation, noise 2e-3 diag, 10% uniform outliers;
// radial normals. Its own xorshift generator (timing input only).
namespace {
struct TuneRng {
  uint64_t s;
  uint64_t next() { s ^= s << 13; s ^= s >> 7; s ^= s << 17; return s; }
  double uni() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
  double gauss() {
    const double u1 = std::max(uni(), 1e-300), u2 = uni();
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
  }
};

void bumpy(TuneRng& g, int64_t n, double zlo, double zhi, std::vector<float>& pts, std::vector<float>* nrm) {
  pts.resize(3 * n);
  if (nrm) nrm->resize(3 * n);
  for (int64_t i = 0; i < n; ++i) {
    const double z = zlo + (zhi - zlo) * g.uni(), ph = 6.283185307179586 * g.uni();
    const double st = std::sqrt(std::max(0.0, 1.0 - z * z)), th = std::acos(z);
    const double u[3] = {st * std::cos(ph), st * std::sin(ph), z};
    const double r = 1.0 + 0.1 * std::sin(3.0 * th) * std::sin(4.0 * ph);
    for (int a = 0; a < 3; ++a) {
      pts[3 * i + a] = (float)(r * u[a]);
      if (nrm) (*nrm)[3 * i + a] = (float)u[a];
    }
  }
}

void tune_pair(int64_t M, int64_t N, std::vector<float>& P, std::vector<float>& Q, std::vector<float>& Qn,
               double* diag) {
  TuneRng g{0x9e3779b97f4a7c15ull ^ (uint64_t)(M * 1000003 + N)};
  bumpy(g, N, -7.0 / 13.0, 1.0, Q, &Qn);
  float lo[3] = {1e30f, 1e30f, 1e30f}, hi[3] = {-1e30f, -1e30f, -1e30f};
  for (int64_t i = 0; i < N; ++i)
    for (int a = 0; a < 3; ++a) { lo[a] = std::min(lo[a], Q[3 * i + a]); hi[a] = std::max(hi[a], Q[3 * i + a]); }
  *diag = std::sqrt(double(hi[0] - lo[0]) * (hi[0] - lo[0]) + double(hi[1] - lo[1]) * (hi[1] - lo[1]) +
                    double(hi[2] - lo[2]) * (hi[2] - lo[2]));
  bumpy(g, M, -1.0, 7.0 / 13.0, P, nullptr);
  const double ang = 20.0 * 3.141592653589793 / 180.0, k[3] = {0.2672612, 0.5345225, 0.8017837};
  const double c = std::cos(ang), s = std::sin(ang);
  const double R[9] = {c + k[0] * k[0] * (1 - c), k[0] * k[1] * (1 - c) - k[2] * s, k[0] * k[2] * (1 - c) + k[1] * s,
                       k[1] * k[0] * (1 - c) + k[2] * s, c + k[1] * k[1] * (1 - c), k[1] * k[2] * (1 - c) - k[0] * s,
                       k[2] * k[0] * (1 - c) - k[1] * s, k[2] * k[1] * (1 - c) + k[0] * s, c + k[2] * k[2] * (1 - c)};
  const double t[3] = {0.05, -0.03, 0.02}, sig = 2e-3 * *diag;
  float plo[3] = {1e30f, 1e30f, 1e30f}, phi[3] = {-1e30f, -1e30f, -1e30f};
  for (int64_t i = 0; i < M; ++i) {
    double x[3];
    for (int a = 0; a < 3; ++a) x[a] = P[3 * i + a] + sig * g.gauss();
    for (int a = 0; a < 3; ++a) {
      P[3 * i + a] = (float)(R[3 * a] * x[0] + R[3 * a + 1] * x[1] + R[3 * a + 2] * x[2] + t[a]);
      plo[a] = std::min(plo[a], P[3 * i + a]);
      phi[a] = std::max(phi[a], P[3 * i + a]);
    }
  }
  for (int64_t i = 0; i < M; ++i)
    if (g.uni() < 0.1)
      for (int a = 0; a < 3; ++a) P[3 * i + a] = (float)(plo[a] + (phi[a] - plo[a]) * g.uni());
}
}  // namespace

extern "C" {

icp_status icp_autotune(icp_ctx* ctx, int64_t M, int64_t N, icp_mode mode, icp_nn_method method,
                        int batch, icp_tuning_entry* best_out) {
  if (!ctx || check_sizes(M, N) != ICP_OK || mode < ICP_P2P_L2 || mode > ICP_P2PL_L2 ||
      method < ICP_NN_AUTO || method > ICP_NN_CLUSTER || (batch != 0 && batch != 1))
    return ICP_ERR_INVALID_ARG;
  method = resolve_method(M, N, method);
  const bool plane = mode_plane(mode);
  std::vector<float> P, Q, Qn;
  double diag = 1.0;
  tune_pair(M, N, P, Q, Qn, &diag);
  icp_params prm;
  icp_params_default(mode, &prm);
  prm.nu_min = mode_l2(mode) ? 0.0 : (plane ? 1e-3 : 1e-3 * diag);
  prm.max_total_iter = 40;
  prm.nn = method;
  prm.engine = ICP_ENGINE_GRAPH;
  const icp_tuning d0 = default_tuning();
  std::vector<icp_tuning> cands{d0};
  for (int grid : {8, 16, 32}) {
    if (batch && grid != d0.grid_per_cu) continue;  // the batch engine's grid is not per pair
    if (method == ICP_NN_CLUSTER) {
      for (int sm : {4, 6, 8, 12})
        for (float mg : {0.04f, 0.08f, 0.16f}) {
          icp_tuning t = d0;
          t.slice_min = sm; t.list_margin = mg; t.grid_per_cu = grid;
          cands.push_back(t);
        }
    } else if (!batch) {
      for (int bi : {2048, 4096, 8192, 12288, 16384, 24576, 32768}) {
        icp_tuning t = d0;
        t.brute_items = bi; t.grid_per_cu = grid;
        cands.push_back(t);
      }
    } else {
      for (int cpi : {4, 8, 16, 32}) {
        icp_tuning t = d0;
        t.brute_clusters = cpi;
        cands.push_back(t);
      }
    }
  }
  icp_tuning_entry e;
  e.m_bucket = size_bucket(M);
  e.n_bucket = size_bucket(N);
  e.mode = mode_family(mode);
  e.method = method;
  e.batch = batch;
  e.tuning = d0;
  e.ms = 0.0;
  // reference result of the defaults (the pair alone)
  icp_result ref{};
  {
    std::lock_guard<std::mutex> g(ctx->sync_mu);
    OwnedRequest r;
    r.P = P; r.Q = Q;
    if (plane) r.Qn = Qn;
    r.M = M; r.N = N; r.prm = prm;
    r.tune = d0;
    r.tune_fixed = true;
    const icp_status rc = run_sync(ctx, r, &ref, nullptr, nullptr, nullptr);
    if (rc != ICP_OK) return rc;
  }
  double best_ms = 1e300;
  icp_tuning best = d0;
  // copies in flight for the batch kind: 16, fewer for large pairs (about
  // 4e6 points in flight)
  const int copies = (int)std::max<int64_t>(2, std::min<int64_t>(16, 4000000 / (M + N)));
  std::vector<icp_request> reqs(batch ? copies : 0);
  for (auto& q : reqs) {
    q.P = P.data(); q.M = M; q.Q = Q.data(); q.Qn = plane ? Qn.data() : nullptr; q.N = N; q.params = prm;
  }
  // the table entry of this bucket while the batch candidates run (restored below)
  std::vector<icp_tuning_entry> saved;
  {
    std::lock_guard<std::mutex> g(ctx->tune_mu);
    saved = ctx->tuning;
  }
  icp_status status = ICP_OK;
  for (size_t ci = 0; ci < cands.size() && status == ICP_OK; ++ci) {
    double ms = 1e300;
    for (int rep = 0; rep < 3 && status == ICP_OK; ++rep) {
      if (!batch) {
        std::lock_guard<std::mutex> g(ctx->sync_mu);
        OwnedRequest r;
        r.P = P; r.Q = Q;
        if (plane) r.Qn = Qn;
        r.M = M; r.N = N; r.prm = prm;
        r.tune = cands[ci];
        r.tune_fixed = true;
        icp_result res{};
        status = run_sync(ctx, r, &res, nullptr, nullptr, nullptr);
        if (status == ICP_OK && (std::memcmp(res.T, ref.T, sizeof ref.T) != 0 || res.nn_passes != ref.nn_passes))
          status = ICP_ERR_DEVICE;  // a partition must never change the result
        if (rep > 0) ms = std::min(ms, res.latency_ms);
      } else {
        icp_tuning_entry t = e;
        t.tuning = cands[ci];
        put_tuning(ctx, t);
        std::vector<uint64_t> tk(reqs.size());
        const auto t0 = Clock::now();
        status = icp_batch_submit(ctx, reqs.data(), (int)reqs.size(), tk.data());
        if (status == ICP_OK) status = icp_batch_wait_all(ctx);
        const double el = std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
        for (uint64_t k : tk) {
          icp_result res{};
          const icp_status pr = icp_poll(ctx, k, &res);
          if (status == ICP_OK && pr != ICP_OK) status = pr;
          if (status == ICP_OK &&
              (std::memcmp(res.T, ref.T, sizeof ref.T) != 0 || res.nn_passes != ref.nn_passes))
            status = ICP_ERR_DEVICE;
        }
        if (rep > 0) ms = std::min(ms, el);
      }
    }
    if (status == ICP_OK && ms < best_ms) { best_ms = ms; best = cands[ci]; }
  }
  if (status != ICP_OK) {
    std::lock_guard<std::mutex> g(ctx->tune_mu);
    ctx->tuning = saved;
    return status;
  }
  e.tuning = best;
  e.ms = best_ms;
  put_tuning(ctx, e);
  if (best_out) *best_out = e;
  return ICP_OK;
}

icp_status icp_batch_wait_all(icp_ctx* ctx) {
  if (!ctx) return ICP_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(ctx->mu);
  // a request is pending while it is queued, being copied by a submission
  // (reserved), between its pop from the queue and its activation or
  // rejection (admitting), or running
  ctx->cv_done.wait(lk, [&] {
    return ctx->failed ||
           (ctx->queue.empty() && ctx->reserved == 0 && ctx->admitting == 0 && ctx->running == 0);
  });
  return ctx->failed ? ICP_ERR_DEVICE : ICP_OK;
}

}  // extern "C"
