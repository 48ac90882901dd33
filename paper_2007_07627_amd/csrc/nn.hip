// Closest-point query of every transformed source point (Sec. 3, eq.
// CorresponcePoint) on gfx950.
//
// Result definition (exact, bit-for-bit): the source point is transformed in
// FP64 with a fixed fused order and rounded once to FP32 (p'); for every target
// q the FP32 distance d2 = fma(dz, dz, fma(dy, dy, dx * dx)) with FP32
// differences is formed; the minimum wins and ties go to the lowest original
// target index. The key (bits(d2) << 32 | index) orders exactly that way.
//
// How it is computed fast without changing that result:
//  * Targets are kept in clusters of 128 Hilbert-ordered points, stored relative
//    to the cluster centre cc together with h = |q - cc|^2 / 2. For a source,
//    the filter value 2 (h - (p' - cc) . (q - cc)) + |p' - cc|^2 equals the
//    squared distance up to a rounding error that is bounded per cluster; it
//    costs 3 FMA per pair and a share of a min tree.
//  * Per lane only the minimum filter value of each 16-target chunk is kept,
//    as certified bounds: the chunk with the smallest upper bound and the
//    smallest lower bounds among the others. At the end the winning chunk is
//    rescanned with the exact FP32 definition; a second chunk that comes
//    within the error bound of the winner is rescanned too, and with a third
//    every cluster the lane can still need is rescanned exactly.
//  * Cluster culling (method NN_CLUSTER): a bounding sphere of the 64-source
//    tile, transformed per pass, against super-cluster and cluster AABBs gives
//    a candidate list; per lane, a cluster whose AABB distance exceeds the
//    current best by more than the error bound is skipped wave-uniformly, and
//    inside a cluster the chunks whose boxes no lane can need are skipped.
//  * Two kernels per pass: the cull kernel (one 64-source tile per wavefront)
//    builds the tile's candidate list and appends slices of it to a per-pair
//    queue; the slice kernel (persistent, dynamic) filters one slice and
//    merges its exact result into the key with a 64-bit atomic min (order
//    independent), so tiles with many candidates (outliers) spread over many
//    wavefronts. A third kernel runs the exhaustive method of a single
//    resident pair: two tiles per wavefront over static ranges of clusters.
//  * Warm start: the previous pass's closest target bounds each lane's exact
//    minimum before any cluster is read; the candidate list keeps only the
//    clusters some lane of the tile can still need.
#include "icp_internal.h"

namespace icp {

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ void xform_f32(const double* T, float x, float y, float z,
                                          float& ox, float& oy, float& oz) {
  const double X = x, Y = y, Z = z;
  ox = (float)__builtin_fma(T[2], Z, __builtin_fma(T[1], Y, __builtin_fma(T[0], X, T[3])));
  oy = (float)__builtin_fma(T[6], Z, __builtin_fma(T[5], Y, __builtin_fma(T[4], X, T[7])));
  oz = (float)__builtin_fma(T[10], Z, __builtin_fma(T[9], Y, __builtin_fma(T[8], X, T[11])));
}

// Relative error bound of the exact FP32 form d2 = fma(dz,dz, fma(dy,dy, dx*dx))
// against the exact squared distance (5 roundings: |d2 - e| <= 5u e, u =
// 2^-24), with margin: gamma = 1e-6. A target j can equal or beat the winner
// only if e_j <= e_min (1 + 2.1 gamma).
__device__ __forceinline__ float winner_threshold(float H) {
  return H + 2.2e-6f * fabsf(H) + 1e-37f;
}


// Exact FP32 scan of n targets of the original-coordinate array.
// Pointers read from a slot descriptor are generic; loading through a global
// pointer makes the load count only against the vector memory counter
// (generic loads also hold the LDS counter, which would serialise a prefetch
// with the LDS work behind it).
typedef float gv4f __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 load_global(const float4* p, size_t i) {
  const gv4f v = ((const __attribute__((address_space(1))) gv4f*)p)[i];
  return make_float4(v.x, v.y, v.z, v.w);
}
typedef int gv4i __attribute__((ext_vector_type(4)));
__device__ __forceinline__ int4 load_global(const int4* p, size_t i) {
  const gv4i v = ((const __attribute__((address_space(1))) gv4i*)p)[i];
  return make_int4(v.x, v.y, v.z, v.w);
}

template <bool kGlobal>
__device__ __forceinline__ unsigned long long exact_scan(const float4* qorg, int base,
                                                         int n, float px, float py, float pz,
                                                         unsigned long long key) {
  // each target is one 16-byte load issued unconditionally (padding is masked
  // after the load), so the loads of an unrolled group are in flight together
#pragma unroll 16
  for (int j = 0; j < n; ++j) {
    const float4 q = kGlobal ? load_global(qorg, (size_t)(base + j)) : qorg[base + j];
    const int id = __float_as_int(q.w);
    const float dx = px - q.x, dy = py - q.y, dz = pz - q.z;
    const float d = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
    // padding (id < 0) maps to the all-ones key by a sign mask, not a branch
    const unsigned long long k = make_key(d, id) | (unsigned long long)(long long)(id >> 31);
    key = k < key ? k : key;
  }
  return key;
}


// The same lower bound with fused multiply-adds (fewer roundings). Callers
// compare it against a threshold raised by 2^-19 for its rounding: lb2 <=
// thr (1 + 2^-19) holds whenever lb2 (1 - 2^-20) <= thr does.
// The offset from the box is p - clamp(p, lo, hi), the clamp a single median
// of three: p - lo below the box, p - hi above it (the negated values of
// lo - p and p - hi, so the squares are those of the two-sided form), 0
// inside. An empty box (lo = +inf, hi = -inf: the padding chunks of a
// pair's last cluster) gives 0, so such a chunk is filtered, which its
// infinite filter values leave without effect.
__device__ __forceinline__ float box_lb2_fma(float px, float py, float pz, float4 lo, float4 hi) {
  const float dx = px - __builtin_amdgcn_fmed3f(px, lo.x, hi.x);
  const float dy = py - __builtin_amdgcn_fmed3f(py, lo.y, hi.y);
  const float dz = pz - __builtin_amdgcn_fmed3f(pz, lo.z, hi.z);
  return __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
}

// Some lane of `lanes` (a ballot of the lanes that take part) has `need`: the
// vote as one 64-bit ballot, kept in scalar registers.
__device__ __forceinline__ bool wave_any_of(bool need, unsigned long long lanes) {
  return (__builtin_amdgcn_ballot_w64(need) & lanes) != 0ull;
}

__device__ __forceinline__ float box_ub2(float px, float py, float pz, float4 lo, float4 hi) {
  const float dx = fmaxf(fabsf(px - lo.x), fabsf(px - hi.x));
  const float dy = fmaxf(fabsf(py - lo.y), fabsf(py - hi.y));
  const float dz = fmaxf(fabsf(pz - lo.z), fabsf(pz - hi.z));
  return dx * dx + dy * dy + dz * dz;
}

// Per-lane filter state over the chunks seen so far: A is the chunk with the
// smallest upper bound H (its lower bound loA); B is the chunk with the
// smallest lower bound S among the others, and S2 the smallest lower bound
// of the rest. The winner lies in a chunk whose lower bound is at most H.
struct LaneBest {
  float H, loA, S, S2;
  int A, B;  // global chunk ids (cluster * kChunksPerCluster + chunk)
};

// Lane j's value of a float, as a wave-uniform scalar.
__device__ __forceinline__ float lane_f(float v, int j) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), j));
}

// Process one cluster with the filter (in chunks of kChunk targets) from its
// copy staged in LDS; every lane reads the same target, so each read is a
// broadcast. With kPrune, chunks that no lane can need are skipped: every
// target of a chunk is at exact squared distance >= lb2 from the lane's point
// (the chunk's box bound, lowered by 2^-20 for its own rounding), and the lane
// needs only targets within winner_threshold(min(H, W)) (W: warm bound), so a
// chunk above that for every lane holds only targets strictly farther than
// each lane's winner (no tie can be lost). The boxes of all chunks are tested
// together before the first chunk is filtered. The exhaustive method filters
// every chunk. The filter value of a target is
// v = 2 (h - pl . ql) + |pl|^2 with pl = p' - cc, h = |ql|^2 / 2, evaluated as
// three FMAs and a final FMA; its distance to the exact squared distance is at
// most u (7 (|pl| + rho)^2 + |v|) (rounding of the centred coordinates, of h,
// of the three FMAs and of the last FMA); 4u is used, so for the chunk
// minimum v: lo = v - 2^-22 |v| - delta, hi = v + 2^-22 |v| + delta,
// delta = 2^-22 7 (|pl| + rho)^2.
// Minimum of n values by a balanced tree of three-way minima (v_min3: one
// instruction per two values).
template <int N>
__device__ __forceinline__ float min_tree(const float* v) {
  if constexpr (N == 1) {
    return v[0];
  } else if constexpr (N == 2) {
    return fminf(v[0], v[1]);
  } else {
    constexpr int M = (N + 2) / 3;
    float w[M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
      const int a = 3 * i;
      if (a + 2 < N) w[i] = fminf(fminf(v[a], v[a + 1]), v[a + 2]);
      else if (a + 1 < N) w[i] = fminf(v[a], v[a + 1]);
      else w[i] = v[a];
    }
    return min_tree<M>(w);
  }
}

__device__ __forceinline__ void filter_chunk(const float4* __restrict__ qc, int id, float npx,
                                             float npy, float npz, float pp, float delta,
                                             LaneBest& L) {
  float sv[kChunk];
#pragma unroll
  for (int j = 0; j < kChunk; ++j) {
    const float4 a = qc[j];
    sv[j] = __builtin_fmaf(npx, a.x, __builtin_fmaf(npy, a.y, __builtin_fmaf(npz, a.z, a.w)));
  }
  const float v = __builtin_fmaf(2.0f, min_tree<kChunk>(sv), pp);
  // an all-padding chunk has v = +inf: keep lo = hi = +inf (no inf - inf)
  const float e = fminf(0x1.0p-22f * fabsf(v) + delta, 1e38f);
  const float lo = v - e, hi = v + e;
  const bool better = hi < L.H;
  const float olo = better ? L.loA : lo;  // the chunk that is not (or no longer) A
  const int oid = better ? L.A : id;
  const bool nb = olo < L.S;
  L.S2 = fminf(L.S2, nb ? L.S : olo);
  L.B = nb ? oid : L.B;
  L.S = nb ? olo : L.S;
  L.loA = better ? lo : L.loA;
  L.A = better ? id : L.A;
  L.H = fminf(L.H, hi);
}

template <bool kPrune>
__device__ __forceinline__ int filter_cluster(const float4* __restrict__ tg,
                                               const float4* __restrict__ bx, int c, float plx,
                                               float ply, float plz, float rho_c, float px,
                                               float py, float pz, unsigned long long vmask, float W,
                                               LaneBest& L) {
  const float npx = -plx, npy = -ply, npz = -plz;
  const float pp = __builtin_fmaf(plz, plz, __builtin_fmaf(ply, ply, plx * plx));
  // the hardware square root (within a few units in the last place) suffices:
  // the bound below carries a 1e-4 relative margin
  const float t = __builtin_amdgcn_sqrtf(pp) + rho_c;
  const float delta = 0x1.0p-22f * 7.0f * 1.0001f * t * t;
  if (kPrune) {
    const float thr = winner_threshold(fminf(L.H, W)) * (1.0f + 0x1.0p-19f);
    unsigned mask = 0;
#pragma unroll
    for (int ch = 0; ch < kChunksPerCluster; ++ch) {
      const float lb2 = box_lb2_fma(px, py, pz, bx[2 * ch], bx[2 * ch + 1]);
      mask |= wave_any_of(lb2 <= thr, vmask) ? (1u << ch) : 0u;
    }
    mask = __builtin_amdgcn_readfirstlane(mask);  // uniform: the chunk loop runs on scalar bits
    const int n = __builtin_popcount(mask);
    for (; mask; mask &= mask - 1u) {
      const int ch = __builtin_ctz(mask);
      filter_chunk(tg + ch * kChunk, c * kChunksPerCluster + ch, npx, npy, npz, pp, delta, L);
    }
    return n;
  } else {
#pragma unroll 1
    for (int ch = 0; ch < kChunksPerCluster; ++ch)
      filter_chunk(tg + ch * kChunk, c * kChunksPerCluster + ch, npx, npy, npz, pp, delta, L);
    return kChunksPerCluster;
  }
}



// Transformed source point of this lane and its warm-start bound W (the exact
// FP32 squared distance to the previous pass's closest target, inflated so
// that it bounds the exact minimum: d2 >= e (1 - gamma)).
__device__ __forceinline__ void lane_point(const SlotDesc& D, const double* T, int si, bool valid,
                                           bool use_prev, float& ptx, float& pty, float& ptz,
                                           float& W) {
  ptx = pty = ptz = 0.f;
  W = __builtin_inff();
  if (!valid) return;
  xform_f32(T, ldg(D.px, si), ldg(D.py, si), ldg(D.pz, si), ptx, pty, ptz);
  if (use_prev) {
    const int prev = ldg(D.nnidx, si);
    if (prev >= 0 && prev < D.N) {
      const float dx = ptx - ldg(D.qx, prev), dy = pty - ldg(D.qy, prev), dz = ptz - ldg(D.qz, prev);
      const float d = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
      W = d * (1.0f + 4e-6f) + 1e-37f;
    }
  }
}

// The same from coordinates and previous index already loaded (prev < 0: no
// warm bound), so that a caller can issue these loads early.
__device__ __forceinline__ void lane_point_from(const SlotDesc& D, const double* T, bool valid,
                                                float x, float y, float z, int prev, float& ptx,
                                                float& pty, float& ptz, float& W) {
  ptx = pty = ptz = 0.f;
  W = __builtin_inff();
  if (!valid) return;
  xform_f32(T, x, y, z, ptx, pty, ptz);
  if (prev >= 0 && prev < D.N) {
    const float dx = ptx - ldg(D.qx, prev), dy = pty - ldg(D.qy, prev), dz = ptz - ldg(D.qz, prev);
    const float d = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
    W = d * (1.0f + 4e-6f) + 1e-37f;
  }
}

constexpr int kCullWaves = 4;

// ------------------------------------------------------------------ cull kernel
// One block of kCullWaves wavefronts per tile of 64 sources (every wavefront
// holds the tile's 64 sources). Cluster mode: candidate clusters from the
// transformed tile sphere against super-cluster and cluster AABBs, then (with
// warm bounds) only the clusters some lane can still need, tested per lane
// against the boxes staged in LDS, the cluster batches shared out among the
// wavefronts. The first wavefront writes the tile record (flags, count, slice
// length, nearest cluster) and queues the slices. Steps that are not shared
// out run identically in every wavefront.
__global__ __launch_bounds__(64 * kCullWaves) void nn_cull_kernel(
    const SlotDesc* __restrict__ descs, const SlotState* __restrict__ states,
    WorkList* __restrict__ wl) {
  __shared__ float4 s_boxes[kCullWaves][128];  // per wavefront: 64 boxes, lo at [j], hi at [64 + j]
  __shared__ int s_cand[kCandCap];
  __shared__ int s_sup[kSupCap];
  __shared__ int s_item, s_n2;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float4* s_box = s_boxes[wv];
  for (int round = 0;; ++round) {
    if (threadIdx.x == 0) s_item = queue_item(wl->q_nn, round);
    __syncthreads();
    const int g = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (g >= wl->nn_total) break;
    const int a = wave_find_slot(wl->nn_base, wl->n_active, g);
    // a wave-uniform slot keeps the descriptor's fields in scalar registers
    const int slot = __builtin_amdgcn_readfirstlane(wl->slot[a]);
    const SlotDesc& D = descs[slot];
    const SlotState& S = states[slot];
    const int tile = g - wl->nn_base[a];
    const int si = tile * kTile + lane;
    const bool valid = si < D.M;
    const double* T = S.Teval;
    int flags = 0, n = 0, first = -1;
    float ptx, pty, ptz, W;
    lane_point(D, T, si, valid, true, ptx, pty, ptz, W);
    const bool warm = __all(!valid || W < __builtin_inff());
    const double4 ts = D.tsph[tile];
    float cx, cy, cz;
    {
      const double X = ts.x, Y = ts.y, Z = ts.z;
      cx = (float)__builtin_fma(T[2], Z, __builtin_fma(T[1], Y, __builtin_fma(T[0], X, T[3])));
      cy = (float)__builtin_fma(T[6], Z, __builtin_fma(T[5], Y, __builtin_fma(T[4], X, T[7])));
      cz = (float)__builtin_fma(T[10], Z, __builtin_fma(T[9], Y, __builtin_fma(T[8], X, T[11])));
    }
    const float cn = sqrtf(cx * cx + cy * cy + cz * cz);
    const float r = (float)ts.w * 1.00001f + 1e-5f * cn + 1e-30f;
    // every lane's winner lies within U of the tile centre's sphere
    float U = warm ? sqrtf(wave_max(valid ? winner_threshold(W) : 0.0f)) * 1.000001f + 1e-30f
                   : __builtin_inff();
    for (int s2 = lane; s2 < D.nsup; s2 += 64)
      U = fminf(U, sqrtf(box_ub2(cx, cy, cz, load_global(D.slo, s2), load_global(D.shi, s2))) * 1.000001f + r);
    U = wave_min(U);
    // Warm lists are kept for later passes while every source stays within
    // the margin of its position now; a later pass's winner is then within
    // its bound here plus twice the margin (the point and its winner's
    // distance each move by at most the margin).
    const float margin = warm ? 2.0f * D.verlet : 0.0f;
    U += margin;
    // per-lane bound with the margin: (sqrt(thr(W)) + margin)^2, rounded up
    const float bw = sqrtf(winner_threshold(W)) * (1.0f + 0x1.0p-20f) + margin;
    const float thr_m = bw * bw * (1.0f + 0x1.0p-20f);
    // candidate super-clusters: tile-level test, then (warm) each lane's own
    // bound against the boxes staged in LDS
    int nsc = 0;
    for (int base = 0; base < D.nsup; base += 64) {
      const int s2 = base + lane;
      bool c = false;
      float4 blo = make_float4(0.f, 0.f, 0.f, 0.f), bhi = blo;
      if (s2 < D.nsup) {
        blo = load_global(D.slo, s2);
        bhi = load_global(D.shi, s2);
        c = sqrtf(box_lb2(cx, cy, cz, blo, bhi)) * 0.999999f - r <= U * 1.00001f;
      }
      unsigned long long bal = __ballot(c);
      if (warm && bal) {
        wave_lds_sync();
        s_box[lane] = blo;
        s_box[64 + lane] = bhi;
        wave_lds_sync();
        const float thr = thr_m;
        unsigned long long need = 0ull;
        for (unsigned long long m = bal; m; m &= m - 1ull) {
          const int j = __builtin_ctzll(m);
          const float lb2 = box_lb2(ptx, pty, ptz, s_box[j], s_box[64 + j]);
          if (__any(valid && lb2 * (1.0f - 0x1.0p-20f) <= thr)) need |= 1ull << j;
        }
        bal = need;
        c = (bal >> lane) & 1ull;
      }
      const int pos = nsc + __popcll(bal & ((1ull << lane) - 1ull));
      if (c && pos < kSupCap) s_sup[pos] = s2;
      nsc += __popcll(bal);
    }
    __syncthreads();
    const int nflat = nsc > kSupCap ? D.ncl : nsc * kSuper;  // all clusters on overflow
    auto flat_cluster = [&](int f) -> int {
      if (nsc > kSupCap) return f;
      const int c = s_sup[f / kSuper] * kSuper + (f % kSuper);
      return c < D.ncl ? c : -1;
    };
    if (warm) {
      // Stream the candidate clusters in batches of 64: tile-level test, then
      // every lane tests the batch's boxes (staged in LDS) against its own
      // bound; the clusters some lane needs are appended to the list.
      const float thr = thr_m;
      // the candidate batches are shared out among the block's wavefronts;
      // needed clusters are appended through a block counter (the list's
      // order varies, its contents do not)
      if (threadIdx.x == 0) s_n2 = 0;
      __syncthreads();
      for (int base = 64 * wv; base < nflat; base += 64 * kCullWaves) {
        const int f = base + lane;
        int cid = f < nflat ? flat_cluster(f) : -1;
        float4 blo = make_float4(0.f, 0.f, 0.f, 0.f), bhi = blo;
        if (cid >= 0) {
          blo = load_global(D.clo, cid);
          bhi = load_global(D.chi, cid);
          if (!(sqrtf(box_lb2(cx, cy, cz, blo, bhi)) * 0.999999f - r <= U * 1.00001f)) cid = -1;
        }
        const unsigned long long cand = __ballot(cid >= 0);
        if (cand == 0ull) continue;
        wave_lds_sync();
        s_box[lane] = blo;
        s_box[64 + lane] = bhi;
        wave_lds_sync();
        unsigned long long need = 0ull;
        for (unsigned long long m = cand; m; m &= m - 1ull) {
          const int j = __builtin_ctzll(m);
          const float lb2 = box_lb2(ptx, pty, ptz, s_box[j], s_box[64 + j]);
          if (__any(valid && lb2 * (1.0f - 0x1.0p-20f) <= thr)) need |= 1ull << j;
        }
        if (need == 0ull) continue;
        int at = 0;
        if (lane == 0) at = atomicAdd(&s_n2, __popcll(need));
        at = __shfl(at, 0, 64);
        const int pos = at + __popcll(need & ((1ull << lane) - 1ull));
        if (((need >> lane) & 1ull) && pos < kListCap) D.clist[(size_t)tile * kListCap + pos] = cid;
      }
      __syncthreads();
      const int n2 = s_n2;
      if (n2 > kListCap || n2 == 0) {
        // more needed clusters than a list holds (or none, which valid lanes
        // exclude): slices over all clusters, tested per lane
        flags = TI_RANGE | TI_LANETEST | TI_WARM;
        n = D.ncl;
      } else {
        flags = TI_LIST | TI_WARM;
        n = n2;
      }
    } else {
      // No warm start (first pass): tile-level candidates, tightened by the
      // best cluster upper bound; the nearest cluster seeds every slice.
      float bestub = __builtin_inff();
      int bestc = 0x7fffffff;
      int ncand = 0;
      for (int base = 0; base < nflat; base += 64) {
        const int f = base + lane;
        bool c = false;
        const int cid = f < nflat ? flat_cluster(f) : -1;
        if (cid >= 0) {
          const float4 blo = load_global(D.clo, cid), bhi = load_global(D.chi, cid);
          const float lb = sqrtf(box_lb2(cx, cy, cz, blo, bhi)) * 0.999999f - r;
          const float ub = sqrtf(box_ub2(cx, cy, cz, blo, bhi)) * 1.000001f + r;
          if (ub < bestub || (ub == bestub && cid < bestc)) { bestub = ub; bestc = cid; }
          c = lb <= U * 1.00001f;
        }
        const unsigned long long bal = __ballot(c);
        const int pos = ncand + __popcll(bal & ((1ull << lane) - 1ull));
        if (c && pos < kCandCap) s_cand[pos] = cid;
        ncand += __popcll(bal);
      }
      const float Uc = wave_min(bestub);
      int cfirst = (bestub == Uc) ? bestc : 0x7fffffff;
      for (int o = 32; o > 0; o >>= 1) cfirst = min(cfirst, __shfl_xor(cfirst, o, 64));
      first = cfirst;
      if (ncand > kListCap) {
        flags = TI_RANGE | TI_LANETEST;
        n = D.ncl;
      } else {
        U = fminf(U, Uc);
        __syncthreads();
        int n2 = 0;
        for (int base = 0; base < ncand; base += 64) {
          const int f = base + lane;
          int cid = -1;
          if (f < ncand) {
            cid = s_cand[f];
            const float lb = sqrtf(box_lb2(cx, cy, cz, load_global(D.clo, cid), load_global(D.chi, cid))) * 0.999999f - r;
            if (!(lb <= U * 1.00001f) || cid == first) cid = -1;
          }
          const unsigned long long keep = __ballot(cid >= 0);
          const int pos = n2 + __popcll(keep & ((1ull << lane) - 1ull));
          if (cid >= 0) D.clist[(size_t)tile * kListCap + pos] = cid;
          n2 += __popcll(keep);
        }
        flags = TI_LIST | TI_LANETEST;
        n = n2;
      }
    }
    __syncthreads();
    // slices of at least slice_min candidates, at most kMaxSlices per tile
    const int smin = D.slice_min;
    int len = max(smin, (n + kMaxSlices - 1) / kMaxSlices);
    int nsl = max(1, (n + len - 1) / len);
    // each slice record carries everything the slice kernel needs, so that
    // its first loads do not wait on a tile record
    if (wv == 0) {
      int base = 0;
      if (lane == 0) {
        if (len > smin) {
          // a long candidate sequence (rare) is cut into shorter slices while
          // the pair's budget of extra slices lasts: its slices would set the tail
          const int l2 = max(smin, (n + kMaxLongSlices - 1) / kMaxLongSlices);
          const int n2 = (n + l2 - 1) / l2;
          if (n2 > nsl && atomicAdd(D.scount + 1, n2 - kMaxSlices) + (n2 - kMaxSlices) <= kExtraSlices) {
            len = l2;
            nsl = n2;
          }
        }
        base = atomicAdd(D.scount, nsl);
      }
      base = __shfl(base, 0, 64);
      len = __shfl(len, 0, 64);
      nsl = __shfl(nsl, 0, 64);
      for (int k = lane; k < nsl; k += 64)
        D.squeue[base + k] = make_int4(tile, k * len, min(n, (k + 1) * len), flags | ((first + 1) << 4));
    }
  }
}

// Exclusive prefix of the per-pair slice counts (one block).
__global__ __launch_bounds__(1024) void slice_plan_kernel(const SlotDesc* __restrict__ descs,
                                                          const SlotState* __restrict__ states,
                                                          WorkList* __restrict__ wl) {
  __shared__ int s[1024];
  const int t = threadIdx.x;
  const int na = wl->n_active;
  int v = 0;
  // slots that search this pass: their slices from this pass's cull or, when
  // the lists are reused, from the last one
  if (t < na && !states[wl->slot[t]].reuse && descs[wl->slot[t]].method != NN_BRUTE)
    v = *descs[wl->slot[t]].scount;
  s[t] = v;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int x = t >= o ? s[t - o] : 0;
    __syncthreads();
    s[t] += x;
    __syncthreads();
  }
  if (t < kSliceQueues) wl->q_s[t * kQueueStride] = 0;
  if (t < kQueues) wl->q_b[t * kQueueStride] = 0;
  if (t < na) wl->s_base[t] = s[t] - v;
  if (t == 1023) {
    wl->s_base[na] = s[1023];
    wl->s_total = s[1023];
  }
}

// ------------------------------------------------------------------ slice kernel
__device__ void multi_brute_items(const SlotDesc* __restrict__ descs,
                                  const SlotState* __restrict__ states, WorkList* __restrict__ wl,
                                  float4* s_tgt);

__global__ __launch_bounds__(64) void nn_slice_kernel(const SlotDesc* __restrict__ descs,
                                                      const SlotState* __restrict__ states,
                                                      WorkList* __restrict__ wl) {
  __shared__ float4 s_tgt[kCluster];
  __shared__ float4 s_box[2 * kChunksPerCluster];
  static_assert(2 * kChunksPerCluster <= 64, "one box entry per lane");
  const int lane = threadIdx.x;
  // one-slot engine: the slice total is the slot's count (from this pass's
  // cull or, with reused lists, from the last one)
  const int s_total = __builtin_amdgcn_readfirstlane(
      wl->s_from_scount ? ldg(descs[wl->slot[0]].scount, 0) : wl->s_total);
  for (int round = 0;; ++round) {
    int g = 0;
    if (lane == 0) g = slice_queue_item(wl->q_s, s_total, round);
    g = __builtin_amdgcn_readfirstlane(__shfl(g, 0, 64));
    if (g >= s_total) break;
    const int a = wave_find_slot(wl->s_base, wl->n_active, g);
    const int slot = __builtin_amdgcn_readfirstlane(wl->slot[a]);
    const SlotDesc& D = descs[slot];
    const SlotState& S = states[slot];
    const int local = g - wl->s_base[a];
    const long long t_begin = D.item_stats ? (long long)__builtin_readcyclecounter() : 0ll;
    const int4 q = load_global(D.squeue, local);
    const int tile = __builtin_amdgcn_readfirstlane(q.x);
    const int p0 = __builtin_amdgcn_readfirstlane(q.y), p1 = __builtin_amdgcn_readfirstlane(q.z);
    const int meta = __builtin_amdgcn_readfirstlane(q.w);
    const int flags = meta & 15, first = (meta >> 4) - 1;
    const int si = tile * kTile + lane;
    const bool valid = si < D.M;
    const int* __restrict__ list = D.clist + (size_t)tile * kListCap;
    const bool from_list = (flags & TI_LIST) != 0;
    // per-lane box test before a cluster is filtered: range tiles, and warm
    // lists (built with the reuse margin, so this pass may need fewer)
    const bool lane_test = (flags & (TI_LANETEST | TI_WARM)) != 0;
    // cluster sequence of this slice: entry 0 is the nearest cluster when the
    // tile has one, then positions p0 .. p1 - 1 (-1: skip)
    const int lead = first >= 0 ? 1 : 0;
    const int nent = lead + max(0, p1 - p0);
    auto cluster_at = [&](int e) -> int {
      if (e < lead) return first;
      const int pos = p0 + e - lead;
      const int c = from_list ? ldg(list, pos) : pos;
      return (!from_list && c == first) ? -1 : c;
    };

    LaneBest L{__builtin_inff(), __builtin_inff(), __builtin_inff(), __builtin_inff(), -1, -1};
    int nproc = 0;  // chunks run through the filter
    // Up to 64 entries at a time: lane j fetches entry j's cluster id, centre
    // and box; the loop reads them across lanes. The first batch's loads are
    // issued together with the source point's (coordinates, previous closest
    // target), so that the slice starts after two round trips.
    auto batch = [&](int gb, int& myc, float4& mcc, float4& mlo, float4& mhi) {
      const int e = gb + lane;
      myc = e < nent ? cluster_at(e) : -1;
      mcc = mlo = mhi = make_float4(0.f, 0.f, 0.f, 0.f);
      if (myc >= 0) {
        mcc = load_global(D.ccen, myc);
        if (lane_test) {
          mlo = load_global(D.clo, myc);
          mhi = load_global(D.chi, myc);
        }
      }
    };
    float spx = 0.f, spy = 0.f, spz = 0.f;
    int prev = -1;
    if (valid) {
      spx = ldg(D.px, si);
      spy = ldg(D.py, si);
      spz = ldg(D.pz, si);
      if (flags & TI_WARM) prev = ldg(D.nnidx, si);
    }
    int myc;
    float4 mcc, mlo, mhi;
    batch(0, myc, mcc, mlo, mhi);
    float ptx, pty, ptz, W;
    lane_point_from(D, S.Teval, valid, spx, spy, spz, prev, ptx, pty, ptz, W);
    // The next cluster's targets are loaded into registers while the current
    // one, staged in LDS, is filtered.
    // every lane's warm bound: a cluster beyond it for every lane is beyond
    // winner_threshold(min(H, W)) too, so the test at filter time would skip
    // it; testing the batch's boxes first keeps such clusters out of the
    // load pipeline (their 2 KB would otherwise be fetched and waited for)
    const float thr_w = winner_threshold(W) * (1.0f + 0x1.0p-19f);
    const unsigned long long vmask = __builtin_amdgcn_ballot_w64(valid);
    for (int gb = 0; gb < nent; gb += 64) {
      if (gb > 0) batch(gb, myc, mcc, mlo, mhi);
      const int gn = min(64, nent - gb);
      unsigned long long live = __ballot(lane < gn && myc >= 0);
      if (lane_test && (flags & TI_WARM)) {
        unsigned long long need = 0ull;
        for (unsigned long long m = live; m; m &= m - 1ull) {
          const int jj = __builtin_ctzll(m);
          if (gb + jj < lead) {  // the nearest cluster is never box-tested
            need |= 1ull << jj;
            continue;
          }
          const float4 blo = make_float4(lane_f(mlo.x, jj), lane_f(mlo.y, jj), lane_f(mlo.z, jj), 0.f);
          const float4 bhi = make_float4(lane_f(mhi.x, jj), lane_f(mhi.y, jj), lane_f(mhi.z, jj), 0.f);
          if (wave_any_of(box_lb2_fma(ptx, pty, ptz, blo, bhi) <= thr_w, vmask)) need |= 1ull << jj;
        }
        live = need;
      }
      if (live == 0ull) continue;
      int j = __builtin_ctzll(live);
      int c = __builtin_amdgcn_readlane(myc, j);
      constexpr int kRows = kCluster / 64;
      constexpr int kBoxes = 2 * kChunksPerCluster;
      float4 r[kRows], rb = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int t = 0; t < kRows; ++t) r[t] = load_global(D.qloc, (size_t)c * kCluster + 64 * t + lane);
      if (lane < kBoxes) rb = load_global(D.kbox, (size_t)c * kBoxes + lane);
      for (unsigned long long rest = live & (live - 1ull);; rest &= rest - 1ull) {
        // the block is one wavefront: its LDS accesses complete in order, so
        // a wavefront fence orders the staging against the filter's reads (a
        // block barrier would also wait for the loads still in flight)
        wave_lds_sync();
#pragma unroll
        for (int t = 0; t < kRows; ++t) s_tgt[64 * t + lane] = r[t];
        if (lane < kBoxes) s_box[lane] = rb;
        wave_lds_sync();
        const int jn = rest ? __builtin_ctzll(rest) : -1;
        const int cn = rest ? __builtin_amdgcn_readlane(myc, jn) : -1;
        if (cn >= 0) {
#pragma unroll
          for (int t = 0; t < kRows; ++t) r[t] = load_global(D.qloc, (size_t)cn * kCluster + 64 * t + lane);
          if (lane < kBoxes) rb = load_global(D.kbox, (size_t)cn * kBoxes + lane);
        }
        bool run = true;
        if (lane_test && gb + j >= lead) {
          // every target of the cluster is at exact squared distance >= lb2
          const float4 blo = make_float4(lane_f(mlo.x, j), lane_f(mlo.y, j), lane_f(mlo.z, j), 0.f);
          const float4 bhi = make_float4(lane_f(mhi.x, j), lane_f(mhi.y, j), lane_f(mhi.z, j), 0.f);
          run = wave_any_of(box_lb2_fma(ptx, pty, ptz, blo, bhi) <=
                                winner_threshold(fminf(L.H, W)) * (1.0f + 0x1.0p-19f),
                            vmask);
        }
        if (run) {
          const float plx = ptx - lane_f(mcc.x, j), ply = pty - lane_f(mcc.y, j),
                      plz = ptz - lane_f(mcc.z, j);
          if (lane_test)
            nproc += filter_cluster<true>(s_tgt, s_box, c, plx, ply, plz, lane_f(mcc.w, j), ptx,
                                          pty, ptz, vmask, W, L);
          else
            nproc += filter_cluster<false>(s_tgt, s_box, c, plx, ply, plz, lane_f(mcc.w, j), ptx,
                                           pty, ptz, vmask, W, L);
        }
        if (cn < 0) break;
        j = jn;
        c = cn;
      }
    }
    const long long t_filter = D.item_stats ? (long long)__builtin_readcyclecounter() : 0ll;

    // Resolution. A slice matters for a lane only if one of its chunks can
    // hold the lane's winner (certified lower bound within the warm bound).
    // Then the chunks that can hold it (lower bound within the threshold of
    // H) are rescanned with the exact definition: chunk A, and B too when it
    // qualifies; when a third chunk qualifies (near-ties, duplicates) the
    // wavefront re-runs the slice's clusters through LDS for those lanes.
    const float thr_h = winner_threshold(L.H);
    const bool has = valid && L.A >= 0 && fminf(L.loA, L.S) <= winner_threshold(W);
    const bool two = has && L.S <= thr_h;
    const bool amb = two && L.S2 <= thr_h;
    unsigned long long key = ~0ull;
    int nexact = 0;
    if (has && !amb) {
      key = exact_scan<true>(D.qorg, L.A * kChunk, kChunk, ptx, pty, ptz, key);
      nexact = kChunk;
      if (two) {
        key = exact_scan<true>(D.qorg, L.B * kChunk, kChunk, ptx, pty, ptz, key);
        nexact += kChunk;
      }
    }
    if (__any(amb)) {
      const float thr = winner_threshold(fminf(L.H, W));
      for (int e = 0; e < nent; ++e) {
        const int c = __builtin_amdgcn_readfirstlane(cluster_at(e));
        if (c < 0) continue;
        const float lb2 = box_lb2(ptx, pty, ptz, load_global(D.clo, c), load_global(D.chi, c));
        const bool need = amb && lb2 * (1.0f - 0x1.0p-20f) <= thr;
        if (!__any(need)) continue;
        __syncthreads();
        for (int t = 0; t < kCluster / 64; ++t)
          s_tgt[64 * t + lane] = load_global(D.qorg, (size_t)c * kCluster + 64 * t + lane);
        __syncthreads();
        if (need) {
          key = exact_scan<false>(s_tgt, 0, kCluster, ptx, pty, ptz, key);
          nexact += kCluster;
        }
      }
    }
    if (has) atomicMin(&D.keys[si], key);
    {
      int nv = valid ? 1 : 0;
      int ne = nexact;
      for (int o = 32; o > 0; o >>= 1) {
        nv += __shfl_xor(nv, o, 64);
        ne += __shfl_xor(ne, o, 64);
      }
      if (lane == 0 && D.stats) {
        // one statistics line per die keeps these atomics off a single address
        unsigned long long* st = D.stats + (blockIdx.x % kQueues) * kStatStride;
        atomicAdd(&st[0], (unsigned long long)nproc * kChunk * (unsigned long long)nv);
        atomicAdd(&st[1], (unsigned long long)ne);
      }
      if (lane == 0 && D.item_stats && local < D.ntile * kMaxSlices) {
        int* row = D.item_stats + 8 * (size_t)local;
        row[0] = (int)((long long)__builtin_readcyclecounter() - t_begin);
        row[1] = nproc;
        row[2] = p1 - p0;
        row[3] = flags | (__any(amb) ? 64 : 0);
        row[4] = p0;
        row[5] = p1;
        row[6] = (int)(t_filter - t_begin);
        row[7] = S.phases;
      }
    }
    __syncthreads();
  }
  if (!wl->single) multi_brute_items(descs, states, wl, s_tgt);
}

// ------------------------------------------------------------------ exhaustive kernel
// Exhaustive method: every target for every source, without a cull pass. The
// wavefront holds two tiles (two sources per lane), so every target read from
// LDS serves two pairs, which halves the LDS traffic per pair. Items are
// (pair of tiles, cluster range), shared out statically (they cost the same):
// in the one-slot engine on a fixed grid of about the slot's brute_items, in
// the multi-slot engine brute_items() per pair (about the slot's
// brute_clusters clusters per item).

// Folds one chunk into a lane's state (the bookkeeping of filter_chunk): m is
// the chunk's minimum of h - pl . ql, v = 2 m + |pl|^2 with bounds lo, hi.
__device__ __forceinline__ void lane_best_update(LaneBest& L, float m, float pp, float delta,
                                                 int id) {
  const float v = __builtin_fmaf(2.0f, m, pp);
  // an all-padding chunk has v = +inf: keep lo = hi = +inf (no inf - inf)
  const float e = fminf(0x1.0p-22f * fabsf(v) + delta, 1e38f);
  const float lo = v - e, hi = v + e;
  const bool better = hi < L.H;
  const float olo = better ? L.loA : lo;
  const int oid = better ? L.A : id;
  const bool nb = olo < L.S;
  L.S2 = fminf(L.S2, nb ? L.S : olo);
  L.B = nb ? oid : L.B;
  L.S = nb ? olo : L.S;
  L.loA = better ? lo : L.loA;
  L.A = better ? id : L.A;
  L.H = fminf(L.H, hi);
}

// One cluster staged in LDS against two sources per lane. The bookkeeping runs
// per group of kBruteGroup targets (the rescan of a winning group covers all
// of it); the targets are read in runs of eight, so that at most eight reads
// are in flight, and each run is folded into the group's minimum with
// three-way minima (32 for the 64 values of a source, the fewest that reduce
// 64 values with them).
constexpr int kBruteGroup = 64;
constexpr int kGroupsPerCluster = kCluster / kBruteGroup;
__device__ __forceinline__ void filter_cluster_pair(const float4* __restrict__ tg, int c,
                                                    const float (&pa)[3], const float (&pb)[3],
                                                    float rho_c, LaneBest& La, LaneBest& Lb) {
  const float ppa = __builtin_fmaf(pa[2], pa[2], __builtin_fmaf(pa[1], pa[1], pa[0] * pa[0]));
  const float ppb = __builtin_fmaf(pb[2], pb[2], __builtin_fmaf(pb[1], pb[1], pb[0] * pb[0]));
  // the hardware square root (within a few units in the last place) suffices:
  // the bound below carries a 1e-4 relative margin
  const float ta = __builtin_amdgcn_sqrtf(ppa) + rho_c, tb = __builtin_amdgcn_sqrtf(ppb) + rho_c;
  const float da = 0x1.0p-22f * 7.0f * 1.0001f * ta * ta;
  const float db = 0x1.0p-22f * 7.0f * 1.0001f * tb * tb;
#pragma unroll 1
  for (int ch = 0; ch < kGroupsPerCluster; ++ch) {
    const float4* qc = tg + ch * kBruteGroup;
    constexpr int kRuns = kBruteGroup / 8;
    float ma = 0.0f, mb = 0.0f;
#pragma unroll
    for (int h = 0; h < kRuns; ++h) {
      float a[8], b[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const float4 q = qc[h * 8 + j];
        a[j] = __builtin_fmaf(-pa[0], q.x, __builtin_fmaf(-pa[1], q.y, __builtin_fmaf(-pa[2], q.z, q.w)));
        b[j] = __builtin_fmaf(-pb[0], q.x, __builtin_fmaf(-pb[1], q.y, __builtin_fmaf(-pb[2], q.z, q.w)));
      }
      if (h == 0) {
        ma = fminf(fminf(fminf(fminf(a[0], a[1]), a[2]), fminf(fminf(a[3], a[4]), a[5])), fminf(a[6], a[7]));
        mb = fminf(fminf(fminf(fminf(b[0], b[1]), b[2]), fminf(fminf(b[3], b[4]), b[5])), fminf(b[6], b[7]));
      } else {
#pragma unroll
        for (int j = 0; j < 8; j += 2) {
          ma = fminf(fminf(ma, a[j]), a[j + 1]);
          mb = fminf(fminf(mb, b[j]), b[j + 1]);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    const int id = c * kGroupsPerCluster + ch;
    lane_best_update(La, ma, ppa, da, id);
    lane_best_update(Lb, mb, ppb, db, id);
  }
}

// One exhaustive item: the tiles 2 pi and 2 pi + 1 of a pair (two sources per
// lane) against clusters [c0, c1).
__device__ __forceinline__ void brute_item(const SlotDesc& D, const SlotState& S, int pi, int c0,
                                           int c1, float4* s_tgt) {
  const int lane = threadIdx.x;
  constexpr int kRows = kCluster / 64;
  const int sa = 2 * pi * kTile + lane, sb = sa + kTile;
  const bool va = sa < D.M, vb = sb < D.M;
  const int ca = va ? sa : D.M - 1, cb = vb ? sb : D.M - 1;
  const float xa = ldg(D.px, ca), ya = ldg(D.py, ca), za = ldg(D.pz, ca);
  const float xb = ldg(D.px, cb), yb = ldg(D.py, cb), zb = ldg(D.pz, cb);
  float4 r[kRows];
#pragma unroll
  for (int t = 0; t < kRows; ++t) r[t] = load_global(D.qloc, (size_t)c0 * kCluster + 64 * t + lane);
  float4 cc = load_global(D.ccen, c0);
  float ax, ay, az, Wa, bx, by, bz, Wb;
  lane_point_from(D, S.Teval, va, xa, ya, za, -1, ax, ay, az, Wa);
  lane_point_from(D, S.Teval, vb, xb, yb, zb, -1, bx, by, bz, Wb);
  LaneBest La{__builtin_inff(), __builtin_inff(), __builtin_inff(), __builtin_inff(), -1, -1};
  LaneBest Lb = La;
  for (int c = c0; c < c1; ++c) {
    wave_lds_sync();
#pragma unroll
    for (int t = 0; t < kRows; ++t) s_tgt[64 * t + lane] = r[t];
    wave_lds_sync();
    const float4 cur = cc;
    if (c + 1 < c1) {
#pragma unroll
      for (int t = 0; t < kRows; ++t) r[t] = load_global(D.qloc, (size_t)(c + 1) * kCluster + 64 * t + lane);
      cc = load_global(D.ccen, c + 1);
    }
    const float pa[3] = {ax - cur.x, ay - cur.y, az - cur.z};
    const float pb[3] = {bx - cur.x, by - cur.y, bz - cur.z};
    filter_cluster_pair(s_tgt, c, pa, pb, cur.w, La, Lb);
  }
  // resolution as in the slice kernel, for both sources of the lane
  int nexact = 0;
  auto resolve = [&](const LaneBest& Lx, float x, float y, float z, bool vx,
                     unsigned long long& keyx, bool& ambx) -> bool {
    const float thr_h = winner_threshold(Lx.H);
    const bool has = vx && Lx.A >= 0;
    const bool two = has && Lx.S <= thr_h;
    ambx = two && Lx.S2 <= thr_h;
    keyx = ~0ull;
    if (has && !ambx) {
      keyx = exact_scan<true>(D.qorg, Lx.A * kBruteGroup, kBruteGroup, x, y, z, keyx);
      nexact += kBruteGroup;
      if (two) {
        keyx = exact_scan<true>(D.qorg, Lx.B * kBruteGroup, kBruteGroup, x, y, z, keyx);
        nexact += kBruteGroup;
      }
    }
    return has;
  };
  unsigned long long ka, kb;
  bool amba, ambb;
  const bool hasa = resolve(La, ax, ay, az, va, ka, amba);
  const bool hasb = resolve(Lb, bx, by, bz, vb, kb, ambb);
  if (__any(amba || ambb)) {
    // near-ties: the item's clusters again, exactly, for those lanes
    const float tha = winner_threshold(La.H), thb = winner_threshold(Lb.H);
    for (int c = c0; c < c1; ++c) {
      const float4 blo = load_global(D.clo, c), bhi = load_global(D.chi, c);
      const bool na = amba && box_lb2(ax, ay, az, blo, bhi) * (1.0f - 0x1.0p-20f) <= tha;
      const bool nb = ambb && box_lb2(bx, by, bz, blo, bhi) * (1.0f - 0x1.0p-20f) <= thb;
      if (!__any(na || nb)) continue;
      wave_lds_sync();
      for (int t = 0; t < kRows; ++t)
        s_tgt[64 * t + lane] = load_global(D.qorg, (size_t)c * kCluster + 64 * t + lane);
      wave_lds_sync();
      if (na) {
        ka = exact_scan<false>(s_tgt, 0, kCluster, ax, ay, az, ka);
        nexact += kCluster;
      }
      if (nb) {
        kb = exact_scan<false>(s_tgt, 0, kCluster, bx, by, bz, kb);
        nexact += kCluster;
      }
    }
  }
  if (hasa) atomicMin(&D.keys[sa], ka);
  if (hasb) atomicMin(&D.keys[sb], kb);
  int nv = (va ? 1 : 0) + (vb ? 1 : 0);
  int ne = nexact;
  for (int o = 32; o > 0; o >>= 1) {
    nv += __shfl_xor(nv, o, 64);
    ne += __shfl_xor(ne, o, 64);
  }
  if (lane == 0 && D.stats) {
    unsigned long long* st = D.stats + (blockIdx.x % kQueues) * kStatStride;
    atomicAdd(&st[0], (unsigned long long)(c1 - c0) * kCluster * (unsigned long long)nv);
    atomicAdd(&st[1], (unsigned long long)ne);
  }
}

__global__ __launch_bounds__(64) void nn_brute_kernel(const SlotDesc* __restrict__ descs,
                                                      const SlotState* __restrict__ states) {
  __shared__ float4 s_tgt[kCluster];
  const SlotDesc& D = descs[0];
  const SlotState& S = states[0];
  if (S.status != ST_RUNNING || S.reuse) return;
  const int ncl = D.ncl;
  const int npair = (D.ntile + 1) / 2;
  const int split = min(ncl, max(1, (D.brute_items + npair - 1) / npair));
  const int len = (ncl + split - 1) / split;
  const int nitems = npair * split;
  for (int g = blockIdx.x; g < nitems; g += gridDim.x) {
    const int pi = g / split, k = g - (g / split) * split;
    const int c0 = k * len, c1 = min(ncl, c0 + len);
    if (c0 >= c1) continue;
    brute_item(D, S, pi, c0, c1, s_tgt);
  }
}

// Multi-slot engine, exhaustive method: the items of every searching pair
// (brute_items per pair, prefixed by the planner), run by the slice kernel's
// wavefronts once the slices are used up: the uniform items fill the uneven
// tail of the slices. Sub-queue x (the workgroups on die x) serves the items
// x, x + kQueues, ...
__device__ void multi_brute_items(const SlotDesc* __restrict__ descs,
                                                  const SlotState* __restrict__ states,
                                                  WorkList* __restrict__ wl, float4* s_tgt) {
  // loop bounds in scalar registers: the exit test is uniform
  const int total = __builtin_amdgcn_readfirstlane(wl->b_total);
  const int na = __builtin_amdgcn_readfirstlane(wl->n_active);
  const int x = (int)(blockIdx.x % kQueues);
  for (;;) {
    int k = 0;
    if (threadIdx.x == 0) k = atomicAdd(&wl->q_b[x * kQueueStride], 1);
    const int g = __builtin_amdgcn_readfirstlane(__shfl(k, 0, 64)) * kQueues + x;
    if (g >= total) break;
    const int a = wave_find_slot(wl->b_base, na, g);
    const int slot = __builtin_amdgcn_readfirstlane(wl->slot[a]);
    const SlotDesc& D = descs[slot];
    const SlotState& S = states[slot];
    const int item = g - __builtin_amdgcn_readfirstlane(wl->b_base[a]);
    const int split = brute_split(D.ncl, D.brute_clusters);
    const int len = (D.ncl + split - 1) / split;
    const int pi = item / split, kk = item - pi * split;
    const int c0 = kk * len, c1 = min(D.ncl, c0 + len);
    if (c0 < c1) brute_item(D, S, pi, c0, c1, s_tgt);
    // The wavefront reconverges here before lane 0 fetches the next item
    // (as in the slice loop). Without this point the compiled loop let lane 0
    // leave after an item while the other lanes went round again on the
    // stale item number, without end.
    __syncthreads();
  }
}

void launch_brute(const SlotDesc* descs, const SlotState* states, int grid, hipStream_t st) {
  hipLaunchKernelGGL(nn_brute_kernel, dim3(grid), dim3(64), 0, st, descs, states);
}

void launch_nn(const SlotDesc* descs, const SlotState* states, WorkList* wl, int grid,
               bool single, hipStream_t st) {
  // every sub-queue needs workgroups of its own (blockIdx mod kQueues, and
  // mod kSliceQueues for the slice kernel)
  grid = std::max(grid, std::max(kQueues * kCullWaves, kSliceQueues));
  // the cull waits on memory most of the time: 7/4 of the search's wavefronts
  // (seven per SIMD at the default grid, which its registers allow)
  hipLaunchKernelGGL(nn_cull_kernel, dim3(grid * 7 / (4 * kCullWaves)), dim3(64 * kCullWaves), 0, st, descs,
                     states, wl);
  if (!single) hipLaunchKernelGGL(slice_plan_kernel, dim3(1), dim3(1024), 0, st, descs, states, wl);
  hipLaunchKernelGGL(nn_slice_kernel, dim3(grid), dim3(64), 0, st, descs, states, wl);
}

}  // namespace icp
