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
//  * Targets are kept in clusters of 128 Morton-ordered points, stored relative
//    to the cluster centre cc together with h = |q - cc|^2 / 2. For a source,
//    the filter value 2 (h - (p' - cc) . (q - cc)) + |p' - cc|^2 equals the
//    squared distance up to a rounding error that is bounded per cluster; it
//    costs 3 FMA per pair (v_fma_f32) and one v_min3_f32 per two pairs.
//  * Only the minimum filter value of each 32-target chunk is kept (with the
//    runner-up chunk value via v_med3_f32). At the end the winning chunk is
//    rescanned with the exact FP32 definition. If another chunk comes within
//    the error bound of the winner, every candidate is rescanned exactly.
//  * Cluster culling (method NN_CLUSTER): a bounding sphere of the 64-source
//    tile, transformed per pass, against super-cluster and cluster AABBs gives
//    a candidate list; per lane, a cluster whose AABB distance exceeds the
//    current best by more than the error bound is skipped wave-uniformly.
//  * Optionally the candidate list of a tile is split over several work
//    items whose keys merge with a 64-bit atomic min (order independent).
#include "icp_internal.h"

namespace icp {

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ void xform_f32(const double* T, float x, float y, float z,
                                          float& ox, float& oy, float& oz) {
  const double X = x, Y = y, Z = z;
  ox = (float)__builtin_fma(T[2], Z, __builtin_fma(T[1], Y, __builtin_fma(T[0], X, T[3])));
  oy = (float)__builtin_fma(T[6], Z, __builtin_fma(T[5], Y, __builtin_fma(T[4], X, T[7])));
  oz = (float)__builtin_fma(T[10], Z, __builtin_fma(T[9], Y, __builtin_fma(T[8], X, T[11])));
}

// Bound on |filter value - exact squared distance| for a target whose exact
// squared distance is at most x, with rho the cluster radius: a 4x margin
// over u (7 (sqrt(x) + 2 rho)^2 + x), u = 2^-24, which covers the rounding of
// the centred coordinates, of h, of the three FMAs and of the final FMA.
__device__ __forceinline__ float err_bound(float x, float rho) {
  const float s = sqrtf(x) + 2.0f * rho;
  return 0x1.0p-22f * (7.0f * s * s + x) * 1.001f;
}

// Threshold on the filter value above which a target can neither beat nor tie
// the exact winner (gamma = 1e-6 bounds the relative error of the exact FP32
// form, 5u).
__device__ __forceinline__ float ambiguity_threshold(float best, float rho) {
  const float X = fmaxf(best, 0.0f);
  const float Xp = X + err_bound(X, rho);
  const float slack = 2.0f * err_bound(Xp * 1.00001f, rho) + 2.2e-6f * Xp;
  return X + slack * 1.01f + 1e-37f;
}

__device__ __forceinline__ unsigned long long make_key(float d2, int idx) {
  return ((unsigned long long)__float_as_uint(d2) << 32) | (unsigned)idx;
}

// Exact FP32 scan of n targets of the original-coordinate array.
__device__ __forceinline__ unsigned long long exact_scan(const float4* __restrict__ qorg, int base,
                                                         int n, float px, float py, float pz,
                                                         unsigned long long key) {
  for (int j = 0; j < n; ++j) {
    const float4 q = qorg[base + j];
    const int id = __float_as_int(q.w);
    if (id < 0) continue;
    const float dx = px - q.x, dy = py - q.y, dz = pz - q.z;
    const float d = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
    const unsigned long long k = make_key(d, id);
    key = k < key ? k : key;
  }
  return key;
}

__device__ __forceinline__ float box_lb2(float px, float py, float pz, float4 lo, float4 hi) {
  const float dx = fmaxf(fmaxf(lo.x - px, px - hi.x), 0.0f);
  const float dy = fmaxf(fmaxf(lo.y - py, py - hi.y), 0.0f);
  const float dz = fmaxf(fmaxf(lo.z - pz, pz - hi.z), 0.0f);
  return dx * dx + dy * dy + dz * dz;
}

__device__ __forceinline__ float box_ub2(float px, float py, float pz, float4 lo, float4 hi) {
  const float dx = fmaxf(fabsf(px - lo.x), fabsf(px - hi.x));
  const float dy = fmaxf(fabsf(py - lo.y), fabsf(py - hi.y));
  const float dz = fmaxf(fabsf(pz - lo.z), fabsf(pz - hi.z));
  return dx * dx + dy * dy + dz * dz;
}

struct LaneBest {
  float best, second;
  int bc;  // global chunk id (cluster * 4 + chunk)
};

// Process one cluster with the filter (all 128 targets, 4 chunks).
__device__ __forceinline__ void filter_cluster(const float4* __restrict__ lds, int c, float plx,
                                               float ply, float plz, LaneBest& L) {
  const float npx = -plx, npy = -ply, npz = -plz;
  const float pp = __builtin_fmaf(plz, plz, __builtin_fmaf(ply, ply, plx * plx));
#pragma unroll
  for (int ch = 0; ch < kChunksPerCluster; ++ch) {
    float m0 = __builtin_inff(), m1 = __builtin_inff();
#pragma unroll
    for (int j = 0; j < kChunk; j += 4) {
      const float4 a = lds[ch * kChunk + j];
      const float4 b = lds[ch * kChunk + j + 1];
      const float4 c2 = lds[ch * kChunk + j + 2];
      const float4 d = lds[ch * kChunk + j + 3];
      const float sa = __builtin_fmaf(npx, a.x, __builtin_fmaf(npy, a.y, __builtin_fmaf(npz, a.z, a.w)));
      const float sb = __builtin_fmaf(npx, b.x, __builtin_fmaf(npy, b.y, __builtin_fmaf(npz, b.z, b.w)));
      const float sc = __builtin_fmaf(npx, c2.x, __builtin_fmaf(npy, c2.y, __builtin_fmaf(npz, c2.z, c2.w)));
      const float sd = __builtin_fmaf(npx, d.x, __builtin_fmaf(npy, d.y, __builtin_fmaf(npz, d.z, d.w)));
      m0 = fminf(m0, fminf(sa, sb));
      m1 = fminf(m1, fminf(sc, sd));
    }
    const float me = __builtin_fmaf(2.0f, fminf(m0, m1), pp);
    L.second = __builtin_amdgcn_fmed3f(L.second, me, L.best);
    const bool lt = me < L.best;
    L.bc = lt ? (c * kChunksPerCluster + ch) : L.bc;
    L.best = fminf(L.best, me);
  }
}

__global__ __launch_bounds__(64) void nn_kernel(const SlotDesc* __restrict__ descs,
                                                const SlotState* __restrict__ states,
                                                WorkList* __restrict__ wl) {
  __shared__ float4 s_tgt[kCluster];
  __shared__ int s_cand[kCandCap];
  __shared__ int s_sup[kSupCap];

  const int lane = threadIdx.x;
  for (;;) {
    int g = 0;
    if (lane == 0) g = atomicAdd(&wl->nn_counter, 1);
    g = __shfl(g, 0, 64);
    if (g >= wl->nn_total) break;
    // decode (slot, tile, split) by binary search over the active prefix
    int lo = 0, hi = wl->n_active - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (wl->nn_base[mid] <= g) lo = mid; else hi = mid - 1;
    }
    const int slot = wl->slot[lo];
    const SlotDesc& D = descs[slot];
    const SlotState& S = states[slot];
    const int local = g - wl->nn_base[lo];
    const int split = D.split;
    const int tile = local / split;
    const int sp = local - tile * split;
    const int si = tile * kTile + lane;
    const bool valid = si < D.M;
    const double* T = S.Teval;

    float ptx = 0.f, pty = 0.f, ptz = 0.f;
    if (valid) xform_f32(T, D.px[si], D.py[si], D.pz[si], ptx, pty, ptz);

    LaneBest L{__builtin_inff(), __builtin_inff(), -1};
    const float rho = D.rho_max;

    // ----------------------------------------------------------------- candidates
    int ncand = 0;       // list length (cluster mode)
    bool use_list = false;
    int first = -1;      // nearest cluster (processed first by every split)
    if (D.method == NN_CLUSTER) {
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
      // level 1: upper bound from super-cluster boxes
      float U = __builtin_inff();
      for (int s = lane; s < D.nsup; s += 64) {
        const float ub = sqrtf(box_ub2(cx, cy, cz, D.slo[s], D.shi[s])) * 1.000001f + r;
        U = fminf(U, ub);
      }
      U = wave_min(U);
      // candidate super-clusters
      int nsc = 0;
      bool overflow = false;
      for (int base = 0; base < D.nsup; base += 64) {
        const int s = base + lane;
        bool c = false;
        if (s < D.nsup) {
          const float lb = sqrtf(box_lb2(cx, cy, cz, D.slo[s], D.shi[s])) * 0.999999f - r;
          c = lb <= U * 1.00001f;
        }
        const unsigned long long bal = __ballot(c);
        const int pos = nsc + __popcll(bal & ((1ull << lane) - 1ull));
        if (c && pos < kSupCap) s_sup[pos] = s;
        nsc += __popcll(bal);
      }
      if (nsc > kSupCap) overflow = true;
      __syncthreads();
      // expand candidate super-clusters to clusters
      float bestub = __builtin_inff();
      int bestc = 0x7fffffff;
      const int nflat = overflow ? 0 : nsc * kSuper;
      for (int base = 0; base < nflat; base += 64) {
        const int f = base + lane;
        bool c = false;
        int cid = 0;
        if (f < nflat) {
          cid = s_sup[f / kSuper] * kSuper + (f % kSuper);
          if (cid < D.ncl) {
            const float4 blo = D.clo[cid], bhi = D.chi[cid];
            const float lb = sqrtf(box_lb2(cx, cy, cz, blo, bhi)) * 0.999999f - r;
            const float ub = sqrtf(box_ub2(cx, cy, cz, blo, bhi)) * 1.000001f + r;
            if (ub < bestub || (ub == bestub && cid < bestc)) { bestub = ub; bestc = cid; }
            c = lb <= U * 1.00001f;
          }
        }
        const unsigned long long bal = __ballot(c);
        const int pos = ncand + __popcll(bal & ((1ull << lane) - 1ull));
        if (c && pos < kCandCap) s_cand[pos] = cid;
        ncand += __popcll(bal);
      }
      // tightest upper bound and the cluster achieving it
      float Uc = wave_min(bestub);
      int cand_first = (bestub == Uc) ? bestc : 0x7fffffff;
      // lowest cluster id among lanes achieving the minimum
      for (int o = 32; o > 0; o >>= 1) cand_first = min(cand_first, __shfl_xor(cand_first, o, 64));
      if (overflow || ncand > kCandCap || nflat == 0) {
        use_list = false;
        first = 0;
      } else {
        use_list = true;
        first = cand_first;
        U = fminf(U, Uc);
        // compact: keep clusters whose lower bound is within the final bound
        __syncthreads();
        int n2 = 0;
        for (int base = 0; base < ncand; base += 64) {
          const int f = base + lane;
          int cid = 0;
          bool keep = false;
          if (f < ncand) {
            cid = s_cand[f];
            const float lb = sqrtf(box_lb2(cx, cy, cz, D.clo[cid], D.chi[cid])) * 0.999999f - r;
            keep = lb <= U * 1.00001f && cid != first;
          }
          const unsigned long long bal = __ballot(keep);
          const int pos = n2 + __popcll(bal & ((1ull << lane) - 1ull));
          __syncthreads();
          if (keep) s_cand[pos] = cid;
          n2 += __popcll(bal);
          __syncthreads();
        }
        ncand = n2;
      }
      __syncthreads();
    }

    // ----------------------------------------------------------------- filter pass
    const float4* __restrict__ qloc = D.qloc;
    const bool culled = D.method == NN_CLUSTER;
    // iteration space: position -1 is the nearest cluster (cluster mode), then
    // this split's share of the list (or of all clusters)
    const int count = culled ? (use_list ? ncand : D.ncl) : D.ncl;
    int it = culled ? -1 : sp;
    const int step = culled ? 1 : split;
    // in cluster mode the split takes list positions sp, sp + split, ...
    for (;;) {
      int c;
      if (culled) {
        if (it < 0) {
          c = first;
        } else {
          const int pos = sp + it * split;
          if (pos >= count) break;
          c = use_list ? s_cand[pos] : pos;
          if (!use_list && c == first) { it += step; continue; }
        }
      } else {
        if (it >= count) break;
        c = it;
      }
      const float4 cc = D.ccen[c];
      const float plx = ptx - cc.x, ply = pty - cc.y, plz = ptz - cc.z;
      if (culled && it >= 0) {
        const float lb2 = box_lb2(ptx, pty, ptz, D.clo[c], D.chi[c]);
        const float pl = sqrtf(__builtin_fmaf(plz, plz, __builtin_fmaf(ply, ply, plx * plx))) + cc.w;
        const float lbv = lb2 * (1.0f - 0x1.0p-20f) - 0x1.0p-20f * 8.0f * pl * pl;
        const bool need = valid && lbv <= ambiguity_threshold(L.best, rho);
        if (!__any(need)) { it += step; continue; }
      }
      __syncthreads();
      s_tgt[lane] = qloc[c * kCluster + lane];
      s_tgt[lane + 64] = qloc[c * kCluster + 64 + lane];
      __syncthreads();
      filter_cluster(s_tgt, c, plx, ply, plz, L);
      it += step;
    }

    // ----------------------------------------------------------------- exact resolution
    if (valid && L.bc >= 0) {
      unsigned long long key = ~0ull;
      const bool amb = L.second <= ambiguity_threshold(L.best, rho);
      if (!amb) {
        key = exact_scan(D.qorg, L.bc * kChunk, kChunk, ptx, pty, ptz, key);
      } else {
        // rescan every cluster this work item could have visited
        if (culled) {
          key = exact_scan(D.qorg, first * kCluster, kCluster, ptx, pty, ptz, key);
          for (int i2 = 0;; ++i2) {
            const int pos = sp + i2 * split;
            if (pos >= count) break;
            const int c = use_list ? s_cand[pos] : pos;
            if (!use_list && c == first) continue;
            key = exact_scan(D.qorg, c * kCluster, kCluster, ptx, pty, ptz, key);
          }
        } else {
          for (int c = sp; c < D.ncl; c += split)
            key = exact_scan(D.qorg, c * kCluster, kCluster, ptx, pty, ptz, key);
        }
      }
      if (split == 1) D.keys[si] = key;
      else atomicMin(&D.keys[si], key);
    }
    __syncthreads();
  }
}

void launch_nn(const SlotDesc* descs, const SlotState* states, WorkList* wl, int grid,
               hipStream_t st) {
  hipLaunchKernelGGL(nn_kernel, dim3(grid), dim3(64), 0, st, descs, states, wl);
}

}  // namespace icp
