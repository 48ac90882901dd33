// Per-request setup on the device (once per registration, before the
// iterations): layout conversion, bounding boxes, Hilbert ordering of both point
// sets with a stable LSD radix sort, the cluster index over the target
// (cluster AABBs, centres, radii, centred coordinates) and bounding spheres of
// the 64-source tiles. Also the planner that rebuilds the active work lists
// before every pass.
#include "icp_internal.h"

namespace icp {

// ------------------------------------------------------------------ layout

__global__ void aos_to_soa_kernel(const float* __restrict__ aos, int n, float* __restrict__ x,
                                  float* __restrict__ y, float* __restrict__ z) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    x[i] = aos[3 * (size_t)i];
    y[i] = aos[3 * (size_t)i + 1];
    z[i] = aos[3 * (size_t)i + 2];
  }
}

// Min/max over n points (one block of 1024 threads); writes the box and its
// FP64 centre.
__global__ __launch_bounds__(1024) void bbox_kernel(const float* __restrict__ x,
                                                    const float* __restrict__ y,
                                                    const float* __restrict__ z, int n,
                                                    float* __restrict__ box,
                                                    double* __restrict__ centre) {
  float mn[3] = {__builtin_inff(), __builtin_inff(), __builtin_inff()};
  float mx[3] = {-__builtin_inff(), -__builtin_inff(), -__builtin_inff()};
  // eight strides' loads in flight at once; folded in index order
  for (int i0 = threadIdx.x; i0 < n; i0 += 8 * 1024) {
    float v[8][3];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + 1024 * u;
      v[u][0] = i < n ? x[i] : __builtin_inff();
      v[u][1] = i < n ? y[i] : __builtin_inff();
      v[u][2] = i < n ? z[i] : __builtin_inff();
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (i0 + 1024 * u < n)
        for (int a = 0; a < 3; ++a) { mn[a] = fminf(mn[a], v[u][a]); mx[a] = fmaxf(mx[a], v[u][a]); }
  }
  __shared__ float s[6][16];
  for (int a = 0; a < 3; ++a) {
    for (int o = 32; o > 0; o >>= 1) {
      mn[a] = fminf(mn[a], __shfl_xor(mn[a], o, 64));
      mx[a] = fmaxf(mx[a], __shfl_xor(mx[a], o, 64));
    }
  }
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0)
    for (int a = 0; a < 3; ++a) { s[a][w] = mn[a]; s[3 + a][w] = mx[a]; }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
    for (int a = 0; a < 3; ++a) {
      float lo = s[a][0], hi = s[3 + a][0];
      for (int k = 1; k < nw; ++k) { lo = fminf(lo, s[a][k]); hi = fmaxf(hi, s[3 + a][k]); }
      box[a] = lo;
      box[3 + a] = hi;
      if (centre) centre[a] = 0.5 * ((double)lo + (double)hi);
    }
  }
}

__device__ inline unsigned spread10(unsigned v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000ffu;
  v = (v | (v << 8)) & 0x0300f00fu;
  v = (v | (v << 4)) & 0x030c30c3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

// 30-bit Hilbert key of the cell of the 1024^3 grid over the bounding box; value = index.
__global__ void hilbert_kernel(const float* __restrict__ x, const float* __restrict__ y,
                               const float* __restrict__ z, int n, const float* __restrict__ box,
                               unsigned* __restrict__ keys, unsigned* __restrict__ vals) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float v[3] = {x[i], y[i], z[i]};
  unsigned c[3];
  for (int a = 0; a < 3; ++a) {
    const float ext = box[3 + a] - box[a];
    float f = ext > 0.0f ? (v[a] - box[a]) / ext * 1024.0f : 0.0f;
    int q = (int)f;
    q = q < 0 ? 0 : (q > 1023 ? 1023 : q);
    c[a] = (unsigned)q;
  }
  // Hilbert index of the cell (Skilling's transpose form: undo the excess
  // work, then Gray-encode; the index interleaves the transposed bits), a
  // curve without the long jumps of the Morton order, so that runs of 64 or
  // 128 consecutive points have tighter boxes.
  unsigned X[3] = {c[0], c[1], c[2]};
  for (unsigned Q = 1u << 9; Q > 1u; Q >>= 1) {
    const unsigned P = Q - 1u;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (X[a] & Q) {
        X[0] ^= P;
      } else {
        const unsigned t = (X[0] ^ X[a]) & P;
        X[0] ^= t;
        X[a] ^= t;
      }
    }
  }
  X[1] ^= X[0];
  X[2] ^= X[1];
  unsigned t = 0u;
  for (unsigned Q = 1u << 9; Q > 1u; Q >>= 1)
    if (X[2] & Q) t ^= Q - 1u;
  X[0] ^= t;
  X[1] ^= t;
  X[2] ^= t;
  keys[i] = (spread10(X[0]) << 2) | (spread10(X[1]) << 1) | spread10(X[2]);
  vals[i] = (unsigned)i;
}

// ------------------------------------------------------------------ radix sort
// Stable LSD sort of (32-bit key, 32-bit value) pairs, 8 bits per pass. Each
// block (one wavefront) owns a contiguous chunk of kSortChunk elements, loads
// all of it at once (kSortPer elements per lane) and ranks it in order, 64 at
// a time, so equal keys keep their input order. Only LDS is shared inside a
// block, so a wavefront fence orders it (no wait on the loads or stores).

constexpr int kSortPer = 16;
constexpr int kSortChunk = 64 * kSortPer;

__global__ __launch_bounds__(64) void rs_hist_kernel(const unsigned* __restrict__ keys, int n,
                                                     int shift, unsigned* __restrict__ hist) {
  __shared__ unsigned h[256];
  const int lane = threadIdx.x;
  const int base = blockIdx.x * kSortChunk + lane;
  unsigned d[kSortPer];
#pragma unroll
  for (int s = 0; s < kSortPer; ++s) {
    const int e = base + 64 * s;
    d[s] = e < n ? (ldg(keys, e) >> shift) & 255u : 256u;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) h[lane + 64 * i] = 0u;
  wave_lds_sync();
#pragma unroll
  for (int s = 0; s < kSortPer; ++s)
    if (d[s] < 256u) atomicAdd(&h[d[s]], 1u);
  wave_lds_sync();
#pragma unroll
  for (int i = 0; i < 4; ++i) hist[(size_t)blockIdx.x * 256 + lane + 64 * i] = h[lane + 64 * i];
}

// Exclusive scan of the block-major histogram hist[block * 256 + digit]: the
// offset of (block, digit) is the count of all smaller digits plus that of
// the digit in earlier blocks. One block of 1024 threads: thread (q, d) owns
// digit d in the q-th quarter of the blocks (reads of 256 consecutive words).
__global__ __launch_bounds__(1024) void rs_scan_kernel(unsigned* __restrict__ hist, int nb) {
  __shared__ unsigned s_part[4][256];
  __shared__ unsigned s_inc[256];
  const int d = threadIdx.x & 255, q = threadIdx.x >> 8;
  const int per = (nb + 3) / 4;
  const int b0 = q * per, b1 = min(nb, b0 + per);
  unsigned sum = 0;
  for (int bb = b0; bb < b1; bb += 8) {
    unsigned v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = bb + j < b1 ? hist[(size_t)(bb + j) * 256 + d] : 0u;
#pragma unroll
    for (int j = 0; j < 8; ++j) sum += v[j];
  }
  s_part[q][d] = sum;
  __syncthreads();
  const unsigned tot = s_part[0][d] + s_part[1][d] + s_part[2][d] + s_part[3][d];
  if (q == 0) s_inc[d] = tot;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    const unsigned v = (q == 0 && d >= o) ? s_inc[d - o] : 0u;
    __syncthreads();
    if (q == 0) s_inc[d] += v;
    __syncthreads();
  }
  unsigned run = s_inc[d] - tot;
  for (int k = 0; k < q; ++k) run += s_part[k][d];
  for (int bb = b0; bb < b1; bb += 8) {
    unsigned v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = bb + j < b1 ? hist[(size_t)(bb + j) * 256 + d] : 0u;
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (bb + j < b1) {
        hist[(size_t)(bb + j) * 256 + d] = run;
        run += v[j];
      }
  }
}

__global__ __launch_bounds__(64) void rs_scatter_kernel(const unsigned* __restrict__ kin,
                                                        const unsigned* __restrict__ vin, int n,
                                                        int shift,
                                                        const unsigned* __restrict__ hist,
                                                        unsigned* __restrict__ kout,
                                                        unsigned* __restrict__ vout) {
  __shared__ unsigned cnt[256];
  const int lane = threadIdx.x;
  const int base = blockIdx.x * kSortChunk + lane;
  unsigned kk[kSortPer], vv[kSortPer];
#pragma unroll
  for (int s = 0; s < kSortPer; ++s) {
    const int e = base + 64 * s;
    kk[s] = e < n ? ldg(kin, e) : 0u;
    vv[s] = e < n ? ldg(vin, e) : 0u;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) cnt[lane + 64 * i] = ldg(hist, (size_t)blockIdx.x * 256 + lane + 64 * i);
  wave_lds_sync();
  const unsigned long long lt = (1ull << lane) - 1ull;
#pragma unroll
  for (int s = 0; s < kSortPer; ++s) {
    const bool valid = base + 64 * s < n;
    const unsigned d = (kk[s] >> shift) & 255u;
    unsigned long long m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const unsigned long long bb = __ballot(valid && bit);
      m &= bit ? bb : ~bb;
    }
    const unsigned rank = (unsigned)__popcll(m & lt);
    const unsigned pos = cnt[d] + rank;
    wave_lds_sync();
    if (valid && rank == 0) cnt[d] += (unsigned)__popcll(m);
    wave_lds_sync();
    if (valid) {
      kout[pos] = kk[s];
      vout[pos] = vv[s];
    }
  }
}

// ------------------------------------------------------------------ cluster index

// One wavefront per cluster of kCluster sorted targets.
__global__ __launch_bounds__(64) void build_clusters_kernel(
    const float* __restrict__ x, const float* __restrict__ y, const float* __restrict__ z,
    const unsigned* __restrict__ order, int n, int ncl, float4* __restrict__ qloc,
    float4* __restrict__ qorg, float4* __restrict__ ccen, float4* __restrict__ clo,
    float4* __restrict__ chi, float4* __restrict__ kbox) {
  const int c = blockIdx.x;
  if (c >= ncl) return;
  const int lane = threadIdx.x;
  constexpr int kRows = kCluster / 64;
  static_assert(kCluster % 64 == 0, "a cluster is whole rows of 64 targets");
  float p[kRows][3];
  int id[kRows];
  float mn[3] = {__builtin_inff(), __builtin_inff(), __builtin_inff()};
  float mx[3] = {-__builtin_inff(), -__builtin_inff(), -__builtin_inff()};
  for (int r = 0; r < kRows; ++r) {
    const int pos = c * kCluster + r * 64 + lane;
    id[r] = pos < n ? (int)order[pos] : -1;
    if (id[r] >= 0) {
      p[r][0] = x[id[r]];
      p[r][1] = y[id[r]];
      p[r][2] = z[id[r]];
      for (int a = 0; a < 3; ++a) { mn[a] = fminf(mn[a], p[r][a]); mx[a] = fmaxf(mx[a], p[r][a]); }
    } else {
      p[r][0] = p[r][1] = p[r][2] = 0.0f;
    }
  }
  // chunk boxes: the kChunk consecutive targets of a chunk sit in kChunk
  // consecutive lanes of one row
  static_assert(64 % kChunk == 0 && (kChunk & (kChunk - 1)) == 0, "chunks tile a row");
  for (int r = 0; r < kRows; ++r) {
    float kmn[3], kmx[3];
    for (int a = 0; a < 3; ++a) {
      kmn[a] = id[r] >= 0 ? p[r][a] : __builtin_inff();
      kmx[a] = id[r] >= 0 ? p[r][a] : -__builtin_inff();
      for (int o = 1; o < kChunk; o <<= 1) {
        kmn[a] = fminf(kmn[a], __shfl_xor(kmn[a], o, 64));
        kmx[a] = fmaxf(kmx[a], __shfl_xor(kmx[a], o, 64));
      }
    }
    if ((lane & (kChunk - 1)) == 0) {
      const size_t k = (size_t)c * kChunksPerCluster + (r * 64 + lane) / kChunk;
      kbox[2 * k] = make_float4(kmn[0], kmn[1], kmn[2], 0.0f);
      kbox[2 * k + 1] = make_float4(kmx[0], kmx[1], kmx[2], 0.0f);
    }
  }
  for (int a = 0; a < 3; ++a)
    for (int o = 32; o > 0; o >>= 1) {
      mn[a] = fminf(mn[a], __shfl_xor(mn[a], o, 64));
      mx[a] = fmaxf(mx[a], __shfl_xor(mx[a], o, 64));
    }
  const float cc[3] = {0.5f * (mn[0] + mx[0]), 0.5f * (mn[1] + mx[1]), 0.5f * (mn[2] + mx[2])};
  double rmax = 0.0;
  for (int r = 0; r < kRows; ++r) {
    const int pos = c * kCluster + r * 64 + lane;
    if (id[r] >= 0) {
      const double ex = (double)p[r][0] - cc[0], ey = (double)p[r][1] - cc[1],
                   ez = (double)p[r][2] - cc[2];
      rmax = fmax(rmax, sqrt(ex * ex + ey * ey + ez * ez));
      const float lx = p[r][0] - cc[0], ly = p[r][1] - cc[1], lz = p[r][2] - cc[2];
      const double h = 0.5 * ((double)lx * lx + (double)ly * ly + (double)lz * lz);
      qloc[pos] = make_float4(lx, ly, lz, (float)h);
      qorg[pos] = make_float4(p[r][0], p[r][1], p[r][2], __int_as_float(id[r]));
    } else {
      qloc[pos] = make_float4(0.0f, 0.0f, 0.0f, __builtin_inff());
      qorg[pos] = make_float4(0.0f, 0.0f, 0.0f, __int_as_float(-1));
    }
  }
  for (int o = 32; o > 0; o >>= 1) rmax = fmax(rmax, __shfl_xor(rmax, o, 64));
  if (lane == 0) {
    // radius rounded up so that it bounds |q - cc| for every member
    ccen[c] = make_float4(cc[0], cc[1], cc[2], (float)(rmax * (1.0 + 1e-6)) + 1e-30f);
    clo[c] = make_float4(mn[0], mn[1], mn[2], 0.0f);
    chi[c] = make_float4(mx[0], mx[1], mx[2], 0.0f);
  }
}

// Super-cluster boxes and the maximum cluster radius (one block of 64).
__global__ __launch_bounds__(64) void build_super_kernel(const float4* __restrict__ clo,
                                                         const float4* __restrict__ chi,
                                                         const float4* __restrict__ ccen, int ncl,
                                                         int nsup, float4* __restrict__ slo,
                                                         float4* __restrict__ shi,
                                                         float* __restrict__ rho_out,
                                                         float verlet_frac) {
  float rmax = 0.0f;
  for (int s = threadIdx.x; s < nsup; s += 64) {
    float4 lo = make_float4(__builtin_inff(), __builtin_inff(), __builtin_inff(), 0.f);
    float4 hi = make_float4(-__builtin_inff(), -__builtin_inff(), -__builtin_inff(), 0.f);
    for (int c = s * kSuper; c < min(ncl, (s + 1) * kSuper); ++c) {
      lo.x = fminf(lo.x, clo[c].x); lo.y = fminf(lo.y, clo[c].y); lo.z = fminf(lo.z, clo[c].z);
      hi.x = fmaxf(hi.x, chi[c].x); hi.y = fmaxf(hi.y, chi[c].y); hi.z = fmaxf(hi.z, chi[c].z);
      rmax = fmaxf(rmax, ccen[c].w);
    }
    slo[s] = lo;
    shi[s] = hi;
  }
  for (int o = 32; o > 0; o >>= 1) rmax = fmaxf(rmax, __shfl_xor(rmax, o, 64));
  // Median cluster radius from a histogram with four bins per octave; the
  // candidate-list margin is a fraction of it (by default about half the
  // sample spacing of a surface cluster).
  __shared__ int hist[256];
  for (int b = threadIdx.x; b < 256; b += 64) hist[b] = 0;
  __syncthreads();
  for (int c = threadIdx.x; c < ncl; c += 64) {
    const float r = ccen[c].w;
    const int b = r > 0.0f ? (int)floorf((log2f(r) + 48.0f) * 4.0f) : 0;
    atomicAdd(&hist[min(255, max(0, b))], 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0, b = 0;
    for (; b < 255; ++b) {
      acc += hist[b];
      if (2 * acc >= ncl) break;
    }
    const float rmed = exp2f((b + 1) * 0.25f - 48.0f);  // upper edge of the median bin
    rho_out[0] = rmax;
    rho_out[1] = verlet_frac * rmed;
  }
}

// Sorted source copy and the bounding sphere of each 64-source tile.
__global__ __launch_bounds__(64) void build_tiles_kernel(
    const float* __restrict__ x, const float* __restrict__ y, const float* __restrict__ z,
    const unsigned* __restrict__ order, int m, int ntile, float* __restrict__ sx,
    float* __restrict__ sy, float* __restrict__ sz, int* __restrict__ perm,
    double4* __restrict__ tsph) {
  const int t = blockIdx.x;
  if (t >= ntile) return;
  const int pos = t * kTile + threadIdx.x;
  const bool valid = pos < m;
  float p[3] = {0.f, 0.f, 0.f};
  float mn[3] = {__builtin_inff(), __builtin_inff(), __builtin_inff()};
  float mx[3] = {-__builtin_inff(), -__builtin_inff(), -__builtin_inff()};
  if (valid) {
    const int o = (int)order[pos];
    p[0] = x[o]; p[1] = y[o]; p[2] = z[o];
    sx[pos] = p[0]; sy[pos] = p[1]; sz[pos] = p[2];
    perm[pos] = o;
    for (int a = 0; a < 3; ++a) { mn[a] = p[a]; mx[a] = p[a]; }
  }
  for (int a = 0; a < 3; ++a)
    for (int o = 32; o > 0; o >>= 1) {
      mn[a] = fminf(mn[a], __shfl_xor(mn[a], o, 64));
      mx[a] = fmaxf(mx[a], __shfl_xor(mx[a], o, 64));
    }
  const double c[3] = {0.5 * ((double)mn[0] + mx[0]), 0.5 * ((double)mn[1] + mx[1]),
                       0.5 * ((double)mn[2] + mx[2])};
  double r = 0.0;
  if (valid) {
    const double ex = p[0] - c[0], ey = p[1] - c[1], ez = p[2] - c[2];
    r = sqrt(ex * ex + ey * ey + ez * ez);
  }
  for (int o = 32; o > 0; o >>= 1) r = fmax(r, __shfl_xor(r, o, 64));
  if (threadIdx.x == 0) tsph[t] = make_double4(c[0], c[1], c[2], r * (1.0 + 1e-9) + 1e-300);
}

__global__ void fill_u64_kernel(unsigned long long* __restrict__ p, int n, unsigned long long v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ------------------------------------------------------------------ planner

// Rebuild the compacted list of RUNNING slots of one branch (slots branch,
// branch + nbranch, ...) and the prefix sums of their closest-point and
// reduction work items; reset the dynamic work counters.
__global__ __launch_bounds__(1024) void plan_kernel(const SlotDesc* __restrict__ descs,
                                                    const SlotState* __restrict__ states,
                                                    WorkList* __restrict__ wl, int capacity,
                                                    int branch, int nbranch) {
  __shared__ int s_act[1024], s_nn[1024], s_epi[1024], s_b[1024];
  const int t = threadIdx.x;
  int act = 0, nn = 0, ep = 0, bi = 0;
  if (t < capacity && t % nbranch == branch && states[t].status == ST_RUNNING) {
    const SlotDesc& D = descs[t];
    act = 1;
    // cluster method: cull items (tiles) when the candidate lists are rebuilt;
    // exhaustive method: its own items whenever the pair searches
    const bool search = !states[t].reuse;
    if (D.method == NN_BRUTE) {
      bi = search ? brute_items(D.ntile, D.ncl, D.brute_clusters) : 0;
    } else {
      nn = (search && states[t].cull) ? D.ntile : 0;
      if (nn) {
        D.scount[0] = 0;
        D.scount[1] = 0;
      }
    }
    ep = D.nepi;
  }
  s_act[t] = act; s_nn[t] = nn; s_epi[t] = ep; s_b[t] = bi;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    int a = 0, b = 0, c = 0, e = 0;
    if (t >= o) { a = s_act[t - o]; b = s_nn[t - o]; c = s_epi[t - o]; e = s_b[t - o]; }
    __syncthreads();
    s_act[t] += a; s_nn[t] += b; s_epi[t] += c; s_b[t] += e;
    __syncthreads();
  }
  if (t < kQueues) {
    wl->q_nn[t * kQueueStride] = 0;
    wl->q_epi[t * kQueueStride] = 0;
  }
  if (act) {
    const int pos = s_act[t] - 1;
    wl->slot[pos] = t;
    wl->nn_base[pos] = s_nn[t] - nn;
    wl->epi_base[pos] = s_epi[t] - ep;
    wl->b_base[pos] = s_b[t] - bi;
  }
  if (t == 1023) {
    wl->single = 0;
    wl->s_from_scount = 0;
    wl->n_active = s_act[t];
    wl->nn_total = s_nn[t];
    wl->epi_total = s_epi[t];
    wl->nn_base[s_act[t]] = s_nn[t];
    wl->epi_base[s_act[t]] = s_epi[t];
    wl->b_total = s_b[t];
    wl->b_base[s_act[t]] = s_b[t];
  }
}

// ------------------------------------------------------------------ launchers

static inline int cdiv(int a, int b) { return (a + b - 1) / b; }

void launch_aos_to_soa(const float* aos, int n, float* x, float* y, float* z, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(aos_to_soa_kernel, dim3(cdiv(n, 256)), dim3(256), 0, st, aos, n, x, y, z);
}

void launch_bbox(const float* x, const float* y, const float* z, int n, float* box,
                 double* centre, hipStream_t st) {
  hipLaunchKernelGGL(bbox_kernel, dim3(1), dim3(1024), 0, st, x, y, z, n, box, centre);
}

size_t sort_scratch_words(int n) {
  const int nb = cdiv(n > 0 ? n : 1, kSortChunk);
  return (size_t)4 * n + (size_t)256 * nb + 64;
}

// Hilbert order of n points: returns (through out_vals) the permutation sorted
// by (cell key, original index). scratch: sort_scratch_words(n) unsigned words.
void launch_hilbert_order(const float* x, const float* y, const float* z, int n, const float* box,
                          unsigned* scratch, unsigned** out_vals, hipStream_t st) {
  unsigned* ka = scratch;
  unsigned* va = ka + n;
  unsigned* kb = va + n;
  unsigned* vb = kb + n;
  unsigned* hist = vb + n;
  const int nb = cdiv(n, kSortChunk);
  hipLaunchKernelGGL(hilbert_kernel, dim3(cdiv(n, 256)), dim3(256), 0, st, x, y, z, n, box, ka, va);
  for (int pass = 0; pass < 4; ++pass) {
    const int shift = 8 * pass;
    hipLaunchKernelGGL(rs_hist_kernel, dim3(nb), dim3(64), 0, st, ka, n, shift, hist);
    hipLaunchKernelGGL(rs_scan_kernel, dim3(1), dim3(1024), 0, st, hist, nb);
    hipLaunchKernelGGL(rs_scatter_kernel, dim3(nb), dim3(64), 0, st, ka, va, n, shift, hist, kb, vb);
    unsigned* t = ka; ka = kb; kb = t;
    t = va; va = vb; vb = t;
  }
  *out_vals = va;
}

void launch_build_clusters(const float* x, const float* y, const float* z, const unsigned* order,
                           int n, int ncl, float4* qloc, float4* qorg, float4* ccen, float4* clo,
                           float4* chi, float4* kbox, hipStream_t st) {
  hipLaunchKernelGGL(build_clusters_kernel, dim3(ncl), dim3(64), 0, st, x, y, z, order, n, ncl, qloc,
                     qorg, ccen, clo, chi, kbox);
}

void launch_build_super(const float4* clo, const float4* chi, const float4* ccen, int ncl, int nsup,
                        float4* slo, float4* shi, float* rho_out, float verlet_frac, hipStream_t st) {
  hipLaunchKernelGGL(build_super_kernel, dim3(1), dim3(64), 0, st, clo, chi, ccen, ncl, nsup, slo, shi,
                     rho_out, verlet_frac);
}

void launch_build_tiles(const float* x, const float* y, const float* z, const unsigned* order, int m,
                        int ntile, float* sx, float* sy, float* sz, int* perm, double4* tsph,
                        hipStream_t st) {
  hipLaunchKernelGGL(build_tiles_kernel, dim3(ntile), dim3(64), 0, st, x, y, z, order, m, ntile, sx, sy,
                     sz, perm, tsph);
}

void launch_fill_u64(unsigned long long* p, int n, unsigned long long v, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_u64_kernel, dim3(cdiv(n, 256)), dim3(256), 0, st, p, n, v);
}

void launch_plan(const SlotDesc* descs, const SlotState* states, WorkList* wl, int capacity,
                 hipStream_t st, int branch, int nbranch) {
  hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(1024), 0, st, descs, states, wl, capacity, branch,
                     nbranch);
}

}  // namespace icp
