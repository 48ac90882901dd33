// Nearest-neighbour statistics of a target set on its cluster index.
//
// Automatic nu_min (Sec. 4.3 for point-to-point, Sec. 5 for point-to-plane,
// rationale in App. C): for every target q_i its six nearest other targets
// (exact FP32 squared distances of q_i - q_j as in the closest-point search,
// ties to the lower index); per target the median (element of rank 3) of
// their distances (point-to-point, taken on squares) or of their distances
// |n_i . (q_j - q_i)| to the tangent plane at q_i (point-to-plane); then the
// median (rank floor(N / 2)) over the targets, Ebar or Hbar, and
// nu_min = sqrt(Ebar) / (3 sqrt 3) or Hbar / 6. Runs once per registration.
//
// Normals for point-to-plane registration of targets given without normals
// (the paper estimates them from 30 nearest neighbours): PCA of each point's
// 30 nearest points, the point included.
#include "icp_internal.h"

namespace icp {

// Inserts a key into the ascending K keys t[0..K-1] (the largest drops out).
template <int K>
__device__ __forceinline__ void insert_k(unsigned long long (&t)[K], unsigned long long k) {
  if (!(k < t[K - 1])) return;
  t[K - 1] = k;
#pragma unroll
  for (int i = K - 1; i > 0; --i) {
    const unsigned long long a = t[i - 1], b = t[i];
    t[i - 1] = b < a ? b : a;
    t[i] = b < a ? a : b;
  }
}

// Squared-distance bound of the K-th key (+inf while fewer than K).
template <int K>
__device__ __forceinline__ float bound_k(const unsigned long long (&t)[K]) {
  return t[K - 1] == ~0ull ? __builtin_inff() : __uint_as_float((unsigned)(t[K - 1] >> 32));
}

// The K nearest points of the set (cluster index qorg/boxes) to each lane's
// point `me` (original index my), as ascending (d2, index) keys; kSelf: the
// point itself counts (at distance 0), otherwise it is excluded. The points'
// own cluster and its two neighbours along the curve give a first bound;
// then every cluster whose box some lane's bound still reaches (super-cluster
// boxes first) is scanned, staged in LDS. Called by the whole wavefront; tile
// is the first cluster-sorted position of the wavefront's 64 points.
template <int K, bool kSelf>
__device__ void knn_search(const float4* __restrict__ qorg, const float4* __restrict__ clo,
                           const float4* __restrict__ chi, const float4* __restrict__ slo,
                           const float4* __restrict__ shi, int ncl, int nsup, int tile, float4 me,
                           int my, bool valid, float4* s_t, unsigned long long (&t)[K]) {
  const int lane = threadIdx.x;
#pragma unroll
  for (int i = 0; i < K; ++i) t[i] = ~0ull;
  auto scan = [&](int c) {
    __syncthreads();
    for (int r = 0; r < kCluster / 64; ++r) s_t[64 * r + lane] = qorg[(size_t)c * kCluster + 64 * r + lane];
    __syncthreads();
    if (!valid) return;
    for (int j = 0; j < kCluster; ++j) {
      const float4 q = s_t[j];
      const int id = __float_as_int(q.w);
      const float dx = me.x - q.x, dy = me.y - q.y, dz = me.z - q.z;
      const float d = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
      // padding (id < 0) never enters; the point itself only with kSelf
      if (id >= 0 && (kSelf || id != my)) insert_k<K>(t, make_key(d, id));
    }
  };
  const int c0 = tile / kCluster;
  for (int c = max(0, c0 - 1); c <= min(ncl - 1, c0 + 1); ++c) scan(c);
  for (int s2 = 0; s2 < nsup; ++s2) {
    const float4 slo2 = slo[s2], shi2 = shi[s2];
    const bool sneed = valid && box_lb2(me.x, me.y, me.z, slo2, shi2) * (1.0f - 0x1.0p-20f) <= bound_k<K>(t);
    if (!__any(sneed)) continue;
    for (int c = s2 * kSuper; c < min(ncl, (s2 + 1) * kSuper); ++c) {
      if (c >= c0 - 1 && c <= c0 + 1) continue;
      const bool need = valid && box_lb2(me.x, me.y, me.z, clo[c], chi[c]) * (1.0f - 0x1.0p-20f) <= bound_k<K>(t);
      if (__any(need)) scan(c);
    }
  }
}

// One wavefront per 64 cluster-sorted targets: their six nearest other
// targets, then the per-target value whose median gives nu_min.
__global__ __launch_bounds__(64) void knn6_kernel(
    const float4* __restrict__ qorg, const float4* __restrict__ clo, const float4* __restrict__ chi,
    const float4* __restrict__ slo, const float4* __restrict__ shi, int ncl, int nsup,
    const float* __restrict__ qx, const float* __restrict__ qy, const float* __restrict__ qz,
    const float* __restrict__ nx, const float* __restrict__ ny, const float* __restrict__ nz,
    int plane, double* __restrict__ vals) {
  __shared__ float4 s_t[kCluster];
  const int pos = blockIdx.x * 64 + threadIdx.x;  // < ncl * kCluster by the grid
  const float4 me = qorg[pos];
  const int my = __float_as_int(me.w);
  const bool valid = my >= 0;
  unsigned long long t[6];
  knn_search<6, false>(qorg, clo, chi, slo, shi, ncl, nsup, blockIdx.x * 64, me, my, valid, s_t, t);
  if (!valid) return;
  if (!plane) {
    vals[my] = (double)__uint_as_float((unsigned)(t[3] >> 32));
    return;
  }
  // distances of the six to the tangent plane at q_i, then their median
  const double n0 = nx[my], n1 = ny[my], n2 = nz[my];
  const double x = qx[my], y = qy[my], z = qz[my];
  double h[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const int j = (int)(unsigned)(t[k] & 0xffffffffull);
    const double dx = (double)qx[j] - x, dy = (double)qy[j] - y, dz = (double)qz[j] - z;
    h[k] = fabs(__builtin_fma(n2, dz, __builtin_fma(n1, dy, n0 * dx)));
  }
  // sorting network for six
#define ICP_CS(a, b) { const double u = fmin(h[a], h[b]), v = fmax(h[a], h[b]); h[a] = u; h[b] = v; }
  ICP_CS(0, 1) ICP_CS(2, 3) ICP_CS(4, 5) ICP_CS(0, 2) ICP_CS(1, 4) ICP_CS(3, 5)
  ICP_CS(0, 1) ICP_CS(2, 3) ICP_CS(4, 5) ICP_CS(1, 2) ICP_CS(3, 4) ICP_CS(2, 3)
#undef ICP_CS
  vals[my] = h[3];
}

// Median (rank floor(n / 2)) of the per-target values by an 8-bit radix
// select on their FP64 bit patterns (all values are >= 0), then nu_min.
__global__ __launch_bounds__(1024) void nu_min_kernel(const double* __restrict__ vals, int n,
                                                      int plane, double* __restrict__ out) {
  __shared__ unsigned hist[256];
  __shared__ unsigned long long s_prefix, s_mask;
  __shared__ long long s_k;
  if (threadIdx.x == 0) {
    s_prefix = 0ull;
    s_mask = 0ull;
    s_k = n / 2;
  }
  __syncthreads();
  for (int shift = 56; shift >= 0; shift -= 8) {
    for (int i = threadIdx.x; i < 256; i += blockDim.x) hist[i] = 0u;
    __syncthreads();
    const unsigned long long pre = s_prefix, msk = s_mask;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const unsigned long long key = (unsigned long long)__double_as_longlong(vals[i]);
      if ((key & msk) == pre) atomicAdd(&hist[(key >> shift) & 255ull], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      long long k = s_k;
      int d = 0;
      for (; d < 256; ++d) {
        if (k < (long long)hist[d]) break;
        k -= hist[d];
      }
      s_k = k;
      s_prefix = pre | ((unsigned long long)d << shift);
      s_mask = msk | (255ull << shift);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double med = __longlong_as_double((long long)s_prefix);
    *out = plane ? med / 6.0 : sqrt(med) / (3.0 * sqrt(3.0));
  }
}

void launch_nu_min_auto(const float4* qorg, const float4* clo, const float4* chi, const float4* slo,
                        const float4* shi, int ncl, int nsup, const float* qx, const float* qy,
                        const float* qz, const float* nx, const float* ny, const float* nz, int n,
                        bool plane, double* vals, double* out, hipStream_t st) {
  hipLaunchKernelGGL(knn6_kernel, dim3(ncl * (kCluster / 64)), dim3(64), 0, st, qorg, clo, chi, slo,
                     shi, ncl, nsup, qx, qy, qz, nx, ny, nz, plane ? 1 : 0, vals);
  hipLaunchKernelGGL(nu_min_kernel, dim3(1), dim3(1024), 0, st, vals, n, plane ? 1 : 0, out);
}

// Normals from the 30 nearest points (the point included): FP64 mean and
// covariance of the 30 in key order, the unit eigenvector of the smallest
// eigenvalue by cyclic Jacobi rotations, oriented so that n . q <= 0
// (towards a viewpoint at the origin). Written in the original order.
__global__ __launch_bounds__(64) void normals_kernel(
    const float4* __restrict__ qorg, const float4* __restrict__ clo, const float4* __restrict__ chi,
    const float4* __restrict__ slo, const float4* __restrict__ shi, int ncl, int nsup,
    const float* __restrict__ qx, const float* __restrict__ qy, const float* __restrict__ qz,
    float* __restrict__ out) {
  constexpr int K = 30;
  __shared__ float4 s_t[kCluster];
  const int pos = blockIdx.x * 64 + threadIdx.x;
  const float4 me = qorg[pos];
  const int my = __float_as_int(me.w);
  const bool valid = my >= 0;
  unsigned long long t[K];
  knn_search<K, true>(qorg, clo, chi, slo, shi, ncl, nsup, blockIdx.x * 64, me, my, valid, s_t, t);
  if (!valid) return;
  double m[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int j = (int)(unsigned)(t[k] & 0xffffffffull);
    m[0] += (double)qx[j];
    m[1] += (double)qy[j];
    m[2] += (double)qz[j];
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) m[a] /= K;
  double C[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int j = (int)(unsigned)(t[k] & 0xffffffffull);
    const double e[3] = {(double)qx[j] - m[0], (double)qy[j] - m[1], (double)qz[j] - m[2]};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) C[3 * a + b] += e[a] * e[b];
  }
#pragma unroll
  for (int a = 0; a < 9; ++a) C[a] /= K;
  // cyclic Jacobi on the symmetric 3x3, rotations accumulated in V
  double V[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  for (int sweep = 0; sweep < 30; ++sweep) {
    const double off = C[1] * C[1] + C[2] * C[2] + C[5] * C[5];
    const double tot = off + C[0] * C[0] + C[4] * C[4] + C[8] * C[8];
    if (off <= 1e-32 * tot || off == 0.0) break;
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int r = p + 1; r < 3; ++r) {
        const double apr = C[3 * p + r];
        if (!(fabs(apr) > 1e-18 * (fabs(C[4 * p]) + fabs(C[4 * r])))) continue;
        const double th = (C[4 * r] - C[4 * p]) / (2.0 * apr);
        const double tt = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        const double c = 1.0 / sqrt(tt * tt + 1.0), sn = tt * c;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const double akp = C[3 * k + p], akr = C[3 * k + r];
          C[3 * k + p] = c * akp - sn * akr;
          C[3 * k + r] = sn * akp + c * akr;
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const double apk = C[3 * p + k], ark = C[3 * r + k];
          C[3 * p + k] = c * apk - sn * ark;
          C[3 * r + k] = sn * apk + c * ark;
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const double vkp = V[3 * k + p], vkr = V[3 * k + r];
          V[3 * k + p] = c * vkp - sn * vkr;
          V[3 * k + r] = sn * vkp + c * vkr;
        }
      }
  }
  int b = 0;
  if (C[4] < C[0]) b = 1;
  if (C[8] < C[4 * b]) b = 2;
  double n[3] = {V[b], V[3 + b], V[6 + b]};
  const double l = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  const double sg = (n[0] * (double)me.x + n[1] * (double)me.y + n[2] * (double)me.z > 0.0) ? -1.0 : 1.0;
  out[3 * (size_t)my + 0] = (float)(sg * n[0] / l);
  out[3 * (size_t)my + 1] = (float)(sg * n[1] / l);
  out[3 * (size_t)my + 2] = (float)(sg * n[2] / l);
}

void launch_estimate_normals(const float4* qorg, const float4* clo, const float4* chi,
                             const float4* slo, const float4* shi, int ncl, int nsup,
                             const float* qx, const float* qy, const float* qz, float* out,
                             hipStream_t st) {
  hipLaunchKernelGGL(normals_kernel, dim3(ncl * (kCluster / 64)), dim3(64), 0, st, qorg, clo, chi,
                     slo, shi, ncl, nsup, qx, qy, qz, out);
}

}  // namespace icp
