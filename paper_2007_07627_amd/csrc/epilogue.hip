// Weight-and-reduce pass after the closest-point search: per source point the
// FP64 residual at the evaluated transform, the Welsch weight and energy term,
// and the moments of the alignment problem; one fixed-order FP64 partial per
// kEpiTile-source item (no floating-point atomics, so results do not depend on
// the batch composition or on scheduling).
//
//  point-to-point (eq. WelschAlignment): w = exp(-r^2 / (2 nu^2)) (w = 1 for
//    L2), energy psi_nu(r) = -expm1(-r^2 / (2 nu^2)) (eq. welsch) or r^2, and
//    sum w, sum w p~, sum w q~, sum w p~ q~^T with p~, q~ centred by fixed
//    per-pair bounding-box centres.
//  point-to-plane (eq. ProxyPointToPlaneAlignment, eq. GNSystem): B = (x - q) . n,
//    g = exp(-B^2 / (2 nu^2)), J from the per-pass derivative matrices
//    (App. D), sum g J J^T (upper triangle), sum g B J, sum g, sum psi_nu(B);
//    classical point-to-plane ICP takes g = 1 and the energy term B^2.
#include "icp_internal.h"

namespace icp {

template <int NV>
__device__ __forceinline__ void block_reduce_store(double (&v)[NV], double* out) {
  __shared__ double s_red[4][32];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double x = v[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
    v[i] = x;
  }
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) s_red[wave][i] = v[i];
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    const int i = threadIdx.x;
    out[i] = ((s_red[0][i] + s_red[1][i]) + s_red[2][i]) + s_red[3][i];
  }
  __syncthreads();
}

// Closest target of sorted source si from this pass's key (or the previous
// pass's index when the transform is unchanged), with the FP64 residual at
// the evaluated transform. Also hands the index on to the next pass.
__device__ __forceinline__ bool source_residual(const SlotDesc& D, const SlotState& S,
                                                const double* T, int si, int& idx, double& px,
                                                double& py, double& pz, double& qxd, double& qyd,
                                                double& qzd, double& dx, double& dy, double& dz) {
  if (si >= D.M) return false;
  if (!S.reuse) {
    const unsigned long long key = D.keys[si];
    idx = (int)(unsigned)(key & 0xffffffffull);
    // every source receives a key from the search; stay in bounds regardless
    if ((unsigned)idx >= (unsigned)D.N) idx = 0;
    const float d2 = __uint_as_float((unsigned)(key >> 32));
    D.nnidx[si] = idx;
    D.nnd2[si] = d2;
    D.keys[si] = ~0ull;  // ready for the next pass's atomic min
    if (D.idx_out) {
      const int o = D.perm[si];
      D.idx_out[o] = idx;
      D.d2_out[o] = d2;
    }
  } else {
    idx = D.nnidx[si];
  }
  px = D.px[si];
  py = D.py[si];
  pz = D.pz[si];
  // FP64 transform with the same fused order as the search, not rounded
  const double x = __builtin_fma(T[2], pz, __builtin_fma(T[1], py, __builtin_fma(T[0], px, T[3])));
  const double y = __builtin_fma(T[6], pz, __builtin_fma(T[5], py, __builtin_fma(T[4], px, T[7])));
  const double z = __builtin_fma(T[10], pz, __builtin_fma(T[9], py, __builtin_fma(T[8], px, T[11])));
  qxd = D.qx[idx];
  qyd = D.qy[idx];
  qzd = D.qz[idx];
  dx = x - qxd;
  dy = y - qyd;
  dz = z - qzd;
  return true;
}

__device__ __forceinline__ void accumulate_p2p(const SlotDesc& D, const SlotState& S,
                                               const double* T, int si, double (&v)[kP2PVals]) {
  int idx = 0;
  double px, py, pz, qxd, qyd, qzd, dx, dy, dz;
  if (!source_residual(D, S, T, si, idx, px, py, pz, qxd, qyd, qzd, dx, dy, dz)) return;
  const double s = S.inv2nu2;
  const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
  double w = 1.0;
  if (D.mode == P2P_L2) {
    v[0] += r2;
  } else {
    v[0] += -expm1(-r2 * s);
    w = exp(-r2 * s);
  }
  if (S.want_median) D.medkey[si] = r2;
  const double a0 = px - S.cP[0], a1 = py - S.cP[1], a2 = pz - S.cP[2];
  const double b0 = qxd - S.cQ[0], b1 = qyd - S.cQ[1], b2 = qzd - S.cQ[2];
  const double wa0 = w * a0, wa1 = w * a1, wa2 = w * a2;
  v[1] += w;
  v[2] += wa0; v[3] += wa1; v[4] += wa2;
  v[5] += w * b0; v[6] += w * b1; v[7] += w * b2;
  v[8] += wa0 * b0; v[9] += wa0 * b1; v[10] += wa0 * b2;
  v[11] += wa1 * b0; v[12] += wa1 * b1; v[13] += wa1 * b2;
  v[14] += wa2 * b0; v[15] += wa2 * b1; v[16] += wa2 * b2;
}

__device__ __forceinline__ void accumulate_p2pl(const SlotDesc& D, const SlotState& S,
                                                const double* T, int si, double (&v)[kP2PLVals]) {
  int idx = 0;
  double px, py, pz, qxd, qyd, qzd, dx, dy, dz;
  if (!source_residual(D, S, T, si, idx, px, py, pz, qxd, qyd, qzd, dx, dy, dz)) return;
  const double s = S.inv2nu2;
  const double n0 = D.nx[idx], n1 = D.ny[idx], n2 = D.nz[idx];
  const double B = __builtin_fma(dz, n2, __builtin_fma(dy, n1, dx * n0));
  // classical point-to-plane ICP: unit weights and energy B^2
  double gam = 1.0;
  if (D.mode == P2PL_L2) {
    v[0] += B * B;
  } else {
    const double B2s = B * B * s;
    gam = exp(-B2s);
    v[0] += -expm1(-B2s);
  }
  v[1] += gam;
  if (S.want_median) D.medkey[si] = fabs(B);
  // J: rotation part n . (dR_j p + dt/d delta_j), translation part (dt/du)^T n
  const double* K = S.K;
  double J[6];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const double* R = K + 9 * j;
    const double r0 = R[0] * px + R[1] * py + R[2] * pz + K[27 + 0 + j];
    const double r1 = R[3] * px + R[4] * py + R[5] * pz + K[27 + 3 + j];
    const double r2 = R[6] * px + R[7] * py + R[8] * pz + K[27 + 6 + j];
    J[j] = n0 * r0 + n1 * r1 + n2 * r2;
    J[3 + j] = K[36 + j] * n0 + K[36 + 3 + j] * n1 + K[36 + 6 + j] * n2;
  }
  int t = 2;
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    const double ga = gam * J[a];
#pragma unroll
    for (int b = a; b < 6; ++b) v[t++] += ga * J[b];
  }
  const double gB = gam * B;
#pragma unroll
  for (int a = 0; a < 6; ++a) v[23 + a] += gB * J[a];
}

__global__ __launch_bounds__(256) void epi_kernel(const SlotDesc* __restrict__ descs,
                                                  const SlotState* __restrict__ states,
                                                  WorkList* __restrict__ wl) {
  __shared__ int s_item;
  for (int round = 0;; ++round) {
    if (threadIdx.x == 0) s_item = queue_item(wl->q_epi, round);
    __syncthreads();
    // the item (and so the slot) is uniform over the block: kept in scalar
    // registers, the descriptor and state fields are scalar loads
    const int g = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (g >= wl->epi_total) break;
    int lo = 0, hi = wl->n_active - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (wl->epi_base[mid] <= g) lo = mid; else hi = mid - 1;
    }
    lo = __builtin_amdgcn_readfirstlane(lo);
    const int slot = __builtin_amdgcn_readfirstlane(wl->slot[lo]);
    const SlotDesc& D = descs[slot];
    const SlotState& S = states[slot];
    const int e = g - wl->epi_base[lo];
    const double* T = S.Teval;
    double* out = D.part + (size_t)e * kPartStride;
    // each thread accumulates kEpiRows sources (one per 256-source row of the
    // item) in row order, then the block reduces in a fixed order
    if (!mode_plane(D.mode)) {
      double v[kP2PVals];
#pragma unroll
      for (int i = 0; i < kP2PVals; ++i) v[i] = 0.0;
#pragma unroll
      for (int r = 0; r < kEpiRows; ++r) accumulate_p2p(D, S, T, e * kEpiTile + 256 * r + threadIdx.x, v);
      block_reduce_store<kP2PVals>(v, out);
    } else {
      double v[kP2PLVals];
#pragma unroll
      for (int i = 0; i < kP2PLVals; ++i) v[i] = 0.0;
#pragma unroll
      for (int r = 0; r < kEpiRows; ++r) accumulate_p2pl(D, S, T, e * kEpiTile + 256 * r + threadIdx.x, v);
      block_reduce_store<kP2PLVals>(v, out);
    }
  }
}

void launch_epi(const SlotDesc* descs, const SlotState* states, WorkList* wl, int grid,
                hipStream_t st) {
  hipLaunchKernelGGL(epi_kernel, dim3(grid), dim3(256), 0, st, descs, states, wl);
}

}  // namespace icp
