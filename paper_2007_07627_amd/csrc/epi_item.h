// One item of the weight-and-reduce pass after the closest-point search: per source point the
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
#pragma once
#include "icp_internal.h"
#include "wave_sum.h"

namespace icp {

// The block's sum of v (NV <= 32 values per thread, four wavefronts): each
// wavefront's sum by recursive halving, then the four in wavefront order.
template <int NV>
__device__ __forceinline__ void block_reduce_store(const double (&v)[NV], double* out) {
  static_assert(NV <= 32, "at most 32 values");
  __shared__ double s_red[4][32];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double w[32];
#pragma unroll
  for (int i = 0; i < 32; ++i) w[i] = i < NV ? v[i] : 0.0;
  const double t = wave_sum32(w);
  if ((lane & 1) == 0) s_red[wave][lane >> 1] = t;
  __syncthreads();
  if (threadIdx.x < NV) {
    const int i = threadIdx.x;
    out[i] = ((s_red[0][i] + s_red[1][i]) + s_red[2][i]) + s_red[3][i];
  }
  __syncthreads();
}

// One reduction item: kEpiRows rows of 256 sorted sources, one source per
// thread and row. Every load of all rows is issued before any store or
// arithmetic (the search keys, or the previous indices when the transform is
// unchanged, and the source coordinates; then the closest targets and their
// normals), so that an item costs two memory round trips. Then the closest
// index is handed on to the next pass and the rows are accumulated in row
// order; the block reduces in a fixed order.
template <bool kPlane>
__device__ __forceinline__ void epi_item(const SlotDesc& D, const SlotState& S, int e) {
  constexpr int R = kEpiRows;
  constexpr int NV = kPlane ? kP2PLVals : kP2PVals;
  const bool reuse = S.reuse != 0;
  int si[R], idx[R];
  bool ok[R];
  unsigned long long key[R];
  float px[R], py[R], pz[R];
  // loads without branches: rows past the end read the last source instead
#pragma unroll
  for (int r = 0; r < R; ++r) {
    si[r] = e * kEpiTile + 256 * r + (int)threadIdx.x;
    ok[r] = si[r] < D.M;
    const int sc = ok[r] ? si[r] : D.M - 1;
    key[r] = ldg(D.keys, sc);
    idx[r] = ldg(D.nnidx, sc);
    px[r] = ldg(D.px, sc);
    py[r] = ldg(D.py, sc);
    pz[r] = ldg(D.pz, sc);
  }
  float qx[R], qy[R], qz[R], nx[R], ny[R], nz[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (!reuse) idx[r] = (int)(unsigned)(key[r] & 0xffffffffull);
    // every source receives a key from the search; stay in bounds regardless
    if ((unsigned)idx[r] >= (unsigned)D.N) idx[r] = 0;
    qx[r] = ldg(D.qx, idx[r]);
    qy[r] = ldg(D.qy, idx[r]);
    qz[r] = ldg(D.qz, idx[r]);
    nx[r] = ny[r] = nz[r] = 0.0f;
    if (kPlane) {
      nx[r] = ldg(D.nx, idx[r]);
      ny[r] = ldg(D.ny, idx[r]);
      nz[r] = ldg(D.nz, idx[r]);
    }
  }
  if (!reuse) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (!ok[r]) continue;
      const float d2 = __uint_as_float((unsigned)(key[r] >> 32));
      D.nnidx[si[r]] = idx[r];
      D.nnd2[si[r]] = d2;
      D.keys[si[r]] = ~0ull;  // ready for the next pass's atomic min
      if (D.idx_out) {
        const int o = D.perm[si[r]];
        D.idx_out[o] = idx[r];
        D.d2_out[o] = d2;
      }
    }
  }
  const double* T = S.Teval;
  const double s = S.inv2nu2;
  double v[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (!ok[r]) continue;
    // FP64 transform with the same fused order as the search, not rounded
    const double p0 = px[r], p1 = py[r], p2 = pz[r];
    const double x = __builtin_fma(T[2], p2, __builtin_fma(T[1], p1, __builtin_fma(T[0], p0, T[3])));
    const double y = __builtin_fma(T[6], p2, __builtin_fma(T[5], p1, __builtin_fma(T[4], p0, T[7])));
    const double z = __builtin_fma(T[10], p2, __builtin_fma(T[9], p1, __builtin_fma(T[8], p0, T[11])));
    const double qxd = qx[r], qyd = qy[r], qzd = qz[r];
    const double dx = x - qxd, dy = y - qyd, dz = z - qzd;
    if (!kPlane) {
      const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
      double w = 1.0;
      if (D.mode == P2P_L2) {
        v[0] += r2;
      } else {
        v[0] += -expm1(-r2 * s);
        w = exp(-r2 * s);
      }
      if (S.want_median) D.medkey[si[r]] = r2;
      const double a0 = p0 - S.cP[0], a1 = p1 - S.cP[1], a2 = p2 - S.cP[2];
      const double b0 = qxd - S.cQ[0], b1 = qyd - S.cQ[1], b2 = qzd - S.cQ[2];
      const double wa0 = w * a0, wa1 = w * a1, wa2 = w * a2;
      v[1] += w;
      v[2] += wa0; v[3] += wa1; v[4] += wa2;
      v[5] += w * b0; v[6] += w * b1; v[7] += w * b2;
      v[8] += wa0 * b0; v[9] += wa0 * b1; v[10] += wa0 * b2;
      v[11] += wa1 * b0; v[12] += wa1 * b1; v[13] += wa1 * b2;
      v[14] += wa2 * b0; v[15] += wa2 * b1; v[16] += wa2 * b2;
    } else {
      const double n0 = nx[r], n1 = ny[r], n2 = nz[r];
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
      if (S.want_median) D.medkey[si[r]] = fabs(B);
      // J: rotation part n . (dR_j p + dt/d delta_j), translation part (dt/du)^T n
      const double* K = S.K;
      double J[6];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const double* Rj = K + 9 * j;
        const double r0 = Rj[0] * p0 + Rj[1] * p1 + Rj[2] * p2 + K[27 + 0 + j];
        const double r1 = Rj[3] * p0 + Rj[4] * p1 + Rj[5] * p2 + K[27 + 3 + j];
        const double r2 = Rj[6] * p0 + Rj[7] * p1 + Rj[8] * p2 + K[27 + 6 + j];
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
  }
  block_reduce_store<NV>(v, D.part + (size_t)e * kPartStride);
}

}  // namespace icp
