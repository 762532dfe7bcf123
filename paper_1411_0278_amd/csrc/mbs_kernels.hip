// HIP kernels of libmbstokes for gfx950 (CDNA4): all-pairs Galerkin pair passes, Krylov
// helpers and the rigid-body stepper.
//
// Pair passes. For spheres n (receiver) and m (source), x = R_n - R_m, r = |x|, P = 1/(8 pi eta).
// The off-diagonal Galerkin matrix elements are derivatives of the unbounded Green's function
// G = I/r + x x / r^3 under the finite-size operators F^l = 1 + a^2/(4l+6) nabla^2 (section III,
// matrix elements for m != n). Because nabla^4 G = 0 every composed operator ends after one
// Laplacian, which gives the closed forms used below (w = Sigma.x, q = x.Sigma.x):
//
//   U <- F      P[(1/r + 2a^2/3r^3) F + (1/r^3 - 2a^2/r^5)(x.F) x]          (Rotne-Prager)
//   U <- T      P (T x x)/r^3
//   U <- Sigma  P[q x (-3/r^5 + 8a^2/r^7) - (16a^2/5) w / r^5]
//   U <- d      (a^5/10)[3 (x.d) x / r^5 - d / r^3]
//   W <- F      P (F x x)/r^3
//   W <- T      (P/2)[3 (x.T) x / r^5 - T / r^3]
//   W <- Sigma  3P (x x w)/r^5
//   E <- F      P[(x.F)(-3/r^5 + 8a^2/r^7) x x - (16a^2/5) sym(F x)/r^5]    (traceless part)
//   E <- T      -3P sym((T x x) x)/r^5
//   E <- Sigma  P[c1 sym(x w) + c2 x x + c3 Sigma],  c1 = -6/r^5 + 24a^2/r^7,
//               c2 = q (15/r^7 - 42a^2/r^9),  c3 = -12a^2/(5 r^5)                (traceless part)
//   E <- d      (a^5/10)[3 (x d + d x)/r^5 - 15 (x.d) x x / r^7]             (traceless part)
//
// Every strain contribution except c3 Sigma has the form sym(x (x) v) for a vector v, so a pass
// accumulates v's contraction with x directly in the 5-component basis (B0..B4, see the public
// header), scaled by (sqrt2, sqrt6, sqrt2, sqrt2, sqrt2) so that no square root appears per pair.
//
// Layout: one thread owns one receiver (coordinates and accumulators in registers); sources
// are staged through LDS in tiles as 64-byte (P2), 96-byte (P1) or 144-byte (P3) records that
// every lane of a wavefront reads at the same address (LDS broadcast). grid.x runs over
// receiver tiles, grid.y over source chunks; chunk partial sums are reduced in a fixed order
// by a finishing kernel, so results are bitwise reproducible. The n == m term is removed by
// setting 1/r to zero when r == 0 (every term carries at least one power of 1/r).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "mbs_device.h"
#include "mbs_grid.h"
#include "mbs_internal.h"
#include "mbs_pair.h"

namespace mbs {

namespace {

// ------------------------------------------------------------------ P1: right-hand side
template <int TJ, bool HAS_T, bool HAS_D>
__global__ void __launch_bounds__(kMaxBlock)
    k_p1(const double* __restrict__ R, const double* __restrict__ Fe, const double* __restrict__ Te,
         const double* __restrict__ D, const double* __restrict__ v2s, double* __restrict__ out,
         int n, int chunk, double P, double a2, double a5_10, double cslip, int direct) {
  __shared__ RecF tile[TJ];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int ii = i < n ? i : n - 1;
  const int b0 = blockIdx.x * blockDim.x;
  const int b1 = min(n, b0 + (int)blockDim.x);
  const double xi = R[3 * ii], yi = R[3 * ii + 1], zi = R[3 * ii + 2];
  const int j0 = blockIdx.y * chunk;
  const int j1 = min(n, j0 + chunk);
  const double A8 = 8.0 * a2, B16 = -3.2 * a2;  // 8a^2, -(16/5) a^2
  Mom6 m;  // raw moments x_i v_j of the per-pair vector v (traceless projection once per receiver)
  for (int jt = j0; jt < j1; jt += TJ) {
    const int cnt = min(TJ, j1 - jt);
    __syncthreads();
    for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
      const int j = jt + t;
      RecF rc;
      rc.x = R[3 * j];
      rc.y = R[3 * j + 1];
      rc.z = R[3 * j + 2];
      rc.fx = P * Fe[3 * j];
      rc.fy = P * Fe[3 * j + 1];
      rc.fz = P * Fe[3 * j + 2];
      if (HAS_T) {
        rc.tx = P * Te[3 * j];
        rc.ty = P * Te[3 * j + 1];
        rc.tz = P * Te[3 * j + 2];
      } else {
        rc.tx = rc.ty = rc.tz = 0.0;
      }
      if (HAS_D) {
        rc.dx = a5_10 * D[3 * j];
        rc.dy = a5_10 * D[3 * j + 1];
        rc.dz = a5_10 * D[3 * j + 2];
      } else {
        rc.dx = rc.dy = rc.dz = 0.0;
      }
      tile[t] = rc;
    }
    __syncthreads();
    if (jt < b1 && jt + cnt > b0) {  // (uniform) the tile may hold a receiver of this workgroup
#pragma unroll 2
      for (int jj = 0; jj < cnt; ++jj) p1_pair<true, HAS_T, HAS_D>(tile[jj], xi, yi, zi, A8, B16, m);
    } else {
      int jj = 0;
      for (; jj + 2 <= cnt; jj += 2) p1_pairs<2, HAS_T, HAS_D>(tile + jj, xi, yi, zi, A8, B16, m);
      for (; jj < cnt; ++jj) p1_pair<false, HAS_T, HAS_D>(tile[jj], xi, yi, zi, A8, B16, m);
    }
  }
  if (i >= n) return;
  double e[5];
  mom6_to_basis(m, e);
  if (direct) {
#pragma unroll
    for (int c = 0; c < 5; ++c)
      out[5 * (int64_t)i + c] = e[c] - (v2s ? cslip * v2s[5 * (int64_t)i + c] : 0.0);
  } else {
    double* o = out + (int64_t)blockIdx.y * 5 * n + 5 * (int64_t)i;
#pragma unroll
    for (int c = 0; c < 5; ++c) o[c] = e[c];
  }
}

__global__ void k_p1_finish(const double* __restrict__ part, const double* __restrict__ v2s,
                            double* __restrict__ b, int64_t len, int split, double cslip) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= len) return;
  double acc = 0.0;
  for (int s = 0; s < split; ++s) acc += part[s * len + k];
  b[k] = acc - (v2s ? cslip * v2s[k] : 0.0);
}

// ------------------------------------------------------------------ P3: rigid-body outputs
// One source record of the output pass: position, P-scaled force, torque and stresslet
// (Cartesian), (a^5/10)-scaled rank-3 trace mode.
template <bool HAS_T, bool HAS_D>
__device__ __forceinline__ RecO make_reco(const double* __restrict__ R, const double* __restrict__ Fe,
                                          const double* __restrict__ Te, const double* __restrict__ Sig,
                                          const double* __restrict__ D, int j, double P, double a5_10) {
  RecO rc;
  rc.x = R[3 * (int64_t)j];
  rc.y = R[3 * (int64_t)j + 1];
  rc.z = R[3 * (int64_t)j + 2];
  rc.fx = P * Fe[3 * (int64_t)j];
  rc.fy = P * Fe[3 * (int64_t)j + 1];
  rc.fz = P * Fe[3 * (int64_t)j + 2];
  if (HAS_T) {
    rc.tx = P * Te[3 * (int64_t)j];
    rc.ty = P * Te[3 * (int64_t)j + 1];
    rc.tz = P * Te[3 * (int64_t)j + 2];
  } else {
    rc.tx = rc.ty = rc.tz = 0.0;
  }
  double sxx, syy, sxy, sxz, syz;
  basis_to_cart(Sig + 5 * (int64_t)j, sxx, syy, sxy, sxz, syz);
  rc.sxx = P * sxx;
  rc.syy = P * syy;
  rc.sxy = P * sxy;
  rc.sxz = P * sxz;
  rc.syz = P * syz;
  if (HAS_D) {
    rc.dx = a5_10 * D[3 * (int64_t)j];
    rc.dy = a5_10 * D[3 * (int64_t)j + 1];
    rc.dz = a5_10 * D[3 * (int64_t)j + 2];
  } else {
    rc.dx = rc.dy = rc.dz = 0.0;
  }
  rc.pad = 0.0;
  return rc;
}
template <int TJ, bool HAS_T, bool HAS_D>
__global__ void __launch_bounds__(kMaxBlock)
    k_p3(const double* __restrict__ R, const double* __restrict__ Fe, const double* __restrict__ Te,
         const double* __restrict__ Sig, const double* __restrict__ D, double* __restrict__ out,
         int n, int chunk, double P, double a2, double a5_10) {
  __shared__ RecO tile[TJ];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int ii = i < n ? i : n - 1;
  const int b0 = blockIdx.x * blockDim.x;
  const int b1 = min(n, b0 + (int)blockDim.x);
  const double xi = R[3 * ii], yi = R[3 * ii + 1], zi = R[3 * ii + 2];
  const int j0 = blockIdx.y * chunk;
  const int j1 = min(n, j0 + chunk);
  const double A2_2 = 2.0 * a2, A2_23 = 2.0 * a2 / 3.0, A8 = 8.0 * a2, B16 = -3.2 * a2;
  UW acc;
  for (int jt = j0; jt < j1; jt += TJ) {
    const int cnt = min(TJ, j1 - jt);
    __syncthreads();
    for (int t = threadIdx.x; t < cnt; t += blockDim.x)
      tile[t] = make_reco<HAS_T, HAS_D>(R, Fe, Te, Sig, D, jt + t, P, a5_10);
    __syncthreads();
    if (jt < b1 && jt + cnt > b0) {  // (uniform) the tile may hold a receiver of this workgroup
#pragma unroll 2
      for (int jj = 0; jj < cnt; ++jj)
        p3_pair<true, HAS_T, HAS_D>(tile[jj], xi, yi, zi, A2_2, A2_23, A8, B16, acc);
    } else {
#pragma unroll 2
      for (int jj = 0; jj < cnt; ++jj)
        p3_pair<false, HAS_T, HAS_D>(tile[jj], xi, yi, zi, A2_2, A2_23, A8, B16, acc);
    }
  }
  if (i >= n) return;
  double* o = out + (int64_t)blockIdx.y * 6 * n + 6 * (int64_t)i;
  o[0] = acc.ux;
  o[1] = acc.uy;
  o[2] = acc.uz;
  o[3] = acc.wx;
  o[4] = acc.wy;
  o[5] = acc.wz;
}

__global__ void k_p3_finish(const double* __restrict__ part, int split, int64_t n,
                            const double* __restrict__ v1s, const double* __restrict__ v2s,
                            const double* __restrict__ Fe, const double* __restrict__ Te,
                            const double* __restrict__ Sig, double* __restrict__ V,
                            double* __restrict__ W, double* __restrict__ S, double mu_t,
                            double mu_r, double slip_S) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int s = 0; s < split; ++s) {
    const double* p = part + (int64_t)s * 6 * n + 6 * i;
#pragma unroll
    for (int c = 0; c < 6; ++c) acc[c] += p[c];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    V[3 * i + c] = acc[c] + mu_t * Fe[3 * i + c] - (v1s ? v1s[3 * i + c] : 0.0);
    W[3 * i + c] = acc[3 + c] + (Te ? mu_r * Te[3 * i + c] : 0.0);
  }
  if (S) {
#pragma unroll
    for (int c = 0; c < 5; ++c) S[5 * i + c] = Sig[5 * i + c] + (v2s ? slip_S * v2s[5 * i + c] : 0.0);
  }
}

// ------------------------------------------------------------------ fused output + operator pass
// The output pass and one binary64 operator application on the same stresslet share the pair
// geometry (separation, powers of 1/r, w = Sigma x, q = x.w), so one pass yields both the rigid-body
// sums and y = Sigma/gamma - E[Sigma]: used for the final residual of a solve. Per receiver and
// source chunk it stores the 5 strain components then the 6 velocity/rotation sums.
template <int TJ, bool HAS_T, bool HAS_D>
__global__ void __launch_bounds__(kMaxBlock)
    k_p23(const double* __restrict__ R, const double* __restrict__ Fe, const double* __restrict__ Te,
          const double* __restrict__ Sig, const double* __restrict__ D, double* __restrict__ out,
          int n, int chunk, double P, double a2, double a5_10) {
  __shared__ RecO tile[TJ];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int ii = i < n ? i : n - 1;
  const int b0 = blockIdx.x * blockDim.x;
  const int b1 = min(n, b0 + (int)blockDim.x);
  const double xi = R[3 * (int64_t)ii], yi = R[3 * (int64_t)ii + 1], zi = R[3 * (int64_t)ii + 2];
  const int j0 = blockIdx.y * chunk;
  const int j1 = min(n, j0 + chunk);
  const double A2_2 = 2.0 * a2, A2_23 = 2.0 * a2 / 3.0, A8 = 8.0 * a2, B16 = -3.2 * a2;
  const double A24 = 24.0 * a2, A42 = 42.0 * a2;
  UW acc;
  Mom<double> m;
  for (int jt = j0; jt < j1; jt += TJ) {
    const int cnt = min(TJ, j1 - jt);
    __syncthreads();
    for (int t = threadIdx.x; t < cnt; t += blockDim.x)
      tile[t] = make_reco<HAS_T, HAS_D>(R, Fe, Te, Sig, D, jt + t, P, a5_10);
    __syncthreads();
    const bool self = jt < b1 && jt + cnt > b0;  // uniform: only these tiles can hold r = 0
    if (self) {
      for (int jj = 0; jj < cnt; ++jj) {
        Geo g;
        pair_geo<true>(tile[jj], xi, yi, zi, g);
        p3_acc<HAS_T, HAS_D>(tile[jj], g, A2_2, A2_23, A8, B16, acc);
        p2_acc(tile[jj], g, A24, A42, m);
      }
    } else {
      for (int jj = 0; jj < cnt; ++jj) {
        Geo g;
        pair_geo<false>(tile[jj], xi, yi, zi, g);
        p3_acc<HAS_T, HAS_D>(tile[jj], g, A2_2, A2_23, A8, B16, acc);
        p2_acc(tile[jj], g, A24, A42, m);
      }
    }
  }
  if (i >= n) return;
  const double v[11] = {m.pxx, m.pyy, m.pzz, m.qxy, m.qxz, m.qyz, m.t0, m.t1, m.t2, m.t3, m.t4};
  double e[5];
  p2_strain(v, 1.0, a2, e);
  double* o = out + (int64_t)blockIdx.y * 11 * n + 11 * (int64_t)i;
#pragma unroll
  for (int c = 0; c < 5; ++c) o[c] = e[c];
  o[5] = acc.ux;
  o[6] = acc.uy;
  o[7] = acc.uz;
  o[8] = acc.wx;
  o[9] = acc.wy;
  o[10] = acc.wz;
}

__global__ void k_p23_finish(const double* __restrict__ part, int split, int64_t n,
                             const double* __restrict__ v1s, const double* __restrict__ v2s,
                             const double* __restrict__ Fe, const double* __restrict__ Te,
                             const double* __restrict__ Sig, double* __restrict__ y,
                             double* __restrict__ V, double* __restrict__ W, double* __restrict__ S,
                             double inv_gamma, double mu_t, double mu_r, double slip_S) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int s = 0; s < split; ++s) {
    const double* p = part + (int64_t)s * 11 * n + 11 * i;
#pragma unroll
    for (int c = 0; c < 11; ++c) acc[c] += p[c];
  }
#pragma unroll
  for (int c = 0; c < 5; ++c) y[5 * i + c] = Sig[5 * i + c] * inv_gamma - acc[c];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    V[3 * i + c] = acc[5 + c] + mu_t * Fe[3 * i + c] - (v1s ? v1s[3 * i + c] : 0.0);
    W[3 * i + c] = acc[8 + c] + (Te ? mu_r * Te[3 * i + c] : 0.0);
  }
  if (S) {
#pragma unroll
    for (int c = 0; c < 5; ++c) S[5 * i + c] = Sig[5 * i + c] + (v2s ? slip_S * v2s[5 * i + c] : 0.0);
  }
}

// ------------------------------------------------------------------ flow at field points
// u(x) = sum_m of the source flows of sphere m at x - R_m (section III: force with its finite-size
// factor 1 + a^2/6 nabla^2, rotlet, flow stresslet with 1 + a^2/10 nabla^2, rank-3 trace mode);
// no finite-size operator acts at the field point:
//   F: P[(1/r + a^2/(3 r^3)) F + (1/r^3 - a^2/r^5)(x.F) x]      T: P (T x x)/r^3
//   Sigma: P[q x (-3/r^5 + 3a^2/r^7) - (6a^2/5) w / r^5]        d: (a^5/10)[3 (x.d) x/r^5 - d/r^3]
// with w = Sigma x, q = x.w. Per (field point, sphere) pair about 70 FLOP. One field point per
// thread, sphere records through LDS tiles, sphere chunks along grid.y summed in a fixed order.
template <int TJ, bool HAS_T, bool HAS_D>
__global__ void __launch_bounds__(kMaxBlock)
    k_flow(const double* __restrict__ X, int m, const double* __restrict__ R, const double* __restrict__ Fe,
           const double* __restrict__ Te, const double* __restrict__ Sig, const double* __restrict__ D,
           double* __restrict__ out, int n, int chunk, double P, double a2, double a5_10) {
  __shared__ RecO tile[TJ];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int ii = i < m ? i : m - 1;
  const double xi = X[3 * (int64_t)ii], yi = X[3 * (int64_t)ii + 1], zi = X[3 * (int64_t)ii + 2];
  const int j0 = blockIdx.y * chunk;
  const int j1 = min(n, j0 + chunk);
  const double A2_3 = a2 / 3.0, A6_5 = 1.2 * a2, A3 = 3.0 * a2;
  double ux = 0.0, uy = 0.0, uz = 0.0;
  for (int jt = j0; jt < j1; jt += TJ) {
    const int cnt = min(TJ, j1 - jt);
    __syncthreads();
    for (int t = threadIdx.x; t < cnt; t += blockDim.x)
      tile[t] = make_reco<HAS_T, HAS_D>(R, Fe, Te, Sig, D, jt + t, P, a5_10);
    __syncthreads();
#pragma unroll 2
    for (int jj = 0; jj < cnt; ++jj) {
      const RecO& sr = tile[jj];
      Geo g;
      pair_geo<true>(sr, xi, yi, zi, g);  // a field point on a centre gets no contribution from it
      const double ri7 = g.ri5 * g.ri2;
      const double xF = fma(g.dx, sr.fx, fma(g.dy, sr.fy, g.dz * sr.fz));
      double cx = xF * fma(-a2, g.ri5, g.ri3) + g.q * fma(A3, ri7, -3.0 * g.ri5);
      const double cF = fma(A2_3, g.ri3, g.ri);
      const double cw = -A6_5 * g.ri5;
      if (HAS_D) cx = fma(3.0 * g.ri5, g.dx * sr.dx + g.dy * sr.dy + g.dz * sr.dz, cx);
      ux = fma(cx, g.dx, fma(cF, sr.fx, fma(cw, g.wx, ux)));
      uy = fma(cx, g.dy, fma(cF, sr.fy, fma(cw, g.wy, uy)));
      uz = fma(cx, g.dz, fma(cF, sr.fz, fma(cw, g.wz, uz)));
      if (HAS_T) {
        ux = fma(g.ri3, sr.ty * g.dz - sr.tz * g.dy, ux);
        uy = fma(g.ri3, sr.tz * g.dx - sr.tx * g.dz, uy);
        uz = fma(g.ri3, sr.tx * g.dy - sr.ty * g.dx, uz);
      }
      if (HAS_D) {
        ux = fma(-g.ri3, sr.dx, ux);
        uy = fma(-g.ri3, sr.dy, uy);
        uz = fma(-g.ri3, sr.dz, uz);
      }
    }
  }
  if (i >= m) return;
  double* o = out + (int64_t)blockIdx.y * 3 * m + 3 * (int64_t)i;
  o[0] = ux;
  o[1] = uy;
  o[2] = uz;
}

__global__ void k_flow_finish(const double* __restrict__ part, int split, int64_t len, double* __restrict__ U) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= len) return;
  double acc = 0.0;
  for (int s = 0; s < split; ++s) acc += part[s * len + k];
  U[k] = acc;
}

// ------------------------------------------------------------------ overlap monitor
template <int TJ>
__global__ void __launch_bounds__(kMaxBlock)
    k_min_dist2(const double* __restrict__ R, int n, double* __restrict__ blockmin,
                const double* __restrict__ have, const GridHdr* __restrict__ hdr) {
  // nothing to do when the grid search already found a pair closer than one cell edge
  if (have[0] < hdr->h * hdr->h) return;
  __shared__ double tx[TJ], ty[TJ], tz[TJ];
  __shared__ double red[kMaxBlock];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int ii = i < n ? i : n - 1;
  const double xi = R[3 * ii], yi = R[3 * ii + 1], zi = R[3 * ii + 2];
  double best = INFINITY;
  for (int jt = 0; jt < n; jt += TJ) {
    const int cnt = min(TJ, n - jt);
    __syncthreads();
    for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
      tx[t] = R[3 * (jt + t)];
      ty[t] = R[3 * (jt + t) + 1];
      tz[t] = R[3 * (jt + t) + 2];
    }
    __syncthreads();
    for (int jj = 0; jj < cnt; ++jj) {
      const double dx = xi - tx[jj], dy = yi - ty[jj], dz = zi - tz[jj];
      const double r2 = dx * dx + dy * dy + dz * dz;
      if (jt + jj != ii) best = fmin(best, r2);
    }
  }
  red[threadIdx.x] = (i < n) ? best : INFINITY;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) blockmin[blockIdx.x] = red[0];
}

// Minimum over the 27 cells around each sphere's own (cell edge h): exact whenever some pair is
// closer than h, since every such pair lies in those cells. A crowded grid yields +inf here, which
// hands the search to the all-pairs scan.
__global__ void __launch_bounds__(256) k_min_grid(GridView G, double* __restrict__ blockmin) {
  if (grid_dense(G.hdr)) {  // crowded grid: leave it to the all-pairs scan
    if (threadIdx.x == 0) blockmin[blockIdx.x] = INFINITY;
    return;
  }
  __shared__ double red[256];
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  double best = INFINITY;
  if (k < G.n) {
    const GridHdr H = *G.hdr;
    const int i = G.perm[k];
    const double xi = G.Rs[4 * (int64_t)k], yi = G.Rs[4 * (int64_t)k + 1], zi = G.Rs[4 * (int64_t)k + 2];
    const int cx = grid_cell1(xi, H.lo[0], H.inv_h, H.g[0]);
    const int cy = grid_cell1(yi, H.lo[1], H.inv_h, H.g[1]);
    const int cz = grid_cell1(zi, H.lo[2], H.inv_h, H.g[2]);
    for (int z = max(cz - 1, 0); z <= min(cz + 1, H.g[2] - 1); ++z)
      for (int y = max(cy - 1, 0); y <= min(cy + 1, H.g[1] - 1); ++y)
        for (int x = max(cx - 1, 0); x <= min(cx + 1, H.g[0] - 1); ++x) {
          const int c = grid_linear(H, x, y, z);
          const int e = G.end[c];
          for (int k2 = G.start[c]; k2 < e; ++k2) {
            const double dx = xi - G.Rs[4 * (int64_t)k2], dy = yi - G.Rs[4 * (int64_t)k2 + 1],
                         dz = zi - G.Rs[4 * (int64_t)k2 + 2];
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (G.perm[k2] != i) best = fmin(best, r2);
          }
        }
  }
  red[threadIdx.x] = best;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) blockmin[blockIdx.x] = red[0];
}

// out[0] = min of the partials; with hdr: only when out[0] (the grid result) is not below h^2
__global__ void k_min_finish(const double* __restrict__ blockmin, int nb, double* __restrict__ out,
                             const GridHdr* __restrict__ hdr) {
  if (hdr && out[0] < hdr->h * hdr->h) return;
  __shared__ double red[kMaxBlock];
  double best = INFINITY;
  for (int k = threadIdx.x; k < nb; k += blockDim.x) best = fmin(best, blockmin[k]);
  red[threadIdx.x] = best;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

__global__ void k_count_nonfinite(const double* __restrict__ a, int64_t len, int* __restrict__ cnt) {
  __shared__ int red[kMaxBlock];
  int bad = 0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < len;
       k += (int64_t)gridDim.x * blockDim.x)
    bad += isfinite(a[k]) ? 0 : 1;
  red[threadIdx.x] = bad;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0 && red[0] != 0) atomicAdd(cnt, red[0]);
}

// rows of p [n x 3] whose length is not within tol of 1 (non-finite rows included)
__global__ void k_count_nonunit(const double* __restrict__ p, int64_t n, double tol, int* __restrict__ cnt) {
  __shared__ int red[kMaxBlock];
  int bad = 0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    const double x = p[3 * k], y = p[3 * k + 1], z = p[3 * k + 2];
    const double len = sqrt(x * x + y * y + z * z);
    bad += fabs(len - 1.0) <= tol ? 0 : 1;
  }
  red[threadIdx.x] = bad;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0 && red[0] != 0) atomicAdd(cnt, red[0]);
}

// ------------------------------------------------------------------ Krylov helpers
constexpr int kDotThreads = 256;

__device__ __forceinline__ double block_sum(double v, double* red) {
  // wavefront reduction (64 lanes), then across the 4 wavefronts of the block through LDS
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int k = 0; k < nw; ++k) s += red[k];
  }
  return s;
}

// part[k * gridDim.x + b] = sum over block b's range of V_k . w
__global__ void __launch_bounds__(kDotThreads)
    k_dots(const double* __restrict__ V, int64_t ld, const double* __restrict__ w, int64_t len,
           int64_t per, double* __restrict__ part) {
  __shared__ double red[kDotThreads / 64];
  const int k = blockIdx.y;
  const double* v = V + (int64_t)k * ld;
  const int64_t beg = (int64_t)blockIdx.x * per;
  const int64_t end = min(len, beg + per);
  double acc = 0.0;
  for (int64_t t = beg + threadIdx.x; t < end; t += blockDim.x) acc = fma(v[t], w[t], acc);
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) part[(int64_t)k * gridDim.x + blockIdx.x] = s;
}

__global__ void __launch_bounds__(kDotThreads)
    k_dots_finish(const double* __restrict__ part, int nb, double* __restrict__ out) {
  __shared__ double red[kDotThreads / 64];
  const int k = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) acc += part[(int64_t)k * nb + b];
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) out[k] = s;
}

__global__ void k_axpy_multi(const double* __restrict__ V, int64_t ld, int nv,
                             const double* __restrict__ h, double sign, double* __restrict__ w,
                             int64_t len) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= len) return;
  double acc = 0.0;
  for (int k = 0; k < nv; ++k) acc = fma(h[k], V[(int64_t)k * ld + t], acc);
  w[t] = fma(sign, acc, w[t]);
}

__global__ void k_scale_by(const double* __restrict__ x, const double* __restrict__ alpha, int inv,
                           double* __restrict__ y, int64_t len) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= len) return;
  const double al = alpha[0];
  if (inv) {
    y[t] = al > 0.0 ? x[t] / al : 0.0;
  } else {
    y[t] = al * x[t];
  }
}

__global__ void k_axpby(double a, const double* __restrict__ x, double b, double* __restrict__ y,
                        int64_t len) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= len) return;
  y[t] = a * x[t] + (b == 0.0 ? 0.0 : b * y[t]);
}

__global__ void k_copy(const double* __restrict__ x, double* __restrict__ y, int64_t len) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < len) y[t] = x[t];
}

__global__ void k_givens(double* __restrict__ H, int m, int k, const double* __restrict__ h1,
                         const double* __restrict__ h2, const double* __restrict__ nsq,
                         double* __restrict__ cs, double* __restrict__ sn, double* __restrict__ g,
                         double* __restrict__ status) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double* col = H + (int64_t)k * (m + 1);
  for (int i = 0; i <= k; ++i) col[i] = h1[i] + (h2 ? h2[i] : 0.0);
  const double hk1 = sqrt(fmax(nsq[0], 0.0));
  col[k + 1] = hk1;
  status[1] = hk1;
  for (int i = 0; i < k; ++i) {
    const double t = cs[i] * col[i] + sn[i] * col[i + 1];
    col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
    col[i] = t;
  }
  const double den = hypot(col[k], hk1);
  if (den > 0.0) {
    cs[k] = col[k] / den;
    sn[k] = hk1 / den;
  } else {
    cs[k] = 1.0;
    sn[k] = 0.0;
  }
  col[k] = den;
  col[k + 1] = 0.0;
  g[k + 1] = -sn[k] * g[k];
  g[k] = cs[k] * g[k];
  status[0] = fabs(g[k + 1]);
}

__global__ void k_backsolve(const double* __restrict__ H, int m, int k, const double* __restrict__ g,
                            double* __restrict__ y) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int i = k - 1; i >= 0; --i) {
    double s = g[i];
    for (int j = i + 1; j < k; ++j) s -= H[(int64_t)j * (m + 1) + i] * y[j];
    const double d = H[(int64_t)i * (m + 1) + i];
    y[i] = d != 0.0 ? s / d : 0.0;
  }
}

__global__ void k_init_g(const double* __restrict__ nsq, double* __restrict__ g, int m,
                         double* __restrict__ status) {
  const int t = threadIdx.x;
  const double beta = sqrt(fmax(nsq[0], 0.0));
  for (int k = t; k <= m; k += blockDim.x) g[k] = (k == 0) ? beta : 0.0;
  if (t == 0) {
    status[0] = beta;
    status[1] = beta;
  }
}

// ------------------------------------------------------------------ stepper
__global__ void k_trap_modes(const double* __restrict__ R, const double* __restrict__ p, double k,
                             double c0, double c1, double c2, double* __restrict__ Fe,
                             double* __restrict__ v1s, double* __restrict__ v2s,
                             double* __restrict__ v3t, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double px = p[3 * i], py = p[3 * i + 1], pz = p[3 * i + 2];
#pragma unroll
  for (int c = 0; c < 3; ++c) Fe[3 * i + c] = -k * R[3 * i + c];
  v1s[3 * i] = c0 * px;
  v1s[3 * i + 1] = c0 * py;
  v1s[3 * i + 2] = c0 * pz;
  // 3 (p p - I/3) in the 5-basis
  v2s[5 * i + 0] = c1 * 3.0 * RS2 * (px * px - py * py);
  v2s[5 * i + 1] = c1 * 3.0 * RS6 * (2.0 * pz * pz - px * px - py * py);
  v2s[5 * i + 2] = c1 * 6.0 * RS2 * px * py;
  v2s[5 * i + 3] = c1 * 6.0 * RS2 * px * pz;
  v2s[5 * i + 4] = c1 * 6.0 * RS2 * py * pz;
  v3t[3 * i] = c2 * px;
  v3t[3 * i + 1] = c2 * py;
  v3t[3 * i + 2] = c2 * pz;
}

__global__ void k_ab_update(double* __restrict__ R, double* __restrict__ p,
                            const double* __restrict__ V, const double* __restrict__ W,
                            double* __restrict__ Vprev, double* __restrict__ Pdprev, double dt,
                            int first, int order, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double px = p[3 * i], py = p[3 * i + 1], pz = p[3 * i + 2];
  const double wx = W[3 * i], wy = W[3 * i + 1], wz = W[3 * i + 2];
  const double pd[3] = {wy * pz - wz * py, wz * px - wx * pz, wx * py - wy * px};
  double q[3] = {px, py, pz};
  const bool euler = first || order == 1;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double v = V[3 * i + c];
    if (euler) {
      R[3 * i + c] += dt * v;
      q[c] += dt * pd[c];
    } else {
      R[3 * i + c] += dt * (1.5 * v - 0.5 * Vprev[3 * i + c]);
      q[c] += dt * (1.5 * pd[c] - 0.5 * Pdprev[3 * i + c]);
    }
    Vprev[3 * i + c] = v;
    Pdprev[3 * i + c] = pd[c];
  }
  const double inv = 1.0 / sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
#pragma unroll
  for (int c = 0; c < 3; ++c) p[3 * i + c] = q[c] * inv;
}

inline unsigned nblk(int64_t len, int b) { return (unsigned)((len + b - 1) / b); }

}  // namespace

// ------------------------------------------------------------------ launchers
Phys make_phys(double eta, double a, double c) {
  Phys p;
  p.eta = eta;
  p.a = a;
  p.P = 1.0 / (8.0 * M_PI * eta);
  p.a2 = a * a;
  p.a5_10 = a * a * a * a * a / 10.0;
  p.gamma = 20.0 / 3.0 * M_PI * eta * a * a * a;
  p.inv_gamma = 1.0 / p.gamma;
  p.mu_t = 1.0 / (6.0 * M_PI * eta * a);
  p.mu_r = 1.0 / (8.0 * M_PI * eta * a * a * a);
  p.slip_S = 8.0 / 3.0 * M_PI * eta * a * a * a;
  p.c_slip = c;
  return p;
}

void launch_p1(const double* R, const double* v2s, const double* v3t, const double* Fe,
               const double* Te, double* b, double* part, int64_t n, const Phys& ph, Tile t,
               hipStream_t s) {
  constexpr int TJ = 128;
  const int bs = tile_block(t);
  const int split = split_for(n, t, TJ);
  const int chunk = (int)((n + split - 1) / split);
  dim3 grid(nblk(n, bs), split);
  double* out = split > 1 ? part : b;
  const int direct = split > 1 ? 0 : 1;
#define MBS_P1(HT, HD)                                                                           \
  hipLaunchKernelGGL((k_p1<TJ, HT, HD>), grid, dim3(bs), 0, s, R, Fe, Te, v3t, v2s, out, (int)n, \
                     chunk, ph.P, ph.a2, ph.a5_10, ph.c_slip, direct)
  if (Te && v3t)
    MBS_P1(true, true);
  else if (Te)
    MBS_P1(true, false);
  else if (v3t)
    MBS_P1(false, true);
  else
    MBS_P1(false, false);
#undef MBS_P1
  if (split > 1)
    hipLaunchKernelGGL(k_p1_finish, dim3(nblk(5 * n, 256)), dim3(256), 0, s, part, v2s, b, 5 * n,
                       split, ph.c_slip);
}

void launch_p3(const double* R, const double* v1s, const double* v2s, const double* v3t,
               const double* Fe, const double* Te, const double* Sig, double* V, double* W,
               double* S, double* part, int64_t n, const Phys& ph, Tile t, hipStream_t s) {
  constexpr int TJ = 128;
  const int bs = tile_block(t);
  // the output pass always goes through the partial buffer (6 values per receiver and chunk)
  const int split = split_for(n, t, TJ);
  const int chunk = (int)((n + split - 1) / split);
  dim3 grid(nblk(n, bs), split);
#define MBS_P3(HT, HD)                                                                          \
  hipLaunchKernelGGL((k_p3<TJ, HT, HD>), grid, dim3(bs), 0, s, R, Fe, Te, Sig, v3t, part, (int)n, \
                     chunk, ph.P, ph.a2, ph.a5_10)
  if (Te && v3t)
    MBS_P3(true, true);
  else if (Te)
    MBS_P3(true, false);
  else if (v3t)
    MBS_P3(false, true);
  else
    MBS_P3(false, false);
#undef MBS_P3
  hipLaunchKernelGGL(k_p3_finish, dim3(nblk(n, 256)), dim3(256), 0, s, part, split, n, v1s, v2s, Fe,
                     Te, Sig, V, W, S, ph.mu_t, ph.mu_r, ph.slip_S);
}

void launch_p23(const double* R, const double* v1s, const double* v2s, const double* v3t,
                const double* Fe, const double* Te, const double* Sig, double* y, double* V, double* W,
                double* S, double* part, int64_t n, const Phys& ph, Tile t, hipStream_t s) {
  constexpr int TJ = 128;
  const int bs = tile_block(t);
  const int split = split_for(n, t, TJ);
  const int chunk = (int)((n + split - 1) / split);
  dim3 grid(nblk(n, bs), split);
#define MBS_P23(HT, HD)                                                                          \
  hipLaunchKernelGGL((k_p23<TJ, HT, HD>), grid, dim3(bs), 0, s, R, Fe, Te, Sig, v3t, part, (int)n, \
                     chunk, ph.P, ph.a2, ph.a5_10)
  if (Te && v3t)
    MBS_P23(true, true);
  else if (Te)
    MBS_P23(true, false);
  else if (v3t)
    MBS_P23(false, true);
  else
    MBS_P23(false, false);
#undef MBS_P23
  hipLaunchKernelGGL(k_p23_finish, dim3(nblk(n, 256)), dim3(256), 0, s, part, split, n, v1s, v2s, Fe, Te,
                     Sig, y, V, W, S, ph.inv_gamma, ph.mu_t, ph.mu_r, ph.slip_S);
}

int flow_split(int64_t m, int64_t n, Tile t) {
  // enough workgroups to fill the GPU: field-point tiles times sphere chunks of >= 128 spheres
  const int64_t ntile = (m + tile_block(t) - 1) / tile_block(t);
  const int64_t target = t.wgs > 0 ? t.wgs : 2048;
  const int64_t s = (target + ntile - 1) / ntile;
  return (int)std::min<int64_t>(std::max<int64_t>(s, 1), std::max<int64_t>(1, (n + 127) / 128));
}

void launch_flow(const double* X, int64_t m, const double* R, const double* Fe, const double* Te,
                 const double* Sig, const double* v3t, double* U, double* part, int64_t n, const Phys& ph,
                 Tile t, hipStream_t s) {
  constexpr int TJ = 128;
  const int bs = tile_block(t);
  const int split = flow_split(m, n, t);
  const int chunk = (int)((n + split - 1) / split);
  dim3 grid(nblk(m, bs), split);
#define MBS_FLOW(HT, HD)                                                                               \
  hipLaunchKernelGGL((k_flow<TJ, HT, HD>), grid, dim3(bs), 0, s, X, (int)m, R, Fe, Te, Sig, v3t, part, (int)n, \
                     chunk, ph.P, ph.a2, ph.a5_10)
  if (Te && v3t)
    MBS_FLOW(true, true);
  else if (Te)
    MBS_FLOW(true, false);
  else if (v3t)
    MBS_FLOW(false, true);
  else
    MBS_FLOW(false, false);
#undef MBS_FLOW
  hipLaunchKernelGGL(k_flow_finish, dim3(nblk(3 * m, 256)), dim3(256), 0, s, part, split, 3 * m, U);
}

void launch_min_dist2(const GridView& g, const double* R, int64_t n, double* out, double* scratch,
                      hipStream_t s) {
  const unsigned nb = nblk(n, 256);
  // grid search first; the all-pairs scan runs (and replaces the result) only if it found no pair
  // closer than one cell edge
  hipLaunchKernelGGL(k_min_grid, dim3(nb), dim3(256), 0, s, g, scratch);
  hipLaunchKernelGGL(k_min_finish, dim3(1), dim3(256), 0, s, scratch, (int)nb, out, nullptr);
  hipLaunchKernelGGL(k_min_dist2<256>, dim3(nb), dim3(256), 0, s, R, (int)n, scratch, out, g.hdr);
  hipLaunchKernelGGL(k_min_finish, dim3(1), dim3(256), 0, s, scratch, (int)nb, out, g.hdr);
}

namespace {
// x = D^{-1} b for the rank <= 3 unknowns (20 per sphere): the stresslet rows scaled by gamma
__global__ void k_rank3_diag(const double* __restrict__ b, int64_t len, double gamma, double* __restrict__ x) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= len) return;
  x[k] = (k % 20) < 5 ? gamma * b[k] : b[k];
}
}  // namespace

void launch_rank3_diag(const double* b, int64_t n, double gamma, double* x, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_rank3_diag, dim3(nblk(20 * n, 256)), dim3(256), 0, s, b, 20 * n, gamma, x);
}

void launch_count_nonfinite(const double* a, int64_t len, int* cnt, hipStream_t s) {
  if (len <= 0) return;
  const unsigned nb = std::min<unsigned>(nblk(len, 256), 1024u);
  hipLaunchKernelGGL(k_count_nonfinite, dim3(nb), dim3(256), 0, s, a, len, cnt);
}

void launch_count_nonunit(const double* p, int64_t n, double tol, int* cnt, hipStream_t s) {
  if (n <= 0) return;
  const unsigned nb = std::min<unsigned>(nblk(n, 256), 1024u);
  hipLaunchKernelGGL(k_count_nonunit, dim3(nb), dim3(256), 0, s, p, n, tol, cnt);
}

int dot_blocks(int64_t len) {
  int64_t b = (len + 2047) / 2048;
  return (int)std::min<int64_t>(std::max<int64_t>(b, 1), 256);
}

void launch_dots(const double* V, int64_t ld, int nv, const double* w, int64_t len, double* part,
                 double* out, hipStream_t s) {
  const int nb = dot_blocks(len);
  const int64_t per = (len + nb - 1) / nb;
  hipLaunchKernelGGL(k_dots, dim3(nb, nv), dim3(kDotThreads), 0, s, V, ld, w, len, per, part);
  hipLaunchKernelGGL(k_dots_finish, dim3(nv), dim3(kDotThreads), 0, s, part, nb, out);
}

void launch_axpy_multi(const double* V, int64_t ld, int nv, const double* h, double sign, double* w,
                       int64_t len, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy_multi, dim3(nblk(len, 256)), dim3(256), 0, s, V, ld, nv, h, sign, w,
                     len);
}

void launch_scale_by(const double* x, const double* alpha, int inv, double* y, int64_t len,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_scale_by, dim3(nblk(len, 256)), dim3(256), 0, s, x, alpha, inv, y, len);
}

void launch_axpby(double a, const double* x, double b, double* y, int64_t len, hipStream_t s) {
  hipLaunchKernelGGL(k_axpby, dim3(nblk(len, 256)), dim3(256), 0, s, a, x, b, y, len);
}

namespace {
// dst[k][c] = src[perm[k]][c] and the reverse; perm is a permutation of 0..n-1
__global__ void k_gather_rows(const double* __restrict__ src, int width, const int32_t* __restrict__ perm,
                              int64_t n, double* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * width) return;
  const int64_t k = t / width;
  dst[t] = src[(int64_t)perm[k] * width + (t - k * width)];
}
__global__ void k_scatter_rows(const double* __restrict__ src, int width, const int32_t* __restrict__ perm,
                               int64_t n, double* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * width) return;
  const int64_t k = t / width;
  dst[(int64_t)perm[k] * width + (t - k * width)] = src[t];
}
}  // namespace

void launch_gather_rows(const double* src, int width, const int32_t* perm, int64_t n, double* dst, hipStream_t s) {
  const int64_t len = n * width;
  hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, s, src, width, perm, n, dst);
}
void launch_scatter_rows(const double* src, int width, const int32_t* perm, int64_t n, double* dst, hipStream_t s) {
  const int64_t len = n * width;
  hipLaunchKernelGGL(k_scatter_rows, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, s, src, width, perm, n, dst);
}

void launch_copy(const double* x, double* y, int64_t len, hipStream_t s) {
  hipLaunchKernelGGL(k_copy, dim3(nblk(len, 256)), dim3(256), 0, s, x, y, len);
}

void launch_givens(double* H, int m, int k, const double* h1, const double* h2, const double* nsq,
                   double* cs, double* sn, double* g, double* status, hipStream_t s) {
  hipLaunchKernelGGL(k_givens, dim3(1), dim3(64), 0, s, H, m, k, h1, h2, nsq, cs, sn, g, status);
}

void launch_backsolve(const double* H, int m, int k, const double* g, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_backsolve, dim3(1), dim3(64), 0, s, H, m, k, g, y);
}

void launch_init_g(const double* nsq, double* g, int m, double* status, hipStream_t s) {
  hipLaunchKernelGGL(k_init_g, dim3(1), dim3(64), 0, s, nsq, g, m, status);
}

void launch_trap_modes(const double* R, const double* p, double k, double c0, double c1, double c2,
                       double* Fe, double* v1s, double* v2s, double* v3t, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_trap_modes, dim3(nblk(n, 256)), dim3(256), 0, s, R, p, k, c0, c1, c2, Fe, v1s,
                     v2s, v3t, n);
}

void launch_ab_update(double* R, double* p, const double* V, const double* W, double* Vprev,
                      double* Pdprev, double dt, int first, int order, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_ab_update, dim3(nblk(n, 256)), dim3(256), 0, s, R, p, V, W, Vprev, Pdprev, dt,
                     first, order, n);
}

}  // namespace mbs
