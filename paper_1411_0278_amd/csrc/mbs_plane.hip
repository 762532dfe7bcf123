// Spheres above a stress-free plane (gfx950): the image passes.
//
// The fluid fills the half space z > z_w above a flat plane on which it slips freely (zero normal
// velocity and zero tangential stress). The Green's function of that half space is the free-space
// one plus its mirror image, so every sphere m acts on the others through its own flow and, on
// every sphere (itself included), through the flow of its mirror image: centre reflected in the
// plane, with M = diag(1, 1, -1) the source coefficients transformed as
//     force F* = M F,   torque T* = -M T (axial),   stresslet Sigma* = M Sigma M,   d* = M d,
// and the receiver's Galerkin projections (the finite-size operators included) act on the image
// flows as on any incident Stokes flow. The free-space passes are unchanged; these passes add the
// images: the strain E of their forces, torques and rank-3 trace modes (the right-hand side), their
// velocity and rotation U, W (the outputs) and their flow at field points. The strain of the images'
// stresslets (the operator's image part, in the solve's precision) is a mode of the operator kernel. Every sphere lies at least a above the plane (checked by the caller), so no image
// comes closer than 2a to a receiver.
//
// A plane no-slip wall (zero velocity on z = z_w) has Blake's Green's function instead: the
// free-space one plus an image part at the mirror point that depends on the source's height as well
// as on the separation (a Stokeslet, a Stokes doublet and a source doublet there). Its blocks take
// each source sphere's surface moments against that image part in the source point; the per-pair
// arithmetic of every target (operator, right-hand side, outputs, flow) is generated from the
// image system into mbs_wall_gen.h and evaluated here in binary64.
//
// Layout: one receiver per thread, image records built from the caller's arrays into LDS tiles, the
// sources split into grid.y chunks whose partial sums a finishing kernel adds into the caller's
// output in a fixed order.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "mbs_device.h"
#include "mbs_internal.h"
#include "mbs_pair.h"
#include "mbs_wall_gen.h"

namespace mbs {
namespace {

constexpr int kImTJ = 64;    // image records per LDS tile
constexpr int kImBlk = 128;  // receivers per workgroup

// image record of sphere j: mirrored centre, P-scaled F*, T*, Cartesian Sigma*, (a^5/10)-scaled d*
// (absent sources are zero)
__device__ __forceinline__ RecO make_image(const double* __restrict__ R, const double* __restrict__ Fe,
                                           const double* __restrict__ Te, const double* __restrict__ Sig,
                                           const double* __restrict__ D, int j, double P, double a5_10,
                                           double zw2) {
  RecO r;
  r.x = R[3 * (int64_t)j];
  r.y = R[3 * (int64_t)j + 1];
  r.z = zw2 - R[3 * (int64_t)j + 2];
  r.fx = Fe ? P * Fe[3 * (int64_t)j] : 0.0;
  r.fy = Fe ? P * Fe[3 * (int64_t)j + 1] : 0.0;
  r.fz = Fe ? -P * Fe[3 * (int64_t)j + 2] : 0.0;
  r.tx = Te ? -P * Te[3 * (int64_t)j] : 0.0;
  r.ty = Te ? -P * Te[3 * (int64_t)j + 1] : 0.0;
  r.tz = Te ? P * Te[3 * (int64_t)j + 2] : 0.0;
  if (Sig) {
    double sxx, syy, sxy, sxz, syz;
    basis_to_cart(Sig + 5 * (int64_t)j, sxx, syy, sxy, sxz, syz);
    r.sxx = P * sxx;
    r.syy = P * syy;
    r.sxy = P * sxy;
    r.sxz = -P * sxz;
    r.syz = -P * syz;
  } else {
    r.sxx = r.syy = r.sxy = r.sxz = r.syz = 0.0;
  }
  r.dx = D ? a5_10 * D[3 * (int64_t)j] : 0.0;
  r.dy = D ? a5_10 * D[3 * (int64_t)j + 1] : 0.0;
  r.dz = D ? -a5_10 * D[3 * (int64_t)j + 2] : 0.0;
  r.pad = 0.0;
  return r;
}

// strain moments of the force, torque and trace-mode flows (the right-hand-side pass's closed form:
// v = x (x.F) r^-5 (8a^2/r^2 - 3) - 3.2 a^2 F r^-5 - 3 (T x x) r^-5 + 6 d r^-5 - 15 (x.d) x r^-7,
// moments sum x_i v_j) from the pair geometry
__device__ __forceinline__ void image_fixed_strain(const RecO& s, const Geo& g, double A8, double B16, Mom6& m) {
  const double dx = g.dx, dy = g.dy, dz = g.dz;
  const double ri5 = g.ri5, ri7 = g.ri5 * g.ri2;
  const double xF = fma(dx, s.fx, fma(dy, s.fy, dz * s.fz));
  const double alpha = xF * ri5 * fma(A8, g.ri2, -3.0);
  const double beta = B16 * ri5;
  double vx = fma(beta, s.fx, alpha * dx);
  double vy = fma(beta, s.fy, alpha * dy);
  double vz = fma(beta, s.fz, alpha * dz);
  const double m3 = -3.0 * ri5;
  vx = fma(m3, s.ty * dz - s.tz * dy, vx);
  vy = fma(m3, s.tz * dx - s.tx * dz, vy);
  vz = fma(m3, s.tx * dy - s.ty * dx, vz);
  const double xd = -15.0 * ri7 * (dx * s.dx + dy * s.dy + dz * s.dz);
  const double six = 6.0 * ri5;
  vx = fma(six, s.dx, fma(xd, dx, vx));
  vy = fma(six, s.dy, fma(xd, dy, vy));
  vz = fma(six, s.dz, fma(xd, dz, vz));
  m.pxx = fma(dx, vx, m.pxx);
  m.pyy = fma(dy, vy, m.pyy);
  m.pzz = fma(dz, vz, m.pzz);
  m.qxy = fma(dx, vy, fma(dy, vx, m.qxy));
  m.qxz = fma(dx, vz, fma(dz, vx, m.qxz));
  m.qyz = fma(dy, vz, fma(dz, vy, m.qyz));
}

// flow of one source record at separation g (no finite-size operator at the field point):
// F: (1/r + a^2/(3 r^3)) F + (1/r^3 - a^2/r^5)(x.F) x; T: (T x x)/r^3;
// Sigma: q x (3a^2/r^7 - 3/r^5) - (6a^2/5) w/r^5; d: 3 (x.d) x/r^5 - d/r^3 (records pre-scaled)
__device__ __forceinline__ void image_flow(const RecO& s, const Geo& g, double a2, double& ux, double& uy,
                                           double& uz) {
  const double ri7 = g.ri5 * g.ri2;
  const double xF = fma(g.dx, s.fx, fma(g.dy, s.fy, g.dz * s.fz));
  double cx = xF * fma(-a2, g.ri5, g.ri3) + g.q * fma(3.0 * a2, ri7, -3.0 * g.ri5);
  cx = fma(3.0 * g.ri5, g.dx * s.dx + g.dy * s.dy + g.dz * s.dz, cx);
  const double cF = fma(a2 / 3.0, g.ri3, g.ri);
  const double cw = -1.2 * a2 * g.ri5;
  ux = fma(cx, g.dx, fma(cF, s.fx, fma(cw, g.wx, ux)));
  uy = fma(cx, g.dy, fma(cF, s.fy, fma(cw, g.wy, uy)));
  uz = fma(cx, g.dz, fma(cF, s.fz, fma(cw, g.wz, uz)));
  ux = fma(g.ri3, s.ty * g.dz - s.tz * g.dy, fma(-g.ri3, s.dx, ux));
  uy = fma(g.ri3, s.tz * g.dx - s.tx * g.dz, fma(-g.ri3, s.dy, uy));
  uz = fma(g.ri3, s.tx * g.dy - s.ty * g.dx, fma(-g.ri3, s.dz, uz));
}

enum { kImOp = 0, kImRhs = 1, kImOut = 2, kImFlow = 3 };
constexpr int im_width(int t) { return t == kImOut ? 6 : (t == kImFlow ? 3 : 5); }

// receivers X [m x 3] (the spheres, or field points for kImFlow) against the images of the n spheres
template <int TGT>
__global__ void __launch_bounds__(kImBlk)
    k_image(const double* __restrict__ X, int m, const double* __restrict__ R, int n, const double* __restrict__ Fe,
            const double* __restrict__ Te, const double* __restrict__ Sig, const double* __restrict__ D, int chunk,
            double P, double a2, double a5_10, double zw2, double* __restrict__ part) {
  __shared__ RecO tile[kImTJ];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int ii = i < m ? i : m - 1;
  const double xi = X[3 * (int64_t)ii], yi = X[3 * (int64_t)ii + 1], zi = X[3 * (int64_t)ii + 2];
  const int j0 = blockIdx.y * chunk;
  const int j1 = min(n, j0 + chunk);
  Mom6 mf;
  UW uw;
  double ux = 0.0, uy = 0.0, uz = 0.0;
  for (int jt = j0; jt < j1; jt += kImTJ) {
    const int cnt = min(kImTJ, j1 - jt);
    __syncthreads();
    for (int t = threadIdx.x; t < cnt; t += blockDim.x)
      tile[t] = make_image(R, Fe, Te, TGT == kImRhs ? nullptr : Sig, D, jt + t, P, a5_10, zw2);
    __syncthreads();
    for (int jj = 0; jj < cnt; ++jj) {
      const RecO& s = tile[jj];
      Geo g;
      pair_geo<false>(s, xi, yi, zi, g);  // an image is never closer than 2a to a sphere
      if (TGT == kImRhs) image_fixed_strain(s, g, 8.0 * a2, -3.2 * a2, mf);
      if (TGT == kImOut) p3_acc<true, true>(s, g, 2.0 * a2, 2.0 * a2 / 3.0, 8.0 * a2, -3.2 * a2, uw);
      if (TGT == kImFlow) image_flow(s, g, a2, ux, uy, uz);
    }
  }
  if (i >= m) return;
  double* o = part + ((int64_t)blockIdx.y * m + i) * im_width(TGT);
  if (TGT == kImRhs) mom6_to_basis(mf, o);
  if (TGT == kImOut) {
    o[0] = uw.ux;
    o[1] = uw.uy;
    o[2] = uw.uz;
    o[3] = uw.wx;
    o[4] = uw.wy;
    o[5] = uw.wz;
  }
  if (TGT == kImFlow) {
    o[0] = ux;
    o[1] = uy;
    o[2] = uz;
  }
}

// source record of the no-slip wall: centre, and the coefficients pre-scaled as the generated
// arithmetic takes them (f = P F, t = P T, s = P Sigma in the 5-basis, q = (a^5/20) d; absent = 0)
struct alignas(16) RecW {
  double x, y, z, f[3], t[3], s[5], q[3], pad;
};

__device__ __forceinline__ RecW make_wall(const double* __restrict__ R, const double* __restrict__ Fe,
                                          const double* __restrict__ Te, const double* __restrict__ Sig,
                                          const double* __restrict__ D, int j, double P, double a5_20) {
  RecW r;
  r.x = R[3 * (int64_t)j];
  r.y = R[3 * (int64_t)j + 1];
  r.z = R[3 * (int64_t)j + 2];
  for (int c = 0; c < 3; ++c) {
    r.f[c] = Fe ? P * Fe[3 * (int64_t)j + c] : 0.0;
    r.t[c] = Te ? P * Te[3 * (int64_t)j + c] : 0.0;
    r.q[c] = D ? a5_20 * D[3 * (int64_t)j + c] : 0.0;
  }
  for (int c = 0; c < 5; ++c) r.s[c] = Sig ? P * Sig[5 * (int64_t)j + c] : 0.0;
  r.pad = 0.0;
  return r;
}

// receivers X [m x 3] against the wall images of the n spheres: kImOp the strain of the stresslets
// Sig (the operator), kImRhs the strain of Fe, Te, D, kImOut U and W of all four, kImFlow the flow
// of all four at field points
template <int TGT>
__global__ void __launch_bounds__(kImBlk)
    k_wall(const double* __restrict__ X, int m, const double* __restrict__ R, int n, const double* __restrict__ Fe,
           const double* __restrict__ Te, const double* __restrict__ Sig, const double* __restrict__ D, int chunk,
           double P, double a2, double a5_20, double zw, double* __restrict__ part) {
  __shared__ RecW tile[kImTJ];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int ii = i < m ? i : m - 1;
  const double xi = X[3 * (int64_t)ii], yi = X[3 * (int64_t)ii + 1], zi = X[3 * (int64_t)ii + 2];
  const int j0 = blockIdx.y * chunk;
  const int j1 = min(n, j0 + chunk);
  constexpr int W = im_width(TGT);
  double acc[W];
#pragma unroll
  for (int c = 0; c < W; ++c) acc[c] = 0.0;
  for (int jt = j0; jt < j1; jt += kImTJ) {
    const int cnt = min(kImTJ, j1 - jt);
    __syncthreads();
    for (int t = threadIdx.x; t < cnt; t += blockDim.x)
      tile[t] = make_wall(R, TGT == kImOp ? nullptr : Fe, TGT == kImOp ? nullptr : Te,
                          TGT == kImRhs ? nullptr : Sig, TGT == kImOp ? nullptr : D, jt + t, P, a5_20);
    __syncthreads();
    for (int jj = 0; jj < cnt; ++jj) {
      const RecW& s = tile[jj];
      // separation from the mirror point and the source's height (at least a above the wall, so
      // |R| >= 2a for a sphere and every image)
      const double h = s.z - zw;
      const double R1 = xi - s.x, R2 = yi - s.y, R3 = zi - zw + h;
      const double ri = 1.0 / sqrt(fma(R1, R1, fma(R2, R2, R3 * R3)));
      if (TGT == kImOp) wall_strain_s(R1, R2, R3, h, ri, a2, s.s, acc);
      if (TGT == kImRhs) wall_strain_ftq(R1, R2, R3, h, ri, a2, s.f, s.t, s.q, acc);
      if (TGT == kImOut) wall_motion_ftsq(R1, R2, R3, h, ri, a2, s.f, s.t, s.s, s.q, acc, acc + 3);
      if (TGT == kImFlow) wall_flow_ftsq(R1, R2, R3, h, ri, a2, s.f, s.t, s.s, s.q, acc);
    }
  }
  if (i >= m) return;
  double* o = part + ((int64_t)blockIdx.y * m + i) * W;
#pragma unroll
  for (int c = 0; c < W; ++c) o[c] = acc[c];
}

// out += sign * (sum of the split partials, in order); widths 3 and 5 go to `out` [m x w], width 6 to
// out [m x 3] (velocity) and out2 [m x 3] (rotation)
template <int TGT>
__global__ void k_image_finish(const double* __restrict__ part, int split, int m, double sign,
                               double* __restrict__ out, double* __restrict__ out2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  constexpr int W = im_width(TGT);
  double acc[W];
  for (int c = 0; c < W; ++c) acc[c] = 0.0;
  for (int s = 0; s < split; ++s)
    for (int c = 0; c < W; ++c) acc[c] += part[((int64_t)s * m + i) * W + c];
  if (TGT == kImOut) {
    for (int c = 0; c < 3; ++c) {
      out[3 * (int64_t)i + c] += sign * acc[c];
      out2[3 * (int64_t)i + c] += sign * acc[3 + c];
    }
  } else {
    for (int c = 0; c < W; ++c) out[(int64_t)W * i + c] += sign * acc[c];
  }
}

// z < zmin or non-finite -> counted
__global__ void k_count_below(const double* __restrict__ R, int64_t n, double zmin, int* __restrict__ cnt) {
  int c = 0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const double z = R[3 * k + 2];
    c += !(z >= zmin);
  }
  for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(cnt, c);
}

// out[0] = min over the spheres of (z - zw); a non-finite height counts as -infinity (one workgroup)
__global__ void __launch_bounds__(256) k_min_height(const double* __restrict__ R, int64_t n, double zw,
                                                    double* __restrict__ out) {
  __shared__ double lo[256];
  double m = INFINITY;
  for (int64_t k = threadIdx.x; k < n; k += blockDim.x) {
    const double h = R[3 * k + 2] - zw;
    m = isfinite(h) ? fmin(m, h) : -INFINITY;
  }
  lo[threadIdx.x] = m;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) lo[threadIdx.x] = fmin(lo[threadIdx.x], lo[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = lo[0];
}

inline unsigned nblk_im(int64_t len, int b) { return (unsigned)((len + b - 1) / b); }

template <int TGT>
void image_launch(int kind, const double* X, int64_t m, const double* R, int64_t n, const double* Fe,
                  const double* Te, const double* Sig, const double* D, double sign, double* out, double* out2,
                  double* part, const Phys& ph, double plane_z, hipStream_t s) {
  const int split = image_split(m, n);
  const int chunk = (int)((n + split - 1) / split);
  const dim3 grid(nblk_im(m, kImBlk), split);
  if (kind == 2)
    hipLaunchKernelGGL(k_wall<TGT>, grid, dim3(kImBlk), 0, s, X, (int)m, R, (int)n, Fe, Te, Sig, D, chunk, ph.P,
                       ph.a2, 0.5 * ph.a5_10, plane_z, part);
  else if constexpr (TGT != kImOp)
    hipLaunchKernelGGL(k_image<TGT>, grid, dim3(kImBlk), 0, s, X, (int)m, R, (int)n, Fe, Te, Sig, D, chunk, ph.P,
                       ph.a2, ph.a5_10, 2.0 * plane_z, part);
  hipLaunchKernelGGL(k_image_finish<TGT>, dim3(nblk_im(m, 256)), dim3(256), 0, s, part, split, (int)m, sign, out,
                     out2);
}

}  // namespace

int image_split(int64_t m, int64_t n) {
  const int64_t blocks = (m + kImBlk - 1) / kImBlk;
  int64_t s = (1024 + blocks - 1) / blocks;
  return (int)std::min<int64_t>(std::max<int64_t>(s, 1), std::max<int64_t>(1, (n + kImTJ - 1) / kImTJ));
}

int64_t image_part_elems(int64_t m, int64_t n) { return (int64_t)image_split(m, n) * 6 * m; }

void launch_wall_op(const double* R, const double* x, double* y, double* part, int64_t n, const Phys& ph,
                    double plane_z, hipStream_t s) {
  if (n <= 0) return;
  image_launch<kImOp>(2, R, n, R, n, nullptr, nullptr, x, nullptr, -1.0, y, nullptr, part, ph, plane_z, s);
}

void launch_image_rhs(int kind, const double* R, const double* Fe, const double* Te, const double* v3t, double* b,
                      double* part, int64_t n, const Phys& ph, double plane_z, hipStream_t s) {
  if (n <= 0 || (!Fe && !Te && !v3t)) return;
  image_launch<kImRhs>(kind, R, n, R, n, Fe, Te, nullptr, v3t, 1.0, b, nullptr, part, ph, plane_z, s);
}

void launch_image_out(int kind, const double* R, const double* Fe, const double* Te, const double* Sig,
                      const double* v3t, double* V, double* W, double* part, int64_t n, const Phys& ph, double plane_z,
                      hipStream_t s) {
  if (n <= 0) return;
  image_launch<kImOut>(kind, R, n, R, n, Fe, Te, Sig, v3t, 1.0, V, W, part, ph, plane_z, s);
}

void launch_image_flow(int kind, const double* X, int64_t m, const double* R, int64_t n, const double* Fe,
                       const double* Te, const double* Sig, const double* v3t, double* U, double* part, const Phys& ph,
                       double plane_z, hipStream_t s) {
  if (m <= 0 || n <= 0) return;
  image_launch<kImFlow>(kind, X, m, R, n, Fe, Te, Sig, v3t, 1.0, U, nullptr, part, ph, plane_z, s);
}

void launch_min_height(const double* R, int64_t n, double plane_z, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_min_height, dim3(1), dim3(256), 0, s, R, n, plane_z, out);
}

void launch_count_below(const double* R, int64_t n, double zmin, int* cnt, hipStream_t s) {
  if (n <= 0) return;
  const unsigned nb = std::min<unsigned>(nblk_im(n, 256), 1024u);
  hipLaunchKernelGGL(k_count_below, dim3(nb), dim3(256), 0, s, R, n, zmin, cnt);
}

}  // namespace mbs
