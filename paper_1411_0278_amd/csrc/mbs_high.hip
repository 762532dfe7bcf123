// Higher slip modes of the minimal truncation as fixed sources (gfx950): the septlet mode gamma
// and the vortlet mode psi (irreducible parts of the quadratic surface-velocity coefficient) and
// the spinlet mode lambda (rank-3 part of the cubic one), section IV. Like the rank-3 trace mode d,
// each keeps its one-body traction, so a sphere m with these slips adds a known flow; it moves no
// lone sphere (the surface means of its slip and of n x slip vanish) and acts on the others through
// that flow. With n the unit normal of sphere m, the slip fields are
//
//   gamma: v = (a^2/2) gamma : n n      psi: v = -(a^2/3) n x (psi . n)      lambda: v = -(a^3/8) n x (lambda : n n)
//
// and their exterior flows at x = R - R_m (the decaying Stokes flows with these surface values;
// g = gamma : x x, Q = g . x, w = psi . x, v = lambda : x x):
//
//   gamma:  u = (7a^5/48) F^2 [grad grad G] : gamma  (F^2 = 1 + a^2/14 nabla^2)
//             = -(7a^5/16) g/r^5 + (35a^5/16) Q x/r^7 + (15a^7/16) g/r^7 - (35a^7/16) Q x/r^9
//   psi:    u = -(a^5/3) (x cross w) / r^5        lambda: u = -(a^7/8) (x cross v) / r^7
//
// The gamma flow carries the pressure (35 eta a^5/8) Q/r^7, the other two none (they are
// harmonic). Projected on a receiving sphere (section III, Faxen form): U = F^0 u, W = curl u / 2,
// E = sym grad F^1 u, which with N = gamma . x (or lambda . x) give
//
//   gamma:  U = (-7a^5/16 r^-5 + 25a^7/8 r^-7) g + (35a^5/16 r^-7 - 175a^7/24 r^-9) Q x
//           W = -(35a^5/16) (x cross g) / r^7
//           E = c1 N + c2 sym(g x) + c3 Q x x,  c1 = -7a^5/8 r^-5 + 9a^7/2 r^-7,
//               c2 = 35a^5/4 r^-7 - 63a^7/2 r^-9,  c3 = -245a^5/16 r^-9 + 189a^7/4 r^-11
//   psi:    U = u,  W = c (w/r^5 - (5/2) (x.w) x/r^7),  E = c [sym(M)/r^5 - 5 sym((x cross w) x)/r^7],
//           c = -a^5/3,  M_ij = (x cross psi_.j)_i
//   lambda: U = u,  W = c (3/2 v/r^7 - 7/2 Q x/r^9),  E = c [2 sym(M)/r^7 - 7 sym((x cross v) x)/r^9],
//           c = -a^7/8,  M_ij = (x cross N_.j)_i,  Q = v . x
//
// (traceless parts; the 5-basis projection drops the trace). One all-pairs pass per target: the
// strain (right-hand side of the stresslet rows), the rigid-body velocities, or the flow at field
// points. Layout as the other passes: one receiver per thread, source records through LDS tiles,
// source chunks along grid.y summed in a fixed order by a finishing kernel that adds into the
// caller's array.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "mbs_device.h"
#include "mbs_internal.h"

namespace mbs {

namespace {

constexpr int kHiTJ = 64;  // source records per LDS tile (224 B each)

// Source record: centre, symmetric traceless gamma and lambda (10 components: xxx xxy xxz xyy xyz
// xzz yyy yyz yzz zzz), Cartesian psi (xx yy xy xz yz; zz = -xx - yy).
struct alignas(16) RecH {
  double x, y, z;
  double g[10];
  double p[5];
  double l[10];
};

struct HiCoef {
  double gA, gB, gCu, gDu, gCf, gDf, gW, e1a, e1b, e2a, e2b, e3a, e3b, cpsi, clam;
};

// symmetric traceless part of a symmetric rank-3 tensor given by its 10 components
__device__ __forceinline__ void stf3(const double* __restrict__ c, double* t) {
  const double tx = c[0] + c[3] + c[5], ty = c[1] + c[6] + c[8], tz = c[2] + c[7] + c[9];
  t[0] = c[0] - 0.6 * tx;
  t[1] = c[1] - 0.2 * ty;
  t[2] = c[2] - 0.2 * tz;
  t[3] = c[3] - 0.2 * tx;
  t[4] = c[4];
  t[5] = c[5] - 0.2 * tx;
  t[6] = c[6] - 0.6 * ty;
  t[7] = c[7] - 0.2 * tz;
  t[8] = c[8] - 0.2 * ty;
  t[9] = c[9] - 0.6 * tz;
}

template <int MASK>
__device__ __forceinline__ RecH make_rech(const double* __restrict__ R, const double* __restrict__ gam,
                                          const double* __restrict__ psi, const double* __restrict__ lam,
                                          int64_t j) {
  RecH rc;
  rc.x = R[3 * j];
  rc.y = R[3 * j + 1];
  rc.z = R[3 * j + 2];
  if (MASK & 1) stf3(gam + 10 * j, rc.g);
  if (MASK & 2) {
    double sxx, syy, sxy, sxz, syz;
    basis_to_cart(psi + 5 * j, sxx, syy, sxy, sxz, syz);
    rc.p[0] = sxx;
    rc.p[1] = syy;
    rc.p[2] = sxy;
    rc.p[3] = sxz;
    rc.p[4] = syz;
  }
  if (MASK & 4) stf3(lam + 10 * j, rc.l);
  return rc;
}

// N = T . x for a symmetric rank-3 T (10 components): Nxx Nyy Nzz Nxy Nxz Nyz
__device__ __forceinline__ void contract3(const double* __restrict__ c, double dx, double dy, double dz,
                                          double* N) {
  N[0] = fma(c[0], dx, fma(c[1], dy, c[2] * dz));
  N[1] = fma(c[3], dx, fma(c[6], dy, c[7] * dz));
  N[2] = fma(c[5], dx, fma(c[8], dy, c[9] * dz));
  N[3] = fma(c[1], dx, fma(c[3], dy, c[4] * dz));
  N[4] = fma(c[2], dx, fma(c[4], dy, c[5] * dz));
  N[5] = fma(c[4], dx, fma(c[7], dy, c[8] * dz));
}

struct Sym6 {  // symmetric matrix accumulator: xx yy zz xy xz yz
  double xx = 0, yy = 0, zz = 0, xy = 0, xz = 0, yz = 0;
};

// s += k1 sym(M) + k2 sym((x cross w) x) with M_ij = (x cross S_.j)_i, S symmetric (xx yy zz xy xz yz)
__device__ __forceinline__ void acc_rot(double dx, double dy, double dz, const double* S, double wx, double wy,
                                        double wz, double k1, double k2, Sym6& s) {
  const double Sxx = S[0], Syy = S[1], Szz = S[2], Sxy = S[3], Sxz = S[4], Syz = S[5];
  const double cx = dy * wz - dz * wy, cy = dz * wx - dx * wz, cz = dx * wy - dy * wx;
  const double Mxx = dy * Sxz - dz * Sxy, Myy = dz * Sxy - dx * Syz, Mzz = dx * Syz - dy * Sxz;
  const double Mxy = (dy * Syz - dz * Syy) + (dz * Sxx - dx * Sxz);
  const double Mxz = (dy * Szz - dz * Syz) + (dx * Sxy - dy * Sxx);
  const double Myz = (dz * Sxz - dx * Szz) + (dx * Syy - dy * Sxy);
  s.xx = fma(k1, Mxx, fma(k2, cx * dx, s.xx));
  s.yy = fma(k1, Myy, fma(k2, cy * dy, s.yy));
  s.zz = fma(k1, Mzz, fma(k2, cz * dz, s.zz));
  const double h1 = 0.5 * k1, h2 = 0.5 * k2;
  s.xy = fma(h1, Mxy, fma(h2, fma(cx, dy, cy * dx), s.xy));
  s.xz = fma(h1, Mxz, fma(h2, fma(cx, dz, cz * dx), s.xz));
  s.yz = fma(h1, Myz, fma(h2, fma(cy, dz, cz * dy), s.yz));
}

// TGT 0: strain (5-basis, 5 values per receiver); 1: velocity and rotation (6); 2: flow (3)
template <int TGT, int MASK>
__device__ __forceinline__ void hi_pair(const RecH& s, double xi, double yi, double zi, const HiCoef& k,
                                        Sym6& e, double* u, double* w) {
  const double dx = xi - s.x, dy = yi - s.y, dz = zi - s.z;
  const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
  const double ri = rinv_or_zero(r2);
  const double ri2 = ri * ri;
  const double ri5 = ri2 * ri2 * ri;
  const double ri7 = ri5 * ri2;
  const double ri9 = ri7 * ri2;
  if (MASK & 1) {  // septlet mode
    double N[6];
    contract3(s.g, dx, dy, dz, N);
    const double gx = fma(N[0], dx, fma(N[3], dy, N[4] * dz));
    const double gy = fma(N[3], dx, fma(N[1], dy, N[5] * dz));
    const double gz = fma(N[4], dx, fma(N[5], dy, N[2] * dz));
    const double Q = fma(gx, dx, fma(gy, dy, gz * dz));
    if (TGT == 0) {
      const double c1 = ri5 * fma(k.e1b, ri2, k.e1a);
      const double c2 = ri7 * fma(k.e2b, ri2, k.e2a);
      const double c3 = Q * ri9 * fma(k.e3b, ri2, k.e3a);
      e.xx = fma(c1, N[0], fma(c2, gx * dx, fma(c3, dx * dx, e.xx)));
      e.yy = fma(c1, N[1], fma(c2, gy * dy, fma(c3, dy * dy, e.yy)));
      e.zz = fma(c1, N[2], fma(c2, gz * dz, fma(c3, dz * dz, e.zz)));
      const double h2 = 0.5 * c2;
      e.xy = fma(c1, N[3], fma(h2, fma(gx, dy, gy * dx), fma(c3, dx * dy, e.xy)));
      e.xz = fma(c1, N[4], fma(h2, fma(gx, dz, gz * dx), fma(c3, dx * dz, e.xz)));
      e.yz = fma(c1, N[5], fma(h2, fma(gy, dz, gz * dy), fma(c3, dy * dz, e.yz)));
    } else {
      const double cg = ri5 * fma(TGT == 1 ? k.gCu : k.gCf, ri2, k.gA);
      const double cq = Q * ri7 * fma(TGT == 1 ? k.gDu : k.gDf, ri2, k.gB);
      u[0] = fma(cg, gx, fma(cq, dx, u[0]));
      u[1] = fma(cg, gy, fma(cq, dy, u[1]));
      u[2] = fma(cg, gz, fma(cq, dz, u[2]));
      if (TGT == 1) {
        const double cw = k.gW * ri7;
        w[0] = fma(cw, dy * gz - dz * gy, w[0]);
        w[1] = fma(cw, dz * gx - dx * gz, w[1]);
        w[2] = fma(cw, dx * gy - dy * gx, w[2]);
      }
    }
  }
  if (MASK & 2) {  // vortlet mode
    const double pxx = s.p[0], pyy = s.p[1], pzz = -(s.p[0] + s.p[1]), pxy = s.p[2], pxz = s.p[3], pyz = s.p[4];
    const double wx = fma(pxx, dx, fma(pxy, dy, pxz * dz));
    const double wy = fma(pxy, dx, fma(pyy, dy, pyz * dz));
    const double wz = fma(pxz, dx, fma(pyz, dy, pzz * dz));
    if (TGT == 0) {
      const double S[6] = {pxx, pyy, pzz, pxy, pxz, pyz};
      acc_rot(dx, dy, dz, S, wx, wy, wz, k.cpsi * ri5, -5.0 * k.cpsi * ri7, e);
    } else {
      const double c = k.cpsi * ri5;
      u[0] = fma(c, dy * wz - dz * wy, u[0]);
      u[1] = fma(c, dz * wx - dx * wz, u[1]);
      u[2] = fma(c, dx * wy - dy * wx, u[2]);
      if (TGT == 1) {
        const double q = fma(wx, dx, fma(wy, dy, wz * dz));
        const double cx = -2.5 * k.cpsi * ri7 * q;
        w[0] = fma(c, wx, fma(cx, dx, w[0]));
        w[1] = fma(c, wy, fma(cx, dy, w[1]));
        w[2] = fma(c, wz, fma(cx, dz, w[2]));
      }
    }
  }
  if (MASK & 4) {  // spinlet mode
    double N[6];
    contract3(s.l, dx, dy, dz, N);
    const double vx = fma(N[0], dx, fma(N[3], dy, N[4] * dz));
    const double vy = fma(N[3], dx, fma(N[1], dy, N[5] * dz));
    const double vz = fma(N[4], dx, fma(N[5], dy, N[2] * dz));
    if (TGT == 0) {
      acc_rot(dx, dy, dz, N, vx, vy, vz, 2.0 * k.clam * ri7, -7.0 * k.clam * ri9, e);
    } else {
      const double c = k.clam * ri7;
      u[0] = fma(c, dy * vz - dz * vy, u[0]);
      u[1] = fma(c, dz * vx - dx * vz, u[1]);
      u[2] = fma(c, dx * vy - dy * vx, u[2]);
      if (TGT == 1) {
        const double Q = fma(vx, dx, fma(vy, dy, vz * dz));
        const double cv = 1.5 * c, cx = -3.5 * k.clam * ri9 * Q;
        w[0] = fma(cv, vx, fma(cx, dx, w[0]));
        w[1] = fma(cv, vy, fma(cx, dy, w[1]));
        w[2] = fma(cv, vz, fma(cx, dz, w[2]));
      }
    }
  }
}

// receivers X [m x 3] (the spheres themselves for targets 0 and 1), sources R [n x 3];
// part[blockIdx.y][m][NOUT]
template <int TGT, int MASK>
__global__ void __launch_bounds__(kMaxBlock)
    k_high(const double* __restrict__ X, int m, const double* __restrict__ R, const double* __restrict__ gam,
           const double* __restrict__ psi, const double* __restrict__ lam, int n, int chunk, HiCoef k,
           double* __restrict__ part) {
  constexpr int NOUT = TGT == 0 ? 5 : (TGT == 1 ? 6 : 3);
  __shared__ RecH tile[kHiTJ];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int ii = i < m ? i : m - 1;
  const double xi = X[3 * (int64_t)ii], yi = X[3 * (int64_t)ii + 1], zi = X[3 * (int64_t)ii + 2];
  const int j0 = blockIdx.y * chunk;
  const int j1 = min(n, j0 + chunk);
  Sym6 e;
  double u[3] = {0.0, 0.0, 0.0}, w[3] = {0.0, 0.0, 0.0};
  for (int jt = j0; jt < j1; jt += kHiTJ) {
    const int cnt = min(kHiTJ, j1 - jt);
    __syncthreads();
    for (int t = threadIdx.x; t < cnt; t += blockDim.x) tile[t] = make_rech<MASK>(R, gam, psi, lam, jt + t);
    __syncthreads();
    for (int jj = 0; jj < cnt; ++jj) hi_pair<TGT, MASK>(tile[jj], xi, yi, zi, k, e, u, w);
  }
  if (i >= m) return;
  double* o = part + ((int64_t)blockIdx.y * m + i) * NOUT;
  if (TGT == 0) {
    o[0] = RS2 * (e.xx - e.yy);
    o[1] = RS6 * (2.0 * e.zz - e.xx - e.yy);
    o[2] = 2.0 * RS2 * e.xy;
    o[3] = 2.0 * RS2 * e.xz;
    o[4] = 2.0 * RS2 * e.yz;
  } else {
    o[0] = u[0];
    o[1] = u[1];
    o[2] = u[2];
    if (TGT == 1) {
      o[3] = w[0];
      o[4] = w[1];
      o[5] = w[2];
    }
  }
}

// a[i][c] += sum_s part[s][i][c] (fixed order), for NOUT values per receiver split over a (c < 3)
// and b (c >= 3)
template <int NOUT>
__global__ void k_high_finish(const double* __restrict__ part, int split, int64_t m, double* __restrict__ a,
                              double* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double acc[NOUT];
#pragma unroll
  for (int c = 0; c < NOUT; ++c) acc[c] = 0.0;
  for (int s = 0; s < split; ++s) {
    const double* p = part + ((int64_t)s * m + i) * NOUT;
#pragma unroll
    for (int c = 0; c < NOUT; ++c) acc[c] += p[c];
  }
  if (NOUT == 5) {
#pragma unroll
    for (int c = 0; c < 5; ++c) a[5 * i + c] += acc[c];
  } else {
#pragma unroll
    for (int c = 0; c < 3; ++c) a[3 * i + c] += acc[c];
    if (NOUT == 6) {
#pragma unroll
      for (int c = 0; c < 3; ++c) b[3 * i + c] += acc[3 + c];
    }
  }
}

inline unsigned nblk(int64_t len, int b) { return (unsigned)((len + b - 1) / b); }

HiCoef hi_coef(const Phys& ph) {
  const double a = ph.a, a2 = a * a, a5 = a2 * a2 * a, a7 = a5 * a2;
  HiCoef k;
  k.gA = -7.0 / 16.0 * a5;
  k.gB = 35.0 / 16.0 * a5;
  k.gCu = 25.0 / 8.0 * a7;
  k.gDu = -175.0 / 24.0 * a7;
  k.gCf = 15.0 / 16.0 * a7;
  k.gDf = -35.0 / 16.0 * a7;
  k.gW = -35.0 / 16.0 * a5;
  k.e1a = -7.0 / 8.0 * a5;
  k.e1b = 4.5 * a7;
  k.e2a = 35.0 / 4.0 * a5;
  k.e2b = -31.5 * a7;
  k.e3a = -245.0 / 16.0 * a5;
  k.e3b = 189.0 / 4.0 * a7;
  k.cpsi = -a5 / 3.0;
  k.clam = -a7 / 8.0;
  return k;
}

template <int TGT>
void high_dispatch(int mask, dim3 grid, int bs, hipStream_t s, const double* X, int m, const double* R,
                   const double* gam, const double* psi, const double* lam, int n, int chunk, const HiCoef& k,
                   double* part) {
#define MBS_HI(M)                                                                                          \
  case M:                                                                                                \
    hipLaunchKernelGGL((k_high<TGT, M>), grid, dim3(bs), 0, s, X, m, R, gam, psi, lam, n, chunk, k, part); \
    break;
  switch (mask) {
    MBS_HI(1)
    MBS_HI(2)
    MBS_HI(3)
    MBS_HI(4)
    MBS_HI(5)
    MBS_HI(6)
    MBS_HI(7)
    default:
      break;
  }
#undef MBS_HI
}

}  // namespace

int high_mask(const HighSlip& h) { return (h.gam ? 1 : 0) | (h.psi ? 2 : 0) | (h.lam ? 4 : 0); }

void launch_high(int target, const double* X, int64_t m, const double* R, int64_t n, const HighSlip& h,
                 double* a, double* b, double* part, int split, const Phys& ph, Tile t, hipStream_t s) {
  const int mask = high_mask(h);
  if (!mask || m < 1 || n < 1) return;
  const int bs = tile_block(t);
  const int chunk = (int)((n + split - 1) / split);
  dim3 grid(nblk(m, bs), split);
  const HiCoef k = hi_coef(ph);
  if (target == 0) {
    high_dispatch<0>(mask, grid, bs, s, X, (int)m, R, h.gam, h.psi, h.lam, (int)n, chunk, k, part);
    hipLaunchKernelGGL(k_high_finish<5>, dim3(nblk(m, 256)), dim3(256), 0, s, part, split, m, a, nullptr);
  } else if (target == 1) {
    high_dispatch<1>(mask, grid, bs, s, X, (int)m, R, h.gam, h.psi, h.lam, (int)n, chunk, k, part);
    hipLaunchKernelGGL(k_high_finish<6>, dim3(nblk(m, 256)), dim3(256), 0, s, part, split, m, a, b);
  } else {
    high_dispatch<2>(mask, grid, bs, s, X, (int)m, R, h.gam, h.psi, h.lam, (int)n, chunk, k, part);
    hipLaunchKernelGGL(k_high_finish<3>, dim3(nblk(m, 256)), dim3(256), 0, s, part, split, m, a, nullptr);
  }
}

int high_split(int64_t m, int64_t n, Tile t) {
  // enough workgroups to fill the GPU: receiver tiles times source chunks of >= kHiTJ sources
  const int64_t ntile = (m + tile_block(t) - 1) / tile_block(t);
  const int64_t target = t.wgs > 0 ? t.wgs : 2048;
  const int64_t sp = (target + ntile - 1) / ntile;
  return (int)std::min<int64_t>(std::max<int64_t>(sp, 1), std::max<int64_t>(1, (n + kHiTJ - 1) / kHiTJ));
}

}  // namespace mbs
