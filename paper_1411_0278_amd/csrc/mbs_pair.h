// Per-pair arithmetic of the three all-pairs passes, shared by the single-configuration and the
// batched kernels. x = R_n - R_m (receiver minus source), P = 1/(8 pi eta); source records carry
// P-scaled force/torque/stresslet and (a^5/10)-scaled trace modes, so no constant appears per pair.
// The closed forms are listed at the top of mbs_kernels.hip.
#pragma once
#include <hip/hip_runtime.h>

#include "mbs_device.h"

namespace mbs {

// ---------------------------------------------------------------- P1: strain of force, torque, d
struct alignas(16) RecF {
  double x, y, z, fx, fy, fz, tx, ty, tz, dx, dy, dz;
};

struct Mom6 {  // raw moments sum x_i v_j of the per-pair strain vector v
  double pxx = 0, pyy = 0, pzz = 0, qxy = 0, qxz = 0, qyz = 0;
};

// SELF: the source range may hold the receiver itself (r = 0 contributes nothing)
template <bool SELF, bool HAS_T, bool HAS_D>
__device__ __forceinline__ void p1_pair(const RecF& s, double xi, double yi, double zi, double A8,
                                        double B16, Mom6& m) {
  const double dx = xi - s.x, dy = yi - s.y, dz = zi - s.z;
  const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
  const double ri = SELF ? rinv_or_zero(r2) : rsq_nr(r2);
  const double ri2 = ri * ri;
  const double ri5 = ri2 * ri2 * ri;
  const double ri7 = ri5 * ri2;
  const double xF = fma(dx, s.fx, fma(dy, s.fy, dz * s.fz));
  const double alpha = xF * ri5 * fma(A8, ri2, -3.0);
  const double beta = B16 * ri5;
  double vx = fma(beta, s.fx, alpha * dx);
  double vy = fma(beta, s.fy, alpha * dy);
  double vz = fma(beta, s.fz, alpha * dz);
  if (HAS_T) {  // -3 (T x x) / r^5
    const double m3 = -3.0 * ri5;
    vx = fma(m3, s.ty * dz - s.tz * dy, vx);
    vy = fma(m3, s.tz * dx - s.tx * dz, vy);
    vz = fma(m3, s.tx * dy - s.ty * dx, vz);
  }
  if (HAS_D) {  // 6 d / r^5 - 15 (x.d) x / r^7
    const double xd = -15.0 * ri7 * (dx * s.dx + dy * s.dy + dz * s.dz);
    const double six = 6.0 * ri5;
    vx = fma(six, s.dx, fma(xd, dx, vx));
    vy = fma(six, s.dy, fma(xd, dy, vy));
    vz = fma(six, s.dz, fma(xd, dz, vz));
  }
  m.pxx = fma(dx, vx, m.pxx);
  m.pyy = fma(dy, vy, m.pyy);
  m.pzz = fma(dz, vz, m.pzz);
  m.qxy = fma(dx, vy, fma(dy, vx, m.qxy));
  m.qxz = fma(dx, vz, fma(dz, vx, m.qxz));
  m.qyz = fma(dy, vz, fma(dz, vy, m.qyz));
}

// K records at once, stage by stage (independent chains in flight in each wave); the moments take
// the records in order, exactly as K calls of p1_pair<false, ...> would.
template <int K, bool HAS_T, bool HAS_D>
__device__ __forceinline__ void p1_pairs(const RecF* s, double xi, double yi, double zi, double A8,
                                         double B16, Mom6& m) {
  double dx[K], dy[K], dz[K], ri[K], vx[K], vy[K], vz[K];
#pragma unroll
  for (int q = 0; q < K; ++q) {
    dx[q] = xi - s[q].x;
    dy[q] = yi - s[q].y;
    dz[q] = zi - s[q].z;
    ri[q] = rsq_nr(fma(dx[q], dx[q], fma(dy[q], dy[q], dz[q] * dz[q])));
  }
#pragma unroll
  for (int q = 0; q < K; ++q) {
    const double ri2 = ri[q] * ri[q];
    const double ri5 = ri2 * ri2 * ri[q];
    const double xF = fma(dx[q], s[q].fx, fma(dy[q], s[q].fy, dz[q] * s[q].fz));
    const double alpha = xF * ri5 * fma(A8, ri2, -3.0);
    const double beta = B16 * ri5;
    vx[q] = fma(beta, s[q].fx, alpha * dx[q]);
    vy[q] = fma(beta, s[q].fy, alpha * dy[q]);
    vz[q] = fma(beta, s[q].fz, alpha * dz[q]);
    if (HAS_T) {
      const double m3 = -3.0 * ri5;
      vx[q] = fma(m3, s[q].ty * dz[q] - s[q].tz * dy[q], vx[q]);
      vy[q] = fma(m3, s[q].tz * dx[q] - s[q].tx * dz[q], vy[q]);
      vz[q] = fma(m3, s[q].tx * dy[q] - s[q].ty * dx[q], vz[q]);
    }
    if (HAS_D) {
      const double ri7 = ri5 * ri2;
      const double xd = -15.0 * ri7 * (dx[q] * s[q].dx + dy[q] * s[q].dy + dz[q] * s[q].dz);
      const double six = 6.0 * ri5;
      vx[q] = fma(six, s[q].dx, fma(xd, dx[q], vx[q]));
      vy[q] = fma(six, s[q].dy, fma(xd, dy[q], vy[q]));
      vz[q] = fma(six, s[q].dz, fma(xd, dz[q], vz[q]));
    }
  }
#pragma unroll
  for (int q = 0; q < K; ++q) {
    m.pxx = fma(dx[q], vx[q], m.pxx);
    m.pyy = fma(dy[q], vy[q], m.pyy);
    m.pzz = fma(dz[q], vz[q], m.pzz);
    m.qxy = fma(dx[q], vy[q], fma(dy[q], vx[q], m.qxy));
    m.qxz = fma(dx[q], vz[q], fma(dz[q], vx[q], m.qxz));
    m.qyz = fma(dy[q], vz[q], fma(dz[q], vy[q], m.qyz));
  }
}

// traceless 5-basis projection of the moments
__device__ __forceinline__ void mom6_to_basis(const Mom6& m, double* e) {
  e[0] = RS2 * (m.pxx - m.pyy);
  e[1] = RS6 * (2.0 * m.pzz - m.pxx - m.pyy);
  e[2] = RS2 * m.qxy;
  e[3] = RS2 * m.qxz;
  e[4] = RS2 * m.qyz;
}

// ---------------------------------------------------------------- P3: velocity and rotation
struct alignas(16) RecO {
  double x, y, z, fx, fy, fz, tx, ty, tz, sxx, syy, sxy, sxz, syz, dx, dy, dz, pad;
};

struct UW {
  double ux = 0, uy = 0, uz = 0, wx = 0, wy = 0, wz = 0;
};

// Pair geometry shared by the output pass and the fused output + operator pass: separation, powers
// of 1/r (all zero for r = 0 when SELF) and w = Sigma x, q = x.w of the source stresslet.
struct Geo {
  double dx, dy, dz, ri, ri2, ri3, ri5, wx, wy, wz, q;
};

template <bool SELF>
__device__ __forceinline__ void pair_geo(const RecO& s, double xi, double yi, double zi, Geo& g) {
  g.dx = xi - s.x;
  g.dy = yi - s.y;
  g.dz = zi - s.z;
  const double r2 = fma(g.dx, g.dx, fma(g.dy, g.dy, g.dz * g.dz));
  g.ri = SELF ? rinv_or_zero(r2) : rsq_nr(r2);
  g.ri2 = g.ri * g.ri;
  g.ri3 = g.ri2 * g.ri;
  g.ri5 = g.ri3 * g.ri2;
  const double szz = -(s.sxx + s.syy);
  g.wx = fma(s.sxx, g.dx, fma(s.sxy, g.dy, s.sxz * g.dz));
  g.wy = fma(s.sxy, g.dx, fma(s.syy, g.dy, s.syz * g.dz));
  g.wz = fma(s.sxz, g.dx, fma(s.syz, g.dy, szz * g.dz));
  g.q = fma(g.dx, g.wx, fma(g.dy, g.wy, g.dz * g.wz));
}

template <bool HAS_T, bool HAS_D>
__device__ __forceinline__ void p3_acc(const RecO& s, const Geo& g, double A2_2, double A2_23, double A8,
                                       double B16, UW& a) {
  const double dx = g.dx, dy = g.dy, dz = g.dz, ri = g.ri, ri2 = g.ri2, ri3 = g.ri3, ri5 = g.ri5;
  const double wx = g.wx, wy = g.wy, wz = g.wz, q = g.q;
  const double xF = fma(dx, s.fx, fma(dy, s.fy, dz * s.fz));
  double cx = xF * fma(-A2_2, ri5, ri3) + q * ri5 * fma(A8, ri2, -3.0);
  const double cF = fma(A2_23, ri3, ri);
  const double cw = B16 * ri5;
  if (HAS_D) cx = fma(3.0 * ri5, dx * s.dx + dy * s.dy + dz * s.dz, cx);
  a.ux = fma(cx, dx, fma(cF, s.fx, fma(cw, wx, a.ux)));
  a.uy = fma(cx, dy, fma(cF, s.fy, fma(cw, wy, a.uy)));
  a.uz = fma(cx, dz, fma(cF, s.fz, fma(cw, wz, a.uz)));
  // rotation: x cross (-F/r^3 + 3 w / r^5)
  const double gx = fma(3.0 * ri5, wx, -ri3 * s.fx);
  const double gy = fma(3.0 * ri5, wy, -ri3 * s.fy);
  const double gz = fma(3.0 * ri5, wz, -ri3 * s.fz);
  a.wx = fma(dy, gz, fma(-dz, gy, a.wx));
  a.wy = fma(dz, gx, fma(-dx, gz, a.wy));
  a.wz = fma(dx, gy, fma(-dy, gx, a.wz));
  if (HAS_T) {
    // U += (T x x)/r^3 ; W += 1.5 (x.T) x / r^5 - 0.5 T / r^3
    a.ux = fma(ri3, s.ty * dz - s.tz * dy, a.ux);
    a.uy = fma(ri3, s.tz * dx - s.tx * dz, a.uy);
    a.uz = fma(ri3, s.tx * dy - s.ty * dx, a.uz);
    const double xT = 1.5 * ri5 * (dx * s.tx + dy * s.ty + dz * s.tz);
    const double h = -0.5 * ri3;
    a.wx = fma(xT, dx, fma(h, s.tx, a.wx));
    a.wy = fma(xT, dy, fma(h, s.ty, a.wy));
    a.wz = fma(xT, dz, fma(h, s.tz, a.wz));
  }
  if (HAS_D) {  // U += -d / r^3 (the (x.d) x part is in cx)
    a.ux = fma(-ri3, s.dx, a.ux);
    a.uy = fma(-ri3, s.dy, a.uy);
    a.uz = fma(-ri3, s.dz, a.uz);
  }
}

template <bool SELF, bool HAS_T, bool HAS_D>
__device__ __forceinline__ void p3_pair(const RecO& s, double xi, double yi, double zi, double A2_2,
                                        double A2_23, double A8, double B16, UW& a) {
  Geo g;
  pair_geo<SELF>(s, xi, yi, zi, g);
  p3_acc<HAS_T, HAS_D>(s, g, A2_2, A2_23, A8, B16, a);
}

// ---------------------------------------------------------------- P2: the system operator
template <typename T>
struct alignas(8 * sizeof(T)) Src8 {
  T x, y, z, sxx, syy, sxy, sxz, syz;
};

template <typename T>
struct Mom {  // per-receiver sums of the operator pass
  T pxx = 0, pyy = 0, pzz = 0, qxy = 0, qxz = 0, qyz = 0, t0 = 0, t1 = 0, t2 = 0, t3 = 0, t4 = 0;
};

template <typename T, bool SELF>
__device__ __forceinline__ void p2_pair(const Src8<T>& s, T xi, T yi, T zi, T A24, T A42, Mom<T>& m) {
  const T dx = xi - s.x, dy = yi - s.y, dz = zi - s.z;
  const T r2 = fma(dx, dx, fma(dy, dy, dz * dz));
  const T ri = SELF ? rinv_or_zero(r2) : rsq_nr(r2);
  const T ri2 = ri * ri;
  const T ri5 = ri2 * ri2 * ri;
  const T ri7 = ri5 * ri2;
  const T szz = -(s.sxx + s.syy);
  const T wx = fma(s.sxx, dx, fma(s.sxy, dy, s.sxz * dz));
  const T wy = fma(s.sxy, dx, fma(s.syy, dy, s.syz * dz));
  const T wz = fma(s.sxz, dx, fma(s.syz, dy, szz * dz));
  const T q = fma(dx, wx, fma(dy, wy, dz * wz));
  const T c1 = ri5 * fma(A24, ri2, (T)-6);
  const T c2 = q * ri7 * fma(-A42, ri2, (T)15);
  const T vx = fma(c1, wx, c2 * dx);
  const T vy = fma(c1, wy, c2 * dy);
  const T vz = fma(c1, wz, c2 * dz);
  m.pxx = fma(dx, vx, m.pxx);
  m.pyy = fma(dy, vy, m.pyy);
  m.pzz = fma(dz, vz, m.pzz);
  m.qxy = fma(dx, vy, fma(dy, vx, m.qxy));
  m.qxz = fma(dx, vz, fma(dz, vx, m.qxz));
  m.qyz = fma(dy, vz, fma(dz, vy, m.qyz));
  m.t0 = fma(ri5, s.sxx, m.t0);
  m.t1 = fma(ri5, s.syy, m.t1);
  m.t2 = fma(ri5, s.sxy, m.t2);
  m.t3 = fma(ri5, s.sxz, m.t3);
  m.t4 = fma(ri5, s.syz, m.t4);
}

// Operator sums of one pair (the arithmetic of p2_pair) from the geometry already formed for the
// output pass; the record's stresslet carries the factor P, so the projection takes P = 1.
__device__ __forceinline__ void p2_acc(const RecO& s, const Geo& g, double A24, double A42, Mom<double>& m) {
  const double ri7 = g.ri5 * g.ri2;
  const double c1 = g.ri5 * fma(A24, g.ri2, -6.0);
  const double c2 = g.q * ri7 * fma(-A42, g.ri2, 15.0);
  const double vx = fma(c1, g.wx, c2 * g.dx);
  const double vy = fma(c1, g.wy, c2 * g.dy);
  const double vz = fma(c1, g.wz, c2 * g.dz);
  m.pxx = fma(g.dx, vx, m.pxx);
  m.pyy = fma(g.dy, vy, m.pyy);
  m.pzz = fma(g.dz, vz, m.pzz);
  m.qxy = fma(g.dx, vy, fma(g.dy, vx, m.qxy));
  m.qxz = fma(g.dx, vz, fma(g.dz, vx, m.qxz));
  m.qyz = fma(g.dy, vz, fma(g.dz, vy, m.qyz));
  m.t0 = fma(g.ri5, s.sxx, m.t0);
  m.t1 = fma(g.ri5, s.syy, m.t1);
  m.t2 = fma(g.ri5, s.sxy, m.t2);
  m.t3 = fma(g.ri5, s.sxz, m.t3);
  m.t4 = fma(g.ri5, s.syz, m.t4);
}

// E[x] at one receiver in the 5-basis from the operator sums (11 values, see Mom)
__device__ __forceinline__ void p2_strain(const double* v, double P, double a2, double* e) {
  const double C3 = -2.4 * a2;  // -12 a^2 / 5
  const double pxx = v[0], pyy = v[1], pzz = v[2], qxy = v[3], qxz = v[4], qyz = v[5];
  const double t0 = v[6], t1 = v[7], t2 = v[8], t3 = v[9], t4 = v[10];
  e[0] = P * RS2 * ((pxx - pyy) + C3 * (t0 - t1));
  e[1] = P * RS6 * ((2.0 * pzz - pxx - pyy) - 3.0 * C3 * (t0 + t1));
  e[2] = P * RS2 * (qxy + 2.0 * C3 * t2);
  e[3] = P * RS2 * (qxz + 2.0 * C3 * t3);
  e[4] = P * RS2 * (qyz + 2.0 * C3 * t4);
}

}  // namespace mbs
