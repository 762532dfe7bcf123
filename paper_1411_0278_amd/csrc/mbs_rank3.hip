// Traction ranks <= 3 (gfx950): the quadratic-order traction modes of the minimal truncation
// (section IV: septlet, vortlet, potential dipole) solved for beside the stresslet.
//
// Each sphere m's exterior flow is written through its flow stresslet Sigma and the equivalent slips
// of the three modes (the slips a lone sphere would need for the same flow of that mode): X^g (a
// symmetric traceless rank-3 tensor), X^p (symmetric traceless rank 2), X^d (a vector), besides the
// fixed sources (body force F, torque T, spinlet slip lambda). The flows at x = R_n - R_m
// (P = 1/(8 pi eta); w = Sigma.x, q = x.w, g = X^g:xx, Q = g.x, v = lambda:xx):
//
//   F      u = P[(1/r + a^2/(3r^3)) F + (x.F)(1/r^3 - a^2/r^5) x]      T  u = P (T x x)/r^3
//   Sigma  u = P[q (3a^2/r^7 - 3/r^5) x - (6a^2/5) w/r^5]
//   X^d    u = (a^5/10)[3 (x.X^d) x/r^5 - X^d/r^3]
//   X^g    u = (-7a^5/(16 r^5) + 15a^7/(16 r^7)) g + (35a^5/(16 r^7) - 35a^7/(16 r^9)) Q x
//   X^p    u = -(a^5/3) (x cross (X^p.x))/r^5                             lambda  u = -(a^7/8) (x cross v)/r^7
//
// and their Laplacians (the finite-size operators need them): F: 2P[F/r^3 - 3 (x.F) x/r^5];
// Sigma: P[30 q x/r^7 - 12 w/r^5]; X^g: (7a^5/24)[45 g/r^7 - 105 Q x/r^9]; the others are harmonic.
//
// Per receiver n, the flows of all other spheres are summed as second-order Taylor data at R_n
// (value, gradient and Hessian of u and of its Laplacian: with the Laplacian known in closed form,
// second order is enough for every projection). The receiver's Galerkin coefficients (section III)
// then follow in closed form:
//   U = u + (a^2/6) lap u,   W = curl u / 2,   E = sym grad (u + (a^2/10) lap u)  (5-basis),
//   V^(3)/a^2 = the part symmetric traceless in (j, k) of d_j d_k (u_i + (a^2/14) lap u_i), whose
//   irreducible parts (section IV) are the septlet (symmetric traceless part, 7-basis), the
//   vortlet (minus the symmetric contraction of eps with i and j, 5-basis) and the potential
//   dipole (the contraction of i with j).
// The system rows: Sigma_n/gamma - E_n = E[fixed sources] - c s_n for the stresslet,
// X^alpha_n + P^alpha_n = v^alpha_n - P^alpha[fixed sources] for the three modes.
//
// Layout: one receiver per thread, source records through LDS tiles, the sources split into
// grid.y chunks whose partial sums a finishing kernel adds in a fixed order.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "mbs_device.h"
#include "mbs_internal.h"

namespace mbs {

namespace {

constexpr double kRs2 = 0.70710678118654752440;  // 1/sqrt(2)
constexpr double kRs6 = 0.40824829046386301637;  // 1/sqrt(6)

// Second-order Taylor data of a scalar field at the receiver:
// f(x0 + h) ~ c0 + sum_j cj h_j + sum_{j <= k} cjk h_j h_k.
struct J2 {
  double c0 = 0, cx = 0, cy = 0, cz = 0, cxx = 0, cxy = 0, cxz = 0, cyy = 0, cyz = 0, czz = 0;
};

// truncated product
__device__ __forceinline__ J2 jmul(const J2& A, const J2& B) {
  J2 C;
  C.c0 = A.c0 * B.c0;
  C.cx = fma(A.c0, B.cx, A.cx * B.c0);
  C.cy = fma(A.c0, B.cy, A.cy * B.c0);
  C.cz = fma(A.c0, B.cz, A.cz * B.c0);
  C.cxx = fma(A.c0, B.cxx, fma(A.cx, B.cx, A.cxx * B.c0));
  C.cyy = fma(A.c0, B.cyy, fma(A.cy, B.cy, A.cyy * B.c0));
  C.czz = fma(A.c0, B.czz, fma(A.cz, B.cz, A.czz * B.c0));
  C.cxy = fma(A.c0, B.cxy, fma(A.cx, B.cy, fma(A.cy, B.cx, A.cxy * B.c0)));
  C.cxz = fma(A.c0, B.cxz, fma(A.cx, B.cz, fma(A.cz, B.cx, A.cxz * B.c0)));
  C.cyz = fma(A.c0, B.cyz, fma(A.cy, B.cz, fma(A.cz, B.cy, A.cyz * B.c0)));
  return C;
}

// acc += s * A
__device__ __forceinline__ void jaxpy(double s, const J2& A, J2& acc) {
  acc.c0 = fma(s, A.c0, acc.c0);
  acc.cx = fma(s, A.cx, acc.cx);
  acc.cy = fma(s, A.cy, acc.cy);
  acc.cz = fma(s, A.cz, acc.cz);
  acc.cxx = fma(s, A.cxx, acc.cxx);
  acc.cxy = fma(s, A.cxy, acc.cxy);
  acc.cxz = fma(s, A.cxz, acc.cxz);
  acc.cyy = fma(s, A.cyy, acc.cyy);
  acc.cyz = fma(s, A.cyz, acc.cyz);
  acc.czz = fma(s, A.czz, acc.czz);
}

// acc += s * w * A, the weight w by Taylor order: w0 on the value, w1 on the gradient, w2 on the
// second-order part. With w = (a^2/6, a^2/10, a^2/14), summing the flow's data with plain weights and
// its Laplacian's with these gives every projection at once: the value is F^0 u, the gradient that
// of F^1 u, the second-order part that of F^2 u (the Laplacian of each flow is a pressure gradient,
// so the curl taken from the gradient is that of u alone).
struct LW {
  double w0, w1, w2;
};
__device__ __forceinline__ void jaxpyL(double s, const J2& A, const LW& w, J2& acc) {
  const double s0 = s * w.w0, s1 = s * w.w1, s2 = s * w.w2;
  acc.c0 = fma(s0, A.c0, acc.c0);
  acc.cx = fma(s1, A.cx, acc.cx);
  acc.cy = fma(s1, A.cy, acc.cy);
  acc.cz = fma(s1, A.cz, acc.cz);
  acc.cxx = fma(s2, A.cxx, acc.cxx);
  acc.cxy = fma(s2, A.cxy, acc.cxy);
  acc.cxz = fma(s2, A.cxz, acc.cxz);
  acc.cyy = fma(s2, A.cyy, acc.cyy);
  acc.cyz = fma(s2, A.cyz, acc.cyz);
  acc.czz = fma(s2, A.czz, acc.czz);
}

// A *= s
__device__ __forceinline__ void jscale(double s, J2& A) {
  A.c0 *= s;
  A.cx *= s;
  A.cy *= s;
  A.cz *= s;
  A.cxx *= s;
  A.cxy *= s;
  A.cxz *= s;
  A.cyy *= s;
  A.cyz *= s;
  A.czz *= s;
}

__device__ __forceinline__ J2 jlin(double c0, double cx, double cy, double cz) {
  J2 A;
  A.c0 = c0;
  A.cx = cx;
  A.cy = cy;
  A.cz = cz;
  return A;
}

// r^-k at x0 with rk = r^-k, rk2 = r^-(k+2), rk4 = r^-(k+4):
// d_j r^-k = -k x_j r^-(k+2),  d_j d_l r^-k = k(k+2) x_j x_l r^-(k+4) - k delta_jl r^-(k+2)
__device__ __forceinline__ J2 jradial(double k, double rk, double rk2, double rk4, double x, double y, double z) {
  J2 A;
  const double a = -k * rk2, b = k * (k + 2.0) * rk4;
  A.c0 = rk;
  A.cx = a * x;
  A.cy = a * y;
  A.cz = a * z;
  A.cxx = 0.5 * fma(b * x, x, a);
  A.cyy = 0.5 * fma(b * y, y, a);
  A.czz = 0.5 * fma(b * z, z, a);
  A.cxy = b * x * y;
  A.cxz = b * x * z;
  A.cyz = b * y * z;
  return A;
}

// Taylor data of g_i = T_ijk x_j x_k (T symmetric, 10 components xxx xxy xxz xyy xyz xzz yyy yyz
// yzz zzz) at x0 (exact: a quadratic), for i = 0, 1, 2, and of Q = T_ijk x_i x_j x_k (cubic).
struct Sym3 {
  double t[3][3][3];
};
__device__ __forceinline__ Sym3 sym3_of(const double* c) {
  Sym3 S;
  const int idx[10][3] = {{0, 0, 0}, {0, 0, 1}, {0, 0, 2}, {0, 1, 1}, {0, 1, 2},
                          {0, 2, 2}, {1, 1, 1}, {1, 1, 2}, {1, 2, 2}, {2, 2, 2}};
#pragma unroll
  for (int q = 0; q < 10; ++q) {
    const int i = idx[q][0], j = idx[q][1], k = idx[q][2];
    S.t[i][j][k] = S.t[i][k][j] = S.t[j][i][k] = S.t[j][k][i] = S.t[k][i][j] = S.t[k][j][i] = c[q];
  }
  return S;
}
__device__ __forceinline__ void quad_jets(const Sym3& T, double x, double y, double z, J2 g[3], J2& Q) {
  const double X[3] = {x, y, z};
  double M[3][3];  // M_ij = T_ijk x_k
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) M[i][j] = fma(T.t[i][j][0], X[0], fma(T.t[i][j][1], X[1], T.t[i][j][2] * X[2]));
  double gv[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    gv[i] = fma(M[i][0], X[0], fma(M[i][1], X[1], M[i][2] * X[2]));
    g[i].c0 = gv[i];
    g[i].cx = 2.0 * M[i][0];
    g[i].cy = 2.0 * M[i][1];
    g[i].cz = 2.0 * M[i][2];
    g[i].cxx = T.t[i][0][0];
    g[i].cyy = T.t[i][1][1];
    g[i].czz = T.t[i][2][2];
    g[i].cxy = 2.0 * T.t[i][0][1];
    g[i].cxz = 2.0 * T.t[i][0][2];
    g[i].cyz = 2.0 * T.t[i][1][2];
  }
  Q.c0 = fma(gv[0], X[0], fma(gv[1], X[1], gv[2] * X[2]));
  Q.cx = 3.0 * gv[0];
  Q.cy = 3.0 * gv[1];
  Q.cz = 3.0 * gv[2];
  Q.cxx = 3.0 * M[0][0];
  Q.cyy = 3.0 * M[1][1];
  Q.czz = 3.0 * M[2][2];
  Q.cxy = 6.0 * M[0][1];
  Q.cxz = 6.0 * M[0][2];
  Q.cyz = 6.0 * M[1][2];
}

// symmetric traceless part of a symmetric rank-3 tensor given by its 10 components
__device__ __forceinline__ void stf10(const double* c, double* t) {
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

// The 7-basis of symmetric traceless rank-3 tensors: B_m = T_m/|T_m|, T_m,ijk = (1/6) d_i d_j d_k p_m for
// the harmonic cubics p_1..p_7 = 2z^3 - 3x^2 z - 3y^2 z, 4xz^2 - x^3 - xy^2, 4yz^2 - x^2 y - y^3,
// x^2 z - y^2 z, xyz, x^3 - 3xy^2, 3x^2 y - y^3. From 7 coordinates to the 10 symmetric components:
__device__ __forceinline__ void from7(const double* c, double* t) {
  const double s10 = 0.31622776601683793320;   // 1/sqrt(10)
  const double s203 = 0.38729833462074168852;  // sqrt(3/20)
  const double s23 = 1.22474487139158904910;   // sqrt(3/2)
  const double s6 = 0.40824829046386301637;    // 1/sqrt(6)
  for (int q = 0; q < 10; ++q) t[q] = 0.0;
  // p1: zzz = 2, xxz = -1, yyz = -1
  t[9] += 2.0 * s10 * c[0];
  t[2] -= s10 * c[0];
  t[7] -= s10 * c[0];
  // p2: xzz = 4/3, xxx = -1, xyy = -1/3
  t[5] += (4.0 / 3.0) * s203 * c[1];
  t[0] -= s203 * c[1];
  t[3] -= (1.0 / 3.0) * s203 * c[1];
  // p3: yzz = 4/3, yyy = -1, xxy = -1/3
  t[8] += (4.0 / 3.0) * s203 * c[2];
  t[6] -= s203 * c[2];
  t[1] -= (1.0 / 3.0) * s203 * c[2];
  // p4: xxz = 1/3, yyz = -1/3
  t[2] += (1.0 / 3.0) * s23 * c[3];
  t[7] -= (1.0 / 3.0) * s23 * c[3];
  // p5: xyz = 1/6, scaled by sqrt(6)
  t[4] += s6 * c[4];
  // p6: xxx = 1, xyy = -1, halved
  t[0] += 0.5 * c[5];
  t[3] -= 0.5 * c[5];
  // p7: xxy = 1, yyy = -1, halved
  t[1] += 0.5 * c[6];
  t[6] -= 0.5 * c[6];
}

// 7 coordinates B_m :. S of a rank-3 tensor S_ijk (any symmetry; the contraction with the symmetric
// traceless B_m takes its symmetric traceless part)
__device__ __forceinline__ void to7(const double S[3][3][3], double* c) {
  const double s10 = 0.31622776601683793320, s203 = 0.38729833462074168852, s23 = 1.22474487139158904910,
               s6 = 0.40824829046386301637;
  auto P3 = [&](int i, int j, int k) { return S[i][j][k] + S[j][k][i] + S[k][i][j]; };  // i, j = i: 3 perms
  const int X = 0, Y = 1, Z = 2;
  c[0] = s10 * (2.0 * S[Z][Z][Z] - P3(X, X, Z) - P3(Y, Y, Z));
  c[1] = s203 * ((4.0 / 3.0) * P3(Z, Z, X) - S[X][X][X] - (1.0 / 3.0) * P3(Y, Y, X));
  c[2] = s203 * ((4.0 / 3.0) * P3(Z, Z, Y) - S[Y][Y][Y] - (1.0 / 3.0) * P3(X, X, Y));
  c[3] = (1.0 / 3.0) * s23 * (P3(X, X, Z) - P3(Y, Y, Z));
  c[4] = s6 * (S[X][Y][Z] + S[X][Z][Y] + S[Y][X][Z] + S[Y][Z][X] + S[Z][X][Y] + S[Z][Y][X]);
  c[5] = 0.5 * (S[X][X][X] - P3(Y, Y, X));
  c[6] = 0.5 * (P3(X, X, Y) - S[Y][Y][Y]);
}

// Source record of one sphere: centre, P-scaled force and torque, P-scaled Cartesian flow stresslet
// (xx yy xy xz yz zz), (a^5/10)-scaled X^d, X^g and lambda as 10 symmetric components (traceless),
// Cartesian X^p (xx yy xy xz yz zz).
struct alignas(16) Rec3 {
  double x, y, z;
  double f[3], t[3];
  double s[6];
  double d[3];
  double g[10];
  double p[6];
  double l[10];
};

constexpr int kR3TJ = 32;   // source records per LDS tile
constexpr int kR3Blk = 128;  // receivers per workgroup
enum { kR3Op = 0, kR3Rhs = 1, kR3Out = 2 };
// Source groups, each swept by its own workgroups (grid.y = groups x source chunks) so that each
// sweep's registers are those of its own sources: the fixed sources (force, torque, spinlet slip),
// the flow stresslet with X^d, X^g, X^p. The operator sweeps the last three separately (then every
// sweep fits two waves per SIMD), the outputs the fixed sources, the stresslet with X^d, and X^g
// with X^p.
enum { kGFix = 1, kGSig = 2, kGSept = 4, kGVort = 8, kGQuad = kGSept | kGVort };
constexpr int r3_ngroups(int mode) { return mode == kR3Op ? 3 : (mode == kR3Rhs ? 1 : 3); }
constexpr int r3_group(int mode, int g) {
  return mode == kR3Op ? (g == 0 ? kGSig : (g == 1 ? kGSept : kGVort)) : (mode == kR3Rhs ? kGFix : (g == 0 ? kGFix : (g == 1 ? kGSig : kGQuad)));
}

struct R3C {  // per-problem constants
  double a2, a5, a7;
  LW w;
};

// add the flow of the sources of group(s) GRP in record s at x = receiver - source, with its
// Laplacian weighted as in jaxpyL, to A[3]
template <int GRP>
__device__ __forceinline__ void r3_pair(const Rec3& s, double x, double y, double z, const R3C& k, J2 A[3]) {
  const double r2 = fma(x, x, fma(y, y, z * z));
  const double ri = rsq_nr(r2);
  const double ri2 = ri * ri;
  const double p3 = ri2 * ri, p5 = p3 * ri2, p7 = p5 * ri2, p9 = p7 * ri2, p11 = p9 * ri2, p13 = p11 * ri2;
  const J2 R3 = jradial(3.0, p3, p5, p7, x, y, z);
  const J2 R5 = jradial(5.0, p5, p7, p9, x, y, z);
  const J2 R7 = jradial(7.0, p7, p9, p11, x, y, z);
  const J2 X[3] = {jlin(x, 1.0, 0.0, 0.0), jlin(y, 0.0, 1.0, 0.0), jlin(z, 0.0, 0.0, 1.0)};
  if (GRP & kGFix) {  // force, torque, spinlet slip
    const J2 R1 = jradial(1.0, ri, p3, p5, x, y, z);
    J2 c1 = R1;
    jaxpy(k.a2 / 3.0, R3, c1);
    J2 c2 = R3;
    jaxpy(-k.a2, R5, c2);
    const J2 xF = jlin(fma(x, s.f[0], fma(y, s.f[1], z * s.f[2])), s.f[0], s.f[1], s.f[2]);
    const J2 t1 = jmul(xF, c2);
    const J2 t2 = jmul(xF, R5);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      jaxpy(s.f[i], c1, A[i]);
      jaxpy(1.0, jmul(t1, X[i]), A[i]);
      jaxpyL(2.0 * s.f[i], R3, k.w, A[i]);
      jaxpyL(-6.0, jmul(t2, X[i]), k.w, A[i]);
    }
    // torque: (T x x)/r^3
    const J2 tx = jlin(s.t[1] * z - s.t[2] * y, 0.0, -s.t[2], s.t[1]);
    const J2 ty = jlin(s.t[2] * x - s.t[0] * z, s.t[2], 0.0, -s.t[0]);
    const J2 tz = jlin(s.t[0] * y - s.t[1] * x, -s.t[1], s.t[0], 0.0);
    jaxpy(1.0, jmul(tx, R3), A[0]);
    jaxpy(1.0, jmul(ty, R3), A[1]);
    jaxpy(1.0, jmul(tz, R3), A[2]);
    // spinlet slip: -(a^7/8) (x cross v)/r^7, v = lambda:xx
    J2 v[3], Qd;
    quad_jets(sym3_of(s.l), x, y, z, v, Qd);
    const J2 cx = jmul(X[1], v[2]), cx2 = jmul(X[2], v[1]);
    const J2 cy = jmul(X[2], v[0]), cy2 = jmul(X[0], v[2]);
    const J2 cz = jmul(X[0], v[1]), cz2 = jmul(X[1], v[0]);
    const double cl = -0.125 * k.a7;
    J2 wx = cx, wy = cy, wz = cz;
    jaxpy(-1.0, cx2, wx);
    jaxpy(-1.0, cy2, wy);
    jaxpy(-1.0, cz2, wz);
    jaxpy(cl, jmul(wx, R7), A[0]);
    jaxpy(cl, jmul(wy, R7), A[1]);
    jaxpy(cl, jmul(wz, R7), A[2]);
  }
  if (GRP & kGSig) {  // flow stresslet and X^d
    const double* S = s.s;
    const J2 w[3] = {jlin(fma(S[0], x, fma(S[2], y, S[3] * z)), S[0], S[2], S[3]),
                     jlin(fma(S[2], x, fma(S[1], y, S[4] * z)), S[2], S[1], S[4]),
                     jlin(fma(S[3], x, fma(S[4], y, S[5] * z)), S[3], S[4], S[5])};
    J2 q = jmul(X[0], w[0]);
    jaxpy(1.0, jmul(X[1], w[1]), q);
    jaxpy(1.0, jmul(X[2], w[2]), q);
    J2 cq = R7;  // 3a^2/r^7 - 3/r^5
    jscale(3.0 * k.a2, cq);
    jaxpy(-3.0, R5, cq);
    const J2 tq = jmul(q, cq);
    const J2 tl = jmul(q, R7);
    // X^d ((a^5/10)-scaled): 3 (x.d) x/r^5 - d/r^3
    const J2 xd = jlin(fma(x, s.d[0], fma(y, s.d[1], z * s.d[2])), s.d[0], s.d[1], s.d[2]);
    const J2 td = jmul(xd, R5);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const J2 r5w = jmul(R5, w[i]);
      jaxpy(1.0, jmul(tq, X[i]), A[i]);
      jaxpy(-1.2 * k.a2, r5w, A[i]);
      jaxpyL(30.0, jmul(tl, X[i]), k.w, A[i]);
      jaxpyL(-12.0, r5w, k.w, A[i]);
      jaxpy(3.0, jmul(td, X[i]), A[i]);
      jaxpy(-s.d[i], R3, A[i]);
    }
  }
  if (GRP & kGSept) {  // X^g
    const J2 R9 = jradial(9.0, p9, p11, p13, x, y, z);
    J2 g[3], Q;
    quad_jets(sym3_of(s.g), x, y, z, g, Q);
    J2 ca = R5;  // -7a^5/(16 r^5) + 15a^7/(16 r^7)
    jscale(-7.0 / 16.0 * k.a5, ca);
    jaxpy(15.0 / 16.0 * k.a7, R7, ca);
    J2 cb = R7;  // 35a^5/(16 r^7) - 35a^7/(16 r^9)
    jscale(35.0 / 16.0 * k.a5, cb);
    jaxpy(-35.0 / 16.0 * k.a7, R9, cb);
    const J2 Qb = jmul(Q, cb);
    const J2 Q9 = jmul(Q, R9);
    const double lg = 7.0 / 24.0 * k.a5;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      jaxpy(1.0, jmul(g[i], ca), A[i]);
      jaxpy(1.0, jmul(Qb, X[i]), A[i]);
      jaxpyL(45.0 * lg, jmul(g[i], R7), k.w, A[i]);
      jaxpyL(-105.0 * lg, jmul(Q9, X[i]), k.w, A[i]);
    }
  }
  if (GRP & kGVort) {  // X^p: -(a^5/3) (x cross (X^p.x))/r^5
    const double* Pp = s.p;
    const J2 pw[3] = {jlin(fma(Pp[0], x, fma(Pp[2], y, Pp[3] * z)), Pp[0], Pp[2], Pp[3]),
                      jlin(fma(Pp[2], x, fma(Pp[1], y, Pp[4] * z)), Pp[2], Pp[1], Pp[4]),
                      jlin(fma(Pp[3], x, fma(Pp[4], y, Pp[5] * z)), Pp[3], Pp[4], Pp[5])};
    J2 xw[3];
    xw[0] = jmul(X[1], pw[2]);
    jaxpy(-1.0, jmul(X[2], pw[1]), xw[0]);
    xw[1] = jmul(X[2], pw[0]);
    jaxpy(-1.0, jmul(X[0], pw[2]), xw[1]);
    xw[2] = jmul(X[0], pw[1]);
    jaxpy(-1.0, jmul(X[1], pw[0]), xw[2]);
    const double cp = -k.a5 / 3.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) jaxpy(cp, jmul(xw[i], R5), A[i]);
  }
}

template <int GRP>
__device__ __forceinline__ Rec3 make_rec3(int j, const double* __restrict__ R, const double* __restrict__ X20,
                                          const double* __restrict__ Fe, const double* __restrict__ Te,
                                          const double* __restrict__ lam, double P, double a5_10) {
  Rec3 r{};
  r.x = R[3 * (int64_t)j];
  r.y = R[3 * (int64_t)j + 1];
  r.z = R[3 * (int64_t)j + 2];
  if (GRP & kGFix) {
    for (int c = 0; c < 3; ++c) {
      r.f[c] = Fe ? P * Fe[3 * (int64_t)j + c] : 0.0;
      r.t[c] = Te ? P * Te[3 * (int64_t)j + c] : 0.0;
    }
    if (lam) stf10(lam + 10 * (int64_t)j, r.l);
  }
  const double* x = X20 + 20 * (int64_t)j;
  if (GRP & kGSig) {
    double sxx, syy, sxy, sxz, syz;
    basis_to_cart(x, sxx, syy, sxy, sxz, syz);
    r.s[0] = P * sxx;
    r.s[1] = P * syy;
    r.s[2] = P * sxy;
    r.s[3] = P * sxz;
    r.s[4] = P * syz;
    r.s[5] = -P * (sxx + syy);
    for (int c = 0; c < 3; ++c) r.d[c] = a5_10 * x[17 + c];
  }
  if (GRP & kGSept) from7(x + 5, r.g);
  if (GRP & kGVort) {
    double pxx, pyy, pxy, pxz, pyz;
    basis_to_cart(x + 12, pxx, pyy, pxy, pxz, pyz);
    r.p[0] = pxx;
    r.p[1] = pyy;
    r.p[2] = pxy;
    r.p[3] = pxz;
    r.p[4] = pyz;
    r.p[5] = -(pxx + pyy);
  }
  return r;
}

// width of the per-receiver partial sums: 20 projections (E, septlet, vortlet, potential dipole) or 6 (U, W)
constexpr int r3_width(int mode) { return mode == kR3Out ? 6 : 20; }

// The receiver's 20 projections from the summed Taylor data: E (5-basis), then V^(3)/a^2 split into
// its septlet (7-basis), vortlet (5-basis) and potential-dipole (3) parts
__device__ __forceinline__ void r3_project(const J2 A[3], double* o) {
  // E = sym grad F^1 u, 5-basis
  o[0] = kRs2 * (A[0].cx - A[1].cy);
  o[1] = kRs6 * (2.0 * A[2].cz - A[0].cx - A[1].cy);
  o[2] = kRs2 * (A[0].cy + A[1].cx);
  o[3] = kRs2 * (A[0].cz + A[2].cx);
  o[4] = kRs2 * (A[1].cz + A[2].cy);
  // S_ijk = part of d_j d_k F^2 u_i symmetric traceless in (j, k)
  double S[3][3][3];
  for (int c = 0; c < 3; ++c) {
    double H[3][3];
    H[0][0] = 2.0 * A[c].cxx;
    H[1][1] = 2.0 * A[c].cyy;
    H[2][2] = 2.0 * A[c].czz;
    H[0][1] = H[1][0] = A[c].cxy;
    H[0][2] = H[2][0] = A[c].cxz;
    H[1][2] = H[2][1] = A[c].cyz;
    const double tr = (H[0][0] + H[1][1] + H[2][2]) / 3.0;
    for (int j = 0; j < 3; ++j)
      for (int kk = 0; kk < 3; ++kk) S[c][j][kk] = H[j][kk] - (j == kk ? tr : 0.0);
  }
  to7(S, o + 5);
  // vortlet: C_lk = -eps_lij S_ijk, symmetric part in the 5-basis
  double C[3][3];
  for (int kk = 0; kk < 3; ++kk) {
    C[0][kk] = S[2][1][kk] - S[1][2][kk];
    C[1][kk] = S[0][2][kk] - S[2][0][kk];
    C[2][kk] = S[1][0][kk] - S[0][1][kk];
  }
  o[12] = kRs2 * (C[0][0] - C[1][1]);
  o[13] = kRs6 * (2.0 * C[2][2] - C[0][0] - C[1][1]);
  o[14] = kRs2 * (C[0][1] + C[1][0]);
  o[15] = kRs2 * (C[0][2] + C[2][0]);
  o[16] = kRs2 * (C[1][2] + C[2][1]);
  // potential dipole: S_iik
  for (int kk = 0; kk < 3; ++kk) o[17 + kk] = S[0][0][kk] + S[1][1][kk] + S[2][2][kk];
}

// Sum over the sources j0 <= j < j1 of group(s) GRP at receiver (xi, yi, zi) (index ii: skipped)
template <int GRP>
__device__ __forceinline__ void r3_sweep(Rec3* tile, int ii, double xi, double yi, double zi, int j0, int j1,
                                         const double* __restrict__ R, const double* __restrict__ X20,
                                         const double* __restrict__ Fe, const double* __restrict__ Te,
                                         const double* __restrict__ lam, double P, const R3C& k, J2 A[3]) {
  for (int jt = j0; jt < j1; jt += kR3TJ) {
    const int cnt = min(kR3TJ, j1 - jt);
    __syncthreads();
    for (int t = threadIdx.x; t < cnt; t += blockDim.x)
      tile[t] = make_rec3<GRP>(jt + t, R, X20, Fe, Te, lam, P, 0.1 * k.a5);
    __syncthreads();
    for (int jj = 0; jj < cnt; ++jj) {
      if (jt + jj == ii) continue;  // a sphere does not act on itself
      const Rec3& s = tile[jj];
      r3_pair<GRP>(s, xi - s.x, yi - s.y, zi - s.z, k, A);
    }
  }
}

// grid: (receiver blocks, groups x chunks); workgroup y sweeps source chunk y % split of group
// y / split and writes partial slice y. Two waves per SIMD: the largest sweep (X^g) then keeps its
// Taylor data in 256 registers with a few bytes spilled, faster than one wave with more registers.
template <int MODE>
__global__ void __launch_bounds__(kR3Blk, 2)
    k_rank3(const double* __restrict__ R, const double* __restrict__ X20, const double* __restrict__ Fe,
            const double* __restrict__ Te, const double* __restrict__ lam, int n, int chunk, int split, double P,
            double a2, double a5, double a7, double* __restrict__ part) {
  __shared__ Rec3 tile[kR3TJ];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int ii = i < n ? i : n - 1;
  const double xi = R[3 * (int64_t)ii], yi = R[3 * (int64_t)ii + 1], zi = R[3 * (int64_t)ii + 2];
  const R3C k{a2, a5, a7, LW{a2 / 6.0, a2 / 10.0, a2 / 14.0}};
  const int grp = blockIdx.y / split;  // uniform
  const int j0 = (blockIdx.y % split) * chunk;
  const int j1 = min(n, j0 + chunk);
  J2 A[3];
  if (grp == 0)
    r3_sweep<r3_group(MODE, 0)>(tile, ii, xi, yi, zi, j0, j1, R, X20, Fe, Te, lam, P, k, A);
  else if (grp == 1)
    r3_sweep<r3_group(MODE, 1)>(tile, ii, xi, yi, zi, j0, j1, R, X20, Fe, Te, lam, P, k, A);
  else
    r3_sweep<r3_group(MODE, 2)>(tile, ii, xi, yi, zi, j0, j1, R, X20, Fe, Te, lam, P, k, A);
  if (i >= n) return;
  double* o = part + ((int64_t)blockIdx.y * n + i) * r3_width(MODE);
  if (MODE == kR3Out) {  // U = F^0 u, W = curl u / 2
    for (int c = 0; c < 3; ++c) o[c] = A[c].c0;
    o[3] = 0.5 * (A[2].cy - A[1].cz);
    o[4] = 0.5 * (A[0].cz - A[2].cx);
    o[5] = 0.5 * (A[1].cx - A[0].cy);
    return;
  }
  r3_project(A, o);
}

// y = [x_Sigma/gamma - E, x_alpha + P_alpha] (operator), b = [E - c s, v_alpha - P_alpha] (right-hand
// side), or V = -v1s + mu_t F + U, W = mu_r T + W, S = Sigma + slip_S s (outputs); sums the split
// partials in a fixed order
template <int MODE>
__global__ void k_rank3_finish(const double* __restrict__ part, int split, int n, const double* __restrict__ X20,
                               const double* __restrict__ v1s, const double* __restrict__ v2s,
                               const double* __restrict__ v3t, const double* __restrict__ gam,
                               const double* __restrict__ psi, const double* __restrict__ Fe,
                               const double* __restrict__ Te, double inv_gamma, double c_slip, double mu_t,
                               double mu_r, double slip_S, double* __restrict__ out, double* __restrict__ out2,
                               double* __restrict__ out3) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  constexpr int W = r3_width(MODE);
  double acc[W];
  for (int c = 0; c < W; ++c) acc[c] = 0.0;
  for (int s = 0; s < split; ++s) {
    const double* p = part + ((int64_t)s * n + i) * W;
    for (int c = 0; c < W; ++c) acc[c] += p[c];
  }
  if (MODE == kR3Op) {
    const double* x = X20 + 20 * (int64_t)i;
    double* y = out + 20 * (int64_t)i;
    for (int c = 0; c < 5; ++c) y[c] = x[c] * inv_gamma - acc[c];
    for (int c = 5; c < 20; ++c) y[c] = x[c] + acc[c];
  } else if (MODE == kR3Rhs) {
    double* b = out + 20 * (int64_t)i;
    for (int c = 0; c < 5; ++c) b[c] = acc[c] - (v2s ? c_slip * v2s[5 * (int64_t)i + c] : 0.0);
    double g7[7] = {0, 0, 0, 0, 0, 0, 0};
    if (gam) {
      double t[10];
      stf10(gam + 10 * (int64_t)i, t);
      const Sym3 T = sym3_of(t);
      to7(T.t, g7);
    }
    for (int c = 0; c < 7; ++c) b[5 + c] = g7[c] - acc[5 + c];
    for (int c = 0; c < 5; ++c) b[12 + c] = (psi ? psi[5 * (int64_t)i + c] : 0.0) - acc[12 + c];
    for (int c = 0; c < 3; ++c) b[17 + c] = (v3t ? v3t[3 * (int64_t)i + c] : 0.0) - acc[17 + c];
  } else {
    double* V = out + 3 * (int64_t)i;
    double* Wo = out2 + 3 * (int64_t)i;
    for (int c = 0; c < 3; ++c) {
      V[c] = acc[c] - (v1s ? v1s[3 * (int64_t)i + c] : 0.0) + (Fe ? mu_t * Fe[3 * (int64_t)i + c] : 0.0);
      Wo[c] = acc[3 + c] + (Te ? mu_r * Te[3 * (int64_t)i + c] : 0.0);
    }
    if (out3)
      for (int c = 0; c < 5; ++c)
        out3[5 * (int64_t)i + c] = X20[20 * (int64_t)i + c] + (v2s ? slip_S * v2s[5 * (int64_t)i + c] : 0.0);
  }
}

// One term of the near-field Neumann series of the rank <= 3 system A = D + B (D = diag(I/gamma, I)
// per sphere, B the couplings): y = D^{-1} (v - B_near z) over the pairs on the neighbour lists,
// z = Z, or D^{-1} v when Z is NULL. B's stresslet rows are -E and its mode rows +P^alpha.
constexpr int kR3NearBlk = 64;
__global__ void __launch_bounds__(kR3NearBlk)
    k_rank3_near(const double* __restrict__ R, const double* __restrict__ V, const double* __restrict__ Z,
                 const int* __restrict__ cnt, const int* __restrict__ list, int n, double P, double a2, double a5,
                 double a7, double gamma, double* __restrict__ Y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const R3C k{a2, a5, a7, LW{a2 / 6.0, a2 / 10.0, a2 / 14.0}};
  const double xi = R[3 * (int64_t)i], yi = R[3 * (int64_t)i + 1], zi = R[3 * (int64_t)i + 2];
  const double* src = Z ? Z : V;
  const double ps = Z ? P : P * gamma;  // D^{-1} v scales the stresslet part by gamma
  J2 A[3];
  const int c = cnt[i];
  for (int q = 0; q < c; ++q) {
    const int j = list[(int64_t)i * kNearCap + q];
    const Rec3 s = make_rec3<kGSig | kGQuad>(j, R, src, nullptr, nullptr, nullptr, ps, 0.1 * a5);
    r3_pair<kGSig | kGQuad>(s, xi - s.x, yi - s.y, zi - s.z, k, A);
  }
  double o[20];
  r3_project(A, o);
  const double* v = V + 20 * (int64_t)i;
  double* y = Y + 20 * (int64_t)i;
  for (int q = 0; q < 5; ++q) y[q] = gamma * (v[q] + o[q]);
  for (int q = 5; q < 20; ++q) y[q] = v[q] - o[q];
}

inline unsigned nblk3(int64_t len, int b) { return (unsigned)((len + b - 1) / b); }

}  // namespace

int rank3_split(int64_t n) {
  const int64_t tiles = (n + kR3Blk - 1) / kR3Blk;
  int64_t s = (1024 + tiles - 1) / tiles;
  s = std::min<int64_t>(std::max<int64_t>(s, 1), std::max<int64_t>(1, (n + kR3TJ - 1) / kR3TJ));
  return (int)s;
}

// the largest of groups x split x width over the three modes (the operator: 3 x split x 20)
int64_t rank3_part_elems(int64_t n) { return (int64_t)rank3_split(n) * 60 * n; }

namespace {
template <int M>
void launch_rank3_mode(const double* R, const double* X20, const double* v1s, const double* v2s, const double* v3t,
                       const double* gam, const double* psi, const double* lam, const double* Fe, const double* Te,
                       double* out, double* out2, double* out3, double* part, int64_t n, const Phys& ph,
                       hipStream_t s) {
  const int split = rank3_split(n);
  const int chunk = (int)((n + split - 1) / split);
  const double a2 = ph.a2, a5 = a2 * a2 * ph.a, a7 = a5 * a2;
  const int slices = r3_ngroups(M) * split;
  hipLaunchKernelGGL(k_rank3<M>, dim3(nblk3(n, kR3Blk), slices), dim3(kR3Blk), 0, s, R, X20, Fe, Te, lam, (int)n,
                     chunk, split, ph.P, a2, a5, a7, part);
  hipLaunchKernelGGL(k_rank3_finish<M>, dim3(nblk3(n, 256)), dim3(256), 0, s, part, slices, (int)n, X20, v1s, v2s,
                     v3t, gam, psi, Fe, Te, ph.inv_gamma, ph.c_slip, ph.mu_t, ph.mu_r, ph.slip_S, out, out2,
                     out3);
}
}  // namespace

void launch_rank3(int mode, const double* R, const double* X20, const double* v1s, const double* v2s,
                  const double* v3t, const double* gam, const double* psi, const double* lam, const double* Fe,
                  const double* Te, double* out, double* out2, double* out3, double* part, int64_t n,
                  const Phys& ph, hipStream_t s) {
  if (n <= 0) return;
  if (mode == 0)
    launch_rank3_mode<kR3Op>(R, X20, v1s, v2s, v3t, gam, psi, lam, Fe, Te, out, out2, out3, part, n, ph, s);
  else if (mode == 1)
    launch_rank3_mode<kR3Rhs>(R, X20, v1s, v2s, v3t, gam, psi, lam, Fe, Te, out, out2, out3, part, n, ph, s);
  else
    launch_rank3_mode<kR3Out>(R, X20, v1s, v2s, v3t, gam, psi, lam, Fe, Te, out, out2, out3, part, n, ph, s);
}

void launch_rank3_near(const double* R, const double* v, const double* z, const int* cnt, const int* list,
                       int64_t n, const Phys& ph, double* y, hipStream_t s) {
  if (n <= 0) return;
  const double a2 = ph.a2, a5 = a2 * a2 * ph.a, a7 = a5 * a2;
  hipLaunchKernelGGL(k_rank3_near, dim3(nblk3(n, kR3NearBlk)), dim3(kR3NearBlk), 0, s, R, v, z, cnt, list, (int)n,
                     ph.P, a2, a5, a7, ph.gamma, y);
}

}  // namespace mbs
