// Spheres in a periodic cubic box (gfx950): Ewald summation of the periodic Oseen tensor.
//
// The paper notes that periodic domains follow from the periodic Green's function, whose direct
// sum converges only conditionally. Hasimoto's procedure fixes it: zero mean velocity over the box
// (the k = 0 Fourier mode left out, a net force balanced by a mean pressure gradient), the tensor
// split with a parameter xi into a screened real-space part, summed over the images within a
// cutoff rc <= L/2 (so the minimum image is the only one), and a smooth Fourier part summed over the
// reciprocal lattice k = 2 pi n / L, 0 < |k| <= kmax. A sphere's own images enter through the
// Fourier sum (which runs over every sphere, the receiver included) minus the smooth part of its own
// flow at its centre, a constant per block (a multiple of the identity, or zero by parity).
//
// One pass (operator, right-hand side or outputs) is five launches:
//   k_per_real    receiver per thread, source records staged through LDS tiles of 64, each lane
//                 marking the records within rc (minimum image) in a bit mask and then evaluating
//                 its own hits with the generated screened blocks (the operator through the
//                 isotropic form of the screened stresslet strain: three generated radial
//                 functions and the contraction here); grid.y chunks of the sources, partial sums
//                 per chunk;
//   k_per_sf      segment of up to kseg consecutive wave vectors of one lattice row per thread:
//                 structure factors sum_m c_m exp(-i k.R_m) of the source coefficients (5, 9 or 14
//                 of them), one sincos per (segment, source) and the row's step exp(-i dk z_m) for
//                 the rest; grid.y chunks of the sources;
//   k_per_mult    wave vector per thread: the chunks added in order, the generated Fourier
//                 multiplier applied, times 2/L^3 (k and -k together) and the splitting factor;
//   k_per_recip   receiver per thread, wave vectors and their complex targets staged through LDS:
//                 Re sum_k exp(i k.R_n) T(k), the phase carried along each lattice row by one complex
//                 factor exp(i dk z_n) (a sincos where a row starts and every 16 steps); grid.y
//                 chunks of the wave vectors;
//   k_per_finish  the chunks added in order, the self constants and the one-body terms.
// With a mesh (smooth particle-mesh Ewald, below) the structure factors and reciprocal sums give way
// to spreading, a 3D FFT, the multipliers per mesh wave vector, the inverse FFT and interpolation,
// and the real-space pass walks the neighbouring cells of the sources' box grid.
// Every sum runs in a fixed order (bitwise reproducible). The arithmetic is binary64 throughout.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "mbs_device.h"
#include "mbs_grid.h"
#include "mbs_internal.h"
#include "mbs_periodic_gen.h"

namespace mbs {
namespace {

constexpr int kPBlk = 128;   // receivers per workgroup (real space, reciprocal sum)
constexpr int kPTJ = 64;     // source records per LDS tile
constexpr int kPKBlk = 64;   // wave vectors per workgroup (structure factors, multipliers)
constexpr int kPKT = 64;     // wave vectors per LDS tile of the reciprocal sum

enum { kPOp = 0, kPRhs = 1, kPOut = 2, kPFlow = 3 };
constexpr int pw(int t) { return t == kPOut ? 6 : (t == kPFlow ? 3 : 5); }  // target width
constexpr int pnc(int t) { return t == kPOp ? 5 : (t == kPRhs ? 9 : 14); }  // source coefficients
constexpr int sft(int t) { return t == kPFlow ? kPOut : t; }  // the structure factors a target uses
// wave vectors per structure-factor thread (consecutive along a lattice row), by target
constexpr int kseg(int t) { return t == kPOp ? 8 : 4; }

// source record: centre and pre-scaled coefficients (f = P F, t = P T, s = P Sigma, q = (a^5/20) d)
struct alignas(16) RecP {
  double x, y, z, f[3], t[3], s[5], q[3], pad;
};

template <int TGT>
__device__ __forceinline__ RecP make_rec(const double* __restrict__ R, const double* __restrict__ Fe,
                                         const double* __restrict__ Te, const double* __restrict__ Sig,
                                         const double* __restrict__ D, int j, double P, double a5_20) {
  RecP r;
  r.x = R[3 * (int64_t)j];
  r.y = R[3 * (int64_t)j + 1];
  r.z = R[3 * (int64_t)j + 2];
  for (int c = 0; c < 3; ++c) {
    r.f[c] = (TGT != kPOp && Fe) ? P * Fe[3 * (int64_t)j + c] : 0.0;
    r.t[c] = (TGT != kPOp && Te) ? P * Te[3 * (int64_t)j + c] : 0.0;
    r.q[c] = (TGT != kPOp && D) ? a5_20 * D[3 * (int64_t)j + c] : 0.0;
  }
  for (int c = 0; c < 5; ++c) r.s[c] = (TGT != kPRhs && Sig) ? P * Sig[5 * (int64_t)j + c] : 0.0;
  r.pad = 0.0;
  return r;
}

// the source coefficients of a record in the order the structure factors hold them
template <int TGT>
__device__ __forceinline__ void coeffs(const RecP& r, double* v) {
  if (TGT == kPOp) {
    for (int c = 0; c < 5; ++c) v[c] = r.s[c];
  } else if (TGT == kPRhs) {
    for (int c = 0; c < 3; ++c) {
      v[c] = r.f[c];
      v[3 + c] = r.t[c];
      v[6 + c] = r.q[c];
    }
  } else {
    for (int c = 0; c < 3; ++c) {
      v[c] = r.f[c];
      v[3 + c] = r.t[c];
      v[11 + c] = r.q[c];
    }
    for (int c = 0; c < 5; ++c) v[6 + c] = r.s[c];
  }
}

__device__ __forceinline__ double wrap(double d, double L, double invL) { return d - L * rint(d * invL); }

// The operator's three radial functions (al, be, ga of the screened stresslet strain's isotropic
// form) tabulated in s = r^2 for the mesh's real-space pass, whose result carries the mesh's own
// error of order 1e-8: Chebyshev series of degree kRtD on kRtK pieces per octave of s / a^2 from
// s = a^2 up (a piece spans 1/8 of its octave, so the powers of 1/r and the splitting's exponentials
// are resolved to about 1e-13 of their values), evaluated by Clenshaw's recurrence; pairs closer
// than a, or beyond the table, take the exact form. No erfc, exp, square root or division per pair.
constexpr int kRtD = 10;                       // degree
constexpr int kRtK = 8;                        // pieces per octave
constexpr int kRtOct = 20;                     // octaves at most (rc up to 1024 a)
constexpr int kRtC = 3 * (kRtD + 1);           // coefficients per piece
constexpr int kRtMax = kRtOct * kRtK * kRtC;   // doubles

// piece (oct, sub) covers s in s_lo 2^oct [1 + sub/K, 1 + (sub + 1)/K): its coefficients from the
// exact radial functions at the D + 1 Chebyshev points (c_0 stored halved)
__global__ void __launch_bounds__(64) k_pm_rtab(int npiece, double s_lo, double xi, double a2,
                                                double* __restrict__ tab) {
  const int iv = blockIdx.x * blockDim.x + threadIdx.x;
  if (iv >= npiece) return;
  const int oct = iv / kRtK, sub = iv % kRtK;
  const double base = ldexp(s_lo, oct);
  const double s0 = base * (1.0 + (double)sub / kRtK), s1 = base * (1.0 + (double)(sub + 1) / kRtK);
  const double mid = 0.5 * (s0 + s1), half = 0.5 * (s1 - s0);
  double v[kRtD + 1][3];
  for (int j = 0; j <= kRtD; ++j) {
    const double th = M_PI * (j + 0.5) / (kRtD + 1);
    const double sj = fma(half, cos(th), mid);
    const double r = sqrt(sj);
    per_real_es_radial(1.0 / r, erfc(xi * r), exp(-xi * xi * sj), xi, a2, v[j]);
  }
  for (int f = 0; f < 3; ++f)
    for (int k = 0; k <= kRtD; ++k) {
      double c = 0.0;
      for (int j = 0; j <= kRtD; ++j) c = fma(v[j][f], cos(M_PI * k * (j + 0.5) / (kRtD + 1)), c);
      c *= 2.0 / (kRtD + 1);
      tab[(int64_t)iv * kRtC + f * (kRtD + 1) + k] = k == 0 ? 0.5 * c : c;
    }
}

// abg from the table in LDS (npiece pieces); false when s lies outside it
__device__ __forceinline__ bool rtab_eval(const double* rt, int npiece, double s, double inv_slo, double* abg) {
  int e;
  const double m = frexp(s * inv_slo, &e);  // s / s_lo = m 2^e, m in [1/2, 1)
  const int oct = e - 1;
  if (oct < 0) return false;
  const double fk = (2.0 * m - 1.0) * kRtK;  // position within the octave, in pieces
  const int sub = min((int)fk, kRtK - 1);
  const int iv = oct * kRtK + sub;
  if (iv >= npiece) return false;
  const double t = 2.0 * (fk - sub) - 1.0, t2 = 2.0 * t;
  const double* c = rt + iv * kRtC;
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    double b1 = 0.0, b2 = 0.0;
#pragma unroll
    for (int k = kRtD; k >= 1; --k) {
      const double b0 = fma(t2, b1, c[f * (kRtD + 1) + k] - b2);
      b2 = b1;
      b1 = b0;
    }
    abg[f] = fma(t, b1, c[f * (kRtD + 1)] - b2);
  }
  return true;
}

// one source record's screened real-space term at a receiver, the separation (dx, dy, dz) already
// the minimum image (the pair within rc, not coincident); the operator's radial functions from the
// table rt when one is given and covers the pair
template <int TGT>
__device__ __forceinline__ void real_pair_d(const RecP& s, double dx, double dy, double dz, double xi, double a2,
                                            double* acc, const double* rt = nullptr, int npiece = 0,
                                            double inv_slo = 0.0) {
  const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
  if (TGT == kPOp) {
    // E = al Sigma + be (x w + w x) + ga q x x (+ a trace the 5-basis drops), w = Sigma x, q = x.w
    double abg[3];
    if (!rt || !rtab_eval(rt, npiece, r2, inv_slo, abg)) {
      const double r = sqrt(r2);
      per_real_es_radial(1.0 / r, erfc(xi * r), exp(-xi * xi * r2), xi, a2, abg);
    }
    double sxx, syy, sxy, sxz, syz;
    basis_to_cart(s.s, sxx, syy, sxy, sxz, syz);
    const double szz = -(sxx + syy);
    const double wx = fma(sxx, dx, fma(sxy, dy, sxz * dz));
    const double wy = fma(sxy, dx, fma(syy, dy, syz * dz));
    const double wz = fma(sxz, dx, fma(syz, dy, szz * dz));
    const double q = fma(dx, wx, fma(dy, wy, dz * wz));
    const double b2 = 2.0 * abg[1], gq = abg[2] * q;
    // M = be (x w + w x) + ga q x x: diagonal M_ii and doubled off-diagonals 2 M_ij
    const double mxx = fma(b2 * dx, wx, gq * dx * dx), myy = fma(b2 * dy, wy, gq * dy * dy),
                 mzz = fma(b2 * dz, wz, gq * dz * dz);
    const double mxy = fma(b2, fma(dx, wy, dy * wx), 2.0 * gq * dx * dy);
    const double mxz = fma(b2, fma(dx, wz, dz * wx), 2.0 * gq * dx * dz);
    const double myz = fma(b2, fma(dy, wz, dz * wy), 2.0 * gq * dy * dz);
    acc[0] = fma(abg[0], s.s[0], fma(RS2, mxx - myy, acc[0]));
    acc[1] = fma(abg[0], s.s[1], fma(RS6, 2.0 * mzz - mxx - myy, acc[1]));
    acc[2] = fma(abg[0], s.s[2], fma(RS2, mxy, acc[2]));
    acc[3] = fma(abg[0], s.s[3], fma(RS2, mxz, acc[3]));
    acc[4] = fma(abg[0], s.s[4], fma(RS2, myz, acc[4]));
    return;
  }
  const double r = sqrt(r2);
  const double ri = 1.0 / r, ec = erfc(xi * r), ex = exp(-xi * xi * r2);
  if (TGT == kPRhs) {
    // E = x a + a x + b x x (+ a trace), a = Af f + Aq q + Dt (x cross t), b = Bf (x.f) + Bq (x.q)
    double rf[5];
    per_real_ftq_radial(ri, ec, ex, xi, a2, rf);
    const double xt0 = dy * s.t[2] - dz * s.t[1], xt1 = dz * s.t[0] - dx * s.t[2], xt2 = dx * s.t[1] - dy * s.t[0];
    const double ax = fma(rf[0], s.f[0], fma(rf[2], s.q[0], rf[4] * xt0));
    const double ay = fma(rf[0], s.f[1], fma(rf[2], s.q[1], rf[4] * xt1));
    const double az = fma(rf[0], s.f[2], fma(rf[2], s.q[2], rf[4] * xt2));
    const double xf = fma(dx, s.f[0], fma(dy, s.f[1], dz * s.f[2]));
    const double xq = fma(dx, s.q[0], fma(dy, s.q[1], dz * s.q[2]));
    const double b = fma(rf[1], xf, rf[3] * xq);
    // diagonal M_ii and doubled off-diagonals 2 M_ij
    const double mxx = dx * fma(b, dx, 2.0 * ax), myy = dy * fma(b, dy, 2.0 * ay), mzz = dz * fma(b, dz, 2.0 * az);
    const double mxy = 2.0 * fma(b * dx, dy, fma(dx, ay, dy * ax));
    const double mxz = 2.0 * fma(b * dx, dz, fma(dx, az, dz * ax));
    const double myz = 2.0 * fma(b * dy, dz, fma(dy, az, dz * ay));
    acc[0] = fma(RS2, mxx - myy, acc[0]);
    acc[1] = fma(RS6, 2.0 * mzz - mxx - myy, acc[1]);
    acc[2] = fma(RS2, mxy, acc[2]);
    acc[3] = fma(RS2, mxz, acc[3]);
    acc[4] = fma(RS2, myz, acc[4]);
  }
  if (TGT == kPOut) {
    // U = F1 f + Q1 q + S1 w + T1 (t cross x) + (F2 (x.f) + Q2 (x.q) + S2 (x.w)) x,
    // W = G1 (f cross x) + Gq (q cross x) + J1 (x cross w) + H1 t + H2 (x.t) x,  w = Sigma x
    double rm[12];
    per_real_motion_radial(ri, ec, ex, xi, a2, rm);
    double sxx, syy, sxy, sxz, syz;
    basis_to_cart(s.s, sxx, syy, sxy, sxz, syz);
    const double szz = -(sxx + syy);
    const double wx = fma(sxx, dx, fma(sxy, dy, sxz * dz));
    const double wy = fma(sxy, dx, fma(syy, dy, syz * dz));
    const double wz = fma(sxz, dx, fma(syz, dy, szz * dz));
    const double xf = fma(dx, s.f[0], fma(dy, s.f[1], dz * s.f[2]));
    const double xq = fma(dx, s.q[0], fma(dy, s.q[1], dz * s.q[2]));
    const double xw = fma(dx, wx, fma(dy, wy, dz * wz));
    const double xt = fma(dx, s.t[0], fma(dy, s.t[1], dz * s.t[2]));
    const double c = fma(rm[1], xf, fma(rm[3], xq, rm[6] * xw));
    const double tx0 = s.t[1] * dz - s.t[2] * dy, tx1 = s.t[2] * dx - s.t[0] * dz, tx2 = s.t[0] * dy - s.t[1] * dx;
    acc[0] += fma(rm[0], s.f[0], fma(rm[2], s.q[0], fma(rm[5], wx, fma(rm[4], tx0, c * dx))));
    acc[1] += fma(rm[0], s.f[1], fma(rm[2], s.q[1], fma(rm[5], wy, fma(rm[4], tx1, c * dy))));
    acc[2] += fma(rm[0], s.f[2], fma(rm[2], s.q[2], fma(rm[5], wz, fma(rm[4], tx2, c * dz))));
    // v = G1 f + Gq q - J1 w gives G1 (f cross x) + Gq (q cross x) + J1 (x cross w) = v cross x
    const double v0 = fma(rm[7], s.f[0], fma(rm[8], s.q[0], -rm[11] * wx));
    const double v1 = fma(rm[7], s.f[1], fma(rm[8], s.q[1], -rm[11] * wy));
    const double v2 = fma(rm[7], s.f[2], fma(rm[8], s.q[2], -rm[11] * wz));
    const double h = rm[10] * xt;
    acc[3] += fma(v1, dz, fma(-v2, dy, fma(rm[9], s.t[0], h * dx)));
    acc[4] += fma(v2, dx, fma(-v0, dz, fma(rm[9], s.t[1], h * dy)));
    acc[5] += fma(v0, dy, fma(-v1, dx, fma(rm[9], s.t[2], h * dz)));
  }
  if (TGT == kPFlow) {
    // u = F1 f + Q1 q + S1 w + T1 (t cross x) + (F2 (x.f) + Q2 (x.q) + S2 (x.w)) x,  w = Sigma x
    double rw[7];
    per_real_flow_radial(ri, ec, ex, xi, a2, rw);
    double sxx, syy, sxy, sxz, syz;
    basis_to_cart(s.s, sxx, syy, sxy, sxz, syz);
    const double szz = -(sxx + syy);
    const double wx = fma(sxx, dx, fma(sxy, dy, sxz * dz));
    const double wy = fma(sxy, dx, fma(syy, dy, syz * dz));
    const double wz = fma(sxz, dx, fma(syz, dy, szz * dz));
    const double xf = fma(dx, s.f[0], fma(dy, s.f[1], dz * s.f[2]));
    const double xq = fma(dx, s.q[0], fma(dy, s.q[1], dz * s.q[2]));
    const double xw = fma(dx, wx, fma(dy, wy, dz * wz));
    const double c = fma(rw[1], xf, fma(rw[3], xq, rw[6] * xw));
    const double tx0 = s.t[1] * dz - s.t[2] * dy, tx1 = s.t[2] * dx - s.t[0] * dz, tx2 = s.t[0] * dy - s.t[1] * dx;
    acc[0] += fma(rw[0], s.f[0], fma(rw[2], s.q[0], fma(rw[5], wx, fma(rw[4], tx0, c * dx))));
    acc[1] += fma(rw[0], s.f[1], fma(rw[2], s.q[1], fma(rw[5], wy, fma(rw[4], tx1, c * dy))));
    acc[2] += fma(rw[0], s.f[2], fma(rw[2], s.q[2], fma(rw[5], wz, fma(rw[4], tx2, c * dz))));
  }
}

template <int TGT>
__device__ __forceinline__ void real_pair(const RecP& s, double xi0, double yi0, double zi0, double L, double invL,
                                          double xi, double a2, double* acc) {
  real_pair_d<TGT>(s, wrap(xi0 - s.x, L, invL), wrap(yi0 - s.y, L, invL), wrap(zi0 - s.z, L, invL), xi, a2, acc);
}

// position of the k-th (from 0) set bit of m
__device__ __forceinline__ int kth_bit(uint64_t m, int k) {
  int pos = 0;
#pragma unroll
  for (int w = 32; w >= 1; w >>= 1) {
    const uint64_t low = (1ull << w) - 1ull;
    const int c = __popcll(m & low);
    if (k >= c) {
      k -= c;
      m >>= w;
      pos += w;
    } else {
      m &= low;
    }
  }
  return pos;
}

// A wavefront's hits (receiver lane, record of the LDS tile) dealt out evenly over its 64 lanes, 64
// per round, in the order of the lanes and then of the records, each lane evaluating one pair; the
// contributions summed back per receiver by a segmented scan across the lanes and added to the
// receiver's sums (a fixed order: bitwise reproducible). Every lane of the wavefront must call it.
// WRAP: the separation taken as the minimum image (else the records already stand at it).
template <int TGT, bool WRAP>
__device__ __forceinline__ void tile_hits(const RecP* tile, uint64_t hits, double xi0, double yi0, double zi0,
                                          double L, double invL, double xi, double a2, double* acc,
                                          const double* rt, int npiece, double inv_slo) {
  constexpr int W = pw(TGT);
  const int lane = threadIdx.x & 63;
  const int c = __popcll(hits);
  int inc = c;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int t = __shfl_up(inc, d, 64);
    if (lane >= d) inc += t;
  }
  const int off = inc - c;
  const int T = __shfl(inc, 63, 64);
  for (int base = 0; base < T; base += 64) {
    const int e = base + lane;
    int src = 0;  // the receiver lane holding entry e: the last lane with off <= e
#pragma unroll
    for (int w = 32; w >= 1; w >>= 1) {
      const int cand = src + w;
      const int o = __shfl(off, cand < 64 ? cand : 63, 64);
      if (cand < 64 && o <= e) src = cand;
    }
    const int osrc = __shfl(off, src, 64);
    const uint64_t hsrc = __shfl(hits, src, 64);
    const double xr = __shfl(xi0, src, 64), yr = __shfl(yi0, src, 64), zr = __shfl(zi0, src, 64);
    double v[W];
#pragma unroll
    for (int cc = 0; cc < W; ++cc) v[cc] = 0.0;
    if (e < T) {
      const RecP& s = tile[kth_bit(hsrc, e - osrc)];
      double dx = xr - s.x, dy = yr - s.y, dz = zr - s.z;
      if (WRAP) {
        dx = wrap(dx, L, invL);
        dy = wrap(dy, L, invL);
        dz = wrap(dz, L, invL);
      }
      real_pair_d<TGT>(s, dx, dy, dz, xi, a2, v, rt, npiece, inv_slo);
    }
    // inclusive scan within each receiver's run of entries (runs are contiguous)
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int sup = __shfl_up(src, d, 64);
#pragma unroll
      for (int cc = 0; cc < W; ++cc) {
        const double t = __shfl_up(v[cc], d, 64);
        if (lane >= d && sup == src) v[cc] += t;
      }
    }
    // each receiver takes the sum at the last of its entries in this round
    const int lo = max(off, base), hi = min(off + c, base + 64);
    const int last = hi > lo ? hi - 1 - base : 0;
#pragma unroll
    for (int cc = 0; cc < W; ++cc) {
      const double t = __shfl(v[cc], last, 64);
      if (hi > lo) acc[cc] += t;
    }
  }
}

template <int TGT>
__global__ void __launch_bounds__(kPBlk)
    k_per_real(const double* __restrict__ X, int m, const double* __restrict__ R, int n,
               const double* __restrict__ Fe, const double* __restrict__ Te, const double* __restrict__ Sig,
               const double* __restrict__ D, int chunk, double L, double invL, double rc2, double xi, double a2,
               double P, double a5_20, double* __restrict__ part) {
  __shared__ RecP tile[kPTJ];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int ii = i < m ? i : m - 1;
  const double xi0 = X[3 * (int64_t)ii], yi0 = X[3 * (int64_t)ii + 1], zi0 = X[3 * (int64_t)ii + 2];
  const int j0 = blockIdx.y * chunk;
  const int j1 = min(n, j0 + chunk);
  constexpr int W = pw(TGT);
  double acc[W];
#pragma unroll
  for (int c = 0; c < W; ++c) acc[c] = 0.0;
  for (int jt = j0; jt < j1; jt += kPTJ) {
    const int cnt = min(kPTJ, j1 - jt);
    __syncthreads();
    for (int t = threadIdx.x; t < cnt; t += blockDim.x) tile[t] = make_rec<TGT>(R, Fe, Te, Sig, D, jt + t, P, a5_20);
    __syncthreads();
    // which records of the tile lie within rc of this receiver (the receiver itself, and its images
    // beyond rc, excluded): a cheap pass over the tile, then each lane evaluates only its own hits,
    // so a wavefront pays for its busiest lane rather than for every record any lane needs
    uint64_t hits = 0;
#pragma unroll 8
    for (int jj = 0; jj < cnt; ++jj) {
      const double dx = wrap(xi0 - tile[jj].x, L, invL), dy = wrap(yi0 - tile[jj].y, L, invL),
                   dz = wrap(zi0 - tile[jj].z, L, invL);
      const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
      hits |= (uint64_t)(r2 < rc2 && r2 > 0.0) << jj;
    }
    // (each lane its own hits: with the exact pair arithmetic and the larger share of pairs within rc
    // of the direct sums, dealing the hits out evenly, as the mesh's cell pass does, was slower here:
    // 70.7 -> 89.4 ms at 10^5 spheres)
    while (hits) {
      const int jj = __ffsll((unsigned long long)hits) - 1;
      hits &= hits - 1;
      real_pair<TGT>(tile[jj], xi0, yi0, zi0, L, invL, xi, a2, acc);
    }
  }
  if (i >= m) return;
  double* o = part + ((int64_t)blockIdx.y * m + i) * W;
#pragma unroll
  for (int c = 0; c < W; ++c) o[c] = acc[c];
}

// structure factors of one source chunk over the segments (first wave vector, count <= kseg) of
// the half lattice: sf[(chunk * K + k) * 2NC] = (re[NC], im[NC])
template <int TGT>
__global__ void __launch_bounds__(kPKBlk)
    k_per_sf(const double* __restrict__ R, int n, const double* __restrict__ Fe, const double* __restrict__ Te,
             const double* __restrict__ Sig, const double* __restrict__ D, const double* __restrict__ kv,
             const int2* __restrict__ seg, int nseg, int K, double dk, int chunk, double P, double a5_20,
             double* __restrict__ sf) {
  __shared__ RecP tile[kPTJ];
  __shared__ double wre[kPTJ], wim[kPTJ];  // exp(-i dk z_m): one step along a row
  constexpr int NC = pnc(TGT), S = kseg(TGT);
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const int2 sg = seg[g < nseg ? g : nseg - 1];
  const double k1 = kv[3 * (int64_t)sg.x], k2 = kv[3 * (int64_t)sg.x + 1], k3 = kv[3 * (int64_t)sg.x + 2];
  const int j0 = blockIdx.y * chunk;
  const int j1 = min(n, j0 + chunk);
  double re[S][NC], im[S][NC];
#pragma unroll
  for (int q = 0; q < S; ++q)
#pragma unroll
    for (int c = 0; c < NC; ++c) re[q][c] = im[q][c] = 0.0;
  for (int jt = j0; jt < j1; jt += kPTJ) {
    const int cnt = min(kPTJ, j1 - jt);
    __syncthreads();
    for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
      tile[t] = make_rec<TGT>(R, Fe, Te, Sig, D, jt + t, P, a5_20);
      double sn, cs;
      sincos(dk * tile[t].z, &sn, &cs);
      wre[t] = cs;
      wim[t] = -sn;
    }
    __syncthreads();
    for (int jj = 0; jj < cnt; ++jj) {
      const RecP& s = tile[jj];
      double sn, cs;
      sincos(fma(k1, s.x, fma(k2, s.y, k3 * s.z)), &sn, &cs);
      double pr = cs, pi = -sn;  // exp(-i k.R_m) at the segment's first wave vector
      const double wr = wre[jj], wi = wim[jj];
      double v[NC];
      coeffs<TGT>(s, v);
#pragma unroll
      for (int q = 0; q < S; ++q) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          re[q][c] = fma(v[c], pr, re[q][c]);
          im[q][c] = fma(v[c], pi, im[q][c]);
        }
        const double t = pr * wr - pi * wi;
        pi = fma(pr, wi, pi * wr);
        pr = t;
      }
    }
  }
  if (g >= nseg) return;
#pragma unroll
  for (int q = 0; q < S; ++q) {
    if (q < sg.y) {
      double* o = sf + ((int64_t)blockIdx.y * K + sg.x + q) * (2 * NC);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        o[c] = re[q][c];
        o[NC + c] = im[q][c];
      }
    }
  }
}

// T[k * 2W] = (2 / L^3) phi(k) M(k) S(k): the chunks' structure factors added in order, the
// generated multiplier applied
template <int TGT>
__global__ void __launch_bounds__(kPKBlk)
    k_per_mult(const double* __restrict__ sf, int nchunk, const double* __restrict__ kv, int K, double xi, double a2,
               double scale, double* __restrict__ T) {
  constexpr int NC = pnc(TGT), W = pw(TGT);
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  double v[2 * NC];
#pragma unroll
  for (int c = 0; c < 2 * NC; ++c) v[c] = 0.0;
  for (int ch = 0; ch < nchunk; ++ch) {
    const double* p = sf + ((int64_t)ch * K + k) * (2 * NC);
#pragma unroll
    for (int c = 0; c < 2 * NC; ++c) v[c] += p[c];
  }
  const double k1 = kv[3 * (int64_t)k], k2 = kv[3 * (int64_t)k + 1], k3 = kv[3 * (int64_t)k + 2];
  const double ksq = fma(k1, k1, fma(k2, k2, k3 * k3));
  const double ik2 = 1.0 / ksq;
  const double q = ksq / (4.0 * xi * xi);
  const double g = scale * (1.0 + q) * exp(-q);
  double tr[W], ti[W];
  const double* re = v;
  const double* im = v + NC;
  if (TGT == kPOp) per_hat_strain_s(k1, k2, k3, ik2, a2, re, im, tr, ti);
  if (TGT == kPRhs) per_hat_strain_ftq(k1, k2, k3, ik2, a2, re, im, re + 3, im + 3, re + 6, im + 6, tr, ti);
  if (TGT == kPOut)
    per_hat_motion_ftsq(k1, k2, k3, ik2, a2, re, im, re + 3, im + 3, re + 6, im + 6, re + 11, im + 11, tr, ti);
  if (TGT == kPFlow)
    per_hat_flow_ftsq(k1, k2, k3, ik2, a2, re, im, re + 3, im + 3, re + 6, im + 6, re + 11, im + 11, tr, ti);
  double* o = T + (int64_t)k * (2 * W);
#pragma unroll
  for (int c = 0; c < W; ++c) {
    o[c] = g * tr[c];
    o[W + c] = g * ti[c];
  }
}

// part[(chunk * n + i) * W] = Re sum_{k in chunk} exp(i k.R_i) T(k)
template <int TGT>
__global__ void __launch_bounds__(kPBlk)
    k_per_recip(const double* __restrict__ R, int n, const double* __restrict__ kv, const double* __restrict__ T,
                int K, double dk, int chunk, double* __restrict__ part) {
  constexpr int W = pw(TGT);
  __shared__ double tk[kPKT][3 + 2 * W];
  __shared__ int step[kPKT];  // 1: same lattice row as the previous wave vector, next k3
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int ii = i < n ? i : n - 1;
  const double x = R[3 * (int64_t)ii], y = R[3 * (int64_t)ii + 1], z = R[3 * (int64_t)ii + 2];
  double wr, wi;  // exp(i dk z): one step along a row
  sincos(dk * z, &wi, &wr);
  const int k0 = blockIdx.y * chunk;
  const int k1e = min(K, k0 + chunk);
  double acc[W];
#pragma unroll
  for (int c = 0; c < W; ++c) acc[c] = 0.0;
  double cs = 1.0, sn = 0.0;
  int run = 0;  // steps since the last sincos (a fresh one every 16 bounds the rounding carried along)
  for (int kt = k0; kt < k1e; kt += kPKT) {
    const int cnt = min(kPKT, k1e - kt);
    __syncthreads();
    for (int t = threadIdx.x; t < cnt * (3 + 2 * W); t += blockDim.x) {
      const int q = t / (3 + 2 * W), c = t % (3 + 2 * W);
      tk[q][c] = c < 3 ? kv[3 * (int64_t)(kt + q) + c] : T[(int64_t)(kt + q) * (2 * W) + (c - 3)];
    }
    for (int q = threadIdx.x; q < cnt; q += blockDim.x) {
      const int k = kt + q;  // the chunk's first wave vector always starts afresh
      step[q] = (k > k0 && kv[3 * (int64_t)k] == kv[3 * (int64_t)(k - 1)] &&
                 kv[3 * (int64_t)k + 1] == kv[3 * (int64_t)(k - 1) + 1] &&
                 fabs(kv[3 * (int64_t)k + 2] - kv[3 * (int64_t)(k - 1) + 2] - dk) < 0.5 * dk) ? 1 : 0;
    }
    __syncthreads();
    for (int q = 0; q < cnt; ++q) {
      if (step[q] && run < 16) {  // uniform across the workgroup
        const double t = cs * wr - sn * wi;
        sn = fma(cs, wi, sn * wr);
        cs = t;
        ++run;
      } else {
        sincos(fma(tk[q][0], x, fma(tk[q][1], y, tk[q][2] * z)), &sn, &cs);
        run = 0;
      }
#pragma unroll
      for (int c = 0; c < W; ++c) acc[c] = fma(tk[q][3 + c], cs, fma(-tk[q][3 + W + c], sn, acc[c]));
    }
  }
  if (i >= n) return;
  double* o = part + ((int64_t)blockIdx.y * n + i) * W;
#pragma unroll
  for (int c = 0; c < W; ++c) o[c] = acc[c];
}

// the chunks added in order, then
//   operator:  y = x (1/gamma + P c_es) - real - recip                  (out = y)
//   rhs:       b = real + recip - c_slip v2s                             (out = b)
//   outputs:   V = real + recip + mu_t F - P c_uf F - (a^5/20) c_ud d - v1s, W = real + recip + mu_r T
//              - P c_wt T, S = Sigma + slip_S v2s                        (out = V, out2 = W, out3 = S)
template <int TGT>
__global__ void k_per_finish(const double* __restrict__ preal, int nreal, const double* __restrict__ precip,
                             int nrecip, int n, const double* __restrict__ X, const double* __restrict__ Fe,
                             const double* __restrict__ Te, const double* __restrict__ D,
                             const double* __restrict__ v1s, const double* __restrict__ v2s, double self0,
                             double self1, double self2, const Phys ph, double* __restrict__ out,
                             double* __restrict__ out2, double* __restrict__ out3) {
  constexpr int W = pw(TGT);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc[W];
  for (int c = 0; c < W; ++c) acc[c] = 0.0;
  for (int ch = 0; ch < nreal; ++ch)
    for (int c = 0; c < W; ++c) acc[c] += preal[((int64_t)ch * n + i) * W + c];
  for (int ch = 0; ch < nrecip; ++ch)
    for (int c = 0; c < W; ++c) acc[c] += precip[((int64_t)ch * n + i) * W + c];
  if (TGT == kPFlow) {
    for (int c = 0; c < 3; ++c) out[3 * (int64_t)i + c] = acc[c];
  } else if (TGT == kPOp) {
    for (int c = 0; c < 5; ++c) out[5 * (int64_t)i + c] = X[5 * (int64_t)i + c] * (ph.inv_gamma + self0) - acc[c];
  } else if (TGT == kPRhs) {
    for (int c = 0; c < 5; ++c) out[5 * (int64_t)i + c] = acc[c] - (v2s ? ph.c_slip * v2s[5 * (int64_t)i + c] : 0.0);
  } else {
    for (int c = 0; c < 3; ++c) {
      const double F = Fe ? Fe[3 * (int64_t)i + c] : 0.0, Tq = Te ? Te[3 * (int64_t)i + c] : 0.0;
      const double d = D ? D[3 * (int64_t)i + c] : 0.0;
      out[3 * (int64_t)i + c] = acc[c] + (ph.mu_t - self0) * F - self1 * d - (v1s ? v1s[3 * (int64_t)i + c] : 0.0);
      out2[3 * (int64_t)i + c] = acc[3 + c] + (ph.mu_r - self2) * Tq;
    }
    for (int c = 0; c < 5; ++c)
      out3[5 * (int64_t)i + c] = X[5 * (int64_t)i + c] + (v2s ? ph.slip_S * v2s[5 * (int64_t)i + c] : 0.0);
  }
}

// the smallest minimum-image distance squared of each workgroup's receivers to every other sphere:
// part[block] (all pairs, positions staged through LDS)
// (skip: when given and *skip < edge, the cell search already found the minimum: nothing to do)
__global__ void __launch_bounds__(256) k_per_min_d2(const double* __restrict__ R, int n, double L, double invL,
                                                    double* __restrict__ part, const double* __restrict__ skip,
                                                    double edge) {
  if (skip && *skip < edge) return;
  __shared__ double tx[256], ty[256], tz[256], red[256];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int ii = i < n ? i : n - 1;
  const double x = R[3 * (int64_t)ii], y = R[3 * (int64_t)ii + 1], z = R[3 * (int64_t)ii + 2];
  double best = INFINITY;
  for (int jt = 0; jt < n; jt += 256) {
    const int cnt = min(256, n - jt);
    __syncthreads();
    if ((int)threadIdx.x < cnt) {
      tx[threadIdx.x] = R[3 * (int64_t)(jt + threadIdx.x)];
      ty[threadIdx.x] = R[3 * (int64_t)(jt + threadIdx.x) + 1];
      tz[threadIdx.x] = R[3 * (int64_t)(jt + threadIdx.x) + 2];
    }
    __syncthreads();
    for (int jj = 0; jj < cnt; ++jj) {
      if (jt + jj == ii) continue;
      const double dx = wrap(x - tx[jj], L, invL), dy = wrap(y - ty[jj], L, invL), dz = wrap(z - tz[jj], L, invL);
      best = fmin(best, fma(dx, dx, fma(dy, dy, dz * dz)));
    }
  }
  red[threadIdx.x] = i < n ? best : INFINITY;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// the smallest minimum-image distance squared from each sphere (box grid order, at least 3 cells per
// axis) to the others in its 27 neighbouring cells: part[block]
__global__ void __launch_bounds__(256) k_pm_min_d2(const GridHdr* __restrict__ hdr, const double* __restrict__ Rs,
                                                   const int32_t* __restrict__ cstart, const int32_t* __restrict__ cend,
                                                   int nc, int n, double L, double invL, double* __restrict__ part) {
  __shared__ double red[256];
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  double best = INFINITY;
  if (k < n) {
    const GridHdr H = *hdr;
    const double x = Rs[4 * (int64_t)k], y = Rs[4 * (int64_t)k + 1], z = Rs[4 * (int64_t)k + 2];
    const int cx = grid_cell1(x, 0.0, H.inv_h, nc), cy = grid_cell1(y, 0.0, H.inv_h, nc),
              cz = grid_cell1(z, 0.0, H.inv_h, nc);
    for (int nb = 0; nb < 27; ++nb) {
      const int jx = (cx + nb % 3 - 1 + nc) % nc, jy = (cy + (nb / 3) % 3 - 1 + nc) % nc,
                jz = (cz + nb / 9 - 1 + nc) % nc;
      const int c = (jz * nc + jy) * nc + jx;
      for (int j = cstart[c]; j < cend[c]; ++j) {
        if (j == k) continue;
        const double dx = wrap(x - Rs[4 * (int64_t)j], L, invL), dy = wrap(y - Rs[4 * (int64_t)j + 1], L, invL),
                     dz = wrap(z - Rs[4 * (int64_t)j + 2], L, invL);
        best = fmin(best, fma(dx, dx, fma(dy, dy, dz * dz)));
      }
    }
  }
  red[threadIdx.x] = best;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// out[0] = sqrt(min over the nb partial minima) (unless skip is given and out[0] < edge already)
__global__ void __launch_bounds__(256) k_min_finish(const double* __restrict__ part, int nb, double* __restrict__ out,
                                                    bool skip, double edge) {
  if (skip && out[0] < edge) return;
  __shared__ double red[256];
  double m = INFINITY;
  for (int k = threadIdx.x; k < nb; k += blockDim.x) m = fmin(m, part[k]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sqrt(red[0]);
}

// ---------------------------------------------------------------- smooth particle-mesh Ewald
// The smooth particle-mesh Ewald method (Essmann, Perera, Berkowitz, Darden, Lee and Pedersen,
// J. Chem. Phys. 103, 8577, 1995), applied here to the Stokes blocks of every pass.
// With a mesh of M^3 points (spacing h = L / M) the Fourier sum runs on the mesh instead of over the
// spheres: exp(-i k.R) is interpolated by cardinal B-splines of order kPmP on the mesh points around
// R (Euler exponential splines, the interpolation's error corrected in Fourier space by |b(m)|^2),
// so the structure factors become one discrete Fourier transform of the source coefficients spread
// onto the mesh, the multiplier is applied per mesh wave vector, and the inverse transform is
// interpolated back at the receivers with the same weights: O(N P^3 + M^3 log M) instead of O(N K).
constexpr int kPmP = 8;    // B-spline order (support of P mesh points per axis)
constexpr int kPmB = 8;    // mesh block edge of the spreading kernel
constexpr int kPmT = 64;   // candidate sources per LDS tile of the spreading kernel

// Workgroups are dealt round-robin over the 8 XCDs, each with its own L2: renumber the first 8 floor(n/8)
// of n so that every XCD takes a contiguous run (neighbouring cells or receivers, which share sources
// and mesh points), the rest unchanged
__device__ __forceinline__ int xcd_order(int b, int n) {
  const int q = n >> 3;
  return b >= 8 * q ? b : (b & 7) * q + (b >> 3);
}

// the weights of mesh points b0 + o, o = 0..P-1, for a scaled coordinate u = floor(u) + t with
// b0 = floor(u) - P + 1: w[o] = M_P(t + P - 1 - o), the B-spline built up from order 2 by its
// two-term recursion M_n(x) = (x M_{n-1}(x) + (n - x) M_{n-1}(x - 1)) / (n - 1)
__host__ __device__ inline void bspline_w(double t, double* w) {
  double v[kPmP];  // v[o] = M_n(t + o), o < n
  v[0] = t;
  v[1] = 1.0 - t;
  for (int n = 3; n <= kPmP; ++n) {
    const double inv = 1.0 / (n - 1);
    v[n - 1] = (1.0 - t) * v[n - 2] * inv;
    for (int o = n - 2; o >= 1; --o) v[o] = ((t + o) * v[o] + (n - t - o) * v[o - 1]) * inv;
    v[0] = t * v[0] * inv;
  }
  for (int o = 0; o < kPmP; ++o) w[o] = v[kPmP - 1 - o];
}

// the c-th source coefficient of sphere j, in the order the structure factors hold them
template <int TGT>
__device__ __forceinline__ double pm_coef(int c, int64_t j, const double* __restrict__ Fe,
                                          const double* __restrict__ Te, const double* __restrict__ Sig,
                                          const double* __restrict__ D, double P, double a5_20) {
  if (TGT == kPOp) return Sig ? P * Sig[5 * j + c] : 0.0;
  if (TGT == kPRhs) {
    if (c < 3) return Fe ? P * Fe[3 * j + c] : 0.0;
    if (c < 6) return Te ? P * Te[3 * j + c - 3] : 0.0;
    return D ? a5_20 * D[3 * j + c - 6] : 0.0;
  }
  if (c < 3) return Fe ? P * Fe[3 * j + c] : 0.0;
  if (c < 6) return Te ? P * Te[3 * j + c - 3] : 0.0;
  if (c < 11) return Sig ? P * Sig[5 * j + c - 6] : 0.0;
  return D ? a5_20 * D[3 * j + c - 11] : 0.0;
}

// per sphere in the box grid's order (wrapped centres Rs): first mesh point and weights per axis
__global__ void __launch_bounds__(256) k_pm_prep(const double* __restrict__ Rs, int n, int M, double inv_h,
                                                 int* __restrict__ b0, double* __restrict__ wts) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  for (int d = 0; d < 3; ++d) {
    const double u = Rs[4 * (int64_t)k + d] * inv_h;
    const double fu = floor(u);
    double w[kPmP];
    bspline_w(u - fu, w);
    b0[4 * (int64_t)k + d] = ((int)fu - (kPmP - 1)) & (M - 1);
    for (int o = 0; o < kPmP; ++o) wts[(3 * (int64_t)k + d) * kPmP + o] = w[o];
  }
  b0[4 * (int64_t)k + 3] = 0;
}

// the real-space pass over the sources' box grid (cells of edge >= rc, at least 3 per axis, so a
// receiver's partners within rc lie in its own and the 26 neighbouring cells, each met once), the
// receivers from a box grid of the same cells (the spheres' own, or the field points'): a
// workgroup per (cell, layer of neighbouring cells along z), its receivers 128 at a time, the 9 cells
// of the layer staged through LDS with the same bit-mask evaluation as k_per_real; partial sums
// part[(layer * m + i) * W] at the receivers' own indices
constexpr int kPmRT = 128;  // threads of the cell real-space kernel (receivers per round)



template <int TGT>
__global__ void __launch_bounds__(kPmRT)
    k_pm_real(const double* __restrict__ RsR, const int32_t* __restrict__ permR, const int32_t* __restrict__ cstartR,
              const int32_t* __restrict__ cendR, const double* __restrict__ Rs, const int32_t* __restrict__ perm,
              const int32_t* __restrict__ cstart, const int32_t* __restrict__ cend, int nc, int m,
              const double* __restrict__ Fe,
              const double* __restrict__ Te, const double* __restrict__ Sig, const double* __restrict__ D, double L,
              double rc2, double xi, double a2, double P, double a5_20, const double* __restrict__ rtab,
              int npiece, double inv_slo, double* __restrict__ part) {
  __shared__ RecP tile[kPTJ];
  extern __shared__ double rt[];  // the operator's radial table (npiece pieces), when given
  constexpr int W = pw(TGT);
  if (rtab) {
    for (int i = threadIdx.x; i < npiece * kRtC; i += blockDim.x) rt[i] = rtab[i];
    __syncthreads();
  }
  const int cell = (gridDim.x & 7) ? (int)blockIdx.x : xcd_order(blockIdx.x, gridDim.x);
  const int ix = cell % nc, iy = (cell / nc) % nc, iz = cell / (nc * nc);
  const int jzr = iz + (int)blockIdx.y - 1;
  const int jz = (jzr + nc) % nc;
  const double shz = jzr < 0 ? -L : (jzr >= nc ? L : 0.0);
  const int r0 = cstartR[cell], r1 = cendR[cell];
  for (int rb = r0; rb < r1; rb += kPmRT) {
    const int k = rb + threadIdx.x;
    const int kk = k < r1 ? k : r1 - 1;
    const double xi0 = RsR[4 * (int64_t)kk], yi0 = RsR[4 * (int64_t)kk + 1], zi0 = RsR[4 * (int64_t)kk + 2];
    double acc[W];
#pragma unroll
    for (int c = 0; c < W; ++c) acc[c] = 0.0;
    for (int nb = 0; nb < 9; ++nb) {
      const int jxr = ix + nb % 3 - 1, jyr = iy + nb / 3 - 1;  // neighbour cell before wrapping
      const int jx = (jxr + nc) % nc, jy = (jyr + nc) % nc;
      const int sc = (jz * nc + jy) * nc + jx;
      // the neighbour's spheres moved by whole boxes to the cell's side of the receiver's: with cells
      // of at least rc and 3 or more per axis this is the minimum image of every pair within rc
      const double shx = jxr < 0 ? -L : (jxr >= nc ? L : 0.0), shy = jyr < 0 ? -L : (jyr >= nc ? L : 0.0);
      const int s0 = cstart[sc], s1 = cend[sc];
      for (int jt = s0; jt < s1; jt += kPTJ) {
        const int cnt = min(kPTJ, s1 - jt);
        __syncthreads();
        for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
          const int64_t j = perm[jt + t];
          RecP r;
          r.pad = 0.0;
          r.x = Rs[4 * (int64_t)(jt + t)] + shx;
          r.y = Rs[4 * (int64_t)(jt + t) + 1] + shy;
          r.z = Rs[4 * (int64_t)(jt + t) + 2] + shz;
          for (int c = 0; c < 3; ++c) {
            r.f[c] = (TGT != kPOp && Fe) ? P * Fe[3 * j + c] : 0.0;
            r.t[c] = (TGT != kPOp && Te) ? P * Te[3 * j + c] : 0.0;
            r.q[c] = (TGT != kPOp && D) ? a5_20 * D[3 * j + c] : 0.0;
          }
          for (int c = 0; c < 5; ++c) r.s[c] = (TGT != kPRhs && Sig) ? P * Sig[5 * j + c] : 0.0;
          tile[t] = r;
        }
        __syncthreads();
        uint64_t hits = 0;
#pragma unroll 8
        for (int q = 0; q < cnt; ++q) {
          const double dx = xi0 - tile[q].x, dy = yi0 - tile[q].y, dz = zi0 - tile[q].z;
          const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
          hits |= (uint64_t)(r2 < rc2 && r2 > 0.0) << q;
        }
        if (k >= r1) hits = 0;  // (a lane past the cell's last receiver)
        tile_hits<TGT, false>(tile, hits, xi0, yi0, zi0, L, 0.0, xi, a2, acc, rtab ? rt : nullptr, npiece, inv_slo);
      }
    }
    if (k < r1) {
      double* o = part + ((int64_t)blockIdx.y * m + permR[k]) * W;
#pragma unroll
      for (int c = 0; c < W; ++c) o[c] = acc[c];
    }
  }
}

// Q_c(g) = sum_j c_j W_j(g) on one 8^3 block of the mesh, coefficients [C0, C0 + CN) (C0 even),
// written in pairs as complex fields (Q_{C0}, Q_{C0+1}), ... from field C0/2 on. A thread holds one
// line of 8 points along x. The candidate spheres (those binned in the cells that reach the block)
// are taken 64 at a time in the grid's order; those whose P^3 points overlap the block (a few
// percent of them) are compacted by a ballot, in order, and only their weights and coefficients go
// through LDS, so every point adds its terms in one fixed order.
template <int TGT, int C0, int CN>
__global__ void __launch_bounds__(64)
    k_pm_spread(const int32_t* __restrict__ perm, const int32_t* __restrict__ cstart,
                const int32_t* __restrict__ cend, const int* __restrict__ b0, const double* __restrict__ wts,
                const double* __restrict__ Fe, const double* __restrict__ Te, const double* __restrict__ Sig,
                const double* __restrict__ D, double P, double a5_20, int M, int nc, double2* __restrict__ fld) {
  __shared__ int tb[kPmT][4];
  __shared__ double tw[kPmT][3 * kPmP];
  __shared__ double tc[kPmT][CN];
  const int nb = M / kPmB;
  const int bx = blockIdx.x % nb, by = (blockIdx.x / nb) % nb, bz = blockIdx.x / (nb * nb);
  const int G0[3] = {bx * kPmB, by * kPmB, bz * kPmB};
  const int gy = G0[1] + (threadIdx.x & 7), gz = G0[2] + (threadIdx.x >> 3);
  double acc[kPmB][CN];
#pragma unroll
  for (int x = 0; x < kPmB; ++x)
#pragma unroll
    for (int c = 0; c < CN; ++c) acc[x][c] = 0.0;
  // cells holding centres with floor(u) in [G0, G0 + B + P - 1) per axis, with a margin for rounding
  int lo[3], cnt[3];
  const double cpm = (double)nc / M;  // cells per mesh spacing
  for (int d = 0; d < 3; ++d) {
    lo[d] = (int)floor((G0[d] - 1e-6) * cpm);
    const int hi = (int)floor((G0[d] + kPmB + kPmP - 1 + 1e-6) * cpm);
    cnt[d] = min(hi - lo[d] + 1, nc);
  }
  for (int cz = 0; cz < cnt[2]; ++cz)
    for (int cy = 0; cy < cnt[1]; ++cy)
      for (int cx = 0; cx < cnt[0]; ++cx) {
        const int ix = ((lo[0] + cx) % nc + nc) % nc, iy = ((lo[1] + cy) % nc + nc) % nc,
                  iz = ((lo[2] + cz) % nc + nc) % nc;
        const int cell = (iz * nc + iy) * nc + ix;
        const int s0 = cstart[cell], s1 = cend[cell];
        for (int st = s0; st < s1; st += kPmT) {
          const int k = st + threadIdx.x;
          int bq[3] = {0, 0, 0};
          bool in = k < s1;
          if (in) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
              bq[d] = b0[4 * (int64_t)k + d];
              in = in && (((G0[d] - bq[d]) & (M - 1)) < kPmP || ((bq[d] - G0[d]) & (M - 1)) < kPmB);
            }
          }
          const uint64_t mask = __ballot(in);
          const int m = __popcll(mask);
          if (m == 0) continue;  // (uniform: one wavefront per workgroup)
          __syncthreads();
          if (in) {
            const int pos = __popcll(mask & ((1ull << threadIdx.x) - 1ull));
            const int64_t j = perm[k];
            for (int d = 0; d < 3; ++d) tb[pos][d] = bq[d];
            for (int o = 0; o < 3 * kPmP; ++o) tw[pos][o] = wts[3 * kPmP * (int64_t)k + o];
#pragma unroll
            for (int c = 0; c < CN; ++c) tc[pos][c] = pm_coef<TGT>(C0 + c, j, Fe, Te, Sig, D, P, a5_20);
          }
          __syncthreads();
          for (int q = 0; q < m; ++q) {
            const int oy = (gy - tb[q][1]) & (M - 1), oz = (gz - tb[q][2]) & (M - 1);
            if (oy >= kPmP || oz >= kPmP) continue;
            const double wyz = tw[q][kPmP + oy] * tw[q][2 * kPmP + oz];
#pragma unroll
            for (int x = 0; x < kPmB; ++x) {
              const int ox = (G0[0] + x - tb[q][0]) & (M - 1);
              if (ox < kPmP) {
                const double w = wyz * tw[q][ox];
#pragma unroll
                for (int c = 0; c < CN; ++c) acc[x][c] = fma(w, tc[q][c], acc[x][c]);
              }
            }
          }
        }
      }
  const int64_t M3 = (int64_t)M * M * M;
#pragma unroll
  for (int x = 0; x < kPmB; ++x) {
    const int64_t idx = ((int64_t)gz * M + gy) * M + G0[0] + x;
#pragma unroll
    for (int f = 0; f < (CN + 1) / 2; ++f)
      fld[(int64_t)f * M3 + idx] = make_double2(acc[x][2 * f], 2 * f + 1 < CN ? acc[x][2 * f + 1] : 0.0);
  }
}

// Radix-4 and radix-8 DFTs in registers: forward exp(-2 pi i q r / R), INV the conjugate.
template <bool INV>
__device__ __forceinline__ void dft4(double2& a0, double2& a1, double2& a2, double2& a3) {
  const double2 t0 = make_double2(a0.x + a2.x, a0.y + a2.y), t1 = make_double2(a0.x - a2.x, a0.y - a2.y);
  const double2 t2 = make_double2(a1.x + a3.x, a1.y + a3.y);
  const double2 d = make_double2(a1.x - a3.x, a1.y - a3.y);
  const double2 t3 = INV ? make_double2(-d.y, d.x) : make_double2(d.y, -d.x);  // (a1 - a3) times -i (i: INV)
  a0 = make_double2(t0.x + t2.x, t0.y + t2.y);
  a2 = make_double2(t0.x - t2.x, t0.y - t2.y);
  a1 = make_double2(t1.x + t3.x, t1.y + t3.y);
  a3 = make_double2(t1.x - t3.x, t1.y - t3.y);
}

template <int R, bool INV>
__device__ __forceinline__ void dft_small(double2* v) {
  if (R == 4) {
    dft4<INV>(v[0], v[1], v[2], v[3]);
  } else {  // 8: the even and odd halves, then exp(-/+ 2 pi i k / 8) on the odd ones
    double2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6], o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<INV>(e0, e1, e2, e3);
    dft4<INV>(o0, o1, o2, o3);
    const double c = 0.70710678118654752440;
    o1 = INV ? make_double2(c * (o1.x - o1.y), c * (o1.x + o1.y)) : make_double2(c * (o1.x + o1.y), c * (o1.y - o1.x));
    o2 = INV ? make_double2(-o2.y, o2.x) : make_double2(o2.y, -o2.x);
    o3 = INV ? make_double2(-c * (o3.x + o3.y), c * (o3.x - o3.y)) : make_double2(c * (o3.y - o3.x), -c * (o3.x + o3.y));
    v[0] = make_double2(e0.x + o0.x, e0.y + o0.y);
    v[4] = make_double2(e0.x - o0.x, e0.y - o0.y);
    v[1] = make_double2(e1.x + o1.x, e1.y + o1.y);
    v[5] = make_double2(e1.x - o1.x, e1.y - o1.y);
    v[2] = make_double2(e2.x + o2.x, e2.y + o2.y);
    v[6] = make_double2(e2.x - o2.x, e2.y - o2.y);
    v[3] = make_double2(e3.x + o3.x, e3.y + o3.y);
    v[7] = make_double2(e3.x - o3.x, e3.y - o3.y);
  }
}

// LDS slot of point idx of line l: rows of M points, the low 4 bits of idx swizzled by the line so
// that lanes reading the same point of consecutive lines meet different banks
__device__ __forceinline__ int fft_slot(int l, int idx, int M) { return l * M + (idx ^ (l & 15)); }

struct FftPlan {
  int nst;
  int r[6];  // radix of each stage (8 or 4), product M
};

// One radix-R Stockham stage over the B lines of a bundle: butterfly j (< M/R) of line l takes the
// points j + r M/R, multiplies them by exp(-/+ 2 pi i r k / (Ns R)) (k = j mod Ns, Ns the product of
// the earlier radices), transforms them and puts them at (j - k) R + k + r Ns: natural order in and
// out. The first stage reads the line from memory and the last one writes it back; the others work
// in LDS, every thread reading all its points before the barrier and writing after it.
template <int R, bool INV, bool CONTIG>
__device__ __forceinline__ void fft_stage(double2* xs, double2* g, bool from_g, bool to_g, int M, int B, int Ns,
                                          int64_t sk, int64_t sb, const double2* __restrict__ tw) {
  constexpr int NB = 16 / R;  // butterflies per thread (B M <= 16 threads)
  const int MR = M / R, nbf = B * MR;
  double2 v[NB][R];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int e = threadIdx.x + q * blockDim.x;
    if (e < nbf) {
      const int l = CONTIG ? e / MR : e % B, j = CONTIG ? e % MR : e / B;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int idx = j + r * MR;
        v[q][r] = from_g ? g[(int64_t)l * sb + (CONTIG ? (int64_t)idx : (int64_t)idx * sk)] : xs[fft_slot(l, idx, M)];
      }
      const int k = j & (Ns - 1), step = M / (Ns * R);
#pragma unroll
      for (int r = 1; r < R; ++r) {
        double2 w = tw[r * k * step];
        if (INV) w.y = -w.y;
        const double2 x = v[q][r];
        v[q][r] = make_double2(w.x * x.x - w.y * x.y, fma(w.x, x.y, w.y * x.x));
      }
      dft_small<R, INV>(v[q]);
    }
  }
  if (!from_g) __syncthreads();
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int e = threadIdx.x + q * blockDim.x;
    if (e < nbf) {
      const int l = CONTIG ? e / MR : e % B, j = CONTIG ? e % MR : e / B;
      const int k = j & (Ns - 1), o = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int idx = o + r * Ns;
        if (to_g)
          g[(int64_t)l * sb + (CONTIG ? (int64_t)idx : (int64_t)idx * sk)] = v[q][r];
        else
          xs[fft_slot(l, idx, M)] = v[q][r];
      }
    }
  }
  if (!to_g) __syncthreads();
}

// One pass of the 3D transform: every line of M points along one axis (point idx of line l of a
// bundle at base + l sb + idx sk), B lines per workgroup (consecutive in memory for the strided axes,
// so that B contiguous points move together). Forward: X(m) = sum_g x(g) exp(-2 pi i m g / M); INV:
// the conjugate exponent, no normalisation. AXIS 0 is the contiguous one (sk = 1). B M / 16 threads.
template <bool INV, int AXIS>
__global__ void __launch_bounds__(512)
    k_fft_lines(double2* __restrict__ a, int M, int B, int64_t sk, int64_t sb, int nbu, int64_t su, int64_t sv,
                int64_t sf, const double2* __restrict__ tw, FftPlan pl) {
  extern __shared__ double2 xs[];
  // workgroups are dealt round-robin over the 8 XCDs: renumber them so that each XCD takes a
  // contiguous run of bundles (neighbouring lines share pages and its L2)
  const int nwg = gridDim.x;
  const int id = (nwg & 7) ? (int)blockIdx.x : (int)(blockIdx.x & 7) * (nwg >> 3) + (int)(blockIdx.x >> 3);
  const int bu = id % nbu, bv = id / nbu;
  double2* base = a + (int64_t)blockIdx.y * sf + (int64_t)bu * su + (int64_t)bv * sv;
  int Ns = 1;
  for (int st = 0; st < pl.nst; ++st) {
    const bool first = st == 0, last = st == pl.nst - 1;
    if (pl.r[st] == 8)
      fft_stage<8, INV, AXIS == 0>(xs, base, first, last, M, B, Ns, sk, sb, tw);
    else
      fft_stage<4, INV, AXIS == 0>(xs, base, first, last, M, B, Ns, sk, sb, tw);
    Ns *= pl.r[st];
  }
}

// At mesh wave vector m = (x, y, z) (k = 2 pi m / L, |m_d| < M/2, m != 0): the coefficients'
// transforms separated from the packed fields at m (zp) and -m (zm) (Z = Q_{2a} + i Q_{2a+1}:
// Q_{2a}(m) = (Z(m) + conj Z(-m)) / 2, Q_{2a+1}(m) = (Z(m) - conj Z(-m)) / 2i), the generated
// multiplier applied with the splitting factor, |b(m)|^2 and 1 / L^3, the targets packed again in
// pairs (T_{2b} + i T_{2b+1}) into Y; zero at m = 0 and on the Nyquist planes.
template <int TGT>
__device__ __forceinline__ void pm_point(const double2* zp, const double2* zm, int x, int y, int z, int M, double dk,
                                         double xi, double a2, double invL3, const double* __restrict__ bmod,
                                         double2* Y) {
  constexpr int NC = pnc(sft(TGT)), W = pw(TGT), NI = (NC + 1) / 2, NO = (W + 1) / 2;
  const int h = M >> 1;
  if ((x == 0 && y == 0 && z == 0) || x == h || y == h || z == h) {
#pragma unroll
    for (int b = 0; b < NO; ++b) Y[b] = make_double2(0.0, 0.0);
    return;
  }
  double re[2 * NI], im[2 * NI];
#pragma unroll
  for (int a = 0; a < NI; ++a) {
    re[2 * a] = 0.5 * (zp[a].x + zm[a].x);
    im[2 * a] = 0.5 * (zp[a].y - zm[a].y);
    re[2 * a + 1] = 0.5 * (zp[a].y + zm[a].y);
    im[2 * a + 1] = 0.5 * (zm[a].x - zp[a].x);
  }
  const double k1 = dk * (x < h ? x : x - M), k2 = dk * (y < h ? y : y - M), k3 = dk * (z < h ? z : z - M);
  const double ksq = fma(k1, k1, fma(k2, k2, k3 * k3));
  const double ik2 = 1.0 / ksq;
  const double q = ksq / (4.0 * xi * xi);
  const double g = invL3 * (1.0 + q) * exp(-q) * bmod[x] * bmod[y] * bmod[z];
  double tr[2 * NO], ti[2 * NO];
  tr[2 * NO - 1] = ti[2 * NO - 1] = 0.0;
  if (TGT == kPOp) per_hat_strain_s(k1, k2, k3, ik2, a2, re, im, tr, ti);
  if (TGT == kPRhs) per_hat_strain_ftq(k1, k2, k3, ik2, a2, re, im, re + 3, im + 3, re + 6, im + 6, tr, ti);
  if (TGT == kPOut)
    per_hat_motion_ftsq(k1, k2, k3, ik2, a2, re, im, re + 3, im + 3, re + 6, im + 6, re + 11, im + 11, tr, ti);
  if (TGT == kPFlow)
    per_hat_flow_ftsq(k1, k2, k3, ik2, a2, re, im, re + 3, im + 3, re + 6, im + 6, re + 11, im + 11, tr, ti);
#pragma unroll
  for (int b = 0; b < NO; ++b) Y[b] = make_double2(g * (tr[2 * b] - ti[2 * b + 1]), g * (ti[2 * b] + tr[2 * b + 1]));
}

// the multiplier at every mesh point, from the transformed packed fields (all three axes)
template <int TGT>
__global__ void __launch_bounds__(256)
    k_pm_mult(const double2* __restrict__ fin, int M, double dk, double xi, double a2, double invL3,
              const double* __restrict__ bmod, double2* __restrict__ fout) {
  constexpr int NC = pnc(sft(TGT)), W = pw(TGT), NI = (NC + 1) / 2, NO = (W + 1) / 2;
  const int64_t M3 = (int64_t)M * M * M;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= M3) return;
  const int x = (int)(idx % M), y = (int)((idx / M) % M), z = (int)(idx / ((int64_t)M * M));
  const int64_t nidx = ((int64_t)((M - z) & (M - 1)) * M + ((M - y) & (M - 1))) * M + ((M - x) & (M - 1));
  double2 zp[NI], zm[NI], Y[NO];
#pragma unroll
  for (int a = 0; a < NI; ++a) {
    zp[a] = fin[(int64_t)a * M3 + idx];
    zm[a] = fin[(int64_t)a * M3 + nidx];
  }
  pm_point<TGT>(zp, zm, x, y, z, M, dk, xi, a2, invL3, bmod, Y);
#pragma unroll
  for (int b = 0; b < NO; ++b) fout[(int64_t)b * M3 + idx] = Y[b];
}

// The x transforms fused with the multiplier: one x line (y, z) of the packed fields and its mirror
// line (-y, -z) (the multiplier at m needs the packed inputs at -m, which lie on the mirror line)
// read once into LDS after the y and z transforms, transformed along x, multiplied point pair by
// point pair (m on this line with -m on the mirror line, each thread reading its pairs before the
// barrier and writing after it), transformed back along x and written to the output fields, which
// then take the inverse y and z transforms. Workgroups enumerate one line of each mirror pair: every y
// for 0 < z < M/2, and 0 <= y <= M/2 for z = 0 and z = M/2 (a line that is its own mirror, y and z
// each 0 or M/2, alone): (M/2 - 1) M + M + 2 of them. Needs 2 NI M <= 4096 (LDS).
template <int TGT>
__global__ void __launch_bounds__(256)
    k_pm_xmult(const double2* __restrict__ fin, int M, double dk, double xi, double a2, double invL3,
               const double* __restrict__ bmod, const double2* __restrict__ tw, FftPlan pl,
               double2* __restrict__ fout) {
  constexpr int NC = pnc(sft(TGT)), W = pw(TGT), NI = (NC + 1) / 2, NO = (W + 1) / 2;
  constexpr int PPT = 2;  // point pairs per thread (M <= 512)
  extern __shared__ double2 xs[];
  const int h = M >> 1, b = blockIdx.x, nmid = (h - 1) * M;
  const int z = b < nmid ? 1 + b / M : ((b - nmid) < h + 1 ? 0 : h);
  const int y = b < nmid ? b % M : (b - nmid) % (h + 1);
  const int yp = (M - y) & (M - 1), zp = (M - z) & (M - 1);
  const bool self = y == yp && z == zp;
  const int nl = self ? NI : 2 * NI;
  const int64_t M3 = (int64_t)M * M * M;
  const int64_t row = ((int64_t)z * M + y) * M, rowp = ((int64_t)zp * M + yp) * M;
  for (int e = threadIdx.x; e < nl * M; e += blockDim.x) {
    const int l = e / M, x = e % M;
    xs[fft_slot(l, x, M)] = fin[(l < NI ? row : rowp) + (int64_t)(l % NI) * M3 + x];
  }
  __syncthreads();
  int Ns = 1;
  for (int st = 0; st < pl.nst; ++st) {
    if (pl.r[st] == 8)
      fft_stage<8, false, true>(xs, nullptr, false, false, M, nl, Ns, 1, M, tw);
    else
      fft_stage<4, false, true>(xs, nullptr, false, false, M, nl, Ns, 1, M, tw);
    Ns *= pl.r[st];
  }
  const int npair = self ? M / 2 + 1 : M;  // (self: x = 0..M/2 with -x on the same line)
  const int lm = self ? 0 : NI;            // first input line of the mirror
  const int lo = self ? 0 : NO;            // first output line of the mirror
  double2 yo[PPT][NO], ym[PPT][NO];
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int x = threadIdx.x + q * 256;
    if (x < npair) {
      const int xm = (M - x) & (M - 1);
      double2 zo[NI], zr[NI];
#pragma unroll
      for (int a = 0; a < NI; ++a) {
        zo[a] = xs[fft_slot(a, x, M)];
        zr[a] = xs[fft_slot(lm + a, xm, M)];
      }
      pm_point<TGT>(zo, zr, x, y, z, M, dk, xi, a2, invL3, bmod, yo[q]);
      pm_point<TGT>(zr, zo, xm, yp, zp, M, dk, xi, a2, invL3, bmod, ym[q]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int x = threadIdx.x + q * 256;
    if (x < npair) {
      const int xm = (M - x) & (M - 1);
#pragma unroll
      for (int b = 0; b < NO; ++b) {
        xs[fft_slot(b, x, M)] = yo[q][b];
        xs[fft_slot(lo + b, xm, M)] = ym[q][b];
      }
    }
  }
  __syncthreads();
  const int nlo = self ? NO : 2 * NO;
  Ns = 1;
  for (int st = 0; st < pl.nst; ++st) {
    if (pl.r[st] == 8)
      fft_stage<8, true, true>(xs, nullptr, false, false, M, nlo, Ns, 1, M, tw);
    else
      fft_stage<4, true, true>(xs, nullptr, false, false, M, nlo, Ns, 1, M, tw);
    Ns *= pl.r[st];
  }
  for (int e = threadIdx.x; e < nlo * M; e += blockDim.x) {
    const int l = e / M, x = e % M;
    fout[(l < NO ? row : rowp) + (int64_t)(l % NO) * M3 + x] = xs[fft_slot(l, x, M)];
  }
}

// part[out(k) * W] = sum over the P^3 mesh points around receiver k of its weights times the
// inverse transform (out(k) = perm[k] when perm is given, else k; receivers at Xr with a stride).
// Eight lanes per receiver, one per x offset, so that each load moves eight consecutive mesh points;
// the lanes' sums are combined by shuffles in a fixed order.
template <int TGT>
__global__ void __launch_bounds__(256)
    k_pm_gather(const double* __restrict__ Xr, int stride, const int32_t* __restrict__ perm, int m, double L,
                int M, const double2* __restrict__ fout, double* __restrict__ part) {
  constexpr int W = pw(TGT), NO = (W + 1) / 2;
  const int k = xcd_order(blockIdx.x, gridDim.x) * (blockDim.x / kPmP) + threadIdx.x / kPmP;
  const int ox = threadIdx.x % kPmP;
  const int kk = k < m ? k : m - 1;
  const int64_t M3 = (int64_t)M * M * M;
  int b[3];
  double w[3][kPmP];
  for (int d = 0; d < 3; ++d) {
    double xw = Xr[(int64_t)stride * kk + d];
    xw -= L * floor(xw / L);
    const double u = xw * (M / L);
    const double fu = floor(u);
    bspline_w(u - fu, w[d]);
    b[d] = ((int)fu - (kPmP - 1)) & (M - 1);
  }
  double wx = w[0][0];
#pragma unroll
  for (int o = 1; o < kPmP; ++o)
    if (ox == o) wx = w[0][o];
  const int px = (b[0] + ox) & (M - 1);
  double acc[2 * NO];
#pragma unroll
  for (int c = 0; c < 2 * NO; ++c) acc[c] = 0.0;
  for (int oz = 0; oz < kPmP; ++oz) {
    const int64_t pz = (int64_t)((b[2] + oz) & (M - 1)) * M;
    const double wz = w[2][oz] * wx;
#pragma unroll
    for (int oy = 0; oy < kPmP; ++oy) {
      const int64_t p = (pz + ((b[1] + oy) & (M - 1))) * M + px;
      const double ww = wz * w[1][oy];
#pragma unroll
      for (int f = 0; f < NO; ++f) {
        const double2 v = fout[(int64_t)f * M3 + p];
        acc[2 * f] = fma(ww, v.x, acc[2 * f]);
        acc[2 * f + 1] = fma(ww, v.y, acc[2 * f + 1]);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 2 * NO; ++c)
#pragma unroll
    for (int sh = kPmP / 2; sh > 0; sh >>= 1) acc[c] += __shfl_xor(acc[c], sh, kPmP);
  if (ox != 0 || k >= m) return;
  const int64_t o = perm ? perm[k] : k;
#pragma unroll
  for (int c = 0; c < W; ++c) part[o * W + c] = acc[c];
}

inline unsigned nblk_p(int64_t len, int b) { return (unsigned)((len + b - 1) / b); }

// launch shapes: source chunks of the real-space pass, source chunks of the structure factors,
// wave-vector chunks of the reciprocal sum (each aiming at about 2048 workgroups)
struct PerShape {
  int nreal, creal, nsf, csf, nrec, crec;
};

PerShape per_shape(int64_t n, int K, int nseg) {
  PerShape p;
  const int64_t rb = std::max<int64_t>((n + kPBlk - 1) / kPBlk, 1), kb = std::max((nseg + kPKBlk - 1) / kPKBlk, 1);
  p.nreal = (int)std::min<int64_t>(std::max<int64_t>((2048 + rb - 1) / rb, 1), (n + kPTJ - 1) / kPTJ);
  p.creal = (int)((n + p.nreal - 1) / p.nreal);
  p.nsf = (int)std::min<int64_t>(std::max<int64_t>((2048 + kb - 1) / kb, 1), std::min<int64_t>(16, (n + kPTJ - 1) / kPTJ));
  p.csf = (int)((n + p.nsf - 1) / p.nsf);
  p.nrec = (int)std::min<int64_t>(std::max<int64_t>((2048 + rb - 1) / rb, 1), (K + kPKT - 1) / kPKT);
  p.crec = (int)((K + p.nrec - 1) / p.nrec);
  return p;
}

inline size_t align256p(size_t b) { return (b + 255) & ~size_t(255); }

struct PmLayout {
  size_t fin, fout, b0, wts, grid, total;
};

// mesh workspace: 7 complex input fields and 3 output fields of M^3 points, per-sphere first mesh
// points and weights, the box grid of the sources
PmLayout pm_layout(int M, int64_t n, int nc) {
  const int64_t M3 = (int64_t)M * M * M;
  PmLayout y{};
  size_t o = 0;
  y.fin = o;
  o += align256p(sizeof(double2) * 7 * (size_t)M3);
  y.fout = o;
  o += align256p(sizeof(double2) * 3 * (size_t)M3);
  y.b0 = o;
  o += align256p(sizeof(int) * 4 * (size_t)n);
  y.wts = o;
  o += align256p(sizeof(double) * 3 * kPmP * (size_t)n);
  y.grid = o;
  o += align256p(grid_ws_bytes((int)n, (int64_t)nc * nc * nc));
  y.total = o;
  return y;
}

// radices of the transform of length M (a power of 2, 16 or more): eights, then one or two fours
FftPlan fft_plan(int M) {
  int lg = 0;
  while ((1 << lg) < M) ++lg;
  FftPlan p{};
  while (lg >= 3 && lg != 4 && lg - 3 != 1) {
    p.r[p.nst++] = 8;
    lg -= 3;
  }
  while (lg >= 2) {
    p.r[p.nst++] = 4;
    lg -= 2;
  }
  return p;
}

// the transform of nf complex fields of M^3 points (x fastest) along the axes in mask (1 x, 2 y,
// 4 z), in place
// the per-workgroup LDS the device allows (gfx950: 160 KB per CU), once
size_t fft_lds_limit() {
  static size_t lim = 0;
  if (!lim) {
    int dev = 0, v = 0;
    lim = 65536;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 65536)
      lim = (size_t)v;
  }
  return lim;
}

void pm_fft(double2* a, int nf, int M, bool inv, const double2* tw, hipStream_t s, int mask = 7) {
  const FftPlan pl = fft_plan(M);
  // lines per workgroup: B M = 4096 points (64 KB) in general; 16 lines (256-byte runs) along z on
  // the 512-point mesh, whose lines stride 4 MB, where the device allows 128 KB of LDS per workgroup
  // (measured: z 4.0 -> 3.35 ms per pass at 512^3 x 3 fields; y, striding 8 KB, gains nothing)
  const int B = std::max(1, std::min(16, 4096 / M));
  const int Bs = (M * 16 * (int)sizeof(double2) <= (int)fft_lds_limit() && 16 * M <= 8192) ? 16 : B;
  const int64_t M2 = (int64_t)M * M, M3 = M2 * M;
#define MBS_FFT_PASS(AX, BB, SK, SB, SU, SV)                                                                    \
  do {                                                                                                          \
    const size_t lds = (size_t)(BB) * M * sizeof(double2);                                                      \
    const dim3 grid((unsigned)(M2 / (BB)), (unsigned)nf), blk((unsigned)((BB) * M / 16));                      \
    if (inv)                                                                                                    \
      hipLaunchKernelGGL((k_fft_lines<true, AX>), grid, blk, lds, s, a, M, BB, SK, SB, M / (BB), SU, SV, M3, tw, \
                         pl);                                                                                   \
    else                                                                                                        \
      hipLaunchKernelGGL((k_fft_lines<false, AX>), grid, blk, lds, s, a, M, BB, SK, SB, M / (BB), SU, SV, M3,  \
                         tw, pl);                                                                               \
  } while (0)
  if (mask & 1) MBS_FFT_PASS(0, B, (int64_t)1, (int64_t)M, (int64_t)B * M, M2);  // x: lines consecutive in y
  if (mask & 2) MBS_FFT_PASS(1, B, (int64_t)M, (int64_t)1, (int64_t)B, M2);       // y: lines consecutive in x
  if (mask & 4) MBS_FFT_PASS(2, Bs, M2, (int64_t)1, (int64_t)Bs, (int64_t)M);     // z: lines consecutive in x
#undef MBS_FFT_PASS
}

template <int TGT>
void pm_launch(const double* X, int64_t m, const double* R, int64_t n, const double* Fe, const double* Te,
               const double* Sig, const double* D, const double* v1s, const double* v2s, double* out, double* out2,
               double* out3, double* part, const PerBox& g, const Phys& ph, hipStream_t s) {
  constexpr int W = pw(TGT), NC = pnc(sft(TGT)), NI = (NC + 1) / 2, NO = (W + 1) / 2;
  const int M = g.M;
  const int64_t M3 = (int64_t)M * M * M;
  const PmLayout Ly = pm_layout(M, n, g.nc);
  char* wb = (char*)g.mws;
  double2* fin = (double2*)(wb + Ly.fin);
  double2* fout = (double2*)(wb + Ly.fout);
  int* b0 = (int*)(wb + Ly.b0);
  double* wts = (double*)(wb + Ly.wts);
  const double2* tw = (const double2*)g.tab;
  const double* bmod = g.tab + 2 * M;
  const double a5_20 = 0.5 * ph.a5_10;
  GridView gv;
  (void)grid_build_box(R, (int)n, g.L, g.nc, wb + Ly.grid, Ly.total - Ly.grid, &gv, s);
  hipLaunchKernelGGL(k_pm_prep, dim3(nblk_p(n, 256)), dim3(256), 0, s, gv.Rs, (int)n, M, M / g.L, b0, wts);
  const dim3 sg((unsigned)(M3 / (kPmB * kPmB * kPmB)));
  if (sft(TGT) == kPOp) {
    hipLaunchKernelGGL((k_pm_spread<kPOp, 0, 5>), sg, dim3(64), 0, s, gv.perm, gv.start, gv.end, b0, wts, Fe, Te, Sig,
                       D, ph.P, a5_20, M, g.nc, fin);
  } else if (sft(TGT) == kPRhs) {
    hipLaunchKernelGGL((k_pm_spread<kPRhs, 0, 6>), sg, dim3(64), 0, s, gv.perm, gv.start, gv.end, b0, wts, Fe, Te,
                       Sig, D, ph.P, a5_20, M, g.nc, fin);
    hipLaunchKernelGGL((k_pm_spread<kPRhs, 6, 3>), sg, dim3(64), 0, s, gv.perm, gv.start, gv.end, b0, wts, Fe, Te,
                       Sig, D, ph.P, a5_20, M, g.nc, fin + 3 * M3);
  } else {
    hipLaunchKernelGGL((k_pm_spread<kPOut, 0, 6>), sg, dim3(64), 0, s, gv.perm, gv.start, gv.end, b0, wts, Fe, Te,
                       Sig, D, ph.P, a5_20, M, g.nc, fin);
    hipLaunchKernelGGL((k_pm_spread<kPOut, 6, 6>), sg, dim3(64), 0, s, gv.perm, gv.start, gv.end, b0, wts, Fe, Te,
                       Sig, D, ph.P, a5_20, M, g.nc, fin + 3 * M3);
    hipLaunchKernelGGL((k_pm_spread<kPOut, 12, 2>), sg, dim3(64), 0, s, gv.perm, gv.start, gv.end, b0, wts, Fe, Te,
                       Sig, D, ph.P, a5_20, M, g.nc, fin + 6 * M3);
  }
  if (2 * NI * M <= 4096) {  // the x transforms fused with the multiplier
    pm_fft(fin, NI, M, false, tw, s, 6);
    hipLaunchKernelGGL(k_pm_xmult<TGT>, dim3((unsigned)((M / 2 - 1) * M + M + 2)), dim3(256),
                       (size_t)2 * NI * M * sizeof(double2), s,
                       fin, M, 2.0 * M_PI / g.L, g.xi, ph.a2, 1.0 / (g.L * g.L * g.L), bmod, tw, fft_plan(M), fout);
    pm_fft(fout, NO, M, true, tw, s, 6);
  } else {
    pm_fft(fin, NI, M, false, tw, s);
    hipLaunchKernelGGL(k_pm_mult<TGT>, dim3(nblk_p(M3, 256)), dim3(256), 0, s, fin, M, 2.0 * M_PI / g.L, g.xi, ph.a2,
                       1.0 / (g.L * g.L * g.L), bmod, fout);
    pm_fft(fout, NO, M, true, tw, s);
  }
  // real space: over the box grid's neighbouring cells when it has at least 3 cells per axis (the
  // spheres as receivers), else over all pairs; the mesh part interpolated at the receivers
  // (field points take the cells too when the caller gave a workspace for their box grid)
  const bool cells = g.nc >= 3 && (TGT != kPFlow || g.fws);
  const PerShape sh = per_shape(m, 0, 0);
  const int nreal = cells ? 3 : sh.nreal;
  double* preal = part;
  double* precip = preal + (int64_t)nreal * W * m;
  if (cells) {
    GridView gr = gv;
    if (TGT == kPFlow) (void)grid_build_box(X, (int)m, g.L, g.nc, g.fws, g.fws_bytes, &gr, s);
    const double* rtab = TGT == kPOp && g.npiece > 0 ? g.rtab : nullptr;
    hipLaunchKernelGGL(k_pm_real<TGT>, dim3((unsigned)g.nc * g.nc * g.nc, 3), dim3(kPmRT),
                       rtab ? (size_t)g.npiece * kRtC * sizeof(double) : 0, s, gr.Rs, gr.perm, gr.start, gr.end,
                       gv.Rs, gv.perm, gv.start, gv.end, g.nc, (int)m, Fe, Te, Sig, D, g.L, g.rc * g.rc, g.xi, ph.a2,
                       ph.P, a5_20, rtab, g.npiece, 1.0 / ph.a2, preal);
  } else {
    const int creal = (int)((n + sh.nreal - 1) / sh.nreal);
    hipLaunchKernelGGL(k_per_real<TGT>, dim3(nblk_p(m, kPBlk), sh.nreal), dim3(kPBlk), 0, s, X, (int)m, R, (int)n,
                       Fe, Te, Sig, D, creal, g.L, 1.0 / g.L, g.rc * g.rc, g.xi, ph.a2, ph.P, a5_20, preal);
  }
  if (TGT == kPFlow)
    hipLaunchKernelGGL(k_pm_gather<TGT>, dim3(nblk_p(m, 256 / kPmP)), dim3(256), 0, s, X, 3,
                       (const int32_t*)nullptr, (int)m, g.L, M, fout, precip);
  else
    hipLaunchKernelGGL(k_pm_gather<TGT>, dim3(nblk_p(m, 256 / kPmP)), dim3(256), 0, s, gv.Rs, 4, gv.perm, (int)m, g.L,
                       M, fout, precip);
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  if (TGT == kPOp) s0 = ph.P * per_self_es(g.xi, ph.a2);
  if (TGT == kPOut) {
    s0 = ph.P * per_self_uf(g.xi, ph.a2);
    s1 = a5_20 * per_self_ud(g.xi, ph.a2);
    s2 = ph.P * per_self_wt(g.xi, ph.a2);
  }
  hipLaunchKernelGGL(k_per_finish<TGT>, dim3(nblk_p(m, 256)), dim3(256), 0, s, preal, nreal, precip, 1, (int)m,
                     Sig, Fe, Te, D, v1s, v2s, s0, s1, s2, ph, out, out2, out3);
}

template <int TGT>
void per_launch(const double* X, int64_t m, const double* R, int64_t n, const double* Fe, const double* Te,
                const double* Sig, const double* D, const double* v1s, const double* v2s, double* out, double* out2,
                double* out3, double* part, const PerBox& g, const Phys& ph, hipStream_t s) {
  if (g.M > 0) {
    pm_launch<TGT>(X, m, R, n, Fe, Te, Sig, D, v1s, v2s, out, out2, out3, part, g, ph, s);
    return;
  }
  constexpr int W = pw(TGT), NC = pnc(TGT);
  // receivers m for the real-space and reciprocal passes, sources n for the structure factors
  const PerShape sh = per_shape(m, g.K, TGT == kPOp ? g.nseg8 : g.nseg4);
  const PerShape shs = per_shape(n, g.K, TGT == kPOp ? g.nseg8 : g.nseg4);
  double* preal = part;
  double* precip = preal + (int64_t)sh.nreal * W * m;
  double* sf = precip + (int64_t)sh.nrec * W * m;
  double* T = sf + (int64_t)shs.nsf * 2 * NC * g.K;
  const double a5_20 = 0.5 * ph.a5_10;
  const int creal = (int)((n + sh.nreal - 1) / sh.nreal);  // sources per real-space chunk
  hipLaunchKernelGGL(k_per_real<TGT>, dim3(nblk_p(m, kPBlk), sh.nreal), dim3(kPBlk), 0, s, X, (int)m, R, (int)n, Fe,
                     Te, Sig, D, creal, g.L, 1.0 / g.L, g.rc * g.rc, g.xi, ph.a2, ph.P, a5_20, preal);
  const int nseg = TGT == kPOp ? g.nseg8 : g.nseg4;
  const double dk = 2.0 * M_PI / g.L;
  hipLaunchKernelGGL(k_per_sf<sft(TGT)>, dim3(nblk_p(nseg, kPKBlk), shs.nsf), dim3(kPKBlk), 0, s, R, (int)n, Fe, Te,
                     Sig, D, g.kv, TGT == kPOp ? g.seg8 : g.seg4, nseg, g.K, dk, shs.csf, ph.P, a5_20, sf);
  hipLaunchKernelGGL(k_per_mult<TGT>, dim3(nblk_p(g.K, kPKBlk)), dim3(kPKBlk), 0, s, sf, shs.nsf, g.kv, g.K, g.xi,
                     ph.a2, 2.0 / (g.L * g.L * g.L), T);
  hipLaunchKernelGGL(k_per_recip<TGT>, dim3(nblk_p(m, kPBlk), sh.nrec), dim3(kPBlk), 0, s, X, (int)m, g.kv, T, g.K,
                     dk, sh.crec, precip);
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  if (TGT == kPOp) s0 = ph.P * per_self_es(g.xi, ph.a2);
  if (TGT == kPOut) {
    s0 = ph.P * per_self_uf(g.xi, ph.a2);
    s1 = a5_20 * per_self_ud(g.xi, ph.a2);
    s2 = ph.P * per_self_wt(g.xi, ph.a2);
  }
  hipLaunchKernelGGL(k_per_finish<TGT>, dim3(nblk_p(m, 256)), dim3(256), 0, s, preal, sh.nreal, precip, sh.nrec,
                     (int)m, Sig, Fe, Te, D, v1s, v2s, s0, s1, s2, ph, out, out2, out3);
}

}  // namespace

std::vector<double> per_kvecs(double L, double kmax) {
  // half of the reciprocal lattice (k and -k give complex conjugate terms): the first nonzero
  // component of the integer vector positive
  std::vector<double> kv;
  const double dk = 2.0 * M_PI / L;
  const int m = (int)floor(kmax / dk);
  for (int a = 0; a <= m; ++a)
    for (int b = -m; b <= m; ++b)
      for (int c = -m; c <= m; ++c) {
        if (a == 0 && (b < 0 || (b == 0 && c <= 0))) continue;
        const double k1 = a * dk, k2 = b * dk, k3 = c * dk;
        if (k1 * k1 + k2 * k2 + k3 * k3 > kmax * kmax) continue;
        kv.push_back(k1);
        kv.push_back(k2);
        kv.push_back(k3);
      }
  return kv;
}

std::vector<int> per_segments(const std::vector<double>& kv, double L, int maxlen) {
  // runs of consecutive k3 within one (k1, k2) row, cut into pieces of at most maxlen
  std::vector<int> seg;
  const int K = (int)(kv.size() / 3);
  const double dk = 2.0 * M_PI / L;
  int k = 0;
  while (k < K) {
    int e = k + 1;
    while (e < K && e - k < maxlen && kv[3 * e] == kv[3 * k] && kv[3 * e + 1] == kv[3 * k + 1] &&
           fabs(kv[3 * e + 2] - kv[3 * (e - 1) + 2] - dk) < 0.5 * dk)
      ++e;
    seg.push_back(k);
    seg.push_back(e - k);
    k = e;
  }
  return seg;
}

int64_t per_part_elems(int64_t m, int64_t n, int K, int nseg) {
  const PerShape sh = per_shape(m, K, nseg), shs = per_shape(n, K, nseg);  // receivers m, sources n
  return (int64_t)(std::max(sh.nreal, 3) + sh.nrec + 1) * 6 * m + (int64_t)shs.nsf * 28 * K + (int64_t)12 * K + 64;
}

size_t pm_ws_bytes(int M, int64_t n, int nc) { return pm_layout(M, n, nc).total; }

size_t pm_flow_ws_bytes(int64_t m, int nc) { return grid_ws_bytes((int)m, (int64_t)nc * nc * nc); }

int pm_radial_pieces(double a2, double rc) {
  const double ratio = rc * rc / a2;
  if (!(ratio > 1.0)) return 0;
  const int noct = (int)ceil(log2(ratio)) + 1;
  return noct > kRtOct ? 0 : noct * kRtK;
}

size_t pm_radial_doubles() { return (size_t)kRtMax; }

hipError_t pm_radial_table(double xi, double a2, double rc, double* tab, hipStream_t s) {
  const int np = pm_radial_pieces(a2, rc);
  if (np == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pm_rtab, dim3((unsigned)((np + 63) / 64)), dim3(64), 0, s, np, a2, xi, a2, tab);
  return hipGetLastError();
}

std::vector<double> pm_tables(int M) {
  // twiddles exp(-2 pi i k / M), k < M, then |b(m)|^2 = 1 / |sum_{k <= P-2} M_P(k + 1) exp(2 pi i m k / M)|^2
  std::vector<double> t(3 * (size_t)M);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int k = 0; k < M; ++k) {
    const long double ang = 2.0L * pi * k / M;
    t[2 * k] = (double)cosl(ang);
    t[2 * k + 1] = (double)-sinl(ang);
  }
  double w[kPmP];
  bspline_w(0.0, w);  // w[o] = M_P(P - 1 - o)
  for (int mm = 0; mm < M; ++mm) {
    const int f = mm < M / 2 ? mm : mm - M;
    long double re = 0.0L, im = 0.0L;
    for (int k = 0; k <= kPmP - 2; ++k) {
      const long double v = w[kPmP - 2 - k], ang = 2.0L * pi * f * k / M;
      re += v * cosl(ang);
      im += v * sinl(ang);
    }
    t[2 * M + mm] = (double)(1.0L / (re * re + im * im));
  }
  return t;
}

void launch_per_op(const double* R, const double* x, double* y, double* part, int64_t n, const PerBox& g,
                   const Phys& ph, hipStream_t s) {
  if (n <= 0) return;
  per_launch<kPOp>(R, n, R, n, nullptr, nullptr, x, nullptr, nullptr, nullptr, y, nullptr, nullptr, part, g, ph, s);
}

void launch_per_rhs(const double* R, const double* v2s, const double* v3t, const double* Fe, const double* Te,
                    double* b, double* part, int64_t n, const PerBox& g, const Phys& ph, hipStream_t s) {
  if (n <= 0) return;
  per_launch<kPRhs>(R, n, R, n, Fe, Te, nullptr, v3t, nullptr, v2s, b, nullptr, nullptr, part, g, ph, s);
}

void launch_per_out(const double* R, const double* v1s, const double* v2s, const double* v3t, const double* Fe,
                    const double* Te, const double* Sig, double* V, double* W, double* S, double* part, int64_t n,
                    const PerBox& g, const Phys& ph, hipStream_t s) {
  if (n <= 0) return;
  per_launch<kPOut>(R, n, R, n, Fe, Te, Sig, v3t, v1s, v2s, V, W, S, part, g, ph, s);
}

int per_min_dist_part(int64_t n) { return (int)((n + 255) / 256); }

void launch_per_min_dist(const double* R, int64_t n, double L, double* part, double* out, hipStream_t s) {
  const int nb = per_min_dist_part(n);
  hipLaunchKernelGGL(k_per_min_d2, dim3(nb), dim3(256), 0, s, R, (int)n, L, 1.0 / L, part, (const double*)nullptr,
                     0.0);
  hipLaunchKernelGGL(k_min_finish, dim3(1), dim3(256), 0, s, part, nb, out, false, 0.0);
}

void launch_pm_min_dist(const double* R, int64_t n, const PerBox& g, double* part, double* out, hipStream_t s) {
  // the box grid's 27 neighbouring cells find every pair closer than a cell edge; only when none is
  // (a sparse box) does the all-pairs scan run, decided on the device
  const int nb = per_min_dist_part(n);
  const PmLayout Ly = pm_layout(g.M, n, g.nc);
  char* wb = (char*)g.mws;
  GridView gv;
  (void)grid_build_box(R, (int)n, g.L, g.nc, wb + Ly.grid, Ly.total - Ly.grid, &gv, s);
  const double edge = g.L / g.nc;
  hipLaunchKernelGGL(k_pm_min_d2, dim3(nb), dim3(256), 0, s, gv.hdr, gv.Rs, gv.start, gv.end, g.nc, (int)n, g.L,
                     1.0 / g.L, part);
  hipLaunchKernelGGL(k_min_finish, dim3(1), dim3(256), 0, s, part, nb, out, false, 0.0);
  hipLaunchKernelGGL(k_per_min_d2, dim3(nb), dim3(256), 0, s, R, (int)n, g.L, 1.0 / g.L, part + nb, out, edge);
  hipLaunchKernelGGL(k_min_finish, dim3(1), dim3(256), 0, s, part + nb, nb, out, true, edge);
}

void launch_per_flow(const double* X, int64_t m, const double* R, int64_t n, const double* Fe, const double* Te,
                     const double* Sig, const double* v3t, double* U, double* part, const PerBox& g, const Phys& ph,
                     hipStream_t s) {
  if (m <= 0 || n <= 0) return;
  per_launch<kPFlow>(X, m, R, n, Fe, Te, Sig, v3t, nullptr, nullptr, U, nullptr, nullptr, part, g, ph, s);
}

}  // namespace mbs
