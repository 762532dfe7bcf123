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
// Every sum runs in a fixed order (bitwise reproducible). The arithmetic is binary64 throughout.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "mbs_device.h"
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
    while (hits) {
      const int jj = __ffsll((unsigned long long)hits) - 1;
      hits &= hits - 1;
      const RecP& s = tile[jj];
      const double dx = wrap(xi0 - s.x, L, invL), dy = wrap(yi0 - s.y, L, invL), dz = wrap(zi0 - s.z, L, invL);
      const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
      const double r = sqrt(r2);
      const double ri = 1.0 / r, ec = erfc(xi * r), ex = exp(-xi * xi * r2);
      if (TGT == kPOp) {
        // E = al Sigma + be (x w + w x) + ga q x x (+ a trace the 5-basis drops), w = Sigma x, q = x.w
        double abg[3];
        per_real_es_radial(ri, ec, ex, xi, a2, abg);
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
      }
      if (TGT == kPRhs) per_real_strain_ftq(dx, dy, dz, ri, ec, ex, xi, a2, s.f, s.t, s.q, acc);
      if (TGT == kPOut) per_real_motion_ftsq(dx, dy, dz, ri, ec, ex, xi, a2, s.f, s.t, s.s, s.q, acc, acc + 3);
      if (TGT == kPFlow) per_real_flow_ftsq(dx, dy, dz, ri, ec, ex, xi, a2, s.f, s.t, s.s, s.q, acc);
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
__global__ void __launch_bounds__(256) k_per_min_d2(const double* __restrict__ R, int n, double L, double invL,
                                                    double* __restrict__ part) {
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

// out[0] = sqrt(min over the nb partial minima)
__global__ void __launch_bounds__(256) k_min_finish(const double* __restrict__ part, int nb, double* __restrict__ out) {
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

inline unsigned nblk_p(int64_t len, int b) { return (unsigned)((len + b - 1) / b); }

// launch shapes: source chunks of the real-space pass, source chunks of the structure factors,
// wave-vector chunks of the reciprocal sum (each aiming at about 2048 workgroups)
struct PerShape {
  int nreal, creal, nsf, csf, nrec, crec;
};

PerShape per_shape(int64_t n, int K, int nseg) {
  PerShape p;
  const int64_t rb = (n + kPBlk - 1) / kPBlk, kb = (nseg + kPKBlk - 1) / kPKBlk;
  p.nreal = (int)std::min<int64_t>(std::max<int64_t>((2048 + rb - 1) / rb, 1), (n + kPTJ - 1) / kPTJ);
  p.creal = (int)((n + p.nreal - 1) / p.nreal);
  p.nsf = (int)std::min<int64_t>(std::max<int64_t>((2048 + kb - 1) / kb, 1), std::min<int64_t>(16, (n + kPTJ - 1) / kPTJ));
  p.csf = (int)((n + p.nsf - 1) / p.nsf);
  p.nrec = (int)std::min<int64_t>(std::max<int64_t>((2048 + rb - 1) / rb, 1), (K + kPKT - 1) / kPKT);
  p.crec = (int)((K + p.nrec - 1) / p.nrec);
  return p;
}

template <int TGT>
void per_launch(const double* X, int64_t m, const double* R, int64_t n, const double* Fe, const double* Te,
                const double* Sig, const double* D, const double* v1s, const double* v2s, double* out, double* out2,
                double* out3, double* part, const PerBox& g, const Phys& ph, hipStream_t s) {
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
  return (int64_t)sh.nreal * 6 * m + (int64_t)sh.nrec * 6 * m + (int64_t)shs.nsf * 28 * K + (int64_t)12 * K + 64;
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
  hipLaunchKernelGGL(k_per_min_d2, dim3(nb), dim3(256), 0, s, R, (int)n, L, 1.0 / L, part);
  hipLaunchKernelGGL(k_min_finish, dim3(1), dim3(256), 0, s, part, nb, out);
}

void launch_per_flow(const double* X, int64_t m, const double* R, int64_t n, const double* Fe, const double* Te,
                     const double* Sig, const double* v3t, double* U, double* part, const PerBox& g, const Phys& ph,
                     hipStream_t s) {
  if (m <= 0 || n <= 0) return;
  per_launch<kPFlow>(X, m, R, n, Fe, Te, Sig, v3t, nullptr, nullptr, U, nullptr, nullptr, part, g, ph, s);
}

}  // namespace mbs
