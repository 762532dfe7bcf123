// The system operator of the stresslet rows (the GMRES matvec), gfx950:
//
//   y_n = x_n / gamma - sum_{m != n} E[x_m](R_n - R_m),
//   E[Sigma](x) = P [ c1 sym(x w) + c2 x x + c3 Sigma ]  (traceless part),  w = Sigma x, q = x.w,
//   c1 = -6/r^5 + 24a^2/r^7,  c2 = q (15/r^7 - 42a^2/r^9),  c3 = -12a^2/(5 r^5),
//
// the off-diagonal Galerkin element between the symmetric l = 1 modes of two spheres: the
// finite-size operators F^1 = 1 + a^2/10 nabla^2 of source and receiver applied to the first
// derivative of the Green's function, reduced with nabla^4 G = 0 (section III).
//
// Per pair the receiver accumulates the raw moments x_i v_j of v = c1 w + c2 x (six sums) and
// r^-5 Sigma (five sums); the traceless 5-basis projection and the constant factors are applied
// once per receiver. Algorithmic work per pair block: 78 FLOP (FMA = 2, rsqrt = 1): differences
// 3, r^2 5, 1/r 1, powers 4, Szz 1, w 15, q 5, c1 3, c2 4, v 9, moments 18, r^-5 Sigma 10.
//
// Two launch variants share that arithmetic:
//  * LDS: the workgroup stages source records (position, Cartesian Sigma) through LDS tiles;
//    every lane reads the same record (broadcast). The binary32 flavour re-centres coordinates on
//    the workgroup's first receiver (in binary64) before rounding.
//  * stream: a pack kernel writes one 64-byte (binary64) or 32-byte (binary32) record per source;
//    the pair kernel walks the records at a wavefront-uniform index, so the compiler issues scalar
//    loads into SGPRs and no LDS or barrier is involved. The binary32 flavour stores coordinates
//    relative to the centre of the bounding box.
// Both split the sources into grid.y chunks whose partial sums a finishing kernel adds in a
// fixed order (bitwise reproducible). Only ranges that can contain the receiver itself test for
// r == 0 (n == m term).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "mbs_device.h"
#include "mbs_internal.h"
#include "mbs_pair.h"

namespace mbs {

const Tile kTileTable[] = {
    {1, 256, 0, 2048}, {1, 128, 0, 2048}, {1, 256, 0, 4096}, {1, 64, 0, 4096},
    {1, 256, 0, 1024}, {0, 256, 128, 2048}, {0, 256, 256, 2048}, {0, 128, 128, 2048},
    {0, 256, 128, 4096}, {0, 256, 64, 2048},
};
const int kTileCount = sizeof(kTileTable) / sizeof(kTileTable[0]);

namespace {

// Total over segments: binary64 adds directly; binary32 uses compensated (Kahan) sums.
template <typename T>
struct Total;
template <>
struct Total<double> {
  Mom<double> s;
  __device__ void add(const Mom<double>& m) {
    s.pxx += m.pxx; s.pyy += m.pyy; s.pzz += m.pzz; s.qxy += m.qxy; s.qxz += m.qxz; s.qyz += m.qyz;
    s.t0 += m.t0; s.t1 += m.t1; s.t2 += m.t2; s.t3 += m.t3; s.t4 += m.t4;
  }
  __device__ void get(double* v) const {
    const double* p = &s.pxx;
#pragma unroll
    for (int k = 0; k < 11; ++k) v[k] = p[k];
  }
};
__device__ __forceinline__ void kahan_add(float& s, float& c, float v) {
  const float y = v - c;
  const float t = s + y;
  c = (t - s) - y;
  s = t;
}
template <>
struct Total<float> {
  Mom<float> s, c;
  __device__ void add(const Mom<float>& m) {
    kahan_add(s.pxx, c.pxx, m.pxx); kahan_add(s.pyy, c.pyy, m.pyy); kahan_add(s.pzz, c.pzz, m.pzz);
    kahan_add(s.qxy, c.qxy, m.qxy); kahan_add(s.qxz, c.qxz, m.qxz); kahan_add(s.qyz, c.qyz, m.qyz);
    kahan_add(s.t0, c.t0, m.t0); kahan_add(s.t1, c.t1, m.t1); kahan_add(s.t2, c.t2, m.t2);
    kahan_add(s.t3, c.t3, m.t3); kahan_add(s.t4, c.t4, m.t4);
  }
  __device__ void get(double* v) const {
    const float* p = &s.pxx;
    const float* q = &c.pxx;
#pragma unroll
    for (int k = 0; k < 11; ++k) v[k] = (double)p[k] - (double)q[k];
  }
};

// Traceless projection and constants; write y (direct) or the chunk partial.
__device__ __forceinline__ void p2_store(const double* v, int i, int n, const double* __restrict__ X,
                                         double* __restrict__ out, double P, double a2,
                                         double inv_gamma, int direct) {
  double e[5];
  p2_strain(v, P, a2, e);
  if (direct) {
#pragma unroll
    for (int c = 0; c < 5; ++c) out[5 * (int64_t)i + c] = X[5 * (int64_t)i + c] * inv_gamma - e[c];
  } else {
    double* o = out + (int64_t)blockIdx.y * 5 * n + 5 * (int64_t)i;
#pragma unroll
    for (int c = 0; c < 5; ++c) o[c] = e[c];
  }
}

// ---------------------------------------------------------------- stream variant
constexpr int kSeg = 64;  // sources per partial sum (binary32: one Kahan update per segment)

template <typename T>
__global__ void k_pack(const double* __restrict__ R, const double* __restrict__ X,
                       Src8<T>* __restrict__ src, int n, const double* __restrict__ orig) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double ox = 0.0, oy = 0.0, oz = 0.0;
  if (orig) {
    ox = orig[0];
    oy = orig[1];
    oz = orig[2];
  }
  double sxx, syy, sxy, sxz, syz;
  basis_to_cart(X + 5 * (int64_t)j, sxx, syy, sxy, sxz, syz);
  Src8<T> r;
  r.x = (T)(R[3 * (int64_t)j] - ox);
  r.y = (T)(R[3 * (int64_t)j + 1] - oy);
  r.z = (T)(R[3 * (int64_t)j + 2] - oz);
  r.sxx = (T)sxx;
  r.syy = (T)syy;
  r.sxy = (T)sxy;
  r.sxz = (T)sxz;
  r.syz = (T)syz;
  src[j] = r;
}

// Centre of the bounding box of R -> orig[0..2] (one workgroup).
__global__ void __launch_bounds__(256) k_bbox(const double* __restrict__ R, int n, double* __restrict__ orig) {
  __shared__ double lo[3][256], hi[3][256];
  double l[3] = {INFINITY, INFINITY, INFINITY}, h[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int j = threadIdx.x; j < n; j += blockDim.x)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double v = R[3 * (int64_t)j + c];
      l[c] = fmin(l[c], v);
      h[c] = fmax(h[c], v);
    }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    lo[c][threadIdx.x] = l[c];
    hi[c][threadIdx.x] = h[c];
  }
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        lo[c][threadIdx.x] = fmin(lo[c][threadIdx.x], lo[c][threadIdx.x + w]);
        hi[c][threadIdx.x] = fmax(hi[c][threadIdx.x], hi[c][threadIdx.x + w]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 3) orig[threadIdx.x] = 0.5 * (lo[threadIdx.x][0] + hi[threadIdx.x][0]);
}

template <typename T, bool SELF>
__device__ __forceinline__ void stream_range(const Src8<T>* __restrict__ src, int jb, int je, T xi,
                                             T yi, T zi, T A24, T A42, Total<T>& tot) {
  for (int j = jb; j < je; j += kSeg) {
    const int jend = min(je, j + kSeg);
    Mom<T> m;
#pragma unroll 2
    for (int jj = j; jj < jend; ++jj) p2_pair<T, SELF>(src[jj], xi, yi, zi, A24, A42, m);
    tot.add(m);
  }
}

template <typename T>
__global__ void __launch_bounds__(kMaxBlock)
    k_p2_stream(const Src8<T>* __restrict__ src, const double* __restrict__ R,
                const double* __restrict__ X, double* __restrict__ out, int n, int chunk,
                const double* __restrict__ orig, double P, double a2, double inv_gamma, int direct) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int ii = i < n ? i : n - 1;
  double ox = 0.0, oy = 0.0, oz = 0.0;
  if (orig) {
    ox = orig[0];
    oy = orig[1];
    oz = orig[2];
  }
  const T xi = (T)(R[3 * (int64_t)ii] - ox), yi = (T)(R[3 * (int64_t)ii + 1] - oy),
          zi = (T)(R[3 * (int64_t)ii + 2] - oz);
  const T A24 = (T)(24.0 * a2), A42 = (T)(42.0 * a2);
  const int j0 = blockIdx.y * chunk;
  const int j1 = min(n, j0 + chunk);
  const int b0 = blockIdx.x * blockDim.x;
  const int b1 = min(n, b0 + (int)blockDim.x);
  // sources that can coincide with a receiver of this workgroup: [max(j0,b0), min(j1,b1))
  const int s0 = max(j0, b0), s1 = min(j1, b1);
  Total<T> tot;
  if (s0 < s1) {
    stream_range<T, false>(src, j0, s0, xi, yi, zi, A24, A42, tot);
    stream_range<T, true>(src, s0, s1, xi, yi, zi, A24, A42, tot);
    stream_range<T, false>(src, s1, j1, xi, yi, zi, A24, A42, tot);
  } else {
    stream_range<T, false>(src, j0, j1, xi, yi, zi, A24, A42, tot);
  }
  if (i >= n) return;
  double v[11];
  tot.get(v);
  p2_store(v, i, n, X, out, P, a2, inv_gamma, direct);
}

// ---------------------------------------------------------------- LDS variant
// binary32 pair arithmetic of the LDS kernel. On gfx950 a binary32 VOP2 instruction whose
// operands are all VGPRs issues at twice the rate of one that reads an SGPR or a literal or that
// needs the VOP3 form (a source negation, an fma whose addend is not its destination). So the
// record carries S_zz (w = S x then needs no negation), the three constants sit in VGPRs, and the
// raw moments accumulated are those of v/15, for which c1/15 = 1.6a^2/r^7 - 0.4/r^5 and
// c2/15 = u - 2.8a^2 u/r^2 with u = q/r^7 are plain multiply and multiply-add chains; the factor 15
// is restored once per receiver. The r^-5 S sums are not scaled.
struct SrcF9 {
  float x, y, z, sxx, syy, szz, sxy, sxz, syz;
};

struct KF32 {
  float a16, n28, n04;  // 1.6 a^2, -2.8 a^2, -0.4
};

template <bool SELF>
__device__ __forceinline__ void p2_pair_f32(const SrcF9& s, float xi, float yi, float zi, const KF32& k,
                                            Mom<float>& m) {
  const float dx = xi - s.x, dy = yi - s.y, dz = zi - s.z;
  const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
  const float ri = SELF ? rinv_or_zero(r2) : rsq_nr(r2);
  const float ri2 = ri * ri;
  const float ri5 = ri2 * ri2 * ri;
  const float ri7 = ri5 * ri2;
  const float wx = fmaf(s.sxx, dx, fmaf(s.sxy, dy, s.sxz * dz));
  const float wy = fmaf(s.sxy, dx, fmaf(s.syy, dy, s.syz * dz));
  const float wz = fmaf(s.sxz, dx, fmaf(s.syz, dy, s.szz * dz));
  const float q = fmaf(dx, wx, fmaf(dy, wy, dz * wz));
  const float c1 = fmaf(k.a16, ri7, k.n04 * ri5);
  const float u = q * ri7;
  const float c2 = fmaf(k.n28, u * ri2, u);
  const float vx = fmaf(c1, wx, c2 * dx);
  const float vy = fmaf(c1, wy, c2 * dy);
  const float vz = fmaf(c1, wz, c2 * dz);
  m.pxx = fmaf(dx, vx, m.pxx);
  m.pyy = fmaf(dy, vy, m.pyy);
  m.pzz = fmaf(dz, vz, m.pzz);
  m.qxy = fmaf(dx, vy, fmaf(dy, vx, m.qxy));
  m.qxz = fmaf(dx, vz, fmaf(dz, vx, m.qxz));
  m.qyz = fmaf(dy, vz, fmaf(dz, vy, m.qyz));
  m.t0 = fmaf(ri5, s.sxx, m.t0);
  m.t1 = fmaf(ri5, s.syy, m.t1);
  m.t2 = fmaf(ri5, s.sxy, m.t2);
  m.t3 = fmaf(ri5, s.sxz, m.t3);
  m.t4 = fmaf(ri5, s.syz, m.t4);
}

// K source records at once, stage by stage, so that K independent chains are in flight in each
// wave (the reciprocal square roots and LDS reads of one step issue together); the sums take the
// records in order, exactly as K calls of p2_pair_f32 would.
template <bool SELF, int K>
__device__ __forceinline__ void p2_pairs_f32(const SrcF9* s, float xi, float yi, float zi, const KF32& k,
                                             Mom<float>& m) {
  float dx[K], dy[K], dz[K], ri[K], ri2[K], ri5[K], ri7[K], wx[K], wy[K], wz[K], c1[K], c2[K];
#pragma unroll
  for (int q = 0; q < K; ++q) {
    dx[q] = xi - s[q].x;
    dy[q] = yi - s[q].y;
    dz[q] = zi - s[q].z;
  }
#pragma unroll
  for (int q = 0; q < K; ++q) {
    const float r2 = fmaf(dx[q], dx[q], fmaf(dy[q], dy[q], dz[q] * dz[q]));
    ri[q] = SELF ? rinv_or_zero(r2) : rsq_nr(r2);
  }
#pragma unroll
  for (int q = 0; q < K; ++q) {
    wx[q] = fmaf(s[q].sxx, dx[q], fmaf(s[q].sxy, dy[q], s[q].sxz * dz[q]));
    wy[q] = fmaf(s[q].sxy, dx[q], fmaf(s[q].syy, dy[q], s[q].syz * dz[q]));
    wz[q] = fmaf(s[q].sxz, dx[q], fmaf(s[q].syz, dy[q], s[q].szz * dz[q]));
  }
#pragma unroll
  for (int q = 0; q < K; ++q) {
    ri2[q] = ri[q] * ri[q];
    ri5[q] = ri2[q] * ri2[q] * ri[q];
    ri7[q] = ri5[q] * ri2[q];
  }
#pragma unroll
  for (int q = 0; q < K; ++q) {
    const float qv = fmaf(dx[q], wx[q], fmaf(dy[q], wy[q], dz[q] * wz[q]));
    c1[q] = fmaf(k.a16, ri7[q], k.n04 * ri5[q]);
    const float u = qv * ri7[q];
    c2[q] = fmaf(k.n28, u * ri2[q], u);
  }
#pragma unroll
  for (int q = 0; q < K; ++q) {
    const float vx = fmaf(c1[q], wx[q], c2[q] * dx[q]);
    const float vy = fmaf(c1[q], wy[q], c2[q] * dy[q]);
    const float vz = fmaf(c1[q], wz[q], c2[q] * dz[q]);
    m.pxx = fmaf(dx[q], vx, m.pxx);
    m.pyy = fmaf(dy[q], vy, m.pyy);
    m.pzz = fmaf(dz[q], vz, m.pzz);
    m.qxy = fmaf(dx[q], vy, fmaf(dy[q], vx, m.qxy));
    m.qxz = fmaf(dx[q], vz, fmaf(dz[q], vx, m.qxz));
    m.qyz = fmaf(dy[q], vz, fmaf(dz[q], vy, m.qyz));
    m.t0 = fmaf(ri5[q], s[q].sxx, m.t0);
    m.t1 = fmaf(ri5[q], s[q].syy, m.t1);
    m.t2 = fmaf(ri5[q], s[q].sxy, m.t2);
    m.t3 = fmaf(ri5[q], s[q].sxz, m.t3);
    m.t4 = fmaf(ri5[q], s[q].syz, m.t4);
  }
}

template <typename T>
struct LdsRec {
  using type = Src8<T>;
};
template <>
struct LdsRec<float> {
  using type = SrcF9;
};

// IMG: the sources are the mirror images of the spheres in the plane z = zw2/2 (centre z -> zw2 - z,
// stresslet M Sigma M with M = diag(1, 1, -1): the xz and yz components change sign); no image
// coincides with a receiver, and the sums always go to the chunk partials.
template <typename T, int TJ, bool IMG>
__global__ void __launch_bounds__(kMaxBlock)
    k_p2_lds(const double* __restrict__ R, const double* __restrict__ X, double* __restrict__ out,
             int n, int chunk, double P, double a2, double inv_gamma, int direct, double zw2) {
  constexpr bool f32 = sizeof(T) == 4;
  using Rec = typename LdsRec<T>::type;
  __shared__ Rec tile[TJ];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int ii = i < n ? i : n - 1;
  const int b0 = blockIdx.x * blockDim.x;
  const int b1 = min(n, b0 + (int)blockDim.x);
  // binary32 re-centres on the workgroup's first receiver; binary64 keeps lab coordinates
  const double ox = f32 ? R[3 * (int64_t)b0] : 0.0, oy = f32 ? R[3 * (int64_t)b0 + 1] : 0.0,
               oz = f32 ? R[3 * (int64_t)b0 + 2] : 0.0;
  const T xi = (T)(R[3 * (int64_t)ii] - ox), yi = (T)(R[3 * (int64_t)ii + 1] - oy),
          zi = (T)(R[3 * (int64_t)ii + 2] - oz);
  const T A24 = (T)(24.0 * a2), A42 = (T)(42.0 * a2);
  KF32 k{(float)(1.6 * a2), (float)(-2.8 * a2), -0.4f};
  // an empty asm with VGPR operands pins the constants to VGPRs (no SGPR or literal operand)
  if constexpr (f32) asm volatile("" : "+v"(k.a16), "+v"(k.n28), "+v"(k.n04));
  const int j0 = blockIdx.y * chunk;
  const int j1 = min(n, j0 + chunk);
  Total<T> tot;
  for (int jt = j0; jt < j1; jt += TJ) {
    const int cnt = min(TJ, j1 - jt);
    __syncthreads();
    for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
      const int j = jt + t;
      double sxx, syy, sxy, sxz, syz;
      basis_to_cart(X + 5 * (int64_t)j, sxx, syy, sxy, sxz, syz);
      Rec r;
      r.x = (T)(R[3 * (int64_t)j] - ox);
      r.y = (T)(R[3 * (int64_t)j + 1] - oy);
      r.z = (T)((IMG ? zw2 - R[3 * (int64_t)j + 2] : R[3 * (int64_t)j + 2]) - oz);
      r.sxx = (T)sxx;
      r.syy = (T)syy;
      r.sxy = (T)sxy;
      r.sxz = (T)(IMG ? -sxz : sxz);
      r.syz = (T)(IMG ? -syz : syz);
      if constexpr (f32) r.szz = (float)(-(sxx + syy));
      tile[t] = r;
    }
    __syncthreads();
    Mom<T> m;
    const bool self = !IMG && jt < b1 && jt + cnt > b0;  // uniform
    if constexpr (f32) {
      if (self) {
#pragma unroll 8
        for (int jj = 0; jj < cnt; ++jj) p2_pair_f32<true>(tile[jj], xi, yi, zi, k, m);
      } else {
        int jj = 0;
#pragma unroll 4
        for (; jj + 2 <= cnt; jj += 2) p2_pairs_f32<false, 2>(tile + jj, xi, yi, zi, k, m);
        for (; jj < cnt; ++jj) p2_pair_f32<false>(tile[jj], xi, yi, zi, k, m);
      }
    } else {
      if (self) {
#pragma unroll 8
        for (int jj = 0; jj < cnt; ++jj) p2_pair<T, true>(tile[jj], xi, yi, zi, A24, A42, m);
      } else {
#pragma unroll 8
        for (int jj = 0; jj < cnt; ++jj) p2_pair<T, false>(tile[jj], xi, yi, zi, A24, A42, m);
      }
    }
    tot.add(m);
  }
  if (i >= n) return;
  double v[11];
  tot.get(v);
  if constexpr (f32)
#pragma unroll
    for (int c = 0; c < 6; ++c) v[c] *= 15.0;
  p2_store(v, i, n, X, out, P, a2, inv_gamma, direct);
}

// y = x/gamma - sum_s part[s]
__global__ void k_p2_finish(const double* __restrict__ X, const double* __restrict__ part,
                            double* __restrict__ y, int64_t len, int split, double inv_gamma) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= len) return;
  double acc = 0.0;
  for (int s = 0; s < split; ++s) acc += part[s * len + k];
  y[k] = X[k] * inv_gamma - acc;
}

// y -= sum_s part[s] (the images' part of the operator)
__global__ void k_p2_finish_sub(const double* __restrict__ part, double* __restrict__ y, int64_t len, int split) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= len) return;
  double acc = 0.0;
  for (int s = 0; s < split; ++s) acc += part[s * len + k];
  y[k] -= acc;
}

inline unsigned nblk(int64_t len, int b) { return (unsigned)((len + b - 1) / b); }

template <typename T>
void p2_launch(const double* R, const double* x, double* y, double* part, double* srcbuf,
               double* orig, int64_t n, const Phys& ph, Tile t, hipStream_t s) {
  const int b = tile_block(t);
  const int tj = t.variant == 0 ? ((t.tj == 64 || t.tj == 256) ? t.tj : 128) : kSeg;
  const int split = split_for(n, t, tj);
  const int chunk = (int)((n + split - 1) / split);
  dim3 grid(nblk(n, b), split);
  double* out = split > 1 ? part : y;
  const int direct = split > 1 ? 0 : 1;
  if (t.variant == 1) {
    const bool f32 = sizeof(T) == 4;
    double* o = f32 ? orig : nullptr;
    if (f32) hipLaunchKernelGGL(k_bbox, dim3(1), dim3(256), 0, s, R, (int)n, orig);
    Src8<T>* src = reinterpret_cast<Src8<T>*>(srcbuf);
    hipLaunchKernelGGL(k_pack<T>, dim3(nblk(n, 256)), dim3(256), 0, s, R, x, src, (int)n, o);
    hipLaunchKernelGGL(k_p2_stream<T>, grid, dim3(b), 0, s, src, R, x, out, (int)n, chunk, o, ph.P,
                       ph.a2, ph.inv_gamma, direct);
  } else if (tj == 64) {
    hipLaunchKernelGGL((k_p2_lds<T, 64, false>), grid, dim3(b), 0, s, R, x, out, (int)n, chunk, ph.P, ph.a2,
                       ph.inv_gamma, direct, 0.0);
  } else if (tj == 256) {
    hipLaunchKernelGGL((k_p2_lds<T, 256, false>), grid, dim3(b), 0, s, R, x, out, (int)n, chunk, ph.P,
                       ph.a2, ph.inv_gamma, direct, 0.0);
  } else {
    hipLaunchKernelGGL((k_p2_lds<T, 128, false>), grid, dim3(b), 0, s, R, x, out, (int)n, chunk, ph.P,
                       ph.a2, ph.inv_gamma, direct, 0.0);
  }
  if (split > 1)
    hipLaunchKernelGGL(k_p2_finish, dim3(nblk(5 * n, 256)), dim3(256), 0, s, x, part, y, 5 * n,
                       split, ph.inv_gamma);
}

// y -= (the images' strain E) with the LDS kernel of tile t (the scalar-streamed variant, which packs
// records once per call, falls back to 128-record tiles of 256 receivers)
template <typename T>
void p2_image_launch(const double* R, const double* x, double* y, double* part, int64_t n, const Phys& ph,
                     double plane_z, Tile t, hipStream_t s) {
  if (t.variant != 0) t = Tile{0, 256, 128, 2048};
  const int b = tile_block(t);
  const int tj = (t.tj == 64 || t.tj == 256) ? t.tj : 128;
  const int split = split_for(n, t, tj);
  const int chunk = (int)((n + split - 1) / split);
  dim3 grid(nblk(n, b), split);
  const double zw2 = 2.0 * plane_z;
  if (tj == 64)
    hipLaunchKernelGGL((k_p2_lds<T, 64, true>), grid, dim3(b), 0, s, R, x, part, (int)n, chunk, ph.P, ph.a2,
                       ph.inv_gamma, 0, zw2);
  else if (tj == 256)
    hipLaunchKernelGGL((k_p2_lds<T, 256, true>), grid, dim3(b), 0, s, R, x, part, (int)n, chunk, ph.P, ph.a2,
                       ph.inv_gamma, 0, zw2);
  else
    hipLaunchKernelGGL((k_p2_lds<T, 128, true>), grid, dim3(b), 0, s, R, x, part, (int)n, chunk, ph.P, ph.a2,
                       ph.inv_gamma, 0, zw2);
  hipLaunchKernelGGL(k_p2_finish_sub, dim3(nblk(5 * n, 256)), dim3(256), 0, s, part, y, 5 * n, split);
}

}  // namespace

int tile_block(Tile t) { return (t.block == 64 || t.block == 128 || t.block == 256) ? t.block : 256; }

int split_for(int64_t n, Tile t, int tj) {
  const int b = tile_block(t);
  const int64_t ntile_i = (n + b - 1) / b;
  const int64_t target = t.wgs > 0 ? t.wgs : 2048;
  const int64_t max_split = std::max<int64_t>(1, (n + std::max(tj, 64) - 1) / std::max(tj, 64));
  int64_t s = (target + ntile_i - 1) / ntile_i;
  s = std::min<int64_t>(std::max<int64_t>(s, 1), max_split);
  return (int)s;
}

int64_t part_elems_max(int64_t n) {
  // up to 11 values per receiver and chunk (the fused output + operator pass)
  int64_t m = 11 * n;
  for (int k = 0; k < kTileCount; ++k) {
    const Tile& t = kTileTable[k];
    for (int tj : {64, 128, 256}) {
      const int s = split_for(n, t, tj);
      if (s > 1) m = std::max<int64_t>(m, (int64_t)s * 11 * n);
    }
  }
  return m;
}

void launch_p2(bool f32, const double* R, const double* x, double* y, double* part, double* src,
               double* orig, int64_t n, const Phys& ph, Tile t, hipStream_t s) {
  if (f32)
    p2_launch<float>(R, x, y, part, src, orig, n, ph, t, s);
  else
    p2_launch<double>(R, x, y, part, src, orig, n, ph, t, s);
}

void launch_p2_image(bool f32, const double* R, const double* x, double* y, double* part, int64_t n,
                     const Phys& ph, double plane_z, Tile t, hipStream_t s) {
  if (n <= 0) return;
  if (f32)
    p2_image_launch<float>(R, x, y, part, n, ph, plane_z, t, s);
  else
    p2_image_launch<double>(R, x, y, part, n, ph, plane_z, t, s);
}

}  // namespace mbs
