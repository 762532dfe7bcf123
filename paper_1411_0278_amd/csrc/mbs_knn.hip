// Neighbourhood features of the learned warm start (gfx950): the 16 nearest other centres of every
// sphere by an all-pairs scan (the same all-pairs traversal as the operator: positions staged in LDS
// tiles, one receiver per thread), kept as a sorted list of (distance^2, index) in registers; ties
// are broken by the smaller index so the result is unique. Features per neighbour, nearest first:
// (R_j - R_i)/|R_j - R_i|, 1/|R_j - R_i|, p_j . p_i.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "mbs_mlp.h"

namespace mbs {
namespace {

constexpr int kTile = 256;

__device__ __forceinline__ bool before(double d, int j, double bd, int bj) {
  return d < bd || (d == bd && j < bj);
}

__global__ void __launch_bounds__(256) k_knn16(const double* __restrict__ R, int n, int32_t* __restrict__ nbr) {
  __shared__ double tx[kTile], ty[kTile], tz[kTile];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int ii = i < n ? i : n - 1;
  const double xi = R[3 * (int64_t)ii], yi = R[3 * (int64_t)ii + 1], zi = R[3 * (int64_t)ii + 2];
  double bd[kNeigh];
  int bj[kNeigh];
#pragma unroll
  for (int k = 0; k < kNeigh; ++k) {
    bd[k] = INFINITY;
    bj[k] = 0x7fffffff;
  }
  for (int jt = 0; jt < n; jt += kTile) {
    const int cnt = min(kTile, n - jt);
    __syncthreads();
    for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
      tx[t] = R[3 * (int64_t)(jt + t)];
      ty[t] = R[3 * (int64_t)(jt + t) + 1];
      tz[t] = R[3 * (int64_t)(jt + t) + 2];
    }
    __syncthreads();
    for (int jj = 0; jj < cnt; ++jj) {
      const int j = jt + jj;
      const double dx = tx[jj] - xi, dy = ty[jj] - yi, dz = tz[jj] - zi;
      const double d2 = dx * dx + dy * dy + dz * dz;
      if (j != ii && before(d2, j, bd[kNeigh - 1], bj[kNeigh - 1])) {
        double d = d2;
        int id = j;
#pragma unroll
        for (int k = 0; k < kNeigh; ++k) {  // insert, keeping the list sorted
          const bool lt = before(d, id, bd[k], bj[k]);
          const double od = bd[k];
          const int oj = bj[k];
          bd[k] = lt ? d : od;
          bj[k] = lt ? id : oj;
          d = lt ? od : d;
          id = lt ? oj : id;
        }
      }
    }
  }
  if (i >= n) return;
#pragma unroll
  for (int k = 0; k < kNeigh; ++k) nbr[(int64_t)i * kNeigh + k] = bj[k];
}

__global__ void k_features(const double* __restrict__ R, const double* __restrict__ p,
                           const int32_t* __restrict__ nbr, int n, float* __restrict__ feat) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * kNeigh) return;
  const int64_t i = t / kNeigh;
  const int k = (int)(t % kNeigh);
  const int64_t j = nbr[t];
  const double rx = R[3 * j] - R[3 * i], ry = R[3 * j + 1] - R[3 * i + 1], rz = R[3 * j + 2] - R[3 * i + 2];
  const double r = sqrt(rx * rx + ry * ry + rz * rz);
  const double inv = 1.0 / r;
  const double pp = p[3 * j] * p[3 * i] + p[3 * j + 1] * p[3 * i + 1] + p[3 * j + 2] * p[3 * i + 2];
  float* f = feat + i * kMlpIn + 5 * k;
  f[0] = (float)(rx * inv);
  f[1] = (float)(ry * inv);
  f[2] = (float)(rz * inv);
  f[3] = (float)inv;
  f[4] = (float)pp;
}

__global__ void k_guess_learned(const double* __restrict__ b, const float* __restrict__ out, double gamma,
                                int64_t len, double* __restrict__ x) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < len) x[k] = gamma * b[k] + (double)out[k];
}

// target of the network: Sigma - gamma b (float32)
__global__ void k_target(const double* __restrict__ Sig, const double* __restrict__ b, double gamma,
                         int64_t len, float* __restrict__ t) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < len) t[k] = (float)(Sig[k] - gamma * b[k]);
}

inline unsigned nblk(int64_t len, int b) { return (unsigned)((len + b - 1) / b); }

}  // namespace

void launch_target(const double* Sig, const double* b, double gamma, int64_t len, float* t,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_target, dim3(nblk(len, 256)), dim3(256), 0, s, Sig, b, gamma, len, t);
}

void launch_knn16(const double* R, int n, int32_t* nbr, hipStream_t s) {
  hipLaunchKernelGGL(k_knn16, dim3(nblk(n, 256)), dim3(256), 0, s, R, n, nbr);
}

void launch_features(const double* R, const double* p, const int32_t* nbr, int n, float* feat,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_features, dim3(nblk((int64_t)n * kNeigh, 256)), dim3(256), 0, s, R, p, nbr, n, feat);
}

void launch_guess_learned(const double* b, const float* out, double gamma, int64_t len, double* x,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_guess_learned, dim3(nblk(len, 256)), dim3(256), 0, s, b, out, gamma, len, x);
}

}  // namespace mbs
