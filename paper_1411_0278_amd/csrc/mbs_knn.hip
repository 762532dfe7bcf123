// Neighbourhood features of the learned warm start (gfx950): the 16 nearest other centres of every
// sphere from a search of the cell grid, kept as a sorted list of (distance^2, index) in registers;
// ties are broken by the smaller index so the result is unique. Features per neighbour, nearest
// first: (R_j - R_i)/|R_j - R_i|, 1/|R_j - R_i|, p_j . p_i.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "mbs_grid.h"
#include "mbs_mlp.h"

namespace mbs {
namespace {

__device__ __forceinline__ bool before(double d, int j, double bd, int bj) {
  return d < bd || (d == bd && j < bj);
}

// One sphere per thread, threads in cell (Morton) order so a wavefront scans overlapping cells.
// The cells are visited in shells of growing Chebyshev radius s around the sphere's own cell; a
// sphere in a cell outside shell s is at least s*h away, so the search ends once the 16th distance
// is below that bound (or every cell has been visited).
__global__ void __launch_bounds__(256) k_knn16(GridView G, int32_t* __restrict__ nbr) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= G.n) return;
  const GridHdr H = *G.hdr;
  const int i = G.perm[k];
  const double xi = G.Rs[4 * (int64_t)k], yi = G.Rs[4 * (int64_t)k + 1], zi = G.Rs[4 * (int64_t)k + 2];
  const int cx = grid_cell1(xi, H.lo[0], H.inv_h, H.g[0]);
  const int cy = grid_cell1(yi, H.lo[1], H.inv_h, H.g[1]);
  const int cz = grid_cell1(zi, H.lo[2], H.inv_h, H.g[2]);
  const int smax = max(max(max(cx, H.g[0] - 1 - cx), max(cy, H.g[1] - 1 - cy)), max(cz, H.g[2] - 1 - cz));
  double bd[kNeigh];
  int bj[kNeigh];
#pragma unroll
  for (int q = 0; q < kNeigh; ++q) {
    bd[q] = INFINITY;
    bj[q] = 0x7fffffff;
  }
  for (int sh = 0; sh <= smax; ++sh) {
    for (int dz = -sh; dz <= sh; ++dz) {
      const int z = cz + dz;
      if (z < 0 || z >= H.g[2]) continue;
      for (int dy = -sh; dy <= sh; ++dy) {
        const int y = cy + dy;
        if (y < 0 || y >= H.g[1]) continue;
        // rows inside the shell contribute only their two end cells
        const int step = (sh > 0 && abs(dz) < sh && abs(dy) < sh) ? 2 * sh : 1;
        for (int dx = -sh; dx <= sh; dx += step) {
          const int x = cx + dx;
          if (x < 0 || x >= H.g[0]) continue;
          const int c = grid_linear(H, x, y, z);
          const int e = G.end[c];
          for (int k2 = G.start[c]; k2 < e; ++k2) {
            const int j = G.perm[k2];
            const double ddx = G.Rs[4 * (int64_t)k2] - xi, ddy = G.Rs[4 * (int64_t)k2 + 1] - yi,
                         ddz = G.Rs[4 * (int64_t)k2 + 2] - zi;
            const double d2 = ddx * ddx + ddy * ddy + ddz * ddz;
            if (j != i && before(d2, j, bd[kNeigh - 1], bj[kNeigh - 1])) {
              double d = d2;
              int id = j;
#pragma unroll
              for (int q = 0; q < kNeigh; ++q) {  // insert, keeping the list sorted
                const bool lt = before(d, id, bd[q], bj[q]);
                const double od = bd[q];
                const int oj = bj[q];
                bd[q] = lt ? d : od;
                bj[q] = lt ? id : oj;
                d = lt ? od : d;
                id = lt ? oj : id;
              }
            }
          }
        }
      }
    }
    const double reach = sh * H.h * (1.0 - 1e-9);
    if (bd[kNeigh - 1] < reach * reach) break;
  }
#pragma unroll
  for (int q = 0; q < kNeigh; ++q) nbr[(int64_t)i * kNeigh + q] = bj[q];
}

__global__ void k_features(const double* __restrict__ R, const double* __restrict__ p,
                           const int32_t* __restrict__ nbr, int n, float* __restrict__ feat,
                           const double* __restrict__ b, double gamma) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * kNeigh) return;
  const int64_t i = t / kNeigh;
  const int k = (int)(t % kNeigh);
  const int64_t j = nbr[t];
  const double rx = R[3 * j] - R[3 * i], ry = R[3 * j + 1] - R[3 * i + 1], rz = R[3 * j + 2] - R[3 * i + 2];
  const double r = sqrt(rx * rx + ry * ry + rz * rz);
  const double inv = 1.0 / r;
  const double pp = p[3 * j] * p[3 * i] + p[3 * j + 1] * p[3 * i + 1] + p[3 * j + 2] * p[3 * i + 2];
  const int per = b ? 10 : 5;  // features per neighbour
  float* f = feat + i * (kNeigh * per) + per * k;
  f[0] = (float)(rx * inv);
  f[1] = (float)(ry * inv);
  f[2] = (float)(rz * inv);
  f[3] = (float)inv;
  f[4] = (float)pp;
  if (b) {
#pragma unroll
    for (int c = 0; c < 5; ++c) f[5 + c] = (float)(gamma * b[5 * j + c]);
  }
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

void launch_knn16(const GridView& g, int32_t* nbr, hipStream_t s) {
  hipLaunchKernelGGL(k_knn16, dim3(nblk(g.n, 256)), dim3(256), 0, s, g, nbr);
}

void launch_features(const double* R, const double* p, const int32_t* nbr, int n, float* feat,
                     hipStream_t s, const double* b, double gamma) {
  hipLaunchKernelGGL(k_features, dim3(nblk((int64_t)n * kNeigh, 256)), dim3(256), 0, s, R, p, nbr, n, feat,
                     b, gamma);
}

void launch_guess_learned(const double* b, const float* out, double gamma, int64_t len, double* x,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_guess_learned, dim3(nblk(len, 256)), dim3(256), 0, s, b, out, gamma, len, x);
}

}  // namespace mbs
