// Near-field right preconditioner of the stresslet system (gfx950).
//
// The system matrix is A = I/gamma - K with K the all-pairs strain-from-stresslet operator. Its
// spread around 1/gamma comes mostly from close pairs, so M = I/gamma - K_near, K_near restricted to
// pairs closer than a cutoff r_c, captures the stiff part. GMRES runs on A M^{-1} with the
// Neumann approximation of even order k, M^{-1} v = gamma (v + X v + ... + X^k v), X = gamma K_near,
// formed by k sparse passes over a few neighbours per sphere (t = gamma v + gamma^2 K_near v, then
// k - 1 times t <- gamma v + gamma K_near t). It is symmetric and, unlike odd truncations, positive
// definite for any X (1 + x + ... + x^k > 0 for every real eigenvalue x of the symmetric X when k
// is even). The solution x = M^{-1} u is unchanged; only the iteration count drops.
//
// Neighbour lists: a search of the cell grid keeps, for each sphere, the kNearCap other spheres of
// smallest index with 2a <= r < r_c, in index order (deterministic); beyond that capacity the
// preconditioner simply ignores the extra pairs. Overlapping pairs (r < 2a, unphysical but
// reachable by a time stepper) stay out: their blocks grow like r^-5 and would make the truncated
// Neumann series a poor, even harmful, approximation.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "mbs_device.h"
#include "mbs_grid.h"
#include "mbs_internal.h"
#include "mbs_pair.h"

namespace mbs {
namespace {

constexpr int kTile = 256;

// All-pairs variant: sources in index order, so the first kNearCap partners are the smallest.
__global__ void __launch_bounds__(256) k_near_build_dense(const double* __restrict__ R, int n,
                                                          const GridHdr* __restrict__ hdr, double rmin2,
                                                          double rc2, int* __restrict__ cnt,
                                                          int* __restrict__ list) {
  if (!grid_dense(hdr)) return;
  __shared__ double tx[kTile], ty[kTile], tz[kTile];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int ii = i < n ? i : n - 1;
  const double xi = R[3 * (int64_t)ii], yi = R[3 * (int64_t)ii + 1], zi = R[3 * (int64_t)ii + 2];
  int c = 0;
  for (int jt = 0; jt < n; jt += kTile) {
    const int m = min(kTile, n - jt);
    __syncthreads();
    for (int t = threadIdx.x; t < m; t += blockDim.x) {
      tx[t] = R[3 * (int64_t)(jt + t)];
      ty[t] = R[3 * (int64_t)(jt + t) + 1];
      tz[t] = R[3 * (int64_t)(jt + t) + 2];
    }
    __syncthreads();
    for (int jj = 0; jj < m; ++jj) {
      const double dx = xi - tx[jj], dy = yi - ty[jj], dz = zi - tz[jj];
      const double r2 = dx * dx + dy * dy + dz * dz;
      const int j = jt + jj;
      if (j != ii && r2 >= rmin2 && r2 < rc2 && c < kNearCap) {
        if (i < n) list[(int64_t)i * kNearCap + c] = j;
        ++c;
      }
    }
  }
  if (i < n) cnt[i] = c;
}

// One sphere per thread, threads in cell (Morton) order. The cell edge is at least r_c, so every
// partner lies in the 27 cells around the sphere's own. The list is a sorted register array that
// keeps the kNearCap smallest partner indices (an insertion network, taken only by candidates
// below the current largest), so a crowded neighbourhood costs one compare per extra candidate.
__global__ void __launch_bounds__(256)
    k_near_build(GridView G, double rmin2, double rc2, int* __restrict__ cnt, int* __restrict__ list) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= G.n || grid_dense(G.hdr)) return;
  const GridHdr H = *G.hdr;
  const int i = G.perm[k];
  const double xi = G.Rs[4 * (int64_t)k], yi = G.Rs[4 * (int64_t)k + 1], zi = G.Rs[4 * (int64_t)k + 2];
  const int cx = grid_cell1(xi, H.lo[0], H.inv_h, H.g[0]);
  const int cy = grid_cell1(yi, H.lo[1], H.inv_h, H.g[1]);
  const int cz = grid_cell1(zi, H.lo[2], H.inv_h, H.g[2]);
  int L[kNearCap];
#pragma unroll
  for (int q = 0; q < kNearCap; ++q) L[q] = 0x7fffffff;
  int c = 0;
  for (int z = max(cz - 1, 0); z <= min(cz + 1, H.g[2] - 1); ++z)
    for (int y = max(cy - 1, 0); y <= min(cy + 1, H.g[1] - 1); ++y)
      for (int x = max(cx - 1, 0); x <= min(cx + 1, H.g[0] - 1); ++x) {
        const int cell = grid_linear(H, x, y, z);
        const int e = G.end[cell];
        for (int k2 = G.start[cell]; k2 < e; ++k2) {
          const int j = G.perm[k2];
          const double dx = xi - G.Rs[4 * (int64_t)k2], dy = yi - G.Rs[4 * (int64_t)k2 + 1],
                       dz = zi - G.Rs[4 * (int64_t)k2 + 2];
          const double r2 = dx * dx + dy * dy + dz * dz;
          if (j == i || !(r2 >= rmin2 && r2 < rc2)) continue;
          ++c;
          if (j < L[kNearCap - 1]) {
            int v = j;
#pragma unroll
            for (int q = 0; q < kNearCap; ++q) {
              const bool lt = v < L[q];
              const int o = L[q];
              L[q] = lt ? v : o;
              v = lt ? o : v;
            }
          }
        }
      }
  c = min(c, kNearCap);
  int* out = list + (int64_t)i * kNearCap;
#pragma unroll
  for (int q = 0; q < kNearCap; ++q)
    if (q < c) out[q] = L[q];
  cnt[i] = c;
}

// y = alpha x + beta K_near z, z = Z or (Z == NULL) x; x = X + kdev[0] * ld when kdev is given (a
// Krylov vector whose index lives on the device)
__global__ void k_near_apply(const double* __restrict__ R, const double* __restrict__ X0,
                             const int* __restrict__ kdev, int64_t ld, const double* __restrict__ Z0,
                             const int* __restrict__ cnt, const int* __restrict__ list, int n, double P,
                             double a2, double alpha, double beta, double* __restrict__ Y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double* __restrict__ X = X0 + (kdev ? (int64_t)kdev[0] * ld : 0);
  const double* __restrict__ Z = Z0 ? Z0 : X;
  const double xi = R[3 * (int64_t)i], yi = R[3 * (int64_t)i + 1], zi = R[3 * (int64_t)i + 2];
  const double A24 = 24.0 * a2, A42 = 42.0 * a2;
  Mom<double> m;
  const int c = cnt[i];
  for (int k = 0; k < c; ++k) {
    const int j = list[(int64_t)i * kNearCap + k];
    Src8<double> s;
    s.x = R[3 * (int64_t)j];
    s.y = R[3 * (int64_t)j + 1];
    s.z = R[3 * (int64_t)j + 2];
    basis_to_cart(Z + 5 * (int64_t)j, s.sxx, s.syy, s.sxy, s.sxz, s.syz);
    p2_pair<double, false>(s, xi, yi, zi, A24, A42, m);
  }
  double e[5];
  p2_strain(&m.pxx, P, a2, e);
#pragma unroll
  for (int q = 0; q < 5; ++q) Y[5 * (int64_t)i + q] = alpha * X[5 * (int64_t)i + q] + beta * e[q];
}

inline unsigned nblk(int64_t len, int b) { return (unsigned)((len + b - 1) / b); }

}  // namespace

void launch_near_build(const GridView& g, const double* R, double rmin, double rc, int* cnt, int* list,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_near_build, dim3(nblk(g.n, 256)), dim3(256), 0, s, g, rmin * rmin, rc * rc, cnt, list);
  hipLaunchKernelGGL(k_near_build_dense, dim3(nblk(g.n, 256)), dim3(256), 0, s, R, g.n, g.hdr, rmin * rmin,
                     rc * rc, cnt, list);
}

void launch_near_apply(const double* R, const double* x, const int* cnt, const int* list, int64_t n,
                       const Phys& ph, double* y, hipStream_t s, const int* kdev, int64_t ld, double* tmp,
                       int order) {
  const double g = ph.gamma;
  if (!tmp || order < 2) {  // first order: y = gamma x + gamma^2 K x
    hipLaunchKernelGGL(k_near_apply, dim3(nblk(n, 128)), dim3(128), 0, s, R, x, kdev, ld, nullptr, cnt, list,
                       (int)n, ph.P, ph.a2, g, g * g, y);
    return;
  }
  // order k: t_1 = gamma x + gamma^2 K x, t_j = gamma x + gamma K t_{j-1} (= gamma sum_{i<=j} X^i x),
  // y = t_k; the partial sums ping-pong between the two halves of tmp
  double* ta = tmp;
  double* tb = tmp + 5 * n;
  hipLaunchKernelGGL(k_near_apply, dim3(nblk(n, 128)), dim3(128), 0, s, R, x, kdev, ld, nullptr, cnt, list,
                     (int)n, ph.P, ph.a2, g, g * g, ta);
  for (int j = 2; j < order; ++j) {
    hipLaunchKernelGGL(k_near_apply, dim3(nblk(n, 128)), dim3(128), 0, s, R, x, kdev, ld, ta, cnt, list,
                       (int)n, ph.P, ph.a2, g, g, tb);
    double* t = ta;
    ta = tb;
    tb = t;
  }
  hipLaunchKernelGGL(k_near_apply, dim3(nblk(n, 128)), dim3(128), 0, s, R, x, kdev, ld, ta, cnt, list,
                     (int)n, ph.P, ph.a2, g, g, y);
}

}  // namespace mbs
