// Batched solves of many independent configurations of uneven size (gfx950).
//
// All configurations advance in lockstep through the same sequence of kernels: one launch of a
// pass covers every configuration at once. The pair passes are decomposed into work items
// (configuration b, tile of 64 receivers); a 64-lane workgroup takes one item and streams the
// sources of its configuration through scalar loads (the index is wavefront-uniform), so large and
// small configurations interleave freely on the CUs and no cross-workgroup synchronisation exists
// inside a kernel. Krylov vectors of all configurations are concatenated: one basis vector is
// [5 N_total] with configuration b's segment at 5 off_b. Per-configuration scalars (Hessenberg
// matrix, Givens rotations, status) live in small arrays indexed by b. A status word per
// configuration lets converged configurations skip every later pass, so a fixed chunk of
// iterations can be replayed from a HIP graph until no configuration is active.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "mbs_batched.h"
#include "mbs_device.h"
#include "mbs_pair.h"

namespace mbs {
namespace {

constexpr int kItemMax = 256;  // receivers per work item: blockDim.x, 64, 128 or 256

// A wavefront whose first receiver lies past its configuration has nothing to do (uniform exit; the
// item kernels have no barriers).
__device__ __forceinline__ bool wave_idle(int first, int o1) { return first + (int)(threadIdx.x & ~63u) >= o1; }

inline unsigned nblk(int64_t len, int b) { return (unsigned)((len + b - 1) / b); }

__global__ void k_bpack_f(const double* __restrict__ R, const double* __restrict__ Fe,
                          const double* __restrict__ Te, const double* __restrict__ D, double P,
                          double a5_10, RecF* __restrict__ rec, int ntot) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ntot) return;
  RecF r;
  r.x = R[3 * (int64_t)j];
  r.y = R[3 * (int64_t)j + 1];
  r.z = R[3 * (int64_t)j + 2];
  r.fx = Fe ? P * Fe[3 * (int64_t)j] : 0.0;
  r.fy = Fe ? P * Fe[3 * (int64_t)j + 1] : 0.0;
  r.fz = Fe ? P * Fe[3 * (int64_t)j + 2] : 0.0;
  r.tx = Te ? P * Te[3 * (int64_t)j] : 0.0;
  r.ty = Te ? P * Te[3 * (int64_t)j + 1] : 0.0;
  r.tz = Te ? P * Te[3 * (int64_t)j + 2] : 0.0;
  r.dx = D ? a5_10 * D[3 * (int64_t)j] : 0.0;
  r.dy = D ? a5_10 * D[3 * (int64_t)j + 1] : 0.0;
  r.dz = D ? a5_10 * D[3 * (int64_t)j + 2] : 0.0;
  rec[j] = r;
}

__global__ void k_bpack_o(const double* __restrict__ R, const double* __restrict__ Fe,
                          const double* __restrict__ Te, const double* __restrict__ Sig,
                          const double* __restrict__ D, double P, double a5_10, RecO* __restrict__ rec,
                          int ntot) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ntot) return;
  RecO r;
  r.x = R[3 * (int64_t)j];
  r.y = R[3 * (int64_t)j + 1];
  r.z = R[3 * (int64_t)j + 2];
  r.fx = Fe ? P * Fe[3 * (int64_t)j] : 0.0;
  r.fy = Fe ? P * Fe[3 * (int64_t)j + 1] : 0.0;
  r.fz = Fe ? P * Fe[3 * (int64_t)j + 2] : 0.0;
  r.tx = Te ? P * Te[3 * (int64_t)j] : 0.0;
  r.ty = Te ? P * Te[3 * (int64_t)j + 1] : 0.0;
  r.tz = Te ? P * Te[3 * (int64_t)j + 2] : 0.0;
  double sxx, syy, sxy, sxz, syz;
  basis_to_cart(Sig + 5 * (int64_t)j, sxx, syy, sxy, sxz, syz);
  r.sxx = P * sxx;
  r.syy = P * syy;
  r.sxy = P * sxy;
  r.sxz = P * sxz;
  r.syz = P * syz;
  r.dx = D ? a5_10 * D[3 * (int64_t)j] : 0.0;
  r.dy = D ? a5_10 * D[3 * (int64_t)j + 1] : 0.0;
  r.dz = D ? a5_10 * D[3 * (int64_t)j + 2] : 0.0;
  r.pad = 0.0;
  rec[j] = r;
}

// source records of the operator from a concatenated 5-basis vector (X + kdev * ld; nothing once the
// Arnoldi index passes maxk, when no configuration is active any more)
__global__ void k_bpack_s(const double* __restrict__ R, const double* __restrict__ X,
                          const int* __restrict__ kdev, int maxk, int64_t ld,
                          Src8<double>* __restrict__ src, int ntot) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ntot) return;
  if (kdev && kdev[0] > maxk) return;
  const double* x = X + (kdev ? (int64_t)kdev[0] * ld : 0);
  double sxx, syy, sxy, sxz, syz;
  basis_to_cart(x + 5 * (int64_t)j, sxx, syy, sxy, sxz, syz);
  Src8<double> r;
  r.x = R[3 * (int64_t)j];
  r.y = R[3 * (int64_t)j + 1];
  r.z = R[3 * (int64_t)j + 2];
  r.sxx = sxx;
  r.syy = syy;
  r.sxy = sxy;
  r.sxz = sxz;
  r.syz = syz;
  src[j] = r;
}

// b = E[F, T, d] - c s for every configuration
template <bool HAS_T, bool HAS_D>
__global__ void __launch_bounds__(kItemMax)
    k_bp1(const int2* __restrict__ items, const int* __restrict__ off, const RecF* __restrict__ rec,
          const double* __restrict__ v2s, double cslip, double a2, double* __restrict__ b) {
  const int2 it = items[blockIdx.x];
  const int o0 = off[it.x], o1 = off[it.x + 1];
  if (wave_idle(it.y, o1)) return;
  const int i = it.y + threadIdx.x;
  const int ii = i < o1 ? i : o1 - 1;
  const double xi = rec[ii].x, yi = rec[ii].y, zi = rec[ii].z;
  const double A8 = 8.0 * a2, B16 = -3.2 * a2;
  Mom6 m;
#pragma unroll 2
  for (int j = o0; j < o1; ++j) p1_pair<true, HAS_T, HAS_D>(rec[j], xi, yi, zi, A8, B16, m);
  if (i >= o1) return;
  double e[5];
  mom6_to_basis(m, e);
#pragma unroll
  for (int c = 0; c < 5; ++c) b[5 * (int64_t)i + c] = e[c] - (v2s ? cslip * v2s[5 * (int64_t)i + c] : 0.0);
}

// y = x/gamma - E[x] for the configurations whose status equals `want`
__global__ void __launch_bounds__(kItemMax)
    k_bp2(const int2* __restrict__ items, const int* __restrict__ off, const int* __restrict__ status,
          int want, const Src8<double>* __restrict__ src, const double* __restrict__ X,
          const int* __restrict__ kdev, int64_t ld, double P, double a2, double inv_gamma,
          double* __restrict__ y) {
  const int2 it = items[blockIdx.x];
  if (status[it.x] != want) return;
  const int o0 = off[it.x], o1 = off[it.x + 1];
  if (wave_idle(it.y, o1)) return;
  const int i = it.y + threadIdx.x;
  const int ii = i < o1 ? i : o1 - 1;
  const double xi = src[ii].x, yi = src[ii].y, zi = src[ii].z;
  const double A24 = 24.0 * a2, A42 = 42.0 * a2;
  Mom<double> m;
  const int s0 = it.y, s1 = min(o1, it.y + (int)blockDim.x);  // sources that can be the receiver itself
#pragma unroll 2
  for (int j = o0; j < s0; ++j) p2_pair<double, false>(src[j], xi, yi, zi, A24, A42, m);
  for (int j = s0; j < s1; ++j) p2_pair<double, true>(src[j], xi, yi, zi, A24, A42, m);
#pragma unroll 2
  for (int j = s1; j < o1; ++j) p2_pair<double, false>(src[j], xi, yi, zi, A24, A42, m);
  if (i >= o1) return;
  const double* x = X + (kdev ? (int64_t)kdev[0] * ld : 0);
  double e[5];
  p2_strain(&m.pxx, P, a2, e);
#pragma unroll
  for (int c = 0; c < 5; ++c) y[5 * (int64_t)i + c] = x[5 * (int64_t)i + c] * inv_gamma - e[c];
}

// Near-field lists of every configuration (partners only within the sphere's own configuration):
// each work item scans its configuration's centres in index order, so a list holds the first
// kNearCap partners with 2a <= r < r_c, as the single-configuration build does.
__global__ void __launch_bounds__(kItemMax)
    k_bnear(const int2* __restrict__ items, const int* __restrict__ off, const double* __restrict__ R,
            double rmin2, double rc2, int* __restrict__ cnt, int* __restrict__ list) {
  const int2 it = items[blockIdx.x];
  const int o0 = off[it.x], o1 = off[it.x + 1];
  const int i = it.y + threadIdx.x;
  if (i >= o1) return;
  const double xi = R[3 * (int64_t)i], yi = R[3 * (int64_t)i + 1], zi = R[3 * (int64_t)i + 2];
  int c = 0;
  for (int j = o0; j < o1; ++j) {
    const double dx = xi - R[3 * (int64_t)j], dy = yi - R[3 * (int64_t)j + 1], dz = zi - R[3 * (int64_t)j + 2];
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (j != i && r2 >= rmin2 && r2 < rc2 && c < kNearCap) list[(int64_t)i * kNearCap + c++] = j;
  }
  cnt[i] = c;
}

// outputs for every configuration
template <bool HAS_T, bool HAS_D>
__global__ void __launch_bounds__(kItemMax)
    k_bp3(const int2* __restrict__ items, const int* __restrict__ off, const RecO* __restrict__ rec,
          double a2, double mu_t, double mu_r, double slip_S, const double* __restrict__ v1s,
          const double* __restrict__ v2s, const double* __restrict__ Fe, const double* __restrict__ Te,
          const double* __restrict__ Sig, double* __restrict__ V, double* __restrict__ W,
          double* __restrict__ S, double* __restrict__ SigOut) {
  const int2 it = items[blockIdx.x];
  const int o0 = off[it.x], o1 = off[it.x + 1];
  if (wave_idle(it.y, o1)) return;
  const int i = it.y + threadIdx.x;
  const int ii = i < o1 ? i : o1 - 1;
  const double xi = rec[ii].x, yi = rec[ii].y, zi = rec[ii].z;
  const double A2_2 = 2.0 * a2, A2_23 = 2.0 * a2 / 3.0, A8 = 8.0 * a2, B16 = -3.2 * a2;
  UW a;
#pragma unroll 2
  for (int j = o0; j < o1; ++j) p3_pair<true, HAS_T, HAS_D>(rec[j], xi, yi, zi, A2_2, A2_23, A8, B16, a);
  if (i >= o1) return;
  const double u[6] = {a.ux, a.uy, a.uz, a.wx, a.wy, a.wz};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    V[3 * (int64_t)i + c] = u[c] + (Fe ? mu_t * Fe[3 * (int64_t)i + c] : 0.0) -
                            (v1s ? v1s[3 * (int64_t)i + c] : 0.0);
    W[3 * (int64_t)i + c] = u[3 + c] + (Te ? mu_r * Te[3 * (int64_t)i + c] : 0.0);
  }
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    const double sg = Sig[5 * (int64_t)i + c];
    S[5 * (int64_t)i + c] = sg + (v2s ? slip_S * v2s[5 * (int64_t)i + c] : 0.0);
    if (SigOut) SigOut[5 * (int64_t)i + c] = sg;
  }
}

__device__ __forceinline__ double block_sum256(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

// h[b][i] = <V_i, w> over configuration b's segment, i < nv (nv = kdev + 1 or nv_fixed): one
// workgroup per (configuration, vector), so a batch keeps the whole GPU busy even when a few large
// configurations dominate; w of a configuration stays in L2 across its vectors.
__global__ void __launch_bounds__(256)
    k_bdots(const double* __restrict__ V, int64_t ld, const int* __restrict__ kdev, int nv_fixed,
            const double* __restrict__ w, const int* __restrict__ off, const int* __restrict__ status,
            int want, double* __restrict__ h, int hstride) {
  __shared__ double red[4];
  const int b = blockIdx.x, i = blockIdx.y;
  const int nv = kdev ? kdev[0] + 1 : nv_fixed;
  if (i >= nv || status[b] != want) return;  // uniform over the workgroup
  const int64_t s0 = 5 * (int64_t)off[b], s1 = 5 * (int64_t)off[b + 1];
  const double* v = V + (int64_t)i * ld;
  double acc = 0.0;
  for (int64_t t = s0 + threadIdx.x; t < s1; t += blockDim.x) acc = fma(v[t], w[t], acc);
  const double sum = block_sum256(acc, red);
  if (threadIdx.x == 0) h[(int64_t)b * hstride + i] = sum;
}

// w += sign * sum_{i < nv} h[b][i] V_i for elements of configurations with status `want`
__global__ void k_baxpy(const double* __restrict__ V, int64_t ld, const int* __restrict__ kdev,
                        const int* __restrict__ nvb, int nv_fixed, const double* __restrict__ h,
                        int hstride, double sign, const int* __restrict__ cid,
                        const int* __restrict__ status, int want, double* __restrict__ w, int64_t len) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= len) return;
  const int b = cid[t / 5];
  if (status[b] != want) return;
  const int nv = nvb ? nvb[b] : (kdev ? kdev[0] + 1 : nv_fixed);
  const double* hb = h + (int64_t)b * hstride;
  double acc = 0.0;
  for (int i = 0; i < nv; ++i) acc = fma(hb[i], V[(int64_t)i * ld + t], acc);
  w[t] = fma(sign, acc, w[t]);
}

struct BState {
  double *H, *cs, *sn, *g, *y, *h1, *h2, *nsq, *bnorm, *hk1, *resid;
  int *status, *kend, *iters;
  unsigned long long *t0, *t1;
};

// Givens update of every active configuration at Arnoldi step k = kdev[0]
__global__ void k_bgivens(BState st, int nconf, int m, const int* __restrict__ kdev, double tol,
                          int max_iter) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nconf || st.status[b] != kActive) return;
  const int k = kdev[0];
  const int hs = m + 2;
  double* col = st.H + (int64_t)b * (m + 1) * (m + 1) + (int64_t)k * (m + 1);
  double* cs = st.cs + (int64_t)b * hs;
  double* sn = st.sn + (int64_t)b * hs;
  double* g = st.g + (int64_t)b * hs;
  const double* h1 = st.h1 + (int64_t)b * hs;
  const double* h2 = st.h2 + (int64_t)b * hs;
  for (int i = 0; i <= k; ++i) col[i] = h1[i] + h2[i];
  const double hk1 = sqrt(fmax(st.nsq[b], 0.0));
  st.hk1[b] = hk1;
  col[k + 1] = hk1;
  for (int i = 0; i < k; ++i) {
    const double t = cs[i] * col[i] + sn[i] * col[i + 1];
    col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
    col[i] = t;
  }
  const double den = hypot(col[k], hk1);
  cs[k] = den > 0.0 ? col[k] / den : 1.0;
  sn[k] = den > 0.0 ? hk1 / den : 0.0;
  col[k] = den;
  col[k + 1] = 0.0;
  g[k + 1] = -sn[k] * g[k];
  g[k] = cs[k] * g[k];
  st.iters[b] += 1;
  const double est = fabs(g[k + 1]);
  if (est <= tol * st.bnorm[b] || k + 1 >= m || !(hk1 > 1e-300 * st.bnorm[b]) || st.iters[b] >= max_iter) {
    st.status[b] = kCycleDone;
    st.kend[b] = k + 1;
  }
}

// V_{k+1} = w / hk1 for configurations still active
__global__ void k_bscale(const double* __restrict__ w, const double* __restrict__ hk1,
                         const int* __restrict__ cid, const int* __restrict__ status,
                         double* __restrict__ V, int64_t ld, const int* __restrict__ kdev, int64_t len) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= len) return;
  const int b = cid[t / 5];
  if (status[b] != kActive) return;
  V[(int64_t)(kdev[0] + 1) * ld + t] = w[t] / hk1[b];
}

__global__ void k_binc(int* __restrict__ kdev) {
  if (threadIdx.x == 0 && blockIdx.x == 0) kdev[0] += 1;
}

__global__ void k_bset_int(int* __restrict__ p, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) p[0] = v;
}

__global__ void k_bset_ints(int* __restrict__ p, int n, int v) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = v;
}

__global__ void k_bfill(double* __restrict__ x, double v, int64_t len) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < len) x[t] = v;
}

// y = H^{-1} g for configurations that finished a cycle
__global__ void k_bbacksolve(BState st, int nconf, int m) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nconf || st.status[b] != kCycleDone) return;
  const int k = st.kend[b], hs = m + 2;
  const double* H = st.H + (int64_t)b * (m + 1) * (m + 1);
  const double* g = st.g + (int64_t)b * hs;
  double* y = st.y + (int64_t)b * hs;
  for (int i = k - 1; i >= 0; --i) {
    double s = g[i];
    for (int j = i + 1; j < k; ++j) s -= H[(int64_t)j * (m + 1) + i] * y[j];
    const double d = H[(int64_t)i * (m + 1) + i];
    y[i] = d != 0.0 ? s / d : 0.0;
  }
}

// r = b - w for configurations that finished a cycle
__global__ void k_bresid(const double* __restrict__ bv, const double* __restrict__ w,
                         const int* __restrict__ cid, const int* __restrict__ status,
                         double* __restrict__ r, int64_t len) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= len) return;
  if (status[cid[t / 5]] != kCycleDone) return;
  r[t] = bv[t] - w[t];
}

// After the true residual: finish, or restart GMRES from the residual.
__global__ void k_bcheck(BState st, int nconf, int m, double tol, int max_iter) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nconf || st.status[b] != kCycleDone) return;
  const double beta = sqrt(fmax(st.nsq[b], 0.0));
  st.resid[b] = st.bnorm[b] > 0.0 ? beta / st.bnorm[b] : 0.0;
  if (beta <= tol * st.bnorm[b] || st.iters[b] >= max_iter) {
    st.status[b] = kFinal;
    st.t1[b] = wall_clock64();
    return;
  }
  double* g = st.g + (int64_t)b * (m + 2);
  g[0] = beta;
  for (int i = 1; i <= m; ++i) g[i] = 0.0;
  st.hk1[b] = beta;  // V_0 = r / beta
  st.status[b] = kRestart;
}

// first cycle: ||b|| known in nsq; x = 0 so r = b
__global__ void k_binit(BState st, int nconf, int m) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nconf) return;
  const double beta = sqrt(fmax(st.nsq[b], 0.0));
  st.bnorm[b] = beta;
  st.iters[b] = 0;
  st.kend[b] = 0;
  st.resid[b] = 0.0;
  st.t0[b] = wall_clock64();
  double* g = st.g + (int64_t)b * (m + 2);
  g[0] = beta;
  for (int i = 1; i <= m; ++i) g[i] = 0.0;
  st.hk1[b] = beta;
  if (beta > 0.0) {
    st.status[b] = kActive;
  } else {
    st.status[b] = kFinal;
    st.t1[b] = st.t0[b];
  }
}

// V_0 = r / hk1[b] (configurations with status `want`)
__global__ void k_bstart(const double* __restrict__ r, const double* __restrict__ hk1,
                         const int* __restrict__ cid, const int* __restrict__ status, int want,
                         double* __restrict__ V0, int64_t len) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= len) return;
  const int b = cid[t / 5];
  if (status[b] != want) return;
  V0[t] = r[t] / hk1[b];
}

__global__ void k_bcount(const int* __restrict__ status, int nconf, int want, int invert, int* __restrict__ out) {
  __shared__ int red[256];
  int c = 0;
  for (int b = threadIdx.x; b < nconf; b += blockDim.x) c += (status[b] == want) != (invert != 0) ? 1 : 0;
  red[threadIdx.x] = c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// One workgroup: once no configuration is inside an Arnoldi cycle, the ones waiting to restart
// become active and the shared step index returns to 0.
__global__ void __launch_bounds__(256) k_bgate(int* __restrict__ status, int nconf, int* __restrict__ kdev) {
  __shared__ int red[256];
  int c = 0;
  for (int b = threadIdx.x; b < nconf; b += blockDim.x) c += status[b] == kActive ? 1 : 0;
  red[threadIdx.x] = c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (red[0] != 0) return;  // (uniform across the workgroup)
  for (int b = threadIdx.x; b < nconf; b += blockDim.x)
    if (status[b] == kRestart) status[b] = kActive;
  if (threadIdx.x == 0) kdev[0] = 0;
}

}  // namespace

// ------------------------------------------------------------------ launchers
void batched_pack_f(const double* R, const double* Fe, const double* Te, const double* D,
                    const Phys& ph, RecF* rec, int ntot, hipStream_t s) {
  hipLaunchKernelGGL(k_bpack_f, dim3(nblk(ntot, 256)), dim3(256), 0, s, R, Fe, Te, D, ph.P, ph.a5_10,
                     rec, ntot);
}

void batched_p1(const int2* items, int nitems, int item, const int* off, const RecF* rec, const double* v2s,
                bool has_t, bool has_d, const Phys& ph, double* b, hipStream_t s) {
#define MBS_BP1(HT, HD)                                                                          \
  hipLaunchKernelGGL((k_bp1<HT, HD>), dim3(nitems), dim3(item), 0, s, items, off, rec, v2s,     \
                     ph.c_slip, ph.a2, b)
  if (has_t && has_d)
    MBS_BP1(true, true);
  else if (has_t)
    MBS_BP1(true, false);
  else if (has_d)
    MBS_BP1(false, true);
  else
    MBS_BP1(false, false);
#undef MBS_BP1
}

void batched_pack_s(const double* R, const double* X, const int* kdev, int maxk, int64_t ld,
                    Src8<double>* src, int ntot, hipStream_t s) {
  hipLaunchKernelGGL(k_bpack_s, dim3(nblk(ntot, 256)), dim3(256), 0, s, R, X, kdev, maxk, ld, src, ntot);
}

void batched_p2(const int2* items, int nitems, int item, const int* off, const int* status, int want,
                const Src8<double>* src, const double* X, const int* kdev, int64_t ld, const Phys& ph,
                double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_bp2, dim3(nitems), dim3(item), 0, s, items, off, status, want, src, X, kdev,
                     ld, ph.P, ph.a2, ph.inv_gamma, y);
}

void batched_near_build(const int2* items, int nitems, int item, const int* off, const double* R, double rmin,
                        double rc, int* cnt, int* list, hipStream_t s) {
  hipLaunchKernelGGL(k_bnear, dim3(nitems), dim3(item), 0, s, items, off, R, rmin * rmin, rc * rc, cnt, list);
}

void batched_pack_o(const double* R, const double* Fe, const double* Te, const double* Sig,
                    const double* D, const Phys& ph, RecO* rec, int ntot, hipStream_t s) {
  hipLaunchKernelGGL(k_bpack_o, dim3(nblk(ntot, 256)), dim3(256), 0, s, R, Fe, Te, Sig, D, ph.P,
                     ph.a5_10, rec, ntot);
}

void batched_p3(const int2* items, int nitems, int item, const int* off, const RecO* rec, bool has_t, bool has_d,
                const Phys& ph, const double* v1s, const double* v2s, const double* Fe,
                const double* Te, const double* Sig, double* V, double* W, double* S, double* SigOut,
                hipStream_t s) {
#define MBS_BP3(HT, HD)                                                                              \
  hipLaunchKernelGGL((k_bp3<HT, HD>), dim3(nitems), dim3(item), 0, s, items, off, rec, ph.a2,      \
                     ph.mu_t, ph.mu_r, ph.slip_S, v1s, v2s, Fe, Te, Sig, V, W, S, SigOut)
  if (has_t && has_d)
    MBS_BP3(true, true);
  else if (has_t)
    MBS_BP3(true, false);
  else if (has_d)
    MBS_BP3(false, true);
  else
    MBS_BP3(false, false);
#undef MBS_BP3
}

void batched_dots(const double* V, int64_t ld, const int* kdev, int nv_fixed, const double* w,
                  const int* off, const int* status, int want, double* h, int hstride, int nconf,
                  hipStream_t s) {
  // with kdev the vector count is read on the device; hstride = m + 2 bounds it by m + 1
  const int nv_max = kdev ? hstride - 1 : nv_fixed;
  hipLaunchKernelGGL(k_bdots, dim3(nconf, nv_max), dim3(256), 0, s, V, ld, kdev, nv_fixed, w, off, status,
                     want, h, hstride);
}

void batched_axpy(const double* V, int64_t ld, const int* kdev, const int* nvb, int nv_fixed,
                  const double* h, int hstride, double sign, const int* cid, const int* status,
                  int want, double* w, int64_t len, hipStream_t s) {
  hipLaunchKernelGGL(k_baxpy, dim3(nblk(len, 256)), dim3(256), 0, s, V, ld, kdev, nvb, nv_fixed, h,
                     hstride, sign, cid, status, want, w, len);
}

void batched_givens(const BatchState& b, int nconf, int m, const int* kdev, double tol, int max_iter,
                    hipStream_t s) {
  BState st{b.H, b.cs, b.sn, b.g, b.y, b.h1, b.h2, b.nsq, b.bnorm, b.hk1, b.resid,
            b.status, b.kend, b.iters, b.t0, b.t1};
  hipLaunchKernelGGL(k_bgivens, dim3(nblk(nconf, 64)), dim3(64), 0, s, st, nconf, m, kdev, tol, max_iter);
}

void batched_scale(const double* w, const double* hk1, const int* cid, const int* status, double* V,
                   int64_t ld, const int* kdev, int64_t len, hipStream_t s) {
  hipLaunchKernelGGL(k_bscale, dim3(nblk(len, 256)), dim3(256), 0, s, w, hk1, cid, status, V, ld, kdev,
                     len);
}

void batched_inc(int* kdev, hipStream_t s) { hipLaunchKernelGGL(k_binc, dim3(1), dim3(64), 0, s, kdev); }
void batched_set_int(int* p, int v, hipStream_t s) {
  hipLaunchKernelGGL(k_bset_int, dim3(1), dim3(64), 0, s, p, v);
}
void batched_set_ints(int* p, int n, int v, hipStream_t s) {
  hipLaunchKernelGGL(k_bset_ints, dim3(nblk(n, 256)), dim3(256), 0, s, p, n, v);
}
void batched_fill(double* x, double v, int64_t len, hipStream_t s) {
  hipLaunchKernelGGL(k_bfill, dim3(nblk(len, 256)), dim3(256), 0, s, x, v, len);
}

void batched_backsolve(const BatchState& b, int nconf, int m, hipStream_t s) {
  BState st{b.H, b.cs, b.sn, b.g, b.y, b.h1, b.h2, b.nsq, b.bnorm, b.hk1, b.resid,
            b.status, b.kend, b.iters, b.t0, b.t1};
  hipLaunchKernelGGL(k_bbacksolve, dim3(nblk(nconf, 64)), dim3(64), 0, s, st, nconf, m);
}

void batched_resid(const double* bv, const double* w, const int* cid, const int* status, double* r,
                   int64_t len, hipStream_t s) {
  hipLaunchKernelGGL(k_bresid, dim3(nblk(len, 256)), dim3(256), 0, s, bv, w, cid, status, r, len);
}

void batched_check(const BatchState& b, int nconf, int m, double tol, int max_iter, hipStream_t s) {
  BState st{b.H, b.cs, b.sn, b.g, b.y, b.h1, b.h2, b.nsq, b.bnorm, b.hk1, b.resid,
            b.status, b.kend, b.iters, b.t0, b.t1};
  hipLaunchKernelGGL(k_bcheck, dim3(nblk(nconf, 64)), dim3(64), 0, s, st, nconf, m, tol, max_iter);
}

void batched_init(const BatchState& b, int nconf, int m, hipStream_t s) {
  BState st{b.H, b.cs, b.sn, b.g, b.y, b.h1, b.h2, b.nsq, b.bnorm, b.hk1, b.resid,
            b.status, b.kend, b.iters, b.t0, b.t1};
  hipLaunchKernelGGL(k_binit, dim3(nblk(nconf, 64)), dim3(64), 0, s, st, nconf, m);
}

void batched_start(const double* r, const double* hk1, const int* cid, const int* status, int want,
                   double* V0, int64_t len, hipStream_t s) {
  hipLaunchKernelGGL(k_bstart, dim3(nblk(len, 256)), dim3(256), 0, s, r, hk1, cid, status, want, V0, len);
}

void batched_count(const int* status, int nconf, int want, int* out, hipStream_t s) {
  hipLaunchKernelGGL(k_bcount, dim3(1), dim3(256), 0, s, status, nconf, want, 0, out);
}

void batched_count_not(const int* status, int nconf, int unwanted, int* out, hipStream_t s) {
  hipLaunchKernelGGL(k_bcount, dim3(1), dim3(256), 0, s, status, nconf, unwanted, 1, out);
}

void batched_gate(int* status, int nconf, int* kdev, hipStream_t s) {
  hipLaunchKernelGGL(k_bgate, dim3(1), dim3(256), 0, s, status, nconf, kdev);
}

}  // namespace mbs
