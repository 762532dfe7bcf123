// Cell grid over the sphere centres (gfx950): bounding box, cell keys, stable radix sort by Morton
// key, per-cell ranges and the centres in sorted order. Five small launches plus the sort; O(n).
//
// The sort is a least-significant-digit radix sort of the 30-bit keys with their sphere indices:
// three passes of 10-bit digits. Each pass counts the digits of every tile of 1024 keys (LDS
// histogram), scans the counts across tiles for each digit (one wavefront per digit) and across
// digits (one workgroup), and scatters: a tile's keys are taken in order, 256 at a time; within a
// wavefront, lanes holding the same digit find each other by ballots over the digit's bits, and a
// key's rank among them plus the counts of the earlier wavefronts and rounds gives its place.
// Keys therefore keep their input order among equal digits (stable), so the final order is by key
// and then by sphere index, and every run produces the same permutation.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "mbs_grid.h"

namespace mbs {
namespace {

constexpr int kBoxParts = 256;  // workgroups of the bounding-box reduction (one per partial)
constexpr int kKeyBits = 3 * kGridAxisBits;

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }
inline unsigned nblk(int64_t len, int b) { return (unsigned)((len + b - 1) / b); }

// 10-bit coordinate -> bits 0, 3, 6, ... of a 30-bit word, and back
__device__ __forceinline__ uint32_t spread3(uint32_t v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000ffu;
  v = (v | (v << 8)) & 0x0300f00fu;
  v = (v | (v << 4)) & 0x030c30c3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}
__device__ __forceinline__ uint32_t compact3(uint32_t v) {
  v &= 0x09249249u;
  v = (v | (v >> 2)) & 0x030c30c3u;
  v = (v | (v >> 4)) & 0x0300f00fu;
  v = (v | (v >> 8)) & 0x030000ffu;
  v = (v | (v >> 16)) & 0x3ffu;
  return v;
}

// per-workgroup min and max of the centres -> part[b][6]
__global__ void __launch_bounds__(256) k_box_part(const double* __restrict__ R, int n, double* __restrict__ part) {
  __shared__ double red[6][256];
  double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double x = R[3 * (int64_t)i + d];
      v[d] = fmin(v[d], x);
      v[3 + d] = fmax(v[3 + d], x);
    }
  }
  const int t = threadIdx.x;
#pragma unroll
  for (int d = 0; d < 6; ++d) red[d][t] = v[d];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        red[d][t] = fmin(red[d][t], red[d][t + w]);
        red[3 + d][t] = fmax(red[3 + d][t], red[3 + d][t + w]);
      }
    }
    __syncthreads();
  }
  if (t < 6) part[6 * blockIdx.x + t] = red[t][0];
}

// bounding box -> cell edge and counts: edge >= h_min, at most max_cells cells, at most 1024 per axis
__global__ void __launch_bounds__(256) k_grid_params(const double* __restrict__ part, int n, double h_min,
                                                     int64_t max_cells, GridHdr* __restrict__ hdr) {
  __shared__ double red[6][kBoxParts];
  const int t = threadIdx.x;
#pragma unroll
  for (int d = 0; d < 6; ++d) red[d][t] = part[6 * t + d];
  __syncthreads();
  for (int w = kBoxParts / 2; w > 0; w >>= 1) {
    if (t < w) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        red[d][t] = fmin(red[d][t], red[d][t + w]);
        red[3 + d][t] = fmax(red[3 + d][t], red[3 + d][t + w]);
      }
    }
    __syncthreads();
  }
  if (t != 0) return;
  double lo[3], ext[3];
  bool ok = true;
  for (int d = 0; d < 3; ++d) {
    lo[d] = red[d][0];
    ext[d] = red[3 + d][0] - red[d][0];
    ok = ok && isfinite(lo[d]) && isfinite(ext[d]);
  }
  GridHdr H;
  int g[3] = {1, 1, 1};
  double h = 1.0;
  if (ok) {
    const double emax = fmax(ext[0], fmax(ext[1], ext[2]));
    // a relative margin keeps pairs closer than h_min within one cell of each other after rounding
    h = fmax(h_min, emax / (double)((1 << kGridAxisBits) - 1)) * (1.0 + 1e-9);
    h = fmax(h, cbrt(fmax(ext[0], h) * fmax(ext[1], h) * fmax(ext[2], h) / (double)max_cells));
    for (int it = 0; it < 512; ++it) {
      for (int d = 0; d < 3; ++d) g[d] = (int)(ext[d] / h) + 1;
      if ((int64_t)g[0] * g[1] * g[2] <= max_cells) break;
      h *= 1.0905077326652577;  // 2^(1/8)
    }
    if ((int64_t)g[0] * g[1] * g[2] > max_cells) g[0] = g[1] = g[2] = 1;
  } else {
    lo[0] = lo[1] = lo[2] = 0.0;
  }
  for (int d = 0; d < 3; ++d) {
    H.lo[d] = lo[d];
    H.g[d] = g[d];
  }
  H.h = h;
  H.inv_h = 1.0 / h;
  H.maxocc = 0;  // raised by the range kernel
  H.n = n;
  H.pad = 0;
  *hdr = H;
}

// a periodic box of side L > 0: the centre wrapped into [0, L); L = 0: unchanged
__device__ __forceinline__ double box_wrap(double x, double L) {
  if (!(L > 0.0)) return x;
  double w = x - L * floor(x / L);
  if (w >= L) w -= L;
  if (w < 0.0) w += L;
  return w;
}

// a periodic box: nc cells of edge L / nc along each axis, from the origin
__global__ void k_grid_params_box(int n, double L, int nc, GridHdr* __restrict__ hdr) {
  if (threadIdx.x != 0) return;
  GridHdr H;
  for (int d = 0; d < 3; ++d) {
    H.lo[d] = 0.0;
    H.g[d] = nc;
  }
  H.h = L / nc;
  H.inv_h = nc / L;
  H.maxocc = 0;
  H.n = n;
  H.pad = 0;
  *hdr = H;
}

__global__ void k_cell_keys(const double* __restrict__ R, int n, double L, const GridHdr* __restrict__ hdr,
                            uint32_t* __restrict__ key, int32_t* __restrict__ idx) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const GridHdr H = *hdr;
  const int cx = grid_cell1(box_wrap(R[3 * (int64_t)i], L), H.lo[0], H.inv_h, H.g[0]);
  const int cy = grid_cell1(box_wrap(R[3 * (int64_t)i + 1], L), H.lo[1], H.inv_h, H.g[1]);
  const int cz = grid_cell1(box_wrap(R[3 * (int64_t)i + 2], L), H.lo[2], H.inv_h, H.g[2]);
  key[i] = spread3(cx) | (spread3(cy) << 1) | (spread3(cz) << 2);
  idx[i] = i;
}

__global__ void k_clear_cells(int32_t* __restrict__ start, int32_t* __restrict__ end, int64_t cells) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cells) return;
  start[c] = 0;
  end[c] = 0;
}

__global__ void k_cell_ranges(const uint32_t* __restrict__ key, const int32_t* __restrict__ perm,
                              const double* __restrict__ R, int n, double L, GridHdr* __restrict__ hdr,
                              int32_t* __restrict__ start, int32_t* __restrict__ end, double* __restrict__ Rs) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const GridHdr H = *hdr;
  const uint32_t kk = key[k];
  const int64_t i = perm[k];
  Rs[4 * (int64_t)k] = box_wrap(R[3 * i], L);
  Rs[4 * (int64_t)k + 1] = box_wrap(R[3 * i + 1], L);
  Rs[4 * (int64_t)k + 2] = box_wrap(R[3 * i + 2], L);
  Rs[4 * (int64_t)k + 3] = 0.0;
  const int c = grid_linear(H, (int)compact3(kk), (int)compact3(kk >> 1), (int)compact3(kk >> 2));
  if (k == 0 || key[k - 1] != kk) start[c] = k;
  if (k == n - 1 || key[k + 1] != kk) {
    end[c] = k + 1;
    int lo = 0, hi = k;  // first position of this key (binary search in the sorted keys)
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (key[mid] < kk)
        lo = mid + 1;
      else
        hi = mid;
    }
    atomicMax(&hdr->maxocc, k + 1 - lo);
  }
}

// ---------------------------------------------------------------- radix sort of the cell keys
constexpr int kSortBits = 10;
constexpr int kSortDigits = 1 << kSortBits;
constexpr int kSortPasses = (kKeyBits + kSortBits - 1) / kSortBits;  // 3
constexpr int kSortThreads = 256;                                      // 4 wavefronts
constexpr int kSortRounds = 4;
constexpr int kSortTile = kSortThreads * kSortRounds;                  // keys per tile
static_assert(kSortPasses % 2 == 1, "an odd number of passes leaves the result in the output buffers");

inline int sort_tiles(int n) { return (n + kSortTile - 1) / kSortTile; }

// digit counts of one tile -> hist[digit * ntiles + tile]
__global__ void __launch_bounds__(kSortThreads) k_sort_hist(const uint32_t* __restrict__ key, int n, int shift,
                                                            int ntiles, int32_t* __restrict__ hist) {
  __shared__ int32_t h[kSortDigits];
  for (int d = threadIdx.x; d < kSortDigits; d += kSortThreads) h[d] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t k = base + r * kSortThreads + threadIdx.x;
    if (k < n) atomicAdd(&h[(key[k] >> shift) & (kSortDigits - 1)], 1);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < kSortDigits; d += kSortThreads) hist[(int64_t)d * ntiles + blockIdx.x] = h[d];
}

__device__ __forceinline__ int wave_incl_scan(int v, int lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int u = __shfl_up(v, off, 64);
    if (lane >= off) v += u;
  }
  return v;
}

// for every digit (one wavefront each): exclusive scan of its tile counts in place; total -> tot[d]
__global__ void __launch_bounds__(kSortThreads) k_sort_scan_tiles(int32_t* __restrict__ hist, int ntiles,
                                                                  int32_t* __restrict__ tot) {
  const int lane = threadIdx.x & 63;
  const int d = blockIdx.x * (kSortThreads / 64) + (threadIdx.x >> 6);
  int32_t* row = hist + (int64_t)d * ntiles;
  int carry = 0;
  for (int t0 = 0; t0 < ntiles; t0 += 64) {
    const int t = t0 + lane;
    const int v = t < ntiles ? row[t] : 0;
    const int s = wave_incl_scan(v, lane);
    if (t < ntiles) row[t] = carry + s - v;
    carry += __shfl(s, 63, 64);
  }
  if (lane == 0) tot[d] = carry;
}

// exclusive scan of the digit totals -> first output position of each digit (one workgroup)
__global__ void __launch_bounds__(kSortDigits) k_sort_scan_digits(const int32_t* __restrict__ tot,
                                                                  int32_t* __restrict__ dbase) {
  __shared__ int32_t wsum[kSortDigits / 64];
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const int v = tot[t];
  const int s = wave_incl_scan(v, lane);
  if (lane == 63) wsum[wid] = s;
  __syncthreads();
  int x = 0, xs = 0;
  if (wid == 0) {
    x = lane < kSortDigits / 64 ? wsum[lane] : 0;
    xs = wave_incl_scan(x, lane);
  }
  __syncthreads();
  if (wid == 0 && lane < kSortDigits / 64) wsum[lane] = xs - x;
  __syncthreads();
  dbase[t] = wsum[wid] + s - v;
}

// stable scatter of one tile by digit
__global__ void __launch_bounds__(kSortThreads) k_sort_scatter(const uint32_t* __restrict__ kin,
                                                               const int32_t* __restrict__ vin, int n, int shift,
                                                               int ntiles, const int32_t* __restrict__ hist,
                                                               const int32_t* __restrict__ dbase,
                                                               uint32_t* __restrict__ kout, int32_t* __restrict__ vout) {
  __shared__ int32_t base[kSortDigits];
  __shared__ int32_t wcnt[kSortThreads / 64][kSortDigits];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  for (int d = tid; d < kSortDigits; d += kSortThreads) {
    base[d] = dbase[d] + hist[(int64_t)d * ntiles + blockIdx.x];
#pragma unroll
    for (int w = 0; w < kSortThreads / 64; ++w) wcnt[w][d] = 0;
  }
  __syncthreads();
  const uint64_t below = (1ull << lane) - 1ull;  // lanes before this one
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t k = (int64_t)blockIdx.x * kSortTile + r * kSortThreads + tid;
    const bool valid = k < n;
    const uint32_t key = valid ? kin[k] : 0u;
    const int d = (int)((key >> shift) & (kSortDigits - 1));
    uint64_t peers = __ballot(valid);  // valid lanes of this wavefront holding the same digit
#pragma unroll
    for (int b = 0; b < kSortBits; ++b) {
      const int bit = (d >> b) & 1;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const int rank = __popcll(peers & below);
    if (valid && rank == 0) wcnt[wid][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int pos = base[d] + rank;
      for (int w = 0; w < wid; ++w) pos += wcnt[w][d];
      kout[pos] = key;
      vout[pos] = vin[k];
    }
    __syncthreads();
    for (int dd = tid; dd < kSortDigits; dd += kSortThreads) {
      int add = 0;
#pragma unroll
      for (int w = 0; w < kSortThreads / 64; ++w) {
        add += wcnt[w][dd];
        wcnt[w][dd] = 0;
      }
      base[dd] += add;
    }
    __syncthreads();
  }
}

struct Layout {
  size_t hdr, part, key_in, key, idx_in, perm, Rs, start, end, hist, tot, dbase, total;
};

Layout layout(int n, int64_t max_cells) {
  Layout L{};
  size_t o = 0;
  L.hdr = o;
  o += align256(sizeof(GridHdr));
  L.part = o;
  o += align256(sizeof(double) * 6 * kBoxParts);
  L.key_in = o;
  o += align256(sizeof(uint32_t) * n);
  L.key = o;
  o += align256(sizeof(uint32_t) * n);
  L.idx_in = o;
  o += align256(sizeof(int32_t) * n);
  L.perm = o;
  o += align256(sizeof(int32_t) * n);
  L.Rs = o;
  o += align256(sizeof(double) * 4 * n);
  L.start = o;
  o += align256(sizeof(int32_t) * max_cells);
  L.end = o;
  o += align256(sizeof(int32_t) * max_cells);
  L.hist = o;
  o += align256(sizeof(int32_t) * (size_t)kSortDigits * sort_tiles(n));
  L.tot = o;
  o += align256(sizeof(int32_t) * kSortDigits);
  L.dbase = o;
  o += align256(sizeof(int32_t) * kSortDigits);
  L.total = o;
  return L;
}

}  // namespace

size_t grid_ws_bytes(int n, int64_t max_cells) { return layout(n, max_cells).total; }

namespace {

// the sort, the cell ranges and the sorted centres, once the header is in place (box > 0: a
// periodic box of that side, centres wrapped into it)
hipError_t grid_finish(const double* R, int n, double box, int64_t max_cells, void* ws, GridView* view,
                       hipStream_t s);

}  // namespace

hipError_t grid_build_box(const double* R, int n, double L, int nc, void* ws, size_t ws_bytes, GridView* view,
                          hipStream_t s) {
  if (n < 1 || nc < 1 || nc > (1 << kGridAxisBits) || !(L > 0.0)) return hipErrorInvalidValue;
  const int64_t cells = (int64_t)nc * nc * nc;
  const Layout Ly = layout(n, cells);
  if (ws_bytes < Ly.total) return hipErrorInvalidValue;
  GridHdr* hdr = (GridHdr*)((char*)ws + Ly.hdr);
  hipLaunchKernelGGL(k_grid_params_box, dim3(1), dim3(64), 0, s, n, L, nc, hdr);
  return grid_finish(R, n, L, cells, ws, view, s);
}

hipError_t grid_build(const double* R, int n, double h_min, int64_t max_cells, void* ws, size_t ws_bytes,
                      GridView* view, hipStream_t s) {
  if (n < 1 || max_cells < 1 || !(h_min > 0.0)) return hipErrorInvalidValue;
  const Layout Ly = layout(n, max_cells);
  if (ws_bytes < Ly.total) return hipErrorInvalidValue;
  char* b = (char*)ws;
  GridHdr* hdr = (GridHdr*)(b + Ly.hdr);
  double* part = (double*)(b + Ly.part);
  hipLaunchKernelGGL(k_box_part, dim3(kBoxParts), dim3(256), 0, s, R, n, part);
  hipLaunchKernelGGL(k_grid_params, dim3(1), dim3(kBoxParts), 0, s, part, n, h_min, max_cells, hdr);
  return grid_finish(R, n, 0.0, max_cells, ws, view, s);
}

namespace {

hipError_t grid_finish(const double* R, int n, double box, int64_t max_cells, void* ws, GridView* view,
                       hipStream_t s) {
  const Layout L = layout(n, max_cells);
  char* b = (char*)ws;
  GridHdr* hdr = (GridHdr*)(b + L.hdr);
  uint32_t* key_in = (uint32_t*)(b + L.key_in);
  uint32_t* key = (uint32_t*)(b + L.key);
  int32_t* idx_in = (int32_t*)(b + L.idx_in);
  int32_t* perm = (int32_t*)(b + L.perm);
  double* Rs = (double*)(b + L.Rs);
  int32_t* start = (int32_t*)(b + L.start);
  int32_t* end = (int32_t*)(b + L.end);
  hipLaunchKernelGGL(k_cell_keys, dim3(nblk(n, 256)), dim3(256), 0, s, R, n, box, hdr, key_in, idx_in);
  {  // stable radix sort (key_in, idx_in) -> (key, perm), ping-ponging through both pairs of buffers
    int32_t* hist = (int32_t*)(b + L.hist);
    int32_t* tot = (int32_t*)(b + L.tot);
    int32_t* dbase = (int32_t*)(b + L.dbase);
    const int ntiles = sort_tiles(n);
    uint32_t* kbuf[2] = {key_in, key};
    int32_t* vbuf[2] = {idx_in, perm};
    for (int p = 0; p < kSortPasses; ++p) {
      const int shift = p * kSortBits;
      const uint32_t* ki = kbuf[p & 1];
      const int32_t* vi = vbuf[p & 1];
      hipLaunchKernelGGL(k_sort_hist, dim3(ntiles), dim3(kSortThreads), 0, s, ki, n, shift, ntiles, hist);
      hipLaunchKernelGGL(k_sort_scan_tiles, dim3(kSortDigits / (kSortThreads / 64)), dim3(kSortThreads), 0, s,
                         hist, ntiles, tot);
      hipLaunchKernelGGL(k_sort_scan_digits, dim3(1), dim3(kSortDigits), 0, s, tot, dbase);
      hipLaunchKernelGGL(k_sort_scatter, dim3(ntiles), dim3(kSortThreads), 0, s, ki, vi, n, shift, ntiles, hist,
                         dbase, kbuf[(p + 1) & 1], vbuf[(p + 1) & 1]);
    }
  }
  hipLaunchKernelGGL(k_clear_cells, dim3(nblk(max_cells, 256)), dim3(256), 0, s, start, end, max_cells);
  hipLaunchKernelGGL(k_cell_ranges, dim3(nblk(n, 256)), dim3(256), 0, s, key, perm, R, n, box, hdr, start, end,
                     Rs);
  view->hdr = hdr;
  view->Rs = Rs;
  view->perm = perm;
  view->start = start;
  view->end = end;
  view->n = n;
  return hipGetLastError();
}

}  // namespace

}  // namespace mbs
