// Warm-start network on the matrix cores (gfx950): an in -> 128 -> 128 -> 5 perceptron with ReLU (in = 80
// or 160 inputs),
// bfloat16 operands and float32 accumulation through v_mfma_f32_16x16x16_bf16, plus the
// kernels of its training step (mean-squared-error gradient, ReLU masks, bias gradients, Adam).
//
// Matrices are row-major. Every GEMM is C[M x N] = A[M x K] B[K x N] with M, N, K multiples of 16,
// in 64 x 64 tiles of C per workgroup (see k_gemm_bf16). MFMA operand layout (wave64):
// lane l holds A[l % 16][4(l/16) .. 4(l/16)+3], B[4(l/16) .. 4(l/16)+3][l % 16] and returns
// C[4(l/16) .. 4(l/16)+3][l % 16]. Long K (weight gradients, K = batch) is split over grid.z into
// partial tiles that a second kernel adds in a fixed order, so every result is reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <math.h>
#include <stdint.h>

#include "mbs_mlp.h"

namespace mbs {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// float32 -> bfloat16, round to nearest, ties to even (finite inputs).
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Tiled GEMM: one workgroup of 256 threads (4 wavefronts) owns a 64 x 64 tile of C; each wavefront
// a 32 x 32 quarter (2 x 2 MFMA tiles). K is walked in panels of 32: the A panel [64 x 32] and the
// B panel [32 x 64] are loaded with one 16-byte global load per thread each (8 consecutive bf16
// along whichever index is contiguous in memory) and stored in LDS as As[m][k] and Bs[n][k], so
// that every MFMA operand (4 consecutive k of one row or column) is one 8-byte LDS read. Rows and
// columns past M or N and k past the panel's end read as zero; M, N and K are multiples of 16.
constexpr int kGT = 64, kGK = 32, kGPad = 8;  // tile edge, K panel, LDS row padding (bank spread)

__global__ void __launch_bounds__(256)
    k_gemm_bf16(const uint16_t* __restrict__ A, int lda, int transA, const uint16_t* __restrict__ B,
                int ldb, int transB, float* __restrict__ C, int M, int N, int K, int kchunk) {
  __shared__ __align__(16) uint16_t As[kGT][kGK + kGPad];
  __shared__ __align__(16) uint16_t Bs[kGT][kGK + kGPad];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * kGT, n0 = blockIdx.x * kGT;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;  // this wavefront's quarter
  const int r = lane & 15, kb = 4 * (lane >> 4);
  const int kbeg = blockIdx.z * kchunk;
  const int kend = min(K, kbeg + kchunk);
  floatx4 acc[2][2] = {};
  // this thread's 16-byte chunk of each panel: 256 chunks of 8 elements
  // contiguous along k (A row-major, B transposed): row = tid / 4, k offset = 8 (tid % 4)
  // contiguous along m or n (A transposed, B row-major): k row = tid / 8, m/n offset = 8 (tid % 8)
  for (int k0 = kbeg; k0 < kend; k0 += kGK) {
    {  // A panel -> As[m][k]
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (!transA) {
        const int mm = tid >> 2, kk = 8 * (tid & 3);
        if (m0 + mm < M && k0 + kk < kend) v = *(const uint4*)(A + (int64_t)(m0 + mm) * lda + k0 + kk);
        *(uint4*)&As[mm][kk] = v;
      } else {
        const int kk = tid >> 3, mm = 8 * (tid & 7);
        if (m0 + mm < M && k0 + kk < kend) v = *(const uint4*)(A + (int64_t)(k0 + kk) * lda + m0 + mm);
        const uint16_t* e = (const uint16_t*)&v;
#pragma unroll
        for (int q = 0; q < 8; ++q) As[mm + q][kk] = e[q];
      }
    }
    {  // B panel -> Bs[n][k]
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (transB) {
        const int nn = tid >> 2, kk = 8 * (tid & 3);
        if (n0 + nn < N && k0 + kk < kend) v = *(const uint4*)(B + (int64_t)(n0 + nn) * ldb + k0 + kk);
        *(uint4*)&Bs[nn][kk] = v;
      } else {
        const int kk = tid >> 3, nn = 8 * (tid & 7);
        if (n0 + nn < N && k0 + kk < kend) v = *(const uint4*)(B + (int64_t)(k0 + kk) * ldb + n0 + nn);
        const uint16_t* e = (const uint16_t*)&v;
#pragma unroll
        for (int q = 0; q < 8; ++q) Bs[nn + q][kk] = e[q];
      }
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < kGK; ks += 16) {
      bf16x4 a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[t] = *(const bf16x4*)&As[wm + 16 * t + r][ks + kb];
        b[t] = *(const bf16x4*)&Bs[wn + 16 * t + r][ks + kb];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  float* Cz = C + (int64_t)blockIdx.z * M * N;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wn + 16 * j + r;
      if (col >= N) continue;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int row = m0 + wm + 16 * i + kb + t;
        if (row < M) Cz[(int64_t)row * N + col] = acc[i][j][t];
      }
    }
}

__global__ void k_sum_partials(const float* __restrict__ P, int parts, int64_t len,
                               float* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= len) return;
  float s = 0.f;
  for (int p = 0; p < parts; ++p) s += P[p * len + k];
  out[k] = s;
}

// X[r, c] = bf16(feat[idx[r], c]) for r < rows (idx NULL: identity), zero for padded rows.
__global__ void k_gather_bf16(const float* __restrict__ feat, const int32_t* __restrict__ idx, int rows,
                              int rows_pad, int cols, uint16_t* __restrict__ X) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (int64_t)rows_pad * cols) return;
  const int r = (int)(k / cols), c = (int)(k % cols);
  float v = 0.f;
  if (r < rows) v = feat[(int64_t)(idx ? idx[r] : r) * cols + c];
  X[k] = f2bf(v);
}

// H = bf16(max(C + b, 0))
__global__ void k_bias_relu(const float* __restrict__ C, const float* __restrict__ b, int64_t len, int N,
                            uint16_t* __restrict__ H) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= len) return;
  H[k] = f2bf(fmaxf(C[k] + b[k % N], 0.f));
}

// out[r, 0:5] = C[r, 0:5] + b3
__global__ void k_out_bias(const float* __restrict__ C, const float* __restrict__ b3, int rows,
                           float* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (int64_t)rows * kMlpOut) return;
  const int r = (int)(k / kMlpOut), c = (int)(k % kMlpOut);
  out[k] = C[(int64_t)r * 16 + c] + b3[c];
}

// dOut = 2 (out - T) / (count * 5) into bf16 [rows_pad x 16] (zero padding) and float32 [rows x 5];
// loss_part[block] = sum of squared errors of the block.
__global__ void __launch_bounds__(256)
    k_mse_grad(const float* __restrict__ C, const float* __restrict__ b3, const float* __restrict__ T,
               const int32_t* __restrict__ idx, int rows, int rows_pad, double scale,
               uint16_t* __restrict__ dOut, float* __restrict__ dOut32, double* __restrict__ loss_part) {
  __shared__ double red[256];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double sq = 0.0;
  if (k < (int64_t)rows_pad * 16) {
    const int r = (int)(k >> 4), c = (int)(k & 15);
    float g = 0.f;
    if (r < rows && c < kMlpOut) {
      const float o = C[k] + b3[c];
      const float t = T[(int64_t)(idx ? idx[r] : r) * kMlpOut + c];
      const float d = o - t;
      sq = (double)d * (double)d;
      g = (float)(2.0 * scale) * d;
      dOut32[(int64_t)r * kMlpOut + c] = g;
    }
    dOut[k] = f2bf(g);
  }
  red[threadIdx.x] = sq;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

// D = bf16(H > 0 ? G : 0), G32 = the float32 masked value (for the bias gradient)
__global__ void k_relu_mask(const float* __restrict__ G, const uint16_t* __restrict__ H, int64_t len,
                            uint16_t* __restrict__ D, float* __restrict__ G32) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= len) return;
  const float g = (H[k] & 0x7FFFu) != 0 && !(H[k] & 0x8000u) ? G[k] : 0.f;
  D[k] = f2bf(g);
  G32[k] = g;
}

// out[c] = sum_r M[r, c] (fixed order; one thread per column)
// column sums of M [rows x cols], stage 1: workgroup (column block, row chunk) -> partial[chunk][col]
__global__ void __launch_bounds__(256) k_colsum_part(const float* __restrict__ M, int rows, int cols,
                                                     int chunk, float* __restrict__ partial) {
  __shared__ float red[4][64];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + tx;
  const int r0 = blockIdx.y * chunk, r1 = min(rows, r0 + chunk);
  float s = 0.f;
  if (c < cols)
    for (int r = r0 + ty; r < r1; r += 4) s += M[(int64_t)r * cols + c];
  red[ty][tx] = s;
  __syncthreads();
  if (ty == 0 && c < cols) partial[(int64_t)blockIdx.y * cols + c] = ((red[0][tx] + red[1][tx]) + red[2][tx]) + red[3][tx];
}

// copy the [rows x ldsrc] float tile's first cols columns into dst [rows x cols]
__global__ void k_copy_cols(const float* __restrict__ src, int ldsrc, int rows, int cols,
                            float* __restrict__ dst) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (int64_t)rows * cols) return;
  const int r = (int)(k / cols), c = (int)(k % cols);
  dst[k] = src[(int64_t)r * ldsrc + c];
}

// Adam (Kingma & Ba) on the float32 master parameters, then refresh of the bf16 weight copies.
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const float gk = g[k];
  const float mk = b1 * m[k] + (1.f - b1) * gk;
  const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  w[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

// bf16 copies: W1 [in x 128], W2 [128x128], W3 [128x16] (columns 5..15 zero)
__global__ void k_weights_bf16(const float* __restrict__ w, MlpLayout L, uint16_t* __restrict__ W1,
                               uint16_t* __restrict__ W2, uint16_t* __restrict__ W3) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < L.in * kMlpHid) W1[k] = f2bf(w[L.offW1 + k]);
  if (k < kMlpHid * kMlpHid) W2[k] = f2bf(w[L.offW2 + k]);
  if (k < kMlpHid * 16) {
    const int r = k >> 4, c = k & 15;
    W3[k] = c < kMlpOut ? f2bf(w[L.offW3 + r * kMlpOut + c]) : (uint16_t)0;
  }
}

inline unsigned nblk(int64_t len, int b) { return (unsigned)((len + b - 1) / b); }

}  // namespace

void mlp_gemm(const uint16_t* A, int lda, bool tA, const uint16_t* B, int ldb, bool tB, float* C,
              float* partial, int M, int N, int K, int ksplit, hipStream_t s) {
  // K chunks of whole panels; every chunk but the last is a multiple of the panel depth
  const int kchunk = ((K + ksplit - 1) / ksplit + kGK - 1) / kGK * kGK;
  const int parts = (K + kchunk - 1) / kchunk;
  float* out = parts > 1 ? partial : C;
  hipLaunchKernelGGL(k_gemm_bf16, dim3((N + kGT - 1) / kGT, (M + kGT - 1) / kGT, parts), dim3(256), 0, s, A, lda,
                     (int)tA, B, ldb, (int)tB, out, M, N, K, kchunk);
  if (parts > 1)
    hipLaunchKernelGGL(k_sum_partials, dim3(nblk((int64_t)M * N, 256)), dim3(256), 0, s, partial,
                       parts, (int64_t)M * N, C);
}

void mlp_gather_bf16(const float* feat, const int32_t* idx, int rows, int rows_pad, int cols,
                     uint16_t* X, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_bf16, dim3(nblk((int64_t)rows_pad * cols, 256)), dim3(256), 0, s, feat,
                     idx, rows, rows_pad, cols, X);
}

void mlp_bias_relu(const float* C, const float* b, int rows_pad, int N, uint16_t* H, hipStream_t s) {
  const int64_t len = (int64_t)rows_pad * N;
  hipLaunchKernelGGL(k_bias_relu, dim3(nblk(len, 256)), dim3(256), 0, s, C, b, len, N, H);
}

void mlp_out_bias(const float* C, const float* b3, int rows, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_out_bias, dim3(nblk((int64_t)rows * kMlpOut, 256)), dim3(256), 0, s, C, b3,
                     rows, out);
}

int mlp_mse_blocks(int rows_pad) { return (int)nblk((int64_t)rows_pad * 16, 256); }

void mlp_mse_grad(const float* C, const float* b3, const float* T, const int32_t* idx, int rows,
                  int rows_pad, double scale, uint16_t* dOut, float* dOut32, double* loss_part,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_mse_grad, dim3(mlp_mse_blocks(rows_pad)), dim3(256), 0, s, C, b3, T, idx, rows,
                     rows_pad, scale, dOut, dOut32, loss_part);
}

void mlp_relu_mask(const float* G, const uint16_t* H, int64_t len, uint16_t* D, float* G32,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_relu_mask, dim3(nblk(len, 256)), dim3(256), 0, s, G, H, len, D, G32);
}

void mlp_colsum(const float* M, int rows, int cols, float* out, float* partial, hipStream_t s) {
  const int parts = std::max(1, std::min(256, (rows + 127) / 128));
  const int chunk = (rows + parts - 1) / parts;
  hipLaunchKernelGGL(k_colsum_part, dim3(nblk(cols, 64), parts), dim3(256), 0, s, M, rows, cols, chunk,
                     partial);
  hipLaunchKernelGGL(k_sum_partials, dim3(nblk(cols, 256)), dim3(256), 0, s, partial, parts, (int64_t)cols,
                     out);
}

void mlp_copy_cols(const float* src, int ldsrc, int rows, int cols, float* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_cols, dim3(nblk((int64_t)rows * cols, 256)), dim3(256), 0, s, src, ldsrc,
                     rows, cols, dst);
}

void mlp_adam(float* w, const float* g, float* m, float* v, int n, float lr, float b1, float b2,
              float eps, int step, hipStream_t s) {
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(nblk(n, 256)), dim3(256), 0, s, w, g, m, v, n, lr, b1, b2, eps, c1, c2);
}

void mlp_weights_bf16(const float* w, const MlpLayout& L, uint16_t* W1, uint16_t* W2, uint16_t* W3, hipStream_t s) {
  const int most = std::max(L.in * kMlpHid, kMlpHid * kMlpHid);
  hipLaunchKernelGGL(k_weights_bf16, dim3(nblk(most, 256)), dim3(256), 0, s, w, L, W1, W2, W3);
}

}  // namespace mbs
