// Warm-start network: sizes, parameter layout and kernel launchers (internal to libmbstokes).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mbs {

constexpr int kMlpIn = 80, kMlpHid = 128, kMlpOut = 5, kNeigh = 16;
// flat float32 parameter vector: W1 [80x128], b1 [128], W2 [128x128], b2 [128], W3 [128x5], b3 [5]
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpIn * kMlpHid;
constexpr int kOffW2 = kOffB1 + kMlpHid;
constexpr int kOffB2 = kOffW2 + kMlpHid * kMlpHid;
constexpr int kOffW3 = kOffB2 + kMlpHid;
constexpr int kOffB3 = kOffW3 + kMlpHid * kMlpOut;
constexpr int kMlpParams = kOffB3 + kMlpOut;  // 27525

// C[M x N] = A B (bfloat16 operands, float32 result); tA: A stored [K x M]; tB: B stored [N x K].
// partial: float32 scratch [ksplit x M x N] when K is split (ksplit > 1).
void mlp_gemm(const uint16_t* A, int lda, bool tA, const uint16_t* B, int ldb, bool tB, float* C,
              float* partial, int M, int N, int K, int ksplit, hipStream_t s);
void mlp_gather_bf16(const float* feat, const int32_t* idx, int rows, int rows_pad, int cols,
                     uint16_t* X, hipStream_t s);
void mlp_bias_relu(const float* C, const float* b, int rows_pad, int N, uint16_t* H, hipStream_t s);
void mlp_out_bias(const float* C, const float* b3, int rows, float* out, hipStream_t s);
int mlp_mse_blocks(int rows_pad);
void mlp_mse_grad(const float* C, const float* b3, const float* T, const int32_t* idx, int rows,
                  int rows_pad, double scale, uint16_t* dOut, float* dOut32, double* loss_part,
                  hipStream_t s);
void mlp_relu_mask(const float* G, const uint16_t* H, int64_t len, uint16_t* D, float* G32,
                   hipStream_t s);
// column sums of M [rows x cols] -> out [cols]; partial: scratch of min(256, ceil(rows/128)) x cols floats
void mlp_colsum(const float* M, int rows, int cols, float* out, float* partial, hipStream_t s);
void mlp_copy_cols(const float* src, int ldsrc, int rows, int cols, float* dst, hipStream_t s);
void mlp_adam(float* w, const float* g, float* m, float* v, int n, float lr, float b1, float b2,
              float eps, int step, hipStream_t s);
void mlp_weights_bf16(const float* w, uint16_t* W1, uint16_t* W2, uint16_t* W3, hipStream_t s);

// 16 nearest other centres of every sphere (ties by index), nearest first: nbr [n x 16], from a
// cell grid of the centres
struct GridView;
void launch_knn16(const GridView& g, int32_t* nbr, hipStream_t s);
// features [n x 80] float32 from the neighbour lists
void launch_features(const double* R, const double* p, const int32_t* nbr, int n, float* feat,
                     hipStream_t s);
// x[k] = gamma * b[k] + out[k] (binary64 guess from the network output)
void launch_guess_learned(const double* b, const float* out, double gamma, int64_t len, double* x,
                          hipStream_t s);

// target of the network from a converged flow stresslet: t = Sigma - gamma b (float32)
void launch_target(const double* Sig, const double* b, double gamma, int64_t len, float* t,
                   hipStream_t s);

}  // namespace mbs
