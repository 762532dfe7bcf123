// Warm-start network: sizes, parameter layout and kernel launchers (internal to libmbstokes).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mbs {

constexpr int kMlpHid = 128, kMlpOut = 5, kNeigh = 16;
// inputs: 16 neighbours x 5 geometric features (feature set 0), or x (5 geometric features + the
// neighbour's one-body stresslet gamma b_j, 5 values) (feature set 1)
constexpr int kMlpIn = 80, kMlpInRhs = 160, kMlpInMax = kMlpInRhs;
// flat float32 parameter vector: W1 [in x 128], b1 [128], W2 [128x128], b2 [128], W3 [128x5], b3 [5]
struct MlpLayout {
  int in, offW1, offB1, offW2, offB2, offW3, offB3, nparam;
};
constexpr MlpLayout mlp_layout(int in) {
  return MlpLayout{in,
                   0,
                   in * kMlpHid,
                   in * kMlpHid + kMlpHid,
                   in * kMlpHid + kMlpHid + kMlpHid * kMlpHid,
                   in * kMlpHid + 2 * kMlpHid + kMlpHid * kMlpHid,
                   in * kMlpHid + 2 * kMlpHid + kMlpHid * kMlpHid + kMlpHid * kMlpOut,
                   in * kMlpHid + 2 * kMlpHid + kMlpHid * kMlpHid + kMlpHid * kMlpOut + kMlpOut};
}
static_assert(mlp_layout(kMlpIn).nparam == 27525, "parameter count of the 80-input network");
static_assert(mlp_layout(kMlpInRhs).nparam == 37765, "parameter count of the 160-input network");
constexpr int kMlpParamsMax = mlp_layout(kMlpInMax).nparam;

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
void mlp_weights_bf16(const float* w, const MlpLayout& L, uint16_t* W1, uint16_t* W2, uint16_t* W3, hipStream_t s);

// 16 nearest other centres of every sphere (ties by index), nearest first: nbr [n x 16], from a
// cell grid of the centres
struct GridView;
void launch_knn16(const GridView& g, int32_t* nbr, hipStream_t s);
// features [n x 80] float32 from the neighbour lists; with b (binary64 [n x 5], the right-hand side)
// the 160-feature set [n x 160]: each neighbour's five geometric features followed by gamma b_j
void launch_features(const double* R, const double* p, const int32_t* nbr, int n, float* feat,
                     hipStream_t s, const double* b = nullptr, double gamma = 0.0);
// x[k] = gamma * b[k] + out[k] (binary64 guess from the network output)
void launch_guess_learned(const double* b, const float* out, double gamma, int64_t len, double* x,
                          hipStream_t s);

// target of the network from a converged flow stresslet: t = Sigma - gamma b (float32)
void launch_target(const double* Sig, const double* b, double gamma, int64_t len, float* t,
                   hipStream_t s);

}  // namespace mbs
