// Internal declarations of the learned pre-screen (k_mlp.hip, tto_api.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace tto {

constexpr int kMlpRowBits = 64;      // bits read per row (TTO_MLP_MAX_ROW_BITS)
constexpr int kMlpMaxTrain = 4096;   // largest training batch (TTO_MLP_MAX_TRAIN)

// Parameters: FP32 master copy (flat: W1b, W1d, b1, W2, b2, W3, b3, W4, b4),
// Adam moments, BF16 copies of the matrices used as MFMA / gather operands.
struct MlpDev {
  int d_bits, d_dense, H;
  size_t n_params;
  float* master;
  float* m;
  float* v;
  float* grad;
  // BF16 copies: W1b, W2 and W3 as stored, and W1d, W2, W3 transposed ([out][in],
  // the forward GEMMs' operand with k contiguous)
  unsigned short* W1b_h;
  unsigned short* W2_h;
  unsigned short* W3_h;
  unsigned short* W1dt_h;
  unsigned short* W2t_h;
  unsigned short* W3t_h;
  // FP32 views into master used directly by kernels
  const float* b1;
  const float* b2;
  const float* b3;
  const float* W4;
  const float* b4;
};

// Views of one flat parameter-shaped FP32 array (master weights or gradients).
struct MlpGrad {
  float *W1b, *W1d, *b1, *W2, *b2, *W3, *b3, *W4, *b4;
};

inline MlpGrad mlp_grad_view(const MlpDev& p, float* base) {
  MlpGrad g;
  const size_t H = p.H;
  g.W1b = base;
  g.W1d = g.W1b + (size_t)p.d_bits * H;
  g.b1 = g.W1d + (size_t)p.d_dense * H;
  g.W2 = g.b1 + H;
  g.b2 = g.W2 + H * H;
  g.W3 = g.b2 + H;
  g.b3 = g.W3 + H * H;
  g.W4 = g.b3 + H;
  g.b4 = g.W4 + 2 * H;
  return g;
}

inline size_t mlp_param_count(int d_bits, int d_dense, int H) {
  const size_t h = H;
  return (size_t)d_bits * h + (size_t)d_dense * h + h + h * h + h + h * h + h + 2 * h + 2;
}

// Per-batch activations and backward buffers.
struct MlpBatch {
  unsigned short *h1, *h2, *h3;      // [B][H] BF16 activations
  unsigned short *dz1, *dz2, *dz3;   // [B][H] BF16 back-propagated pre-activation grads
  int* cnt;                          // [d_bits] bucket sizes of the first-layer gradient
  int* start;                        // [d_bits + 1] bucket offsets
  int* cursor;                       // [d_bits] fill cursors
  int* list;                         // [B * kMlpRowBits] samples per bit
  unsigned short* Xd;                // [B][d_dense] BF16 dense inputs
  float* zd;                         // [B][H] dense inputs times W1d (FP32)
  float* y;                          // [B][2]
  float* dy;                         // [B][2]
  float* lterm;                      // [B]
  float* part;                       // [ceil(B / 64)][2 H] chunk partial sums
  float* gpart;                      // split-K partials of the weight-gradient GEMMs
};

// Floats of MlpBatch::gpart: the most any split weight-gradient GEMM needs for
// width H, dense width dd and training batch Bt.
size_t mlp_split_floats(int H, int dd, int Bt);

void mlp_forward(const MlpDev& p, const MlpBatch& wb, const int* off, const int* idx,
                 const float* dense, int B, float* y, hipStream_t s);
void mlp_gradients(const MlpDev& p, const MlpBatch& wb, const int* off, const int* idx,
                   const float* dense, const float* target, int B, float* grad, float* loss,
                   hipStream_t s);
void mlp_adam(const MlpDev& p, const float* grad, float lr, int step, hipStream_t s);
void mlp_refresh_bf16(const MlpDev& p, hipStream_t s);
void topk_smallest(const float* score, int n, int stride, int k, int* out, hipStream_t s);
void batch_gather(const int* open, const int* sbus, const int* moff, const int* mbr,
                  const double* mp, int n_src, int no, int ns, int T, const int* idx, int k,
                  int* d_open, int* d_sbus, int* d_moff, int* d_mbr, int cap, double* d_mp,
                  hipStream_t s);

}  // namespace tto
