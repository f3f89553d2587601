// Learned pre-screen: a 4-layer perceptron over a candidate's action bitmask
// and an injection summary, predicting (maximum loading, log-overload).
// Forward and backward on the GPU: embedding-bag first layer, BF16 MFMA GEMMs
// with FP32 accumulation for the hidden layers (fused bias + ReLU, or ReLU
// mask in the backward pass), VALU output layer, Adam on FP32 master weights,
// and a deterministic single-workgroup radix top-k for the screen.
#include "tto_common.h"
#include "tto_mlp.h"

#include <limits.h>

#include <algorithm>

namespace tto {

typedef float v4f32m __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf16m __attribute__((ext_vector_type(8)));
typedef unsigned short v8u16m __attribute__((ext_vector_type(8)));

__device__ inline unsigned short bf16_rne(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ inline float bf16_to_f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

// ---------------------------------------------------------------------------
// One TILE x BK operand tile of a GEMM step (TILE = 64 or 128, BK = 32 or
// 64), held in registers between its global load and its LDS store
// (TILE BK / 2048 pieces of 16 bytes per thread), stored in LDS as T[r][k]
// (k contiguous, row stride BK + 8 halfwords so that every 8-element MFMA
// fragment is one aligned 16-byte read).  ROWK: the operand is stored [rows][ld] with k contiguous; otherwise
// [k][ld] with the rows contiguous (each piece is 8 rows at one k, written
// transposed).  k beyond kend and rows beyond `rows` read as zero.  `vec`:
// 16-byte global loads (the contiguous extent is a multiple of 8).
template <bool ROWK, int TILE, int BK>
struct GemmStage {
  static constexpr int HS = TILE * BK / 2048;   // pieces per thread
  static constexpr int RG = TILE / 8;           // 8-row groups (non-ROWK)
  static constexpr int KP = BK / 8;             // pieces per row (ROWK)
  v8u16m v[HS];
  __device__ __forceinline__ void load(const unsigned short* __restrict__ X, int rows, int ld,
                                       int kend, int r0, int k0, bool vec, int tid) {
#pragma unroll
    for (int h = 0; h < HS; ++h) {
      const int pc = tid + 256 * h;
      if constexpr (ROWK) {
        const int gr = r0 + pc / KP, gk = k0 + (pc % KP) * 8;
        if (vec && gr < rows && gk + 8 <= kend) {
          v[h] = *(const v8u16m*)(X + (size_t)gr * ld + gk);
        } else {
#pragma unroll
          for (int u = 0; u < 8; ++u)
            v[h][u] = (gr < rows && gk + u < kend) ? X[(size_t)gr * ld + gk + u] : (unsigned short)0;
        }
      } else {
        const int gk = k0 + pc / RG, gr = r0 + (pc % RG) * 8;
        if (vec && gk < kend && gr + 8 <= rows) {
          v[h] = *(const v8u16m*)(X + (size_t)gk * ld + gr);
        } else {
#pragma unroll
          for (int u = 0; u < 8; ++u)
            v[h][u] = (gk < kend && gr + u < rows) ? X[(size_t)gk * ld + gr + u] : (unsigned short)0;
        }
      }
    }
  }
  __device__ __forceinline__ void store(unsigned short (*T)[BK + 8], int tid) const {
#pragma unroll
    for (int h = 0; h < HS; ++h) {
      const int pc = tid + 256 * h;
      if constexpr (ROWK) {
        *(v8u16m*)&T[pc / KP][(pc % KP) * 8] = v[h];
      } else {
        const int kr = pc / RG, rc = (pc % RG) * 8;
#pragma unroll
        for (int u = 0; u < 8; ++u) T[rc + u][kr] = v[h][u];
      }
    }
  }
};

// C[M x N] = op(A) op(B), BF16 operands, FP32 accumulation on
// v_mfma_f32_16x16x32_bf16.  A_COL: A stored [K][M] (else [M][K]); B_COL: B
// stored [N][K] (else [K][N]).  Workgroup of 256 threads = TILE x TILE tile
// (128 for large outputs, 64 when 128-tiles would leave CUs idle), each wave
// a quarter (TILE / 32 x TILE / 32 MFMA tiles per step); K in steps of 32
// through two LDS buffers: the next step's tiles are loaded from global
// memory while the current one is multiplied, then stored to the other
// buffer, one barrier per step.  Tiles are dealt so that the workgroups of
// one XCD take consecutive tiles (n fastest): the n tiles that share an A
// block meet in one L2.  Split K (gridDim.y > 1, EPI 0 only): workgroup y
// multiplies the K range [y kc, (y + 1) kc) and writes its FP32 partial to
// Cf + y M N; the partials are added in y order afterwards.  Epilogue EPI:
// 0 = FP32 store, 1 = + bias, ReLU, BF16 store, 2 = times the ReLU mask
// (mask[i][j] > 0) and BF16 store.
template <bool A_COL, bool B_COL, int EPI, int TILE, int BK>
__global__ __launch_bounds__(256) void k_gemm_bf16(const unsigned short* __restrict__ A,
                                                   const unsigned short* __restrict__ Bm,
                                                   int M, int N, int K, int kc, int n_tn,
                                                   float* __restrict__ Cf,
                                                   unsigned short* __restrict__ Cb,
                                                   const float* __restrict__ bias,
                                                   const unsigned short* __restrict__ mask) {
  constexpr int WT = TILE / 2, MI = TILE / 32;
  __shared__ __attribute__((aligned(16))) unsigned short As[2][TILE][BK + 8];
  __shared__ __attribute__((aligned(16))) unsigned short Bs[2][TILE][BK + 8];
  const int n_tm = (M + TILE - 1) / TILE;
  // grid.x is a multiple of 8; hardware deals workgroups to the 8 XCDs in turn
  const int q = (int)((blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3));
  if (q >= n_tm * n_tn) return;   // whole workgroup
  const int tm = q / n_tn, tn = q - (q / n_tn) * n_tn;
  const int m0 = tm * TILE, n0 = tn * TILE;
  const int kb = (int)blockIdx.y * kc, ke = min(K, kb + kc);
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = (wid >> 1) * WT, wn = (wid & 1) * WT;
  // contiguous extents: A_COL -> M, else K; B_COL -> K, else N
  const bool vec_a = ((A_COL ? M : K) & 7) == 0;
  const bool vec_b = ((B_COL ? K : N) & 7) == 0;
  v4f32m acc[MI][MI];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < MI; ++j) acc[i][j] = v4f32m{0.f, 0.f, 0.f, 0.f};
  GemmStage<!A_COL, TILE, BK> sa;
  GemmStage<B_COL, TILE, BK> sb;
  sa.load(A, M, A_COL ? M : K, ke, m0, kb, vec_a, tid);
  sb.load(Bm, N, B_COL ? K : N, ke, n0, kb, vec_b, tid);
  sa.store(As[0], tid);
  sb.store(Bs[0], tid);
  __syncthreads();
  const int fr = lane & 15, fk = (lane >> 4) * 8;
  int buf = 0;
  for (int k0 = kb; k0 < ke; k0 += BK) {
    const bool more = k0 + BK < ke;
    if (more) {
      sa.load(A, M, A_COL ? M : K, ke, m0, k0 + BK, vec_a, tid);
      sb.load(Bm, N, B_COL ? K : N, ke, n0, k0 + BK, vec_b, tid);
    }
#pragma unroll
    for (int kk = 0; kk < BK; kk += 32) {   // 32-deep MFMA steps in k order
      v8u16m fa[MI], fb[MI];
#pragma unroll
      for (int i = 0; i < MI; ++i) fa[i] = *(const v8u16m*)&As[buf][wm + i * 16 + fr][kk + fk];
#pragma unroll
      for (int j = 0; j < MI; ++j) fb[j] = *(const v8u16m*)&Bs[buf][wn + j * 16 + fr][kk + fk];
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < MI; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf16m, fa[i]),
                                                              __builtin_bit_cast(v8bf16m, fb[j]),
                                                              acc[i][j], 0, 0, 0);
    }
    if (more) {
      sa.store(As[buf ^ 1], tid);
      sb.store(Bs[buf ^ 1], tid);
    }
    __syncthreads();
    buf ^= 1;
  }
  // ---- epilogue: lane holds rows 4*(lane/16)+v of column lane%16
  float* Co = Cf ? Cf + (size_t)blockIdx.y * M * N : nullptr;
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < MI; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm + i * 16 + 4 * (lane >> 4) + v;
        const int col = n0 + wn + j * 16 + (lane & 15);
        if (row < M && col < N) {
          float x = acc[i][j][v];
          const size_t o = (size_t)row * N + col;
          if constexpr (EPI == 0) {
            Co[o] = x;
          } else if constexpr (EPI == 1) {
            x += bias[col];
            x = x > 0.f ? x : 0.f;
            Cb[o] = bf16_rne(x);
            if (Co) Co[o] = x;
          } else {
            x = (mask[o] != 0) ? x : 0.f;   // bf16 activation > 0 <=> nonzero bits
            Cb[o] = bf16_rne(x);
          }
        }
      }
}

// A row's bit set: the distinct ids in [0, d_bits) among its first
// kMlpRowBits entries (repeats and out-of-range ids are ignored).
__device__ inline bool row_bit_ok(const int* __restrict__ idx, int lo, int p, int i, int d_bits) {
  if (i < 0 || i >= d_bits) return false;
  for (int q = lo; q < p; ++q)
    if (idx[q] == i) return false;
  return true;
}

// First layer (embedding bag): z1[b][j] = b1[j] + (dense W1d)[b][j] + sum over
// the row's bit set of W1b[i][j] (BF16 weights, FP32 sum); h1 = relu(z1).  The
// dense product comes from the BF16 MFMA GEMM (zd, FP32) or is absent.
__global__ __launch_bounds__(256) void k_mlp_l1(const int* __restrict__ off,
                                                const int* __restrict__ idx,
                                                const float* __restrict__ zd, int d_bits,
                                                const unsigned short* __restrict__ W1b,
                                                const float* __restrict__ b1, int H,
                                                unsigned short* __restrict__ h1) {
  const int b = blockIdx.x;
  const int lo = off[b], hi = off[b + 1];
  for (int j = threadIdx.x; j < H; j += 256) {
    float z = b1[j];
    if (zd) z += zd[(size_t)b * H + j];   // dense part, from the MFMA GEMM
    const int end = min(hi, lo + kMlpRowBits);
    for (int p = lo; p < end; ++p) {
      const int i = idx[p];
      if (row_bit_ok(idx, lo, p, i, d_bits)) z += bf16_to_f(W1b[(size_t)i * H + j]);
    }
    h1[(size_t)b * H + j] = bf16_rne(z > 0.f ? z : 0.f);
  }
}

// Output layer y[b][k] = b4[k] + sum_j h3[b][j] W4[j][k], one wave per sample.
__global__ __launch_bounds__(64) void k_mlp_out(const unsigned short* __restrict__ h3,
                                                const float* __restrict__ W4,
                                                const float* __restrict__ b4, int H,
                                                float* __restrict__ y) {
  const int b = blockIdx.x, lane = threadIdx.x;
  float s0 = 0.f, s1 = 0.f;
  for (int j = lane; j < H; j += 64) {
    const float h = bf16_to_f(h3[(size_t)b * H + j]);
    s0 += h * W4[j * 2];
    s1 += h * W4[j * 2 + 1];
  }
  for (int o = 32; o > 0; o >>= 1) {
    s0 += __shfl_xor(s0, o);
    s1 += __shfl_xor(s1, o);
  }
  if (lane == 0) {
    y[b * 2] = s0 + b4[0];
    y[b * 2 + 1] = s1 + b4[1];
  }
}

// dy = (y - t) / B; per-sample terms of the loss 1/(2B) sum (y - t)^2
// (summed in a fixed order later).
__global__ __launch_bounds__(256) void k_mlp_dy(const float* __restrict__ y,
                                                const float* __restrict__ t, int B,
                                                float* __restrict__ dy,
                                                float* __restrict__ lterm) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= B) return;
  const float e0 = y[b * 2] - t[b * 2], e1 = y[b * 2 + 1] - t[b * 2 + 1];
  dy[b * 2] = e0 / (float)B;
  dy[b * 2 + 1] = e1 / (float)B;
  lterm[b] = 0.5f * (e0 * e0 + e1 * e1) / (float)B;
}

// Output-layer backward: gW4[j][k] = sum_b h3[b][j] dy[b][k], gb4 = sum_b dy,
// and dz3[b][j] = (dy[b] . W4[j]) where h3 > 0 (BF16).  Batch sums in two
// fixed-order stages: per chunk of kRowChunk rows, then over the chunks.
constexpr int kRowChunk = 64;

__global__ __launch_bounds__(256) void k_mlp_out_bwd_w_part(const unsigned short* __restrict__ h3,
                                                            const float* __restrict__ dy, int B,
                                                            int H, float* __restrict__ part) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  const int r = blockIdx.y;
  if (j >= H) return;
  const int b0 = r * kRowChunk, b1 = min(B, b0 + kRowChunk);
  float s0 = 0.f, s1 = 0.f;
  for (int b = b0; b < b1; ++b) {
    const float h = bf16_to_f(h3[(size_t)b * H + j]);
    s0 += h * dy[b * 2];
    s1 += h * dy[b * 2 + 1];
  }
  part[((size_t)r * H + j) * 2] = s0;
  part[((size_t)r * H + j) * 2 + 1] = s1;
}

__global__ __launch_bounds__(256) void k_mlp_out_bwd_x(const unsigned short* __restrict__ h3,
                                                       const float* __restrict__ dy,
                                                       const float* __restrict__ W4, int B,
                                                       int H, unsigned short* __restrict__ dz3) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (size_t)B * H) return;
  const int b = (int)(i / H), j = (int)(i - (size_t)b * H);
  const float g = dy[b * 2] * W4[j * 2] + dy[b * 2 + 1] * W4[j * 2 + 1];
  dz3[i] = h3[i] != 0 ? bf16_rne(g) : (unsigned short)0;
}

// Column sums over the batch of a [B][n] matrix (BF16 or FP32): per chunk of
// kRowChunk rows into part[chunk][n], then k_chunk_sum over the chunks.
template <typename T>
__global__ __launch_bounds__(256) void k_colsum_part(const T* __restrict__ x, int B, int n,
                                                     float* __restrict__ part) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  const int r = blockIdx.y;
  if (j >= n) return;
  const int b0 = r * kRowChunk, b1 = min(B, b0 + kRowChunk);
  float s = 0.f;
  for (int b = b0; b < b1; ++b) {
    if constexpr (sizeof(T) == 2) s += bf16_to_f(x[(size_t)b * n + j]);
    else s += x[(size_t)b * n + j];
  }
  part[(size_t)r * n + j] = s;
}

// out[j] = sum over chunks r (in order) of part[r][j].
__global__ __launch_bounds__(256) void k_chunk_sum(const float* __restrict__ part, int R, int n,
                                                   float* __restrict__ out) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  float s = 0.f;
  for (int r = 0; r < R; ++r) s += part[(size_t)r * n + j];
  out[j] = s;
}

// The same sum for few columns and many chunks (the bias gradients): 64
// columns per workgroup, wave w adds the w-th contiguous quarter of the
// chunks in order, and the four quarter sums are added in order.
__global__ __launch_bounds__(256) void k_chunk_sum4(const float* __restrict__ part, int R, int n,
                                                    float* __restrict__ out) {
  __shared__ float q[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + lane;
  const int per = (R + 3) / 4;
  const int r0 = w * per, r1 = min(R, r0 + per);
  float s = 0.f;
  if (j < n)
    for (int r = r0; r < r1; ++r) s += part[(size_t)r * n + j];
  q[w][lane] = s;
  __syncthreads();
  if (w == 0 && j < n) out[j] = ((q[0][lane] + q[1][lane]) + q[2][lane]) + q[3][lane];
}

// First-layer weight gradient gW1b[i] = sum of dz1[b] over the samples b
// whose bit set holds i.  The (bit, sample) pairs are bucketed by bit
// (count, exclusive scan, fill); each bit's bucket is then put in sample
// order in LDS and summed over fixed runs of it, the runs' partials added in
// order, so the result does not depend on scheduling.
__global__ __launch_bounds__(256) void k_zero_i32(int* __restrict__ p, int n) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) p[i] = 0;
}

template <bool FILL>
__global__ __launch_bounds__(256) void k_bits_bucket(const int* __restrict__ off,
                                                     const int* __restrict__ idx, int B,
                                                     int d_bits, int* __restrict__ cnt,
                                                     int* __restrict__ list) {
  for (int b = blockIdx.x * 256 + threadIdx.x; b < B; b += gridDim.x * 256) {
    const int lo = off[b], end = min(off[b + 1], lo + kMlpRowBits);
    for (int p = lo; p < end; ++p) {
      const int i = idx[p];
      if (!row_bit_ok(idx, lo, p, i, d_bits)) continue;
      const int pos = atomicAdd(&cnt[i], 1);
      if constexpr (FILL) list[pos] = b;
    }
  }
}

// Exclusive scan of cnt[0..n) into start[0..n] and cursor[0..n) (one workgroup).
__global__ __launch_bounds__(1024) void k_scan_counts(const int* __restrict__ cnt, int n,
                                                      int* __restrict__ start,
                                                      int* __restrict__ cursor) {
  __shared__ int s_w[16];
  __shared__ int s_base;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  if (tid == 0) s_base = 0;
  __syncthreads();
  for (int i0 = 0; i0 < n; i0 += 1024) {
    const int i = i0 + tid;
    const int v = i < n ? cnt[i] : 0;
    int x = v;
    for (int o = 1; o < 64; o <<= 1) {
      const int u = __shfl_up(x, o);
      if (lane >= o) x += u;
    }
    if (lane == 63) s_w[wid] = x;
    __syncthreads();
    int pre = s_base;
    for (int q = 0; q < wid; ++q) pre += s_w[q];
    if (i < n) { start[i] = pre + x - v; cursor[i] = pre + x - v; }
    __syncthreads();
    if (tid == 0) {
      int t = 0;
      for (int q = 0; q < 16; ++q) t += s_w[q];
      s_base += t;
    }
    __syncthreads();
  }
  if (tid == 0) start[n] = s_base;
}

__global__ __launch_bounds__(256) void k_w1b_grad(const int* __restrict__ start,
                                                  const int* __restrict__ list,
                                                  const unsigned short* __restrict__ dz1, int H,
                                                  float* __restrict__ g) {
  constexpr int kWords = kMlpMaxTrain / 32;
  static_assert(kWords <= 256 && kWords % 64 == 0, "one bitmap word per thread, whole waves");
  __shared__ unsigned s_bits[kWords];
  __shared__ int s_sorted[kMlpMaxTrain];
  __shared__ int s_wtot[kWords / 64];
  __shared__ float s_part[2048];   // G run partials of H columns (G H = 2048)
  const int i = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
  const int lo = start[i], L = min(start[i + 1] - lo, kMlpMaxTrain);
  // the bucket's sample ids (distinct) as a bitmap, then listed in ascending
  // order: the column sums below add them in sample order, whatever order
  // the bucketing wrote them in
  if (tid < kWords) s_bits[tid] = 0u;
  __syncthreads();
  for (int q = tid; q < L; q += 256) {
    const int v = list[lo + q];
    atomicOr(&s_bits[v >> 5], 1u << (v & 31));
  }
  __syncthreads();
  unsigned word = 0u;
  int pos = 0;
  if (tid < kWords) {
    word = s_bits[tid];
    const int n = __popc(word);
    int x = n;
    for (int o = 1; o < 64; o <<= 1) {
      const int u = __shfl_up(x, o);
      if (lane >= o) x += u;
    }
    if (lane == 63) s_wtot[tid >> 6] = x;
    pos = x - n;
  }
  __syncthreads();
  if (tid < kWords) {
    for (int q = 0; q < (tid >> 6); ++q) pos += s_wtot[q];
    while (word) {
      const int b = __ffs(word) - 1;
      s_sorted[pos++] = tid * 32 + b;
      word &= word - 1u;
    }
  }
  __syncthreads();
  // column sums: each thread takes 8 adjacent columns (one 16-byte load per
  // sample) over one of G contiguous runs of the sorted bucket; the G run
  // partials are then added in run order
  const int nb = H / 8, G = 256 / nb;   // H is a multiple of 64 and at most 2048
  if (tid < nb * G) {
    const int cb = tid % nb, gr = tid / nb;
    const int q0 = (int)(((long)gr * L) / G), q1 = (int)(((long)(gr + 1) * L) / G);
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int q = q0; q < q1; ++q) {
      const v8u16m v = *(const v8u16m*)(dz1 + (size_t)s_sorted[q] * H + cb * 8);
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] += bf16_to_f(v[u]);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) s_part[gr * H + cb * 8 + u] = acc[u];
  }
  __syncthreads();
  for (int j = tid; j < H; j += 256) {
    float acc = 0.f;
    for (int gr = 0; gr < G; ++gr) acc += s_part[gr * H + j];
    g[(size_t)i * H + j] = acc;
  }
}

__global__ __launch_bounds__(256) void k_to_bf16(const float* __restrict__ x, size_t n,
                                                 unsigned short* __restrict__ y) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = bf16_rne(x[i]);
}

// y[c][r] = bf16(x[r][c]) for x [R][C]: 32 x 32 tiles through LDS.
__global__ __launch_bounds__(256) void k_to_bf16_t(const float* __restrict__ x, int R, int C,
                                                   unsigned short* __restrict__ y) {
  __shared__ float t[32][33];
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int i = ty; i < 32; i += 8) {
    const int r = r0 + i, c = c0 + tx;
    t[i][tx] = (r < R && c < C) ? x[(size_t)r * C + c] : 0.f;
  }
  __syncthreads();
  for (int i = ty; i < 32; i += 8) {
    const int c = c0 + i, r = r0 + tx;
    if (c < C && r < R) y[(size_t)c * R + r] = bf16_rne(t[tx][i]);
  }
}

// Adam (bias-corrected moments) on FP32 master weights; refreshes the BF16 copy.
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ w, float* __restrict__ m,
                                              float* __restrict__ v,
                                              const float* __restrict__ g, size_t n, float lr,
                                              float b1, float b2, float c1, float c2, float eps,
                                              unsigned short* __restrict__ wb) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[i] = wi;
  if (wb) wb[i] = bf16_rne(wi);
}

// Fixed-order sum of per-sample loss terms (single wave).
__global__ __launch_bounds__(64) void k_sum(const float* __restrict__ x, int n,
                                            float* __restrict__ out) {
  float s = 0.f;
  for (int i = threadIdx.x; i < n; i += 64) s += x[i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (threadIdx.x == 0) *out = s;
}

// ---------------------------------------------------------------------------
// k smallest scores, deterministically: radix select of the k-th smallest
// key over 4 digits of 8 bits in one workgroup, then an ordered compaction
// (all keys below the threshold, then threshold ties in index order).
__device__ inline unsigned int key_of(float f) {
  const unsigned int u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);   // ascending order of floats
}

__global__ __launch_bounds__(1024) void k_topk_smallest(const float* __restrict__ score, int n,
                                                        int stride, int k,
                                                        int* __restrict__ out) {
  __shared__ unsigned int hist[256];
  __shared__ unsigned int s_prefix, s_mask, s_need;
  __shared__ int s_wc[16];
  __shared__ int s_base;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  if (tid == 0) { s_prefix = 0; s_mask = 0; s_need = (unsigned)k; }
  __syncthreads();
  for (int shift = 24; shift >= 0; shift -= 8) {
    for (int i = tid; i < 256; i += 1024) hist[i] = 0;
    __syncthreads();
    const unsigned int pre = s_prefix, msk = s_mask;
    for (int i = tid; i < n; i += 1024) {
      const unsigned int key = key_of(score[(size_t)i * stride]);
      if ((key & msk) == pre) atomicAdd(&hist[(key >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (tid == 0) {
      unsigned int need = s_need, d = 0;
      while (d < 255 && hist[d] < need) { need -= hist[d]; ++d; }
      s_prefix = pre | (d << shift);
      s_mask = msk | (255u << shift);
      s_need = need;   // how many of the keys equal to the threshold to take
    }
    __syncthreads();
  }
  const unsigned int thr = s_prefix;
  const int ties = (int)s_need;
  // pass 1: keys strictly below the threshold; pass 2: first `ties` equal keys
  if (tid == 0) s_base = 0;
  __syncthreads();
  for (int pass = 0; pass < 2; ++pass) {
    for (int i0 = 0; i0 < n; i0 += 1024) {
      const int i = i0 + tid;
      bool take = false;
      if (i < n) {
        const unsigned int key = key_of(score[(size_t)i * stride]);
        take = pass == 0 ? key < thr : key == thr;
      }
      const unsigned long long msk64 = __ballot(take);
      if (lane == 0) s_wc[wid] = __popcll(msk64);
      __syncthreads();
      int pos = s_base;
      for (int q = 0; q < wid; ++q) pos += s_wc[q];
      pos += __popcll(msk64 & ((1ull << lane) - 1ull));
      const int limit = pass == 0 ? k : (k - ties) + ties;
      if (take && pos < limit) out[pos] = i;
      __syncthreads();
      if (tid == 0) {
        int s = 0;
        for (int q = 0; q < 16; ++q) s += s_wc[q];
        s_base += s;
      }
      __syncthreads();
    }
    if (pass == 0) {
      if (tid == 0) s_base = k - ties;
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// Batch gather: copy the genomes idx[0..k) into a compact batch.  One
// workgroup scans the gathered split slots in order (moved-list offsets and
// split buses); a second, machine-wide kernel copies the openings, moved
// lists and moved injections.
__global__ __launch_bounds__(1024) void k_gather_scan(
    const int* __restrict__ sbus, const int* __restrict__ moff, int n_src, int ns,
    const int* __restrict__ idx, int k, int* __restrict__ d_sbus, int* __restrict__ d_moff,
    int cap) {
  __shared__ int s_wsum[16];
  __shared__ int s_base;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  if (tid == 0) { s_base = 0; d_moff[0] = 0; }
  __syncthreads();
  const int slots = k * ns;
  for (int s0 = 0; s0 < slots; s0 += 1024) {
    const int sl = s0 + tid;
    int len = 0, src = 0, j = 0;
    bool okc = false;
    if (sl < slots) {
      const int c = sl / ns;
      j = sl - c * ns;
      src = idx[c];
      okc = src >= 0 && src < n_src;
      if (okc) len = moff[(size_t)src * ns + j + 1] - moff[(size_t)src * ns + j];
      if (len < 0) len = 0;
    }
    // inclusive wave scan of len, then across waves in order
    int v = len;
    for (int o = 1; o < 64; o <<= 1) {
      const int u = __shfl_up(v, o);
      if (lane >= o) v += u;
    }
    if (lane == 63) s_wsum[wid] = v;
    __syncthreads();
    int pre = s_base;
    for (int q = 0; q < wid; ++q) pre += s_wsum[q];
    const int start = pre + v - len;
    if (sl < slots) {
      const bool fits = start + len <= cap;
      const int bus = okc ? sbus[(size_t)src * ns + j] : -2;
      d_sbus[sl] = fits ? bus : (bus == -1 ? -1 : -2);
      // clipped end: monotone and inside [0, cap] even past the first overflow
      d_moff[sl + 1] = min(start + len, cap);
    }
    __syncthreads();
    if (tid == 0) {
      int sum = 0;
      for (int q = 0; q < 16; ++q) sum += s_wsum[q];
      s_base += sum;
    }
    __syncthreads();
  }
}

// One thread per gathered split slot and per gathered opening slot.  A slot's
// moved list is copied when its range got its full length (it fitted).
__global__ __launch_bounds__(256) void k_gather_copy(
    const int* __restrict__ open, const int* __restrict__ moff, const int* __restrict__ mbr,
    const double* __restrict__ mp, int n_src, int no, int ns, int T,
    const int* __restrict__ idx, int k, int* __restrict__ d_open,
    const int* __restrict__ d_moff, int* __restrict__ d_mbr, double* __restrict__ d_mp) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < k * ns) {
    const int c = i / ns, j = i - c * ns;
    const int src = idx[c];
    const bool okc = src >= 0 && src < n_src;
    if (okc) {
      const int lo = moff[(size_t)src * ns + j];
      const int len = moff[(size_t)src * ns + j + 1] - lo;
      const int dlo = d_moff[i], dhi = d_moff[i + 1];
      if (len > 0 && dhi - dlo == len)
        for (int q = 0; q < len; ++q) d_mbr[dlo + q] = mbr[lo + q];
    }
    if (d_mp)
      for (int t = 0; t < T; ++t)
        d_mp[(size_t)i * T + t] = (okc && mp) ? mp[((size_t)src * ns + j) * T + t] : 0.0;
  }
  if (i < k * no) {
    const int c = i / no, q = i - c * no;
    const int src = idx[c];
    d_open[i] = (src >= 0 && src < n_src) ? open[(size_t)src * no + q] : -2;
  }
}

void batch_gather(const int* open, const int* sbus, const int* moff, const int* mbr,
                  const double* mp, int n_src, int no, int ns, int T, const int* idx, int k,
                  int* d_open, int* d_sbus, int* d_moff, int* d_mbr, int cap, double* d_mp,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_gather_scan, dim3(1), dim3(1024), 0, s, sbus, moff, n_src, ns, idx, k,
                     d_sbus, d_moff, cap);
  const int n = k * (ns > no ? ns : no);
  if (n > 0)
    hipLaunchKernelGGL(k_gather_copy, dim3((n + 255) / 256), dim3(256), 0, s, open, moff, mbr, mp,
                       n_src, no, ns, T, idx, k, d_open, (const int*)d_moff, d_mbr, d_mp);
}

static inline int cdiv_m(long a, int b) { return (int)((a + b - 1) / b); }

// Tile edge of a GEMM: 128 when that still gives at least 512 workgroups
// (K step 32: 40 KB of LDS, three workgroups per CU), else 64 (K step 64).
static int gemm_tile(int M, int N) {
  return cdiv_m(M, 128) * cdiv_m(N, 128) >= 512 ? 128 : 64;
}

// K splits of a GEMM with FP32 output: enough workgroups to fill the chip
// (about 1024 with the tiles), each split at least 256 deep, at most 16.
int gemm_splits(int M, int N, int K) {
  const int t = gemm_tile(M, N);
  const int tiles = cdiv_m(M, t) * cdiv_m(N, t);
  const int s = std::max(1, cdiv_m(1024, tiles));
  return std::min(s, std::max(1, std::min(16, cdiv_m(K, 256))));
}

size_t mlp_split_floats(int H, int dd, int Bt) {
  const size_t a = (size_t)gemm_splits(H, H, Bt) * H * H;
  const size_t b = dd > 0 ? (size_t)gemm_splits(dd, H, Bt) * dd * H : 0;
  return std::max(std::max(a, b), (size_t)1);
}

// part: room for the split partials (gemm_splits(M, N, K) x M x N floats) or
// NULL for a single pass; splitting applies to the FP32 epilogue only.
template <bool AC, bool BC, int EPI>
static void gemm(const unsigned short* A, const unsigned short* B, int M, int N, int K, float* Cf,
                 unsigned short* Cb, const float* bias, const unsigned short* mask, float* part,
                 hipStream_t s) {
  const int t = gemm_tile(M, N);
  const int n_tn = cdiv_m(N, t), tiles = cdiv_m(M, t) * n_tn;
  int kc = K, S = 1;
  if (EPI == 0 && part) {
    const int want = gemm_splits(M, N, K);
    if (want > 1) {
      kc = cdiv_m(cdiv_m(K, want), 64) * 64;   // whole steps per split
      S = cdiv_m(K, kc);
    }
  }
  const dim3 grid((unsigned)(cdiv_m(tiles, 8) * 8), (unsigned)S);
  float* co = S > 1 ? part : Cf;
  if (t == 128)
    hipLaunchKernelGGL((k_gemm_bf16<AC, BC, EPI, 128, 32>), grid, dim3(256), 0, s, A, B, M, N, K,
                       kc, n_tn, co, Cb, bias, mask);
  else
    hipLaunchKernelGGL((k_gemm_bf16<AC, BC, EPI, 64, 64>), grid, dim3(256), 0, s, A, B, M, N, K,
                       kc, n_tn, co, Cb, bias, mask);
  if (S > 1)
    hipLaunchKernelGGL(k_chunk_sum, dim3(cdiv_m((long)M * N, 256)), dim3(256), 0, s, part, S,
                       M * N, Cf);
}

template <typename T>
static void colsum(const T* x, int B, int n, float* part, float* out, hipStream_t s) {
  const int R = cdiv_m(B, kRowChunk);
  hipLaunchKernelGGL((k_colsum_part<T>), dim3(cdiv_m(n, 256), R), dim3(256), 0, s, x, B, n, part);
  hipLaunchKernelGGL(k_chunk_sum4, dim3(cdiv_m(n, 64)), dim3(256), 0, s, part, R, n, out);
}

// ---------------------------------------------------------------------------
void mlp_forward(const MlpDev& p, const MlpBatch& wb, const int* off, const int* idx,
                 const float* dense, int B, float* y, hipStream_t s) {
  const int H = p.H, dd = p.d_dense;
  if (dd > 0) {
    hipLaunchKernelGGL(k_to_bf16, dim3(cdiv_m((long)B * dd, 256)), dim3(256), 0, s, dense,
                       (size_t)B * dd, wb.Xd);
    gemm<false, true, 0>(wb.Xd, p.W1dt_h, B, H, dd, wb.zd, nullptr, nullptr, nullptr, nullptr, s);
  }
  hipLaunchKernelGGL(k_mlp_l1, dim3(B), dim3(256), 0, s, off, idx,
                     dd > 0 ? (const float*)wb.zd : (const float*)nullptr, p.d_bits, p.W1b_h,
                     p.b1, H, wb.h1);
  gemm<false, true, 1>(wb.h1, p.W2t_h, B, H, H, nullptr, wb.h2, p.b2, nullptr, nullptr, s);
  gemm<false, true, 1>(wb.h2, p.W3t_h, B, H, H, nullptr, wb.h3, p.b3, nullptr, nullptr, s);
  hipLaunchKernelGGL(k_mlp_out, dim3(B), dim3(64), 0, s, wb.h3, p.W4, p.b4, H, y);
}

void mlp_gradients(const MlpDev& p, const MlpBatch& wb, const int* off, const int* idx,
                   const float* dense, const float* target, int B, float* grad, float* loss,
                   hipStream_t s) {
  const int H = p.H, db = p.d_bits, dd = p.d_dense;
  mlp_forward(p, wb, off, idx, dense, B, wb.y, s);
  hipLaunchKernelGGL(k_mlp_dy, dim3(cdiv_m(B, 256)), dim3(256), 0, s, wb.y, target, B, wb.dy,
                     wb.lterm);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(64), 0, s, wb.lterm, B, loss);
  MlpGrad g = mlp_grad_view(p, grad);
  // output layer
  const int R = cdiv_m(B, kRowChunk);
  hipLaunchKernelGGL(k_mlp_out_bwd_w_part, dim3(cdiv_m(H, 256), R), dim3(256), 0, s, wb.h3,
                     wb.dy, B, H, wb.part);
  hipLaunchKernelGGL(k_chunk_sum4, dim3(cdiv_m(2 * H, 64)), dim3(256), 0, s, wb.part, R, 2 * H,
                     g.W4);
  colsum<float>(wb.dy, B, 2, wb.part, g.b4, s);
  hipLaunchKernelGGL(k_mlp_out_bwd_x, dim3(cdiv_m((long)B * H, 256)), dim3(256), 0, s, wb.h3,
                     wb.dy, p.W4, B, H, wb.dz3);
  // layer 3: gW3 = h2^T dz3, gb3 = colsum dz3, dz2 = (dz3 W3^T) * [h2 > 0]
  gemm<true, false, 0>(wb.h2, wb.dz3, H, H, B, g.W3, nullptr, nullptr, nullptr, wb.gpart, s);
  colsum<unsigned short>(wb.dz3, B, H, wb.part, g.b3, s);
  gemm<false, true, 2>(wb.dz3, p.W3_h, B, H, H, nullptr, wb.dz2, nullptr, wb.h2, nullptr, s);
  // layer 2
  gemm<true, false, 0>(wb.h1, wb.dz2, H, H, B, g.W2, nullptr, nullptr, nullptr, wb.gpart, s);
  colsum<unsigned short>(wb.dz2, B, H, wb.part, g.b2, s);
  gemm<false, true, 2>(wb.dz2, p.W2_h, B, H, H, nullptr, wb.dz1, nullptr, wb.h1, nullptr, s);
  // layer 1: gW1b = X^T dz1 over the 0/1 bitmask, gW1d = dense^T dz1
  colsum<unsigned short>(wb.dz1, B, H, wb.part, g.b1, s);
  const int nb = std::min(cdiv_m(B, 256), 1024);
  hipLaunchKernelGGL(k_zero_i32, dim3(std::min(cdiv_m(db, 256), 1024)), dim3(256), 0, s, wb.cnt, db);
  hipLaunchKernelGGL((k_bits_bucket<false>), dim3(nb), dim3(256), 0, s, off, idx, B, db, wb.cnt,
                     (int*)nullptr);
  hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, s, wb.cnt, db, wb.start, wb.cursor);
  hipLaunchKernelGGL((k_bits_bucket<true>), dim3(nb), dim3(256), 0, s, off, idx, B, db,
                     wb.cursor, wb.list);
  hipLaunchKernelGGL(k_w1b_grad, dim3(db), dim3(256), 0, s, wb.start, wb.list, wb.dz1, H, g.W1b);
  if (dd > 0)   // wb.Xd holds the BF16 dense inputs from the forward pass
    gemm<true, false, 0>(wb.Xd, wb.dz1, dd, H, B, g.W1d, nullptr, nullptr, nullptr, wb.gpart, s);
}

void mlp_adam(const MlpDev& p, const float* grad, float lr, int step, hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  const size_t n = p.n_params;
  hipLaunchKernelGGL(k_adam, dim3(cdiv_m((long)n, 256)), dim3(256), 0, s, p.master, p.m, p.v,
                     grad, n, lr, b1, b2, c1, c2, eps, (unsigned short*)nullptr);
  mlp_refresh_bf16(p, s);
}

void mlp_refresh_bf16(const MlpDev& p, hipStream_t s) {
  const int H = p.H;
  MlpGrad w = mlp_grad_view(p, p.master);
  hipLaunchKernelGGL(k_to_bf16, dim3(cdiv_m((long)p.d_bits * H, 256)), dim3(256), 0, s, w.W1b,
                     (size_t)p.d_bits * H, p.W1b_h);
  hipLaunchKernelGGL(k_to_bf16, dim3(cdiv_m((long)H * H, 256)), dim3(256), 0, s, w.W2,
                     (size_t)H * H, p.W2_h);
  hipLaunchKernelGGL(k_to_bf16, dim3(cdiv_m((long)H * H, 256)), dim3(256), 0, s, w.W3,
                     (size_t)H * H, p.W3_h);
  if (p.d_dense > 0)
    hipLaunchKernelGGL(k_to_bf16_t, dim3(cdiv_m(H, 32), cdiv_m(p.d_dense, 32)), dim3(256), 0, s,
                       w.W1d, p.d_dense, H, p.W1dt_h);
  hipLaunchKernelGGL(k_to_bf16_t, dim3(cdiv_m(H, 32), cdiv_m(H, 32)), dim3(256), 0, s, w.W2, H, H,
                     p.W2t_h);
  hipLaunchKernelGGL(k_to_bf16_t, dim3(cdiv_m(H, 32), cdiv_m(H, 32)), dim3(256), 0, s, w.W3, H, H,
                     p.W3t_h);
}

void topk_smallest(const float* score, int n, int stride, int k, int* out, hipStream_t s) {
  hipLaunchKernelGGL(k_topk_smallest, dim3(1), dim3(1024), 0, s, score, n, stride, k, out);
}

}  // namespace tto
