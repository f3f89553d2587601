// Importer on the device: PTDF of the pre-optimisation topology and its
// bridges (Importer section: the DC optimizer starts from the PTDF of the
// grid; branches whose opening splits the grid are left out of the
// disconnectable set).
//
// PTDF[e][j] = b_e (X[from_e][j] - X[to_e][j]) with X = B'^{-1} (the nodal
// susceptance matrix without the slack row and column; slack row and column
// of X zero).  B' is symmetric positive definite, so it is inverted in place
// by blocked Gauss-Jordan elimination without pivoting on 64 x 64 blocks:
// for each diagonal block k, P = A_kk^{-1} (one workgroup, LDS), then
//   A_kj <- P A_kj (j != k),  A_ij <- A_ij - A_ik A_kj (i, j != k),
//   A_ik <- -A_ik P (i != k),  A_kk <- P,
// the three products on the FP64 MFMA (16x16x4): 2 N^3 flops in all.
// A branch is a bridge iff all of a transfer across it stays on it:
// H_ee = b_e S_ee = 1 (S = A X A^T), tested as 1 - H_ee < 1e-9.
#include "tto_common.h"

namespace tto {

namespace {

constexpr int kGjB = 64;   // block size

typedef double v4f64_t __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_fill_zero(double* __restrict__ A, size_t n) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    A[i] = 0.0;
}

// B' (padded to Np with unit diagonal) from the bus adjacency in CSR form:
// one thread per row, entries added in adjacency order (the matrix is zero).
__global__ __launch_bounds__(256) void k_lap_rows(const int* __restrict__ off,
                                                  const int* __restrict__ nbr,
                                                  const double* __restrict__ wgt, int n,
                                                  int slack, int Np, double* __restrict__ A) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= Np) return;
  double* row = A + (size_t)r * Np;
  if (r >= n - 1) { row[r] = 1.0; return; }
  const int v = r + (r >= slack ? 1 : 0);        // bus of this row
  double d = 0.0;
  for (int p = off[v]; p < off[v + 1]; ++p) {
    const int u = nbr[p];
    d += wgt[p];
    if (u != slack) row[u - (u > slack ? 1 : 0)] -= wgt[p];
  }
  row[r] = d;
}

// In-place Gauss-Jordan inverse of the 64 x 64 diagonal block (SPD).  Thread
// t holds the 4 x 4 sub-block at rows 4 (t / 16), columns 4 (t % 16) in
// registers; for pivot p the owners of row p and of column p publish them
// through LDS, double-buffered by the pivot's parity, so one barrier per
// pivot separates the writes from the reads (a buffer is rewritten two pivots
// later, after every thread has passed the barrier in between).
__global__ __launch_bounds__(256) void k_gj_diag(double* __restrict__ A, int Np, int kb,
                                                 double* __restrict__ Pbuf) {
  __shared__ double prow[2][kGjB], pcol[2][kGjB];
  const int tid = threadIdx.x;
  const int i0 = 4 * (tid >> 4), j0 = 4 * (tid & 15);
  const size_t k0 = (size_t)kb * kGjB;
  double a[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) a[r][c] = A[(k0 + i0 + r) * Np + k0 + j0 + c];
  for (int p = 0; p < kGjB; ++p) {
    const int buf = p & 1;
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (i0 + r == p) {
#pragma unroll
        for (int c = 0; c < 4; ++c) prow[buf][j0 + c] = a[r][c];
      }
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (j0 + c == p) {
#pragma unroll
        for (int r = 0; r < 4; ++r) pcol[buf][i0 + r] = a[r][c];
      }
    __syncthreads();
    const double inv = 1.0 / prow[buf][p];
    double rw[4], cl[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) rw[c] = j0 + c == p ? inv : prow[buf][j0 + c] * inv;
#pragma unroll
    for (int r = 0; r < 4; ++r) cl[r] = pcol[buf][i0 + r];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c)
        a[r][c] = i0 + r == p ? rw[c] : (j0 + c == p ? 0.0 : a[r][c]) - cl[r] * rw[c];
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) Pbuf[(size_t)(i0 + r) * kGjB + j0 + c] = a[r][c];
}

// 64 x 64 tile product on the MFMA: wave w computes rows 32 (w / 2) + [0, 32)
// and columns 32 (w % 2) + [0, 32) of X Y (X: 64 x 64 at ldx, Y: 64 x 64 at
// ldy), four 16x16 tiles; lane L of a tile holds rows L/16 + 4v, column L%16.
__device__ inline void tile_mfma(const double* __restrict__ X, size_t ldx,
                                 const double* __restrict__ Y, size_t ldy, v4f64_t c[2][2]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int r0 = 32 * (w >> 1), c0 = 32 * (w & 1);
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) c[a][b] = (v4f64_t){0.0, 0.0, 0.0, 0.0};
  for (int q = 0; q < kGjB; q += 4) {
    const double x0 = X[(size_t)(r0 + li) * ldx + q + lg];
    const double x1 = X[(size_t)(r0 + 16 + li) * ldx + q + lg];
    const double y0 = Y[(size_t)(q + lg) * ldy + c0 + li];
    const double y1 = Y[(size_t)(q + lg) * ldy + c0 + 16 + li];
    c[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, y0, c[0][0], 0, 0, 0);
    c[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, y1, c[0][1], 0, 0, 0);
    c[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, y0, c[1][0], 0, 0, 0);
    c[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, y1, c[1][1], 0, 0, 0);
  }
}

// element (row, col) of the workgroup's 64 x 64 tile held in c[a][b][v]
#define TILE_FOR(a, b, v, row, col)                                              \
  for (int a = 0; a < 2; ++a)                                                    \
    for (int b = 0; b < 2; ++b)                                                  \
      for (int v = 0; v < 4; ++v)                                                \
        if (const int row = 32 * ((threadIdx.x >> 6) >> 1) + 16 * a +           \
                            ((threadIdx.x & 63) >> 4) + 4 * v,                   \
                      col = 32 * ((threadIdx.x >> 6) & 1) + 16 * b + (threadIdx.x & 15); \
            true)

// A_kj <- P A_kj for the column tile j (j != k); all products before writes.
__global__ __launch_bounds__(256) void k_gj_row(double* __restrict__ A, int Np, int kb,
                                                const double* __restrict__ Pbuf) {
  const int jb = blockIdx.x >= (unsigned)kb ? blockIdx.x + 1 : blockIdx.x;
  double* T = A + (size_t)kb * kGjB * Np + (size_t)jb * kGjB;
  v4f64_t c[2][2];
  tile_mfma(Pbuf, kGjB, T, Np, c);
  __syncthreads();
  TILE_FOR(a, b, v, row, col) T[(size_t)row * Np + col] = c[a][b][v];
}

// A_ij <- A_ij - A_ik A_kj (i, j != k)
__global__ __launch_bounds__(256) void k_gj_update(double* __restrict__ A, int Np, int kb) {
  const int ib = blockIdx.y >= (unsigned)kb ? blockIdx.y + 1 : blockIdx.y;
  const int jb = blockIdx.x >= (unsigned)kb ? blockIdx.x + 1 : blockIdx.x;
  const double* X = A + (size_t)ib * kGjB * Np + (size_t)kb * kGjB;
  const double* Y = A + (size_t)kb * kGjB * Np + (size_t)jb * kGjB;
  double* C = A + (size_t)ib * kGjB * Np + (size_t)jb * kGjB;
  v4f64_t c[2][2];
  tile_mfma(X, Np, Y, Np, c);
  TILE_FOR(a, b, v, row, col) C[(size_t)row * Np + col] -= c[a][b][v];
}

// A_ik <- -A_ik P for the row tile i (i != k); all products before writes.
__global__ __launch_bounds__(256) void k_gj_col(double* __restrict__ A, int Np, int kb,
                                                const double* __restrict__ Pbuf) {
  const int ib = blockIdx.x >= (unsigned)kb ? blockIdx.x + 1 : blockIdx.x;
  double* T = A + (size_t)ib * kGjB * Np + (size_t)kb * kGjB;
  v4f64_t c[2][2];
  tile_mfma(T, Np, Pbuf, kGjB, c);
  __syncthreads();
  TILE_FOR(a, b, v, row, col) T[(size_t)row * Np + col] = -c[a][b][v];
}

__global__ __launch_bounds__(256) void k_gj_setdiag(double* __restrict__ A, int Np, int kb,
                                                    const double* __restrict__ Pbuf) {
  const size_t k0 = (size_t)kb * kGjB;
  for (int idx = threadIdx.x; idx < kGjB * kGjB; idx += 256)
    A[(k0 + idx / kGjB) * Np + k0 + idx % kGjB] = Pbuf[idx];
}

// PTDF[e][j] = b_e (X[from][j] - X[to][j]), slack rows and columns of X zero
__global__ __launch_bounds__(256) void k_ptdf_rows(const double* __restrict__ X, int Np, int n,
                                                   int slack, const int* __restrict__ from,
                                                   const int* __restrict__ to,
                                                   const double* __restrict__ b,
                                                   double* __restrict__ ptdf) {
  const int e = blockIdx.y;
  const int f = from[e], t = to[e];
  const int rf = f - (f > slack ? 1 : 0), rt = t - (t > slack ? 1 : 0);
  const double be = b[e];
  for (int j = blockIdx.x * 256 + threadIdx.x; j < n; j += gridDim.x * 256) {
    double v = 0.0;
    if (j != slack) {
      const int rj = j - (j > slack ? 1 : 0);
      const double xf = f == slack ? 0.0 : X[(size_t)rf * Np + rj];
      const double xt = t == slack ? 0.0 : X[(size_t)rt * Np + rj];
      v = be * (xf - xt);
    }
    ptdf[(size_t)e * n + j] = v;
  }
}

__global__ __launch_bounds__(256) void k_bridges(const double* __restrict__ S,
                                                 const double* __restrict__ b, int m,
                                                 uint8_t* __restrict__ out) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= m) return;
  out[e] = (1.0 - b[e] * S[(size_t)e * m + e]) < kTauCont ? 1 : 0;
}

}  // namespace

int gj_padded(int n) { return ((n - 1 + kGjB - 1) / kGjB) * kGjB; }

hipError_t launch_ptdf(const int* off, const int* nbr, const double* wgt, int n, int m,
                       int slack, const int* from, const int* to, const double* b, double* A,
                       double* Pbuf, double* ptdf, hipStream_t s) {
  const int Np = gj_padded(n);
  const int nbk = Np / kGjB;
  hipLaunchKernelGGL(k_fill_zero, dim3(2048), dim3(256), 0, s, A, (size_t)Np * Np);
  hipLaunchKernelGGL(k_lap_rows, dim3((Np + 255) / 256), dim3(256), 0, s, off, nbr, wgt, n, slack,
                     Np, A);
  for (int kb = 0; kb < nbk; ++kb) {
    hipLaunchKernelGGL(k_gj_diag, dim3(1), dim3(256), 0, s, A, Np, kb, Pbuf);
    if (nbk > 1) {
      hipLaunchKernelGGL(k_gj_row, dim3(nbk - 1), dim3(256), 0, s, A, Np, kb, (const double*)Pbuf);
      hipLaunchKernelGGL(k_gj_update, dim3(nbk - 1, nbk - 1), dim3(256), 0, s, A, Np, kb);
      hipLaunchKernelGGL(k_gj_col, dim3(nbk - 1), dim3(256), 0, s, A, Np, kb, (const double*)Pbuf);
    }
    hipLaunchKernelGGL(k_gj_setdiag, dim3(1), dim3(256), 0, s, A, Np, kb, (const double*)Pbuf);
  }
  hipLaunchKernelGGL(k_ptdf_rows, dim3((n + 255) / 256, m), dim3(256), 0, s, (const double*)A, Np,
                     n, slack, from, to, b, ptdf);
  return hipGetLastError();
}

hipError_t launch_bridges(const double* S, const double* b, int m, uint8_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_bridges, dim3((m + 255) / 256), dim3(256), 0, s, S, b, m, out);
  return hipGetLastError();
}

}  // namespace tto
