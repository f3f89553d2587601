// Grid-level kernels: the symmetric sensitivity matrix S = A L^-1 A^T, the
// monitored x contingency block of H = diag(b) S, precision conversions, and the base-flow GEMM f0 = PTDF * P on
// MFMA (Importer: PTDF of the pre-optimisation topology; DC-Optimizer: flows
// are linear in the injections).
#include "tto_common.h"

namespace tto {

typedef double v4f64 __attribute__((ext_vector_type(4)));
typedef float v4f32 __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf16 __attribute__((ext_vector_type(8)));
typedef _Float16 v8f16 __attribute__((ext_vector_type(8)));
typedef unsigned short v8u16 __attribute__((ext_vector_type(8)));

// S[e][l] = (PTDF[e][from(l)] - PTDF[e][to(l)]) / b_e: with PTDF = diag(b) A L^-1
// this is (A L^-1 A^T)_el, symmetric in exact arithmetic.
__global__ __launch_bounds__(256) void k_build_S(const double* __restrict__ ptdf,
                                                 const int* __restrict__ from,
                                                 const int* __restrict__ to,
                                                 const double* __restrict__ b, int m, int n,
                                                 double* __restrict__ S) {
  const int e = blockIdx.y;
  const int l = blockIdx.x * 256 + threadIdx.x;
  if (l >= m) return;
  const double* row = ptdf + (size_t)e * n;
  S[(size_t)e * m + l] = (row[from[l]] - row[to[l]]) / b[e];
}

// In-place symmetrisation S <- (S + S^T) / 2 over 64x64 tile pairs (I <= J),
// so that rows and columns of S are bit-identical.
__global__ __launch_bounds__(256) void k_symmetrize(double* __restrict__ S, int m) {
  __shared__ double a[64][65], c[64][65];
  const int I = blockIdx.y, J = blockIdx.x;
  if (I > J) return;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int r = ty; r < 64; r += 4) {
    const int ra = I * 64 + r, ca = J * 64 + tx;   // tile (I, J)
    const int rc = J * 64 + r, cc = I * 64 + tx;   // tile (J, I)
    a[r][tx] = (ra < m && ca < m) ? S[(size_t)ra * m + ca] : 0.0;
    c[r][tx] = (rc < m && cc < m) ? S[(size_t)rc * m + cc] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const int ra = I * 64 + r, ca = J * 64 + tx;
    const int rc = J * 64 + r, cc = I * 64 + tx;
    const double va = 0.5 * (a[r][tx] + c[tx][r]);
    const double vc = 0.5 * (c[r][tx] + a[tx][r]);
    if (ra < m && ca < m) S[(size_t)ra * m + ca] = va;
    if (rc < m && cc < m) S[(size_t)rc * m + cc] = vc;
  }
}

// Column-compacted copy of S: SMC[s][j] = S[s][col_j], col = M then C.
__global__ __launch_bounds__(256) void k_build_SMC(const double* __restrict__ S,
                                                   const int* __restrict__ mon,
                                                   const int* __restrict__ cont, int m, int nM,
                                                   int nC, double* __restrict__ SMC) {
  const int s = blockIdx.y;
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= nM + nC) return;
  const int col = j < nM ? mon[j] : cont[j - nM];
  SMC[(size_t)s * (nM + nC) + j] = S[(size_t)s * m + col];
}

// Per-row scalars of the monitored then contingency rows, contiguous in the
// row index: bMC[j] = b of row j, limM[ei] = limit of M[ei], sllC[li] = S_ll of
// l = C[li].
__global__ __launch_bounds__(256) void k_build_rows(const double* __restrict__ S,
                                                    const double* __restrict__ b,
                                                    const double* __restrict__ lim,
                                                    const int* __restrict__ mon,
                                                    const int* __restrict__ cont, int m, int nM,
                                                    int nC, double* __restrict__ bMC,
                                                    double* __restrict__ limM,
                                                    double* __restrict__ sllC) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= nM + nC) return;
  const int e = j < nM ? mon[j] : cont[j - nM];
  bMC[j] = b[e];
  if (j < nM) limM[j] = lim[e];
  else sllC[j - nM] = S[(size_t)e * m + e];
}

// Base flows of the monitored then contingency rows, timestep-major:
// f0MC[t][j] = f0[row j][t], so that the lanes of a row loop read one
// contiguous run per timestep.
__global__ __launch_bounds__(256) void k_f0_rows(const double* __restrict__ f0,
                                                 const int* __restrict__ mon,
                                                 const int* __restrict__ cont, int T, int nM,
                                                 int nC, double* __restrict__ f0MC,
                                                 float* __restrict__ f0M32) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  const int t = blockIdx.y;
  if (j >= nM + nC) return;
  const int e = j < nM ? mon[j] : cont[j - nM];
  const double v = f0[(size_t)e * T + t];
  f0MC[(size_t)t * (nM + nC) + j] = v;
  if (f0M32 && j < nM) f0M32[(size_t)t * nM + j] = (float)v;
}

// Contingency-major monitored block: HMC[li][ei] = H[M[ei], C[li]], with the
// line-outage convention that the outaged branch's own entry is H_ll - 1 so
// that its post-contingency flow f_l + (H'_ll - 1) f_l / (1 - H'_ll) is zero.
__global__ __launch_bounds__(256) void k_build_HMC(const double* __restrict__ S,
                                                   const double* __restrict__ b,
                                                   const int* __restrict__ mon,
                                                   const int* __restrict__ cont, int m, int nM,
                                                   float* __restrict__ H32,
                                                   double* __restrict__ H64) {
  const int li = blockIdx.y;
  const int ei = blockIdx.x * 256 + threadIdx.x;
  if (ei >= nM) return;
  const int l = cont[li], e = mon[ei];
  double v = b[e] * S[(size_t)l * m + e];
  if (e == l) v -= 1.0;
  H32[(size_t)li * nM + ei] = (float)v;
  H64[(size_t)li * nM + ei] = v;
}

__device__ inline unsigned short f32_to_bf16_rne(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

__device__ inline float bf16_bits_to_f32(unsigned short h) {
  return __uint_as_float((unsigned int)h << 16);
}

// Element i of a padded operand in the GEMM precision.  The split modes keep
// two planes of 16-bit values, hi = round(v) and lo = round(v - hi), the lo
// plane `plane` elements after the hi plane.
template <int PREC>
__device__ inline void store_prec(void* out, size_t i, double v, size_t plane) {
  if constexpr (PREC == TTO_GEMM_F64) {
    ((double*)out)[i] = v;
  } else if constexpr (PREC == TTO_GEMM_F32) {
    ((float*)out)[i] = (float)v;
  } else if constexpr (PREC == TTO_GEMM_BF16) {
    ((unsigned short*)out)[i] = f32_to_bf16_rne((float)v);
  } else if constexpr (PREC == TTO_GEMM_F16) {
    ((_Float16*)out)[i] = (_Float16)(float)v;
  } else if constexpr (PREC == TTO_GEMM_BF16X3) {
    const unsigned short hi = f32_to_bf16_rne((float)v);
    const double rest = v - (double)bf16_bits_to_f32(hi);
    ((unsigned short*)out)[i] = hi;
    ((unsigned short*)out)[plane + i] = f32_to_bf16_rne((float)rest);
  } else {
    const _Float16 hi = (_Float16)(float)v;
    ((_Float16*)out)[i] = hi;
    ((_Float16*)out)[plane + i] = (_Float16)(float)(v - (double)(float)hi);
  }
}

// Padded copy of the PTDF in the GEMM precision: [m_pad][ld], zeros outside.
template <int PREC>
__global__ __launch_bounds__(256) void k_convert_ptdf(const double* __restrict__ ptdf, int m,
                                                      int n, int ld, void* out, size_t plane) {
  const int row = blockIdx.y;
  for (int k = blockIdx.x * 256 + threadIdx.x; k < ld; k += gridDim.x * 256) {
    const double v = (row < m && k < n) ? ptdf[(size_t)row * n + k] : 0.0;
    store_prec<PREC>(out, (size_t)row * ld + k, v, plane);
  }
}

// Injections transposed and padded: PT[t][k] for t < kGemmN, k < ld.
template <int PREC>
__global__ __launch_bounds__(256) void k_pack_injections(const double* __restrict__ p, int n,
                                                         int T, int ld, void* out, size_t plane) {
  const int t = blockIdx.y;
  for (int k = blockIdx.x * 256 + threadIdx.x; k < ld; k += gridDim.x * 256) {
    const double v = (t < T && k < n) ? p[(size_t)k * T + t] : 0.0;
    store_prec<PREC>(out, (size_t)t * ld + k, v, plane);
  }
}

// f0 partial products on MFMA.  One wave owns 16 branch rows x 32 timestep
// columns (two 16x16 output tiles) over one k-chunk.  The order of the k
// index inside a chunk is free, so every lane group reads a contiguous run
// of its row (A) and of its timestep column (PT) and feeds consecutive MFMAs.
// Output layout of a 16x16 FP32-accumulating MFMA tile: lane L holds rows
// 4*(L/16)+v, v<4, of column L%16 (FP64: rows L/16 + 4v).
template <int PREC>
__global__ __launch_bounds__(64) void k_gemm_f0(const void* __restrict__ Av,
                                                const void* __restrict__ PTv, int m, int ld,
                                                int T, int kchunk, float* __restrict__ part32,
                                                double* __restrict__ part64, size_t a_plane,
                                                size_t p_plane) {
  const int lane = threadIdx.x;
  const int li = lane & 15, lg = lane >> 4;
  const int row0 = blockIdx.x * 16;
  const int ks = blockIdx.y;
  const int k0 = ks * kchunk;
  const int k1 = min(ld, k0 + kchunk);
  const size_t arow = (size_t)(row0 + li) * ld;
  const size_t b0row = (size_t)li * ld, b1row = (size_t)(16 + li) * ld;
  if constexpr (PREC == TTO_GEMM_F64) {
    const double* A = (const double*)Av;
    const double* PT = (const double*)PTv;
    v4f64 c0 = {0, 0, 0, 0}, c1 = {0, 0, 0, 0};
    for (int k = k0 + 4 * lg; k < k1; k += 16) {
      const double4 a = *(const double4*)(A + arow + k);
      const double4 b0 = *(const double4*)(PT + b0row + k);
      const double4 b1 = *(const double4*)(PT + b1row + k);
      c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b0.x, c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b1.x, c1, 0, 0, 0);
      c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b0.y, c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b1.y, c1, 0, 0, 0);
      c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a.z, b0.z, c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a.z, b1.z, c1, 0, 0, 0);
      c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a.w, b0.w, c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a.w, b1.w, c1, 0, 0, 0);
    }
    // the FP64 16x16x4 MFMA interleaves its rows: lane L holds rows L/16 + 4v
    double* out = part64 + (size_t)ks * m * kGemmN;
    for (int v = 0; v < 4; ++v) {
      const int row = row0 + lg + 4 * v;
      if (row < m) {
        if (li < T) out[(size_t)row * kGemmN + li] = c0[v];
        if (16 + li < T) out[(size_t)row * kGemmN + 16 + li] = c1[v];
      }
    }
  } else {
    v4f32 c0 = {0, 0, 0, 0}, c1 = {0, 0, 0, 0};
    if constexpr (PREC == TTO_GEMM_F32) {
      const float* A = (const float*)Av;
      const float* PT = (const float*)PTv;
      for (int k = k0 + 4 * lg; k < k1; k += 16) {
        const float4 a = *(const float4*)(A + arow + k);
        const float4 b0 = *(const float4*)(PT + b0row + k);
        const float4 b1 = *(const float4*)(PT + b1row + k);
        c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b0.x, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b1.x, c1, 0, 0, 0);
        c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b0.y, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b1.y, c1, 0, 0, 0);
        c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b0.z, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b1.z, c1, 0, 0, 0);
        c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b0.w, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b1.w, c1, 0, 0, 0);
      }
    } else if constexpr (PREC == TTO_GEMM_BF16X3 || PREC == TTO_GEMM_F16X3) {
      // (A_hi + A_lo)(P_hi + P_lo) without the lo*lo term: three products
      const unsigned short* A = (const unsigned short*)Av;
      const unsigned short* PT = (const unsigned short*)PTv;
      for (int k = k0 + 8 * lg; k < k1; k += 32) {
        const v8u16 ah = *(const v8u16*)(A + arow + k);
        const v8u16 al = *(const v8u16*)(A + a_plane + arow + k);
        const v8u16 ph = *(const v8u16*)(PT + b0row + k);
        const v8u16 pl = *(const v8u16*)(PT + p_plane + b0row + k);
        const v8u16 qh = *(const v8u16*)(PT + b1row + k);
        const v8u16 ql = *(const v8u16*)(PT + p_plane + b1row + k);
        if constexpr (PREC == TTO_GEMM_BF16X3) {
          const v8bf16 AH = __builtin_bit_cast(v8bf16, ah), AL = __builtin_bit_cast(v8bf16, al);
          c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(AL, __builtin_bit_cast(v8bf16, ph), c0, 0, 0, 0);
          c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(AL, __builtin_bit_cast(v8bf16, qh), c1, 0, 0, 0);
          c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(AH, __builtin_bit_cast(v8bf16, pl), c0, 0, 0, 0);
          c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(AH, __builtin_bit_cast(v8bf16, ql), c1, 0, 0, 0);
          c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(AH, __builtin_bit_cast(v8bf16, ph), c0, 0, 0, 0);
          c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(AH, __builtin_bit_cast(v8bf16, qh), c1, 0, 0, 0);
        } else {
          const v8f16 AH = __builtin_bit_cast(v8f16, ah), AL = __builtin_bit_cast(v8f16, al);
          c0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(AL, __builtin_bit_cast(v8f16, ph), c0, 0, 0, 0);
          c1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(AL, __builtin_bit_cast(v8f16, qh), c1, 0, 0, 0);
          c0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(AH, __builtin_bit_cast(v8f16, pl), c0, 0, 0, 0);
          c1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(AH, __builtin_bit_cast(v8f16, ql), c1, 0, 0, 0);
          c0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(AH, __builtin_bit_cast(v8f16, ph), c0, 0, 0, 0);
          c1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(AH, __builtin_bit_cast(v8f16, qh), c1, 0, 0, 0);
        }
      }
    } else {
      const unsigned short* A = (const unsigned short*)Av;
      const unsigned short* PT = (const unsigned short*)PTv;
      for (int k = k0 + 16 * lg; k < k1; k += 64) {
        const v8u16 a0 = *(const v8u16*)(A + arow + k);
        const v8u16 a1 = *(const v8u16*)(A + arow + k + 8);
        const v8u16 p0 = *(const v8u16*)(PT + b0row + k);
        const v8u16 p1 = *(const v8u16*)(PT + b0row + k + 8);
        const v8u16 q0 = *(const v8u16*)(PT + b1row + k);
        const v8u16 q1 = *(const v8u16*)(PT + b1row + k + 8);
        if constexpr (PREC == TTO_GEMM_BF16) {
          c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf16, a0),
                                                       __builtin_bit_cast(v8bf16, p0), c0, 0, 0, 0);
          c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf16, a0),
                                                       __builtin_bit_cast(v8bf16, q0), c1, 0, 0, 0);
          c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf16, a1),
                                                       __builtin_bit_cast(v8bf16, p1), c0, 0, 0, 0);
          c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf16, a1),
                                                       __builtin_bit_cast(v8bf16, q1), c1, 0, 0, 0);
        } else {
          c0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(v8f16, a0),
                                                      __builtin_bit_cast(v8f16, p0), c0, 0, 0, 0);
          c1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(v8f16, a0),
                                                      __builtin_bit_cast(v8f16, q0), c1, 0, 0, 0);
          c0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(v8f16, a1),
                                                      __builtin_bit_cast(v8f16, p1), c0, 0, 0, 0);
          c1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(v8f16, a1),
                                                      __builtin_bit_cast(v8f16, q1), c1, 0, 0, 0);
        }
      }
    }
    float* out = part32 + (size_t)ks * m * kGemmN;
    for (int v = 0; v < 4; ++v) {
      const int row = row0 + 4 * lg + v;
      if (row < m) {
        if (li < T) out[(size_t)row * kGemmN + li] = c0[v];
        if (16 + li < T) out[(size_t)row * kGemmN + 16 + li] = c1[v];
      }
    }
  }
}

// f0[e][t] = sum over k-chunks of the partial products, in chunk order.
template <typename P>
__global__ __launch_bounds__(256) void k_reduce_f0(const P* __restrict__ part, int m, int T,
                                                   int ksplit, double* __restrict__ f0) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= m * T) return;
  const int e = i / T, t = i - e * T;
  double s = 0.0;
  for (int k = 0; k < ksplit; ++k) s += (double)part[((size_t)k * m + e) * kGemmN + t];
  f0[i] = s;
}

// out = max_i |a_i - b_i| (one workgroup; max is order independent).
__global__ __launch_bounds__(1024) void k_max_abs_diff(const double* __restrict__ a,
                                                       const double* __restrict__ b, size_t n,
                                                       double* __restrict__ out) {
  __shared__ double s_w[16];
  double v = 0.0;
  for (size_t i = threadIdx.x; i < n; i += 1024) v = fmax(v, fabs(a[i] - b[i]));
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int q = 0; q < 16; ++q) m = fmax(m, s_w[q]);
    *out = m;
  }
}

hipError_t launch_max_abs_diff(const double* a, const double* b, size_t n, double* out,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_max_abs_diff, dim3(1), dim3(1024), 0, s, a, b, n, out);
  return hipGetLastError();
}

static inline int cdiv(int a, int b) { return (a + b - 1) / b; }

hipError_t launch_build_S(const double* ptdf, const int* from, const int* to, const double* b,
                          int m, int n, double* S, hipStream_t s) {
  hipLaunchKernelGGL(k_build_S, dim3(cdiv(m, 256), m), dim3(256), 0, s, ptdf, from, to, b, m, n, S);
  hipLaunchKernelGGL(k_symmetrize, dim3(cdiv(m, 64), cdiv(m, 64)), dim3(256), 0, s, S, m);
  return hipGetLastError();
}

hipError_t launch_build_SMC(const double* S, const int* mon, const int* cont, int m, int nM,
                            int nC, double* SMC, hipStream_t s) {
  hipLaunchKernelGGL(k_build_SMC, dim3(cdiv(nM + nC, 256), m), dim3(256), 0, s, S, mon, cont, m,
                     nM, nC, SMC);
  return hipGetLastError();
}

hipError_t launch_build_rows(const double* S, const double* b, const double* lim, const int* mon,
                             const int* cont, int m, int nM, int nC, double* bMC, double* limM,
                             double* sllC, hipStream_t s) {
  hipLaunchKernelGGL(k_build_rows, dim3(cdiv(nM + nC, 256)), dim3(256), 0, s, S, b, lim, mon,
                     cont, m, nM, nC, bMC, limM, sllC);
  return hipGetLastError();
}

hipError_t launch_f0_rows(const double* f0, const int* mon, const int* cont, int T, int nM, int nC,
                          double* f0MC, float* f0M32, hipStream_t s) {
  hipLaunchKernelGGL(k_f0_rows, dim3(cdiv(nM + nC, 256), T), dim3(256), 0, s, f0, mon, cont, T,
                     nM, nC, f0MC, f0M32);
  return hipGetLastError();
}

hipError_t launch_build_HMC(const double* S, const double* b, const int* mon, const int* cont,
                            int m, int nM, int nC, float* HMC32, double* HMC64, hipStream_t s) {
  hipLaunchKernelGGL(k_build_HMC, dim3(cdiv(nM, 256), nC), dim3(256), 0, s, S, b, mon, cont, m,
                     nM, HMC32, HMC64);
  return hipGetLastError();
}

static inline int gemm_ld(int n) { return ((n + 63) / 64) * 64; }
static inline int gemm_mpad(int m) { return ((m + 15) / 16) * 16; }

hipError_t launch_convert_ptdf(const double* ptdf, int m, int n, int prec, void* out,
                               hipStream_t s) {
  const int ld = gemm_ld(n), mp = gemm_mpad(m);
  const dim3 grid(std::min(cdiv(ld, 256), 64), mp);
  const size_t plane = (size_t)mp * ld;
  switch (prec) {
    case TTO_GEMM_F64: hipLaunchKernelGGL(k_convert_ptdf<TTO_GEMM_F64>, grid, dim3(256), 0, s, ptdf, m, n, ld, out, plane); break;
    case TTO_GEMM_F32: hipLaunchKernelGGL(k_convert_ptdf<TTO_GEMM_F32>, grid, dim3(256), 0, s, ptdf, m, n, ld, out, plane); break;
    case TTO_GEMM_BF16: hipLaunchKernelGGL(k_convert_ptdf<TTO_GEMM_BF16>, grid, dim3(256), 0, s, ptdf, m, n, ld, out, plane); break;
    case TTO_GEMM_F16: hipLaunchKernelGGL(k_convert_ptdf<TTO_GEMM_F16>, grid, dim3(256), 0, s, ptdf, m, n, ld, out, plane); break;
    case TTO_GEMM_BF16X3: hipLaunchKernelGGL(k_convert_ptdf<TTO_GEMM_BF16X3>, grid, dim3(256), 0, s, ptdf, m, n, ld, out, plane); break;
    default: hipLaunchKernelGGL(k_convert_ptdf<TTO_GEMM_F16X3>, grid, dim3(256), 0, s, ptdf, m, n, ld, out, plane); break;
  }
  return hipGetLastError();
}

hipError_t launch_pack_injections(const double* p, int n, int T, int prec, void* PT,
                                  hipStream_t s) {
  const int ld = gemm_ld(n);
  const dim3 grid(std::min(cdiv(ld, 256), 64), kGemmN);
  const size_t plane = (size_t)kGemmN * ld;
  switch (prec) {
    case TTO_GEMM_F64: hipLaunchKernelGGL(k_pack_injections<TTO_GEMM_F64>, grid, dim3(256), 0, s, p, n, T, ld, PT, plane); break;
    case TTO_GEMM_F32: hipLaunchKernelGGL(k_pack_injections<TTO_GEMM_F32>, grid, dim3(256), 0, s, p, n, T, ld, PT, plane); break;
    case TTO_GEMM_BF16: hipLaunchKernelGGL(k_pack_injections<TTO_GEMM_BF16>, grid, dim3(256), 0, s, p, n, T, ld, PT, plane); break;
    case TTO_GEMM_F16: hipLaunchKernelGGL(k_pack_injections<TTO_GEMM_F16>, grid, dim3(256), 0, s, p, n, T, ld, PT, plane); break;
    case TTO_GEMM_BF16X3: hipLaunchKernelGGL(k_pack_injections<TTO_GEMM_BF16X3>, grid, dim3(256), 0, s, p, n, T, ld, PT, plane); break;
    default: hipLaunchKernelGGL(k_pack_injections<TTO_GEMM_F16X3>, grid, dim3(256), 0, s, p, n, T, ld, PT, plane); break;
  }
  return hipGetLastError();
}

// Split the k range so that the launch has several waves per CU.
int gemm_ksplit(int m, int n) {
  const int ld = gemm_ld(n);
  const int tiles = gemm_mpad(m) / 16;
  int ks = std::max(1, 4096 / std::max(tiles, 1));
  ks = std::min(ks, ld / 64);
  return std::max(ks, 1);
}

hipError_t launch_gemm_f0(int prec, const void* A, const void* PT, int m, int n, int T,
                          int ksplit, float* part32, double* part64, double* f0,
                          hipStream_t s) {
  const int ld = gemm_ld(n);
  int kchunk = cdiv(cdiv(ld, ksplit), 64) * 64;
  const dim3 grid(gemm_mpad(m) / 16, ksplit);
  const size_t ap = (size_t)gemm_mpad(m) * ld, pp = (size_t)kGemmN * ld;
  switch (prec) {
    case TTO_GEMM_F64: hipLaunchKernelGGL(k_gemm_f0<TTO_GEMM_F64>, grid, dim3(64), 0, s, A, PT, m, ld, T, kchunk, part32, part64, ap, pp); break;
    case TTO_GEMM_F32: hipLaunchKernelGGL(k_gemm_f0<TTO_GEMM_F32>, grid, dim3(64), 0, s, A, PT, m, ld, T, kchunk, part32, part64, ap, pp); break;
    case TTO_GEMM_BF16: hipLaunchKernelGGL(k_gemm_f0<TTO_GEMM_BF16>, grid, dim3(64), 0, s, A, PT, m, ld, T, kchunk, part32, part64, ap, pp); break;
    case TTO_GEMM_F16: hipLaunchKernelGGL(k_gemm_f0<TTO_GEMM_F16>, grid, dim3(64), 0, s, A, PT, m, ld, T, kchunk, part32, part64, ap, pp); break;
    case TTO_GEMM_BF16X3: hipLaunchKernelGGL(k_gemm_f0<TTO_GEMM_BF16X3>, grid, dim3(64), 0, s, A, PT, m, ld, T, kchunk, part32, part64, ap, pp); break;
    default: hipLaunchKernelGGL(k_gemm_f0<TTO_GEMM_F16X3>, grid, dim3(64), 0, s, A, PT, m, ld, T, kchunk, part32, part64, ap, pp); break;
  }
  if (prec == TTO_GEMM_F64)
    hipLaunchKernelGGL(k_reduce_f0<double>, dim3(cdiv(m * T, 256)), dim3(256), 0, s, part64, m, T, ksplit, f0);
  else
    hipLaunchKernelGGL(k_reduce_f0<float>, dim3(cdiv(m * T, 256)), dim3(256), 0, s, part32, m, T, ksplit, f0);
  return hipGetLastError();
}

}  // namespace tto
