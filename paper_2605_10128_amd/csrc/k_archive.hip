// One-elite-per-cell repertoire update (High-level loop, Alg. 3: insert each
// new individual into the cell given by beta; a cell keeps one elite, replaced
// only by a strictly better fitness).
//
// The batch's winner per cell comes from an order-free 64-bit atomic max of a
// monotone key of the fitness, then the lowest index among exact ties; the
// result equals offering the candidates one at a time in index order.  The
// genome variant also copies the winner's genome and takes candidate ids from
// the device-side generation counter (ids generation * B + i), so that a
// captured generation can be replayed unchanged.
#include "tto_common.h"
#include "tto_evolve.h"

#include <limits.h>

#include <mutex>
#include <vector>

namespace tto {

__device__ inline unsigned long long order_key(double d) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(d);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

__global__ __launch_bounds__(256) void k_arch_init(unsigned long long* key, int* idx, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) { key[i] = 0ull; idx[i] = INT_MAX; }
}

__global__ __launch_bounds__(256) void k_arch_key(const double* fit, const int* cell,
                                                  const uint8_t* st, int B, int n_cells,
                                                  unsigned long long* key) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= B) return;
  const int cl = cell[i];
  if ((st[i] & (TTO_ST_ISLANDED | TTO_ST_INVALID)) || cl < 0 || cl >= n_cells) return;
  atomicMax(key + cl, order_key(fit[i]));
}

__global__ __launch_bounds__(256) void k_arch_idx(const double* fit, const int* cell,
                                                  const uint8_t* st, int B, int n_cells,
                                                  const unsigned long long* key, int* idx) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= B) return;
  const int cl = cell[i];
  if ((st[i] & (TTO_ST_ISLANDED | TTO_ST_INVALID)) || cl < 0 || cl >= n_cells) return;
  if (order_key(fit[i]) == key[cl]) atomicMin(idx + cl, i);
}

__global__ __launch_bounds__(256) void k_arch_apply(const double* fit, const int* idx,
                                                    int n_cells, int64_t id_base,
                                                    double* elite_fit, int64_t* elite_id) {
  const int cl = blockIdx.x * 256 + threadIdx.x;
  if (cl >= n_cells) return;
  const int i = idx[cl];
  if (i == INT_MAX) return;
  const double f = fit[i];
  if (elite_id[cl] == -1 || f > elite_fit[cl]) {
    elite_fit[cl] = f;
    elite_id[cl] = id_base + i;
  }
}

__global__ __launch_bounds__(256) void k_arch_apply_genome(
    const double* fit, const int* idx, int n_cells, const int64_t* generation,
    const int* id_map, int id_stride, double* elite_fit, int64_t* elite_id, int* elite_genome,
    const int* genomes, int G) {
  const int cl = blockIdx.x * 256 + threadIdx.x;
  if (cl >= n_cells) return;
  const int i = idx[cl];
  if (i == INT_MAX) return;
  const double f = fit[i];
  if (elite_id[cl] == -1 || f > elite_fit[cl]) {
    elite_fit[cl] = f;
    elite_id[cl] = *generation * (int64_t)id_stride + (id_map ? id_map[i] : i);
    for (int j = 0; j < G; ++j) elite_genome[(size_t)cl * G + j] = genomes[(size_t)i * G + j];
  }
}

static inline int cdiv(int a, int b) { return (a + b - 1) / b; }

static void launch_winners(int n_cells, const double* fit, const int* cell,
                           const uint8_t* status, int B, unsigned long long* key, int* idx,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_arch_init, dim3(cdiv(n_cells, 256)), dim3(256), 0, s, key, idx, n_cells);
  if (B > 0) {
    hipLaunchKernelGGL(k_arch_key, dim3(cdiv(B, 256)), dim3(256), 0, s, fit, cell, status, B,
                       n_cells, key);
    hipLaunchKernelGGL(k_arch_idx, dim3(cdiv(B, 256)), dim3(256), 0, s, fit, cell, status, B,
                       n_cells, key, idx);
  }
}

hipError_t launch_cell_winners(int n_cells, const double* fit, const int* cell,
                               const uint8_t* status, int B, unsigned long long* key, int* idx,
                               hipStream_t s) {
  launch_winners(n_cells, fit, cell, status, B, key, idx, s);
  return hipGetLastError();
}

hipError_t launch_archive(double* elite_fit, int64_t* elite_id, int n_cells, const double* fit,
                          const int* cell, const uint8_t* status, int B, int64_t id_base,
                          unsigned long long* key, int* idx, hipStream_t s) {
  launch_winners(n_cells, fit, cell, status, B, key, idx, s);
  hipLaunchKernelGGL(k_arch_apply, dim3(cdiv(n_cells, 256)), dim3(256), 0, s, fit, idx, n_cells,
                     id_base, elite_fit, elite_id);
  return hipGetLastError();
}

// Scratch of the allocation-free insertion: per cell a 64-bit key, then per
// cell a 32-bit winner index (the layout of the caller's workspace in
// tto_archive_insert).  One copy per GPU, held until the process ends; its
// address on each device is taken once, with that device current, when the
// first grid is created there.
static __device__ __align__(256) unsigned char scratch[16 * (size_t)kArchiveStaticCells];

namespace {
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;   // device address of `scratch`, per device
}  // namespace

hipError_t archive_scratch_init(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0) return hipErrorInvalidDevice;
  if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize((size_t)device + 1, nullptr);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

void* archive_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0 || device >= (int)g_scratch_ptr.size()) return nullptr;
  return g_scratch_ptr[device];
}

hipError_t launch_archive_genome(double* elite_fit, int64_t* elite_id, int* elite_genome,
                                 int n_cells, const double* fit, const int* cell,
                                 const uint8_t* status, int B, const int64_t* generation,
                                 const int* genomes, int G, const int* id_map, int id_stride,
                                 unsigned long long* key, int* idx, hipStream_t s) {
  launch_winners(n_cells, fit, cell, status, B, key, idx, s);
  hipLaunchKernelGGL(k_arch_apply_genome, dim3(cdiv(n_cells, 256)), dim3(256), 0, s, fit, idx,
                     n_cells, generation, id_map, id_stride, elite_fit, elite_id, elite_genome,
                     genomes, G);
  return hipGetLastError();
}

}  // namespace tto
