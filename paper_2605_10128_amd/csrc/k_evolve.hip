// Variation step of the MapElites loop on the device (DC-Optimizer: Mutation,
// Alg. 1; Crossover, Alg. 2; High-level loop, Alg. 3) and the expansion of
// genomes into the candidate batch encoding.
//
//   k_vary          one lane per child: parents uniform over the occupied
//                   cells (compacted per workgroup in LDS), children
//                   [0, b_mc) mutate one parent, the rest cross two.
//   k_expand_scan   one workgroup: slots of every child in canonical order,
//                   moved-list lengths, exclusive scan into the CSR offsets,
//                   split buses and opened branch ids.
//   k_expand_copy   grid-stride copy of the moved branch lists.
//   k_gen_bump      generation counter += 1 (ends a generation).
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC 2011),
// draw j of child i in generation g = word (j mod 4) of
// Philox(counter (j div 4, i, g mod 2^32, g div 2^32), key (seed mod 2^32,
// seed div 2^32)); child index 0xFFFFFFFF holds the generation's own draw
// (b_mc).  A draw r maps to an index in [0, n) as (r n) div 2^32.  Draw
// positions per child: 0, 1 parents; mutation 2 = N_mut, 3 + 3s .. 5 + 3s
// action step s (operation, slot, item), 3 + 3 N_a .. 5 + 3 N_a the
// disconnection step; crossover 2 + 2i, 3 + 2i action slot i (parent, entry),
// 2 + 2 N_a + 2i, 3 + 2 N_a + 2i disconnection slot i.
//
// Sampling rules (each a reading of the paper's operator description):
//   - "u-th element" of a set of actions: in station order (bus, id); of a
//     set of disconnections: ascending D index; u-th empty / filled slot:
//     ascending slot index.
//   - Add (action): a uniform action outside every substation the individual
//     splits, into a uniform empty slot.  Change (action): a uniform action
//     among the other actions of the split substations, into the slot of its
//     substation.  Remove: a uniform filled slot.  Disconnection Add / Change
//     sample D minus the current entries (Change into a uniform filled slot).
//   - The operation is drawn with the integer weights over the feasible
//     operations; the disconnection step takes Add when the individual holds
//     nothing (and Add is feasible).
//   - Crossover: per child slot, parent 1 with probability p_c1 (the other
//     parent when one has nothing left), then a uniform remaining entry of
//     that parent (empty entries included); the taken value also leaves the
//     other parent once; an action at an already split substation becomes
//     empty.
//   - Parents are first made feasible: out-of-range entries, actions at a
//     substation an earlier slot splits and repeated disconnections read as
//     empty.
#include "tto_common.h"
#include "tto_evolve.h"

#include <algorithm>

#include <float.h>
#include <limits.h>

namespace tto {

namespace {

constexpr uint32_t kGenChild = 0xFFFFFFFFu;
enum { OP_ADD = 0, OP_REMOVE = 1, OP_CHANGE = 2, OP_IDENTITY = 3, OP_NONE = -1 };

__device__ inline uint32_t philox_word(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                       uint32_t k0, uint32_t k1, int w) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  return w == 0 ? c0 : w == 1 ? c1 : w == 2 ? c2 : c3;
}

struct Rng {
  uint32_t k0, k1, child, g0, g1;
  __device__ uint32_t operator()(int j) const {
    return philox_word((uint32_t)(j >> 2), child, g0, g1, k0, k1, j & 3);
  }
};

__device__ inline int uidx(uint32_t r, int n) {
  return (int)(((unsigned long long)r * (unsigned long long)(unsigned)n) >> 32);
}

// k-th (from 0) empty or filled slot, ascending
__device__ inline int kth_slot(const int* x, int n, int k, bool empty) {
  int seen = 0;
  for (int i = 0; i < n; ++i) {
    if ((x[i] == -1) == empty) {
      if (seen == k) return i;
      ++seen;
    }
  }
  return 0;   // not reached: k < number of such slots by feasibility
}

// u-th integer not covered by the disjoint ranges [st, st + ln)
__device__ inline int complement_element(int u, int* st, int* ln, int nr) {
  for (int i = 1; i < nr; ++i) {
    const int s = st[i], l = ln[i];
    int j = i - 1;
    while (j >= 0 && st[j] > s) { st[j + 1] = st[j]; ln[j + 1] = ln[j]; --j; }
    st[j + 1] = s; ln[j + 1] = l;
  }
  int x = u;
  for (int i = 0; i < nr; ++i)
    if (x >= st[i]) x += ln[i];
  return x;
}

__device__ inline int weighted(uint32_t r, const int* w, bool f0, bool f1, bool f2, bool f3) {
  const int a0 = f0 ? w[0] : 0, a1 = f1 ? w[1] : 0, a2 = f2 ? w[2] : 0, a3 = f3 ? w[3] : 0;
  const int tot = a0 + a1 + a2 + a3;
  if (tot == 0) return OP_NONE;
  const int x = uidx(r, tot);
  if (x < a0) return OP_ADD;
  if (x < a0 + a1) return OP_REMOVE;
  if (x < a0 + a1 + a2) return OP_CHANGE;
  return OP_IDENTITY;
}

__device__ void action_step(const GenomeDev& gd, int* a, uint32_t r_op, uint32_t r_slot,
                            uint32_t r_item) {
  const int na = gd.n_a;
  int n_full = 0, sum_cnt = 0, n_chg = 0;
  for (int j = 0; j < na; ++j) {
    if (a[j] == -1) continue;
    const int c = gd.count[a[j]];
    ++n_full; sum_cnt += c; n_chg += c - 1;
  }
  const int n_empty = na - n_full, n_add = gd.n_actions - sum_cnt;
  const int op = weighted(r_op, gd.w_act, n_empty >= 1 && n_add >= 1, n_full >= 1, n_chg >= 1,
                          true);
  if (op == OP_ADD) {
    const int slot = kth_slot(a, na, uidx(r_slot, n_empty), true);
    int st[kGenomeSlots], ln[kGenomeSlots], nr = 0;
    for (int j = 0; j < na; ++j)
      if (a[j] != -1) { st[nr] = gd.first[a[j]]; ln[nr] = gd.count[a[j]]; ++nr; }
    const int p = complement_element(uidx(r_item, n_add), st, ln, nr);
    a[slot] = gd.st_order[p];
  } else if (op == OP_REMOVE) {
    a[kth_slot(a, na, uidx(r_slot, n_full), false)] = -1;
  } else if (op == OP_CHANGE) {
    int u = uidx(r_item, n_chg);
    for (int j = 0; j < na; ++j) {
      const int v = a[j];
      if (v == -1) continue;
      const int c = gd.count[v] - 1;
      if (u < c) {
        const int own = gd.pos[v] - gd.first[v];
        a[j] = gd.st_order[gd.first[v] + u + (u >= own ? 1 : 0)];
        break;
      }
      u -= c;
    }
  }
}

__device__ void disc_step(const GenomeDev& gd, int* d, bool force_add, uint32_t r_op,
                          uint32_t r_slot, uint32_t r_item) {
  const int nd = gd.n_d;
  int n_full = 0;
  for (int j = 0; j < nd; ++j) n_full += d[j] != -1;
  const int n_empty = nd - n_full, n_add = gd.n_disc - n_full;
  const bool f_add = n_empty >= 1 && n_add >= 1;
  const int op = (force_add && f_add)
                     ? OP_ADD
                     : weighted(r_op, gd.w_disc, f_add, n_full >= 1, n_full >= 1 && n_add >= 1,
                                true);
  if (op == OP_ADD || op == OP_CHANGE) {
    int st[kGenomeSlots], ln[kGenomeSlots], nr = 0;
    for (int j = 0; j < nd; ++j)
      if (d[j] != -1) { st[nr] = d[j]; ln[nr] = 1; ++nr; }
    const int item = complement_element(uidx(r_item, n_add), st, ln, nr);
    const int slot = op == OP_ADD ? kth_slot(d, nd, uidx(r_slot, n_empty), true)
                                  : kth_slot(d, nd, uidx(r_slot, n_full), false);
    d[slot] = item;
  } else if (op == OP_REMOVE) {
    d[kth_slot(d, nd, uidx(r_slot, n_full), false)] = -1;
  }
}

// One crossover part (actions when bus != nullptr, disconnections otherwise).
__device__ void cross_part(const int* p1, const int* p2, int n, unsigned long long thr,
                           const Rng& rnd, int j0, const int* bus, int* child) {
  int rem[2][kGenomeSlots];
  int cnt[2] = {n, n};
  for (int i = 0; i < n; ++i) { rem[0][i] = p1[i]; rem[1][i] = p2[i]; }
  int taken[kGenomeSlots], nt = 0;
  for (int i = 0; i < n; ++i) {
    int side = (unsigned long long)rnd(j0 + 2 * i) < thr ? 0 : 1;
    if (cnt[side] == 0) side = 1 - side;
    if (cnt[side] == 0) { child[i] = -1; continue; }
    const int k = uidx(rnd(j0 + 2 * i + 1), cnt[side]);
    int v = rem[side][k];
    for (int q = k; q + 1 < cnt[side]; ++q) rem[side][q] = rem[side][q + 1];
    --cnt[side];
    const int o = 1 - side;
    for (int q = 0; q < cnt[o]; ++q) {
      if (rem[o][q] == v) {
        for (int w = q; w + 1 < cnt[o]; ++w) rem[o][w] = rem[o][w + 1];
        --cnt[o];
        break;
      }
    }
    if (v != -1 && bus) {
      const int b = bus[v];
      bool dup = false;
      for (int q = 0; q < nt; ++q) dup |= taken[q] == b;
      if (dup) v = -1;
      else taken[nt++] = b;
    }
    child[i] = v;
  }
}

// Read a parent genome and make it feasible (see the header comment).
__device__ void load_parent(const GenomeDev& gd, const int* src, int* a, int* d) {
  for (int j = 0; j < gd.n_a; ++j) {
    int v = src ? src[j] : -1;
    if (v < -1 || v >= gd.n_actions) v = -1;
    if (v != -1) {
      const int b = gd.bus[v];
      for (int q = 0; q < j; ++q)
        if (a[q] != -1 && gd.bus[a[q]] == b) v = -1;
    }
    a[j] = v;
  }
  for (int j = 0; j < gd.n_d; ++j) {
    int v = src ? src[gd.n_a + j] : -1;
    if (v < -1 || v >= gd.n_disc) v = -1;
    for (int q = 0; q < j; ++q)
      if (v != -1 && d[q] == v) v = -1;
    d[j] = v;
  }
}

__global__ __launch_bounds__(256) void k_vary(GenomeDev gd, const int64_t* __restrict__ elite_id,
                                              const int* __restrict__ elite_genome, int n_cells,
                                              uint32_t k0, uint32_t k1,
                                              const int64_t* __restrict__ generation, int n_child,
                                              int* __restrict__ children, int* __restrict__ b_mc_out) {
  __shared__ int occ[kMaxCells];
  __shared__ int part[256];
  __shared__ int n_occ;
  const int tid = threadIdx.x;
  // ordered compaction of the occupied cells
  const int chunk = (n_cells + 255) / 256;
  const int lo = min(tid * chunk, n_cells), hi = min(lo + chunk, n_cells);
  int c = 0;
  for (int q = lo; q < hi; ++q) c += elite_id[q] != -1;
  part[tid] = c;
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    for (int q = 0; q < 256; ++q) { const int v = part[q]; part[q] = acc; acc += v; }
    n_occ = acc;
  }
  __syncthreads();
  int w = part[tid];
  for (int q = lo; q < hi; ++q)
    if (elite_id[q] != -1) occ[w++] = q;
  __syncthreads();

  const uint64_t g = (uint64_t)*generation;
  const uint32_t g0 = (uint32_t)g, g1 = (uint32_t)(g >> 32);
  const Rng grng{k0, k1, kGenChild, g0, g1};
  const int b_mc = uidx(grng(0), n_child + 1);
  if (blockIdx.x == 0 && tid == 0 && b_mc_out) *b_mc_out = b_mc;
  const int i = blockIdx.x * 256 + tid;
  if (i >= n_child) return;
  const Rng rnd{k0, k1, (uint32_t)i, g0, g1};
  const int G = gd.n_a + gd.n_d;
  const int no = n_occ;
  auto parent = [&](int j) -> const int* {
    if (no == 0) return nullptr;
    return elite_genome + (size_t)occ[uidx(rnd(j), no)] * G;
  };
  int a[kGenomeSlots], d[kGenomeSlots];
  if (i < b_mc) {
    load_parent(gd, parent(0), a, d);
    int n_mut = 0;
    if (gd.n_a > 0) {
      const uint32_t r = rnd(2);
      n_mut = 1;
      for (int k = 0; k + 1 < gd.n_a; ++k) n_mut += (unsigned long long)r >= gd.poisson[k];
    }
    for (int s = 0; s < n_mut; ++s) action_step(gd, a, rnd(3 + 3 * s), rnd(4 + 3 * s), rnd(5 + 3 * s));
    bool empty = true;
    for (int j = 0; j < gd.n_a; ++j) empty &= a[j] == -1;
    for (int j = 0; j < gd.n_d; ++j) empty &= d[j] == -1;
    const int j = 3 + 3 * gd.n_a;
    disc_step(gd, d, empty, rnd(j), rnd(j + 1), rnd(j + 2));
  } else {
    int a1[kGenomeSlots], d1[kGenomeSlots], a2[kGenomeSlots], d2[kGenomeSlots];
    load_parent(gd, parent(0), a1, d1);
    load_parent(gd, parent(1), a2, d2);
    cross_part(a1, a2, gd.n_a, gd.thr_c1, rnd, 2, gd.bus, a);
    cross_part(d1, d2, gd.n_d, gd.thr_c1, rnd, 2 + 2 * gd.n_a, nullptr, d);
  }
  int* out = children + (size_t)i * G;
  for (int j = 0; j < gd.n_a; ++j) out[j] = a[j];
  for (int j = 0; j < gd.n_d; ++j) out[gd.n_a + j] = d[j];
}

__device__ inline int action_len(const GenomeDev& gd, int v) {
  return (v >= 0 && v < gd.n_actions) ? gd.moff[v + 1] - gd.moff[v] : 0;
}

// Canonical slot order of an expanded candidate: valid entries ascending by
// (bus or branch id, id), then out-of-range entries, then empty slots, so
// that the evaluation of an individual does not depend on its slot order.
__device__ inline long long slot_key(int v, int n, const int* site) {
  if (v == -1) return LLONG_MAX;
  if (v < 0 || v >= n) return LLONG_MAX - 1;
  return ((long long)site[v] << 32) | (unsigned)v;
}

__device__ inline void sorted_slots(const int* src, int k, int n, const int* site, int* out) {
  long long key[kGenomeSlots];
  for (int j = 0; j < k; ++j) {
    const int v = src[j];
    const long long kv = slot_key(v, n, site);
    int q = j - 1;
    while (q >= 0 && key[q] > kv) { key[q + 1] = key[q]; out[q + 1] = out[q]; --q; }
    key[q + 1] = kv;
    out[q + 1] = v;
  }
}

__global__ __launch_bounds__(1024) void k_expand_scan(GenomeDev gd, const int* __restrict__ genomes,
                                                      int n, int* __restrict__ open,
                                                      int* __restrict__ sbus,
                                                      int* __restrict__ moff) {
  __shared__ int sums[1024];
  const int tid = threadIdx.x;
  const int G = gd.n_a + gd.n_d;
  const int chunk = (n + 1023) / 1024;
  const int lo = min(tid * chunk, n), hi = min(lo + chunk, n);
  int srt[kGenomeSlots];
  int c_sum = 0;
  for (int c = lo; c < hi; ++c) {
    sorted_slots(genomes + (size_t)c * G, gd.n_a, gd.n_actions, gd.bus, srt);
    for (int j = 0; j < gd.n_a; ++j) c_sum += action_len(gd, srt[j]);
  }
  sums[tid] = c_sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int v = tid >= off ? sums[tid - off] : 0;
    __syncthreads();
    sums[tid] += v;
    __syncthreads();
  }
  int run = sums[tid] - c_sum;
  for (int c = lo; c < hi; ++c) {
    const int* gc = genomes + (size_t)c * G;
    if (gd.n_a > 0) {
      sorted_slots(gc, gd.n_a, gd.n_actions, gd.bus, srt);
      for (int j = 0; j < gd.n_a; ++j) {
        const int v = srt[j];
        const size_t s = (size_t)c * gd.n_a + j;
        moff[s] = run;
        run += action_len(gd, v);
        sbus[s] = v == -1 ? -1 : (v >= 0 && v < gd.n_actions ? gd.bus[v] : -2);
      }
    }
    if (gd.n_d > 0) {
      sorted_slots(gc + gd.n_a, gd.n_d, gd.n_disc, gd.disc, srt);
      for (int j = 0; j < gd.n_d; ++j) {
        const int v = srt[j];
        open[(size_t)c * gd.n_d + j] = v == -1 ? -1 : (v >= 0 && v < gd.n_disc ? gd.disc[v] : -2);
      }
    }
  }
  if (tid == 1023 && gd.n_a > 0) moff[(size_t)n * gd.n_a] = sums[1023];
}

__global__ __launch_bounds__(256) void k_expand_copy(GenomeDev gd, const int* __restrict__ genomes,
                                                     int n, const int* __restrict__ moff,
                                                     int* __restrict__ mbr) {
  const int G = gd.n_a + gd.n_d;
  int srt[kGenomeSlots];
  for (int c = blockIdx.x * 256 + threadIdx.x; c < n; c += gridDim.x * 256) {
    sorted_slots(genomes + (size_t)c * G, gd.n_a, gd.n_actions, gd.bus, srt);
    for (int j = 0; j < gd.n_a; ++j) {
      const int v = srt[j];
      const int len = action_len(gd, v);
      const int dst = moff[(size_t)c * gd.n_a + j];
      for (int q = 0; q < len; ++q) mbr[dst + q] = gd.mbr[gd.moff[v] + q];
    }
  }
}

__global__ void k_gen_bump(int64_t* generation) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *generation += 1;
}

// ---------------------------------------------------------------------------
// Screened generation: the learned pre-screen's inputs taken from the
// children's genomes, and the survivors compacted in child order.

// Feature bits of each genome as a fixed-stride row of G entries: action a ->
// bit n_disc + a, disconnection d -> bit d (the bit vocabulary of the
// network: one bit per disconnectable branch, then one per action), empty or
// out-of-range slots -> -1, which the network's first layer skips.
__global__ __launch_bounds__(256) void k_genome_bits(GenomeDev gd, const int* __restrict__ genomes,
                                                     int n, int* __restrict__ off,
                                                     int* __restrict__ ids) {
  const int G = gd.n_a + gd.n_d;
  const size_t total = (size_t)n * G;
  const size_t stride = (size_t)gridDim.x * 256;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < total; i += stride) {
    const int j = (int)(i % (size_t)G);
    const int v = genomes[i];
    int bit = -1;
    if (j < gd.n_a) {
      if (v >= 0 && v < gd.n_actions) bit = gd.n_disc + v;
    } else if (v >= 0 && v < gd.n_disc) {
      bit = v;
    }
    ids[i] = bit;
  }
  for (size_t c = (size_t)blockIdx.x * 256 + threadIdx.x; c <= (size_t)n; c += stride)
    off[c] = (int)(c * G);
}

// The same dense row for every child.
__global__ __launch_bounds__(256) void k_bcast_row(const float* __restrict__ row, int d, int n,
                                                   float* __restrict__ out) {
  const size_t total = (size_t)n * d;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (size_t)gridDim.x * 256)
    out[i] = row[i % (size_t)d];
}

__global__ __launch_bounds__(256) void k_fill_i32(int* __restrict__ p, int v, int n) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) p[i] = v;
}

__global__ __launch_bounds__(256) void k_mark(const int* __restrict__ idx, int k, int n,
                                              int* __restrict__ mask) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < k) {
    const int c = idx[i];
    if (c >= 0 && c < n) mask[c] = 1;
  }
}

// Marked children in increasing index order (one workgroup, ordered scan).
__global__ __launch_bounds__(1024) void k_compact_marked(const int* __restrict__ mask, int n,
                                                         int cap, int* __restrict__ list) {
  __shared__ int s_w[16];
  __shared__ int s_base;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  if (tid == 0) s_base = 0;
  __syncthreads();
  for (int i0 = 0; i0 < n; i0 += 1024) {
    const int i = i0 + tid;
    const bool f = i < n && mask[i] != 0;
    const unsigned long long m = __ballot(f);
    if (lane == 0) s_w[wid] = __popcll(m);
    __syncthreads();
    int pos = s_base;
    for (int q = 0; q < wid; ++q) pos += s_w[q];
    pos += __popcll(m & ((1ull << lane) - 1ull));
    if (f && pos < cap) list[pos] = i;
    __syncthreads();
    if (tid == 0) {
      int t = 0;
      for (int q = 0; q < 16; ++q) t += s_w[q];
      s_base += t;
    }
    __syncthreads();
  }
}

// Archive-aware screen, first step: each child's predicted cell (from its
// genome: switch count, or the three-axis map's counts; and the predicted
// maximum loading) and predicted fitness (minus the predicted overload), and
// whether it is predicted to enter the repertoire (its predicted cell empty,
// or its predicted fitness above that cell's elite); children that are not
// get status INVALID so that the per-cell winner step ignores them.
__global__ __launch_bounds__(256) void k_screen_predict(
    GenomeDev gd, const int* __restrict__ genomes, int n, const float* __restrict__ y,
    ScreenScoreCfg sc, const double* __restrict__ edges, const double* __restrict__ elite_fit,
    const int64_t* __restrict__ elite_id, double* __restrict__ fit_pred,
    int* __restrict__ cell_pred, uint8_t* __restrict__ st_pred) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int G = gd.n_a + gd.n_d;
  const int* g = genomes + (size_t)i * G;
  int na = 0, nd = 0, moved = 0;
  for (int j = 0; j < gd.n_a; ++j) {
    const int v = g[j];
    if (v >= 0 && v < gd.n_actions) { ++na; moved += action_len(gd, v); }
  }
  for (int j = 0; j < gd.n_d; ++j) {
    const int v = g[gd.n_a + j];
    nd += (v >= 0 && v < gd.n_disc) ? 1 : 0;
  }
  const double rho = (double)y[2 * i] * sc.sd[0] + sc.mu[0] + sc.ref[0];
  const double lo = (double)y[2 * i + 1] * sc.sd[1] + sc.mu[1] + sc.ref[1];
  const double fit = -sc.overload_scale * fmax(expm1(lo), 0.0);
  int cell;
  if (sc.desc_kind == TTO_DESC_PAPER) {
    cell = min(nd, 2) + 3 * (min(na, 3) + 4 * min(moved, 45));
  } else {
    int bin = 0;
    for (int q = 0; q < sc.n_load_bins - 1; ++q) bin += (edges[q] <= rho) ? 1 : 0;
    cell = min(na + nd, sc.n_count_bins - 1) * sc.n_load_bins + bin;
  }
  const bool in_range = cell >= 0 && cell < sc.n_cells;
  const bool enters = in_range && (elite_id[cell] < 0 || fit > elite_fit[cell]);
  fit_pred[i] = fit;
  cell_pred[i] = in_range ? cell : -1;
  st_pred[i] = enters ? (uint8_t)0 : (uint8_t)TTO_ST_INVALID;
}

// Second step: the per-cell winners (best predicted fitness among the
// children predicted to enter, ties to the lower index) come first; every
// other child is ranked by its predicted overload term (column 1).
__global__ __launch_bounds__(256) void k_screen_tier(const float* __restrict__ y,
                                                     const int* __restrict__ cell_pred,
                                                     const uint8_t* __restrict__ st_pred,
                                                     const int* __restrict__ winner, int n,
                                                     float* __restrict__ score) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int cl = cell_pred[i];
  const bool first = st_pred[i] == 0 && cl >= 0 && winner[cl] == i;
  score[i] = first ? -FLT_MAX : y[2 * i + 1];
}

__global__ __launch_bounds__(256) void k_gather_rows(const int* __restrict__ src,
                                                     const int* __restrict__ list, int k, int G,
                                                     int* __restrict__ dst) {
  const size_t total = (size_t)k * G;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (size_t)gridDim.x * 256) {
    const size_t r = i / (size_t)G;
    dst[i] = src[(size_t)list[r] * G + (i - r * G)];
  }
}

}  // namespace

hipError_t launch_vary(const GenomeDev& gd, const int64_t* elite_id, const int* elite_genome,
                       int n_cells, uint64_t seed, const int64_t* generation, int n_child,
                       int* children, int* b_mc, hipStream_t s) {
  const int grid = n_child > 0 ? (n_child + 255) / 256 : 1;
  hipLaunchKernelGGL(k_vary, dim3(grid), dim3(256), 0, s, gd, elite_id, elite_genome, n_cells,
                     (uint32_t)seed, (uint32_t)(seed >> 32), generation, n_child, children, b_mc);
  return hipGetLastError();
}

hipError_t launch_expand(const GenomeDev& gd, const int* genomes, int n, int* open, int* sbus,
                         int* moff, int* mbr, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_expand_scan, dim3(1), dim3(1024), 0, s, gd, genomes, n, open, sbus, moff);
  if (gd.n_a > 0) {
    const int grid = min((n + 255) / 256, 2048);
    hipLaunchKernelGGL(k_expand_copy, dim3(grid), dim3(256), 0, s, gd, genomes, n, moff, mbr);
  }
  return hipGetLastError();
}

hipError_t launch_genome_bits(const GenomeDev& gd, const int* genomes, int n, int* off, int* ids,
                              hipStream_t s) {
  const long total = (long)n * (gd.n_a + gd.n_d) + n + 1;
  const int grid = (int)std::min<long>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(k_genome_bits, dim3(grid), dim3(256), 0, s, gd, genomes, n, off, ids);
  return hipGetLastError();
}

hipError_t launch_broadcast_row(const float* row, int d, int n, float* out, hipStream_t s) {
  if (d <= 0 || n <= 0) return hipSuccess;
  const int grid = (int)std::min<long>(((long)n * d + 255) / 256, 4096);
  hipLaunchKernelGGL(k_bcast_row, dim3(grid), dim3(256), 0, s, row, d, n, out);
  return hipGetLastError();
}

hipError_t launch_keep_in_order(const int* idx, int k, int n, int* mask, int* list, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_i32, dim3(std::min((n + 255) / 256, 1024)), dim3(256), 0, s, mask, 0,
                     n);
  if (k > 0)
    hipLaunchKernelGGL(k_mark, dim3((k + 255) / 256), dim3(256), 0, s, idx, k, n, mask);
  hipLaunchKernelGGL(k_compact_marked, dim3(1), dim3(1024), 0, s, (const int*)mask, n, k, list);
  return hipGetLastError();
}

hipError_t launch_screen_predict(const GenomeDev& gd, const int* genomes, int n, const float* y,
                                 const ScreenScoreCfg& sc, const double* edges,
                                 const double* elite_fit, const int64_t* elite_id,
                                 double* fit_pred, int* cell_pred, uint8_t* st_pred,
                                 hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_screen_predict, dim3((n + 255) / 256), dim3(256), 0, s, gd, genomes, n, y,
                     sc, edges, elite_fit, elite_id, fit_pred, cell_pred, st_pred);
  return hipGetLastError();
}

hipError_t launch_screen_tier(const float* y, const int* cell_pred, const uint8_t* st_pred,
                              const int* winner, int n, float* score, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_screen_tier, dim3((n + 255) / 256), dim3(256), 0, s, y, cell_pred, st_pred,
                     winner, n, score);
  return hipGetLastError();
}

hipError_t launch_gather_rows(const int* src, const int* list, int k, int G, int* dst,
                              hipStream_t s) {
  if (k <= 0 || G <= 0) return hipSuccess;
  const int grid = (int)std::min<long>(((long)k * G + 255) / 256, 4096);
  hipLaunchKernelGGL(k_gather_rows, dim3(grid), dim3(256), 0, s, src, list, k, G, dst);
  return hipGetLastError();
}

hipError_t launch_generation_bump(int64_t* generation, hipStream_t s) {
  hipLaunchKernelGGL(k_gen_bump, dim3(1), dim3(64), 0, s, generation);
  return hipGetLastError();
}

}  // namespace tto
