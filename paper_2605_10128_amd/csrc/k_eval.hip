// Per-candidate kernels of the batched DC N-1 screen.
//
//   k_setup    FP64 rank-r update of the pre-computed distribution factors for
//              the candidate's openings and bus splits (DC-Optimizer: topology
//              changes enter as low-rank updates of the PTDF), islanding pivot
//              test, post-switch flows f', per-contingency LODF denominators
//              1 - H'_ll and the compacted list of non-islanding contingencies.
//   k_sweep    N-1 flows f^(l)_e(t) = f'_e(t) + H'_el f'_l(t) / (1 - H'_ll) for
//              every monitored e, active contingency l and timestep t, with the
//              running max |f| fused in (f^max of the Fitness function
//              heuristics section) and the per-branch overload sums reduced
//              per block.
//   k_finalize deterministic combination of the block partials, arg-max
//              contingency, fitness lambda_f1 and the descriptor cell.
//   k_n1_dump  full N-1 flow tensor for small debugging batches.
//   k_arch_*   one-elite-per-cell repertoire update.
//
// Algebra of a candidate (standard DC sensitivities; the paper cites, but does
// not print, its low-rank formulas).  H = PTDF A^T, H_el = flow on e per MW
// sent across l.  Opening branch k is modelled as a transfer x_k across k that
// cancels k's own flow; splitting bus i into busbars A and B as an unknown
// angle step Delta_j applied to every moved branch b (sign sg_b = +1 if b
// leaves i).  With u_j = sum_b sg_b b_b (e_b - H_:,b) the unknowns z = (x, Delta)
// solve the r x r bordered system
//    [ I - H_KK      -u_j(K)   ] [x]   [ f0_K           ]
//    [ Y_jK          S - Q     ] [D] = [ p_j - phi_j    ]
// with Y_jk = sum_b sg_b H_bk, Q_jj' = sum_{b,b'} sg_b sg_b' b_b' H_bb',
// S_jj' = sum_{b in S_j and S_j'} sg sg' b_b, phi_j = sum_b sg_b f0_b, p_j the
// moved injection.  Split rows are divided by s_j = sum_b b_b.  Then
// f' = f0 + U z with U = [H_:,K, u_j], zero on opened branches, and the
// post-switch factor column of contingency l is H'_:,l = H_:,l + U V_l with
// V_l the solution for right-hand side [H_Kl ; ps_l - Y_jl] (ps_l = sg_l if l
// itself is moved by split j).
#include "tto_common.h"

#include <float.h>
#include <limits.h>
#include <math.h>

namespace tto {

__device__ inline unsigned long long ballot64(bool p) { return __ballot(p); }

// LU solve with the factors in s_M (row swaps in s_piv), in place on x[0..r).
__device__ inline void lu_solve(const double (*s_M)[kMaxRank], const int* s_piv, int r,
                                double* x) {
#pragma unroll
  for (int i = 0; i < kMaxRank; ++i) {
    if (i < r) {
      const int p = s_piv[i];
      // swap x[i] and x[p] (p >= i) with selects only: no dynamic indexing
      const double xi = x[i];
      double xp = xi;
#pragma unroll
      for (int q = 0; q < kMaxRank; ++q)
        if (q > i) xp = (q == p) ? x[q] : xp;
#pragma unroll
      for (int q = 0; q < kMaxRank; ++q)
        if (q > i) x[q] = (q == p) ? xi : x[q];
      x[i] = xp;
    }
  }
#pragma unroll
  for (int i = 0; i < kMaxRank; ++i) {
    if (i < r) {
#pragma unroll
      for (int q = 0; q < kMaxRank; ++q)
        if (q < i) x[i] -= s_M[i][q] * x[q];
    }
  }
#pragma unroll
  for (int i = kMaxRank - 1; i >= 0; --i) {
    if (i < r) {
#pragma unroll
      for (int q = 0; q < kMaxRank; ++q)
        if (q > i && q < r) x[i] -= s_M[i][q] * x[q];
      x[i] /= s_M[i][i];
    }
  }
}

// Compiler barrier: keeps the per-column LDS reads of x(t) inside the column
// loops instead of hoisting 8 x TT doubles into registers.
__device__ inline void keep_in_loop() { __asm__ volatile("" ::: "memory"); }

// Shared description of one candidate inside k_setup.
struct SetupShared {
  int open[kMaxRank];      // opened branch ids (column q < k)
  double bK[kMaxRank];     // their susceptances
  int sslot[kMaxRank];     // genome slot of split j (for the moved injection)
  int sbus[kMaxRank];      // split buses
  int moff[kMaxRank + 1];  // moved-branch ranges per split j
  int mbr[kMaxMoved];      // moved branch ids
  int mj[kMaxMoved];       // split index of each moved branch
  double msign[kMaxMoved]; // sg_b = +1 if b leaves the split bus
  double msg[kMaxMoved];   // sg_b * b_b
  double inv_s[kMaxRank];  // 1 / sum_b b_b per split
  double M[kMaxRank][kMaxRank];
  int piv[kMaxRank];
  int hdr[4];              // valid, k, ns, islanded
};

// Column gather for branch e: W[q] = S[K_q][e] (q < k) and
// W[k + j] = sum_{b in S_j} sg_b b_b S[b][e]; loads issued four at a time.
// Written to the per-thread row wrow[0..7] (dynamic q), zero beyond r.
__device__ inline void gather_column(const GridDev& g, const SetupShared& sh, int e, int k,
                                     int ns, double* wrow) {
  const size_t m = g.n_branch;
  const int r = k + ns;
#pragma unroll 4
  for (int q = 0; q < k; ++q) wrow[q] = g.S[(size_t)sh.open[q] * m + e];
  for (int j = 0; j < ns; ++j) {
    double acc = 0.0;
    const int p1 = sh.moff[j + 1];
#pragma unroll 4
    for (int p = sh.moff[j]; p < p1; ++p) acc += sh.msg[p] * g.S[(size_t)sh.mbr[p] * m + e];
    wrow[k + j] = acc;
  }
  for (int q = r; q < kMaxRank; ++q) wrow[q] = 0.0;
}

template <typename F, int TT>
__global__ __launch_bounds__(256) void k_setup(GridDev g, BatchDev bt, SweepBufs<F> w,
                                               double* __restrict__ base_out) {
  constexpr int RS = rec_stride(TT);
  const int c = blockIdx.x;
  const int tid = threadIdx.x;
  const int m = g.n_branch, T = g.T, nM = g.nM, nC = g.nC;

  __shared__ SetupShared sh;
  __shared__ double s_x[kMaxRank][TT];
  __shared__ double s_w[256][kMaxRank + 1];   // per-thread column gather (padded)
  __shared__ int s_wcnt[4];
  __shared__ int s_base, s_n0, s_nisl;

  if (tid == 0) {
    int valid = 1, k = 0, s = 0, nm = 0;
    for (int i = 0; i < bt.no; ++i) {
      const int v = bt.open[(size_t)c * bt.no + i];
      if (v == -1) continue;
      if (v < 0 || v >= m) { valid = 0; continue; }
      for (int q = 0; q < k; ++q) if (sh.open[q] == v) valid = 0;
      if (k >= kMaxRank) { valid = 0; continue; }
      sh.bK[k] = g.b[v];
      sh.open[k++] = v;
    }
    for (int j = 0; j < bt.ns; ++j) {
      const int bus = bt.sbus[(size_t)c * bt.ns + j];
      if (bus == -1) continue;
      if (bus < 0 || bus >= g.n_bus || s >= kMaxRank) { valid = 0; continue; }
      for (int q = 0; q < s; ++q) if (sh.sbus[q] == bus) valid = 0;
      const int lo = bt.moff[(size_t)c * bt.ns + j], hi = bt.moff[(size_t)c * bt.ns + j + 1];
      // CSR sanity: offsets inside [0, total moved] and increasing
      const int tot = bt.moff[(size_t)bt.B * bt.ns];
      if (lo < 0 || hi > tot || hi <= lo) { valid = 0; continue; }
      sh.moff[s] = nm;
      double ssum = 0.0;
      for (int p = lo; p < hi; ++p) {
        const int e = bt.mbr[p];
        if (e < 0 || e >= m) { valid = 0; continue; }
        const int f = g.from[e], t = g.to[e];
        if (f != bus && t != bus) valid = 0;
        for (int q = sh.moff[s]; q < nm; ++q) if (sh.mbr[q] == e) valid = 0;
        for (int q = 0; q < k; ++q) if (sh.open[q] == e) valid = 0;
        if (nm >= kMaxMoved) { valid = 0; continue; }
        const double sg = (f == bus) ? 1.0 : -1.0;
        sh.mbr[nm] = e;
        sh.mj[nm] = s;
        sh.msign[nm] = sg;
        sh.msg[nm] = sg * g.b[e];
        ssum += g.b[e];
        ++nm;
      }
      sh.sbus[s] = bus;
      sh.sslot[s] = j;
      sh.inv_s[s] = ssum > 0.0 ? 1.0 / ssum : 0.0;
      ++s;
    }
    sh.moff[s] = nm;
    if (k + s > kMaxRank) valid = 0;
    sh.hdr[0] = valid;
    sh.hdr[1] = k;
    sh.hdr[2] = s;
    sh.hdr[3] = 0;
    s_base = 0;
    s_n0 = 0;
    s_nisl = 0;
  }
  __syncthreads();
  const int valid = sh.hdr[0], k = sh.hdr[1], ns = sh.hdr[2];
  const int r = k + ns;
  CandInfo* inf = w.info + c;
  if (!valid) {
    if (tid == 0) {
      inf->status = TTO_ST_INVALID;
      inf->r = 0; inf->k = 0; inf->n_act = 0; inf->n_act_pad = 0; inf->n_island = 0;
      inf->n_crit_n0 = 0;
    }
    return;
  }

  // bordered matrix M_c, one entry per thread; H_ab = b_a S_ab
  if (tid < r * r) {
    const int i = tid / r, q = tid - (tid / r) * r;
    const size_t mm = m;
    double v = 0.0;
    if (i < k) {
      const size_t ki = (size_t)sh.open[i] * mm;
      if (q < k) {
        v = (i == q ? 1.0 : 0.0) - sh.bK[i] * g.S[ki + sh.open[q]];
      } else {
        const int j = q - k;
        for (int p = sh.moff[j]; p < sh.moff[j + 1]; ++p) v += sh.msg[p] * g.S[ki + sh.mbr[p]];
        v *= sh.bK[i];
      }
    } else {
      const int j = i - k;
      if (q < k) {
        for (int p = sh.moff[j]; p < sh.moff[j + 1]; ++p)
          v += sh.msg[p] * g.S[(size_t)sh.mbr[p] * mm + sh.open[q]];
      } else {
        const int j2 = q - k;
        for (int p = sh.moff[j]; p < sh.moff[j + 1]; ++p) {
          const size_t bp = (size_t)sh.mbr[p] * mm;
          for (int p2 = sh.moff[j2]; p2 < sh.moff[j2 + 1]; ++p2) {
            v -= sh.msg[p] * sh.msg[p2] * g.S[bp + sh.mbr[p2]];
            if (sh.mbr[p] == sh.mbr[p2]) v += sh.msign[p] * sh.msign[p2] * g.b[sh.mbr[p]];
          }
        }
      }
      v *= sh.inv_s[j];
    }
    sh.M[i][q] = v;
  }
  __syncthreads();
  if (tid == 0) {
    double minpiv = DBL_MAX;
    for (int p = 0; p < r; ++p) {
      int best = p;
      double bv = fabs(sh.M[p][p]);
      for (int i = p + 1; i < r; ++i)
        if (fabs(sh.M[i][p]) > bv) { bv = fabs(sh.M[i][p]); best = i; }
      sh.piv[p] = best;
      if (best != p)
        for (int q = 0; q < r; ++q) { const double t = sh.M[p][q]; sh.M[p][q] = sh.M[best][q]; sh.M[best][q] = t; }
      minpiv = fmin(minpiv, bv);
      if (bv > 0.0) {
        for (int i = p + 1; i < r; ++i) {
          const double f = sh.M[i][p] / sh.M[p][p];
          sh.M[i][p] = f;
          for (int q = p + 1; q < r; ++q) sh.M[i][q] -= f * sh.M[p][q];
        }
      }
    }
    sh.hdr[3] = (r > 0 && minpiv < kTauIsland) ? 1 : 0;
  }
  __syncthreads();
  if (sh.hdr[3]) {
    if (tid == 0) {
      inf->status = TTO_ST_ISLANDED;
      inf->r = r; inf->k = k; inf->n_act = 0; inf->n_act_pad = 0; inf->n_island = 0;
      inf->n_crit_n0 = 0;
    }
    return;
  }

  // x(t) = M_c^{-1} rhs(t), rhs = [f0_K ; (p_j - phi_j) / s_j]
  if (tid < TT) {
    const int t = tid;
    double x[kMaxRank];
#pragma unroll
    for (int q = 0; q < kMaxRank; ++q) {
      double v = 0.0;
      if (t < T) {
        if (q < k) {
          v = g.f0[(size_t)sh.open[q] * T + t];
        } else if (q < r) {
          const int j = q - k;
          double phi = 0.0;
          for (int p = sh.moff[j]; p < sh.moff[j + 1]; ++p) phi += sh.msign[p] * g.f0[(size_t)sh.mbr[p] * T + t];
          const double pj = bt.mp ? bt.mp[((size_t)c * bt.ns + sh.sslot[j]) * T + t] : 0.0;
          v = (pj - phi) * sh.inv_s[j];
        }
      }
      x[q] = v;
    }
    if (t < T) lu_solve(sh.M, sh.piv, r, x);
#pragma unroll
    for (int q = 0; q < kMaxRank; ++q) s_x[q][t] = (t < T) ? x[q] : 0.0;
  }
  __syncthreads();

  double* wrow = s_w[tid];
  const int nm = sh.moff[ns];
  // U row of branch e from its column gather: U_q = b_e W_q (openings),
  // U_{k+j} = -b_e W_{k+j} + sum_{b in S_j, b = e} sg_b b_b (moved-branch term)
  auto u_from_w = [&](int e, double be, double* U) {
#pragma unroll
    for (int q = 0; q < kMaxRank; ++q) U[q] = (q < k ? be : -be) * wrow[q];
    for (int p = 0; p < nm; ++p) {
      if (sh.mbr[p] == e) {
        const int qq = k + sh.mj[p];
#pragma unroll
        for (int q = 0; q < kMaxRank; ++q)
          if (q == qq) U[q] += sh.msg[p];
      }
    }
  };

  // monitored rows: f'_M and U_M
  int n0 = 0;
  for (int ei = tid; ei < nM; ei += 256) {
    keep_in_loop();
    const int e = g.mon[ei];
    bool opened = false;
    for (int q = 0; q < k; ++q) opened |= (sh.open[q] == e);
    gather_column(g, sh, e, k, ns, wrow);
    double U[kMaxRank];
    u_from_w(e, g.b[e], U);
    const double lim = g.lim[e];
    F* fo = w.fM + ((size_t)c * nM + ei) * TT;
#pragma unroll
    for (int t = 0; t < TT; ++t) {
      double fp = 0.0;
      if (t < T && !opened) {
        fp = g.f0[(size_t)e * T + t];
#pragma unroll
        for (int q = 0; q < kMaxRank; ++q) fp += U[q] * s_x[q][t];
        n0 += fabs(fp) > lim;
      }
      fo[t] = (F)fp;
    }
    F* uo = w.UM + ((size_t)c * nM + ei) * kVSlots;
#pragma unroll
    for (int q = 0; q < kVSlots; ++q) uo[q] = opened ? (F)0 : (F)U[q];
  }
  if (n0) atomicAdd(&s_n0, n0);

  // optional full post-switch base flows
  if (base_out) {
    for (int e = tid; e < m; e += 256) {
      keep_in_loop();
      bool opened = false;
      for (int q = 0; q < k; ++q) opened |= (sh.open[q] == e);
      gather_column(g, sh, e, k, ns, wrow);
      double U[kMaxRank];
      u_from_w(e, g.b[e], U);
      for (int t = 0; t < T; ++t) {
        double fp = 0.0;
        if (!opened) {
          fp = g.f0[(size_t)e * T + t];
#pragma unroll
          for (int q = 0; q < kMaxRank; ++q) fp += U[q] * s_x[q][t];
        }
        base_out[((size_t)c * m + e) * T + t] = fp;
      }
    }
  }

  // contingencies: V_l, denominators, phi_l, ordered compaction
  const int lane = tid & 63, wid = tid >> 6;
  F* rec = w.rec + (size_t)c * (nC + 1) * RS;
  int* act = w.act + (size_t)c * (nC + 1);
  int nisl = 0;
  for (int base = 0; base < nC; base += 256) {
    keep_in_loop();
    const int li = base + tid;
    bool active = false, island = false, opened = false;
    int l = 0;
    double V[kMaxRank], U[kMaxRank];
    double inv_d = 0.0;
#pragma unroll
    for (int q = 0; q < kMaxRank; ++q) { V[q] = 0.0; U[q] = 0.0; }
    if (li < nC) {
      l = g.cont[li];
      for (int q = 0; q < k; ++q) opened |= (sh.open[q] == l);
      if (opened) {
        active = true;  // already open: the N-0 state (phi = 0)
      } else {
        gather_column(g, sh, l, k, ns, wrow);
        const double bl = g.b[l];
        // right-hand side of the factor column: R_q = b_{K_q} W_q (openings),
        // R_{k+j} = (ps_j - W_{k+j}) / s_j with ps_j = sg_l if l is moved by j
#pragma unroll
        for (int q = 0; q < kMaxRank; ++q) {
          double v = 0.0;
          if (q < k) v = sh.bK[q] * wrow[q];
          else if (q < r) v = -wrow[q] * sh.inv_s[q - k];
          V[q] = v;
        }
        for (int p = 0; p < nm; ++p) {
          if (sh.mbr[p] == l) {
            const int qq = k + sh.mj[p];
            const double add = sh.msign[p] * sh.inv_s[sh.mj[p]];
#pragma unroll
            for (int q = 0; q < kMaxRank; ++q)
              if (q == qq) V[q] += add;
          }
        }
        u_from_w(l, bl, U);
        lu_solve(sh.M, sh.piv, r, V);
        double hll = bl * g.S[(size_t)l * m + l];
#pragma unroll
        for (int q = 0; q < kMaxRank; ++q) hll += U[q] * V[q];
        const double d = 1.0 - hll;
        if (fabs(d) < kTauCont) {
          island = true;
        } else {
          active = true;
          inv_d = 1.0 / d;
        }
      }
    }
    nisl += island;
    const unsigned long long mask = ballot64(active);
    if (lane == 0) s_wcnt[wid] = __popcll(mask);
    __syncthreads();
    int off = s_base;
    for (int q = 0; q < wid; ++q) off += s_wcnt[q];
    off += __popcll(mask & ((1ull << lane) - 1ull));
    if (active) {
      // phi_l(t) = f'_l(t) / (1 - H'_ll), zero for an already opened l
      F* ro = rec + (size_t)off * RS;
#pragma unroll
      for (int t = 0; t < TT; ++t) {
        double ph = 0.0;
        if (t < T && !opened) {
          double fl = g.f0[(size_t)l * T + t];
#pragma unroll
          for (int q = 0; q < kMaxRank; ++q) fl += U[q] * s_x[q][t];
          ph = fl * inv_d;
        }
        ro[t] = (F)ph;
      }
#pragma unroll
      for (int q = 0; q < kVSlots; ++q) ro[TT + q] = (F)V[q];
#pragma unroll
      for (int q = TT + kVSlots; q < RS; ++q) ro[q] = (F)0;
      act[off] = li;
    }
    if (w.slot && li < nC) w.slot[(size_t)c * nC + li] = active ? off : -1;
    __syncthreads();
    if (tid == 0) s_base += s_wcnt[0] + s_wcnt[1] + s_wcnt[2] + s_wcnt[3];
    __syncthreads();
  }
  if (nisl) atomicAdd(&s_nisl, nisl);
  __syncthreads();
  const int n_act = s_base;
  // even length for the paired sweep: duplicate the last record (max unchanged)
  if (n_act & 1) {
    const F* src = rec + (size_t)(n_act - 1) * RS;
    F* dst = rec + (size_t)n_act * RS;
    for (int q = tid; q < RS; q += 256) dst[q] = src[q];
    if (tid == 0) act[n_act] = act[n_act - 1];
  }
  if (tid == 0) {
    inf->status = 0;
    inf->r = r;
    inf->k = k;
    inf->n_act = n_act;
    inf->n_act_pad = n_act + (n_act & 1);
    inf->n_island = s_nisl;
    inf->n_crit_n0 = s_n0;
    for (int q = 0; q < kMaxRank; ++q) inf->open_br[q] = q < k ? sh.open[q] : -1;
  }
}

// ---------------------------------------------------------------------------
// N-1 sweep.  Thread = (candidate, monitored branch), all timesteps in
// registers; contingencies are consumed in pairs so that the running maximum
// takes one 3-input max per two flows.  Contingency records (phi, V) are
// wave-uniform; the H row entries are per lane.
__device__ inline float fabs_t(float v) { return fabsf(v); }
__device__ inline double fabs_t(double v) { return fabs(v); }
__device__ inline float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ inline float max3_t(float a, float b, float c) { return fmaxf(a, fmaxf(b, c)); }
__device__ inline double max3_t(double a, double b, double c) { return fmax(a, fmax(b, c)); }

template <typename F, int TT, int R>
__device__ __forceinline__ void sweep_core(const GridDev& g, const SweepBufs<F>& w,
                                           const F* __restrict__ HMC, int c, int ei_c,
                                           int n_act_pad, F* acc, F* a) {
  constexpr int RS = rec_stride(TT);
  const int nM = g.nM, nC = g.nC;
  F U[R > 0 ? R : 1];
  const F* fa = w.fM + ((size_t)c * nM + ei_c) * TT;
  const F* ua = w.UM + ((size_t)c * nM + ei_c) * kVSlots;
#pragma unroll
  for (int t = 0; t < TT; ++t) { a[t] = fa[t]; acc[t] = (F)0; }
#pragma unroll
  for (int j = 0; j < R; ++j) U[j] = ua[j];
  const F* __restrict__ rec = w.rec + (size_t)c * (nC + 1) * RS;
  const int* __restrict__ act = w.act + (size_t)c * (nC + 1);
  if (n_act_pad == 0) return;
  // software pipeline: the H entries of the next pair are in flight while the
  // current pair is consumed (the last prefetch re-reads an in-range pair)
  F hn0 = HMC[(size_t)act[0] * nM + ei_c];
  F hn1 = HMC[(size_t)act[1] * nM + ei_c];
  for (int i = 0; i < n_act_pad; i += 2) {
    F h0 = hn0, h1 = hn1;
    const int nx = (i + 2 < n_act_pad) ? i + 2 : i;
    hn0 = HMC[(size_t)act[nx] * nM + ei_c];
    hn1 = HMC[(size_t)act[nx + 1] * nM + ei_c];
    const F* r0 = rec + (size_t)i * RS;
    const F* r1 = r0 + RS;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      h0 = fma_t(U[j], r0[TT + j], h0);
      h1 = fma_t(U[j], r1[TT + j], h1);
    }
#pragma unroll
    for (int t = 0; t < TT; ++t) {
      const F g0 = fma_t(h0, r0[t], a[t]);
      const F g1 = fma_t(h1, r1[t], a[t]);
      acc[t] = max3_t(acc[t], fabs_t(g0), fabs_t(g1));
    }
  }
}

#ifndef TTO_SWEEP_WPE
#define TTO_SWEEP_WPE 0
#endif
#if TTO_SWEEP_WPE > 0
#define TTO_SWEEP_ATTR __attribute__((amdgpu_waves_per_eu(TTO_SWEEP_WPE, 8)))
#else
#define TTO_SWEEP_ATTR
#endif

template <typename F, int TT>
__global__ __launch_bounds__(256) TTO_SWEEP_ATTR void k_sweep(GridDev g, SweepBufs<F> w,
                                               const F* __restrict__ HMC,
                                               double* __restrict__ fmax_out) {
  const int c = blockIdx.y;
  const CandInfo* inf = w.info + c;
  const int status = inf->status;
  if (status & (TTO_ST_ISLANDED | TTO_ST_INVALID)) return;
  const int r = inf->r, k = inf->k, n_act_pad = inf->n_act_pad;
  const int nM = g.nM, T = g.T;
  const int ei = blockIdx.x * 256 + threadIdx.x;
  const bool valid = ei < nM;
  const int ei_c = valid ? ei : nM - 1;
  F acc[TT], a[TT];
  switch (r) {
    case 0: sweep_core<F, TT, 0>(g, w, HMC, c, ei_c, n_act_pad, acc, a); break;
    case 1: sweep_core<F, TT, 1>(g, w, HMC, c, ei_c, n_act_pad, acc, a); break;
    case 2: sweep_core<F, TT, 2>(g, w, HMC, c, ei_c, n_act_pad, acc, a); break;
    case 3: sweep_core<F, TT, 3>(g, w, HMC, c, ei_c, n_act_pad, acc, a); break;
    case 4: sweep_core<F, TT, 4>(g, w, HMC, c, ei_c, n_act_pad, acc, a); break;
    case 5: sweep_core<F, TT, 5>(g, w, HMC, c, ei_c, n_act_pad, acc, a); break;
    case 6: sweep_core<F, TT, 6>(g, w, HMC, c, ei_c, n_act_pad, acc, a); break;
    case 7: sweep_core<F, TT, 7>(g, w, HMC, c, ei_c, n_act_pad, acc, a); break;
    default: sweep_core<F, TT, 8>(g, w, HMC, c, ei_c, n_act_pad, acc, a); break;
  }
  // per-thread reduction over timesteps
  const int e = g.mon[ei_c];
  bool opened = false;
  for (int q = 0; q < k; ++q) opened |= (inf->open_br[q] == e);
  double so = 0.0, best = -1.0;
  int cc = 0, bt = 0;
  if (valid) {
    const double lim = g.lim[e];
#pragma unroll
    for (int t = 0; t < TT; ++t) {
      if (t < T) {
        // an opened monitored branch carries no flow in any state
        const double fm = opened ? 0.0 : (double)acc[t];
        if (fmax_out) fmax_out[((size_t)c * nM + ei) * T + t] = fm;
        const double ov = fm - lim;
        if (ov > 0.0) so += ov;
        cc += fm > lim;
        const double ratio = fm / lim;
        if (ratio > best) { best = ratio; bt = t; }
      }
    }
  }
  // deterministic block tree reduction
  __shared__ double s_so[256], s_best[256];
  __shared__ int s_cc[256], s_be[256], s_bt[256];
  const int tid = threadIdx.x;
  s_so[tid] = so; s_best[tid] = best; s_cc[tid] = cc; s_be[tid] = ei; s_bt[tid] = bt;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) {
      s_so[tid] += s_so[tid + st];
      s_cc[tid] += s_cc[tid + st];
      const double b2 = s_best[tid + st];
      if (b2 > s_best[tid]) { s_best[tid] = b2; s_be[tid] = s_be[tid + st]; s_bt[tid] = s_bt[tid + st]; }
    }
    __syncthreads();
  }
  if (tid == 0) {
    Partial p;
    p.sum_o = s_so[0]; p.best = s_best[0]; p.cnt_c = s_cc[0]; p.best_e = s_be[0];
    p.best_t = s_bt[0]; p.pad_ = 0;
    w.part[(size_t)c * w.n_eblk + blockIdx.x] = p;
  }
}

// ---------------------------------------------------------------------------
template <typename F, int TT>
__global__ __launch_bounds__(64) void k_finalize(GridDev g, SweepBufs<F> w,
                                                 const F* __restrict__ HMC, tto_outputs o) {
  constexpr int RS = rec_stride(TT);
  const int c = blockIdx.x;
  const int lane = threadIdx.x;
  const CandInfo inf = w.info[c];
  const int nM = g.nM, nC = g.nC;
  if (inf.status & (TTO_ST_ISLANDED | TTO_ST_INVALID)) {
    if (lane == 0) {
      const double nan = __builtin_nan("");
      if (o.status) o.status[c] = (uint8_t)inf.status;
      if (o.n_island_cont) o.n_island_cont[c] = 0;
      if (o.overload_mw) o.overload_mw[c] = nan;
      if (o.n_crit_n1) o.n_crit_n1[c] = 0;
      if (o.n_crit_n0) o.n_crit_n0[c] = 0;
      if (o.max_loading) o.max_loading[c] = nan;
      if (o.worst_branch) o.worst_branch[c] = -1;
      if (o.worst_cont) o.worst_cont[c] = -1;
      if (o.worst_t) o.worst_t[c] = -1;
      if (o.fitness) o.fitness[c] = -__builtin_inf();
      if (o.cell) o.cell[c] = -1;
    }
    return;
  }
  __shared__ double s_sum, s_best;
  __shared__ int s_cc, s_be, s_bt;
  if (lane == 0) {
    double so = 0.0, best = -1.0;
    int cc = 0, be = -1, bt = 0;
    const Partial* p = w.part + (size_t)c * w.n_eblk;
    for (int b = 0; b < w.n_eblk; ++b) {
      so += p[b].sum_o;
      cc += p[b].cnt_c;
      if (p[b].best > best) { best = p[b].best; be = p[b].best_e; bt = p[b].best_t; }
    }
    s_sum = so; s_best = best; s_cc = cc; s_be = be; s_bt = bt;
  }
  __syncthreads();
  const int be = s_be, bt = s_bt;
  // arg-max contingency at (e*, t*), same arithmetic as the sweep
  double bv = -1.0;
  int bi = INT_MAX;
  bool be_open = false;
  if (be >= 0)
    for (int q = 0; q < inf.k; ++q) be_open |= (inf.open_br[q] == g.mon[be]);
  if (be >= 0 && be_open) {
    // every state gives zero flow on an opened branch: first active contingency
    if (inf.n_act > 0 && lane == 0) { bv = 0.0; bi = 0; }
  } else if (be >= 0) {
    const F a = w.fM[((size_t)c * nM + be) * TT + bt];
    const F* ua = w.UM + ((size_t)c * nM + be) * kVSlots;
    const F* rec = w.rec + (size_t)c * (nC + 1) * RS;
    const int* act = w.act + (size_t)c * (nC + 1);
    for (int i = lane; i < inf.n_act; i += 64) {
      const F* ri = rec + (size_t)i * RS;
      F h = HMC[(size_t)act[i] * nM + be];
      for (int j = 0; j < inf.r; ++j) h = fma_t(ua[j], ri[TT + j], h);
      const double v = (double)fabs_t(fma_t(h, ri[bt], a));
      if (v > bv) { bv = v; bi = i; }
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(bv, off);
    const int oi = __shfl_xor(bi, off);
    if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
  }
  if (lane == 0) {
    const double so = s_sum, best = s_best;
    const int cc = s_cc;
    const int n0 = inf.n_crit_n0;
    const double fit = -(so + g.w_c0 * n0 + g.w_c * cc);
    int bin = 0;
    for (int q = 0; q < g.n_load_bins - 1; ++q) bin += (g.edges[q] <= best) ? 1 : 0;
    const int cnt = inf.r < g.n_count_bins - 1 ? inf.r : g.n_count_bins - 1;
    const int* act = w.act + (size_t)c * (nC + 1);
    if (o.status) o.status[c] = (uint8_t)inf.status;
    if (o.n_island_cont) o.n_island_cont[c] = inf.n_island;
    if (o.overload_mw) o.overload_mw[c] = so;
    if (o.n_crit_n1) o.n_crit_n1[c] = cc;
    if (o.n_crit_n0) o.n_crit_n0[c] = n0;
    if (o.max_loading) o.max_loading[c] = best < 0.0 ? 0.0 : best;
    if (o.worst_branch) o.worst_branch[c] = be >= 0 ? g.mon[be] : -1;
    if (o.worst_t) o.worst_t[c] = be >= 0 ? bt : -1;
    if (o.worst_cont) o.worst_cont[c] = (bi != INT_MAX) ? g.cont[act[bi]] : -1;
    if (o.fitness) o.fitness[c] = fit;
    if (o.cell) o.cell[c] = cnt * g.n_load_bins + bin;
  }
}

// ---------------------------------------------------------------------------
// Full N-1 flow tensor for debugging-sized batches: n1[c][li][ei][t].
template <typename F, int TT>
__global__ __launch_bounds__(256) void k_n1_dump(GridDev g, SweepBufs<F> w,
                                                 const F* __restrict__ HMC,
                                                 double* __restrict__ n1) {
  constexpr int RS = rec_stride(TT);
  const int c = blockIdx.y;
  const int ei = blockIdx.x * 256 + threadIdx.x;
  const int nM = g.nM, nC = g.nC, T = g.T;
  if (ei >= nM) return;
  const CandInfo inf = w.info[c];
  const double nan = __builtin_nan("");
  const bool bad = inf.status & (TTO_ST_ISLANDED | TTO_ST_INVALID);
  const int e = g.mon[ei];
  bool opened = false;
  for (int q = 0; q < inf.k; ++q) opened |= (inf.open_br[q] == e);
  const F* fa = w.fM + ((size_t)c * nM + ei) * TT;
  const F* ua = w.UM + ((size_t)c * nM + ei) * kVSlots;
  const F* rec = w.rec + (size_t)c * (nC + 1) * RS;
  for (int li = 0; li < nC; ++li) {
    double* out = n1 + (((size_t)c * nC + li) * nM + ei) * T;
    const int slot = bad ? -1 : w.slot[(size_t)c * nC + li];
    if (slot < 0) {
      for (int t = 0; t < T; ++t) out[t] = nan;
      continue;
    }
    if (opened || g.cont[li] == e) {
      for (int t = 0; t < T; ++t) out[t] = 0.0;
      continue;
    }
    const F* ri = rec + (size_t)slot * RS;
    F h = HMC[(size_t)li * nM + ei];
    for (int j = 0; j < inf.r; ++j) h = fma_t(ua[j], ri[TT + j], h);
    for (int t = 0; t < T; ++t) out[t] = (double)fma_t(h, ri[t], fa[t]);
  }
}

// ---------------------------------------------------------------------------
// Archive: per-cell best of the batch by an order-free 64-bit atomic max of a
// monotone key, then the lowest index among exact ties, then the strict
// replacement test against the stored elite.
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

static inline int cdiv(int a, int b) { return (a + b - 1) / b; }

hipError_t launch_archive(double* elite_fit, int64_t* elite_id, int n_cells, const double* fit,
                          const int* cell, const uint8_t* status, int B, int64_t id_base,
                          unsigned long long* key, int* idx, hipStream_t s) {
  hipLaunchKernelGGL(k_arch_init, dim3(cdiv(n_cells, 256)), dim3(256), 0, s, key, idx, n_cells);
  if (B > 0) {
    hipLaunchKernelGGL(k_arch_key, dim3(cdiv(B, 256)), dim3(256), 0, s, fit, cell, status, B, n_cells, key);
    hipLaunchKernelGGL(k_arch_idx, dim3(cdiv(B, 256)), dim3(256), 0, s, fit, cell, status, B, n_cells, key, idx);
  }
  hipLaunchKernelGGL(k_arch_apply, dim3(cdiv(n_cells, 256)), dim3(256), 0, s, fit, idx, n_cells, id_base, elite_fit, elite_id);
  return hipGetLastError();
}

template <typename F, int TT>
static hipError_t launch_eval_tt(const GridDev& g, const BatchDev& bt, const SweepBufs<F>& w,
                                 const tto_outputs& o, hipStream_t s, hipEvent_t* ev) {
  const F* HMC;
  if constexpr (sizeof(F) == 4) HMC = g.HMC32; else HMC = g.HMC64;
  if (ev) hipEventRecord(ev[0], s);
  hipLaunchKernelGGL((k_setup<F, TT>), dim3(bt.B), dim3(256), 0, s, g, bt, w, o.base_flows);
  if (ev) hipEventRecord(ev[1], s);
  hipLaunchKernelGGL((k_sweep<F, TT>), dim3(w.n_eblk, bt.B), dim3(256), 0, s, g, w, HMC, o.fmax);
  if (ev) hipEventRecord(ev[2], s);
  hipLaunchKernelGGL((k_finalize<F, TT>), dim3(bt.B), dim3(64), 0, s, g, w, HMC, o);
  if (ev) hipEventRecord(ev[3], s);
  if (o.n1_flows)
    hipLaunchKernelGGL((k_n1_dump<F, TT>), dim3(w.n_eblk, bt.B), dim3(256), 0, s, g, w, HMC, o.n1_flows);
  return hipGetLastError();
}

template <typename F>
hipError_t launch_evaluate(const GridDev& g, const BatchDev& bt, const SweepBufs<F>& w,
                           const tto_outputs& o, hipStream_t s, hipEvent_t* ev) {
  switch (g.TT) {
    case 1: return launch_eval_tt<F, 1>(g, bt, w, o, s, ev);
    case 8: return launch_eval_tt<F, 8>(g, bt, w, o, s, ev);
    case 24: return launch_eval_tt<F, 24>(g, bt, w, o, s, ev);
    default: return launch_eval_tt<F, 32>(g, bt, w, o, s, ev);
  }
}

template hipError_t launch_evaluate<float>(const GridDev&, const BatchDev&, const SweepBufs<float>&,
                                           const tto_outputs&, hipStream_t, hipEvent_t*);
template hipError_t launch_evaluate<double>(const GridDev&, const BatchDev&, const SweepBufs<double>&,
                                            const tto_outputs&, hipStream_t, hipEvent_t*);

}  // namespace tto
