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
//   (The repertoire update lives in k_archive.hip.)
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
  // flattened sources of the column gathers: row src_row[s] of S enters
  // column slot q with coefficient coef[s][q] (1 for an opening, sg_b b_b for
  // a moved branch of its split)
  int nsrc;
  int src_row[kMaxRank + kMaxMoved];
  double coef[kMaxRank + kMaxMoved][kMaxRank];
  // staging of the genome slots
  int oval[kMaxRank], sval[kMaxRank], slo[kMaxRank], shi[kMaxRank], stot;
  int mfrom[kMaxMoved], mto[kMaxMoved];
  double mb[kMaxMoved];
};

// Column gather: W[q] = sum_s coef[s][q] tab[src_row[s]][col], i.e. W[q] =
// S[K_q][e] for openings and W[k+j] = sum_{b in S_j} sg_b b_b S[b][e] for
// splits.  Eight independent row loads are in flight per step.
__device__ inline void gather_column(const double* __restrict__ tab, size_t ld, int col,
                                     const SetupShared& sh, double* W) {
#pragma unroll
  for (int q = 0; q < kMaxRank; ++q) W[q] = 0.0;
  const int nsrc = sh.nsrc;
  for (int s0 = 0; s0 < nsrc; s0 += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      v[u] = (s0 + u < nsrc) ? tab[(size_t)sh.src_row[s0 + u] * ld + col] : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (s0 + u < nsrc) {
#pragma unroll
        for (int q = 0; q < kMaxRank; ++q) W[q] = fma(sh.coef[s0 + u][q], v[u], W[q]);
      }
    }
  }
}

template <typename F, int TT>
__global__ __launch_bounds__(256) void k_setup(GridDev g, BatchDev bt, SweepBufs<F> w,
                                               double* __restrict__ base_out) {
  constexpr int RS = rec_stride(TT);
  const int c = blockIdx.x;
  const int tid = threadIdx.x;
  const int m = g.n_branch, T = g.T, nM = g.nM, nC = g.nC;
  // genome index: refinement passes evaluate map[c] for c < live count
  int cb = c;
  if (bt.map) {
    if (c >= min(*bt.live, bt.B)) return;
    cb = bt.map[c];
  }

  __shared__ SetupShared sh;
  __shared__ double s_x[kMaxRank][TT];
  __shared__ int s_wcnt[4];
  __shared__ int s_base, s_n0, s_nisl, s_bad;
  // record staging, one slab per wave (contingency rows); before that the
  // same LDS holds the S entries among the gather sources (bordered matrix)
  __shared__ __align__(16) char s_raw[sizeof(F) * 4 * 64 * 17];
  F (*s_stage)[64][17] = reinterpret_cast<F (*)[64][17]>(s_raw);
  double* s_sub = reinterpret_cast<double*>(s_raw);
  static_assert(sizeof(F) * 4 * 64 * 17 >= sizeof(double) * kSubMax * kSubMax, "LDS reuse");

  // -- genome parse in stages: slot values, ranges, moved-branch data, checks
  if (tid < bt.no) sh.oval[tid] = bt.open[(size_t)cb * bt.no + tid];
  if (tid < bt.ns) {
    sh.sval[tid] = bt.sbus[(size_t)cb * bt.ns + tid];
    sh.slo[tid] = bt.moff[(size_t)cb * bt.ns + tid];
    sh.shi[tid] = bt.moff[(size_t)cb * bt.ns + tid + 1];
  }
  if (tid == 0) sh.stot = bt.ns > 0 ? bt.moff[(size_t)bt.n_genomes * bt.ns] : 0;
  __syncthreads();
  if (tid == 0) {
    int valid = 1, k = 0, s = 0, nm = 0;
    for (int i = 0; i < bt.no; ++i) {
      const int v = sh.oval[i];
      if (v == -1) continue;
      if (v < 0 || v >= m) { valid = 0; continue; }
      for (int q = 0; q < k; ++q) if (sh.open[q] == v) valid = 0;
      if (k >= kMaxRank) { valid = 0; continue; }
      sh.open[k++] = v;
    }
    for (int j = 0; j < bt.ns; ++j) {
      const int bus = sh.sval[j];
      if (bus == -1) continue;
      if (bus < 0 || bus >= g.n_bus || s >= kMaxRank) { valid = 0; continue; }
      for (int q = 0; q < s; ++q) if (sh.sbus[q] == bus) valid = 0;
      const int lo = sh.slo[j], hi = sh.shi[j];
      // CSR sanity: offsets inside [0, total moved] and increasing
      if (lo < 0 || hi > sh.stot || hi <= lo || nm + (hi - lo) > kMaxMoved) { valid = 0; continue; }
      sh.moff[s] = nm;
      sh.slo[s] = lo;     // compacted: raw start of split s
      sh.sbus[s] = bus;
      sh.sslot[s] = j;
      nm += hi - lo;
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
    s_bad = 0;
  }
  __syncthreads();
  {
    const int k0 = sh.hdr[1], ns0 = sh.hdr[2], nm0 = sh.moff[ns0];
    if (sh.hdr[0] && tid < nm0) {
      int s = 0;
      while (s + 1 < ns0 && sh.moff[s + 1] <= tid) ++s;
      const int e = bt.mbr[sh.slo[s] + (tid - sh.moff[s])];
      sh.mbr[tid] = e;
      sh.mj[tid] = s;
      const bool ok = e >= 0 && e < m;
      sh.mfrom[tid] = ok ? g.from[e] : -1;
      sh.mto[tid] = ok ? g.to[e] : -1;
      sh.mb[tid] = ok ? g.b[e] : 0.0;
    }
    if (sh.hdr[0] && tid >= 64 && tid - 64 < k0) sh.bK[tid - 64] = g.b[sh.open[tid - 64]];
  }
  __syncthreads();
  if (tid == 0 && sh.hdr[0]) {
    int valid = 1;
    const int k = sh.hdr[1], ns = sh.hdr[2];
    for (int s = 0; s < ns; ++s) {
      const int bus = sh.sbus[s];
      double ssum = 0.0;
      for (int p = sh.moff[s]; p < sh.moff[s + 1]; ++p) {
        const int e = sh.mbr[p];
        if (e < 0 || e >= m) { valid = 0; continue; }
        if (sh.mfrom[p] != bus && sh.mto[p] != bus) valid = 0;
        for (int q = sh.moff[s]; q < p; ++q) if (sh.mbr[q] == e) valid = 0;
        for (int q = 0; q < k; ++q) if (sh.open[q] == e) valid = 0;
        const double sg = (sh.mfrom[p] == bus) ? 1.0 : -1.0;
        sh.msign[p] = sg;
        sh.msg[p] = sg * sh.mb[p];
        ssum += sh.mb[p];
      }
      sh.inv_s[s] = ssum > 0.0 ? 1.0 / ssum : 0.0;
    }
    // flattened gather sources
    int ns_ = 0;
    for (int q = 0; q < k; ++q) {
      sh.src_row[ns_] = sh.open[q];
      for (int qq = 0; qq < kMaxRank; ++qq) sh.coef[ns_][qq] = (qq == q) ? 1.0 : 0.0;
      ++ns_;
    }
    for (int p = 0; p < sh.moff[ns]; ++p) {
      sh.src_row[ns_] = sh.mbr[p] >= 0 && sh.mbr[p] < m ? sh.mbr[p] : 0;
      const int slot = k + sh.mj[p];
      for (int qq = 0; qq < kMaxRank; ++qq) sh.coef[ns_][qq] = (qq == slot) ? sh.msg[p] : 0.0;
      ++ns_;
    }
    sh.nsrc = ns_;
    sh.hdr[0] = valid;
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

  // S entries among the gather sources (openings, then moved branches), one
  // load per thread, so that the bordered matrix is built from LDS; more
  // than kSubMax sources read S directly
  const int nsrc = sh.nsrc;
  const bool sub = nsrc <= kSubMax;
  if (sub)
    for (int i = tid; i < nsrc * nsrc; i += 256) {
      const int a = i / nsrc, a2 = i - (i / nsrc) * nsrc;
      s_sub[i] = g.S[(size_t)sh.src_row[a] * m + sh.src_row[a2]];
    }
  __syncthreads();
  // S between sources a and a2 (a < k: opening a; a >= k: moved branch a - k)
  auto Sv = [&](int a, int a2) -> double {
    return sub ? s_sub[a * nsrc + a2] : g.S[(size_t)sh.src_row[a] * m + sh.src_row[a2]];
  };

  // bordered matrix M_c, one entry per thread; H_ab = b_a S_ab
  if (tid < r * r) {
    const int i = tid / r, q = tid - (tid / r) * r;
    double v = 0.0;
    if (i < k) {
      if (q < k) {
        v = (i == q ? 1.0 : 0.0) - sh.bK[i] * Sv(i, q);
      } else {
        const int j = q - k;
        for (int p = sh.moff[j]; p < sh.moff[j + 1]; ++p) v += sh.msg[p] * Sv(i, k + p);
        v *= sh.bK[i];
      }
    } else {
      const int j = i - k;
      if (q < k) {
        for (int p = sh.moff[j]; p < sh.moff[j + 1]; ++p) v += sh.msg[p] * Sv(k + p, q);
      } else {
        const int j2 = q - k;
        for (int p = sh.moff[j]; p < sh.moff[j + 1]; ++p) {
          for (int p2 = sh.moff[j2]; p2 < sh.moff[j2 + 1]; ++p2) {
            v -= sh.msg[p] * sh.msg[p2] * Sv(k + p, k + p2);
            if (sh.mbr[p] == sh.mbr[p2]) v += sh.msign[p] * sh.msign[p2] * sh.mb[p];
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
      inf->n_moved = sh.moff[ns];
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
          const double pj = bt.mp ? bt.mp[((size_t)cb * bt.ns + sh.sslot[j]) * T + t] : 0.0;
          v = (pj - phi) * sh.inv_s[j];
        }
      }
      x[q] = v;
    }
    if (t < T) lu_solve(sh.M, sh.piv, r, x);
    // a non-finite moved injection reaches x(t) (NaN times 0 stays NaN)
    bool bad = false;
#pragma unroll
    for (int q = 0; q < kMaxRank; ++q) {
      s_x[q][t] = (t < T) ? x[q] : 0.0;
      bad |= (t < T) && !isfinite(x[q]);
    }
    if (bad) atomicAdd(&s_bad, 1);
  }
  __syncthreads();

  const int nm = sh.moff[ns];
  const size_t nMC = (size_t)nM + nC;
  // U row of branch e from its column gather: U_q = b_e W_q (openings),
  // U_{k+j} = -b_e W_{k+j} + sum_{b in S_j, b = e} sg_b b_b (moved-branch term)
  auto u_from_w = [&](int e, double be, const double* W, double* U) {
#pragma unroll
    for (int q = 0; q < kMaxRank; ++q) U[q] = (q < k ? be : -be) * W[q];
    for (int p = 0; p < nm; ++p) {
      if (sh.mbr[p] == e) {
        const int qq = k + sh.mj[p];
#pragma unroll
        for (int q = 0; q < kMaxRank; ++q)
          if (q == qq) U[q] += sh.msg[p];
      }
    }
  };

  // monitored rows: f'_M and U_M.  A non-finite grid injection makes every
  // base flow non-finite (the product with a zero PTDF entry included), so
  // the monitored rows' f0 see it.
  int n0 = 0, nbad = 0;
  for (int ei = tid; ei < nM; ei += 256) {
    keep_in_loop();
    const int e = g.mon[ei];
    bool opened = false;
    for (int q = 0; q < k; ++q) opened |= (sh.open[q] == e);
    // loads that depend on the row alone go out before the column gather,
    // so that their latency overlaps it
    double f0e[TT];
#pragma unroll
    for (int t = 0; t < TT; ++t) f0e[t] = t < T ? g.f0MC[(size_t)t * nMC + ei] : 0.0;
#pragma unroll
    for (int t = 0; t < TT; ++t) nbad += !isfinite(f0e[t]);
    const double be = g.bMC[ei], lim = g.limM[ei];
    double W[kMaxRank], U[kMaxRank];
    gather_column(g.SMC, nMC, ei, sh, W);
    u_from_w(e, be, W, U);
    F* fo = w.fM + (size_t)c * TT * nM + ei;   // [c][t][ei]: coalesced across threads
#pragma unroll
    for (int t = 0; t < TT; ++t) {
      double fp = 0.0;
      if (t < T && !opened) {
        fp = f0e[t];
#pragma unroll
        for (int q = 0; q < kMaxRank; ++q) fp += U[q] * s_x[q][t];
        n0 += fabs(fp) > lim;
      }
      fo[(size_t)t * nM] = (F)fp;
    }
    F* uo = w.UM + (size_t)c * kVSlots * nM + ei;   // [c][q][ei]
#pragma unroll
    for (int q = 0; q < kVSlots; ++q) uo[(size_t)q * nM] = opened ? (F)0 : (F)U[q];
  }
  if (n0) atomicAdd(&s_n0, n0);
  if (nbad) atomicAdd(&s_bad, nbad);

  // optional full post-switch base flows
  if (base_out) {
    for (int e = tid; e < m; e += 256) {
      keep_in_loop();
      bool opened = false;
      for (int q = 0; q < k; ++q) opened |= (sh.open[q] == e);
      double W[kMaxRank], U[kMaxRank];
      gather_column(g.S, (size_t)m, e, sh, W);
      u_from_w(e, g.b[e], W, U);
      for (int t = 0; t < T; ++t) {
        double fp = 0.0;
        if (!opened) {
          fp = g.f0[(size_t)e * T + t];
#pragma unroll
          for (int q = 0; q < kMaxRank; ++q) fp += U[q] * s_x[q][t];
        }
        base_out[((size_t)cb * m + e) * T + t] = fp;
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
    double f0l[TT];
    double s_ll = 0.0, b_l = 0.0;
#pragma unroll
    for (int q = 0; q < kMaxRank; ++q) { V[q] = 0.0; U[q] = 0.0; }
    if (li < nC) {
      l = g.cont[li];
      // row-only loads first (their latency overlaps the column gather)
      s_ll = g.sllC[li];
      b_l = g.bMC[nM + li];
#pragma unroll
      for (int t = 0; t < TT; ++t) f0l[t] = t < T ? g.f0MC[(size_t)t * nMC + nM + li] : 0.0;
      for (int q = 0; q < k; ++q) opened |= (sh.open[q] == l);
      if (opened) {
        active = true;  // already open: the N-0 state (phi = 0)
      } else {
        double W[kMaxRank];
        gather_column(g.SMC, nMC, nM + li, sh, W);
        const double bl = b_l;
        // right-hand side of the factor column: R_q = b_{K_q} W_q (openings),
        // R_{k+j} = (ps_j - W_{k+j}) / s_j with ps_j = sg_l if l is moved by j
#pragma unroll
        for (int q = 0; q < kMaxRank; ++q) {
          double v = 0.0;
          if (q < k) v = sh.bK[q] * W[q];
          else if (q < r) v = -W[q] * sh.inv_s[q - k];
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
        u_from_w(l, bl, W, U);
        lu_solve(sh.M, sh.piv, r, V);
        double hll = bl * s_ll;
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
    int o0 = s_base;
    for (int q = 0; q < wid; ++q) o0 += s_wcnt[q];
    const int rank = __popcll(mask & ((1ull << lane) - 1ull));
    const int na = __popcll(mask);
    const int off = o0 + rank;
    // Records go out through LDS in 16-entry passes so that every store
    // instruction writes whole contiguous runs (direct per-thread 128-byte
    // records leave partially written lines thrashing the L2).
#pragma unroll
    for (int p0 = 0; p0 < RS; p0 += 16) {
      if (active) {
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int slot = p0 + u;
          if (slot < RS) {
            double v = 0.0;
            if (slot < TT) {
              // phi_l(t) = f'_l(t) / (1 - H'_ll), zero for an already opened l
              if (slot < T && !opened) {
                double fl = f0l[slot];
#pragma unroll
                for (int q = 0; q < kMaxRank; ++q) fl += U[q] * s_x[q][slot];
                v = fl * inv_d;
              }
            } else if (slot < TT + kVSlots) {
              v = V[slot - TT];
            }
            s_stage[wid][rank][u] = (F)v;
          }
        }
      }
      __syncthreads();
      const int nsl = (RS - p0) < 16 ? (RS - p0) : 16;
      for (int idx = lane; idx < na * 16; idx += 64) {
        const int i = idx >> 4, u = idx & 15;
        if (u < nsl) rec[(size_t)(o0 + i) * RS + p0 + u] = s_stage[wid][i][u];
      }
      __syncthreads();
    }
    if (active) act[off] = li;
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
  if (tid == 0 && s_bad) {
    // non-finite injections: no metric is defined, the candidate is skipped
    inf->status = TTO_ST_INVALID | TTO_ST_NONFINITE;
    inf->r = r; inf->k = k; inf->n_act = 0; inf->n_act_pad = 0; inf->n_island = 0;
    inf->n_moved = sh.moff[ns];
    inf->n_crit_n0 = 0;
  } else if (tid == 0) {
    inf->status = 0;
    inf->r = r;
    inf->k = k;
    inf->n_act = n_act;
    inf->n_act_pad = n_act + (n_act & 1);
    inf->n_island = s_nisl;
    inf->n_crit_n0 = s_n0;
    inf->n_moved = sh.moff[ns];
    for (int q = 0; q < kMaxRank; ++q) inf->open_br[q] = q < k ? sh.open[q] : -1;
  }
}

// ---------------------------------------------------------------------------
// N-1 sweep.  The unit of work is one wave: a candidate and NP consecutive
// chunks of 64 monitored branches (one lane per branch of each chunk, NP = 1
// or 2 branches per lane), all timesteps in registers.  Contingencies are
// consumed in pairs, so that the running maximum takes one 3-input max per
// two flows.  The contingency records (phi_l(t), V_l) are wave-uniform
// scalar loads, each feeding NP branches per lane; the H[M, C] entries are
// per lane.  Waves share nothing (no LDS, no barrier): a workgroup is a
// group of independent waves.
__device__ inline float fabs_t(float v) { return fabsf(v); }
__device__ inline double fabs_t(double v) { return fabs(v); }
__device__ inline float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ inline float max3_t(float a, float b, float c) { return fmaxf(a, fmaxf(b, c)); }
__device__ inline double max3_t(double a, double b, double c) { return fmax(a, fmax(b, c)); }

// Contingency pairs [i0, i1) of candidate c for the lanes' monitored
// positions ei[p] (p < NP, clamped into range): acc[p][t] = max |f^(l)|.
template <typename F, int TT, int R, int NP>
__device__ __forceinline__ void sweep_core(const GridDev& g, const SweepBufs<F>& w,
                                           const F* __restrict__ HMC, int c, const int* ei,
                                           int i0, int i1, F (*acc)[TT]) {
  constexpr int RS = rec_stride(TT);
  const int nM = g.nM, nC = g.nC;
  F U[NP][R > 0 ? R : 1], a[NP][TT];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const F* fa = w.fM + (size_t)c * TT * nM + ei[p];
    const F* ua = w.UM + (size_t)c * kVSlots * nM + ei[p];
#pragma unroll
    for (int t = 0; t < TT; ++t) { a[p][t] = fa[(size_t)t * nM]; acc[p][t] = (F)0; }
#pragma unroll
    for (int j = 0; j < R; ++j) U[p][j] = ua[(size_t)j * nM];
  }
  const F* __restrict__ rec = w.rec + (size_t)c * (nC + 1) * RS;
  const int* __restrict__ act = w.act + (size_t)c * (nC + 1);
  if (i1 <= i0) return;
  // Software pipeline: the H entries of the next pair are in flight while the
  // current pair is consumed (the last prefetch re-reads an in-range pair).
  F hn0[NP], hn1[NP];
  {
    const size_t c0 = (size_t)act[i0] * nM, c1 = (size_t)act[i0 + 1] * nM;
#pragma unroll
    for (int p = 0; p < NP; ++p) { hn0[p] = HMC[c0 + ei[p]]; hn1[p] = HMC[c1 + ei[p]]; }
  }
  for (int i = i0; i < i1; i += 2) {
    F h0[NP], h1[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) { h0[p] = hn0[p]; h1[p] = hn1[p]; }
    const int nx = (i + 2 < i1) ? i + 2 : i;
    {
      const size_t c0 = (size_t)act[nx] * nM, c1 = (size_t)act[nx + 1] * nM;
#pragma unroll
      for (int p = 0; p < NP; ++p) { hn0[p] = HMC[c0 + ei[p]]; hn1[p] = HMC[c1 + ei[p]]; }
    }
    const F* r0 = rec + (size_t)i * RS;
    const F* r1 = r0 + RS;
#pragma unroll
    for (int j = 0; j < R; ++j) {
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        h0[p] = fma_t(U[p][j], r0[TT + j], h0[p]);
        h1[p] = fma_t(U[p][j], r1[TT + j], h1[p]);
      }
    }
#pragma unroll
    for (int t = 0; t < TT; ++t) {
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const F g0 = fma_t(h0[p], r0[t], a[p][t]);
        const F g1 = fma_t(h1[p], r1[t], a[p][t]);
        acc[p][t] = max3_t(acc[p][t], fabs_t(g0), fabs_t(g1));
      }
    }
  }
}

// Rank dispatch: the rank-r factor is a compile-time loop bound.
template <typename F, int TT, int NP>
__device__ __forceinline__ void sweep_rank(const GridDev& g, const SweepBufs<F>& w,
                                           const F* __restrict__ HMC, int c, int r,
                                           const int* ei, int i0, int i1, F (*acc)[TT]) {
  switch (r) {
    case 0: sweep_core<F, TT, 0, NP>(g, w, HMC, c, ei, i0, i1, acc); break;
    case 1: sweep_core<F, TT, 1, NP>(g, w, HMC, c, ei, i0, i1, acc); break;
    case 2: sweep_core<F, TT, 2, NP>(g, w, HMC, c, ei, i0, i1, acc); break;
    case 3: sweep_core<F, TT, 3, NP>(g, w, HMC, c, ei, i0, i1, acc); break;
    case 4: sweep_core<F, TT, 4, NP>(g, w, HMC, c, ei, i0, i1, acc); break;
    case 5: sweep_core<F, TT, 5, NP>(g, w, HMC, c, ei, i0, i1, acc); break;
    case 6: sweep_core<F, TT, 6, NP>(g, w, HMC, c, ei, i0, i1, acc); break;
    case 7: sweep_core<F, TT, 7, NP>(g, w, HMC, c, ei, i0, i1, acc); break;
    default: sweep_core<F, TT, 8, NP>(g, w, HMC, c, ei, i0, i1, acc); break;
  }
}

// Reduction of one 64-branch chunk of candidate c: f^max out (optional),
// then over timesteps and lanes the chunk's overload sum, critical count,
// top-2 loading and arg-max, written to part[c][chunk] by lane 0.  The wave
// butterfly is fixed and the finalize kernel adds the chunks in increasing
// order, so every launch shape gives bitwise the same outputs.
template <typename F, int TT>
__device__ __forceinline__ void chunk_epilogue(const GridDev& g, const SweepBufs<F>& w,
                                               double* __restrict__ fmax_out, int c, int chunk,
                                               int oc, const F* acc) {
  const CandInfo* inf = w.info + c;
  const int k = inf->k;
  const int nM = g.nM, T = g.T;
  const int lane = threadIdx.x & 63;
  const int ei = chunk * 64 + lane;
  const bool valid = ei < nM;
  const int ei_c = valid ? ei : nM - 1;
  const int e = g.mon[ei_c];
  bool opened = false;
  for (int q = 0; q < k; ++q) opened |= (inf->open_br[q] == e);
  double so = 0.0, best = -1.0, best2 = -1.0;
  int bt = 0, be = 0;
  int cc = 0;
  if (valid) {
    const double lim = g.lim[e];
#pragma unroll
    for (int t = 0; t < TT; ++t) {
      if (t < T) {
        // an opened monitored branch carries no flow in any state
        const double fm = opened ? 0.0 : (double)acc[t];
        if (fmax_out) fmax_out[((size_t)oc * nM + ei) * T + t] = fm;
        const double ov = fm - lim;
        if (ov > 0.0) so += ov;
        cc += fm > lim;
        const double ratio = fm / lim;
        if (ratio > best) { best2 = best; best = ratio; }
        else if (ratio > best2) best2 = ratio;
      }
    }
  }
  // deterministic wave butterfly (every lane ends with the same values);
  // best2 tracks the runner-up loading for the near-tie test of the FP32 pass
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    so += __shfl_xor(so, off);
    cc += __shfl_xor(cc, off);
    const double b2 = __shfl_xor(best, off), s2 = __shfl_xor(best2, off);
    const double lo = fmin(best, b2);
    best2 = fmax(fmax(best2, s2), lo);
    best = fmax(best, b2);
  }
  // arg-max with the loading tie band: the smallest (e, t) of the chunk whose
  // loading is at least best (1 - TTO_LOAD_TIE_REL); the ratios are recomputed
  // by the same operations as above, so they are bitwise the same
  const double thr = best * (1.0 - kLoadTieRel);
  int key = INT_MAX;
  if (valid) {
    const double lim = g.lim[e];
#pragma unroll
    for (int t = TT - 1; t >= 0; --t) {
      if (t < T) {
        const double fm = opened ? 0.0 : (double)acc[t];
        if (fm / lim >= thr) key = ei * TT + t;
      }
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) key = min(key, __shfl_xor(key, off));
  be = key / TT;
  bt = key - be * TT;
  if (lane == 0) {
    Partial p;
    p.sum_o = so; p.best = best; p.best2 = best2; p.cnt_c = cc; p.best_e = be; p.best_t = bt;
    p.pad_ = 0;
    w.part[(size_t)c * w.n_eblk + chunk] = p;
  }
}

// One wave: candidate c, chunks [wb * NPL, wb * NPL + NPL) clipped to the
// monitored set (a candidate's last wave may hold one chunk only).
template <typename F, int TT, int NPL>
__device__ __forceinline__ void sweep_wave(const GridDev& g, const SweepBufs<F>& w,
                                           const F* __restrict__ HMC,
                                           double* __restrict__ fmax_out, int c, int wb, int oc) {
  // stated wave-uniform: the per-candidate pointers stay in scalar registers
  // and the contingency loop stays a scalar loop (records through the scalar
  // cache)
  c = __builtin_amdgcn_readfirstlane(c);
  wb = __builtin_amdgcn_readfirstlane(wb);
  oc = __builtin_amdgcn_readfirstlane(oc);
  const CandInfo* inf = w.info + c;
  if (inf->status & (TTO_ST_ISLANDED | TTO_ST_INVALID)) return;   // uniform per wave
  const int r = __builtin_amdgcn_readfirstlane(inf->r);
  const int n_pairs = __builtin_amdgcn_readfirstlane(inf->n_act_pad);
  const int nM = g.nM;
  const int lane = threadIdx.x & 63;
  const int ch0 = wb * NPL;
  const int np = min(NPL, w.n_eblk - ch0);
  int ei[NPL];
#pragma unroll
  for (int p = 0; p < NPL; ++p) ei[p] = min((ch0 + p) * 64 + lane, nM - 1);
  F acc[NPL][TT];
  if (NPL == 2 && np == 2) {
    sweep_rank<F, TT, NPL>(g, w, HMC, c, r, ei, 0, n_pairs, acc);
    chunk_epilogue<F, TT>(g, w, fmax_out, c, ch0, oc, acc[0]);
    chunk_epilogue<F, TT>(g, w, fmax_out, c, ch0 + 1, oc, acc[NPL - 1]);
  } else {
    sweep_rank<F, TT, 1>(g, w, HMC, c, r, ei, 0, n_pairs, acc);
    chunk_epilogue<F, TT>(g, w, fmax_out, c, ch0, oc, acc[0]);
  }
}

// Work item u of a sweep: (candidate, wave block) in the plan's order.
__device__ __forceinline__ void sweep_item(int u, int nc, int n_wb, int order, int* c, int* wb) {
  if (order == 2) { *wb = u / nc; *c = u - *wb * nc; }
  else { *c = u / n_wb; *wb = u - *c * n_wb; }
}

// One wave per work item.  Workgroups are dealt to the 8 XCDs round-robin;
// order != 0 remaps workgroup q so that each XCD takes a contiguous range of
// the item order: order 1 candidate-major (the waves of a candidate share its
// records in one L2), order 2 block-major (an XCD streams few column blocks
// of H[M, C] for many candidates).  The grid is a multiple of 8.
template <typename F, int TT, int NPL>
__global__ __launch_bounds__(256) void k_sweep(GridDev g, SweepBufs<F> w,
                                               const F* __restrict__ HMC,
                                               double* __restrict__ fmax_out, int n_cand,
                                               int order, const int* __restrict__ map,
                                               const int* __restrict__ live) {
  int nc = n_cand;
  if (live) nc = min(*live, n_cand);
  const int n_wb = (w.n_eblk + NPL - 1) / NPL;
  const int wpg = (int)(blockDim.x >> 6);
  int q = blockIdx.x;
  if (order) q = (q & 7) * (int)(gridDim.x >> 3) + (q >> 3);
  const int u = q * wpg + (int)(threadIdx.x >> 6);
  if (u >= nc * n_wb) return;   // uniform per wave
  int c, wb;
  sweep_item(u, nc, n_wb, order, &c, &wb);
  sweep_wave<F, TT, NPL>(g, w, HMC, fmax_out, c, wb, map ? map[c] : c);
}

// ---------------------------------------------------------------------------
// Finalize one candidate per wave.  Main pass: outputs at index c.  FP64
// refinement pass (map != NULL): workgroup c < min(*live, cap) finalizes
// candidate map[c] and marks it REFINED.  With rc.list set (FP32 main pass),
// candidates whose discrete outputs lie within the flow error margin of a
// decision (a load-bin edge, a runner-up (e, t) loading, a runner-up
// contingency at (e*, t*)) are queued for the FP64 pass.
// Dynamic LDS of k_finalize: one flow per active contingency when it fits in
// 32 KB (else the second pass recomputes the flows).
template <typename F>
static inline size_t finalize_lds_bytes(int nC) {
  const size_t b = sizeof(F) * ((size_t)nC + 1);
  return b <= 32768 ? b : 0;
}

template <typename F, int TT>
__global__ __launch_bounds__(64) void k_finalize(GridDev g, SweepBufs<F> w,
                                                 const F* __restrict__ HMC, tto_outputs o,
                                                 const int* __restrict__ map,
                                                 const int* __restrict__ live, int cap,
                                                 RefineCtl rc, int cache_flows) {
  // cache_flows: the launch provides (nC + 1) F of dynamic LDS for the flows
  // of the worst-contingency passes
  extern __shared__ unsigned char fin_lds[];
  constexpr int RS = rec_stride(TT);
  const int c = blockIdx.x;
  if (map && c >= min(*live, cap)) return;
  const int oc = map ? map[c] : c;
  const int lane = threadIdx.x;
  const CandInfo inf = w.info[c];
  const int nM = g.nM, nC = g.nC;
  const uint8_t refined = map ? (uint8_t)TTO_ST_REFINED : (uint8_t)0;
  if (inf.status & (TTO_ST_ISLANDED | TTO_ST_INVALID)) {
    if (lane == 0) {
      const double nan = __builtin_nan("");
      if (rc.flags) rc.flags[c] = 0;
      if (o.status) o.status[oc] = (uint8_t)inf.status | refined;
      if (o.n_island_cont) o.n_island_cont[oc] = 0;
      if (o.overload_mw) o.overload_mw[oc] = nan;
      if (o.n_crit_n1) o.n_crit_n1[oc] = 0;
      if (o.n_crit_n0) o.n_crit_n0[oc] = 0;
      if (o.max_loading) o.max_loading[oc] = nan;
      if (o.worst_branch) o.worst_branch[oc] = -1;
      if (o.worst_cont) o.worst_cont[oc] = -1;
      if (o.worst_t) o.worst_t[oc] = -1;
      if (o.fitness) o.fitness[oc] = -__builtin_inf();
      if (o.cell) o.cell[oc] = -1;
    }
    return;
  }
  __shared__ double s_sum, s_best, s_best2;
  __shared__ int s_cc, s_be, s_bt;
  if (lane == 0) {
    double so = 0.0, best = -1.0, best2 = -1.0;
    int cc = 0, be = -1, bt = 0;
    const Partial* p = w.part + (size_t)c * w.n_eblk;
    for (int b = 0; b < w.n_eblk; ++b) {
      so += p[b].sum_o;
      cc += p[b].cnt_c;
      best2 = fmax(fmax(best2, p[b].best2), fmin(best, p[b].best));
      best = fmax(best, p[b].best);
    }
    // (e*, t*): the smallest (e, t) whose loading is within the tie band of
    // rho; chunks hold increasing monitored positions, so the first chunk
    // reaching the band holds it
    const double thr = best * (1.0 - kLoadTieRel);
    for (int b = 0; b < w.n_eblk; ++b) {
      if (p[b].best >= thr) { be = p[b].best_e; bt = p[b].best_t; break; }
    }
    s_sum = so; s_best = best; s_best2 = best2; s_cc = cc; s_be = be; s_bt = bt;
  }
  __syncthreads();
  const int be = s_be, bt = s_bt;
  // worst contingency at (e*, t*), same arithmetic as the sweep: the first
  // active contingency (C order) whose |flow| is within the tie tolerance of
  // the maximum.  Pass 1 finds the maximum, pass 2 the first index above the
  // cut and whether any flow sits within the decision margin of the cut.
  const double mg = decision_margin(g);
  double bv = -1.0;
  int bi = INT_MAX;
  bool band = false;
  bool be_open = false;
  if (be >= 0)
    for (int q = 0; q < inf.k; ++q) be_open |= (inf.open_br[q] == g.mon[be]);
  if (be >= 0 && be_open) {
    // every state gives zero flow on an opened branch: first active contingency
    if (inf.n_act > 0 && lane == 0) { bv = 0.0; bi = 0; }
  } else if (be >= 0) {
    const F a = w.fM[((size_t)c * TT + bt) * nM + be];
    const F* ua = w.UM + (size_t)c * kVSlots * nM + be;
    const F* rec = w.rec + (size_t)c * (nC + 1) * RS;
    const int* act = w.act + (size_t)c * (nC + 1);
    auto flow = [&](int i) -> double {
      const F* ri = rec + (size_t)i * RS;
      F h = HMC[(size_t)act[i] * nM + be];
      for (int j = 0; j < inf.r; ++j) h = fma_t(ua[(size_t)j * nM], ri[TT + j], h);
      return (double)fabs_t(fma_t(h, ri[bt], a));
    };
    F* vbuf = cache_flows ? (F*)fin_lds : nullptr;   // lane i mod 64 owns entry i
    for (int i = lane; i < inf.n_act; i += 64) {
      const double v = flow(i);
      if (vbuf) vbuf[i] = (F)v;
      bv = fmax(bv, v);
    }
    for (int off = 32; off > 0; off >>= 1) bv = fmax(bv, __shfl_xor(bv, off));
    const double cut = bv - kWorstContTieMW;
    for (int i = lane; i < inf.n_act; i += 64) {
      const double v = vbuf ? (double)vbuf[i] : flow(i);
      if (v >= cut && i < bi) bi = i;
      band |= fabs(v - cut) <= 2.0 * mg;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    bi = min(bi, __shfl_xor(bi, off));
    band |= __shfl_xor((int)band, off) != 0;
  }
  if (lane == 0) {
    const double so = s_sum, best = s_best;
    const int cc = s_cc;
    const int n0 = inf.n_crit_n0;
    const double fit = -(so + g.w_c0 * n0 + g.w_c * cc);
    int bin = 0;
    for (int q = 0; q < g.n_load_bins - 1; ++q) bin += (g.edges[q] <= best) ? 1 : 0;
    const int cnt = inf.r < g.n_count_bins - 1 ? inf.r : g.n_count_bins - 1;
    int cell = cnt * g.n_load_bins + bin;
    if (g.desc_kind == TTO_DESC_PAPER) {
      // (disconnections, splits, reassigned assets) clamped to 0..2, 0..3, 0..45
      const int ld = min(inf.k, 2), ls = min(inf.r - inf.k, 3), lr = min(inf.n_moved, 45);
      cell = ld + 3 * (ls + 4 * lr);
    }
    const int* act = w.act + (size_t)c * (nC + 1);
    uint8_t st = (uint8_t)inf.status | refined;
    if (rc.flags) {
      int near = 0;
      if (be >= 0) {
        const double lim_e = g.lim[g.mon[be]];
        near = (best - s_best2) * g.lim_min <= mg;                     // runner-up (e, t)
        near |= band;                                                  // worst-contingency cut
        if (g.desc_kind == TTO_DESC_COUNT_LOAD)
          for (int q = 0; q < g.n_load_bins - 1; ++q)                  // load-bin edge
            near |= fabs(best - g.edges[q]) * lim_e <= mg;
      }
      rc.flags[c] = near;
    }
    if (o.status) o.status[oc] = st;
    if (o.n_island_cont) o.n_island_cont[oc] = inf.n_island;
    if (o.overload_mw) o.overload_mw[oc] = so;
    if (o.n_crit_n1) o.n_crit_n1[oc] = cc;
    if (o.n_crit_n0) o.n_crit_n0[oc] = n0;
    if (o.max_loading) o.max_loading[oc] = best < 0.0 ? 0.0 : best;
    if (o.worst_branch) o.worst_branch[oc] = be >= 0 ? g.mon[be] : -1;
    if (o.worst_t) o.worst_t[oc] = be >= 0 ? bt : -1;
    if (o.worst_cont) o.worst_cont[oc] = (bi != INT_MAX) ? g.cont[act[bi]] : -1;
    if (o.fitness) o.fitness[oc] = fit;
    if (o.cell) o.cell[oc] = cell;
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
  const F* fa = w.fM + (size_t)c * TT * nM + ei;
  const F* ua = w.UM + (size_t)c * kVSlots * nM + ei;
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
    for (int j = 0; j < inf.r; ++j) h = fma_t(ua[(size_t)j * nM], ri[TT + j], h);
    for (int t = 0; t < T; ++t) out[t] = (double)fma_t(h, ri[t], fa[(size_t)t * nM]);
  }
}

// ---------------------------------------------------------------------------
// FP64 refinement sweep, split over contingency ranges so that a handful of
// queued candidates still fill the machine: wave (candidate, 64-branch chunk,
// range s of S) merges the f^max of its range into fbuf by an atomic max on
// the bit patterns (the values are >= 0, so the integer order is the numeric
// order: order-free and exact); k_sweep_split_epi then runs the chunk
// epilogue on the merged maxima.
__global__ __launch_bounds__(256) void k_zero_live_u64(unsigned long long* __restrict__ p,
                                                       const int* __restrict__ live, int cap,
                                                       size_t per) {
  const size_t n = (size_t)min(*live, cap) * per;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    p[i] = 0ull;
}

template <int TT>
__global__ __launch_bounds__(256) void k_sweep_split(GridDev g, SweepBufs<double> w,
                                                     const double* __restrict__ HMC, int n_cand,
                                                     int S, const int* __restrict__ live,
                                                     unsigned long long* __restrict__ fbuf) {
  const int nc = min(*live, n_cand);
  int u = blockIdx.x * 4 + (int)(threadIdx.x >> 6);   // one wave per (range, chunk, candidate)
  if (u >= nc * w.n_eblk * S) return;
  const int sr = __builtin_amdgcn_readfirstlane(u % S);
  u /= S;
  const int c = __builtin_amdgcn_readfirstlane(u / w.n_eblk);
  const int chunk = __builtin_amdgcn_readfirstlane(u - c * w.n_eblk);
  const CandInfo* inf = w.info + c;
  if (inf->status & (TTO_ST_ISLANDED | TTO_ST_INVALID)) return;
  const int r = inf->r, n_act_pad = inf->n_act_pad, nM = g.nM;
  const int per = ((n_act_pad >> 1) + S - 1) / S;       // pairs per range
  const int i0 = __builtin_amdgcn_readfirstlane(2 * sr * per);
  const int i1 = __builtin_amdgcn_readfirstlane(min(n_act_pad, 2 * (sr + 1) * per));
  const int ei = chunk * 64 + (int)(threadIdx.x & 63);
  const bool valid = ei < nM;
  const int ei_c[1] = {valid ? ei : nM - 1};
  double acc[1][TT];
  sweep_rank<double, TT, 1>(g, w, HMC, c, r, ei_c, i0, i1, acc);
  if (valid && i0 < i1) {
    unsigned long long* out = fbuf + (size_t)c * TT * nM + ei;
#pragma unroll
    for (int t = 0; t < TT; ++t)
      atomicMax(out + (size_t)t * nM, (unsigned long long)__double_as_longlong(acc[0][t]));
  }
}

template <int TT>
__global__ __launch_bounds__(256) void k_sweep_split_epi(GridDev g, SweepBufs<double> w,
                                                         double* __restrict__ fmax_out,
                                                         int n_cand, const int* __restrict__ map,
                                                         const int* __restrict__ live,
                                                         const unsigned long long* __restrict__ fbuf) {
  const int nc = min(*live, n_cand);
  const int u = blockIdx.x * 4 + (int)(threadIdx.x >> 6);   // one wave per (candidate, chunk)
  if (u >= nc * w.n_eblk) return;
  const int c = __builtin_amdgcn_readfirstlane(u / w.n_eblk);
  const int chunk = __builtin_amdgcn_readfirstlane(u - c * w.n_eblk);
  const int oc = __builtin_amdgcn_readfirstlane(map[c]);
  if (w.info[c].status & (TTO_ST_ISLANDED | TTO_ST_INVALID)) return;
  const int nM = g.nM;
  const int ei_c = min(chunk * 64 + (int)(threadIdx.x & 63), nM - 1);
  const unsigned long long* in = fbuf + (size_t)c * TT * nM + ei_c;
  double acc[TT];
#pragma unroll
  for (int t = 0; t < TT; ++t) acc[t] = __longlong_as_double((long long)in[(size_t)t * nM]);
  chunk_epilogue<double, TT>(g, w, fmax_out, c, chunk, oc, acc);
}

// Sweep launch for a plan: 256-lane workgroups of four independent waves,
// 1 or 2 monitored branches per lane, and the item order.
template <typename F, int TT, int NPL>
static void launch_sweep_npl(const GridDev& g, const BatchDev& bt, const SweepBufs<F>& w,
                             const F* HMC, double* fmax_out, hipStream_t s, const SweepPlan& plan) {
  const int wpg = plan.lanes / 64;
  const long n_items = (long)bt.B * ((w.n_eblk + NPL - 1) / NPL);
  const long groups = (n_items + wpg - 1) / wpg;
  hipLaunchKernelGGL((k_sweep<F, TT, NPL>), dim3((unsigned)((groups + 7) / 8 * 8)),
                     dim3(plan.lanes), 0, s, g, w, HMC, fmax_out, bt.B, plan.order, bt.map,
                     bt.live);
}

template <typename F, int TT>
static void launch_sweep(const GridDev& g, const BatchDev& bt, const SweepBufs<F>& w,
                         const F* HMC, double* fmax_out, hipStream_t s, const SweepPlan& plan) {
  if constexpr (sizeof(F) == 4) {
    if (plan.npl == 2) { launch_sweep_npl<F, TT, 2>(g, bt, w, HMC, fmax_out, s, plan); return; }
  }
  launch_sweep_npl<F, TT, 1>(g, bt, w, HMC, fmax_out, s, plan);
}

// Refinement queue: the flagged candidates in index order, the first `cap`
// of them queued for the FP64 pass, the rest marked REFINE_SKIPPED; one
// workgroup, ordered scan, so the choice does not depend on scheduling.
__global__ __launch_bounds__(1024) void k_refine_queue(const int* __restrict__ flags, int B,
                                                       int cap, int* __restrict__ list,
                                                       int* __restrict__ count,
                                                       uint8_t* __restrict__ status) {
  __shared__ int s_w[16];
  __shared__ int s_base;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  if (tid == 0) s_base = 0;
  __syncthreads();
  for (int i0 = 0; i0 < B; i0 += 1024) {
    const int i = i0 + tid;
    const bool f = i < B && flags[i] != 0;
    const unsigned long long m = __ballot(f);
    if (lane == 0) s_w[wid] = __popcll(m);
    __syncthreads();
    int pos = s_base;
    for (int q = 0; q < wid; ++q) pos += s_w[q];
    pos += __popcll(m & ((1ull << lane) - 1ull));
    if (f) {
      if (pos < cap) list[pos] = i;
      else if (status) status[i] |= (uint8_t)TTO_ST_REFINE_SKIPPED;
    }
    __syncthreads();
    if (tid == 0) {
      int t = 0;
      for (int q = 0; q < 16; ++q) t += s_w[q];
      s_base += t;
    }
    __syncthreads();
  }
  if (tid == 0) *count = s_base;
}

template <typename F, int TT>
static void launch_pass(const GridDev& g, const BatchDev& bt, SweepBufs<F> w,
                        const tto_outputs& o, hipStream_t s, hipEvent_t* ev,
                        const SweepPlan& plan, const RefineCtl& rc) {
  const F* HMC;
  if constexpr (sizeof(F) == 4) HMC = g.HMC32; else HMC = g.HMC64;
  w.n_eblk = (g.nM + 63) / 64;   // partials per candidate: one per 64-branch chunk
  if (ev) hipEventRecord(ev[0], s);
  hipLaunchKernelGGL((k_setup<F, TT>), dim3(bt.B), dim3(256), 0, s, g, bt, w, o.base_flows);
  if (ev) hipEventRecord(ev[1], s);
  launch_sweep<F, TT>(g, bt, w, HMC, o.fmax, s, plan);
  if (ev) hipEventRecord(ev[2], s);
  const size_t fin_lds = finalize_lds_bytes<F>(g.nC);
  hipLaunchKernelGGL((k_finalize<F, TT>), dim3(bt.B), dim3(64), fin_lds, s, g, w, HMC, o, bt.map,
                     bt.live, bt.B, rc, fin_lds > 0 ? 1 : 0);
  if (ev) hipEventRecord(ev[3], s);
}

template <typename F, int TT>
static hipError_t launch_eval_tt(const GridDev& g, const BatchDev& bt, const SweepBufs<F>& w,
                                 const tto_outputs& o, hipStream_t s, hipEvent_t* ev,
                                 const SweepPlan& plan, const SweepBufs<double>* rw,
                                 const RefineCtl& rc) {
  const bool refine = (sizeof(F) == 4) && rw && rc.cap > 0;
  RefineCtl main_rc = rc;
  if (!refine) { main_rc.list = nullptr; main_rc.flags = nullptr; }
  GridDev gm = g;
  gm.near_margin = refine ? rc.margin : -1.0;
  launch_pass<F, TT>(gm, bt, w, o, s, ev, plan, main_rc);
  if (refine)
    hipLaunchKernelGGL(k_refine_queue, dim3(1), dim3(1024), 0, s, (const int*)rc.flags, bt.B,
                       rc.cap, rc.list, rc.count, o.status);
  if (o.n1_flows) {
    const F* HMC;
    if constexpr (sizeof(F) == 4) HMC = g.HMC32; else HMC = g.HMC64;
    const int nb = (g.nM + 255) / 256;
    hipLaunchKernelGGL((k_n1_dump<F, TT>), dim3(nb, bt.B), dim3(256), 0, s, g, w, HMC, o.n1_flows);
  }
  if (refine) {
    // FP64 re-evaluation of the queued candidates (no host synchronisation:
    // grids are sized for the capacity and idle workgroups exit at once)
    BatchDev rb = bt;
    rb.B = rc.cap;
    rb.map = rc.list;
    rb.live = rc.count;
    tto_outputs ro = o;
    ro.base_flows = nullptr;
    ro.n1_flows = nullptr;
    RefineCtl none = rc;
    none.list = nullptr;
    none.flags = nullptr;
    GridDev gh = g;
    gh.f0 = g.f0_hi;   // FP64-GEMM base flows
    gh.f0MC = g.f0MC_hi;
    gh.near_margin = -1.0;
    SweepBufs<double> w64 = *rw;
    w64.n_eblk = (g.nM + 63) / 64;
    constexpr int kSplit = 8;
    hipLaunchKernelGGL((k_setup<double, TT>), dim3(rb.B), dim3(256), 0, s, gh, rb, w64,
                       (double*)nullptr);
    hipLaunchKernelGGL(k_zero_live_u64, dim3(1024), dim3(256), 0, s, rc.fbuf,
                       (const int*)rc.count, rc.cap, (size_t)TT * g.nM);
    hipLaunchKernelGGL((k_sweep_split<TT>), dim3((rb.B * w64.n_eblk * kSplit + 3) / 4), dim3(256),
                       0, s, gh, w64, (const double*)g.HMC64, rb.B, kSplit, (const int*)rc.count,
                       rc.fbuf);
    hipLaunchKernelGGL((k_sweep_split_epi<TT>), dim3((rb.B * w64.n_eblk + 3) / 4), dim3(256), 0,
                       s, gh, w64, ro.fmax, rb.B, (const int*)rc.list, (const int*)rc.count,
                       (const unsigned long long*)rc.fbuf);
    const size_t fin_lds = finalize_lds_bytes<double>(g.nC);
    hipLaunchKernelGGL((k_finalize<double, TT>), dim3(rb.B), dim3(64), fin_lds, s, gh, w64,
                       (const double*)g.HMC64, ro, rb.map, rb.live, rb.B, none,
                       fin_lds > 0 ? 1 : 0);
  }
  if (ev) hipEventRecord(ev[4], s);
  return hipGetLastError();
}

template <typename F>
hipError_t launch_evaluate(const GridDev& g, const BatchDev& bt, const SweepBufs<F>& w,
                           const tto_outputs& o, hipStream_t s, hipEvent_t* ev,
                           const SweepPlan& plan, const SweepBufs<double>* rw,
                           const RefineCtl& rc) {
  switch (g.TT) {
    case 1: return launch_eval_tt<F, 1>(g, bt, w, o, s, ev, plan, rw, rc);
    case 8: return launch_eval_tt<F, 8>(g, bt, w, o, s, ev, plan, rw, rc);
    case 24: return launch_eval_tt<F, 24>(g, bt, w, o, s, ev, plan, rw, rc);
    default: return launch_eval_tt<F, 32>(g, bt, w, o, s, ev, plan, rw, rc);
  }
}

// ---------------------------------------------------------------------------
// Worst-k contingencies (the AC validator's pre-filter: the overload energy
// of every N-1 case on its own, the k largest written out).
// k_cont_energy: tile = (candidate, 256 monitored branches) as in the sweep;
// per active contingency every lane forms sum_t max(|f^(l)_e(t)| - fbar_e, 0)
// (an opened monitored branch carries no flow), the wave adds it in a fixed
// butterfly and the four waves add in order into part[c][tile][i].
template <typename F, int TT>
__global__ __launch_bounds__(256) void k_cont_energy(GridDev g, SweepBufs<F> w,
                                                     const F* __restrict__ HMC, int n_eblk,
                                                     double* __restrict__ part) {
  constexpr int RS = rec_stride(TT);
  const int c = blockIdx.y, eb = blockIdx.x;
  const CandInfo* inf = w.info + c;
  if (inf->status & (TTO_ST_ISLANDED | TTO_ST_INVALID)) return;   // uniform per workgroup
  const int nM = g.nM, nC = g.nC, T = g.T;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int ei = eb * 256 + tid;
  const bool valid = ei < nM;
  const int ei_c = valid ? ei : nM - 1;
  const int e = g.mon[ei_c];
  const int k = inf->k, r = inf->r, n_act = inf->n_act;
  bool opened = false;
  for (int q = 0; q < k; ++q) opened |= (inf->open_br[q] == e);
  const bool live = valid && !opened;
  const F lim = (F)g.lim[e];
  F a[TT], U[kVSlots];
  const F* fa = w.fM + (size_t)c * TT * nM + ei_c;
  const F* ua = w.UM + (size_t)c * kVSlots * nM + ei_c;
#pragma unroll
  for (int t = 0; t < TT; ++t) a[t] = fa[(size_t)t * nM];
#pragma unroll
  for (int j = 0; j < kVSlots; ++j) U[j] = j < r ? ua[(size_t)j * nM] : (F)0;
  const F* __restrict__ rec = w.rec + (size_t)c * (nC + 1) * RS;
  const int* __restrict__ act = w.act + (size_t)c * (nC + 1);
  double* out = part + ((size_t)c * n_eblk + eb) * (nC + 1);
  __shared__ double s_w[4][64];
  for (int i0 = 0; i0 < n_act; i0 += 64) {
    const int cnt = min(64, n_act - i0);
    for (int q = 0; q < cnt; ++q) {
      const F* ri = rec + (size_t)(i0 + q) * RS;
      F h = HMC[(size_t)act[i0 + q] * nM + ei_c];
#pragma unroll
      for (int j = 0; j < kVSlots; ++j)
        if (j < r) h = fma_t(U[j], ri[TT + j], h);
      F ov = (F)0;
#pragma unroll
      for (int t = 0; t < TT; ++t) {
        const F f = fabs_t(fma_t(h, ri[t], a[t]));
        if (t < T && f > lim) ov += f - lim;
      }
      double v = live ? (double)ov : 0.0;
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
      if (lane == 0) s_w[wv][q] = v;
    }
    __syncthreads();
    if (tid < cnt) out[i0 + tid] = ((s_w[0][tid] + s_w[1][tid]) + s_w[2][tid]) + s_w[3][tid];
    __syncthreads();
  }
}

// k_worst_k: one workgroup per candidate; tiles summed in order into the
// first tile's row, then k rounds of a block arg-max over the total order
// (energy descending, position in the contingency list ascending), each round
// restricted to keys below the previous pick.
template <typename F>
__global__ __launch_bounds__(256) void k_worst_k(GridDev g, SweepBufs<F> w, int n_eblk,
                                                 double* __restrict__ part, int kk,
                                                 int* __restrict__ ids,
                                                 double* __restrict__ energy) {
  const int c = blockIdx.x, tid = threadIdx.x;
  const CandInfo* inf = w.info + c;
  const int nC = g.nC;
  const int n_act = (inf->status & (TTO_ST_ISLANDED | TTO_ST_INVALID)) ? 0 : inf->n_act;
  const int* act = w.act + (size_t)c * (nC + 1);
  double* row = part + (size_t)c * n_eblk * (nC + 1);
  for (int i = tid; i < n_act; i += 256) {
    double sum = row[i];
    for (int b = 1; b < n_eblk; ++b) sum += row[(size_t)b * (nC + 1) + i];
    row[i] = sum;
  }
  __syncthreads();
  __shared__ double s_v[256];
  __shared__ int s_p[256];
  __shared__ double s_prev_v;
  __shared__ int s_prev_p;
  if (tid == 0) { s_prev_v = __builtin_inf(); s_prev_p = -1; }
  __syncthreads();
  for (int round = 0; round < kk; ++round) {
    const double pv = s_prev_v;
    const int pp = s_prev_p;
    double bv = -1.0;
    int bp = INT_MAX;   // position in the active list (C order)
    for (int i = tid; i < n_act; i += 256) {
      const double v = row[i];
      const bool below = v < pv || (v == pv && i > pp);
      if (below && (v > bv || (v == bv && i < bp))) { bv = v; bp = i; }
    }
    s_v[tid] = bv;
    s_p[tid] = bp;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if (tid < off) {
        const double ov = s_v[tid + off];
        const int op = s_p[tid + off];
        if (ov > s_v[tid] || (ov == s_v[tid] && op < s_p[tid])) { s_v[tid] = ov; s_p[tid] = op; }
      }
      __syncthreads();
    }
    if (tid == 0) {
      const int p = s_p[0];
      const bool got = p != INT_MAX;
      ids[(size_t)c * kk + round] = got ? g.cont[act[p]] : -1;
      energy[(size_t)c * kk + round] = got ? s_v[0] : __builtin_nan("");
      if (got) { s_prev_v = s_v[0]; s_prev_p = p; }
      else { s_prev_v = -2.0; }      // nothing left: later rounds find nothing
    }
    __syncthreads();
  }
}

template <typename F, int TT>
static hipError_t launch_worst_k_tt(const GridDev& g, const BatchDev& bt, const SweepBufs<F>& w,
                                    int kk, int* ids, double* energy, double* part,
                                    hipStream_t s) {
  const F* HMC;
  if constexpr (sizeof(F) == 4) HMC = g.HMC32; else HMC = g.HMC64;
  const int n_eblk = (g.nM + 255) / 256;
  hipLaunchKernelGGL((k_setup<F, TT>), dim3(bt.B), dim3(256), 0, s, g, bt, w, (double*)nullptr);
  if (g.nC > 0)
    hipLaunchKernelGGL((k_cont_energy<F, TT>), dim3(n_eblk, bt.B), dim3(256), 0, s, g, w, HMC,
                       n_eblk, part);
  hipLaunchKernelGGL((k_worst_k<F>), dim3(bt.B), dim3(256), 0, s, g, w, n_eblk, part, kk, ids,
                     energy);
  return hipGetLastError();
}

template <typename F>
hipError_t launch_worst_k(const GridDev& g, const BatchDev& bt, const SweepBufs<F>& w, int kk,
                          int* ids, double* energy, double* part, hipStream_t s) {
  switch (g.TT) {
    case 1: return launch_worst_k_tt<F, 1>(g, bt, w, kk, ids, energy, part, s);
    case 8: return launch_worst_k_tt<F, 8>(g, bt, w, kk, ids, energy, part, s);
    case 24: return launch_worst_k_tt<F, 24>(g, bt, w, kk, ids, energy, part, s);
    default: return launch_worst_k_tt<F, 32>(g, bt, w, kk, ids, energy, part, s);
  }
}

// Candidate set-up alone (f', U and the contingency records), for the
// busbar-outage pass that reuses the candidate's U rows.
template <typename F>
hipError_t launch_setup(const GridDev& g, const BatchDev& bt, const SweepBufs<F>& w,
                        hipStream_t s) {
  switch (g.TT) {
    case 1: hipLaunchKernelGGL((k_setup<F, 1>), dim3(bt.B), dim3(256), 0, s, g, bt, w, (double*)nullptr); break;
    case 8: hipLaunchKernelGGL((k_setup<F, 8>), dim3(bt.B), dim3(256), 0, s, g, bt, w, (double*)nullptr); break;
    case 24: hipLaunchKernelGGL((k_setup<F, 24>), dim3(bt.B), dim3(256), 0, s, g, bt, w, (double*)nullptr); break;
    default: hipLaunchKernelGGL((k_setup<F, 32>), dim3(bt.B), dim3(256), 0, s, g, bt, w, (double*)nullptr); break;
  }
  return hipGetLastError();
}

template hipError_t launch_setup<float>(const GridDev&, const BatchDev&, const SweepBufs<float>&,
                                        hipStream_t);
template hipError_t launch_setup<double>(const GridDev&, const BatchDev&,
                                         const SweepBufs<double>&, hipStream_t);

template hipError_t launch_worst_k<float>(const GridDev&, const BatchDev&, const SweepBufs<float>&,
                                          int, int*, double*, double*, hipStream_t);
template hipError_t launch_worst_k<double>(const GridDev&, const BatchDev&,
                                           const SweepBufs<double>&, int, int*, double*, double*,
                                           hipStream_t);

template hipError_t launch_evaluate<float>(const GridDev&, const BatchDev&, const SweepBufs<float>&,
                                           const tto_outputs&, hipStream_t, hipEvent_t*,
                                           const SweepPlan&, const SweepBufs<double>*,
                                           const RefineCtl&);
template hipError_t launch_evaluate<double>(const GridDev&, const BatchDev&, const SweepBufs<double>&,
                                            const tto_outputs&, hipStream_t, hipEvent_t*,
                                            const SweepPlan&, const SweepBufs<double>*,
                                            const RefineCtl&);

}  // namespace tto
