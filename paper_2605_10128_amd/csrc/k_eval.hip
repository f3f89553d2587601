// Per-candidate kernels of the batched DC N-1 screen.
//
//   k_setup_cand, k_setup_rows
//              FP64 rank-r update of the pre-computed distribution factors for
//              the candidate's openings and bus splits (DC-Optimizer: topology
//              changes enter as low-rank updates of the PTDF): the bordered
//              system, its LU factors and the islanding pivot test (one wave
//              per candidate), then the U rows of the monitored branches,
//              per-contingency records (phi_l(t), V_l) with the LODF
//              denominators 1 - H'_ll and the compacted list of non-islanding
//              contingencies (one workgroup per candidate, rank fixed at
//              compile time).  The monitored post-switch flows f'_M are not
//              stored: every reader forms them from the shared base-flow table,
//              the U row and x(t) (post_flow).
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

// Orders LDS writes and reads among the lanes of one wave (a wave's LDS
// operations complete in issue order; the fences keep the compiler from
// moving them across).
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Shared description of one candidate inside k_setup_cand.
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
  int perm[kMaxRank];      // row i of the pivoted system is row perm[i] of M_c
  int hdr[4];              // valid, k, ns, islanded
  int nsrc;
  int src_row[kMaxSrc];    // gather sources: the openings, then the moved branches
  // staging of the genome slots
  int oval[kMaxRank], sval[kMaxRank], slo[kMaxRank], shi[kMaxRank], stot;
  int mfrom[kMaxMoved], mto[kMaxMoved];
  double mb[kMaxMoved];
};

// Set-up, first kernel: one wave per candidate.  Genome parse and checks, the
// rank-r bordered system M_c in FP64 with its LU factors (partial pivoting)
// and the islanding pivot test, x(t) = M_c^-1 rhs(t), and the candidate's
// SetupDesc for the row kernel: the gather sources with their coefficients
// for W (the column of U before the b_e factor) and for the pivoted
// right-hand side of V_l, the factors, x(t) and the moved-branch fix-ups.
template <typename F, int TT>
__global__ __launch_bounds__(64) void k_setup_cand(GridDev g, BatchDev bt, SweepBufs<F> w) {
  const int c = blockIdx.x;
  const int tid = threadIdx.x;
  const int m = g.n_branch, T = g.T;
  int cb = c;
  if (bt.map) {
    if (c >= min(*bt.live, bt.B)) return;
    cb = bt.map[c];
  }
  __shared__ SetupShared sh;
  __shared__ double s_sub[kSubMax * kSubMax];
  __shared__ int s_bad;
  SetupDesc* D = w.desc + c;

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
    if (sh.hdr[0] && tid < k0) sh.bK[tid] = g.b[sh.open[tid]];
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
    int ns_ = 0;
    for (int q = 0; q < k; ++q) sh.src_row[ns_++] = sh.open[q];
    for (int p = 0; p < sh.moff[ns]; ++p)
      sh.src_row[ns_++] = sh.mbr[p] >= 0 && sh.mbr[p] < m ? sh.mbr[p] : 0;
    sh.nsrc = ns_;
    sh.hdr[0] = valid;
  }
  __syncthreads();
  const int valid = sh.hdr[0], k = sh.hdr[1], ns = sh.hdr[2];
  const int r = k + ns;
  CandInfo* inf = w.info + c;
  if (!valid) {
    if (tid == 0) {
      D->status = TTO_ST_INVALID;
      inf->status = TTO_ST_INVALID;
      inf->r = 0; inf->k = 0; inf->n_act = 0; inf->n_act_pad = 0; inf->n_island = 0;
      inf->n_crit_n0 = 0;
    }
    return;
  }

  // S entries among the gather sources (openings, then moved branches), so
  // that the bordered matrix is built from LDS; more than kSubMax sources
  // read S directly
  const int nsrc = sh.nsrc;
  const bool sub = nsrc <= kSubMax;
  if (sub)
    for (int i = tid; i < nsrc * nsrc; i += 64) {
      const int a = i / nsrc, a2 = i - (i / nsrc) * nsrc;
      s_sub[i] = g.S[(size_t)sh.src_row[a] * m + sh.src_row[a2]];
    }
  __syncthreads();
  // S between sources a and a2 (a < k: opening a; a >= k: moved branch a - k)
  auto Sv = [&](int a, int a2) -> double {
    return sub ? s_sub[a * nsrc + a2] : g.S[(size_t)sh.src_row[a] * m + sh.src_row[a2]];
  };

  // bordered matrix M_c, one entry per lane; H_ab = b_a S_ab
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
    for (int q = 0; q < kMaxRank; ++q) sh.perm[q] = q;
    for (int p = 0; p < r; ++p) {
      int best = p;
      double bv = fabs(sh.M[p][p]);
      for (int i = p + 1; i < r; ++i)
        if (fabs(sh.M[i][p]) > bv) { bv = fabs(sh.M[i][p]); best = i; }
      sh.piv[p] = best;
      if (best != p) {
        for (int q = 0; q < r; ++q) { const double t = sh.M[p][q]; sh.M[p][q] = sh.M[best][q]; sh.M[best][q] = t; }
        const int t = sh.perm[p]; sh.perm[p] = sh.perm[best]; sh.perm[best] = t;
      }
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
      D->status = TTO_ST_ISLANDED;
      inf->status = TTO_ST_ISLANDED;
      inf->r = r; inf->k = k; inf->n_act = 0; inf->n_act_pad = 0; inf->n_island = 0;
      inf->n_moved = sh.moff[ns];
      inf->n_crit_n0 = 0;
    }
    return;
  }

  // x(t) = M_c^{-1} rhs(t), rhs = [f0_K ; (p_j - phi_j) / s_j], one lane per t
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
      D->x[t][q] = (t < T) ? x[q] : 0.0;
      D->x32[t][q] = (t < T) ? (float)x[q] : 0.0f;
      bad |= (t < T) && !isfinite(x[q]);
    }
    if (bad) atomicAdd(&s_bad, 1);
  }

  // the description: coefficient rows per source, zero rows up to the next
  // multiple of 8 (the row kernel reads sources in groups of 8)
  const int nm = sh.moff[ns];
  const int nsrc8 = (nsrc + 7) & ~7;
  for (int i = tid; i < nsrc8 * kMaxRank; i += 64) {
    const int s = i / kMaxRank, q = i - (i / kMaxRank) * kMaxRank;
    // column slot of source s and its coefficient: an opening enters its own
    // slot with 1, a moved branch its split's slot with sg_b b_b
    int slot = -1;
    double cf = 0.0;
    if (s < k) { slot = s; cf = 1.0; }
    else if (s < nsrc) { slot = k + sh.mj[s - k]; cf = sh.msg[s - k]; }
    D->coefW[s][q] = (q == slot) ? cf : 0.0;
    // pivoted right-hand side of V_l: row q takes slot perm[q] scaled by
    // b_K (openings) or -1/s_j (splits)
    double cv = 0.0;
    if (q < r && sh.perm[q] == slot) cv = slot < k ? sh.bK[slot] * cf : -sh.inv_s[slot - k] * cf;
    D->coefV[s][q] = cv;
    if (q == 0) D->src_row[s] = s < nsrc ? sh.src_row[s] : 0;
  }
  for (int p = tid; p < nm; p += 64) {
    const int slot = k + sh.mj[p];
    int pos = 0;
    for (int q = 0; q < r; ++q) pos = (sh.perm[q] == slot) ? q : pos;
    D->mbr[p] = sh.mbr[p];
    D->mslot[p] = slot;
    D->mpos[p] = pos;
    D->msg[p] = sh.msg[p];
    D->madd[p] = sh.msign[p] * sh.inv_s[sh.mj[p]];
  }
  {
    const int i = tid >> 3, q = tid & 7;
    D->LU[i][q] = (i < r && q < r) ? sh.M[i][q] : 0.0;
    if (q == 0) {
      D->inv_diag[i] = i < r ? 1.0 / sh.M[i][i] : 0.0;
      D->uscale[i] = i < k ? 1.0 : -1.0;
      D->open[i] = i < k ? sh.open[i] : -1;
    }
  }
  __syncthreads();
  if (tid == 0) {
    D->status = 0;
    D->r = r; D->k = k; D->ns = ns; D->nsrc = nsrc; D->nm = nm;
    D->bad = s_bad;
  }
}

// Set-up, second kernel: one workgroup per candidate, one lane per row of
// M and then of C, rank R fixed at compile time.  The candidate's
// description is copied to LDS once and read there as broadcasts (reads
// through the scalar cache would each wait on its latency, and holding the
// uniform values in scalar registers runs out of them).
typedef const __attribute__((address_space(4))) SetupDesc CSetupDesc;

// Post-switch flow of a monitored branch, f'_e(t) = f0_e(t) + sum_q U_eq x_q(t),
// formed in the flow type from the stored U row: FP64 flows from the FP64
// base-flow table and x(t); FP32 flows from their FP32 copies (f0 and x each
// rounded once), so that the loads land in the flow registers directly.  Every
// reader takes the steps in increasing q from the table entry, so f'_e(t) is
// bitwise the same wherever it is formed.  Both tables have zero rows past T,
// as has x(t).
template <typename F>
__device__ __forceinline__ F post_base(const GridDev& g, int ei, int t) {
  if constexpr (sizeof(F) == 4) return g.f0M32[(size_t)t * g.nM + ei];
  else return g.f0MC[(size_t)t * ((size_t)g.nM + g.nC) + ei];
}
template <typename F, typename D_>
__device__ __forceinline__ F post_x(const D_* D, int t, int j) {
  if constexpr (sizeof(F) == 4) return D->x32[t][j];
  else return D->x[t][j];
}
__device__ __forceinline__ float post_step(float u, float x, float fp) { return __builtin_fmaf(u, x, fp); }
__device__ __forceinline__ double post_step(double u, double x, double fp) { return __builtin_fma(u, x, fp); }

// f'_e(t) of monitored position ei with run-time rank r (U row at ua, stride nM).
template <typename F>
__device__ __forceinline__ F post_flow(const GridDev& g, const SetupDesc* D, const F* ua, int r,
                                       int ei, int t) {
  F fp = post_base<F>(g, ei, t);
  for (int j = 0; j < r; ++j) fp = post_step(ua[(size_t)j * g.nM], post_x<F>(D, t, j), fp);
  return fp;
}

// A uniform stride passed through an opaque register copy: the per-timestep
// offsets of a row are formed inside the iteration rather than kept in
// scalar registers for the whole loop.
__device__ __forceinline__ int at_use(int v) {
  __asm__ volatile("" : "+s"(v));
  return v;
}

// Arguments of k_setup_rows: only what the row loops read and write, so that
// few scalar registers hold kernel arguments.
template <typename F>
struct RowsArgs {
  const int* mon;
  const int* cont;
  const double* f0MC;
  const double* bMC;
  const double* limM;
  const double* sllC;
  const double* SMC;
  const double* S;     // full S and f0 and b: the optional base-flow output only
  const double* f0;
  const double* b;
  F* UM;
  F* rec;
  int* act;
  int* slot;
  CandInfo* info;
  const SetupDesc* desc;
  int m, T, nM, nC;
};

// Row scratch of k_setup_rows in LDS.
template <typename F>
struct RowsShared {
  static constexpr int SP = 128 / (int)sizeof(F);  // record entries per staging pass
  F stage[4][64][SP + 1];   // one slab per wave
  SetupDesc d;              // the candidate's description (the parts in use)
  int wcnt[2][4];
  int n0, nisl, bad;
};

// W_q = sum_s coefW[s][q] tab[src_row[s]][col] (and the pivoted right-hand
// side Y when V is wanted), eight independent row loads in flight; the
// coefficient rows past the sources are zero.
template <int R, bool WITH_V>
__device__ __forceinline__ void gather_rows(const SetupDesc& D, int nsrc, const double* __restrict__ tab,
                                            size_t ld, int col, double* W, double* Y) {
#pragma unroll
  for (int q = 0; q < R; ++q) { W[q] = 0.0; if (WITH_V) Y[q] = 0.0; }
  for (int s0 = 0; s0 < nsrc; s0 += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      v[u] = (s0 + u < nsrc)
                 ? tab[(size_t)__builtin_amdgcn_readfirstlane(D.src_row[s0 + u]) * ld + col]
                 : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
#pragma unroll
      for (int q = 0; q < R; ++q) {
        W[q] = fma(D.coefW[s0 + u][q], v[u], W[q]);
        if (WITH_V) Y[q] = fma(D.coefV[s0 + u][q], v[u], Y[q]);
      }
    }
  }
}

// Row e is an opening of the candidate / a branch moved by one of its splits.
__device__ __forceinline__ void row_kind(const SetupDesc& D, int k, int nm, int e, bool* opened,
                                         bool* moved) {
  bool op = false, mv = false;
  for (int q = 0; q < k; ++q) op |= (D.open[q] == e);
  for (int p = 0; p < nm; ++p) mv |= (D.mbr[p] == e);
  *opened = op;
  *moved = mv;
}

template <typename F, int TT, int R>
__device__ __forceinline__ void setup_rows(const RowsArgs<F>& a, double* __restrict__ base_out,
                                           int c, int cb, CSetupDesc* D, RowsShared<F>& sm) {
  const SetupDesc& L = sm.d;
  constexpr int RS = rec_stride_r(TT, R);   // this candidate's record stride
  constexpr int SP = RowsShared<F>::SP;
  const int tid = threadIdx.x;
  const int m = a.m, T = a.T, nM = a.nM, nC = a.nC;
  const size_t nMC = (size_t)nM + nC;
  const int k = D->k, nsrc = D->nsrc, nm = D->nm;

  // U row of branch e: U_q = (+-) b_e W_q, plus sg_b b_b in its split's slot
  // when e itself is moved (rare: a branch of the candidate)
  auto finish_u = [&](int e, double be, bool moved, const double* W, double* U) {
#pragma unroll
    for (int q = 0; q < R; ++q) U[q] = L.uscale[q] * be * W[q];
    if (moved) {
      for (int p = 0; p < nm; ++p) {
        if (L.mbr[p] == e) {
          const int qq = L.mslot[p];
#pragma unroll
          for (int q = 0; q < R; ++q)
            if (q == qq) U[q] += L.msg[p];
        }
      }
    }
  };

  // monitored rows: U_M and the N-0 overload count (f'_M itself is formed
  // by its readers).  A non-finite grid injection makes every base flow of
  // its timestep non-finite (the product with a zero PTDF entry included), so
  // the first monitored row sees it.
  int n0 = 0, nbad = 0;
  F* const UM = a.UM + (size_t)c * kVSlots * nM;  // [q][ei]: coalesced across lanes
  for (int ei = tid; ei < nM; ei += 256) {
    keep_in_loop();
    const int sM = at_use(nM), sMC = at_use((int)nMC);
    const int e = a.mon[ei];
    double f0e[TT];
#pragma unroll
    for (int t = 0; t < TT; ++t) f0e[t] = a.f0MC[t * sMC + ei];   // zero rows past T
    if (ei == 0)
#pragma unroll
      for (int t = 0; t < TT; ++t) nbad += !isfinite(f0e[t]);
    const double be = a.bMC[ei];
    bool opened, moved;
    row_kind(L, k, nm, e, &opened, &moved);
    // an opened monitored branch carries no flow: never counted, its stored
    // rows are zeroed below
    const double lim = opened ? HUGE_VAL : a.limM[ei];
    double W[R > 0 ? R : 1], U[R > 0 ? R : 1];
    gather_rows<R, false>(L, nsrc, a.SMC, nMC, ei, W, nullptr);
    finish_u(e, be, moved, W, U);
#pragma unroll
    for (int t = 0; t < TT; ++t) {
      double fp = f0e[t];
#pragma unroll
      for (int q = 0; q < R; ++q) fp += U[q] * L.x[t][q];
      // past T: x(t) = 0 and f0 = 0, so fp = 0
      n0 += fabs(fp) > lim;
    }
    // only the R slots in use: every reader of U stops at the candidate's rank;
    // an opened row (rare: one of the candidate's openings) is zero, and every
    // reader gives it zero flow by its own test
#pragma unroll
    for (int q = 0; q < R; ++q) UM[q * sM + ei] = opened ? (F)0 : (F)U[q];
  }
  if (n0) atomicAdd(&sm.n0, n0);
  if (nbad) atomicAdd(&sm.bad, nbad);

  // optional full post-switch base flows
  if (base_out) {
    for (int e = tid; e < m; e += 256) {
      keep_in_loop();
      bool opened, moved;
      row_kind(L, k, nm, e, &opened, &moved);
      double W[R > 0 ? R : 1], U[R > 0 ? R : 1];
      gather_rows<R, false>(L, nsrc, a.S, (size_t)m, e, W, nullptr);
      finish_u(e, a.b[e], moved, W, U);
      for (int t = 0; t < T; ++t) {
        double fp = 0.0;
        if (!opened) {
          fp = a.f0[(size_t)e * T + t];
#pragma unroll
          for (int q = 0; q < R; ++q) fp += U[q] * L.x[t][q];
        }
        base_out[((size_t)cb * m + e) * T + t] = fp;
      }
    }
  }

  // contingencies: V_l, denominators, phi_l, ordered compaction
  const int lane = tid & 63, wid = tid >> 6;
  F* rec = a.rec + (size_t)c * (nC + 1) * rec_stride(TT);
  int* act = a.act + (size_t)c * (nC + 1);
  int nisl = 0;
  int run = 0;   // records written by the chunks before (same in every lane)
  for (int base = 0; base < nC; base += 256) {
    keep_in_loop();
    const int sMC = at_use((int)nMC);
    const int li = base + tid;
    const bool row = li < nC;
    const int lc = row ? li : nC - 1;
    const int l = a.cont[lc];
    // row-only loads first (their latency overlaps the column gather)
    const double s_ll = a.sllC[lc];
    const double b_l = a.bMC[nM + lc];
    double f0l[TT];
#pragma unroll
    for (int t = 0; t < TT; ++t) f0l[t] = a.f0MC[t * sMC + nM + lc];
    bool opened, moved;
    row_kind(L, k, nm, l, &opened, &moved);
    double W[R > 0 ? R : 1], U[R > 0 ? R : 1], V[R > 0 ? R : 1];
    gather_rows<R, true>(L, nsrc, a.SMC, nMC, nM + lc, W, V);
    finish_u(l, b_l, moved, W, U);
    // the contingency itself moved by split j: ps_j = sg_l enters the
    // right-hand side as sg_l / s_j, in its pivoted position
    if (moved) {
      for (int p = 0; p < nm; ++p) {
        if (L.mbr[p] == l) {
          const int pp = L.mpos[p];
#pragma unroll
          for (int q = 0; q < R; ++q)
            if (q == pp) V[q] += L.madd[p];
        }
      }
    }
    // V_l = M_c^-1 rhs from the LU factors (the right-hand side is already
    // in pivoted order)
#pragma unroll
    for (int i = 0; i < R; ++i) {
#pragma unroll
      for (int q = 0; q < i; ++q) V[i] -= L.LU[i][q] * V[q];
    }
#pragma unroll
    for (int i = R - 1; i >= 0; --i) {
#pragma unroll
      for (int q = i + 1; q < R; ++q) V[i] -= L.LU[i][q] * V[q];
      V[i] *= L.inv_diag[i];
    }
    double hll = b_l * s_ll;
#pragma unroll
    for (int q = 0; q < R; ++q) hll += U[q] * V[q];
    const double d = 1.0 - hll;
    // an already opened contingency is the N-0 state: phi = 0, V = 0
    const bool island = row && !opened && fabs(d) < kTauCont;
    const bool active = row && !island;
    const double inv_d = (opened || island) ? 0.0 : 1.0 / d;
    nisl += island;
    // ordered compaction: one barrier per chunk, the wave counts double
    // buffered so that a wave one chunk ahead never overwrites unread counts
    const unsigned long long mask = ballot64(active);
    const int par = (base >> 8) & 1;
    if (lane == 0) sm.wcnt[par][wid] = __popcll(mask);
    __syncthreads();
    int o0 = run;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int v = sm.wcnt[par][q];
      o0 += q < wid ? v : 0;
      run += v;
    }
    const int rank = __popcll(mask & ((1ull << lane) - 1ull));
    const int na = __popcll(mask);
    const int off = o0 + rank;
    // Records go out through the wave's own LDS slab, one 128-byte line of
    // each record per pass, so that every store instruction writes whole
    // lines (direct per-lane 128-byte records leave partially written lines
    // thrashing the L2); only the wave's lanes meet there.
    F (*slab)[SP + 1] = sm.stage[wid];
#pragma unroll
    for (int p0 = 0; p0 < RS; p0 += SP) {
      if (active) {
#pragma unroll
        for (int u = 0; u < SP; ++u) {
          const int slot = p0 + u;
          if (slot < RS) {
            double v = 0.0;
            if (slot < TT) {
              // phi_l(t) = f'_l(t) / (1 - H'_ll), zero for an already opened l
              // (and past T, where f0 and x(t) are zero)
              if (!opened) {
                double fl = f0l[slot];
#pragma unroll
                for (int q = 0; q < R; ++q) fl += U[q] * L.x[slot][q];
                v = fl * inv_d;
              }
            } else if (slot < TT + R) {
              v = opened ? 0.0 : V[slot - TT < R ? slot - TT : 0];
            }
            slab[rank][u] = (F)v;
          }
        }
      }
      wave_lds_sync();
      // slots p0 .. p0 + nsl of the wave's na records, every lane busy (one
      // contiguous run when a record fits in one pass)
      const int nsl = (RS - p0) < SP ? (RS - p0) : SP;
      for (int idx = lane; idx < na * nsl; idx += 64) {
        const int i = idx / nsl, u = idx - (idx / nsl) * nsl;
        rec[(size_t)(o0 + i) * RS + p0 + u] = slab[i][u];
      }
      wave_lds_sync();
    }
    if (active) act[off] = li;
    if (a.slot && row) a.slot[(size_t)c * nC + li] = active ? off : -1;
  }
  if (nisl) atomicAdd(&sm.nisl, nisl);
  __syncthreads();
  const int n_act = run;
  // even length for the paired sweep: duplicate the last record (max unchanged)
  if (n_act & 1) {
    const F* src = rec + (size_t)(n_act - 1) * RS;
    F* dst = rec + (size_t)n_act * RS;
    for (int q = tid; q < RS; q += 256) dst[q] = src[q];
    if (tid == 0) act[n_act] = act[n_act - 1];
  }
  CandInfo* inf = a.info + c;
  if (tid == 0 && sm.bad) {
    // non-finite injections: no metric is defined, the candidate is skipped
    inf->status = TTO_ST_INVALID | TTO_ST_NONFINITE;
    inf->r = R; inf->k = k; inf->n_act = 0; inf->n_act_pad = 0; inf->n_island = 0;
    inf->n_moved = nm;
    inf->n_crit_n0 = 0;
  } else if (tid == 0) {
    inf->status = 0;
    inf->r = R;
    inf->k = k;
    inf->n_act = n_act;
    inf->n_act_pad = n_act + (n_act & 1);
    inf->n_island = sm.nisl;
    inf->n_crit_n0 = sm.n0;
    inf->n_moved = nm;
    for (int q = 0; q < kMaxRank; ++q) inf->open_br[q] = L.open[q];
  }
}

template <typename F, int TT>
__global__ __launch_bounds__(256) void k_setup_rows(RowsArgs<F> a, const int* __restrict__ map,
                                                    const int* __restrict__ live, int B,
                                                    double* __restrict__ base_out) {
  const int c = blockIdx.x;
  int cb = c;
  if (map) {
    if (c >= min(*live, B)) return;
    cb = map[c];
  }
  __shared__ RowsShared<F> sm;
  CSetupDesc* D = (CSetupDesc*)(a.desc + c);
  if (D->status) return;   // invalid or islanded: the first kernel wrote its outputs
  if (threadIdx.x == 0) { sm.n0 = 0; sm.nisl = 0; sm.bad = D->bad; }
  // the description's parts in use: openings, sources and their coefficient
  // rows (padded to 8), moved branches, factors, x(t)
  {
    const int tid = threadIdx.x;
    const int nsrc8 = (D->nsrc + 7) & ~7, nm = D->nm;
    SetupDesc& L = sm.d;
    if (tid < 8) { L.open[tid] = D->open[tid]; L.uscale[tid] = D->uscale[tid]; L.inv_diag[tid] = D->inv_diag[tid]; }
    if (tid < 64) L.LU[tid >> 3][tid & 7] = D->LU[tid >> 3][tid & 7];
    if (tid < nsrc8) L.src_row[tid] = D->src_row[tid];
    if (tid < nm) {
      L.mbr[tid] = D->mbr[tid]; L.mslot[tid] = D->mslot[tid]; L.mpos[tid] = D->mpos[tid];
      L.msg[tid] = D->msg[tid]; L.madd[tid] = D->madd[tid];
    }
    for (int i = tid; i < nsrc8 * kMaxRank; i += 256) {
      L.coefW[i >> 3][i & 7] = D->coefW[i >> 3][i & 7];
      L.coefV[i >> 3][i & 7] = D->coefV[i >> 3][i & 7];
    }
    for (int i = tid; i < TT * kMaxRank; i += 256) L.x[i >> 3][i & 7] = D->x[i >> 3][i & 7];
  }
  __syncthreads();
  switch (D->r) {
    case 0: setup_rows<F, TT, 0>(a, base_out, c, cb, D, sm); break;
    case 1: setup_rows<F, TT, 1>(a, base_out, c, cb, D, sm); break;
    case 2: setup_rows<F, TT, 2>(a, base_out, c, cb, D, sm); break;
    case 3: setup_rows<F, TT, 3>(a, base_out, c, cb, D, sm); break;
    case 4: setup_rows<F, TT, 4>(a, base_out, c, cb, D, sm); break;
    case 5: setup_rows<F, TT, 5>(a, base_out, c, cb, D, sm); break;
    case 6: setup_rows<F, TT, 6>(a, base_out, c, cb, D, sm); break;
    case 7: setup_rows<F, TT, 7>(a, base_out, c, cb, D, sm); break;
    default: setup_rows<F, TT, 8>(a, base_out, c, cb, D, sm); break;
  }
}

// Both set-up kernels of a batch (bt.B workgroups each).
template <typename F, int TT>
static void launch_setup_tt(const GridDev& g, const BatchDev& bt, const SweepBufs<F>& w,
                            double* base_out, hipStream_t s) {
  hipLaunchKernelGGL((k_setup_cand<F, TT>), dim3(bt.B), dim3(64), 0, s, g, bt, w);
  RowsArgs<F> a;
  a.mon = g.mon; a.cont = g.cont; a.f0MC = g.f0MC; a.bMC = g.bMC; a.limM = g.limM;
  a.sllC = g.sllC; a.SMC = g.SMC; a.S = g.S; a.f0 = g.f0; a.b = g.b;
  a.UM = w.UM; a.rec = w.rec; a.act = w.act; a.slot = w.slot; a.info = w.info;
  a.desc = w.desc;
  a.m = g.n_branch; a.T = g.T; a.nM = g.nM; a.nC = g.nC;
  hipLaunchKernelGGL((k_setup_rows<F, TT>), dim3(bt.B), dim3(256), 0, s, a, bt.map, bt.live, bt.B,
                     base_out);
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

// Lane entry of one H[M, C] column through a raw buffer load: the resource is
// based at the column (wave-uniform, built in scalar registers) and the lane's
// byte offset is fixed for the whole contingency loop, so no per-load vector
// address arithmetic is issued.  The column holds nM entries and every offset
// is below that (ei is clamped into the monitored set).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t col_rsrc(const void* col, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(col), (short)0, bytes, 0x00020000);
}
__device__ __forceinline__ float col_ld(__amdgpu_buffer_rsrc_t rs, int off, float*) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0));
}
__device__ __forceinline__ double col_ld(__amdgpu_buffer_rsrc_t rs, int off, double*) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
}

// Contingency pairs [i0, i1) of candidate c for the lanes' monitored
// positions ei[p] (p < NP, clamped into range): acc[p][t] = max |f^(l)|.
template <typename F, int TT, int R, int NP>
__device__ __forceinline__ void sweep_core(const GridDev& g, const SweepBufs<F>& w,
                                           const F* __restrict__ HMC, int c, const int* ei,
                                           int i0, int i1, F (*acc)[TT]) {
  constexpr int RS = rec_stride_r(TT, R);
  const int nM = g.nM, nC = g.nC;
  F U[NP][R > 0 ? R : 1], a[NP][TT];
  CSetupDesc* D = (CSetupDesc*)(w.desc + c);   // x(t): wave-uniform
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const F* ua = w.UM + (size_t)c * kVSlots * nM + ei[p];
#pragma unroll
    for (int j = 0; j < R; ++j) U[p][j] = ua[(size_t)j * nM];
  }
#pragma unroll
  for (int p = 0; p < NP; ++p) {
#pragma unroll
    for (int t = 0; t < TT; ++t) {
      F fp = post_base<F>(g, ei[p], t);   // f'_e(t), as post_flow forms it
#pragma unroll
      for (int j = 0; j < R; ++j) fp = post_step(U[p][j], post_x<F>(D, t, j), fp);
      a[p][t] = fp;
      acc[p][t] = (F)0;
    }
  }
  const F* __restrict__ rec = w.rec + (size_t)c * (nC + 1) * rec_stride(TT);
  const int* __restrict__ act = w.act + (size_t)c * (nC + 1);
  if (i1 <= i0) return;
  // The H entries of a pair are loaded once the previous pair has been
  // consumed, into the same registers (no copies); the latency is covered by
  // the other waves of the SIMD.  The resource of each column is based at the
  // column and the lane's byte offset is fixed, so the loads issue no vector
  // address arithmetic.
  const int col_bytes = nM * (int)sizeof(F);
  int eoff[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) eoff[p] = ei[p] * (int)sizeof(F);
  F h0[NP], h1[NP];
  auto load_pair = [&](int i) {
    const auto q0 = col_rsrc(HMC + (size_t)act[i] * nM, col_bytes);
    const auto q1 = col_rsrc(HMC + (size_t)act[i + 1] * nM, col_bytes);
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      h0[p] = col_ld(q0, eoff[p], (F*)nullptr);
      h1[p] = col_ld(q1, eoff[p], (F*)nullptr);
    }
  };
  load_pair(i0);
  for (int i = i0; i < i1; i += 2) {
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
    load_pair((i + 2 < i1) ? i + 2 : i);   // the last one re-reads an in-range pair
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
  else if (order == 3) {
    // two passes over the batch, each candidate-major over one half of the
    // wave blocks
    const int h0 = (n_wb + 1) >> 1, h1 = n_wb - h0;
    if (u < nc * h0) { *c = u / h0; *wb = u - *c * h0; }
    else { const int v = u - nc * h0; *c = v / h1; *wb = h0 + v - *c * h1; }
  }
  else { *c = u / n_wb; *wb = u - *c * n_wb; }
}

// One wave per work item.  Workgroups are dealt to the 8 XCDs round-robin;
// order != 0 remaps workgroup q so that each XCD takes a contiguous range of
// the item order: order 1 candidate-major (the waves of a candidate share its
// records in one L2), order 2 block-major (an XCD streams few column blocks
// of H[M, C] for many candidates), order 3 candidate-major over the first
// half of every candidate's wave blocks and then over the second (half of
// the H column blocks in flight at a time).  The grid is a multiple of 8.
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
// |f^(l)| at (e*, t*) for the active contingencies i = lane + 64 u of a
// candidate, four per lane per step so that their loads are in flight
// together; the rank is a compile-time bound.  Pass 1 keeps the maximum
// (and the flows, when vbuf is given).
template <typename F, int TT, int R>
__device__ __forceinline__ double fin_flows(const F* __restrict__ HMC, const F* rec,
                                            const int* act, const F* ua, int nM, int be, int bt,
                                            F a, int n_act, F* vbuf) {
  constexpr int RS = rec_stride_r(TT, R);
  const int lane = threadIdx.x;
  F u[R > 0 ? R : 1];
#pragma unroll
  for (int j = 0; j < R; ++j) u[j] = ua[(size_t)j * nM];
  double bv = -1.0;
  for (int i0 = lane; i0 < n_act; i0 += 256) {
    F h[4], ph[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = min(i0 + 64 * q, n_act - 1);
      const F* ri = rec + (size_t)i * RS;
      h[q] = HMC[(size_t)act[i] * nM + be];
      ph[q] = ri[bt];
#pragma unroll
      for (int j = 0; j < R; ++j) h[q] = fma_t(u[j], ri[TT + j], h[q]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = i0 + 64 * q;
      if (i < n_act) {
        const double v = (double)fabs_t(fma_t(h[q], ph[q], a));
        if (vbuf) vbuf[i] = (F)v;
        bv = fmax(bv, v);
      }
    }
  }
  return bv;
}

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
    const F* ua = w.UM + (size_t)c * kVSlots * nM + be;
    const F a = post_flow(g, w.desc + c, ua, inf.r, be, bt);
    const F* rec = w.rec + (size_t)c * (nC + 1) * RS;
    const int* act = w.act + (size_t)c * (nC + 1);
    const int rs = rec_stride_r(TT, inf.r);
    auto flow = [&](int i) -> double {
      const F* ri = rec + (size_t)i * rs;
      F h = HMC[(size_t)act[i] * nM + be];
      for (int j = 0; j < inf.r; ++j) h = fma_t(ua[(size_t)j * nM], ri[TT + j], h);
      return (double)fabs_t(fma_t(h, ri[bt], a));
    };
    F* vbuf = cache_flows ? (F*)fin_lds : nullptr;   // lane i mod 64 owns entry i
    switch (inf.r) {
      case 0: bv = fin_flows<F, TT, 0>(HMC, rec, act, ua, nM, be, bt, a, inf.n_act, vbuf); break;
      case 1: bv = fin_flows<F, TT, 1>(HMC, rec, act, ua, nM, be, bt, a, inf.n_act, vbuf); break;
      case 2: bv = fin_flows<F, TT, 2>(HMC, rec, act, ua, nM, be, bt, a, inf.n_act, vbuf); break;
      case 3: bv = fin_flows<F, TT, 3>(HMC, rec, act, ua, nM, be, bt, a, inf.n_act, vbuf); break;
      case 4: bv = fin_flows<F, TT, 4>(HMC, rec, act, ua, nM, be, bt, a, inf.n_act, vbuf); break;
      case 5: bv = fin_flows<F, TT, 5>(HMC, rec, act, ua, nM, be, bt, a, inf.n_act, vbuf); break;
      case 6: bv = fin_flows<F, TT, 6>(HMC, rec, act, ua, nM, be, bt, a, inf.n_act, vbuf); break;
      case 7: bv = fin_flows<F, TT, 7>(HMC, rec, act, ua, nM, be, bt, a, inf.n_act, vbuf); break;
      default: bv = fin_flows<F, TT, 8>(HMC, rec, act, ua, nM, be, bt, a, inf.n_act, vbuf); break;
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
  const F* ua = w.UM + (size_t)c * kVSlots * nM + ei;
  const F* rec = w.rec + (size_t)c * (nC + 1) * RS;
  F fa[TT];
#pragma unroll
  for (int t = 0; t < TT; ++t) fa[t] = bad ? (F)0 : post_flow(g, w.desc + c, ua, inf.r, ei, t);
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
    const F* ri = rec + (size_t)slot * rec_stride_r(TT, inf.r);
    F h = HMC[(size_t)li * nM + ei];
    for (int j = 0; j < inf.r; ++j) h = fma_t(ua[(size_t)j * nM], ri[TT + j], h);
#pragma unroll
    for (int t = 0; t < TT; ++t)
      if (t < T) out[t] = (double)fma_t(h, ri[t], fa[t]);
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
  launch_setup_tt<F, TT>(g, bt, w, o.base_flows, s);
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
    launch_setup_tt<double, TT>(gh, rb, w64, nullptr, s);
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
  const F* ua = w.UM + (size_t)c * kVSlots * nM + ei_c;
#pragma unroll
  for (int j = 0; j < kVSlots; ++j) U[j] = j < r ? ua[(size_t)j * nM] : (F)0;
#pragma unroll
  for (int t = 0; t < TT; ++t) a[t] = post_flow(g, w.desc + c, ua, r, ei_c, t);
  const F* __restrict__ rec = w.rec + (size_t)c * (nC + 1) * RS;
  const int* __restrict__ act = w.act + (size_t)c * (nC + 1);
  double* out = part + ((size_t)c * n_eblk + eb) * (nC + 1);
  __shared__ double s_w[4][64];
  for (int i0 = 0; i0 < n_act; i0 += 64) {
    const int cnt = min(64, n_act - i0);
    for (int q = 0; q < cnt; ++q) {
      const F* ri = rec + (size_t)(i0 + q) * rec_stride_r(TT, r);
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
  launch_setup_tt<F, TT>(g, bt, w, nullptr, s);
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
    case 1: launch_setup_tt<F, 1>(g, bt, w, nullptr, s); break;
    case 8: launch_setup_tt<F, 8>(g, bt, w, nullptr, s); break;
    case 24: launch_setup_tt<F, 24>(g, bt, w, nullptr, s); break;
    default: launch_setup_tt<F, 32>(g, bt, w, nullptr, s); break;
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
