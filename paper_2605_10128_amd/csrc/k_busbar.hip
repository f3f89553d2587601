// Busbar outages (Fitness function heuristics: busbar penalty lambda_b; High-
// level loop: lambda_f2 = lambda_f1 - max(lambda_b - lambda_b_pre, 0)).
//
// A busbar outage b removes every in-service branch on bus b's node of the
// post-switch grid (a split's busbar B is another node and keeps its branches
// and its moved injection) and loses the injection P_A(t) left on that node,
// which the slack picks up.  On the device this is the candidate's bordered
// system on the base grid with the busbar's branches as extra openings, all
// but one of them: once P_A has moved to the slack, the node carries no
// injection, so the one branch kept in service carries no flow (opening all
// of them would make the system singular).  The base flows are shifted to
// f0 - PTDF_{:,b} P_A.  An outage whose system fails the pivot test islands
// the grid and is skipped and counted.
//
//   k_bb_setup     one wave per (candidate, busbar): genome parse in the set-up
//                  kernel's column order, bordered matrix, FP64 LU with the
//                  islanding test, solutions z(t) and P_A(t) stored.
//   k_bb_sweep     tile (candidate, 256 monitored branches) as in the N-1
//                  sweep: the candidate's U rows from the set-up, the busbar's
//                  own columns gathered per outage, the maximum over outages
//                  kept in registers; tile sums of max(f^max - fbar, 0).
//   k_bb_finalize  fixed-order sums: lambda_b, islanding count, lambda_f2.
#include "tto_busbar.h"

#include <float.h>
#include <limits.h>
#include <math.h>

namespace tto {

namespace {

__global__ __launch_bounds__(256) void k_bb_tables(const double* __restrict__ ptdf, int n_bus,
                                                   int m, const int* __restrict__ mon, int nM,
                                                   const int* __restrict__ bus, int nb,
                                                   double* __restrict__ PB,
                                                   double* __restrict__ PBM,
                                                   float* __restrict__ PBM32) {
  const int ib = blockIdx.y;
  const int b = bus[ib];
  for (int x = blockIdx.x * 256 + threadIdx.x; x < m; x += gridDim.x * 256)
    PB[(size_t)ib * m + x] = ptdf[(size_t)x * n_bus + b];
  for (int ei = blockIdx.x * 256 + threadIdx.x; ei < nM; ei += gridDim.x * 256) {
    const double v = ptdf[(size_t)mon[ei] * n_bus + b];
    PBM[(size_t)ib * nM + ei] = v;
    PBM32[(size_t)ib * nM + ei] = (float)v;
  }
}

// H of the busbars' branches against the monitored set: HB[p][ei] = b_e S_{x,e}
__global__ __launch_bounds__(256) void k_bb_htile(const double* __restrict__ S,
                                                  const double* __restrict__ bsus,
                                                  const int* __restrict__ mon, int nM, int m,
                                                  const int* __restrict__ inc_br,
                                                  double* __restrict__ HB,
                                                  float* __restrict__ HB32) {
  const int p = blockIdx.y;
  const size_t x = (size_t)inc_br[p];
  for (int ei = blockIdx.x * 256 + threadIdx.x; ei < nM; ei += gridDim.x * 256) {
    const int e = mon[ei];
    const double v = bsus[e] * S[x * m + e];
    HB[(size_t)p * nM + ei] = v;
    HB32[(size_t)p * nM + ei] = (float)v;
  }
}

struct BbShared {
  int op[kBbMaxR];            // openings: the candidate's, then the busbar's
  int sbus[kMaxRank], sslot[kMaxRank];
  int moff[kMaxRank + 1];
  int mbr[kMaxMoved];
  double msg[kMaxMoved], msign[kMaxMoved];
  double inv_s[kMaxRank];
  double bK[kBbMaxR];
  int ids[kBbMaxDeg], pos[kBbMaxDeg];  // the busbar's branches and their H-tile rows
  int rm[kBbMaxDeg], rmc[kBbMaxDeg];   // moved branches opened by the outage
  int k, kk, s, R, d, jb, skip, nrm;
  double M[kBbMaxR][kBbMaxR + 1];
  int piv[kBbMaxR];
  int perm[kBbMaxR];   // row q of the factors is row perm[q] of the system
  double pa[32];
};

// One thread per candidate: the genome parse shared by all busbar outages
// (same column order as the set-up kernel).
template <typename F>
__global__ __launch_bounds__(256) void k_bb_parse(GridDev g, BatchDev bt, SweepBufs<F> w,
                                                  BbCand* __restrict__ out) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= bt.B) return;
  BbCand& cd = out[c];
  if (w.info[c].status & (TTO_ST_ISLANDED | TTO_ST_INVALID)) { cd.k = 0; cd.s = 0; cd.nm = 0; return; }
  const int m = g.n_branch;
  int k = 0, s = 0, nm = 0;
  for (int i = 0; i < bt.no; ++i) {
    const int v = bt.open[(size_t)c * bt.no + i];
    if (v >= 0 && v < m && k < kMaxRank) cd.op[k++] = v;
  }
  for (int j = 0; j < bt.ns; ++j) {
    const int sb = bt.sbus[(size_t)c * bt.ns + j];
    if (sb == -1 || s >= kMaxRank) continue;
    cd.sbus[s] = sb;
    cd.sslot[s] = j;
    cd.moff[s] = nm;
    const int lo = bt.moff[(size_t)c * bt.ns + j], hi = bt.moff[(size_t)c * bt.ns + j + 1];
    for (int p = lo; p < hi && nm < kMaxMoved; ++p) {
      const int e = bt.mbr[p];
      cd.mbr[nm] = e;
      cd.msgn[nm] = g.from[e] == sb ? 1 : -1;
      cd.mb[nm] = g.b[e];
      ++nm;
    }
    ++s;
  }
  cd.moff[s] = nm;
  cd.k = k; cd.s = s; cd.nm = nm;
}

template <typename F, int TT>
__global__ __launch_bounds__(64) void k_bb_setup(GridDev g, BatchDev bt, SweepBufs<F> w,
                                                 BusbarDev bb, const double* __restrict__ P,
                                                 BusbarRecs<F> rr) {
  const int ib = blockIdx.x, c = blockIdx.y, tid = threadIdx.x;
  const int T = g.T, m = g.n_branch, nb = bb.nb;
  const size_t rec = (size_t)c * nb + ib;
  int* H = rr.hdr + rec * kBbHdr;
  __shared__ BbShared sh;
  const int status = w.info[c].status;
  if (status & (TTO_ST_ISLANDED | TTO_ST_INVALID)) {
    if (tid == 0) { H[0] = 0; H[1] = 0; H[2] = 0; H[3] = 2; }
    return;
  }
  const int bus = bb.bus[ib];
  __shared__ BbCand cd;
  {
    const int* src = (const int*)(rr.cand + c);
    int* dst = (int*)&cd;
    for (int i = tid; i < (int)(sizeof(BbCand) / 4); i += 64) dst[i] = src[i];
  }
  __syncthreads();
  // The outage's lists, one lane per element (the workgroup is one wave):
  // openings, the busbar's in-service branches, the moved lists without the
  // branches this outage opens, in the set-up kernel's order.
  {
    const int k = cd.k, s = cd.s, nmc = cd.nm;
    const unsigned long long below = (1ull << tid) - 1ull;
    if (tid < k) sh.op[tid] = cd.op[tid];
    if (tid < s) { sh.sbus[tid] = cd.sbus[tid]; sh.sslot[tid] = cd.sslot[tid]; }
    const unsigned long long jm = __ballot(tid < s && cd.sbus[tid] == bus);
    const int jb = jm ? 63 - __clzll(jm) : -1;
    // branches on the busbar's node: incident in the base grid, in service,
    // not moved to busbar B of a split of this bus (at most kBbMaxDeg)
    const int p0 = bb.inc_off[ib], n_inc = bb.inc_off[ib + 1] - p0;
    bool keep = false;
    int x = -1;
    if (tid < n_inc) {
      x = bb.inc_br[p0 + tid];
      bool off = false;
      for (int q = 0; q < k; ++q) off |= cd.op[q] == x;
      if (jb >= 0)
        for (int q = cd.moff[jb]; q < cd.moff[jb + 1]; ++q) off |= cd.mbr[q] == x;
      keep = !off;
    }
    const unsigned long long km = __ballot(keep);
    const int d = min(__popcll(km), kBbMaxDeg);
    const int rk = __popcll(km & below);
    if (keep && rk < kBbMaxDeg) { sh.ids[rk] = x; sh.pos[rk] = p0 + tid; }
    __syncthreads();
    const int kk = k + (d > 0 ? d - 1 : 0);
    if (tid + 1 < d) sh.op[k + tid] = sh.ids[tid];
    // moved branches: kept in their split, or opened by this outage (then
    // recorded with their index among the busbar's branches)
    bool kept = false, rem = false;
    int e = -1, jme = 0, here = -1;
    double sg = 0.0, mbv = 0.0;
    if (tid < nmc) {
      e = cd.mbr[tid];
      while (jme + 1 < s && cd.moff[jme + 1] <= tid) ++jme;
      sg = (double)cd.msgn[tid];
      mbv = cd.mb[tid];
      for (int q = 0; q + 1 < d; ++q) here = sh.ids[q] == e ? q : here;
      rem = here >= 0;
      kept = !rem;
    }
    const unsigned long long kmask = __ballot(kept), rmask = __ballot(rem);
    const int kr = __popcll(kmask & below), rr_ = __popcll(rmask & below);
    if (kept) { sh.mbr[kr] = e; sh.msign[kr] = sg; sh.msg[kr] = sg * mbv; }
    if (rem && rr_ < kBbMaxDeg) {
      sh.rm[rr_] = e;
      sh.rmc[rr_] = 2 * jme + (sg > 0.0 ? 1 : 0) + 256 * here;
    }
    if (tid <= s) {
      const int first = cd.moff[tid];
      sh.moff[tid] = __popcll(kmask & (first >= 64 ? ~0ull : (1ull << first) - 1ull));
    }
    if (tid < s) {
      double ssum = 0.0;
      for (int p = cd.moff[tid]; p < cd.moff[tid + 1]; ++p)
        if ((kmask >> p) & 1ull) ssum += cd.mb[p];
      sh.inv_s[tid] = ssum > 0.0 ? 1.0 / ssum : 0.0;
    }
    __syncthreads();
    if (tid < kk) sh.bK[tid] = g.b[sh.op[tid]];
    if (tid == 0) {
      sh.k = k; sh.kk = kk; sh.s = s; sh.R = kk + s; sh.d = d; sh.jb = jb;
      sh.nrm = min(__popcll(rmask), kBbMaxDeg);
    }
  }
  __syncthreads();
  const int k = sh.k, kk = sh.kk, R = sh.R, d = sh.d, jb = sh.jb;
  if (tid < TT) {
    double pa = 0.0;
    if (tid < T) {
      pa = P[(size_t)bus * T + tid];
      if (jb >= 0 && bt.mp) pa -= bt.mp[((size_t)c * bt.ns + sh.sslot[jb]) * T + tid];
    }
    sh.pa[tid] = pa;
  }
  // bordered matrix, as in the set-up with the extended opening list
  const size_t mm = m;
  for (int idx = tid; idx < R * R; idx += 64) {
    const int i = idx / R, q = idx - i * R;
    double v = 0.0;
    if (i < kk) {
      const size_t ki = (size_t)sh.op[i] * mm;
      if (q < kk) {
        v = (i == q ? 1.0 : 0.0) - sh.bK[i] * g.S[ki + sh.op[q]];
      } else {
        const int j = q - kk;
        for (int p = sh.moff[j]; p < sh.moff[j + 1]; ++p) v += sh.msg[p] * g.S[ki + sh.mbr[p]];
        v *= sh.bK[i];
      }
    } else {
      const int j = i - kk;
      if (q < kk) {
        for (int p = sh.moff[j]; p < sh.moff[j + 1]; ++p)
          v += sh.msg[p] * g.S[(size_t)sh.mbr[p] * mm + sh.op[q]];
      } else {
        const int j2 = q - kk;
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
  // LU with partial pivoting by one wave: the pivot row is the first row of
  // largest |entry| (shuffle arg-max), each lane eliminates its own row
  double minpiv = DBL_MAX;
  for (int p = 0; p < R; ++p) {
    double bv = (tid >= p && tid < R) ? fabs(sh.M[tid][p]) : -1.0;
    int bi = tid;
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(bv, off);
      const int oi = __shfl_xor(bi, off);
      if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
    }
    minpiv = fmin(minpiv, bv);
    if (bi != p && tid < R) {
      const double t = sh.M[p][tid];
      sh.M[p][tid] = sh.M[bi][tid];
      sh.M[bi][tid] = t;
    }
    if (tid == 0) sh.piv[p] = bi;
    __syncthreads();
    if (bv > 0.0 && tid > p && tid < R) {
      const double f = sh.M[tid][p] / sh.M[p][p];
      sh.M[tid][p] = f;
      for (int q = p + 1; q < R; ++q) sh.M[tid][q] -= f * sh.M[p][q];
    }
    __syncthreads();
  }
  if (tid == 0) {
    // the row interchanges composed: the factors hold whole swapped rows, so
    // the right-hand side is permuted once before the triangular solves
    for (int q = 0; q < R; ++q) sh.perm[q] = q;
    for (int p = 0; p < R; ++p) {
      const int pv = sh.piv[p];
      const int t = sh.perm[p]; sh.perm[p] = sh.perm[pv]; sh.perm[pv] = t;
    }
    sh.skip = (R > 0 && minpiv < kTauIsland) ? 1 : 0;
    H[0] = R; H[1] = k; H[2] = d; H[3] = sh.skip;
    for (int q = 0; q < kBbMaxDeg; ++q) {
      H[kBbIds + q] = q < d ? sh.ids[q] : -1;
      H[kBbRm + q] = q < sh.nrm ? sh.rm[q] : -1;
      H[kBbRmc + q] = q < sh.nrm ? sh.rmc[q] : -1;
      H[kBbPos + q] = q < d ? sh.pos[q] : -1;
    }
  }
  __syncthreads();
  F* z = rr.z + rec * kBbMaxR * TT;
  if (tid < TT) {
    rr.pa[rec * TT + tid] = (F)sh.pa[tid];
  }
  if (sh.skip) return;
  // z(t) = M^{-1} rhs(t) with the base flows shifted by the lost injection;
  // every index into x is a compile-time constant, so x stays in registers
  if (tid < TT) {
    const int t = tid;
    double x[kBbMaxR];
#pragma unroll
    for (int q = 0; q < kBbMaxR; ++q) x[q] = 0.0;
    if (t < T) {
      const double pa = sh.pa[t];
      const double* PBr = bb.PB + (size_t)ib * m;
#pragma unroll
      for (int q = 0; q < kBbMaxR; ++q) {
        if (q < R) {
          const int row = sh.perm[q];
          double v;
          if (row < kk) {
            const int x0 = sh.op[row];
            v = g.f0[(size_t)x0 * T + t] - PBr[x0] * pa;
          } else {
            const int j = row - kk;
            double phi = 0.0;
            for (int p = sh.moff[j]; p < sh.moff[j + 1]; ++p) {
              const int e = sh.mbr[p];
              phi += sh.msign[p] * (g.f0[(size_t)e * T + t] - PBr[e] * pa);
            }
            const double pj = bt.mp ? bt.mp[((size_t)c * bt.ns + sh.sslot[j]) * T + t] : 0.0;
            v = (pj - phi) * sh.inv_s[j];
          }
          x[q] = v;
        }
      }
#pragma unroll
      for (int p = 0; p < kBbMaxR; ++p) {
        if (p < R) {
#pragma unroll
          for (int i = p + 1; i < kBbMaxR; ++i)
            if (i < R) x[i] -= sh.M[i][p] * x[p];
        }
      }
#pragma unroll
      for (int p = kBbMaxR - 1; p >= 0; --p) {
        if (p < R) {
          double v = x[p];
#pragma unroll
          for (int q = p + 1; q < kBbMaxR; ++q)
            if (q < R) v -= sh.M[p][q] * x[q];
          x[p] = v / sh.M[p][p];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < kBbMaxR; ++q) z[(size_t)q * TT + t] = (F)x[q];
  }
}

template <typename F, int TT>
__global__ __launch_bounds__(256) void k_bb_sweep(GridDev g, SweepBufs<F> w, BusbarDev bb,
                                                  BusbarRecs<F> rr, int n_eblk) {
  const int c = blockIdx.y, eb = blockIdx.x, tid = threadIdx.x;
  const int nM = g.nM, T = g.T, nb = bb.nb;
  const CandInfo* inf = w.info + c;
  const bool bad = inf->status & (TTO_ST_ISLANDED | TTO_ST_INVALID);
  const int ei = eb * 256 + tid;
  const bool valid = ei < nM && !bad;
  const int ei_c = ei < nM ? ei : nM - 1;
  const int e = g.mon[ei_c];
  const int kc = bad ? 0 : inf->k, rc = bad ? 0 : inf->r;
  bool opened = false;
  for (int q = 0; q < kc; ++q) opened |= (inf->open_br[q] == e);
  F U[kVSlots];
  const F* ua = w.UM + (size_t)c * kVSlots * nM + ei_c;
#pragma unroll
  for (int q = 0; q < kVSlots; ++q) U[q] = q < rc ? ua[(size_t)q * nM] : (F)0;
  F f0e[TT], acc[TT];
#pragma unroll
  for (int t = 0; t < TT; ++t) { f0e[t] = t < T ? (F)g.f0[(size_t)e * T + t] : (F)0; acc[t] = (F)0; }
  const F* HB;
  const F* PBM;
  if constexpr (sizeof(F) == 4) { HB = bb.HB32; PBM = bb.PBM32; } else { HB = bb.HB; PBM = bb.PBM; }
  // records staged through LDS, double-buffered: the workgroup loads outage
  // ib + 1 into registers (coalesced) while it computes outage ib from LDS
  constexpr int ZN = kBbMaxR * TT, ZP = ZN + TT;
  constexpr int PER = (ZP + 255) / 256;
  __shared__ F zs[2][ZP];
  __shared__ int hs[2][kBbHdr];
  F rz[PER];
  int rh = 0;
  auto fetch = [&](int ib) {
    const size_t rec = (size_t)c * nb + ib;
    const F* zsrc = rr.z + rec * ZN;
    const F* psrc = rr.pa + rec * TT;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int i = tid + 256 * u;
      rz[u] = i < ZN ? zsrc[i] : (i < ZP ? psrc[i - ZN] : (F)0);
    }
    if (tid < kBbHdr) rh = rr.hdr[rec * kBbHdr + tid];
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int i = tid + 256 * u;
      if (i < ZP) zs[buf][i] = rz[u];
    }
    if (tid < kBbHdr) hs[buf][tid] = rh;
  };
  if (!bad && nb > 0) {
    fetch(0);
    stash(0);
  }
  __syncthreads();
  for (int ib = 0; ib < nb && !bad; ++ib) {
    const int buf = ib & 1;
    if (ib + 1 < nb) fetch(ib + 1);
    const int* H = hs[buf];
    if (H[3] == 0) {
      const int k = H[1], d = H[2];
      const int kk = k + (d > 0 ? d - 1 : 0);
      bool removed = opened;
      for (int q = 0; q < d; ++q) removed |= H[kBbIds + q] == e;
      const F* z = zs[buf];
      const F* pa = zs[buf] + ZN;
      const F pb = PBM[(size_t)ib * nM + ei_c];
      F f[TT];
#pragma unroll
      for (int t = 0; t < TT; ++t) f[t] = f0e[t] - pb * pa[t];
#pragma unroll
      for (int q = 0; q < kMaxRank; ++q) {
        if (q < k) {
          const F u = U[q];
#pragma unroll
          for (int t = 0; t < TT; ++t) f[t] += u * z[q * TT + t];
        }
      }
      for (int q = k; q < kk; ++q) {
        const F u = HB[(size_t)H[kBbPos + q - k] * nM + ei_c];
#pragma unroll
        for (int t = 0; t < TT; ++t) f[t] += u * z[q * TT + t];
      }
      // split columns without the moved branches the outage opens:
      // u_j(e) + b_e msg_r S_re for each such branch r of split j
      F uj[kMaxRank];
#pragma unroll
      for (int j = 0; j < kMaxRank; ++j) uj[j] = (k + j < rc) ? U[k + j] : (F)0;
      for (int q = 0; q < kBbMaxDeg; ++q) {
        const int r = H[kBbRm + q];
        if (r < 0) break;
        const int code = H[kBbRmc + q];
        const F msg = (code & 1 ? (F)1 : (F)-1) * (F)g.b[r];
        const F add = msg * HB[(size_t)H[kBbPos + (code >> 8)] * nM + ei_c];
        const int jr = (code >> 1) & 127;
#pragma unroll
        for (int j = 0; j < kMaxRank; ++j)
          if (j == jr) uj[j] += add;
      }
#pragma unroll
      for (int j = 0; j < kMaxRank; ++j) {
        if (k + j < rc) {
          const F u = uj[j];
          const int q = kk + j;
#pragma unroll
          for (int t = 0; t < TT; ++t) f[t] += u * z[q * TT + t];
        }
      }
      if (!removed) {
#pragma unroll
        for (int t = 0; t < TT; ++t) {
          const F v = f[t] < (F)0 ? -f[t] : f[t];
          acc[t] = acc[t] > v ? acc[t] : v;
        }
      }
    }
    __syncthreads();                      // everyone is done with buffer buf
    if (ib + 1 < nb) stash(buf ^ 1);
    __syncthreads();
  }
  double ov = 0.0;
  if (valid) {
    const double lim = g.lim[e];
    for (int t = 0; t < T && t < TT; ++t) {
      const double v = (double)acc[t] - lim;
      if (v > 0.0) ov += v;
    }
  }
  for (int off = 32; off > 0; off >>= 1) ov += __shfl_xor(ov, off);
  __shared__ double s_w[4];
  if ((tid & 63) == 0) s_w[tid >> 6] = ov;
  __syncthreads();
  if (tid == 0) rr.part[(size_t)c * n_eblk + eb] = ((s_w[0] + s_w[1]) + s_w[2]) + s_w[3];
}

template <typename F>
__global__ __launch_bounds__(256) void k_bb_finalize(SweepBufs<F> w, BusbarDev bb,
                                                     BusbarRecs<F> rr, int B, int n_eblk,
                                                     double pre, const double* __restrict__ f1,
                                                     double* __restrict__ lam,
                                                     int* __restrict__ n_isl,
                                                     double* __restrict__ f2) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= B) return;
  const bool bad = w.info[c].status & (TTO_ST_ISLANDED | TTO_ST_INVALID);
  double sum = 0.0;
  for (int b = 0; b < n_eblk; ++b) sum += rr.part[(size_t)c * n_eblk + b];
  int cnt = 0;
  for (int ib = 0; ib < bb.nb; ++ib) cnt += rr.hdr[((size_t)c * bb.nb + ib) * kBbHdr + 3] == 1;
  if (lam) lam[c] = bad ? __builtin_nan("") : sum;
  if (n_isl) n_isl[c] = bad ? 0 : cnt;
  if (f2 && f1) f2[c] = bad ? -__builtin_inf() : f1[c] - fmax(sum - pre, 0.0);
}

template <typename F, int TT>
hipError_t launch_busbar_tt(const GridDev& g, const BatchDev& bt, const SweepBufs<F>& w,
                            const BusbarDev& bb, const BusbarRecs<F>& rr, const double* P,
                            double pre, const double* f1, double* lam, int* n_isl, double* f2,
                            hipStream_t s) {
  const int n_eblk = (g.nM + 255) / 256;
  if (bb.nb > 0) {
    hipLaunchKernelGGL((k_bb_parse<F>), dim3((bt.B + 255) / 256), dim3(256), 0, s, g, bt, w, rr.cand);
    hipLaunchKernelGGL((k_bb_setup<F, TT>), dim3(bb.nb, bt.B), dim3(64), 0, s, g, bt, w, bb, P, rr);
  }
  hipLaunchKernelGGL((k_bb_sweep<F, TT>), dim3(n_eblk, bt.B), dim3(256), 0, s, g, w, bb, rr,
                     n_eblk);
  hipLaunchKernelGGL((k_bb_finalize<F>), dim3((bt.B + 255) / 256), dim3(256), 0, s, w, bb, rr,
                     bt.B, n_eblk, pre, f1, lam, n_isl, f2);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_busbar_tables(const double* ptdf, int n_bus, int m, const int* mon, int nM,
                                const int* bus, int nb, double* PB, double* PBM, float* PBM32,
                                const double* S, const double* b, const int* inc_br, int n_inc,
                                double* HB, float* HB32, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bb_tables, dim3((m + 255) / 256, nb), dim3(256), 0, s, ptdf, n_bus, m,
                     mon, nM, bus, nb, PB, PBM, PBM32);
  if (n_inc > 0)
    hipLaunchKernelGGL(k_bb_htile, dim3((nM + 255) / 256, n_inc), dim3(256), 0, s, S, b, mon, nM,
                       m, inc_br, HB, HB32);
  return hipGetLastError();
}

template <typename F>
hipError_t launch_busbar(const GridDev& g, const BatchDev& bt, const SweepBufs<F>& w,
                         const BusbarDev& bb, const BusbarRecs<F>& rr, const double* P,
                         double pre, const double* f1, double* lam, int* n_isl, double* f2,
                         hipStream_t s) {
  switch (g.TT) {
    case 1: return launch_busbar_tt<F, 1>(g, bt, w, bb, rr, P, pre, f1, lam, n_isl, f2, s);
    case 8: return launch_busbar_tt<F, 8>(g, bt, w, bb, rr, P, pre, f1, lam, n_isl, f2, s);
    case 24: return launch_busbar_tt<F, 24>(g, bt, w, bb, rr, P, pre, f1, lam, n_isl, f2, s);
    default: return launch_busbar_tt<F, 32>(g, bt, w, bb, rr, P, pre, f1, lam, n_isl, f2, s);
  }
}

template hipError_t launch_busbar<float>(const GridDev&, const BatchDev&, const SweepBufs<float>&,
                                         const BusbarDev&, const BusbarRecs<float>&,
                                         const double*, double, const double*, double*, int*,
                                         double*, hipStream_t);
template hipError_t launch_busbar<double>(const GridDev&, const BatchDev&,
                                          const SweepBufs<double>&, const BusbarDev&,
                                          const BusbarRecs<double>&, const double*, double,
                                          const double*, double*, int*, double*, hipStream_t);

}  // namespace tto
