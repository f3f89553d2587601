// Busbar outages (Fitness function heuristics: busbar penalty lambda_b;
// High-level loop: lambda_f2) on the device.
#pragma once

#include "tto_common.h"

namespace tto {

constexpr int kBbMaxDeg = 16;                        // branches on one busbar
constexpr int kBbMaxR = kMaxRank + kBbMaxDeg - 1;    // candidate rank + busbar openings
// record header: R, k, d, state (0 solved, 1 islanding, 2 candidate skipped),
// the busbar's branches (kBbMaxDeg ids), the moved branches that the outage
// removes from their split (kBbMaxDeg ids, kBbMaxDeg codes 2 j + (sg > 0) +
// 256 q with q the branch's index among the busbar's branches), and the
// busbar's branches' positions in the set's H tile (kBbMaxDeg)
constexpr int kBbHdr = 4 + 4 * kBbMaxDeg;
constexpr int kBbIds = 4, kBbRm = 4 + kBbMaxDeg, kBbRmc = 4 + 2 * kBbMaxDeg,
              kBbPos = 4 + 3 * kBbMaxDeg;

// Busbar set: the buses whose (main) busbar can fail, their base-grid
// incident branches and the PTDF columns of those buses.
struct BusbarDev {
  int nb;
  const int* bus;       // [nb]
  const int* inc_off;   // [nb + 1]
  const int* inc_br;    // incident branch ids (base grid)
  const double* PB;     // [nb][m]  PTDF_{x, bus}
  const double* PBM;    // [nb][nM] PTDF_{mon[ei], bus}
  const float* PBM32;   // the same in FP32
  int n_inc;
  const double* HB;     // [n_inc][nM] H_{mon[ei], inc_br[p]} = b_e S_{e, x}
  const float* HB32;    // the same in FP32
};

// A candidate's genome parsed once for all its busbar outages (openings in
// slot order, splits in slot order with their moved branches).
struct BbCand {
  int k, s, nm, pad;
  int op[kMaxRank];
  int sbus[kMaxRank], sslot[kMaxRank];
  int moff[kMaxRank + 1];
  int pad2[3];
  int mbr[kMaxMoved];
  int msgn[kMaxMoved];       // +1 if the branch leaves the split bus
  double mb[kMaxMoved];      // susceptance of each moved branch
};

// Per (candidate, busbar) solution of the bordered system.
template <typename F>
struct BusbarRecs {
  BbCand* cand;   // [B]
  int* hdr;   // [B][nb][kBbHdr]
  F* z;       // [B][nb][kBbMaxR][TT]
  F* pa;      // [B][nb][TT] injection lost with the busbar
  double* part;   // [B][n_eblk] tile sums of lambda_b
};

hipError_t launch_busbar_tables(const double* ptdf, int n_bus, int m, const int* mon, int nM,
                                const int* bus, int nb, double* PB, double* PBM, float* PBM32,
                                const double* S, const double* b, const int* inc_br, int n_inc,
                                double* HB, float* HB32, hipStream_t s);

template <typename F>
hipError_t launch_busbar(const GridDev& g, const BatchDev& bt, const SweepBufs<F>& w,
                         const BusbarDev& bb, const BusbarRecs<F>& rr, const double* P,
                         double lambda_b_pre, const double* fit_f1, double* lambda_b,
                         int* n_island, double* fit_f2, hipStream_t s);

}  // namespace tto
