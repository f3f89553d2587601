// Busbar outages (Fitness function heuristics: busbar penalty lambda_b;
// High-level loop: lambda_f2) on the device.
#pragma once

#include "tto_common.h"

namespace tto {

constexpr int kBbMaxDeg = 16;                        // branches on one busbar
constexpr int kBbMaxR = kMaxRank + kBbMaxDeg - 1;    // candidate rank + busbar openings
// record header: R, k, d, state (0 solved, 1 islanding, 2 candidate skipped),
// the busbar's branches (kBbMaxDeg), then the moved branches that the outage
// removes from their split (kBbMaxDeg ids and kBbMaxDeg codes 2 j + (sg > 0))
constexpr int kBbHdr = 4 + 3 * kBbMaxDeg;

// Busbar set: the buses whose (main) busbar can fail, their base-grid
// incident branches and the PTDF columns of those buses.
struct BusbarDev {
  int nb;
  const int* bus;       // [nb]
  const int* inc_off;   // [nb + 1]
  const int* inc_br;    // incident branch ids (base grid)
  const double* PB;     // [nb][m]  PTDF_{x, bus}
  const double* PBM;    // [nb][nM] PTDF_{mon[ei], bus}
};

// Per (candidate, busbar) solution of the bordered system.
template <typename F>
struct BusbarRecs {
  int* hdr;   // [B][nb][kBbHdr]
  F* z;       // [B][nb][kBbMaxR][TT]
  F* pa;      // [B][nb][TT] injection lost with the busbar
  double* part;   // [B][n_eblk] tile sums of lambda_b
};

hipError_t launch_busbar_tables(const double* ptdf, int n_bus, int m, const int* mon, int nM,
                                const int* bus, int nb, double* PB, double* PBM, hipStream_t s);

template <typename F>
hipError_t launch_busbar(const GridDev& g, const BatchDev& bt, const SweepBufs<F>& w,
                         const BusbarDev& bb, const BusbarRecs<F>& rr, const double* P,
                         double lambda_b_pre, const double* fit_f1, double* lambda_b,
                         int* n_island, double* fit_f2, hipStream_t s);

}  // namespace tto
