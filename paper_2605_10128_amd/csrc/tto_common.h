// Internal declarations shared by the HIP translation units of libtto.
// gfx950 only: 64-lane wavefronts, MFMA, 160 KB LDS per CU.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/tto.h"

namespace tto {

constexpr int kWave = 64;
constexpr int kMaxRank = TTO_MAX_RANK;
constexpr int kMaxMoved = TTO_MAX_MOVED;
constexpr int kVSlots = 8;          // V entries per contingency record
constexpr double kTauIsland = 1e-9; // |pivot| of the scaled bordered system
constexpr double kTauCont = 1e-9;   // |1 - H'_ll| of a contingency
constexpr double kWorstContTieMW = TTO_WORST_CONT_TIE_MW;  // worst-contingency tie tolerance
constexpr double kLoadTieRel = TTO_LOAD_TIE_REL;          // worst (branch, timestep) tie band
constexpr int kGemmN = 32;          // timestep columns of the f0 GEMM (T padded)
constexpr int kSubMax = 32;         // gather sources whose mutual S entries the set-up stages in LDS
constexpr int kMaxSrc = kMaxRank + kMaxMoved;   // gather sources of a candidate
static_assert(kMaxSrc % 8 == 0, "sources are read in groups of 8");

// Record of one active contingency in a candidate's sweep list: phi(t) for
// t < TT, then V_j for j < r, padded to a multiple of 4 entries.  A
// candidate of rank r packs its records at rec_stride_r(TT, r) within its
// region of the record table, whose size per candidate is set by the largest
// stride, rec_stride(TT) (r = 8).
__host__ __device__ constexpr int rec_stride_r(int TT, int r) { return ((TT + r + 3) / 4) * 4; }
__host__ __device__ constexpr int rec_stride(int TT) { return rec_stride_r(TT, kVSlots); }

// Timestep tile used by the templated kernels: smallest supported >= T.
inline int tile_T(int T) {
  if (T <= 1) return 1;
  if (T <= 8) return 8;
  if (T <= 24) return 24;
  return 32;
}

struct GridDev {
  int n_bus, n_branch, slack, T, TT, nM, nC;
  const int* from;
  const int* to;
  const double* b;
  const double* lim;
  // S = A L^-1 A^T, symmetric [m][m]; the flow on e per MW sent across l is
  // H_el = b_e S_el, so any row or column of H is a contiguous row of S.
  const double* S;
  // S restricted to the monitored then contingency columns, [m][nM + nC]:
  // column gathers of a candidate's rows are contiguous across threads
  const double* SMC;
  const float* HMC32;   // [nC][nM], H[M[ei], C[li]] with -1 where M[ei] == C[li]
  const double* HMC64;  // same in FP64
  const double* f0;     // [m][T] base flows of the unswitched grid (GEMM precision)
  const double* f0_hi;  // [m][T] the same from the FP64 GEMM (refinement pass)
  const int* mon;       // [nM]
  const int* cont;      // [nC]
  // Tables of the monitored then contingency rows, contiguous in the row
  // index so that the lanes of a row loop read them coalesced:
  const double* f0MC;     // [TT][nM + nC] base flows f0 at row j, zero rows past T
  const double* f0MC_hi;  // the same from f0_hi
  const float* f0M32;     // [TT][nM] f0 of the monitored rows in FP32, zero rows past T
  const double* bMC;      // [nM + nC] susceptance of row j
  const double* limM;     // [nM] limit of M[ei]
  const double* sllC;     // [nC] S_ll of l = C[li]
  const double* edges;  // [n_load_bins - 1]
  double lim_min;       // smallest monitored limit
  int n_count_bins, n_load_bins;
  int desc_kind;        // TTO_DESC_*
  double w_c0, w_c;
  // Decision margin of an FP32 pass that queues FP64 refinement (< 0: none):
  // near_margin + 4 max|f0 - f0_hi| MW, the second term read from gemm_err
  // (device scalar written with the base flows; NULL when f0 is FP64).
  double near_margin;
  const double* gemm_err;
};

// Decision margin in MW of the current pass (negative: no refinement).
__device__ inline double decision_margin(const GridDev& g) {
  if (g.near_margin < 0.0) return -1.0;
  return g.near_margin + (g.gemm_err ? 4.0 * *g.gemm_err : 0.0);
}

struct BatchDev {
  int B, no, ns;
  int n_genomes;      // rows of the genome arrays (B of the caller's batch)
  const int* open;
  const int* sbus;
  const int* moff;
  const int* mbr;
  const double* mp;
  // refinement pass: workgroup c < min(*live, B) evaluates genome map[c]
  const int* map;
  const int* live;
};

// FP32 pass -> FP64 refinement hand-over.
struct RefineCtl {
  int* list;        // [cap] candidates to re-evaluate in FP64, in index order
  int* count;       // number flagged (may exceed cap)
  int* flags;       // [B] 1 if the candidate's FP32 decisions are near a threshold
  unsigned long long* fbuf;   // [cap][TT][nM] f^max bit patterns of the FP64 pass
  int cap;
  double margin;    // flow error margin in MW
};

// Per-candidate summary written by the set-up kernel.
struct CandInfo {
  int status;      // TTO_ST_* bits
  int r;           // filled slots (openings + splits)
  int k;           // openings
  int n_act;       // active (non-islanding) contingencies
  int n_act_pad;   // n_act rounded up to even (duplicate of the last record)
  int n_island;    // islanding contingencies
  int n_crit_n0;   // lambda_c0 from the FP64 post-switch flows
  int n_moved;     // branches moved by the candidate's splits (reassigned assets)
  int open_br[kMaxRank];
};

// Per-candidate description left by the first set-up kernel for the second:
// the gather sources (openings, then moved branches) with their coefficients
// for W_q (the column of U before the b_e factor) and for the pivoted
// right-hand side of V_l, the LU factors of the bordered system, x(t) and
// the moved-branch fix-ups.  Coefficient rows past nsrc are zero up to the
// next multiple of 8.
struct SetupDesc {
  int status;              // 0, or the TTO_ST_* bits of a candidate with no row work
  int r, k, ns, nsrc, nm;  // rank, openings, splits, sources, moved branches
  int bad;                 // x(t) not finite
  int pad_;
  int open[kMaxRank];      // opened branches, -1 past k
  int src_row[kMaxSrc];
  int mbr[kMaxMoved];      // moved branches
  int mslot[kMaxMoved];    // their split's slot k + j
  int mpos[kMaxMoved];     // that slot's row in the pivoted order
  double msg[kMaxMoved];   // sg_b b_b
  double madd[kMaxMoved];  // sg_b / s_j
  double uscale[kMaxRank]; // +1 openings, -1 splits: U_q = uscale_q b_e W_q
  double coefW[kMaxSrc][kMaxRank];
  double coefV[kMaxSrc][kMaxRank];
  double LU[kMaxRank][kMaxRank];   // unit L below the diagonal, U on and above
  double inv_diag[kMaxRank];
  double x[32][kMaxRank];          // x(t), zero for t >= T
  float x32[32][kMaxRank];         // x(t) rounded to FP32 (the FP32 flows' f'_M)
};

// Per (candidate, monitored block) reduction of the sweep.
struct Partial {
  double sum_o;     // sum of max(fmax - lim, 0)
  double best;      // max loading in this block
  double best2;     // second largest loading (another (e, t)) in this block
  int cnt_c;        // fmax > lim count
  int best_e;       // smallest (monitored index, timestep) within the tie band
                    // of this block's max loading
  int best_t;
  int pad_;
};

// Batch workspace views (carved from the caller's batch workspace).
template <typename F>
struct SweepBufs {
  CandInfo* info;   // [B]
  F* UM;            // [B][8][nM] rank-r factor rows (slots past r not written)
  F* rec;           // [B][(nC+1) rec_stride(TT)]: records at rec_stride_r(TT, r)
  int* act;         // [B][nC+1] contingency index of each record
  int* slot;        // [B][nC] record of each contingency or -1 (optional)
  Partial* part;    // [B][n_eblk] one per chunk of 64 monitored branches
  SetupDesc* desc;  // [B] set-up description of each candidate
  int n_eblk;       // ceil(nM / 64)
};

// Launch shape of the N-1 sweep (chosen by the autotuner).  The unit of
// work is one wave: a candidate and npl chunks of 64 monitored branches.
struct SweepPlan {
  int lanes;        // workgroup size: 256 (four independent waves)
  int npl;          // monitored branches per lane: 1 or 2 (2: FP32 flows only)
  int order;        // 0 hardware, 1 XCD candidate-major, 2 XCD chunk-major
};

// ---- launchers (k_grid.hip) -------------------------------------------------
hipError_t launch_build_S(const double* ptdf, const int* from, const int* to, const double* b,
                          int m, int n, double* S, hipStream_t s);
hipError_t launch_build_SMC(const double* S, const int* mon, const int* cont, int m, int nM,
                            int nC, double* SMC, hipStream_t s);
hipError_t launch_build_HMC(const double* S, const double* b, const int* mon, const int* cont,
                            int m, int nM, int nC, float* HMC32, double* HMC64, hipStream_t s);
hipError_t launch_build_rows(const double* S, const double* b, const double* lim, const int* mon,
                             const int* cont, int m, int nM, int nC, double* bMC, double* limM,
                             double* sllC, hipStream_t s);
hipError_t launch_f0_rows(const double* f0, const int* mon, const int* cont, int T, int nM, int nC,
                          double* f0MC, float* f0M32, hipStream_t s);
hipError_t launch_convert_ptdf(const double* ptdf, int m, int n, int prec, void* out, hipStream_t s);
hipError_t launch_pack_injections(const double* p, int n, int T, int prec, void* PT, hipStream_t s);
hipError_t launch_gemm_f0(int prec, const void* A, const void* PT, int m, int n, int T,
                          int ksplit, float* part32, double* part64, double* f0, hipStream_t s);
hipError_t launch_max_abs_diff(const double* a, const double* b, size_t n, double* out,
                               hipStream_t s);
int gemm_ksplit(int m, int n);

// ---- launchers (k_eval.hip) -------------------------------------------------
// ev: NULL or 5 events recorded before set-up, after set-up, after the sweep,
// after finalize and after the FP64 refinement pass.  rw/rc: refinement
// buffers and control (FP32 flows only; rc.cap == 0 disables).
// importer on the device (k_ptdf.hip)
int gj_padded(int n_bus);
hipError_t launch_ptdf(const int* off, const int* nbr, const double* wgt, int n, int m,
                       int slack, const int* from, const int* to, const double* b, double* A,
                       double* Pbuf, double* ptdf, hipStream_t s);
hipError_t launch_bridges(const double* S, const double* b, int m, uint8_t* out, hipStream_t s);

template <typename F>
hipError_t launch_setup(const GridDev& g, const BatchDev& bt, const SweepBufs<F>& w,
                        hipStream_t s);
template <typename F>
hipError_t launch_worst_k(const GridDev& g, const BatchDev& bt, const SweepBufs<F>& w, int kk,
                          int* ids, double* energy, double* part, hipStream_t s);
template <typename F>
hipError_t launch_evaluate(const GridDev& g, const BatchDev& bt, const SweepBufs<F>& w,
                           const tto_outputs& out, hipStream_t s, hipEvent_t* ev,
                           const SweepPlan& plan, const SweepBufs<double>* rw,
                           const RefineCtl& rc);
// Allocation-free insertion: cells covered by the static scratch, its set-up
// (once per device, that device current) and its device address (NULL before).
constexpr int kArchiveStaticCells = 65536;
hipError_t archive_scratch_init(int device);
void* archive_scratch(int device);
hipError_t launch_archive(double* elite_fit, int64_t* elite_id, int n_cells, const double* fit,
                          const int* cell, const uint8_t* status, int B, int64_t id_base,
                          unsigned long long* key, int* idx, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, size_t n, hipStream_t s);

}  // namespace tto
