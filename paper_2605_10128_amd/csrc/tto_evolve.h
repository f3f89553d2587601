// Device side of the MapElites generation (DC-Optimizer: Repertoire design,
// Mutation Alg. 1, Crossover Alg. 2, High-level loop Alg. 3).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tto {

constexpr int kGenomeSlots = 8;      // per kind (action, disconnection)
constexpr int kMaxCells = 4096;      // repertoire cells compacted in LDS by k_vary

// Genome tables and operator parameters.  Actions are addressed in "station
// order" (ascending (bus, action id)); the actions of one substation form one
// contiguous range of station positions.
struct GenomeDev {
  int n_a, n_d, n_actions, n_disc, max_len;
  const int* st_order;   // [n_actions] station position -> action id
  const int* pos;        // [n_actions] action id -> station position
  const int* first;      // [n_actions] first station position of the action's substation
  const int* count;      // [n_actions] number of actions at that substation
  const int* bus;        // [n_actions]
  const int* moff;       // [n_actions + 1] moved-branch CSR
  const int* mbr;
  const int* disc;       // [n_disc] branch id of each disconnection
  int w_act[4];          // Add, Remove, Change, Identity
  int w_disc[4];
  unsigned long long thr_c1;               // parent 1 iff draw < thr_c1 (<= 2^32)
  unsigned long long poisson[kGenomeSlots]; // floor(P(K <= k) 2^32), k = 1 .. n_a - 1
};

hipError_t launch_vary(const GenomeDev& gd, const int64_t* elite_id, const int* elite_genome,
                       int n_cells, uint64_t seed, const int64_t* generation, int n_child,
                       int* children, int* b_mc, hipStream_t s);

hipError_t launch_expand(const GenomeDev& gd, const int* genomes, int n, int* open, int* sbus,
                         int* moff, int* mbr, hipStream_t s);

// Insertion with genomes; the new elite's id is generation * id_stride +
// (id_map ? id_map[i] : i) for batch entry i.
hipError_t launch_archive_genome(double* elite_fit, int64_t* elite_id, int* elite_genome,
                                 int n_cells, const double* fit, const int* cell,
                                 const uint8_t* status, int B, const int64_t* generation,
                                 const int* genomes, int G, const int* id_map, int id_stride,
                                 unsigned long long* key, int* idx, hipStream_t s);

hipError_t launch_generation_bump(int64_t* generation, hipStream_t s);

// Screened generation helpers: the network's feature rows from genomes
// (off [n+1], ids [n*G]), one dense row broadcast to n rows, the k chosen
// children (idx) listed in increasing index order (mask [n] scratch), and a
// row gather dst[i] = src[list[i]].
hipError_t launch_genome_bits(const GenomeDev& gd, const int* genomes, int n, int* off, int* ids,
                              hipStream_t s);
hipError_t launch_broadcast_row(const float* row, int d, int n, float* out, hipStream_t s);
hipError_t launch_keep_in_order(const int* idx, int k, int n, int* mask, int* list, hipStream_t s);
hipError_t launch_gather_rows(const int* src, const int* list, int k, int G, int* dst,
                              hipStream_t s);

// Archive-aware screen: the network's outputs de-standardised (raw = y sd +
// mu + ref), the descriptor of the grid, the repertoire's cells.  Step 1
// predicts each child's cell, fitness and whether it would enter; the
// per-cell winners among those come from the archive's winner kernels; step
// 2 ranks the winners first and every other child by its overload term.
struct ScreenScoreCfg {
  double mu[2], sd[2], ref[2];
  double overload_scale;
  int desc_kind, n_count_bins, n_load_bins, n_cells;
};
hipError_t launch_screen_predict(const GenomeDev& gd, const int* genomes, int n, const float* y,
                                 const ScreenScoreCfg& sc, const double* edges,
                                 const double* elite_fit, const int64_t* elite_id,
                                 double* fit_pred, int* cell_pred, uint8_t* st_pred,
                                 hipStream_t s);
hipError_t launch_screen_tier(const float* y, const int* cell_pred, const uint8_t* st_pred,
                              const int* winner, int n, float* score, hipStream_t s);
// Per-cell winners of a batch (best fitness among entries whose status has
// neither ISLANDED nor INVALID, ties to the lowest index; INT_MAX if none).
hipError_t launch_cell_winners(int n_cells, const double* fit, const int* cell,
                               const uint8_t* status, int B, unsigned long long* key, int* idx,
                               hipStream_t s);

}  // namespace tto
