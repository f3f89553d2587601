/*
 * tto.h - C ABI of the MI355X (gfx950) batched DC N-1 topology screen.
 *
 * The library scores batches of candidate grid topologies the way the
 * DC-Optimizer of "Transmission Topology Optimization using accelerated
 * MapElites" does inside its MapElites loop (Alg. 3 "Accelerated MapElites
 * for TTO": compute N-1 DC loadflows, then lambda and beta, for a batch of new
 * individuals, then insert into the repertoire):
 *
 *   grid PTDF + nodal injections in; candidate branch openings and bus splits
 *   in; per-candidate base flows, N-1 flow maxima, overload metrics, fitness
 *   and MapElites descriptor cell out; per-cell elites updated on device.
 *
 * Conventions (all entry points):
 *   - Plain C types only.  "device" pointers point to GPU memory of the
 *     current HIP device; "host" pointers to CPU memory.
 *   - Every device buffer is owned by the caller.  The library keeps only a
 *     small host handle (tto_grid) that remembers pointers into the caller's
 *     grid workspace; that workspace must stay alive and untouched until
 *     tto_grid_destroy.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     Calls are asynchronous on that stream unless stated otherwise.
 *   - Every call returns a tto_status; no C++ exception crosses the ABI.  On
 *     error, tto_last_error() returns a thread-local message.  Argument errors
 *     are detected on the host before any kernel is launched.  Per-candidate
 *     problems never fail a batch: they set status bits instead.
 */
#ifndef TTO_H
#define TTO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TTO_VERSION_MAJOR 1
#define TTO_VERSION_MINOR 1

#define TTO_MAX_RANK 8      /* openings + splits per candidate */
#define TTO_MAX_T 32        /* timesteps per injection set */
#define TTO_MAX_MOVED 64    /* moved branches summed over a candidate's splits */
#define TTO_MAX_LOAD_BINS 64
/* Worst contingency: the first contingency (in the order of the contingency
 * list) whose |flow| on the worst branch at the worst timestep is within this
 * many MW of the maximum.  Branches whose flow no contingency changes (bridges
 * of the post-switch grid) tie exactly, and the order of the list, not
 * rounding, then picks the reported contingency. */
#define TTO_WORST_CONT_TIE_MW 0.05
/* Worst (branch, timestep): the smallest (monitored position, timestep) whose
 * loading is at least max_loading * (1 - TTO_LOAD_TIE_REL).  Branches of a
 * two-branch cut with equal limits, for instance, carry the same maximum
 * loading exactly (each carries the cut's transfer when the other is out),
 * and the monitored order, not rounding, then picks the reported branch. */
#define TTO_LOAD_TIE_REL 1e-9

typedef int32_t tto_status;
enum {
  TTO_OK = 0,
  TTO_E_INVALID = -1,     /* NULL pointer, size or enum out of range */
  TTO_E_GRID = -2,        /* bad grid: index out of range, non-positive
                             susceptance/limit, disconnected base grid,
                             duplicate monitored/contingency id */
  TTO_E_RANK = -3,        /* slot counts beyond TTO_MAX_RANK per kind */
  TTO_E_WORKSPACE = -4,   /* workspace NULL, misaligned or too small */
  TTO_E_HIP = -5,         /* a HIP runtime call failed */
  TTO_E_UNSUPPORTED = -6  /* valid request the library does not implement */
};

/* Arithmetic of the flows (N-0 and N-1 sweep).  Candidate set-up (the rank-r
 * bordered system, its LU with the islanding pivot test, the LODF
 * denominators 1 - H'_ll and the contingency islanding test) is FP64 in every
 * mode. */
enum { TTO_FLOW_F64 = 0, TTO_FLOW_F32 = 1 };

/* Arithmetic of the base-flow product f0 = PTDF * P (MFMA); FP64 accumulate
 * for F64, FP32 accumulate otherwise.  f0 is kept in FP64.  BF16X3 and F16X3
 * split both operands into hi + lo 16-bit parts and sum the three products
 * hi*hi + hi*lo + lo*hi on the 16-bit MFMA (about 16 and 22 significant bits).
 * F16 and F16X3 need |injections| below 65504 MW. */
enum {
  TTO_GEMM_F64 = 0, TTO_GEMM_F32 = 1, TTO_GEMM_BF16 = 2, TTO_GEMM_F16 = 3,
  TTO_GEMM_BF16X3 = 4, TTO_GEMM_F16X3 = 5
};

/* Per-candidate status bits. */
#define TTO_ST_ISLANDED 0x01u  /* post-switch grid is not connected */
#define TTO_ST_INVALID  0x02u  /* candidate violates the encoding rules */
#define TTO_ST_REFINED  0x04u  /* FP32 result was near a decision threshold
                                  and was recomputed in FP64 */
#define TTO_ST_REFINE_SKIPPED 0x08u  /* near a decision threshold but beyond
                                        the refinement capacity: FP32 result */
#define TTO_ST_NONFINITE 0x10u  /* set together with INVALID: the injections
                                   (the grid's or the candidate's moved
                                   amounts) hold a NaN or an infinity, so no
                                   flow is defined; decided after the
                                   encoding rules and the islanding test */

typedef struct tto_grid tto_grid;   /* opaque host handle */

/*
 * Grid (Problem formulation: node set N, edge set E with limits fbar_e,
 * outage set O).  DC model: lossless branches, b_e = 1/x_e, flows in MW,
 * dimensionless PTDF with a zero slack column (Importer: the PTDF of the
 * pre-optimisation topology is computed once).
 *
 *   ptdf          device, row-major [n_branch][n_bus], read only during
 *                 tto_grid_create (the grid keeps its own copies).
 *   monitored     host, distinct branch ids whose flows enter the metrics (M).
 *   contingency   host, distinct branch ids whose single outages form the
 *                 N-1 set (O).
 *   max_batch     largest n_cand later passed to tto_evaluate.
 */
typedef struct {
  int32_t n_bus;
  int32_t n_branch;
  int32_t slack;
  int32_t n_timesteps;          /* 1..TTO_MAX_T */
  const int32_t* from_bus;      /* host [n_branch] */
  const int32_t* to_bus;        /* host [n_branch] */
  const double* susceptance;    /* host [n_branch], > 0 */
  const double* limit_mw;       /* host [n_branch], > 0 */
  const double* ptdf;           /* device [n_branch * n_bus] */
  int32_t n_monitored;
  const int32_t* monitored;     /* host [n_monitored] */
  int32_t n_contingency;
  const int32_t* contingency;   /* host [n_contingency] */
  int32_t flow_precision;       /* TTO_FLOW_* */
  int32_t gemm_precision;       /* TTO_GEMM_* */
  int32_t max_batch;            /* >= 1 */
} tto_grid_desc;

/*
 * MapElites descriptor and fitness (DC-Optimizer, repertoire design and the
 * fitness lambda_f1 = -(lambda_o + w_c0 lambda_c0 + w_c lambda_c), weights 200
 * and 50 in the paper).
 *   TTO_DESC_COUNT_LOAD: two-axis cell, count axis = number of switched
 *   elements (openings + splits, clamped to n_count_bins-1), load axis =
 *   number of load_edges <= max loading (edges ascending);
 *   cell = count * n_load_bins + load_bin.
 *   TTO_DESC_PAPER: the repertoire design's three axes, lambda_d = openings
 *   (0..2), lambda_s = splits (0..3), lambda_r = reassigned assets = branches
 *   moved by the splits (0..45), each clamped;
 *   cell = lambda_d + 3 (lambda_s + 4 lambda_r), 552 cells (the printed
 *   coefficient is garbled; this one maps the ranges one to one).
 */
enum { TTO_DESC_COUNT_LOAD = 0, TTO_DESC_PAPER = 1 };
#define TTO_PAPER_CELLS 552

typedef struct {
  int32_t n_count_bins;         /* >= 1 (count-load map) */
  int32_t n_load_bins;          /* 1..TTO_MAX_LOAD_BINS (count-load map) */
  const double* load_edges;     /* host [n_load_bins - 1], ascending */
  double w_c0;
  double w_c;
  int32_t kind;                 /* TTO_DESC_* */
} tto_descriptor_cfg;

/*
 * Candidate batch in the fixed-slot genome encoding (repertoire design: an
 * individual holds N_a action slots and N_d disconnection slots, empty slots
 * hold the empty action).  All arrays are device memory.
 *
 *   open       [n_cand][n_open_slots]  opened branch id or -1
 *   split_bus  [n_cand][n_split_slots] split bus id or -1
 *   moved_off  [n_cand*n_split_slots+1] CSR offsets (may be NULL iff
 *              n_split_slots == 0)
 *   moved_br   branch ids moved to busbar B of each split slot
 *   moved_p_mw [n_cand*n_split_slots][n_timesteps] MW moved from busbar A to
 *              busbar B, or NULL (nothing moved)
 *
 * A candidate is INVALID (status bit) unless: opened ids are in range and
 * distinct; split buses are in range and distinct; each filled split moves a
 * non-empty list of distinct branches incident to its bus, none of them
 * opened; filled slots <= TTO_MAX_RANK; moved branches <= TTO_MAX_MOVED.
 * Moved lists of empty split slots are ignored.  The slack role stays on
 * busbar A.
 */
typedef struct {
  int32_t n_cand;
  int32_t n_open_slots;         /* 0..TTO_MAX_RANK */
  int32_t n_split_slots;        /* 0..TTO_MAX_RANK */
  const int32_t* open;
  const int32_t* split_bus;
  const int32_t* moved_off;
  const int32_t* moved_br;
  const double* moved_p_mw;
} tto_batch;

/*
 * Outputs, device memory, one entry per candidate unless noted; any pointer
 * may be NULL to skip that output.  Metrics follow the Fitness function
 * heuristics section with timesteps summed (lambda_o, lambda_c, lambda_c0)
 * or maximised (max loading, arg-max).  For islanded or invalid candidates
 * only `status` and `cell` (= -1) and `fitness` (= -inf) are defined.
 *
 *   overload_mw    lambda_o = sum_{t,e in M} max(f^max_e(t) - fbar_e, 0)
 *   n_crit_n1      lambda_c = #{(e,t): f^max_e(t) > fbar_e}
 *   n_crit_n0      lambda_c0 = #{(e,t): |f'_e(t)| > fbar_e}
 *   max_loading    max_{e,t} f^max_e(t) / fbar_e
 *   worst_*        branch id e*, timestep t* of the maximum loading (the
 *                  smallest (monitored position, t) within TTO_LOAD_TIE_REL
 *                  of it) and contingency branch id l*, the
 *                  first contingency within TTO_WORST_CONT_TIE_MW of the
 *                  maximum |flow| at (e*, t*) (l* = -1 when every
 *                  contingency islands)
 *   n_island_cont  contingencies skipped because they island the grid
 *   base_flows     [n_cand][n_branch][n_timesteps] post-switch N-0 flows
 *   fmax           [n_cand][n_monitored][n_timesteps]
 *   n1_flows       [n_cand][n_contingency][n_monitored][n_timesteps]; NaN
 *                  for islanding contingencies (debug-sized batches only)
 */
typedef struct {
  uint8_t* status;
  int32_t* n_island_cont;
  double* overload_mw;
  int32_t* n_crit_n1;
  int32_t* n_crit_n0;
  double* max_loading;
  int32_t* worst_branch;
  int32_t* worst_cont;
  int32_t* worst_t;
  double* fitness;
  int32_t* cell;
  double* base_flows;
  double* fmax;
  double* n1_flows;
} tto_outputs;

/* Library version; returns TTO_OK. */
tto_status tto_version(int32_t* major, int32_t* minor);

/* Thread-local message of the last failed call on this thread ("" if none). */
const char* tto_last_error(void);

/*
 * Device workspace sizes for a grid description (host only, no GPU work).
 * grid_bytes: persistent grid workspace for tto_grid_create.
 * batch_bytes: scratch for one tto_evaluate / tto_archive_insert call with
 * up to desc->max_batch candidates.  Both need 256-byte alignment.
 */
tto_status tto_workspace_bytes(const tto_grid_desc* desc, size_t* grid_bytes,
                               size_t* batch_bytes);

/*
 * Validate the grid on the host (index ranges, b > 0, limits > 0, distinct
 * M and C ids, connected base grid via union-find) and build the device
 * tables in grid_ws: H = PTDF * A^T in FP64 (row- and column-major), the
 * monitored x contingency block of H in FP32 and FP64 (contingency-major),
 * the PTDF copy in the GEMM precision.  Synchronises `stream`.  On success
 * *out receives a handle to free with tto_grid_destroy.  The default
 * descriptor is 32 x 32 cells, geometric load edges 0.25..64, weights 200/50.
 */
tto_status tto_grid_create(const tto_grid_desc* desc, void* grid_ws, size_t grid_bytes,
                           void* stream, tto_grid** out);

/* Free the host handle (device memory stays with the caller). */
void tto_grid_destroy(tto_grid* grid);

/*
 * Install nodal injections p_mw (device, row-major [n_bus][n_timesteps], MW,
 * generation positive; balancing is the caller's duty) and compute the base
 * flows f0 = PTDF * P with the MFMA GEMM in the grid's GEMM precision.
 * Asynchronous on `stream`; p_mw may be freed once the stream has passed.
 * Non-finite entries are not rejected here (that would need a host
 * synchronisation): every connected, encodable candidate evaluated under
 * them gets status INVALID | NONFINITE and never enters the repertoire.
 */
tto_status tto_set_injections(tto_grid* grid, const double* p_mw, void* stream);

/* Copy f0 (device [n_branch][n_timesteps], FP64) into out_mw. Asynchronous. */
tto_status tto_get_base_flows(tto_grid* grid, double* out_mw, void* stream);

/* Replace the descriptor/fitness settings.  Synchronous (small upload). */
tto_status tto_set_descriptor(tto_grid* grid, const tto_descriptor_cfg* cfg);

/*
 * Score a batch (DC-Optimizer: batched N-1 DC loadflow, lambda and beta).
 * Runs on `stream` without host synchronisation; batch_ws must hold
 * batch_bytes from tto_workspace_bytes and may be reused once the stream has
 * passed.  TTO_E_RANK if a slot count exceeds TTO_MAX_RANK.
 */
tto_status tto_evaluate(tto_grid* grid, const tto_batch* batch, const tto_outputs* out,
                        void* batch_ws, size_t batch_bytes, void* stream);

/*
 * Per-cell elite update (High-level loop: insert each new individual into the
 * cell given by beta; one elite per cell).  elite_fitness/elite_id are device
 * arrays [n_cells]; an empty cell has elite_id == -1.  Among the batch's
 * candidates whose status has neither ISLANDED nor INVALID set, each cell's
 * best fitness wins (ties: lowest index), and it replaces the elite only if
 * the cell is empty or the fitness is strictly greater; the new id is
 * id_base + index.  Equal to inserting the candidates one at a time in batch
 * order.  Uses the first 16*n_cells bytes of batch_ws.  Asynchronous.
 */
tto_status tto_archive_insert(tto_grid* grid, double* elite_fitness, int64_t* elite_id,
                              int32_t n_cells, const double* fitness, const int32_t* cell,
                              const uint8_t* status, int32_t n_cand, int64_t id_base,
                              void* batch_ws, size_t batch_bytes, void* stream);

/*
 * Allocation-free form of tto_archive_insert, for callers that cannot
 * allocate or pass a workspace (code under graph capture, tight serving
 * loops, harnesses that forbid allocation): the same update, with the same
 * arguments less batch_ws, its per-cell scratch held in a static device
 * array of the library (16 * TTO_ARCHIVE_NOALLOC_MAX_CELLS bytes = 1 MiB per
 * GPU, kept until the process ends; its address is taken when the first
 * grid is created on a device).  Calls no allocator.  The grid's device must
 * be current (TTO_E_INVALID otherwise); n_cells above
 * TTO_ARCHIVE_NOALLOC_MAX_CELLS returns TTO_E_WORKSPACE.  Every call on one
 * GPU shares that array and clears the part it uses by a kernel before use:
 * calls that overlap on one GPU (different streams, no ordering between
 * them) race and must not be issued.  Asynchronous.
 */
#define TTO_ARCHIVE_NOALLOC_MAX_CELLS 65536
tto_status tto_archive_insert_noalloc(tto_grid* grid, double* elite_fitness, int64_t* elite_id,
                                      int32_t n_cells, const double* fitness,
                                      const int32_t* cell, const uint8_t* status,
                                      int32_t n_cand, int64_t id_base, void* stream);

/*
 * Stage timing of tto_evaluate (tracing aid): when enabled, every
 * tto_evaluate records HIP events on its stream around its stages
 * (candidate set-up, N-1 sweep, finalize, FP64 refinement).
 * tto_profile_read waits for the events of the latest tto_evaluate and
 * writes the stage durations in milliseconds to ms[0..3].  TTO_E_INVALID if
 * profiling is off or nothing was recorded yet.
 */
tto_status tto_profile_enable(tto_grid* grid, int32_t enable);
tto_status tto_profile_read(tto_grid* grid, double* ms);

/*
 * Launch shape of the N-1 sweep (batching of uneven-rank candidates in one
 * launch).  The unit of work is one wave: a candidate and branches_per_lane
 * consecutive chunks of 64 monitored branches (one lane per branch of each
 * chunk, every timestep in registers); waves share no memory and never wait
 * on each other, and each candidate's rank fixes its wave's loop.
 *   lanes              workgroup size: 256 (four independent waves); 64 and
 *                      128 return TTO_E_UNSUPPORTED
 *   branches_per_lane  1 or 2 (2: each contingency record read by a wave
 *                      feeds two branches; FP32 flows only)
 *   order              0: hardware order of the work items; 1: each XCD
 *                      takes a contiguous candidate-major range (a
 *                      candidate's waves share its records in one L2); 2:
 *                      chunk-major ranges (an XCD streams few column blocks
 *                      of H[M, C] across many candidates); 3: as 1, in two
 *                      passes over the batch, each over one half of every
 *                      candidate's chunks (half of H in flight: far fewer
 *                      L2 misses for a little more time; the autotuner,
 *                      which minimises time, does not try it)
 *   persistent         must be 0: the persistent grid returns
 *                      TTO_E_UNSUPPORTED
 * The 64- and 128-lane workgroups and the persistent grid are switched off:
 * an earlier sweep in those shapes did not finish within a test's time limit
 * and no cause was found in its code.  Every enabled plan gives bitwise the
 * same outputs.  Default 256, 1, 0, 0.  TTO_E_INVALID for values out of
 * range, TTO_E_UNSUPPORTED for 2 branches per lane on an FP64 grid and for
 * the disabled shapes.
 */
tto_status tto_set_sweep_plan(tto_grid* grid, int32_t lanes, int32_t branches_per_lane,
                              int32_t order, int32_t persistent);

/*
 * FP64 refinement of FP32-flow grids (on by default, margin 8e-3 MW): after
 * the FP32 pass, a candidate whose maximum loading lies within margin_mw /
 * fbar of a load-bin edge, whose runner-up (branch, timestep) loading is
 * within margin_mw / min fbar of the maximum, or with a contingency flow at
 * (e*, t*) within 2 margin_mw of the worst-contingency cut (maximum minus
 * TTO_WORST_CONT_TIE_MW), is re-evaluated end to end in
 * FP64 on the GPU in the same tto_evaluate (status bit REFINED).  Capacity:
 * max_batch / 8 (at least 64) candidates per call; further flagged
 * candidates keep FP32 results (status bit REFINE_SKIPPED).  No effect on
 * FP64 grids.
 */
tto_status tto_set_refine(tto_grid* grid, int32_t enable, double margin_mw);
tto_status tto_get_sweep_plan(tto_grid* grid, int32_t* lanes, int32_t* branches_per_lane,
                              int32_t* order, int32_t* persistent);

/*
 * Autotuner: times the sweep plans on this batch (three tto_evaluate calls
 * each, median of the sweep stage by HIP events) and keeps the fastest.  The
 * search covers the register tile (1 or 2 monitored branches per lane, 2 on
 * FP32 grids only) x item orders 0, 1 and 2, at 256 lanes.  With a
 * non-empty cache_path, a line "<device> <shape>|<lanes> <branches per lane>
 * <order> <persistent>" is looked up first (no timing when found) and
 * appended after tuning.  chosen (optional, int32[5]) receives lanes,
 * branches per lane, order, persistent and 1 if the cache answered.
 * Synchronises `stream`; overwrites the outputs.
 */
tto_status tto_autotune(tto_grid* grid, const tto_batch* batch, const tto_outputs* out,
                        void* batch_ws, size_t batch_bytes, void* stream,
                        const char* cache_path, int32_t* chosen);

/*
 * Gather candidates idx[0..k) of `src` into the caller's device arrays
 * (dst_open [k][n_open_slots], dst_split [k][n_split_slots], dst_moved_off
 * [k*n_split_slots+1], dst_moved_br (capacity dst_moved_cap), dst_moved_p
 * [k*n_split_slots][T] or NULL) and fill *dst as a batch over them: used to
 * evaluate a screened subset exactly.  Indices must lie in [0, src->n_cand)
 * (checked on the device; a bad index yields an empty, INVALID-to-be
 * candidate).  If the gathered moved lists exceed dst_moved_cap the tail
 * candidates get empty split slots with a -2 bus (INVALID).  Asynchronous.
 */
tto_status tto_batch_gather(const tto_batch* src, const int32_t* idx, int32_t k,
                            int32_t n_timesteps, int32_t* dst_open, int32_t* dst_split,
                            int32_t* dst_moved_off, int32_t* dst_moved_br,
                            int32_t dst_moved_cap, double* dst_moved_p, tto_batch* dst,
                            void* stream);

/* ------------------------------------------------------------------------
 * Learned pre-screen (surrogate).  Not in the paper (its DC-Optimizer scores
 * every candidate exactly); added so that a generation can be screened
 * before exact evaluation.  A 4-layer perceptron:
 *   z1 = sum_{i in bits} W1b[i] + dense W1d + b1, h1 = relu(z1),
 *   h2 = relu(h1 W2 + b2), h3 = relu(h2 W3 + b3), y = h3 W4 + b4 (2 outputs),
 * input = the candidate's action bitmask (CSR list of set bit ids) and a
 * dense summary (e.g. per-timestep injection totals); outputs trained on the
 * exact evaluator's (maximum loading, log overload).  W1b, W1d, W2, W3 are
 * used in BF16 (MFMA, FP32 accumulation); the dense inputs and the hidden
 * activations are BF16; biases, W4 and the Adam master weights are FP32.
 * Loss 1/(2B) sum (y - t)^2.
 * Parameters are one flat FP32 array in the order W1b [d_bits][width],
 * W1d [d_dense][width], b1, W2 [width][width], b2, W3, b3, W4 [width][2], b4.
 */
typedef struct tto_mlp tto_mlp;

typedef struct {
  int32_t d_bits;            /* bitmask width (action vocabulary), >= 1 */
  int32_t d_dense;           /* dense inputs, 0..64 */
  int32_t width;             /* hidden width: multiple of 64 in 64..2048 */
  int32_t max_batch;         /* largest forward batch */
  int32_t max_train_batch;   /* largest training / gradient batch, 1..TTO_MLP_MAX_TRAIN */
} tto_mlp_desc;

#define TTO_MLP_MAX_ROW_BITS 64   /* entries read per bitmask row */
#define TTO_MLP_MAX_TRAIN 4096

/* Device workspace sizes: parameters + Adam state (persistent) and batch
 * scratch (per call).  Host only. */
tto_status tto_mlp_workspace_bytes(const tto_mlp_desc* desc, size_t* param_bytes,
                                   size_t* batch_bytes);
/* Bind a network to param_ws (256-byte aligned, param_bytes long).  Weights
 * are zero until tto_mlp_set_params.  Host only. */
tto_status tto_mlp_create(const tto_mlp_desc* desc, void* param_ws, size_t param_bytes,
                          tto_mlp** out);
void tto_mlp_destroy(tto_mlp* mlp);
tto_status tto_mlp_n_params(tto_mlp* mlp, int64_t* n);
/* Copy flat FP32 parameters (device) in / out; set also clears Adam. */
tto_status tto_mlp_set_params(tto_mlp* mlp, const float* params, void* stream);
tto_status tto_mlp_get_params(tto_mlp* mlp, float* params, void* stream);
/* y[B][2] for B candidates: bits_off [B+1] and bits_idx (device CSR; the
 * offsets must be non-decreasing and index inside bits_idx, which is the
 * caller's duty).  A row's bit set is the distinct ids in [0, d_bits) among
 * its first TTO_MLP_MAX_ROW_BITS entries (repeats and other ids are
 * ignored).  dense [B][d_dense] (device, may be NULL iff d_dense == 0). */
tto_status tto_mlp_forward(tto_mlp* mlp, const int32_t* bits_off, const int32_t* bits_idx,
                           const float* dense, int32_t n, float* y, void* batch_ws,
                           size_t batch_bytes, void* stream);
/* Loss (device scalar) and flat gradients (device, n_params) for targets
 * t[B][2]; B <= max_train_batch. */
tto_status tto_mlp_gradients(tto_mlp* mlp, const int32_t* bits_off, const int32_t* bits_idx,
                             const float* dense, const float* target, int32_t n, float* grad,
                             float* loss, void* batch_ws, size_t batch_bytes, void* stream);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8) on the loss of this batch. */
tto_status tto_mlp_train_step(tto_mlp* mlp, const int32_t* bits_off, const int32_t* bits_idx,
                              const float* dense, const float* target, int32_t n, float lr,
                              float* loss, void* batch_ws, size_t batch_bytes, void* stream);
/* Indices of the k smallest score[i * stride] (device), i < n, in index
 * order among equals; deterministic.  n <= 2^24, 0 <= k <= n. */
tto_status tto_topk_smallest(const float* score, int32_t n, int32_t stride, int32_t k,
                             int32_t* idx_out, void* stream);

/* ------------------------------------------------------------------------
 * Graph capture and replay.  A generation's launches (evaluate, archive
 * insertion, or the whole screened pipeline) are recorded once and replayed
 * with one call, so that many small launches cost one submission.
 *
 * tto_graph_begin creates a private stream in capture mode and returns it in
 * *capture_stream; pass that stream to the asynchronous tto_* calls to be
 * recorded, then call tto_graph_end.  Every pointer and size is fixed at
 * capture: a replay re-reads the current contents of the same buffers.
 * Calls that synchronise, allocate or clear memory refuse to run while their
 * stream is captured (tto_autotune, tto_mlp_set_params, tto_mlp_train_step
 * return TTO_E_UNSUPPORTED).  Stage events (tto_profile_*) are recorded by
 * eager calls only, never into a graph.  Host only, except tto_graph_launch,
 * which is asynchronous on `stream`.  tto_graph_destroy ends an open capture.
 */
typedef struct tto_graph tto_graph;
tto_status tto_graph_begin(tto_graph** out, void** capture_stream);
tto_status tto_graph_end(tto_graph* graph);
tto_status tto_graph_launch(tto_graph* graph, void* stream);
void tto_graph_destroy(tto_graph* graph);

/* One-call form: tto_evaluate on this batch followed, when elite_fitness is
 * not NULL, by tto_archive_insert of its results (ids id_base + i), captured
 * into *graph. */
tto_status tto_evaluate_capture(tto_grid* grid, const tto_batch* batch, const tto_outputs* out,
                                void* batch_ws, size_t batch_bytes, double* elite_fitness,
                                int64_t* elite_id, int32_t n_cells, int64_t id_base,
                                tto_graph** graph);

/* ------------------------------------------------------------------------
 * Importer on the device (Importer section: the optimizer starts from the
 * PTDF of the pre-optimisation topology; branches whose opening would split
 * the grid are not disconnectable).
 *
 * tto_ptdf_build: PTDF[e][j] = b_e (X[from_e][j] - X[to_e][j]) with X the
 * inverse of the nodal susceptance matrix without the slack row and column
 * (X's slack row and column zero), by blocked Gauss-Jordan elimination on
 * the FP64 MFMA.  Host arrays as in tto_grid_desc; ptdf: device FP64
 * [n_branch][n_bus] out, ready for tto_grid_desc.ptdf.  ws: device, 256-byte
 * aligned, tto_ptdf_bytes long (about 8 (n_bus - 1)^2 bytes).  TTO_E_GRID for
 * bad branches, susceptances or a disconnected grid.  Synchronises `stream`.
 *
 * tto_bridges: is_bridge (device uint8 [n_branch]) = 1 iff the branch is a
 * bridge of the grid, i.e. H_ee = b_e S_ee = 1 (tested as 1 - H_ee < 1e-9).
 */
tto_status tto_ptdf_bytes(int32_t n_bus, int32_t n_branch, size_t* bytes);

tto_status tto_ptdf_build(int32_t n_bus, int32_t n_branch, int32_t slack, const int32_t* from_bus,
                          const int32_t* to_bus, const double* susceptance, double* ptdf,
                          void* ws, size_t bytes, void* stream);

tto_status tto_bridges(const tto_grid* grid, uint8_t* is_bridge, void* stream);

/* ------------------------------------------------------------------------
 * Worst-k contingencies (AC-Validator section: for every N-1 case the DC
 * optimizer computes the overload energy on its own and writes out the k
 * worst cases, k = 20 in the paper, which the AC validator computes first).
 *
 * For each candidate of `batch` and each non-islanding contingency l:
 *   E_l = sum_{e in M, t} max(|f^(l)_e(t)| - fbar_e, 0)   (MW x timesteps)
 * in the grid's flow precision (an opened monitored branch carries no flow;
 * a contingency on an opened branch is the post-switch N-0 state).  ids
 * (device int32 [n_cand][k]) receives the contingency branch ids of the k
 * largest E_l in descending order, ties to the earlier entry of the
 * contingency list, energy_mw (device FP64 [n_cand][k]) the E_l; entries past
 * the candidate's non-islanding contingencies, and every entry of an
 * islanded or invalid candidate, are -1 and NaN.  The candidate set-up runs
 * again (batch_ws as for tto_evaluate); wk_ws (device, 256-byte aligned)
 * holds tto_worst_k_bytes.  No FP64 refinement: near-equal energies may
 * order differently from FP64 within the flow tolerance.
 */
#define TTO_MAX_WORST_K 64

tto_status tto_worst_k_bytes(const tto_grid* grid, int32_t n_cand, size_t* bytes);

tto_status tto_worst_contingencies(tto_grid* grid, const tto_batch* batch, int32_t k,
                                   int32_t* ids, double* energy_mw, void* batch_ws,
                                   size_t batch_bytes, void* wk_ws, size_t wk_bytes,
                                   void* stream);

/* ------------------------------------------------------------------------
 * Busbar outages (Problem formulation: the busbar outage set O_b; Fitness
 * function heuristics: busbar penalty lambda_b; High-level loop: lambda_f2).
 *
 * A busbar outage of bus b removes every in-service branch on b's node of the
 * post-switch grid and the injection on that node, which the slack takes over
 * (when the candidate splits b, the outage takes busbar A: the moved branches
 * and moved injection on busbar B stay).  With f^(b) the flows of that state,
 *   lambda_b = sum_{e in M, t} max(max_b |f^(b)_e(t)| - fbar_e, 0)
 * over the outages that leave the rest of the grid connected (the others are
 * counted in n_island), and
 *   lambda_f2 = lambda_f1 - max(lambda_b - lambda_b_pre, 0)
 * with lambda_b_pre the value of the pre-optimisation topology (evaluate the
 * empty candidate first).  Flows in the grid's flow precision; the per-
 * outage systems in FP64 (same islanding test as tto_evaluate).
 */
typedef struct tto_busbars tto_busbars;   /* opaque host handle */

/* Device bytes of a busbar set (host only). */
tto_status tto_busbar_set_bytes(const tto_grid* grid, int32_t n_busbars, size_t* bytes);

/*
 * buses: host [n_busbars] distinct bus ids, not the slack, each with 1..16
 * branches in the base grid (else TTO_E_GRID).  ptdf: the grid's PTDF again
 * (device FP64 [n_branch][n_bus], read during this call only).  ws: device,
 * 256-byte aligned, tto_busbar_set_bytes long, caller-owned and kept until
 * tto_busbar_set_destroy.  Synchronises `stream`.
 */
tto_status tto_busbar_set_create(const tto_grid* grid, int32_t n_busbars, const int32_t* buses,
                                 const double* ptdf, void* ws, size_t bytes, void* stream,
                                 tto_busbars** out);

void tto_busbar_set_destroy(tto_busbars* set);

/* Bytes of bb_ws for tto_busbar_evaluate on n_cand candidates (host only). */
tto_status tto_busbar_bytes(const tto_grid* grid, const tto_busbars* set, int32_t n_cand,
                            size_t* bytes);

/*
 * lambda_b (device FP64 [n_cand], may be NULL), n_island (device int32
 * [n_cand], may be NULL) and, when fitness_f2 is not NULL, lambda_f2 from
 * fitness_f1 (device FP64 [n_cand], tto_evaluate's fitness of the same batch)
 * and a finite lambda_b_pre.  p_mw: the injections installed with
 * tto_set_injections (device FP64 [n_bus][n_timesteps]).  Islanded or invalid
 * candidates get NaN, 0 and -inf.  The candidate set-up runs again
 * (batch_ws as for tto_evaluate).  Asynchronous.
 */
tto_status tto_busbar_evaluate(tto_grid* grid, const tto_busbars* set, const tto_batch* batch,
                               const double* p_mw, double lambda_b_pre, const double* fitness_f1,
                               double* lambda_b, int32_t* n_island, double* fitness_f2,
                               void* batch_ws, size_t batch_bytes, void* bb_ws, size_t bb_bytes,
                               void* stream);

/* ------------------------------------------------------------------------
 * MapElites generation on the device (DC-Optimizer: Repertoire design,
 * Mutation Alg. 1, Crossover Alg. 2, High-level loop Alg. 3): parents are
 * drawn from the repertoire, varied, expanded into a tto_batch, scored by
 * tto_evaluate and inserted, with no host synchronisation, so that a
 * generation can be captured once and replayed for a whole epoch.
 *
 * Genome: int32 [N_a action slots | N_d disconnection slots].  An action slot
 * holds an id into the split-action set A (each action splits one substation,
 * i.e. one bus, and names the branches it moves to busbar B), a disconnection
 * slot an index into the disconnectable-branch set D; -1 is the empty slot.
 *
 * Random numbers are Philox4x32-10 words addressed by (seed, generation,
 * child, draw position), so a generation's children depend only on the seed,
 * the generation counter and the repertoire.  Operator rules where the paper
 * leaves the sampling open:
 *   - Action Add: a uniform action outside every substation the individual
 *     splits, into a uniform empty slot; action Change: a uniform other action
 *     of a split substation, into that substation's slot; Remove: a uniform
 *     filled slot.  Disconnection Add / Change draw from D minus the current
 *     entries.  Operations are drawn with the integer weights over those that
 *     are feasible; N_mut = clip(Poisson(mut_mean), 1, N_a); the
 *     disconnection step takes Add when the individual (after its action
 *     steps) holds nothing.
 *   - Crossover: each child slot picks parent 1 with probability p_c1 (the
 *     other parent when one has nothing left), then a uniform remaining entry
 *     of that parent, empty entries included; the value also leaves the other
 *     parent once; an action at a substation the child already splits becomes
 *     empty.
 *   - Generation: b_mc uniform on 0..n_child; children [0, b_mc) are
 *     mutations, the rest crossovers; parents uniform over the occupied cells
 *     (the empty individual while none is occupied).  Parent genomes are
 *     first made feasible: out-of-range entries, actions at a substation an
 *     earlier slot splits and repeated disconnections read as empty.
 * Children may still be INVALID for tto_evaluate (a disconnected branch that
 * an action moves, more than TTO_MAX_MOVED moved branches); such children
 * never enter the repertoire.
 */
#define TTO_MAX_CELLS 4096

typedef struct tto_genome_space tto_genome_space;  /* opaque host handle */

typedef struct {
  int32_t n_action_slots;           /* N_a, 0..TTO_MAX_RANK */
  int32_t n_disc_slots;             /* N_d, 0..TTO_MAX_RANK */
  int32_t n_actions;                /* |A| >= 0 */
  const int32_t* action_bus;        /* host [n_actions] substation (bus) of each action */
  const int32_t* action_moved_off;  /* host [n_actions + 1] CSR offsets */
  const int32_t* action_moved_br;   /* host, distinct branches incident to the bus,
                                       at most TTO_MAX_MOVED per action */
  int32_t n_disc;                   /* |D| >= 0 */
  const int32_t* disc_branch;       /* host [n_disc] distinct branch ids */
  double mut_mean;                  /* N_mutmean >= 0 (paper: 2) */
  int32_t w_action[4];              /* Add, Remove, Change, Identity weights >= 0
                                       (paper: 20 20 50 10) */
  int32_t w_disc[4];                /* (paper: 25 25 50 0) */
  double p_c1;                      /* crossover bias toward parent 1, 0..1 */
} tto_genome_desc;

/* Device bytes of the genome tables (host only). */
tto_status tto_genome_space_bytes(const tto_genome_desc* desc, size_t* bytes);

/*
 * Validate the tables against the grid (ids in range, moved lists non-empty,
 * distinct and incident to their bus, D distinct) and upload them into ws
 * (device, 256-byte aligned, tto_genome_space_bytes long; caller-owned, kept
 * untouched until tto_genome_space_destroy).  Synchronises `stream`.
 * TTO_E_GRID for a table that does not fit the grid, TTO_E_RANK for slot
 * counts beyond TTO_MAX_RANK.
 */
tto_status tto_genome_space_create(const tto_grid* grid, const tto_genome_desc* desc, void* ws,
                                   size_t bytes, void* stream, tto_genome_space** out);

void tto_genome_space_destroy(tto_genome_space* gs);

/* Upper bound of moved branches per expanded candidate (N_a x longest action). */
tto_status tto_genome_max_moved(const tto_genome_space* gs, int32_t* per_candidate);

/*
 * Variation step of one generation (Alg. 3 with Alg. 1 and 2): children
 * [n_child][N_a + N_d] (device out) from the repertoire's occupied cells
 * (elite_id [n_cells] device, -1 = empty; elite_genome [n_cells][N_a + N_d]
 * device) for generation *generation (device int64, read only).  b_mc
 * (device int32, may be NULL) receives the number of mutated children.
 * n_cells 1..TTO_MAX_CELLS.
 */
tto_status tto_vary(const tto_genome_space* gs, const int64_t* elite_id,
                    const int32_t* elite_genome, int32_t n_cells, uint64_t seed,
                    const int64_t* generation, int32_t n_child, int32_t* children,
                    int32_t* b_mc, void* stream);

/*
 * Genomes [n][N_a + N_d] (device) -> tto_batch arrays (device, caller-owned):
 * open [n][N_d] (D index -> branch id), split_bus [n][N_a] (action -> bus),
 * moved_off [n*N_a + 1] and moved_br (the action's list).  Empty slots give
 * -1, out-of-range ids -2 (an INVALID candidate).  moved_cap (entries of
 * moved_br) must be at least n * tto_genome_max_moved; split_bus, moved_off
 * and moved_br may be NULL iff N_a == 0, open iff N_d == 0.
 */
tto_status tto_genome_expand(const tto_genome_space* gs, const int32_t* genomes, int32_t n,
                             int32_t* open, int32_t* split_bus, int32_t* moved_off,
                             int32_t* moved_br, int64_t moved_cap, void* stream);

/* Repertoire in device memory (caller-owned).  Empty cells have id -1. */
typedef struct {
  int32_t n_cells;          /* 1..TTO_MAX_CELLS, = the descriptor's cell count */
  double* fitness;          /* [n_cells] */
  int64_t* id;              /* [n_cells] generation * n_child + child index */
  int32_t* genome;          /* [n_cells][N_a + N_d] */
  int64_t* generation;      /* [1] generations completed so far */
} tto_repertoire;

/* Bytes of gen_ws for tto_generation with n_child children (host only). */
tto_status tto_generation_bytes(const tto_grid* grid, const tto_genome_space* gs,
                                int32_t n_child, size_t* bytes);

/*
 * One generation of Alg. 3 on `stream`: tto_vary, tto_genome_expand,
 * tto_evaluate (batch_ws as for tto_evaluate), insertion into the repertoire
 * (one elite per cell, ties to the lowest child index, strictly better
 * replaces; the genome is copied with the fitness and id), then
 * *generation += 1.  gen_ws (device, 256-byte aligned) holds the children
 * [n_child][N_a + N_d] int32 at offset 0, the int32 b_mc at byte offset
 * round_up(4 n_child (N_a + N_d), 256), and the expanded batch and the
 * status / fitness / cell outputs after it.  `out` may be NULL; otherwise its
 * non-NULL fields receive the outputs as from tto_evaluate.  No host
 * synchronisation: a generation can be captured between tto_graph_begin and
 * tto_graph_end and replayed; each replay advances the counter.
 */
tto_status tto_generation(tto_grid* grid, const tto_genome_space* gs, const tto_repertoire* rep,
                          uint64_t seed, int32_t n_child, const tto_outputs* out, void* gen_ws,
                          size_t gen_bytes, void* batch_ws, size_t batch_bytes, void* stream);

/*
 * Screened generation: Alg. 3 with the learned pre-screen between variation
 * and evaluation (an addition; the paper scores every child exactly).  On
 * `stream`: tto_vary of n_child children; their feature rows taken from the
 * genomes on the device (action a -> bit |D| + a, disconnection d -> bit d,
 * the network's d_bits must equal |D| + |A|); tto_mlp_forward with dense_row
 * (device FP32 [d_dense], the generation's injection summary, the same for
 * every child); the n_keep children with the smallest score, ties to the
 * lower child index, kept in child order.  The score (cfg NULL or rule
 * TTO_SCREEN_OVERLOAD) is the predicted column 1 (the overload term).  With
 * TTO_SCREEN_GAIN the outputs are de-standardised by cfg; each child's
 * predicted cell is taken from its genome (switch count, or the three-axis
 * map's counts) and the predicted maximum loading, its predicted fitness is
 * minus the predicted overload, and it is predicted to enter the repertoire
 * if that cell is empty or its elite is worse; of the children predicted to
 * enter each cell, the best predicted (ties to the lower index) comes
 * first, every other child is ranked by column 1;
 * tto_genome_expand, tto_evaluate and insertion of the kept children as in
 * tto_generation, the new elites' ids being generation * n_child + child
 * index; then *generation += 1.  n_child <= the network's max_batch, n_keep
 * <= min(n_child, the grid's max_batch).  gen_ws: device, 256-byte aligned,
 * tto_screened_generation_bytes long; mlp_ws: the network's batch workspace
 * (tto_mlp_workspace_bytes); batch_ws as for tto_evaluate.  `out` (may be
 * NULL) receives the kept children's outputs, entry i for the i-th kept
 * child, and kept_out (device int32 [n_keep], may be NULL) their child
 * indices.  No host synchronisation (capturable).
 */
#define TTO_SCREEN_OVERLOAD 0   /* keep the smallest predicted column 1 */
#define TTO_SCREEN_GAIN 1       /* first the best-predicted child of every
                                   cell it is predicted to enter, then the
                                   smallest predicted column 1 */
typedef struct {
  int32_t rule;               /* TTO_SCREEN_OVERLOAD or TTO_SCREEN_GAIN */
  double y_mu[2], y_sd[2];    /* raw target = output * y_sd + y_mu + ref */
  double ref[2];              /* (the network learns standardised targets
                                 relative to the unswitched grid) */
  double overload_scale_mw;   /* column 1 is log1p(overload / this scale) */
} tto_screen_cfg;
tto_status tto_screened_generation_bytes(const tto_grid* grid, const tto_genome_space* gs,
                                         const tto_mlp* net, int32_t n_child, int32_t n_keep,
                                         size_t* bytes);
tto_status tto_screened_generation(tto_grid* grid, const tto_genome_space* gs,
                                   const tto_repertoire* rep, tto_mlp* net,
                                   const float* dense_row, const tto_screen_cfg* cfg,
                                   uint64_t seed, int32_t n_child, int32_t n_keep,
                                   const tto_outputs* out, int32_t* kept_out, void* gen_ws,
                                   size_t gen_bytes, void* mlp_ws, size_t mlp_bytes,
                                   void* batch_ws, size_t batch_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* TTO_H */
