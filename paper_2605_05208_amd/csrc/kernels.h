// kernels.h -- host-side launch interface between the C-ABI layer and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace mdvrp {

// Compacted improving-move list (structure of arrays, caller-owned device arrays).
struct MoveList {
  int64_t* dF = nullptr;
  int64_t* dD = nullptr;
  uint64_t* id = nullptr;
  uint8_t* kind = nullptr;
  uint8_t* variant = nullptr;
  uint8_t* changed = nullptr;
  int32_t* unit = nullptr;
  int32_t* a = nullptr;
  int32_t* b = nullptr;
  int32_t* res = nullptr;  // [cap][3]
  int64_t cap = 0;
  unsigned long long* count = nullptr;  // null: no list
};

// Optional outputs of an evaluation: every evaluated move (rec/count/cap), the
// improving moves (ml), or per-anchor improving flags (label, pair kinds only,
// full lists).
struct DenseOut {
  DenseRec* rec = nullptr;
  unsigned long long* count = nullptr;
  int64_t cap = 0;
  uint8_t* label = nullptr;
  MoveList ml;
};

// Everything a launch needs about a batch.
struct LaunchCtx {
  hipStream_t stream;
  const UnitDesc* units;    // device array [n_units]
  int n_units;
  int has_tw, open;
  int t_is_c_all;           // every instance's travel times are its costs (one matrix)
  // item classes: 0 pairs, 1 depot-insert, 2 depot-replace, 3 route slots, 4 one block per unit
  const int32_t* tile_off[4];  // device arrays [n_units + 1]
  int tiles[4];
  int per_unit[4];             // tiles of each unit when all units have the same count, else 0
  // compact grids: pair evaluation of a search with a filter (blocks per unit = filtered
  // tiles; used when compact is set), and Depot-Replace (blocks per unit for the
  // expected routes); tiles_* = 0 when absent
  const int32_t* tile_off_f;
  int tiles_f, per_unit_f;
  const int32_t* tile_off_r;
  int tiles_r, per_unit_r;
  int compact;
  int max_nd;                  // largest depot count over the batch's instances
  int32_t* active_count;       // device int
  // active map of the local search's current pass (written by launch_pass_begin; null
  // outside the search): the evaluation kernels then map their first blocks onto the
  // active units' tiles
  int32_t* act;
  // dynamic penalty weights of a local search: the fused step writes each unit's new
  // weights into this array (the device copy of units) after a step that applied
  // moves; null = fixed weights
  UnitDesc* adapt_units;
  AdaptBounds adapt;
};

// One item class: 0 pair kinds, 1 depot-insert, 2 depot-replace (no launch when it has no work).
// shape: tile shape index (threads per block = tile_shape_threads(shape)); dense, label and
// footprint launches always use shape 0.
constexpr int kNumTileShapes = 3;
int tile_shape_threads(int shape);
void launch_eval_class(const LaunchCtx& L, uint32_t fam_mask, int cls, const DenseOut* dense, int shape = 0);
// Same evaluation, also marking every matrix entry read in the units' footprint bitmaps.
void launch_eval_footprint(const LaunchCtx& L, uint32_t fam_mask, int cls);
// Item classes an evaluation of fam_mask fills (bit 0 pairs, 1 depot-insert, 2 depot-replace).
uint32_t eval_classes(const LaunchCtx& L, uint32_t fam_mask);
// scored = the filtered lists were re-scored before this step's evaluation.
// apply = true: the selection kernel also rebuilds the new routes (the local search's fused step)
void launch_select(const LaunchCtx& L, uint32_t fam_mask, int leader_only, int scored = 0, bool apply = false);
void launch_rebuild(const LaunchCtx& L);
void launch_pass_begin(const LaunchCtx& L);
void launch_pass_end(const LaunchCtx& L);
void launch_cost(const LaunchCtx& L, int64_t* F, int64_t* terms);
void launch_export(const LaunchCtx& L, int32_t* nodes, int32_t* offs, int32_t* starts, int32_t* ends,
                   int32_t* counts, const int32_t* node_base, const int32_t* route_base);
void launch_load(const LaunchCtx& L, const int32_t* nodes, const int32_t* offs, const int32_t* starts,
                 const int32_t* ends, const int32_t* unit_route_off);
// Moves evaluated by every unit in the latest evaluation (out[n_units]).
void launch_evaluated_export(const LaunchCtx& L, int64_t* out);
void launch_sel_export(const LaunchCtx& L, uint64_t* ids, int64_t* dF, int32_t* counts, int32_t cap_per_unit);
constexpr int kStateWords = 16;  // per-unit counters and weights exported by launch_state_export
void launch_state_export(const LaunchCtx& L, int64_t* out /* [n_units][kStateWords] */);

// ---- learned move filter
// Device buffers of one network: fp32 master parameters, Adam moments, and the
// bf16 operand copies the kernels read (W1 / W2 in MFMA fragment order, W2 in the
// fragment order of the hidden-layer backward, w3 rounded and widened back to fp32); scratch holds the loss kernel's weight
// sum and per-block partials (2 + kBceBlocks floats).
struct MlpDev {
  float *P, *m, *v;
  void *w1f, *w2f, *w2b;
  float* w3b;
  float* scratch;
};
constexpr int kBceBlocks = 1024;  // loss-kernel blocks of a network's own scratch
int mlp_param_count();
int mlp_row_pad();  // activation buffers hold n rounded up to a multiple of this
void launch_mlp_pack(hipStream_t s, const MlpDev& M);
void launch_mlp_zero(hipStream_t s, float* p, int n);
void launch_features(const LaunchCtx& L, uint16_t* out);
// Incremental ranking state of a batch: cached logits of every anchor, the queue of
// anchors to rescore and its length, per-customer flags, anchor offsets per unit.
struct FilterQueue {
  float* lcache;         // [n_anchors]
  int32_t* queue;        // [n_anchors]
  int32_t* count;        // [1]
  uint8_t* cmark;        // [n_customers of the batch]
  const int64_t* anchor_off;  // [n_units + 1]
  int64_t n_anchors;
  int64_t max_unit_anchors;   // largest n_customers * theta of a unit
};
// Rank the lists: all = 1 every anchor of every unit, all = 0 the stale anchors of
// active filtered units; then the top-k of every customer that owns a rescored anchor.
void launch_rank(const LaunchCtx& L, const int32_t* cust_off, int n_cust, const MlpDev& M, const FilterQueue& Q,
                 int all);
void launch_eta_lists(const LaunchCtx& L, const int32_t* cust_off, int n_tasks);
void launch_mlp_forward(hipStream_t s, const MlpDev& M, const uint16_t* x, int n, float* logits, uint16_t* h1,
                        uint16_t* h2);
// Blocks of the loss kernel for n samples (at most max_blocks; one partial sum each).
int bce_blocks(int n, int max_blocks);
// scratch: [0] weight sum, [1] unused, [2 .. 2 + nb) per-block loss partials; nb = bce_blocks(n, ...).
void launch_bce(hipStream_t s, const float* z, const float* y, const float* w, int n, float* scratch, int nb,
                float* dz, float* loss);
// Floats of partial sums the backward pass of n samples needs.
size_t mlp_grad_part_floats(int n);
void launch_mlp_backward(hipStream_t s, const MlpDev& M, const uint16_t* x, int n, const float* dz, const uint16_t* h1,
                         const uint16_t* h2, float* g, uint16_t* G2, uint16_t* G1, float* part);
void launch_adam(hipStream_t s, const MlpDev& M, const float* g, float lr, int step);

// population measures (Section 3.4)
constexpr int kPopMaxMembers = 1024;  // members of one population call
constexpr int kPopMaxClose = 16;      // largest n_close of the population distance (Eq. 6)
// Edge keys of the members (units list[0..n)) into keys[n][nc], |E| into n_edges[n], then
// Eq. 7 for every pair into dist[n][n] (and the common arc counts into common, nullable).
void launch_pop_distance(const LaunchCtx& L, const int32_t* list, int n, int nc, int2* keys, int64_t* n_edges,
                         double* dist, int64_t* common);
void launch_pop_reduce(hipStream_t s, const double* dist, const int64_t* f, int n, int mu, double xi, int n_close,
                       int32_t* keep, int32_t* order, double* chi, double* dpop);

// repair insertion (Section 3.3): missing-customer lists, then one insertion per unit and
// round (op: MDVRP_REPAIR_*; order[order_base[u] + i] = the i-th customer inserted in unit u)
void launch_ins_begin(const LaunchCtx& L);
void launch_ins_export(const LaunchCtx& L, int64_t* out);  // insertion positions evaluated per unit
void launch_ins_round(const LaunchCtx& L, int op, uint64_t seed, int max_unrouted, int32_t* order,
                      const int32_t* order_base);

// DCREX crossover pieces (Algorithm 3) and discounted UCB1 (Eq. 4)
constexpr int kOccMax = 8;  // occurrences of one customer in an offspring the counts accept
size_t dcrex_ws_bytes(int n_nodes, int ns, int np, int p_len);
void launch_dcrex_counts(hipStream_t s, int n_nodes, int n_depots, int ns, int s_len, const int32_t* s_nodes,
                         const int32_t* s_offs, const int32_t* s_start, const int32_t* s_end, const int32_t* s_intro,
                         int np, int p_len, const int32_t* p_nodes, const int32_t* p_offs, const int32_t* p_start,
                         const int32_t* p_end, int32_t* EI, int32_t* NR, int32_t* NM, int32_t* NC, void* ws,
                         int32_t** err_out);
void launch_dcrex_pick(hipStream_t s, int ns, int np, const int32_t* EI, const int32_t* NR, const int32_t* NM,
                       const int32_t* NC, uint64_t seed, int32_t* out);
void launch_ucb_select(hipStream_t s, int n_arms, const double* R, const double* N, int32_t* arm);
void launch_ucb_update(hipStream_t s, int n_arms, double* R, double* N, const int32_t* arm, const double* reward,
                       double gamma);

// instance preprocessing
void launch_inst_stats(hipStream_t s, const int32_t* c, const int32_t* t, int n, int64_t* partial, int nblocks);
int inst_stats_blocks(int n);
void launch_inst_stats_final(hipStream_t s, const int64_t* partial, int nblocks, int64_t* out);
// Packs q, s, e, l into one int4 per node.
void launch_node_attr(hipStream_t s, const int32_t* q, const int32_t* sv, const int32_t* e, const int32_t* l, int n,
                      int4* attr);
// Depot-arc table of an instance: {c(d,x), t(d,x), c(x,d), t(x,d)} at [(x - nd) * nd + d].
void launch_depot_arcs(hipStream_t s, const int32_t* c, const int32_t* t, int nd, int nc, int4* out);
// Locality layout of an instance: landmarks (lm[6]), node keys, rank pi[x], its inverse,
// customers in layout order, and the reordered copies of c (and of t when tl != null).
void launch_layout(hipStream_t s, const int32_t* c, const int32_t* t, int n, int nd, int64_t* lm, uint64_t* keys,
                   int32_t* pi, int32_t* inv, int32_t* corder, int32_t* cl, int32_t* tl);
// Sum of c(u, first list entry) over customers with a list, and their count (out[0..1]).
void launch_nn_sum(hipStream_t s, const int32_t* c, const int32_t* nbr, const int32_t* nbr_len, int nd, int nc,
                   int theta, int64_t* out);
void launch_nbr_lists(hipStream_t s, const int32_t* c, const int32_t* t, const int32_t* sv, const int32_t* ev,
                      const int32_t* lv, int nd, int nc, int theta, int has_tw, int64_t gnum, int64_t gden,
                      int32_t* nbr, int32_t* nbr_len);
// {c(u, v), t(u, v)} of every granular-list slot (0 past the end of a list).
void launch_nbr_arcs(hipStream_t s, const int32_t* c, const int32_t* t, const int32_t* nbr, const int32_t* nbr_len,
                     int nd, int nc, int theta, int2* out);

}  // namespace mdvrp
