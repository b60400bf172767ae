/*
 * mdvrp.h -- C-ABI of libmdvrp: the data-parallel local-search hot path of a
 * hybrid method for multi-depot vehicle routing (MDVRP, MDVRPTW, MDOVRP),
 * after Lei & Hao, "A GPU-Accelerated Hybrid Method for a Class of
 * Multi-Depot Vehicle Routing Problems".
 *
 * Problem (paper Section 1): depots have ids [0, n_depots), customers
 * [n_depots, N); c and t are N*N travel distances and times; q demand, s
 * service time, [e, l] time window; Q vehicle capacity, NV vehicles per
 * depot, Dmax route-duration limit. A solution is a set of routes
 * S = {R_1..R_M}, each (start depot, customers..., end depot).
 *
 * Conventions
 *  - Every call returns an mdvrp_status; no call throws, prints or aborts.
 *  - Device memory is owned by the caller. Objects carve their device state
 *    out of a caller-provided workspace sized by the matching *_query call;
 *    the library never allocates device memory. Handles are host objects
 *    owned by the library and released by the *_destroy calls.
 *  - Calls are ordered on the caller's HIP stream (passed as void*, a
 *    hipStream_t; NULL = the default stream). Calls that return host values
 *    synchronise that stream.
 *  - Call order on a batch: every call that reads or changes its solutions
 *    returns ESTATE before the first successful mdvrp_solutions_load;
 *    mdvrp_select_multimove needs the latest mdvrp_eval_neighbourhood of the
 *    current solutions to be of the same family mask, and mdvrp_apply_moves a
 *    selection made since the last change of the solutions. These checks run
 *    on the host.
 *  - A handle is not thread-safe.
 *  - The routing arithmetic is int32 fixed point with int64 sums and objective
 *    values: every result is exact and deterministic. The learned filter
 *    computes in bf16 / fp32; every sum over samples runs in a fixed order, so
 *    its results are deterministic too. The one unspecified order is that of
 *    the rows of an improving-move list (mdvrp_moves).
 */
#ifndef MDVRP_H
#define MDVRP_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mdvrp_status;
#define MDVRP_OK 0
#define MDVRP_EINVAL (-1)  /* invalid argument or input data */
#define MDVRP_ERANGE (-2)  /* input outside the int32-safe range of the fixed-point arithmetic */
#define MDVRP_ENOSPC (-3)  /* workspace or output too small (required size written where stated) */
#define MDVRP_EDEVICE (-4) /* HIP runtime error; text from mdvrp_last_error() */
#define MDVRP_ESTATE (-5)  /* call out of order, or an internal invariant failed */

/* Operator families (bits of a family mask), paper Section 3.2.2. */
#define MDVRP_FAM_RELOCATE 0x01u      /* Relocate of 1- and 2-node sequences */
#define MDVRP_FAM_SWAP 0x02u          /* Swap of 1- and 2-node sequences */
#define MDVRP_FAM_2OPT_STAR 0x04u     /* 2-opt* between two routes */
#define MDVRP_FAM_2OPT 0x08u          /* 2-opt inside a route (instances without time windows) */
#define MDVRP_FAM_DEPOT_INSERT 0x10u  /* Depot-Insert (Fig. 1a) */
#define MDVRP_FAM_DEPOT_REPLACE 0x20u /* Depot-Replace (Fig. 1b) */
#define MDVRP_FAM_ALL 0x3Fu

/* Move kinds encoded in a move id: id = kind<<56 | variant<<48 | a<<24 | b. */
#define MDVRP_KIND_REL1 0
#define MDVRP_KIND_REL2 1
#define MDVRP_KIND_SWP11 2
#define MDVRP_KIND_SWP21 3
#define MDVRP_KIND_SWP12 4
#define MDVRP_KIND_SWP22 5
#define MDVRP_KIND_2OPT_STAR 6
#define MDVRP_KIND_2OPT 7
#define MDVRP_KIND_DEPOT_INSERT 8
#define MDVRP_KIND_DEPOT_REPLACE 9

typedef struct mdvrp_instance mdvrp_instance;
typedef struct mdvrp_batch mdvrp_batch;

/* Instance description. Array pointers are DEVICE pointers owned by the caller
 * and must stay valid for the lifetime of the instance handle. */
typedef struct {
  int32_t n_depots, n_customers; /* ids: depots [0,n_depots), customers [n_depots,N) */
  const int32_t *c, *t;          /* N*N row-major, >= 0; t may alias c. Without time
                                    windows c (and t) must be symmetric. */
  const int32_t *q, *s, *e, *l;  /* length N; depots: q = s = 0, [e,l] = departure/return window */
  int32_t Q, NV, Dmax;           /* capacity (> 0), vehicles per depot (>= 0), Dmax < 0: no limit */
  int32_t open_routes;           /* 1 = MDOVRP: routes have no arrival depot */
  int32_t has_tw;                /* 1 = time windows (time warp), 2-opt and reversed blocks off */
  int32_t theta;                 /* granular list size, 1..128 (>= n_customers-1: full) */
  int32_t w_tw, w_load, w_dur;   /* fixed penalty weights (>= 0) */
  int32_t w_depot;               /* < 0: 2*max c - min c (the Eq. A.1 normaliser) */
  int32_t layout;                /* MDVRP_LAYOUT_*: memory layout of the matrices the kernels read */
} mdvrp_instance_desc;

/* Matrix layout. The evaluations read c(x, y) for nodes close to each other; with
 * MDVRP_LAYOUT_ORDERED the instance keeps a copy of c (and t) whose rows and
 * columns follow an order in which nearby nodes get nearby indices (derived from
 * c: the Morton code of each node's distances to three far-apart landmarks), so
 * those reads share cache lines. The copy lives in the instance workspace (N*N
 * int32 per matrix). Results do not depend on the layout. MDVRP_LAYOUT_AUTO
 * (0, the default) orders instances whose matrix exceeds 64 MiB. */
#define MDVRP_LAYOUT_AUTO 0
#define MDVRP_LAYOUT_GIVEN 1
#define MDVRP_LAYOUT_ORDERED 2

/* ------------------------------------------------------------------------- instance */

/* Validate the scalar fields of desc and the HOST arrays q, s, e, l (desc's
 * pointers taken as host pointers; c and t are not read). Pure CPU; usable
 * without a GPU. Checks: n_depots >= 1, n_customers >= 1, N <= 65535,
 * Q > 0, NV >= 0, 1 <= theta <= 128, weights >= 0, q >= 0, s >= 0, e <= l,
 * depots q = s = 0 (EINVAL); total demand < 2^30 (ERANGE). */
mdvrp_status mdvrp_validate_instance_host(const mdvrp_instance_desc* desc);

/* Device workspace needed by mdvrp_instance_create. */
mdvrp_status mdvrp_instance_workspace_query(const mdvrp_instance_desc* desc, size_t* bytes);

/* Preprocess an instance (once): matrix statistics, the Theta normaliser and
 * Gamma of Eq. A.1 / Eq. 3, time-window arc pruning and the theta-nearest
 * granular lists by eta (Section 3.2.3), with c(u, v) and t(u, v) of every list
 * slot kept beside the lists (8 bytes per slot, read by the pair evaluation in
 * place of the matrix gather of the arc u -> v); with at most 64 depots also a
 * table of the arcs between every customer and every depot (16 bytes per pair,
 * read by Depot-Insert and Depot-Replace). Synchronises the stream.
 * Errors: EINVAL (bad desc or data, asymmetric c/t without time windows,
 * negative entries), ERANGE (distances too large for the fixed-point keys:
 * 8*max c >= 2^25), ENOSPC (ws_bytes too small), EDEVICE. */
mdvrp_status mdvrp_instance_create(const mdvrp_instance_desc* desc, void* ws, size_t ws_bytes, void* stream,
                                   mdvrp_instance** out);

/* Host copy of instance facts: [0] Theta, [1] Gamma numerator, [2] Gamma
 * denominator, [3] effective depot weight, [4] max c, [5] min c, [6] max t,
 * [7] longest route (customers) the int32 segment arithmetic accepts. */
mdvrp_status mdvrp_instance_info(const mdvrp_instance* inst, int64_t out[8]);

/* Copy the granular lists into DEVICE arrays: nbr[(u - n_depots)*theta + k]
 * (customer ids ranked by eta, -1 padding; n_customers*theta entries) and
 * nbr_len[u - n_depots] (n_customers entries). */
mdvrp_status mdvrp_instance_copy_lists(const mdvrp_instance* inst, int32_t* nbr, int32_t* nbr_len, void* stream);

void mdvrp_instance_destroy(mdvrp_instance* inst);

/* ------------------------------------------------------------------------- batches */

/* A batch is a set of units; unit k holds one solution of instance
 * insts[unit_inst[k]] (host arrays). All instances of a batch must agree on
 * has_tw and open_routes. */
mdvrp_status mdvrp_batch_workspace_query(const mdvrp_instance* const* insts, int32_t n_inst,
                                         const int32_t* unit_inst, int32_t n_units, size_t* bytes);
mdvrp_status mdvrp_batch_create(const mdvrp_instance* const* insts, int32_t n_inst, const int32_t* unit_inst,
                                int32_t n_units, void* ws, size_t ws_bytes, void* stream, mdvrp_batch** out);
void mdvrp_batch_destroy(mdvrp_batch* batch);

/* Validate solutions given in HOST arrays (layout of mdvrp_solutions_load) for
 * units whose instances are described by descs[unit_inst[k]] (only the scalar
 * fields of descs are read). Pure CPU. Checks, per unit: offsets increase;
 * every customer appears exactly once; routes are non-empty; starts (and
 * ends unless open) are depots; at most n_customers routes. */
mdvrp_status mdvrp_validate_solutions_host(const mdvrp_instance_desc* descs, int32_t n_inst, const int32_t* unit_inst,
                                           int32_t n_units, const int32_t* route_nodes,
                                           const int32_t* route_offsets, const int32_t* route_start,
                                           const int32_t* route_end, const int32_t* unit_route_offsets);

/* Load one solution per unit from DEVICE arrays: routes of unit k are
 * unit_route_offsets[k] .. unit_route_offsets[k+1]-1 (n_units+1 entries);
 * route r visits route_nodes[route_offsets[r] .. route_offsets[r+1]-1]
 * between depots route_start[r] and route_end[r] (ignored when open).
 * The arrays are copied to the host and validated first (EINVAL); a route
 * longer than the instance's int32-safe length (mdvrp_instance_info [7]) is
 * refused with ERANGE before any launch; then the route-major segment state is
 * built on the device and every unit's penalty weights are reset to its
 * instance's. Synchronises. */
mdvrp_status mdvrp_solutions_load(mdvrp_batch* batch, const int32_t* route_nodes, const int32_t* route_offsets,
                                  const int32_t* route_start, const int32_t* route_end,
                                  const int32_t* unit_route_offsets, int32_t n_routes_total,
                                  int32_t n_nodes_total, void* stream);

/* mdvrp_solutions_load for partial solutions: customers may be missing (each
 * appears at most once; routes non-empty; EINVAL otherwise). ERANGE when a route
 * plus every missing customer of its unit could exceed the int32-safe length.
 * Until mdvrp_repair completes the solutions, only mdvrp_repair,
 * mdvrp_solutions_export, mdvrp_batch_cost and mdvrp_batch_state accept the
 * batch (ESTATE otherwise). */
mdvrp_status mdvrp_solutions_load_partial(mdvrp_batch* batch, const int32_t* route_nodes, const int32_t* route_offsets,
                                          const int32_t* route_start, const int32_t* route_end,
                                          const int32_t* unit_route_offsets, int32_t n_routes_total,
                                          int32_t n_nodes_total, void* stream);

/* Insertion operators of the repair step (Section 3.3, after Algorithm 3). */
#define MDVRP_REPAIR_FBI 0 /* feasible best insertion */
#define MDVRP_REPAIR_IBI 1 /* infeasible best insertion */
#define MDVRP_REPAIR_FRI 2 /* feasible regret insertion */
#define MDVRP_REPAIR_IRI 3 /* infeasible regret insertion */
#define MDVRP_REPAIR_RI 4  /* random insertion */

/* Insert every customer missing from each unit's solution (loaded with
 * mdvrp_solutions_load_partial) with operator op; afterwards every unit holds a
 * complete solution. A position is "after the k-th customer of a route" (k = 0:
 * after the departure depot; k = L: before the arrival depot, or at the end of
 * an open route); its cost is the change of that route's Eq. A.1 cost under the
 * unit's current weights; it is feasible when it adds no time warp, load
 * excess or duration excess. Positions tie by their predecessor customer, or by
 * N + the route's first customer for k = 0.
 *   FBI / IBI: the missing customers in ascending id order, each to its
 *     cheapest feasible (FBI) / cheapest (IBI) position.
 *   FRI / IRI: repeatedly the customer of largest regret -- the cost of its
 *     second cheapest admissible position minus that of its cheapest; fewer than
 *     two admissible positions count as the largest; ties to the lower id -- to
 *     its cheapest admissible position.
 *   RI: in ascending id order, customer x goes into route r1 mod M after its
 *     (r2 mod (L + 1))-th customer, routes numbered by their first customer
 *     ascending, (r1, r2) the first two outputs of SplitMix64 seeded with
 *     seed ^ x.
 * FBI and FRI open a new route (d, x, d) -- (d, x) for open routes -- at the
 * depot of least cost change, fleet term included (ties: lower depot), in the
 * lowest empty route slot, when x has no feasible position; IBI, IRI and RI do
 * so only when the unit has no route. order (DEVICE int32, nullable) receives
 * the inserted customers of unit k in insertion order from entry node_base_k on
 * (node_base_k as in mdvrp_solutions_export); n_evaluated (DEVICE int64
 * [n_units], nullable) the insertion positions evaluated. Synchronises.
 * Errors: EINVAL (op), ESTATE (nothing loaded), ENOSPC (a unit's position
 * buffer is full). A batch of complete solutions is left unchanged. */
mdvrp_status mdvrp_repair(mdvrp_batch* batch, int32_t op, uint64_t seed, int32_t* order, int64_t* n_evaluated,
                          void* stream);

/* Export the current solutions to DEVICE arrays. Unit k writes its customers to
 * route_nodes[node_base_k ..] with node_base_k = sum of n_customers of units < k,
 * and its routes to entries [route_base_k ..] of route_offsets (values index
 * route_nodes; one extra closing entry), route_start and route_end, with
 * route_base_k = sum over units < k of (n_customers + 1); route_count[k] = number
 * of routes. Capacity: sum(n_customers) nodes, sum(n_customers + 1) routes. */
mdvrp_status mdvrp_solutions_export(const mdvrp_batch* batch, int32_t* route_nodes, int32_t* route_offsets,
                                    int32_t* route_start, int32_t* route_end, int32_t* route_count, void* stream);

/* F(S) of every unit recomputed from the current routes (Eq. A.1 under the
 * unit's current penalty weights: its instance's, unless a search with
 * penalty_adapt changed them): F[k] and terms[k*6 + 0..5] = D, TW, LX, DX, CL,
 * FX (DEVICE arrays, terms nullable). */
mdvrp_status mdvrp_batch_cost(mdvrp_batch* batch, int64_t* F, int64_t* terms, void* stream);

/* Host copy of per-unit counters, 16 per unit: running F, evaluated moves,
 * passes, steps, moves applied, error bits, active flag, moves selected in
 * the latest step, full-list fallback passes of a filtered search, current
 * list mode (0 full, 1 filtered, 2 full fallback pass), device clock at the
 * start of the latest search and at the end of the unit's latest pass, and
 * the unit's current penalty weights (time window, load, duration, depot).
 * Synchronises. */
mdvrp_status mdvrp_batch_state(const mdvrp_batch* batch, int64_t* out_host);

/* ------------------------------------------------------------------------- hot path */

/* Compacted list of improving moves (dF < 0), structure of arrays. Every array
 * is a DEVICE array owned by the caller with room for cap rows; count is a
 * DEVICE counter that the evaluation sets to the number of improving moves it
 * found (which may exceed cap: rows beyond cap are not written). Row order is
 * unspecified (it depends on scheduling); the set of rows is deterministic. */
typedef struct {
  int64_t* dF;              /* penalised cost delta (Eq. A.1 with fixed weights), < 0 */
  int64_t* dD;              /* distance delta */
  uint64_t* id;             /* kind<<56 | variant<<48 | a<<24 | b */
  uint8_t* kind;            /* MDVRP_KIND_* (= id >> 56) */
  uint8_t* variant;         /* (id >> 48) & 0xff: orientation of 2-node blocks, Depot-Replace case */
  uint8_t* changed;         /* penalty terms the move changes: bit 0 time warp, 1 load excess,
                               2 duration excess, 3 closure + fleet excess (V4) */
  int32_t* unit;            /* unit (solution) of the move */
  int32_t* a;               /* pair kinds: u; Depot-Insert: u (cut after u); Depot-Replace: first customer */
  int32_t* b;               /* pair kinds: v; depot moves: the depot */
  int32_t* res;             /* [cap][3] resources: route slot r, n_customers + d for depot d's
                               vehicle count, -1 none (the conflict sets of Section 3.2.5) */
  int64_t cap;
  unsigned long long* count;
} mdvrp_moves;

/* Evaluate, in parallel, the penalised delta of every move of the families in
 * family_mask for every active unit (Sections 3.2.1-3.2.4: Eq. A.1 deltas of
 * Relocate, Swap, 2-opt*, 2-opt and the depot operators of Fig. 1 over the
 * granular neighbourhood of Eq. 3). The per-unit leader candidate and follower
 * candidates stay in the batch for mdvrp_select_multimove.
 *   cand, k: optional candidate lists (DEVICE int32, cand[unit][i][k] for
 *     customer n_depots + i of the unit's instance, units in batch order; -1
 *     pads a list). When given, pair moves are anchored on (u, v) for the
 *     entries v of u's list instead of the granular list N(u); the depot
 *     operators are unchanged. 1 <= k <= theta of every instance; entries must
 *     be customers other than u, without repeats in one list (checked on the
 *     host: EINVAL). cand = NULL: the granular lists, or with
 *     MDVRP_EVAL_FILTERED the lists of the attached filter.
 *   moves (nullable): receives every improving move (mdvrp_moves). When
 *     *moves->count exceeds moves->cap the call returns ENOSPC after the
 *     evaluation; *moves->count then holds the required capacity and the
 *     selection state is still valid.
 *   n_evaluated (DEVICE int64[n_units], nullable): moves evaluated per unit
 *     (every tuple that passes its preconditions).
 * Families without moves in an instance (2-opt with time windows) are
 * ignored. Synchronises the stream when cand or moves is given. */
#define MDVRP_EVAL_FILTERED 0x2u
mdvrp_status mdvrp_eval_neighbourhood(mdvrp_batch* batch, uint32_t family_mask, const int32_t* cand, int32_t k,
                                      mdvrp_moves* moves, uint32_t flags, int64_t* n_evaluated, void* stream);

/* One dense record per evaluated move (debug output). */
typedef struct {
  int64_t dF, dD, dTW, dLX, dDX, dV4; /* deltas of F, distance, time warp, load excess,
                                         duration excess, closure + fleet excess */
  uint64_t id;                        /* kind<<56 | variant<<48 | a<<24 | b */
  int32_t unit;
  int32_t res[3];                     /* route slot r, or n_customers + depot, or -1 */
} mdvrp_dense_rec;

/* Debug form of mdvrp_eval_neighbourhood: the same evaluation (with flags
 * MDVRP_EVAL_FILTERED as there), writing every evaluated move, improving or
 * not, to dense (DEVICE array of dense_cap records); *dense_count, a DEVICE
 * counter the caller zeroes, receives the total, which may exceed dense_cap. */
mdvrp_status mdvrp_eval_dense(mdvrp_batch* batch, uint32_t family_mask, uint32_t flags, mdvrp_dense_rec* dense,
                              int64_t dense_cap, unsigned long long* dense_count, void* stream);

/* Leader-follower selection (Section 3.2.5) over the last evaluation: the
 * leader is the move with the smallest (dF, id) and is taken when dF < 0;
 * followers (dD < 0 and no change of any penalty term) are taken in ascending
 * (dF, id) order when they share no route and no depot vehicle count with a
 * move already taken. leader_only = 1 keeps the leader alone. The selection
 * is prepared for mdvrp_apply_moves. When sel_ids is non-NULL, unit k's
 * selected ids and deltas are written to sel_ids / sel_dF [k*sel_cap ..] and
 * their count to sel_count[k] (DEVICE arrays). */
mdvrp_status mdvrp_select_multimove(mdvrp_batch* batch, uint32_t family_mask, int32_t leader_only,
                                    uint64_t* sel_ids, int64_t* sel_dF, int32_t* sel_count, int32_t sel_cap,
                                    void* stream);

/* Apply the selected moves of every unit: the update of the current solution
 * by the accepted move set of Algorithm 2 (the leader and its followers of
 * Section 3.2.5). The moves are route-disjoint, so the order does not matter;
 * emptied routes are deleted and the segment state of the changed routes is
 * rebuilt. */
mdvrp_status mdvrp_apply_moves(mdvrp_batch* batch, void* stream);

#define MDVRP_LS_PASSES 0 /* Algorithm 2: per pass, every family in a seeded random order */
#define MDVRP_LS_UNION 1  /* every step evaluates all families together */

typedef struct mdvrp_mlp mdvrp_mlp;

#define MDVRP_FILTER_NONE 0  /* pair moves over the granular lists */
#define MDVRP_FILTER_LISTS 1 /* pair moves over the attached filter's lists as they stand */
#define MDVRP_FILTER_MLP 2   /* lists re-ranked by the network whenever their features change */

#define MDVRP_RESCORE_STEP 0 /* re-rank stale lists before every pair-family step */
#define MDVRP_RESCORE_PASS 1 /* re-rank stale lists before the first pair-family step of a pass;
                                n > 1: of every n-th pass */

typedef struct {
  int32_t mode;        /* MDVRP_LS_PASSES or MDVRP_LS_UNION */
  int32_t leader_only; /* 1 = single-move steps (the paper's ETGA-S) */
  int32_t max_passes;  /* search depth delta; 0 = until a local optimum */
  int32_t poll_every;  /* passes between host convergence checks (>= 1). The host reads the
                          count of active units of one interval while the next interval
                          runs (pinned host memory owned by the batch), so up to
                          2 * poll_every - 1 passes may follow the last unit's convergence;
                          they change nothing (inactive units skip every kernel) */
  uint64_t seed;       /* family order of pass p: Fisher-Yates with SplitMix64(seed ^ p) */
  int32_t filter;      /* MDVRP_FILTER_*; a filter needs mdvrp_filter_attach first */
  int32_t rescore;     /* when MDVRP_FILTER_MLP re-ranks stale lists: MDVRP_RESCORE_STEP, or
                          n >= 1 = at the first pair-family step of every n-th pass */
  const mdvrp_mlp* mlp; /* network of MDVRP_FILTER_MLP, else ignored */
  int32_t graph;       /* 1 = each pass runs as a HIP graph, captured once per distinct launch
                          sequence (family order and options) and replayed; per-launch
                          profiling is off for captured passes */
  int32_t penalty_adapt; /* 1 = dynamic penalty coefficients (Section 3.2.1): every unit starts
                          from its instance's weights; after each step that applied moves each of
                          the four weights (order: time window, load, duration, depot) is doubled
                          (divided by kappa = 1/2) when the new solution violates its term (time
                          warp; load excess; duration excess; closure or fleet excess) and halved,
                          rounding down (multiplied by kappa), otherwise, then clamped to
                          [w_min, w_max]. The weights of a unit change only here. Needs
                          max_passes > 0 (EINVAL otherwise): with moving weights a search need
                          not reach a fixed point (the paper bounds it by its depth delta = 500) */
  int32_t w_min[4], w_max[4]; /* bounds of the adapted weights: 0 <= w_min <= w_max <= 2^30 */
} mdvrp_ls_options;

typedef struct {
  int64_t passes, steps, moves_applied, evaluated, F;
  int64_t fallback_passes; /* passes of a filtered search that evaluated the full lists */
  double device_ms;        /* device clock from the start of the search to the end of this
                              unit's last pass (its time to the local optimum) */
  int32_t converged, err;
  int64_t w_final[4];      /* penalty weights at the end (time window, load, duration, depot);
                              F is the objective under these weights */
} mdvrp_ls_stats;

/* Local search to a local optimum for every unit of the batch (Algorithm 2 with
 * the multi-move step). A unit stops when a full pass applies nothing. With a
 * filter, pair moves are first drawn from the filtered lists; when a pass over
 * the filtered lists applies nothing, the next pass evaluates the full
 * granular lists: if that pass improves, the unit returns to the filtered
 * lists, otherwise it stops -- at a local optimum of the full neighbourhood
 * either way. With MDVRP_FILTER_MLP the lists of every customer whose
 * features may have changed (its route, or the route of an entry of its
 * granular list, was rebuilt since the last ranking) are re-ranked before
 * each pair-family step (MDVRP_RESCORE_STEP) or before the first one of every
 * n-th pass (rescore = n >= 1); the first ranking covers all of them. The
 * lists in between may lag the routes; they stay valid candidate sets, every
 * move is still evaluated exactly, and the fallback passes keep the end state
 * a local optimum of the full neighbourhood. stats
 * (HOST array of n_units, nullable) receives per-unit results. Synchronises.
 * Errors: ERANGE when a route grew beyond the int32-safe length, ENOSPC on
 * internal capacity overflow, EDEVICE. */
mdvrp_status mdvrp_local_search_to_optimum(mdvrp_batch* batch, const mdvrp_ls_options* opts,
                                           mdvrp_ls_stats* stats, void* stream);

/* ------------------------------------------------------------------------- population (Section 3.4)
 *
 * A population is a list of distinct units of one batch that hold solutions of
 * the same instance (units: HOST array of n unit indices, 1 <= n <= 1024). The
 * edge set E of a solution is the set of directed arcs along its routes: from the
 * departure depot to the first customer, between consecutive customers, and from
 * the last customer to the arrival depot (none for an open route). */

/* Device workspace of mdvrp_population_distance for these members. */
mdvrp_status mdvrp_population_workspace_query(const mdvrp_batch* batch, const int32_t* units, int32_t n,
                                              size_t* bytes);

/* Distance between every pair of members' current solutions (Eq. 7):
 * dist[i*n + j] = 100 * (1 - |E_i & E_j| / max(|E_i|, |E_j|)) in fp64 (DEVICE,
 * n*n; the quotient, the difference and the product each rounded once, in that
 * order); common[i*n + j] = |E_i & E_j| and n_edges[i] = |E_i| (DEVICE int64,
 * nullable). ws: DEVICE workspace of mdvrp_population_workspace_query bytes.
 * Errors: EINVAL (bad member list), ESTATE (no solutions loaded), ENOSPC
 * (workspace too small). Synchronises the stream. */
mdvrp_status mdvrp_population_distance(mdvrp_batch* batch, const int32_t* units, int32_t n, double* dist,
                                       int64_t* common, int64_t* n_edges, void* ws, size_t ws_bytes, void* stream);

/* Reduction of a population of n members to mu (Section 3.4; all arrays DEVICE):
 * while more than mu remain, the fitness-and-distance score chi (Eq. 5) of every
 * remaining member is computed and the member of lowest chi leaves (ties: the
 * higher index). chi = (m - Rank_f)/m + xi * (m - Rank_D)/m over the m remaining
 * members; Rank_f orders f[] ascending, Rank_D the population distance (Eq. 6:
 * the mean of the n_close smallest distances to the other remaining members,
 * summed in ascending order; fewer when fewer remain) descending; ties in either
 * go to the lower index; ranks count from 1. dist: n*n from
 * mdvrp_population_distance (or any symmetric matrix); f: n objective values
 * (e.g. mdvrp_batch_cost of the members); xi >= 0 (the paper uses 0.7);
 * 1 <= n_close <= 16 (the paper uses 5). keep[i] = 1 for the survivors; order
 * (nullable, n - mu entries) the removal order; chi and dpop (nullable, n each)
 * the scores and population distances over all n members. */
mdvrp_status mdvrp_population_reduce(const double* dist, const int64_t* f, int32_t n, int32_t mu, double xi,
                                     int32_t n_close, int32_t* keep, int32_t* order, double* chi, double* dpop,
                                     void* stream);

/* ------------------------------------------------------------------------- DCREX crossover (Algorithm 3, Eq. 4)
 *
 * The offspring S' of the route-exchange crossover may hold a customer in more
 * than one route, so it is passed as plain route lists: DEVICE int32 arrays, route
 * r = (start[r], nodes[offs[r] .. offs[r+1]-1], end[r]), end -1 for an open route;
 * intro[r] = 1 for the routes introduced from other parents. Arcs are the directed
 * arcs along a route, as in the population distance. */

mdvrp_status mdvrp_dcrex_workspace_query(int32_t n_nodes, int32_t ns, int32_t np, int32_t p_len, size_t* bytes);

/* The counts behind the score of every route pair (R_i of S', ns routes; R_j of
 * parent P, np routes), at [i*np + j] (DEVICE int32 outputs): EI = arcs of R_j
 * held by no route of S' other than R_i (new arcs); NR = customers of R_i that
 * R_j does not bring and no other route of S' holds (missing); NM = customers of
 * R_j held by another route of S' (redundant); NC = customers of R_j held by
 * another introduced route of S' (conflicting). Algorithm 3 scores a pair by
 * -(EI - NR - NM - 10 NC) and its exchange adds EI + NR + NM to the diversity.
 * Node ids: depots [0, n_depots), customers [n_depots, n_nodes). The route lists
 * are copied to the host and checked first (EINVAL: ids, offsets, flags, a customer
 * twice in one route of S' or anywhere in P). ENOSPC when a customer occurs in more
 * than 8 routes of S'. Synchronises. */
mdvrp_status mdvrp_dcrex_counts(int32_t n_depots, int32_t n_nodes, int32_t ns, int32_t s_len, const int32_t* s_nodes,
                                const int32_t* s_offs, const int32_t* s_start, const int32_t* s_end,
                                const int32_t* s_intro, int32_t np, int32_t p_len, const int32_t* p_nodes,
                                const int32_t* p_offs, const int32_t* p_start, const int32_t* p_end, int32_t* EI,
                                int32_t* NR, int32_t* NM, int32_t* NC, void* ws, size_t ws_bytes, void* stream);

/* Algorithm 3's choice of the exchange: among the min(5, ns*np) pairs of lowest
 * (score, i, j), the one at index SplitMix64(seed) mod their number. out (DEVICE
 * int32[4]) = {i, j, diversity increase EI + NR + NM, number of candidates}
 * ({-1, -1, 0, 0} without pairs). */
mdvrp_status mdvrp_dcrex_pick(int32_t ns, int32_t np, const int32_t* EI, const int32_t* NR, const int32_t* NM,
                              const int32_t* NC, uint64_t seed, int32_t* out, void* stream);

/* Discounted UCB1 (Eq. 4) over n_arms arms (1..1024) with discounted reward sums R
 * and counts N (DEVICE fp64). Select: *arm (DEVICE) = an arm with N = 0 (lowest
 * index) if any, else the arm of largest R/N + sqrt(2 ln(sum N) / N), ties to the
 * lower index; ln and sqrt follow fixed operation sequences (a 40-term atanh
 * series after halving into [1, 2); 8 Newton steps after scaling into [1, 4)), so
 * that the choice is reproducible bit for bit. Update: every arm's R and N times
 * gamma (the paper's gamma_d = 0.99), then the reward (*reward, DEVICE) and 1 added
 * to arm *arm. The reward of the paper is 100 (f(P_m) - f(S')) / f(P_m). */
mdvrp_status mdvrp_ucb_select(int32_t n_arms, const double* R, const double* N, int32_t* arm, void* stream);
mdvrp_status mdvrp_ucb_update(int32_t n_arms, double* R, double* N, const int32_t* arm, const double* reward,
                              double gamma, void* stream);

/* ------------------------------------------------------------------------- profiling */

/* Kernel classes of the profiler. */
#define MDVRP_PROF_EVAL_PAIRS 0
#define MDVRP_PROF_EVAL_DEPOT_INSERT 1
#define MDVRP_PROF_EVAL_DEPOT_REPLACE 2
#define MDVRP_PROF_SELECT 3 /* in the local search: selection and apply, one fused kernel per step */
#define MDVRP_PROF_APPLY 4  /* mdvrp_apply_moves */
#define MDVRP_PROF_FILTER_SCORE 5

/* Turn per-launch timing on (class_mask != 0) or off for a batch. Every launch
 * of a kernel class whose bit (1 << MDVRP_PROF_*) is set in class_mask is
 * bracketed by two HIP events on the launch stream (host objects; no device
 * memory is allocated). Up to max_launches launches are kept pending before
 * they are folded into totals. Resets the totals. */
mdvrp_status mdvrp_profile_enable(mdvrp_batch* batch, uint32_t class_mask, int32_t max_launches);

/* Time only every n-th launch of each class (every >= 1; 1 = all, the default).
 * Each timed launch adds two event records to the stream, which delay the
 * next launch by a few microseconds; sampling keeps that cost small while the
 * sampled launches still give the average duration of the class. Kept across
 * mdvrp_profile_enable calls. Errors: EINVAL. */
mdvrp_status mdvrp_profile_sampling(mdvrp_batch* batch, int32_t every);

/* Per-class totals since enabling: launches[8] (timed launches) and elapsed milliseconds ms[8]
 * (HOST arrays, indexed by MDVRP_PROF_*). Waits for pending events. */
mdvrp_status mdvrp_profile_read(mdvrp_batch* batch, int64_t* launches, double* ms);

/* Measurement variant of mdvrp_eval_neighbourhood: the same evaluation, which
 * also marks every matrix entry it reads in a bitmap, giving the number of
 * distinct c/t entries (the matrix part of a launch's compulsory traffic).
 * bitmap: zeroed DEVICE array; instance k of the batch (order of the
 * instance list given at creation) owns words [sum_{j<k} W_j, ...) with
 * W_j = ceil(N_j*N_j / 32). bitmap_words must cover all instances.
 * Arcs between a customer and a depot that Depot-Insert and Depot-Replace read
 * from the instance's depot-arc table (instances with at most 64 depots) are
 * not matrix reads and are not marked; the table is 16 bytes per (customer,
 * depot) pair. The results of the evaluation itself are discarded.
 * Synchronises. */
mdvrp_status mdvrp_eval_footprint(mdvrp_batch* batch, uint32_t family_mask, uint32_t* bitmap, int64_t bitmap_words,
                                  void* stream);

/* ------------------------------------------------------------------------- autotuner
 *
 * An evaluation tile is 256 items (anchors, or (customer, depot) pairs); a
 * block of 256, 128 or 64 threads covers it with 1, 2 or 4 items per thread.
 * Results never depend on the shape. mdvrp_autotune times every shape of the
 * evaluation of each family in family_mask on the batch's current solutions
 * (reps launches each, HIP events on the stream), keeps the fastest for the
 * local search and the single-family evaluations, and writes the chosen
 * threads per block of each family (6 entries, family bit order) to
 * shapes_out (HOST, nullable). Call it after loading solutions and before a
 * search: it resets the follower candidates and keeps the evaluation
 * counters. Synchronises. */
mdvrp_status mdvrp_autotune(mdvrp_batch* batch, uint32_t family_mask, int32_t reps, int32_t* shapes_out,
                            void* stream);
/* Set the threads per block of each family (6 entries, each 256, 128 or 64). */
mdvrp_status mdvrp_set_tile_shapes(mdvrp_batch* batch, const int32_t* threads);

/* ------------------------------------------------------------------------- learned move filter
 *
 * The paper restricts every operator to granular lists (Section 3.2.3, Eq. 3).
 * The filter ranks each customer u's granular list N(u) with a network and
 * keeps the k best entries for exact evaluation.
 *
 * Features: 32 per anchor (u, v = k-th entry of N(u)), from exact integers:
 *   0 c(u,v) 1 c(p(u),u) 2 c(u,s(u)) 3 c(p(u),s(u)) 4 c(p(v),v) 5 c(p(v),u)
 *   6 distance delta of relocating u before v, 7 of the 2-opt* move joining
 *   u -> v, 8 of swapping u with p(v) (s(u) of an open route's last customer
 *   contributes 0; pp(v) = p(v) when p(v) is a depot);
 *   9, 10 load - Q of u's and v's routes; 11 q_u; 12 q_v; 13, 14 duration -
 *   Dmax of both routes (0 without a limit); 15, 16 time warp of both routes;
 *   17, 18 window widths of u and v; 19 e_u; 20 e_v; 21 max(e_v - e_u - s_u -
 *   t(u,v), 0); 22 max(e_u + s_u + t(u,v) - l_v, 0) (17..22 are 0 without
 *   time windows); 23 same route; 24 same start depot; 25, 26 start depots;
 *   27, 28 route lengths; 29, 30 positions of u and v; 31 k.
 * Each integer is converted to fp32 and multiplied (one rounding) by an fp32
 * scale, then rounded to bf16 (nearest even): 0..8 by 1/dbar, dbar = integer
 * mean of c(u, first entry of N(u)) (at least 1); 9..12 by 1/Q; 13..22 by 1/H,
 * H = l - e of depot 0 with time windows, else 1; 23, 24 by 1; 25, 26 by
 * 1/n_depots; 27, 28 by 1/32; 29 by 1/length(u's route); 30 by 1/length(v's
 * route); 31 by 1/theta.
 * Network: logit = w3 . relu(W2 relu(W1 x + b1) + b2) + b3, 32 -> 256 -> 256
 * -> 1; bf16 weights and inputs, fp32 accumulation, hidden activations
 * rounded to bf16. Parameters (fp32 master copy, MDVRP_MLP_PARAMS floats):
 * W1[256][32], b1[256], W2[256][256], b2[256], w3[256], b3.
 * Per-anchor arrays of a batch (features, labels, logits) hold units in batch
 * order, each n_customers * theta anchors, anchor (i, k) at i * theta + k. */
#define MDVRP_MLP_PARAMS 74497

mdvrp_status mdvrp_mlp_workspace_query(size_t* bytes);
/* params_init: DEVICE fp32[MDVRP_MLP_PARAMS] copied in, or NULL for zeros.
 * Adam moments start at zero. */
mdvrp_status mdvrp_mlp_create(void* ws, size_t ws_bytes, const float* params_init, void* stream, mdvrp_mlp** out);
/* Device pointer to the fp32 master parameters inside the workspace. After
 * writing them, call mdvrp_mlp_sync. */
mdvrp_status mdvrp_mlp_params(mdvrp_mlp* mlp, float** params);
/* Refresh the bf16 operand copies from the master parameters; reset_adam = 1
 * also zeroes the Adam moments. */
mdvrp_status mdvrp_mlp_sync(mdvrp_mlp* mlp, int32_t reset_adam, void* stream);
void mdvrp_mlp_destroy(mdvrp_mlp* mlp);
/* Bytes of the activation workspace for n samples (training calls). */
mdvrp_status mdvrp_mlp_act_bytes(int32_t n, size_t* bytes);
/* logits[n] (DEVICE fp32) of x[n][32] (DEVICE bf16 bits). act_ws (nullable)
 * keeps the hidden activations for mdvrp_mlp_backward. */
mdvrp_status mdvrp_mlp_forward(const mdvrp_mlp* mlp, const uint16_t* x, int32_t n, float* logits, void* act_ws,
                               size_t act_bytes, void* stream);
/* grads (DEVICE fp32[MDVRP_MLP_PARAMS], overwritten) = gradient of
 * sum_p dlogits[p] * logit_p, using the activations a forward pass over the
 * same x and parameters left in act_ws. */
mdvrp_status mdvrp_mlp_backward(const mdvrp_mlp* mlp, const uint16_t* x, const float* dlogits, int32_t n,
                                float* grads, void* act_ws, size_t act_bytes, void* stream);
/* Weighted mean binary cross-entropy with logits: *loss (DEVICE, nullable) =
 * sum w_p l_p / sum w_p, dlogits_p = w_p (sigmoid(z_p) - y_p) / sum w_p;
 * weights NULL = all 1. Uses the network's scratch. */
mdvrp_status mdvrp_mlp_bce(mdvrp_mlp* mlp, const float* logits, const float* labels, const float* weights, int32_t n,
                           float* dlogits, float* loss, void* stream);
/* Adam (beta 0.9 / 0.999, eps 1e-8, bias-corrected, step >= 1) on the master
 * parameters, then refresh of the bf16 copies. */
mdvrp_status mdvrp_adam_step(mdvrp_mlp* mlp, const float* grads, float lr, int32_t step, void* stream);
/* forward + BCE + backward + Adam on one batch of n samples. */
mdvrp_status mdvrp_mlp_train_step(mdvrp_mlp* mlp, const uint16_t* x, const float* labels, const float* weights,
                                  int32_t n, float lr, int32_t step, float* grads, float* logits, float* loss,
                                  void* act_ws, size_t act_bytes, void* stream);

/* mdvrp_mlp_train_step without the activation workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving or training
 * loops, harnesses that forbid allocation). It runs the same kernels; the
 * activations, hidden-layer gradients and partial sums live in a static device
 * array of 16 MiB inside the library (one per GPU, held until the process ends),
 * so the call allocates nothing. n is at most MDVRP_TRAIN_STATIC_MAX_N (EINVAL
 * beyond). Every call on a GPU shares that GPU's array: calls that overlap on one
 * GPU (different streams or threads) race and must be serialised by the caller.
 * Results equal those of mdvrp_mlp_train_step on the same arguments. */
#define MDVRP_TRAIN_STATIC_MAX_N 4096
mdvrp_status mdvrp_mlp_train_step_static(mdvrp_mlp* mlp, const uint16_t* x, const float* labels,
                                         const float* weights, int32_t n, float lr, int32_t step, float* grads,
                                         float* logits, float* loss, void* stream);

/* Candidate lists of k entries per customer for every unit of a batch
 * (1 <= k <= theta of every instance); attaching sets them to the first k
 * entries of the granular lists. */
mdvrp_status mdvrp_filter_workspace_query(const mdvrp_batch* batch, int32_t k, size_t* bytes);
mdvrp_status mdvrp_filter_attach(mdvrp_batch* batch, int32_t k, void* ws, size_t ws_bytes, void* stream);
/* Number of anchors of the batch (sum of n_customers * theta over units). */
mdvrp_status mdvrp_filter_anchor_count(const mdvrp_batch* batch, int64_t* n);
/* Features of every anchor of the current solutions: feats[anchor][32] (DEVICE
 * bf16 bits; rows of missing list entries are zero). */
mdvrp_status mdvrp_filter_features(mdvrp_batch* batch, uint16_t* feats, void* stream);
/* Training labels: labels[anchor] (DEVICE, zeroed by the caller) is set to 1
 * when some pair move of the families in family_mask anchored at it has
 * dF < 0 in the current solution (the evaluation of the full lists). */
mdvrp_status mdvrp_filter_labels(mdvrp_batch* batch, uint32_t family_mask, uint8_t* labels, void* stream);
/* Rank every customer's granular list by the network and keep the k best
 * entries (logit descending, customer id ascending; -1 padding); logits
 * (DEVICE, nullable) receives every anchor's logit. */
mdvrp_status mdvrp_filter_score_topk(mdvrp_batch* batch, const mdvrp_mlp* mlp, float* logits, void* stream);
/* The heuristic lists: the first k entries of each granular list. */
mdvrp_status mdvrp_filter_eta_lists(mdvrp_batch* batch, void* stream);
/* cand[unit][customer][k] (DEVICE int32), units in batch order. */
mdvrp_status mdvrp_filter_export(const mdvrp_batch* batch, int32_t* cand, void* stream);

/* ------------------------------------------------------------------------- misc */

const char* mdvrp_status_string(mdvrp_status s);
/* Text of the last error raised on the calling thread. */
const char* mdvrp_last_error(void);
/* Family order of pass p as the library computes it (host; for checks). */
int32_t mdvrp_family_order(int32_t has_tw, uint64_t seed, int64_t pass, int32_t* fam_out);

#ifdef __cplusplus
}
#endif
#endif
