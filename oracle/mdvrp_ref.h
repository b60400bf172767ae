/*
 * mdvrp_ref.h -- plain CPU oracle for the MDVRP local-search hot path.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library. The product path (the
 * HIP library) never links, calls or includes anything from this directory,
 * and this directory includes nothing from the product.
 *
 * What it computes (paper: Lei & Hao, "A GPU-Accelerated Hybrid Method for a
 * Class of Multi-Depot Vehicle Routing Problems"):
 *   - the multi-penalty evaluation function F(S) (Section 3.2.1, Eq. 2, and
 *     its full form Eq. A.1 in the supplementary material), with fixed integer
 *     penalty weights in place of the dynamic coefficients;
 *   - time warp and duration by Vidal's sequence concatenation (cited in
 *     Section 3.2.2 and in Appendix A);
 *   - the neighbourhood of Relocate, Swap, 2-opt*, 2-opt (Section 3.2.2) and
 *     the two depot operators Depot-Insert / Depot-Replace (Section 3.2.2,
 *     Fig. 1), restricted to granular lists (Section 3.2.3, Eq. 3);
 *   - the leader-follower multi-move selection (Section 3.2.5);
 *   - the local search loop (Algorithm 2), optionally with the dynamic
 *     penalty coefficients of Section 3.2.1;
 *   - the population measures of Section 3.4 (Eq. 5-7; pop_ref.c).
 * Every move is evaluated by rebuilding the changed routes as explicit node
 * lists and recomputing their cost from scratch.
 *
 * All pointers are host pointers. Functions return 0 on success, a negative
 * code on error (-1 invalid input, -3 output capacity too small: the required
 * count is written to the count argument).
 */
#ifndef MDVRP_REF_H
#define MDVRP_REF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t n_depots, n_customers;
  const int32_t *c, *t;            /* N*N row-major */
  const int32_t *q, *s, *e, *l;    /* length N */
  int32_t Q, NV, Dmax;             /* Dmax < 0: no duration limit */
  int32_t open_routes, has_tw, theta;
  int32_t w_tw, w_load, w_dur, w_depot; /* w_depot < 0: use 2*max c - min c */
} ref_instance;

/* Move kinds (id = kind<<56 | variant<<48 | a<<24 | b). */
enum { REF_REL1 = 0, REF_REL2 = 1, REF_SWP11 = 2, REF_SWP21 = 3, REF_SWP12 = 4, REF_SWP22 = 5,
       REF_X2 = 6, REF_2OPT = 7, REF_DINS = 8, REF_DREP = 9 };
/* Operator families (bit positions of a family mask). */
enum { REF_FAM_REL = 0, REF_FAM_SWP = 1, REF_FAM_X2 = 2, REF_FAM_2OPT = 3, REF_FAM_DINS = 4,
       REF_FAM_DREP = 5 };

typedef struct {
  int64_t dF, dD, dTW, dLX, dDX, dV4;
  uint64_t id;
  int32_t res[3]; /* route index r >= 0, depot d as -2-d, -1 none */
} ref_move;

/* Instance statistics: out[0] = Theta = 2*max c - min c over u != v,
 * out[1], out[2] = Gamma = sum c / sum t reduced to num/den,
 * out[3] = effective depot weight. */
int ref_instance_stats(const ref_instance* I, int64_t out[4]);

/* Granular lists (Section 3.2.3): nbr[(u - n_depots)*theta + k], nbr_len[u - n_depots]. */
int ref_neighbours(const ref_instance* I, int32_t* nbr, int32_t* nbr_len);

/* F(S) and its terms: terms[0..5] = D, TW, LX, DX, CL, FX. Returns 0. */
int ref_cost(const ref_instance* I, int32_t n_routes, const int32_t* nodes, const int32_t* offs,
             const int32_t* start, const int32_t* end, int64_t* F, int64_t terms[6]);

/* Terms of one route walked node by node (start depot, customers xs[0..L-1],
 * end depot or -1 when open): out[0] distance, out[1] load, out[2] duration
 * and out[3] time warp by the left fold of Vidal's concatenation (Section 3.2.2,
 * Appendix A; without time windows duration = travel + service, warp 0). */
int ref_route_terms(const ref_instance* I, int32_t start, const int32_t* xs, int32_t L, int32_t end, int64_t out[4]);

/* Every evaluated move of the families in fam_mask (dense list). */
int ref_eval(const ref_instance* I, const int32_t* nbr, const int32_t* nbr_len,
             int32_t n_routes, const int32_t* nodes, const int32_t* offs,
             const int32_t* start, const int32_t* end, uint32_t fam_mask,
             ref_move* out, int64_t cap, int64_t* count);

/* One step: evaluate fam_mask, select (leader + followers), apply.
 * The new solution is written to the out arrays (capacity: n_customers
 * nodes, n_customers routes). sel_ids receives the selected ids in
 * selection order. */
int ref_step(const ref_instance* I, const int32_t* nbr, const int32_t* nbr_len,
             int32_t n_routes, const int32_t* nodes, const int32_t* offs,
             const int32_t* start, const int32_t* end, uint32_t fam_mask, int32_t leader_only,
             int32_t* o_nroutes, int32_t* o_nodes, int32_t* o_offs, int32_t* o_start,
             int32_t* o_end, uint64_t* sel_ids, int64_t* sel_dF, int32_t* n_sel,
             int64_t* n_eval);

/* Apply the (route-disjoint) moves with the given ids; output as in ref_step. */
int ref_apply_ids(const ref_instance* I, int32_t n_routes, const int32_t* nodes, const int32_t* offs,
                  const int32_t* start, const int32_t* end, const uint64_t* ids, int32_t n_ids,
                  int32_t* o_nroutes, int32_t* o_nodes, int32_t* o_offs, int32_t* o_start, int32_t* o_end);

typedef struct {
  int32_t mode;        /* 0 = passes over a permutation of families, 1 = union */
  int32_t leader_only; /* 1 = apply the leader alone */
  int32_t max_passes;  /* 0 = until a local optimum (the depth delta of Algorithm 2 otherwise) */
  int32_t penalty_adapt; /* 1 = dynamic penalty coefficients (Section 3.2.1), see w_min/w_max;
                            needs max_passes > 0 (the search depth of Algorithm 2): with moving
                            weights a search can revisit solutions forever */
  uint64_t seed;
  /* Bounds of the adapted weights, order time window, load, duration, depot
   * (lambda_1..lambda_4): after every step that applied moves, each weight is
   * doubled (divided by kappa = 1/2) when the new solution violates its constraint
   * and halved, rounding down, otherwise, then clamped to [w_min, w_max]. */
  int32_t w_min[4], w_max[4];
} ref_ls_options;

typedef struct {
  int64_t passes, steps, moves_applied, evaluated, F; /* F under the final weights */
  int64_t w_final[4];                                 /* weights at the end (tw, load, dur, depot) */
} ref_ls_stats;

/* Local search to a local optimum for each of n_sol solutions (OpenMP over
 * solutions). Input/output in the batch layout: routes of solution k are
 * sol_offs[k]..sol_offs[k+1]-1. Output capacity: n_sol*n_customers routes. */
int ref_local_search(const ref_instance* I, const int32_t* nbr, const int32_t* nbr_len,
                     int32_t n_sol, const int32_t* nodes, const int32_t* offs,
                     const int32_t* start, const int32_t* end, const int32_t* sol_offs,
                     const ref_ls_options* opt, int32_t* o_nodes, int32_t* o_offs,
                     int32_t* o_start, int32_t* o_end, int32_t* o_sol_offs, ref_ls_stats* stats);

/* ---- learned move filter (mlp_ref.c) ---- */

/* fp32 -> bf16, round to nearest even; bf16 -> fp32. */
uint16_t ref_bf16(float f);
float ref_bf16_to_f32(uint16_t h);

/* 32 bf16 features of every anchor (u, k-th entry of N(u)):
 * out[((u - n_depots)*theta + k)*32 + f]; rows of missing entries are zero. */
int ref_filter_features(const ref_instance* I, const int32_t* nbr, const int32_t* nbr_len, int32_t n_routes,
                        const int32_t* nodes, const int32_t* offs, const int32_t* start, const int32_t* end,
                        uint16_t* out);

/* MLP 32 -> 256 -> 256 -> 1 (ReLU). Parameters fp32, layout W1[256][32], b1[256],
 * W2[256][256], b2[256], w3[256], b3. round_act = 1 rounds weights, input and
 * hidden activations to bf16 where the GPU path does. */
int ref_mlp_param_count(void);
int ref_mlp_forward(const float* params, const uint16_t* x, int32_t n, int32_t round_act, double* logits);
/* gradient of sum_p dlogits[p] * logit_p (fp64) */
int ref_mlp_backward(const float* params, const uint16_t* x, int32_t n, const double* dlogits, int32_t round_act,
                     double* grads);
double ref_bce(const double* logits, const float* labels, const float* weights, int32_t n);
int ref_adam(float* params, float* m, float* v, const float* grads, int32_t n, float lr, int32_t step);
/* k largest scores per customer (ties -> lower customer id), -1 padding */
int ref_topk(const int32_t* nbr, const int32_t* nbr_len, int32_t n_customers, int32_t theta, const float* score,
             int32_t k, int32_t* out);

/* One output of SplitMix64 (Steele, Lea and Flood 2014); advances *state. */
uint64_t ref_splitmix64(uint64_t* state);

/* Family order of pass p: Fisher-Yates driven by SplitMix64 seeded with seed ^ p. */
int ref_family_order(int32_t has_tw, uint64_t seed, int64_t pass, int32_t* fam_out);

/* ---- population measures (pop_ref.c; Section 3.4) ---- */

/* Distance between every pair of n_sol solutions (batch layout of
 * ref_local_search), Eq. 7: dist[i*n_sol + j] = 100 * (1 - |E_i & E_j| /
 * max(|E_i|, |E_j|)), with E the set of directed arcs of a solution's routes
 * (departure depot to first customer, consecutive customers, last customer to
 * arrival depot unless the route is open). common[i*n_sol + j] = |E_i & E_j|
 * and n_edges[i] = |E_i| (both nullable). */
int ref_population_distance(const ref_instance* I, int32_t n_sol, const int32_t* nodes, const int32_t* offs,
                            const int32_t* start, const int32_t* end, const int32_t* sol_offs, double* dist,
                            int64_t* common, int64_t* n_edges);

/* Reduction of a population of n solutions to mu (Section 3.4): while more than
 * mu remain, chi (Eq. 5, with the population distance of Eq. 6 over the n_close
 * nearest other solutions, fewer when fewer remain) is computed over the
 * remaining ones and the one of lowest chi leaves (ties: higher index).
 * Rank_f: objective f ascending; Rank_D: population distance descending (ties in
 * either: lower index first), both from 1. keep[i] = 1 for the survivors,
 * order[0 .. n-mu) the removal order, chi_first / dpop_first (nullable) the
 * scores and population distances over all n solutions. */
int ref_population_reduce(int32_t n, const double* dist, const int64_t* f, int32_t mu, double xi, int32_t n_close,
                          int32_t* keep, int32_t* order, double* chi_first, double* dpop_first);

/* ---- repair insertion (repair_ref.c; Section 3.3, after Algorithm 3) ---- */

/* Insert every customer missing from the partial solution (routes as in ref_cost;
 * each customer at most once, routes non-empty) with operator op: 0 FBI, 1 IBI,
 * 2 FRI, 3 IRI, 4 RI. A position is "after the k-th customer of a route" (k = 0:
 * after the departure depot, k = L: before the arrival depot or at the end of an
 * open route); its cost is the change of that route's Eq. A.1 cost; it is
 * feasible when it adds no time warp, load excess or duration excess. Positions
 * tie by their predecessor customer (or N + the first customer for k = 0).
 * FBI / IBI take the customers in ascending id order, each to its cheapest
 * (feasible) position; FRI / IRI repeatedly take the customer of largest regret
 * (second cheapest minus cheapest admissible cost; fewer than two admissible
 * positions count as the largest regret; ties to the lower id) to its cheapest
 * position. FBI / FRI open a new route (d, x, d) -- (d, x) when open -- at the
 * depot of least cost change, fleet term included (ties: lower depot), when x
 * has no feasible position; IBI / IRI only when the solution has no route. RI
 * takes the customers in ascending id order and inserts x into route
 * r1 mod M after customer r2 mod (L + 1), routes numbered by their first
 * customer ascending, (r1, r2) the first two outputs of SplitMix64 seeded with
 * seed ^ x. Output routes are ordered by their first customer (capacity:
 * n_customers routes); order[0 .. n_order) lists the inserted customers in
 * insertion order; n_evaluated counts the positions evaluated. */
int ref_repair(const ref_instance* I, int32_t n_routes, const int32_t* nodes, const int32_t* offs,
               const int32_t* start, const int32_t* end, int32_t op, uint64_t seed, int32_t* o_nroutes,
               int32_t* o_nodes, int32_t* o_offs, int32_t* o_start, int32_t* o_end, int32_t* order,
               int32_t* n_order, int64_t* n_evaluated);

/* ---- DCREX crossover (dcrex_ref.c; Algorithm 3, Eq. 4) ---- */

/* The counts behind the score of every route pair (R_i of the offspring S',
 * R_j of a parent P), at [i*np + j]: EI new arcs (arcs of R_j held by no route
 * of S' other than R_i), NR missing nodes (customers of R_i that R_j does not
 * bring and no other route of S' holds), NM redundant nodes (customers of R_j
 * held by another route of S'), NC conflicting nodes (customers of R_j held by
 * another route of S' introduced from a parent: intro[r] = 1). Score =
 * -(EI - NR - NM - 10 NC); diversity increase = EI + NR + NM. */
int ref_dcrex_counts(int32_t ns, const int32_t* s_nodes, const int32_t* s_offs, const int32_t* s_start,
                     const int32_t* s_end, const int32_t* s_intro, int32_t np, const int32_t* p_nodes,
                     const int32_t* p_offs, const int32_t* p_start, const int32_t* p_end, int32_t* EI, int32_t* NR,
                     int32_t* NM, int32_t* NC);

/* Discounted UCB1 (Eq. 4) over n_arms arms with discounted reward sums R and
 * counts N: the arm of largest R/N + sqrt(2 ln(sum N) / N) (an arm with N = 0
 * first; ties to the lower index); the update discounts every arm by gamma and
 * adds the reward and 1 to the played one. ln and sqrt are computed by the fixed
 * operation sequences below. */
int32_t ref_ucb_select(int32_t n_arms, const double* R, const double* N);
void ref_ucb_update(int32_t n_arms, double* R, double* N, int32_t arm, double reward, double gamma);
double ref_ucb_ln(double x);
double ref_ucb_sqrt(double x);

/* OpenMP threads of the solution-parallel local search (timing only). */
void ref_set_threads(int32_t n);
int32_t ref_get_threads(void);

#ifdef __cplusplus
}
#endif
#endif
