/*
 * repair_ref.c -- plain CPU oracle of the insertion operators that put unrouted
 * customers back into a solution (Section 3.3, after Algorithm 3): feasible and
 * infeasible best insertion (FBI, IBI), feasible and infeasible regret
 * insertion (FRI, IRI) and random insertion (RI).
 * TEST INFRASTRUCTURE ONLY (see mdvrp_ref.h). Shares no code with the HIP path.
 *
 * Every candidate insertion is materialised as the explicit node list of the new
 * route, whose terms are recomputed by walking it (ref_route_terms).
 */
#include <stdlib.h>
#include <string.h>

#include "mdvrp_ref.h"

typedef struct {
  int32_t start, end, len;
  int32_t* x;
} prt;

typedef struct {
  int64_t dF;
  int feasible;
  int64_t posid; /* predecessor customer, or N + first customer for the slot after the departure depot */
  int32_t route, k; /* insert after the k-th customer of route (k = 0: after the departure depot) */
} ins_t;

static int64_t route_cost(const ref_instance* I, int64_t wdep, int32_t start, const int32_t* xs, int32_t L,
                          int32_t end, int64_t term[3]) {
  (void)wdep;
  int64_t t[4];
  ref_route_terms(I, start, xs, L, end, t);
  const int64_t lx = t[1] > I->Q ? t[1] - I->Q : 0;
  const int64_t dx = (I->Dmax >= 0 && t[2] > I->Dmax) ? t[2] - I->Dmax : 0;
  term[0] = t[3];
  term[1] = lx;
  term[2] = dx;
  return t[0] + (int64_t)I->w_tw * t[3] + (int64_t)I->w_load * lx + (int64_t)I->w_dur * dx;
}

/* The cost change of inserting customer x after the k-th customer of route R. */
static ins_t eval_insert(const ref_instance* I, int64_t wdep, const prt* R, int32_t ri, int32_t k, int32_t x,
                         int32_t* buf) {
  const int64_t N = (int64_t)I->n_depots + I->n_customers;
  int64_t t0[3], t1[3];
  const int64_t c0 = route_cost(I, wdep, R->start, R->x, R->len, R->end, t0);
  for (int32_t i = 0; i < k; ++i) buf[i] = R->x[i];
  buf[k] = x;
  for (int32_t i = k; i < R->len; ++i) buf[i + 1] = R->x[i];
  const int64_t c1 = route_cost(I, wdep, R->start, buf, R->len + 1, R->end, t1);
  ins_t r;
  r.dF = c1 - c0;
  r.feasible = t1[0] == t0[0] && t1[1] == t0[1] && t1[2] == t0[2];
  r.posid = k > 0 ? R->x[k - 1] : N + R->x[0];
  r.route = ri;
  r.k = k;
  return r;
}

static int ins_less(const ins_t* a, const ins_t* b) {
  return a->dF < b->dF || (a->dF == b->dF && a->posid < b->posid);
}

/* The depot of a new route (d, x, d) -- (d, x) when open: least cost change including
 * the fleet term, ties to the lower depot. */
static int32_t best_new_route(const ref_instance* I, int64_t wdep, const prt* R, int32_t nr, int32_t x,
                              int64_t* dF_out) {
  int32_t best = -1;
  int64_t bF = 0;
  for (int32_t d = 0; d < I->n_depots; ++d) {
    int64_t used = 0, term[3];
    for (int32_t r = 0; r < nr; ++r) used += R[r].start == d;
    const int64_t fx0 = used > I->NV ? used - I->NV : 0, fx1 = used + 1 > I->NV ? used + 1 - I->NV : 0;
    const int64_t f = route_cost(I, wdep, d, &x, 1, I->open_routes ? -1 : d, term) + wdep * (fx1 - fx0);
    if (best < 0 || f < bF) { best = d; bF = f; }
  }
  *dF_out = bF;
  return best;
}

static void insert_at(prt* R, int32_t k, int32_t x) {
  R->x = (int32_t*)realloc(R->x, sizeof(int32_t) * (size_t)(R->len + 1));
  memmove(R->x + k + 1, R->x + k, sizeof(int32_t) * (size_t)(R->len - k));
  R->x[k] = x;
  R->len += 1;
}

static int cmp_first(const void* a, const void* b) {
  const prt *x = (const prt*)a, *y = (const prt*)b;
  return x->x[0] - y->x[0];
}

int ref_repair(const ref_instance* I, int32_t n_routes, const int32_t* nodes, const int32_t* offs,
               const int32_t* start, const int32_t* end, int32_t op, uint64_t seed, int32_t* o_nroutes,
               int32_t* o_nodes, int32_t* o_offs, int32_t* o_start, int32_t* o_end, int32_t* order,
               int32_t* n_order, int64_t* n_evaluated) {
  const int32_t nd = I->n_depots, nc = I->n_customers;
  if (op < 0 || op > 4) return -1;
  int64_t st[4];
  ref_instance_stats(I, st);
  const int64_t wdep = st[3];
  prt* R = (prt*)calloc((size_t)nc + 1, sizeof(prt));
  char* routed = (char*)calloc((size_t)nd + nc, 1);
  int32_t nr = 0;
  for (int32_t r = 0; r < n_routes; ++r) {
    const int32_t L = offs[r + 1] - offs[r];
    if (L <= 0) continue;
    R[nr].start = start[r];
    R[nr].end = I->open_routes ? -1 : end[r];
    R[nr].len = L;
    R[nr].x = (int32_t*)malloc(sizeof(int32_t) * (size_t)L);
    for (int32_t i = 0; i < L; ++i) {
      R[nr].x[i] = nodes[offs[r] + i];
      routed[nodes[offs[r] + i]] = 1;
    }
    ++nr;
  }
  int32_t* U = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nc > 0 ? nc : 1));
  int32_t nu = 0;
  for (int32_t x = nd; x < nd + nc; ++x)
    if (!routed[x]) U[nu++] = x; /* ascending ids */
  int32_t* buf = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nc + 2));
  int64_t evals = 0;
  int32_t done = 0;
  char* taken = (char*)calloc((size_t)(nu > 0 ? nu : 1), 1);
  while (done < nu) {
    int32_t pick = -1; /* index into U */
    ins_t where;
    memset(&where, 0, sizeof where);
    int have = 0;
    if (op == 4) {
      /* random insertion: routes numbered by their first customer, ascending */
      pick = done;
      const int32_t x = U[pick];
      if (nr > 0) {
        qsort(R, (size_t)nr, sizeof(prt), cmp_first);
        uint64_t s = seed ^ (uint64_t)x;
        const uint64_t r1 = ref_splitmix64(&s), r2 = ref_splitmix64(&s);
        const int32_t ri = (int32_t)(r1 % (uint64_t)nr);
        const int32_t k = (int32_t)(r2 % (uint64_t)(R[ri].len + 1));
        where = eval_insert(I, wdep, &R[ri], ri, k, x, buf);
        evals += 1;
        have = 1;
      }
    } else {
      const int feas_only = op == 0 || op == 2, regret = op == 2 || op == 3;
      int64_t best_regret = 0;
      for (int32_t j = 0; j < nu; ++j) {
        if (taken[j]) continue;
        if (!regret && pick >= 0) break; /* best insertion: the next customer in id order */
        ins_t b1, b2;
        memset(&b1, 0, sizeof b1);
        memset(&b2, 0, sizeof b2);
        int n_adm = 0;
        for (int32_t r = 0; r < nr; ++r)
          for (int32_t k = 0; k <= R[r].len; ++k) {
            const ins_t c = eval_insert(I, wdep, &R[r], r, k, U[j], buf);
            evals += 1;
            if (feas_only && !c.feasible) continue;
            if (n_adm == 0 || ins_less(&c, &b1)) { b2 = b1; b1 = c; }
            else if (n_adm == 1 || ins_less(&c, &b2)) { b2 = c; }
            ++n_adm;
          }
        if (!regret) {
          pick = j;
          have = n_adm > 0;
          if (have) where = b1;
        } else {
          /* regret: second best minus best; fewer than two admissible positions first */
          const int64_t rg = n_adm >= 2 ? b2.dF - b1.dF : INT64_MAX;
          if (pick < 0 || rg > best_regret) {
            pick = j;
            best_regret = rg;
            have = n_adm > 0;
            if (have) where = b1;
          }
        }
      }
    }
    const int32_t x = U[pick];
    taken[pick] = 1;
    if (have) {
      insert_at(&R[where.route], where.k, x);
    } else {
      int64_t f;
      const int32_t d = best_new_route(I, wdep, R, nr, x, &f);
      R[nr].start = d;
      R[nr].end = I->open_routes ? -1 : d;
      R[nr].len = 1;
      R[nr].x = (int32_t*)malloc(sizeof(int32_t));
      R[nr].x[0] = x;
      ++nr;
    }
    order[done++] = x;
  }
  /* output: routes ordered by their first customer */
  qsort(R, (size_t)nr, sizeof(prt), cmp_first);
  int32_t w = 0;
  o_offs[0] = 0;
  for (int32_t r = 0; r < nr; ++r) {
    for (int32_t i = 0; i < R[r].len; ++i) o_nodes[w++] = R[r].x[i];
    o_offs[r + 1] = w;
    o_start[r] = R[r].start;
    o_end[r] = R[r].end;
    free(R[r].x);
  }
  *o_nroutes = nr;
  *n_order = nu;
  if (n_evaluated) *n_evaluated = evals;
  free(R);
  free(routed);
  free(U);
  free(buf);
  free(taken);
  return 0;
}
