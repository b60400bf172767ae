/*
 * pop_ref.c -- plain CPU oracle of the population measures of Section 3.4:
 * the distance between two solutions (Eq. 7), the distance of a solution to
 * the population (Eq. 6), the fitness-and-distance score chi (Eq. 5), and the
 * reduction of an expanded population back to mu solutions.
 * TEST INFRASTRUCTURE ONLY (see mdvrp_ref.h). Shares no code with the HIP path.
 *
 * Every edge set is built explicitly as a sorted list of arcs; the intersection
 * is a merge of two sorted lists. Ranks are found by sorting.
 */
#include <stdlib.h>
#include <string.h>

#include "mdvrp_ref.h"

/* The edges of one solution: the arcs (n_k, n_{k+1}) along each route,
 * from its departure depot to its last customer and, unless the route is open
 * (end < 0), on to its arrival depot. Each arc a -> b is coded a * N + b. */
static int cmp_i64(const void* x, const void* y) {
  const int64_t a = *(const int64_t*)x, b = *(const int64_t*)y;
  return a < b ? -1 : (a > b ? 1 : 0);
}

static int64_t edge_set(int64_t N, int32_t r0, int32_t r1, const int32_t* nodes, const int32_t* offs,
                        const int32_t* start, const int32_t* end, int64_t** out) {
  int64_t cap = 0;
  for (int32_t r = r0; r < r1; ++r) cap += (offs[r + 1] - offs[r]) + 1;
  int64_t* e = (int64_t*)malloc(sizeof(int64_t) * (size_t)(cap > 0 ? cap : 1));
  int64_t n = 0;
  for (int32_t r = r0; r < r1; ++r) {
    int32_t prev = start[r];
    for (int32_t k = offs[r]; k < offs[r + 1]; ++k) {
      e[n++] = (int64_t)prev * N + nodes[k];
      prev = nodes[k];
    }
    if (end[r] >= 0) e[n++] = (int64_t)prev * N + end[r];
  }
  qsort(e, (size_t)n, sizeof(int64_t), cmp_i64);
  *out = e;
  return n;
}

static int64_t common_count(const int64_t* a, int64_t na, const int64_t* b, int64_t nb) {
  int64_t i = 0, j = 0, c = 0;
  while (i < na && j < nb) {
    if (a[i] < b[j]) ++i;
    else if (a[i] > b[j]) ++j;
    else { ++c; ++i; ++j; }
  }
  return c;
}

int ref_population_distance(const ref_instance* I, int32_t n_sol, const int32_t* nodes, const int32_t* offs,
                            const int32_t* start, const int32_t* end, const int32_t* sol_offs, double* dist,
                            int64_t* common, int64_t* n_edges) {
  if (n_sol < 1) return -1;
  const int64_t N = (int64_t)I->n_depots + I->n_customers;
  int64_t** E = (int64_t**)calloc((size_t)n_sol, sizeof(int64_t*));
  int64_t* nE = (int64_t*)calloc((size_t)n_sol, sizeof(int64_t));
  for (int32_t k = 0; k < n_sol; ++k) nE[k] = edge_set(N, sol_offs[k], sol_offs[k + 1], nodes, offs, start, end, &E[k]);
  for (int32_t i = 0; i < n_sol; ++i)
    for (int32_t j = 0; j < n_sol; ++j) {
      const int64_t c = common_count(E[i], nE[i], E[j], nE[j]);
      const int64_t m = nE[i] > nE[j] ? nE[i] : nE[j];
      /* Eq. 7 */
      dist[(int64_t)i * n_sol + j] = m > 0 ? 100.0 * (1.0 - (double)c / (double)m) : 0.0;
      if (common) common[(int64_t)i * n_sol + j] = c;
    }
  if (n_edges)
    for (int32_t k = 0; k < n_sol; ++k) n_edges[k] = nE[k];
  for (int32_t k = 0; k < n_sol; ++k) free(E[k]);
  free(E);
  free(nE);
  return 0;
}

/* sort keys of the rankings */
typedef struct {
  double v;
  int64_t f;
  int32_t idx;
} rkey;

static int cmp_near(const void* x, const void* y) { /* distance ascending, index ascending */
  const rkey *a = (const rkey*)x, *b = (const rkey*)y;
  if (a->v != b->v) return a->v < b->v ? -1 : 1;
  return a->idx - b->idx;
}
static int cmp_f(const void* x, const void* y) { /* objective ascending, index ascending */
  const rkey *a = (const rkey*)x, *b = (const rkey*)y;
  if (a->f != b->f) return a->f < b->f ? -1 : 1;
  return a->idx - b->idx;
}
static int cmp_far(const void* x, const void* y) { /* population distance descending, index ascending */
  const rkey *a = (const rkey*)x, *b = (const rkey*)y;
  if (a->v != b->v) return a->v > b->v ? -1 : 1;
  return a->idx - b->idx;
}

/* chi of every alive solution (Eq. 5 and Eq. 6) given the distance matrix. */
static void chi_scores(int32_t n, const double* dist, const int64_t* f, const int* alive, double xi, int32_t n_close,
                       double* dpop, double* chi) {
  int32_t m = 0;
  for (int32_t i = 0; i < n; ++i) m += alive[i];
  rkey* tmp = (rkey*)malloc(sizeof(rkey) * (size_t)(n > 0 ? n : 1));
  int32_t* rank_f = (int32_t*)calloc((size_t)n, sizeof(int32_t));
  int32_t* rank_d = (int32_t*)calloc((size_t)n, sizeof(int32_t));
  /* Eq. 6: mean distance to the n_close nearest other solutions */
  for (int32_t i = 0; i < n; ++i) {
    if (!alive[i]) continue;
    int32_t k = 0;
    for (int32_t j = 0; j < n; ++j)
      if (alive[j] && j != i) { tmp[k].v = dist[(int64_t)i * n + j]; tmp[k].idx = j; ++k; }
    qsort(tmp, (size_t)k, sizeof(rkey), cmp_near);
    const int32_t c = k < n_close ? k : n_close;
    double s = 0.0;
    for (int32_t z = 0; z < c; ++z) s += tmp[z].v;
    dpop[i] = c > 0 ? s / (double)c : 0.0;
  }
  int32_t k = 0;
  for (int32_t i = 0; i < n; ++i)
    if (alive[i]) { tmp[k].f = f[i]; tmp[k].v = dpop[i]; tmp[k].idx = i; ++k; }
  qsort(tmp, (size_t)k, sizeof(rkey), cmp_f);
  for (int32_t z = 0; z < k; ++z) rank_f[tmp[z].idx] = z + 1;
  qsort(tmp, (size_t)k, sizeof(rkey), cmp_far);
  for (int32_t z = 0; z < k; ++z) rank_d[tmp[z].idx] = z + 1;
  /* Eq. 5 */
  for (int32_t i = 0; i < n; ++i) {
    if (!alive[i]) continue;
    const double a = (double)(m - rank_f[i]) / (double)m;
    const double b = (double)(m - rank_d[i]) / (double)m;
    chi[i] = a + xi * b;
  }
  free(tmp);
  free(rank_f);
  free(rank_d);
}

int ref_population_reduce(int32_t n, const double* dist, const int64_t* f, int32_t mu, double xi, int32_t n_close,
                          int32_t* keep, int32_t* order, double* chi_first, double* dpop_first) {
  if (n < 1 || mu < 1 || n_close < 1) return -1;
  int* alive = (int*)malloc(sizeof(int) * (size_t)n);
  double* chi = (double*)malloc(sizeof(double) * (size_t)n);
  double* dpop = (double*)malloc(sizeof(double) * (size_t)n);
  for (int32_t i = 0; i < n; ++i) alive[i] = 1;
  int32_t m = n, removed = 0;
  for (int first = 1;; first = 0) {
    chi_scores(n, dist, f, alive, xi, n_close, dpop, chi);
    if (first) {
      for (int32_t i = 0; i < n; ++i) {
        if (chi_first) chi_first[i] = chi[i];
        if (dpop_first) dpop_first[i] = dpop[i];
      }
    }
    if (m <= mu) break;
    /* the solution of lowest chi leaves; on a tie the one of higher index */
    int32_t w = -1;
    for (int32_t i = 0; i < n; ++i)
      if (alive[i] && (w < 0 || chi[i] <= chi[w])) w = i;
    alive[w] = 0;
    order[removed++] = w;
    --m;
  }
  for (int32_t i = 0; i < n; ++i) keep[i] = alive[i];
  free(alive);
  free(chi);
  free(dpop);
  return 0;
}
