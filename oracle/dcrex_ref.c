/*
 * dcrex_ref.c -- plain CPU oracle of the diversity-controlled route-exchange
 * crossover (Algorithm 3, Section 3.3): the four counts behind the score of a
 * route pair, the crossover itself, and the discounted UCB1 rule (Eq. 4) that
 * picks the diversity degree and the insertion operator.
 * TEST INFRASTRUCTURE ONLY (see mdvrp_ref.h). Shares no code with the HIP path.
 *
 * Every count is taken by scanning the explicit node lists of the routes.
 */
#include <stdlib.h>
#include <string.h>

#include "mdvrp_ref.h"

typedef struct {
  int32_t n;
  const int32_t *nodes, *offs, *start, *end;
} rset;

static int32_t rlen(const rset* S, int r) { return S->offs[r + 1] - S->offs[r]; }
static int32_t rnode(const rset* S, int r, int k) { return S->nodes[S->offs[r] + k]; }

/* the k-th arc of route r: (start, x1), (x1, x2), ..., (xL, end) unless open */
static int32_t n_arcs(const rset* S, int r) { return rlen(S, r) + (S->end[r] >= 0 ? 1 : 0); }
static void arc_at(const rset* S, int r, int k, int32_t* a, int32_t* b) {
  const int32_t L = rlen(S, r);
  *a = k == 0 ? S->start[r] : rnode(S, r, k - 1);
  *b = k < L ? rnode(S, r, k) : S->end[r];
}

static int route_has_arc(const rset* S, int r, int32_t a, int32_t b) {
  for (int k = 0; k < n_arcs(S, r); ++k) {
    int32_t x, y;
    arc_at(S, r, k, &x, &y);
    if (x == a && y == b) return 1;
  }
  return 0;
}

static int route_has_node(const rset* S, int r, int32_t y) {
  for (int k = 0; k < rlen(S, r); ++k)
    if (rnode(S, r, k) == y) return 1;
  return 0;
}

int ref_dcrex_counts(int32_t ns, const int32_t* s_nodes, const int32_t* s_offs, const int32_t* s_start,
                     const int32_t* s_end, const int32_t* s_intro, int32_t np, const int32_t* p_nodes,
                     const int32_t* p_offs, const int32_t* p_start, const int32_t* p_end, int32_t* EI, int32_t* NR,
                     int32_t* NM, int32_t* NC) {
  const rset S = {ns, s_nodes, s_offs, s_start, s_end};
  const rset P = {np, p_nodes, p_offs, p_start, p_end};
  for (int i = 0; i < ns; ++i)
    for (int j = 0; j < np; ++j) {
      int32_t ei = 0, nr = 0, nm = 0, nc = 0;
      /* new arcs: arcs of R_j that no other route of the offspring has */
      for (int k = 0; k < n_arcs(&P, j); ++k) {
        int32_t a, b;
        arc_at(&P, j, k, &a, &b);
        int found = 0;
        for (int r = 0; r < ns && !found; ++r)
          if (r != i && route_has_arc(&S, r, a, b)) found = 1;
        ei += !found;
      }
      /* redundant and conflicting nodes: customers of R_j already routed elsewhere in
         the offspring, and among those, in routes introduced from other parents */
      for (int k = 0; k < rlen(&P, j); ++k) {
        const int32_t y = rnode(&P, j, k);
        int other = 0, intro = 0;
        for (int r = 0; r < ns; ++r)
          if (r != i && route_has_node(&S, r, y)) {
            other = 1;
            if (s_intro[r]) intro = 1;
          }
        nm += other;
        nc += intro;
      }
      /* missing nodes: customers of R_i that R_j does not bring and no other route holds */
      for (int k = 0; k < rlen(&S, i); ++k) {
        const int32_t y = rnode(&S, i, k);
        if (route_has_node(&P, j, y)) continue;
        int other = 0;
        for (int r = 0; r < ns && !other; ++r)
          if (r != i && route_has_node(&S, r, y)) other = 1;
        nr += !other;
      }
      EI[(int64_t)i * np + j] = ei;
      NR[(int64_t)i * np + j] = nr;
      NM[(int64_t)i * np + j] = nm;
      NC[(int64_t)i * np + j] = nc;
    }
  return 0;
}

/* ---------------------------------------------------------------- discounted UCB1 (Eq. 4) */

/* ln x for x >= 1 from ln x = k ln 2 + 2 atanh((m - 1) / (m + 1)), m = x / 2^k in
 * [1, 2): the atanh series summed to a fixed 40 terms, every operation rounded on its
 * own. The same sequence runs in the library, so both take their argmax decisions on
 * identical doubles. */
double ref_ucb_ln(double x) {
  int k = 0;
  while (x >= 2.0) { x = x / 2.0; ++k; }
  const double z = (x - 1.0) / (x + 1.0), z2 = z * z;
  double term = z, s = 0.0;
  for (int n = 0; n < 40; ++n) {
    s = s + term / (double)(2 * n + 1);
    term = term * z2;
  }
  return (double)k * 0.6931471805599453 + 2.0 * s;
}

/* square root by Newton's iteration on x scaled into [1, 4) by powers of 4 (exact),
 * a fixed 8 steps from 1.5, every operation rounded on its own (the library runs the
 * same sequence). */
double ref_ucb_sqrt(double x) {
  if (!(x > 0.0)) return 0.0;
  double scale = 1.0;
  while (x >= 4.0) { x = x / 4.0; scale = scale * 2.0; }
  while (x < 1.0) { x = x * 4.0; scale = scale / 2.0; }
  double y = 1.5;
  for (int n = 0; n < 8; ++n) y = 0.5 * (y + x / y);
  return y * scale;
}

int32_t ref_ucb_select(int32_t n_arms, const double* R, const double* N) {
  /* an arm never played (count exactly 0) first, lowest index */
  for (int32_t a = 0; a < n_arms; ++a)
    if (N[a] == 0.0) return a;
  double tot = 0.0;
  for (int32_t a = 0; a < n_arms; ++a) tot = tot + N[a];
  const double ln_tot = tot > 1.0 ? ref_ucb_ln(tot) : 0.0;
  int32_t best = 0;
  double bv = 0.0;
  for (int32_t a = 0; a < n_arms; ++a) {
    const double v = R[a] / N[a] + ref_ucb_sqrt(2.0 * ln_tot / N[a]);
    if (a == 0 || v > bv) { bv = v; best = a; }
  }
  return best;
}

void ref_ucb_update(int32_t n_arms, double* R, double* N, int32_t arm, double reward, double gamma) {
  for (int32_t a = 0; a < n_arms; ++a) {
    R[a] = gamma * R[a];
    N[a] = gamma * N[a];
  }
  R[arm] = R[arm] + reward;
  N[arm] = N[arm] + 1.0;
}
