/*
 * mdvrp_ref.c -- plain, slow, deliberately literal CPU oracle.
 * TEST INFRASTRUCTURE ONLY (see mdvrp_ref.h). Shares no code with the HIP path.
 *
 * Every move is materialised as the explicit node lists of the routes it
 * produces; their cost is recomputed by walking the nodes. No prefix or
 * suffix data is kept anywhere in this file.
 */
#include "mdvrp_ref.h"

#include <omp.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int32_t start, end, len;
  int32_t* x;
} rroute;

typedef struct {
  int32_t nr;
  rroute* r;
} rsol;

#define NT(I) ((int64_t)(I)->n_depots + (I)->n_customers)
static int64_t cc(const ref_instance* I, int a, int b) { return I->c[(int64_t)a * NT(I) + b]; }
static int64_t tt(const ref_instance* I, int a, int b) { return I->t[(int64_t)a * NT(I) + b]; }
static int64_t mx(int64_t a, int64_t b) { return a > b ? a : b; }
static int64_t mn(int64_t a, int64_t b) { return a < b ? a : b; }
static int symmetric(const ref_instance* I) { return !I->has_tw; }

/* ------------------------------------------------------------------ instance statistics */

static int64_t gcd64(int64_t a, int64_t b) {
  if (a < 0) a = -a;
  if (b < 0) b = -b;
  while (b) { int64_t r = a % b; a = b; b = r; }
  return a;
}

/* Theta = 2*max c - min c over all edges (Eq. A.1); Gamma = sum c / sum t (Eq. 3, A.1). */
int ref_instance_stats(const ref_instance* I, int64_t out[4]) {
  int64_t n = NT(I), cmax = INT64_MIN, cmin = INT64_MAX, sc = 0, st = 0;
  for (int64_t a = 0; a < n; ++a)
    for (int64_t b = 0; b < n; ++b) {
      if (a == b) continue;
      int64_t v = cc(I, (int)a, (int)b);
      cmax = mx(cmax, v);
      cmin = mn(cmin, v);
      sc += v;
      st += tt(I, (int)a, (int)b);
    }
  if (n < 2) { cmax = 0; cmin = 0; }
  int64_t g = gcd64(sc, st);
  if (g == 0) g = 1;
  out[0] = 2 * cmax - cmin;
  out[1] = (st == 0) ? 1 : sc / g;
  out[2] = (st == 0) ? 1 : st / g;
  out[3] = I->w_depot < 0 ? out[0] : I->w_depot;
  return 0;
}

/* ------------------------------------------------------------------ granular lists */

typedef struct { __int128 key; int32_t v; } nkey;

static int nkey_cmp(const void* pa, const void* pb) {
  const nkey* a = (const nkey*)pa;
  const nkey* b = (const nkey*)pb;
  if (a->key != b->key) return a->key < b->key ? -1 : 1;
  return (a->v > b->v) - (a->v < b->v);
}

/* Section 3.2.3: drop arc i->j when e_i + s_i + t_ij > l_j (time windows only),
 * then keep the theta customers with the smallest correlation
 *   eta_ij = c_ij + Gamma*(alpha*max(e_j - l_i - s_i - t_ij, 0) + beta*max(l_i + s_i + t_ij - l_j, 0)),
 * alpha = 1, beta = 10 (Eq. 3), compared exactly as eta*den with Gamma = num/den;
 * ties go to the lower customer id. Without time windows eta = c. */
int ref_neighbours(const ref_instance* I, int32_t* nbr, int32_t* nbr_len) {
  int nd = I->n_depots, nc = I->n_customers, n = nd + nc, th = I->theta;
  if (th < 1) return -1;
  int64_t st[4];
  ref_instance_stats(I, st);
  __int128 num = st[1], den = st[2];
  nkey* buf = (nkey*)malloc(sizeof(nkey) * (size_t)(nc > 0 ? nc : 1));
  for (int u = nd; u < n; ++u) {
    int m = 0;
    for (int v = nd; v < n; ++v) {
      if (v == u) continue;
      __int128 key;
      if (I->has_tw) {
        int64_t ei = I->e[u], li = I->l[u], si = I->s[u], tij = tt(I, u, v), ej = I->e[v], lj = I->l[v];
        if (ei + si + tij > lj) continue; /* pruned arc */
        int64_t early = mx(ej - li - si - tij, 0);
        int64_t late = mx(li + si + tij - lj, 0);
        key = (__int128)cc(I, u, v) * den + num * ((__int128)1 * early + (__int128)10 * late);
      } else {
        key = cc(I, u, v);
      }
      buf[m].key = key;
      buf[m].v = v;
      ++m;
    }
    qsort(buf, (size_t)m, sizeof(nkey), nkey_cmp);
    int k = m < th ? m : th;
    for (int j = 0; j < th; ++j) nbr[(int64_t)(u - nd) * th + j] = j < k ? buf[j].v : -1;
    nbr_len[u - nd] = k;
  }
  free(buf);
  return 0;
}

/* ------------------------------------------------------------------ route cost */

/* Vidal's segment data: duration D, time warp TW, earliest start E, latest start L. */
typedef struct { int64_t D, TW, E, L; } twseg;

static twseg tw_node(const ref_instance* I, int x) {
  twseg r = {I->s[x], 0, I->e[x], I->l[x]};
  return r;
}

/* Concatenation of two segments joined by travel time tab (Vidal et al. 2013). */
static twseg tw_cat(twseg a, int64_t tab, twseg b) {
  int64_t delta = a.D - a.TW + tab;
  int64_t wait = mx(b.E - delta - a.L, 0);
  int64_t warp = mx(a.E + delta - b.L, 0);
  twseg r;
  r.D = a.D + b.D + tab + wait;
  r.TW = a.TW + b.TW + warp;
  r.E = mx(b.E - delta, a.E) - wait;
  r.L = mn(b.L - delta, a.L) + warp;
  return r;
}

typedef struct { int64_t dist, load, dur, tw; } rterm;

/* Walk one route (start depot, customers, end depot or -1 when open). */
static rterm route_terms(const ref_instance* I, int start, const int32_t* xs, int L, int end) {
  rterm o = {0, 0, 0, 0};
  int prev = start;
  twseg sg = tw_node(I, start);
  int64_t dur = I->s[start];
  for (int k = 0; k < L; ++k) {
    int x = xs[k];
    o.dist += cc(I, prev, x);
    o.load += I->q[x];
    if (I->has_tw) sg = tw_cat(sg, tt(I, prev, x), tw_node(I, x));
    else dur += tt(I, prev, x) + I->s[x];
    prev = x;
  }
  if (end >= 0) {
    o.dist += cc(I, prev, end);
    if (I->has_tw) sg = tw_cat(sg, tt(I, prev, end), tw_node(I, end));
    else dur += tt(I, prev, end) + I->s[end];
  }
  o.dur = I->has_tw ? sg.D : dur;
  o.tw = I->has_tw ? sg.TW : 0;
  return o;
}

int ref_route_terms(const ref_instance* I, int32_t start, const int32_t* xs, int32_t L, int32_t end, int64_t out[4]) {
  rterm t = route_terms(I, start, xs, L, end);
  out[0] = t.dist; out[1] = t.load; out[2] = t.dur; out[3] = t.tw;
  return 0;
}

static int64_t lx_of(const ref_instance* I, rterm t) { return mx(t.load - I->Q, 0); }
static int64_t dx_of(const ref_instance* I, rterm t) { return I->Dmax >= 0 ? mx(t.dur - I->Dmax, 0) : 0; }
static int64_t cost_of(const ref_instance* I, rterm t) {
  return t.dist + (int64_t)I->w_tw * t.tw + (int64_t)I->w_load * lx_of(I, t) + (int64_t)I->w_dur * dx_of(I, t);
}

/* Eq. A.1 with fixed weights: F = D + w_tw*TW + w_load*LX + w_dur*DX + w_depot*(CL + FX). */
int ref_cost(const ref_instance* I, int32_t n_routes, const int32_t* nodes, const int32_t* offs,
             const int32_t* start, const int32_t* end, int64_t* F, int64_t terms[6]) {
  int64_t st[4];
  ref_instance_stats(I, st);
  int64_t D = 0, TW = 0, LX = 0, DX = 0, CL = 0, FX = 0, cost = 0;
  int64_t* cnt = (int64_t*)calloc((size_t)I->n_depots, sizeof(int64_t));
  for (int r = 0; r < n_routes; ++r) {
    int L = offs[r + 1] - offs[r];
    if (L == 0) continue;
    rterm t = route_terms(I, start[r], nodes + offs[r], L, I->open_routes ? -1 : end[r]);
    D += t.dist; TW += t.tw; LX += lx_of(I, t); DX += dx_of(I, t);
    cost += cost_of(I, t);
    if (!I->open_routes && start[r] != end[r]) CL += 1;
    cnt[start[r]] += 1;
  }
  for (int d = 0; d < I->n_depots; ++d) FX += mx(cnt[d] - I->NV, 0);
  free(cnt);
  if (terms) { terms[0] = D; terms[1] = TW; terms[2] = LX; terms[3] = DX; terms[4] = CL; terms[5] = FX; }
  *F = cost + st[3] * (CL + FX);
  return 0;
}

/* ------------------------------------------------------------------ solutions */

static rsol sol_load(const ref_instance* I, int32_t n_routes, const int32_t* nodes, const int32_t* offs,
                     const int32_t* start, const int32_t* end) {
  rsol S;
  S.nr = 0;
  S.r = (rroute*)calloc((size_t)(n_routes > 0 ? n_routes : 1), sizeof(rroute));
  for (int r = 0; r < n_routes; ++r) {
    int L = offs[r + 1] - offs[r];
    if (L == 0) continue;
    rroute* R = &S.r[S.nr++];
    R->start = start[r];
    R->end = I->open_routes ? -1 : end[r];
    R->len = L;
    R->x = (int32_t*)malloc(sizeof(int32_t) * (size_t)L);
    memcpy(R->x, nodes + offs[r], sizeof(int32_t) * (size_t)L);
  }
  return S;
}

static void sol_free(rsol* S) {
  for (int r = 0; r < S->nr; ++r) free(S->r[r].x);
  free(S->r);
  S->r = NULL;
  S->nr = 0;
}

/* route index and 0-based index inside the route, per node */
typedef struct { int32_t* rt; int32_t* ix; int32_t* ndep; } rloc;

static rloc loc_build(const ref_instance* I, const rsol* S) {
  rloc L;
  int n = (int)NT(I);
  L.rt = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  L.ix = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  L.ndep = (int32_t*)calloc((size_t)I->n_depots, sizeof(int32_t));
  for (int i = 0; i < n; ++i) { L.rt[i] = -1; L.ix[i] = -1; }
  for (int r = 0; r < S->nr; ++r) {
    for (int k = 0; k < S->r[r].len; ++k) { L.rt[S->r[r].x[k]] = r; L.ix[S->r[r].x[k]] = k; }
    L.ndep[S->r[r].start] += 1;
  }
  return L;
}

static void loc_free(rloc* L) { free(L->rt); free(L->ix); free(L->ndep); }

/* ------------------------------------------------------------------ neighbours of a move */

/* A move replaces n_old existing routes by n_new new routes (new routes may be empty). */
typedef struct {
  int n_old, old[2];
  int n_new;
  int32_t nstart[2], nend[2], nlen[2];
  int32_t* nx[2];
} nbh;

static void push(nbh* m, int w, int x) { m->nx[w][m->nlen[w]++] = x; }
static void push_range(nbh* m, int w, const rroute* R, int a, int b) {
  for (int k = a; k <= b; ++k) push(m, w, R->x[k]);
}

/* node before / after index k of route R: a customer, the depot, or -1 (open end) */
static int pred_of(const rroute* R, int k) { return k > 0 ? R->x[k - 1] : R->start; }
static int succ_of(const rroute* R, int k) { return k + 1 < R->len ? R->x[k + 1] : R->end; }

/* Blocks: X is taken from route A at indices [xa, xb]; placed as X (in placement order).
 * Y is taken from route B at [ya, yb] (immediately before v). */

/* Relocate (Section 3.2.2): remove the block [xa,xb] of A and insert its placement
 * immediately before v (index j of B). */
static void build_rel(nbh* m, const rroute* A, int ai, const rroute* B, int bi, int xa, int xb,
                      const int* place, int np, int j) {
  m->n_new = 0;
  if (ai != bi) {
    m->n_old = 2; m->old[0] = ai; m->old[1] = bi;
    m->n_new = 2;
    m->nstart[0] = A->start; m->nend[0] = A->end; m->nlen[0] = 0;
    push_range(m, 0, A, 0, xa - 1);
    push_range(m, 0, A, xb + 1, A->len - 1);
    m->nstart[1] = B->start; m->nend[1] = B->end; m->nlen[1] = 0;
    push_range(m, 1, B, 0, j - 1);
    for (int k = 0; k < np; ++k) push(m, 1, place[k]);
    push_range(m, 1, B, j, B->len - 1);
  } else {
    m->n_old = 1; m->old[0] = ai;
    m->n_new = 1;
    m->nstart[0] = A->start; m->nend[0] = A->end; m->nlen[0] = 0;
    for (int k = 0; k < A->len; ++k) {
      if (k == j) for (int z = 0; z < np; ++z) push(m, 0, place[z]);
      if (k >= xa && k <= xb) continue;
      push(m, 0, A->x[k]);
    }
  }
}

/* Swap (Section 3.2.2): the X block goes to Y's place (before v), the Y block to X's place. */
static void build_swp(nbh* m, const rroute* A, int ai, const rroute* B, int bi, int xa, int xb,
                      const int* xplace, int nxp, int ya, int yb, const int* yplace, int nyp) {
  if (ai != bi) {
    m->n_old = 2; m->old[0] = ai; m->old[1] = bi;
    m->n_new = 2;
    m->nstart[0] = A->start; m->nend[0] = A->end; m->nlen[0] = 0;
    push_range(m, 0, A, 0, xa - 1);
    for (int k = 0; k < nyp; ++k) push(m, 0, yplace[k]);
    push_range(m, 0, A, xb + 1, A->len - 1);
    m->nstart[1] = B->start; m->nend[1] = B->end; m->nlen[1] = 0;
    push_range(m, 1, B, 0, ya - 1);
    for (int k = 0; k < nxp; ++k) push(m, 1, xplace[k]);
    push_range(m, 1, B, yb + 1, B->len - 1);
  } else {
    m->n_old = 1; m->old[0] = ai;
    m->n_new = 1;
    m->nstart[0] = A->start; m->nend[0] = A->end; m->nlen[0] = 0;
    for (int k = 0; k < A->len; ++k) {
      if (k == xa) for (int z = 0; z < nyp; ++z) push(m, 0, yplace[z]);
      if (k == ya) for (int z = 0; z < nxp; ++z) push(m, 0, xplace[z]);
      if ((k >= xa && k <= xb) || (k >= ya && k <= yb)) continue;
      push(m, 0, A->x[k]);
    }
  }
}

/* X block of u for 2-node kinds: o = 0 -> (p(u), u) in place; o = 1 -> (u, s(u)) placed as
 * (s(u), u). Returns 0 when the block does not exist. */
static int x_block(const ref_instance* I, const rroute* A, int i, int o, int* xa, int* xb, int* place) {
  if (o == 0) {
    if (i < 1) return 0;
    *xa = i - 1; *xb = i; place[0] = A->x[i - 1]; place[1] = A->x[i];
  } else {
    if (i + 1 >= A->len) return 0;
    *xa = i; *xb = i + 1; place[0] = A->x[i + 1]; place[1] = A->x[i];
  }
  (void)I;
  return 1;
}

/* Build the neighbour for a pair move anchored on (u, v): creates the arc u -> v. */
static int build_pair(const ref_instance* I, const rsol* S, const rloc* Lc, int kind, int var,
                      int u, int v, nbh* m) {
  int ai = Lc->rt[u], bi = Lc->rt[v];
  const rroute* A = &S->r[ai];
  const rroute* B = &S->r[bi];
  int i = Lc->ix[u], j = Lc->ix[v];
  int intra = (ai == bi);
  int su = succ_of(A, i);
  int pv = pred_of(B, j);
  int place[2], yplace[2], xa, xb, ya, yb;
  switch (kind) {
    case REF_REL1:
      if (var != 0) return 0;
      if (intra && v == su) return 0;
      place[0] = u;
      build_rel(m, A, ai, B, bi, i, i, place, 1, j);
      return 1;
    case REF_REL2:
      if (var > 1) return 0;
      if (var == 1 && !symmetric(I)) return 0;
      if (!x_block(I, A, i, var, &xa, &xb, place)) return 0;
      if (intra && j >= xa && j <= xb) return 0; /* v inside X */
      if (intra && v == su) return 0;            /* same place */
      build_rel(m, A, ai, B, bi, xa, xb, place, 2, j);
      return 1;
    case REF_SWP11:
      if (var != 0) return 0;
      if (j < 1 || pv == u) return 0;
      place[0] = u; yplace[0] = pv;
      build_swp(m, A, ai, B, bi, i, i, place, 1, j - 1, j - 1, yplace, 1);
      return 1;
    case REF_SWP21:
      if (var == 1 && !symmetric(I)) return 0;
      if (var > 1) return 0;
      if (!x_block(I, A, i, var, &xa, &xb, place)) return 0;
      if (j < 1) return 0;
      ya = yb = j - 1;
      if (intra && ((ya >= xa && ya <= xb) || (j >= xa && j <= xb))) return 0;
      yplace[0] = pv;
      build_swp(m, A, ai, B, bi, xa, xb, place, 2, ya, yb, yplace, 1);
      return 1;
    case REF_SWP12:
      if (var == 1 && !symmetric(I)) return 0;
      if (var > 1) return 0;
      if (j < 2) return 0;
      ya = j - 2; yb = j - 1;
      if (intra && i >= ya && i <= yb) return 0;
      place[0] = u;
      if (var == 0) { yplace[0] = B->x[j - 2]; yplace[1] = B->x[j - 1]; }
      else { yplace[0] = B->x[j - 1]; yplace[1] = B->x[j - 2]; }
      build_swp(m, A, ai, B, bi, i, i, place, 1, ya, yb, yplace, 2);
      return 1;
    case REF_SWP22: {
      int ox = var & 1, oy = (var >> 1) & 1;
      if (var > 3) return 0;
      if ((ox || oy) && !symmetric(I)) return 0;
      if (!x_block(I, A, i, ox, &xa, &xb, place)) return 0;
      if (j < 2) return 0;
      ya = j - 2; yb = j - 1;
      if (intra && ((ya <= xb && xa <= yb) || (j >= xa && j <= xb))) return 0;
      if (oy == 0) { yplace[0] = B->x[j - 2]; yplace[1] = B->x[j - 1]; }
      else { yplace[0] = B->x[j - 1]; yplace[1] = B->x[j - 2]; }
      build_swp(m, A, ai, B, bi, xa, xb, place, 2, ya, yb, yplace, 2);
      return 1;
    }
    case REF_X2:
      if (var != 0 || intra) return 0;
      /* 2-opt* (Section 3.2.2): A' = A[..i] + B[j..], B' = B[..j-1] + A[i+1..]; tails swap depots */
      m->n_old = 2; m->old[0] = ai; m->old[1] = bi;
      m->n_new = 2;
      m->nstart[0] = A->start; m->nend[0] = B->end; m->nlen[0] = 0;
      push_range(m, 0, A, 0, i);
      push_range(m, 0, B, j, B->len - 1);
      m->nstart[1] = B->start; m->nend[1] = A->end; m->nlen[1] = 0;
      push_range(m, 1, B, 0, j - 1);
      push_range(m, 1, A, i + 1, A->len - 1);
      return 1;
    case REF_2OPT:
      /* 2-opt (Section 3.2.2): reverse A[i+1..j]; creates u -> v and s(u) -> s(v). */
      if (var != 0 || !intra || !symmetric(I)) return 0;
      if (!(i < j - 1)) return 0;
      m->n_old = 1; m->old[0] = ai;
      m->n_new = 1;
      m->nstart[0] = A->start; m->nend[0] = A->end; m->nlen[0] = 0;
      push_range(m, 0, A, 0, i);
      for (int k = j; k >= i + 1; --k) push(m, 0, A->x[k]);
      push_range(m, 0, A, j + 1, A->len - 1);
      return 1;
    default:
      return 0;
  }
}

/* Depot-Insert (Section 3.2.2, Fig. 1a): cut route r after index k and put depot d
 * between the two parts, giving (start..x_k, d) and (d, x_{k+1}..end). */
static void build_dins(const ref_instance* I, const rsol* S, int r, int k, int d, nbh* m) {
  const rroute* A = &S->r[r];
  m->n_old = 1; m->old[0] = r;
  m->n_new = 2;
  m->nstart[0] = A->start; m->nend[0] = I->open_routes ? -1 : d; m->nlen[0] = 0;
  push_range(m, 0, A, 0, k);
  m->nstart[1] = d; m->nend[1] = A->end; m->nlen[1] = 0;
  push_range(m, 1, A, k + 1, A->len - 1);
}

/* Depot-Replace (Section 3.2.2, Fig. 1b): case 0 replaces the departure depot,
 * case 1 the arrival depot, case 2 both. */
static void build_drep(const rsol* S, int r, int d, int cs, nbh* m) {
  const rroute* A = &S->r[r];
  m->n_old = 1; m->old[0] = r;
  m->n_new = 1;
  m->nstart[0] = (cs == 0 || cs == 2) ? d : A->start;
  m->nend[0] = (cs == 1 || cs == 2) ? d : A->end;
  m->nlen[0] = 0;
  push_range(m, 0, A, 0, A->len - 1);
}

/* Delta of a neighbour: every changed route is recomputed from scratch. */
static void eval_nbh(const ref_instance* I, const rsol* S, const rloc* Lc, int64_t wdep, const nbh* m,
                     ref_move* o) {
  int64_t dc = 0, dD = 0, dTW = 0, dLX = 0, dDX = 0, dCL = 0;
  int dep[6], dd[6], nd = 0;
  for (int k = 0; k < m->n_old; ++k) {
    const rroute* R = &S->r[m->old[k]];
    rterm t = route_terms(I, R->start, R->x, R->len, R->end);
    dc -= cost_of(I, t); dD -= t.dist; dTW -= t.tw; dLX -= lx_of(I, t); dDX -= dx_of(I, t);
    if (R->end >= 0 && R->start != R->end) dCL -= 1;
    int f = -1;
    for (int z = 0; z < nd; ++z) if (dep[z] == R->start) f = z;
    if (f < 0) { f = nd++; dep[f] = R->start; dd[f] = 0; }
    dd[f] -= 1;
  }
  for (int k = 0; k < m->n_new; ++k) {
    if (m->nlen[k] == 0) continue; /* an emptied route is deleted */
    rterm t = route_terms(I, m->nstart[k], m->nx[k], m->nlen[k], m->nend[k]);
    dc += cost_of(I, t); dD += t.dist; dTW += t.tw; dLX += lx_of(I, t); dDX += dx_of(I, t);
    if (m->nend[k] >= 0 && m->nstart[k] != m->nend[k]) dCL += 1;
    int f = -1;
    for (int z = 0; z < nd; ++z) if (dep[z] == m->nstart[k]) f = z;
    if (f < 0) { f = nd++; dep[f] = m->nstart[k]; dd[f] = 0; }
    dd[f] += 1;
  }
  int64_t dFX = 0;
  int nres = 0;
  for (int k = 0; k < 3; ++k) o->res[k] = -1;
  for (int k = 0; k < m->n_old; ++k) o->res[nres++] = m->old[k];
  for (int z = 0; z < nd; ++z) {
    if (dd[z] == 0) continue;
    int64_t n0 = Lc->ndep[dep[z]];
    dFX += mx(n0 + dd[z] - I->NV, 0) - mx(n0 - I->NV, 0);
    if (nres < 3) o->res[nres] = -2 - dep[z];
    nres++;
  }
  o->dD = dD; o->dTW = dTW; o->dLX = dLX; o->dDX = dDX; o->dV4 = dCL + dFX;
  o->dF = dc + wdep * (dCL + dFX);
}

static uint64_t mk_id(int kind, int var, int a, int b) {
  return ((uint64_t)kind << 56) | ((uint64_t)var << 48) | ((uint64_t)a << 24) | (uint64_t)b;
}

typedef struct {
  ref_move* v;
  int64_t n, cap;
} mvec;

static void mv_push(mvec* M, const ref_move* m) {
  if (M->n == M->cap) {
    M->cap = M->cap ? 2 * M->cap : 1024;
    M->v = (ref_move*)realloc(M->v, sizeof(ref_move) * (size_t)M->cap);
  }
  M->v[M->n++] = *m;
}

static const int kinds_of_family[6][4] = {
    {REF_REL1, REF_REL2, -1, -1}, {REF_SWP11, REF_SWP21, REF_SWP12, REF_SWP22},
    {REF_X2, -1, -1, -1}, {REF_2OPT, -1, -1, -1}, {REF_DINS, -1, -1, -1}, {REF_DREP, -1, -1, -1}};

/* Evaluate every move of the families in fam_mask (Section 3.2.2 operators on the
 * granular lists of Section 3.2.3). */
static void eval_all(const ref_instance* I, const int32_t* nbr, const int32_t* nbr_len, const rsol* S,
                     uint32_t fam_mask, int64_t wdep, mvec* M) {
  rloc Lc = loc_build(I, S);
  nbh m;
  m.nx[0] = (int32_t*)malloc(sizeof(int32_t) * (size_t)(I->n_customers + 2));
  m.nx[1] = (int32_t*)malloc(sizeof(int32_t) * (size_t)(I->n_customers + 2));
  ref_move o;
  if (!symmetric(I)) fam_mask &= ~(1u << REF_FAM_2OPT);
  /* pair families */
  for (int fam = REF_FAM_REL; fam <= REF_FAM_2OPT; ++fam) {
    if (!(fam_mask & (1u << fam))) continue;
    for (int u = I->n_depots; u < (int)NT(I); ++u) {
      int ui = u - I->n_depots;
      for (int k = 0; k < nbr_len[ui]; ++k) {
        int v = nbr[(int64_t)ui * I->theta + k];
        for (int q = 0; q < 4; ++q) {
          int kind = kinds_of_family[fam][q];
          if (kind < 0) continue;
          for (int var = 0; var < 4; ++var) {
            if (!build_pair(I, S, &Lc, kind, var, u, v, &m)) continue;
            eval_nbh(I, S, &Lc, wdep, &m, &o);
            o.id = mk_id(kind, var, u, v);
            mv_push(M, &o);
          }
        }
      }
    }
  }
  if (fam_mask & (1u << REF_FAM_DINS)) {
    for (int r = 0; r < S->nr; ++r)
      for (int k = 0; k + 1 < S->r[r].len; ++k)
        for (int d = 0; d < I->n_depots; ++d) {
          build_dins(I, S, r, k, d, &m);
          eval_nbh(I, S, &Lc, wdep, &m, &o);
          o.id = mk_id(REF_DINS, 0, S->r[r].x[k], d);
          mv_push(M, &o);
        }
  }
  if (fam_mask & (1u << REF_FAM_DREP)) {
    for (int r = 0; r < S->nr; ++r) {
      const rroute* A = &S->r[r];
      for (int d = 0; d < I->n_depots; ++d) {
        int have = 0;
        ref_move best;
        int best_case = -1;
        for (int cs = 0; cs < 3; ++cs) {
          if (A->end < 0 && cs != 0) continue; /* open routes have no arrival depot */
          int ns = (cs == 0 || cs == 2) ? d : A->start;
          int ne = (cs == 1 || cs == 2) ? d : A->end;
          if (ns == A->start && ne == A->end) continue; /* identity */
          int dup = 0;                                 /* same route as an earlier case */
          for (int c2 = 0; c2 < cs; ++c2) {
            int s2 = (c2 == 0 || c2 == 2) ? d : A->start;
            int e2 = (c2 == 1 || c2 == 2) ? d : A->end;
            if (!(s2 == A->start && e2 == A->end) && s2 == ns && e2 == ne) dup = 1;
          }
          if (dup) continue;
          build_drep(S, r, d, cs, &m);
          eval_nbh(I, S, &Lc, wdep, &m, &o);
          if (!have || o.dF < best.dF) { best = o; best_case = cs; have = 1; }
        }
        if (have) {
          best.id = mk_id(REF_DREP, best_case, A->x[0], d);
          mv_push(M, &best);
        }
      }
    }
  }
  free(m.nx[0]);
  free(m.nx[1]);
  loc_free(&Lc);
}

int ref_eval(const ref_instance* I, const int32_t* nbr, const int32_t* nbr_len, int32_t n_routes,
             const int32_t* nodes, const int32_t* offs, const int32_t* start, const int32_t* end,
             uint32_t fam_mask, ref_move* out, int64_t cap, int64_t* count) {
  rsol S = sol_load(I, n_routes, nodes, offs, start, end);
  mvec M = {NULL, 0, 0};
  int64_t st[4];
  ref_instance_stats(I, st);
  eval_all(I, nbr, nbr_len, &S, fam_mask, st[3], &M);
  *count = M.n;
  int rc = 0;
  if (M.n > cap) rc = -3;
  else if (M.n) memcpy(out, M.v, sizeof(ref_move) * (size_t)M.n);
  free(M.v);
  sol_free(&S);
  return rc;
}

/* ------------------------------------------------------------------ selection */

static int key_cmp(const void* pa, const void* pb) {
  const ref_move* a = (const ref_move*)pa;
  const ref_move* b = (const ref_move*)pb;
  if (a->dF != b->dF) return a->dF < b->dF ? -1 : 1;
  return (a->id > b->id) - (a->id < b->id);
}

static int shares(const ref_move* a, const ref_move* b) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      if (a->res[i] != -1 && a->res[i] == b->res[j]) return 1;
  return 0;
}

/* Section 3.2.5: the leader is the best move; followers (dD < 0, no change in any
 * penalty term) are taken in ascending order when they share no route (and no
 * depot count) with a move already taken. Moves are sorted in place. */
static int64_t select_moves(ref_move* mv, int64_t n, int leader_only, ref_move* sel) {
  if (n == 0) return 0;
  qsort(mv, (size_t)n, sizeof(ref_move), key_cmp);
  if (mv[0].dF >= 0) return 0;
  int64_t ns = 0;
  sel[ns++] = mv[0];
  if (leader_only) return ns;
  for (int64_t k = 1; k < n; ++k) {
    const ref_move* f = &mv[k];
    if (!(f->dD < 0 && f->dTW == 0 && f->dLX == 0 && f->dDX == 0 && f->dV4 == 0)) continue;
    int ok = 1;
    for (int64_t z = 0; z < ns && ok; ++z) if (shares(f, &sel[z])) ok = 0;
    if (ok) sel[ns++] = *f;
  }
  return ns;
}

/* ------------------------------------------------------------------ apply */

static int rebuild_move(const ref_instance* I, const rsol* S, const rloc* Lc, uint64_t id, nbh* m) {
  int kind = (int)(id >> 56), var = (int)((id >> 48) & 0xff);
  int a = (int)((id >> 24) & 0xffffff), b = (int)(id & 0xffffff);
  if (kind <= REF_2OPT) return build_pair(I, S, Lc, kind, var, a, b, m);
  if (kind == REF_DINS) { build_dins(I, S, Lc->rt[a], Lc->ix[a], b, m); return 1; }
  if (kind == REF_DREP) { build_drep(S, Lc->rt[a], b, var, m); return 1; }
  return 0;
}

/* Apply a route-disjoint set of moves: changed routes are replaced, emptied routes
 * deleted, new routes appended. */
static void apply_moves(const ref_instance* I, rsol* S, const ref_move* sel, int64_t ns) {
  rloc Lc = loc_build(I, S);
  int nr = S->nr;
  char* gone = (char*)calloc((size_t)(nr > 0 ? nr : 1), 1);
  rroute* out = (rroute*)calloc((size_t)(nr + 2 * ns + 1), sizeof(rroute));
  int no = 0;
  nbh m;
  m.nx[0] = (int32_t*)malloc(sizeof(int32_t) * (size_t)(I->n_customers + 2));
  m.nx[1] = (int32_t*)malloc(sizeof(int32_t) * (size_t)(I->n_customers + 2));
  rroute* fresh = (rroute*)calloc((size_t)(2 * ns + 1), sizeof(rroute));
  int nf = 0;
  for (int64_t k = 0; k < ns; ++k) {
    rebuild_move(I, S, &Lc, sel[k].id, &m);
    for (int z = 0; z < m.n_old; ++z) gone[m.old[z]] = 1;
    for (int z = 0; z < m.n_new; ++z) {
      if (m.nlen[z] == 0) continue;
      rroute* R = &fresh[nf++];
      R->start = m.nstart[z]; R->end = m.nend[z]; R->len = m.nlen[z];
      R->x = (int32_t*)malloc(sizeof(int32_t) * (size_t)m.nlen[z]);
      memcpy(R->x, m.nx[z], sizeof(int32_t) * (size_t)m.nlen[z]);
    }
  }
  for (int r = 0; r < nr; ++r) {
    if (gone[r]) { free(S->r[r].x); continue; }
    out[no++] = S->r[r];
  }
  for (int z = 0; z < nf; ++z) out[no++] = fresh[z];
  free(S->r);
  S->r = out;
  S->nr = no;
  free(fresh);
  free(gone);
  free(m.nx[0]);
  free(m.nx[1]);
  loc_free(&Lc);
}

static void sol_store(const rsol* S, int32_t* o_nroutes, int32_t* o_nodes, int32_t* o_offs,
                      int32_t* o_start, int32_t* o_end, int32_t off0) {
  int32_t p = off0;
  for (int r = 0; r < S->nr; ++r) {
    o_offs[r] = p;
    o_start[r] = S->r[r].start;
    o_end[r] = S->r[r].end;
    for (int k = 0; k < S->r[r].len; ++k) o_nodes[p++] = S->r[r].x[k];
  }
  o_offs[S->nr] = p;
  if (o_nroutes) *o_nroutes = S->nr;
}

int ref_step(const ref_instance* I, const int32_t* nbr, const int32_t* nbr_len, int32_t n_routes,
             const int32_t* nodes, const int32_t* offs, const int32_t* start, const int32_t* end,
             uint32_t fam_mask, int32_t leader_only, int32_t* o_nroutes, int32_t* o_nodes,
             int32_t* o_offs, int32_t* o_start, int32_t* o_end, uint64_t* sel_ids, int64_t* sel_dF,
             int32_t* n_sel, int64_t* n_eval) {
  rsol S = sol_load(I, n_routes, nodes, offs, start, end);
  mvec M = {NULL, 0, 0};
  int64_t st[4];
  ref_instance_stats(I, st);
  eval_all(I, nbr, nbr_len, &S, fam_mask, st[3], &M);
  *n_eval = M.n;
  ref_move* sel = (ref_move*)malloc(sizeof(ref_move) * (size_t)(M.n + 1));
  int64_t ns = select_moves(M.v, M.n, leader_only, sel);
  for (int64_t k = 0; k < ns; ++k) { sel_ids[k] = sel[k].id; sel_dF[k] = sel[k].dF; }
  *n_sel = (int32_t)ns;
  if (ns) apply_moves(I, &S, sel, ns);
  sol_store(&S, o_nroutes, o_nodes, o_offs, o_start, o_end, 0);
  free(sel);
  free(M.v);
  sol_free(&S);
  return 0;
}

/* ------------------------------------------------------------------ local search */

/* SplitMix64 (Steele, Lea and Flood, 2014): state += golden gamma, then two
 * xor-shift-multiply rounds and a final xor-shift. */
/* SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): advance the state by the golden
 * gamma, then mix with two xor-shift-multiply rounds and a final xor-shift. */
uint64_t ref_splitmix64(uint64_t* s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* Algorithm 2 visits the operators in a random permutation each pass. */
int ref_family_order(int32_t has_tw, uint64_t seed, int64_t pass, int32_t* fam) {
  int n = 0;
  fam[n++] = REF_FAM_REL;
  fam[n++] = REF_FAM_SWP;
  fam[n++] = REF_FAM_X2;
  if (!has_tw) fam[n++] = REF_FAM_2OPT;
  fam[n++] = REF_FAM_DINS;
  fam[n++] = REF_FAM_DREP;
  uint64_t st = seed ^ (uint64_t)pass;
  for (int i = n - 1; i >= 1; --i) {
    int j = (int)(ref_splitmix64(&st) % (uint64_t)(i + 1));
    int tmp = fam[i]; fam[i] = fam[j]; fam[j] = tmp;
  }
  return n;
}

/* Terms of Eq. A.1 of a solution, every route walked node by node:
 * t = {D, TW, LX, DX, CL, FX}. */
static void sol_terms(const ref_instance* I, const rsol* S, int64_t t[6]) {
  int64_t* cnt = (int64_t*)calloc((size_t)I->n_depots, sizeof(int64_t));
  for (int k = 0; k < 6; ++k) t[k] = 0;
  for (int r = 0; r < S->nr; ++r) {
    const rroute* R = &S->r[r];
    rterm x = route_terms(I, R->start, R->x, R->len, R->end);
    t[0] += x.dist; t[1] += x.tw; t[2] += lx_of(I, x); t[3] += dx_of(I, x);
    if (R->end >= 0 && R->start != R->end) t[4] += 1;
    cnt[R->start] += 1;
  }
  for (int d = 0; d < I->n_depots; ++d) t[5] += mx(cnt[d] - I->NV, 0);
  free(cnt);
}

/* Dynamic penalty coefficients (Section 3.2.1; kappa = 0.5 in Table 1), integer form.
 * After an accepted step each coefficient is updated on its own: lambda / kappa (twice
 * the weight, at most w_max) when the current solution violates the constraint of its
 * term, lambda * kappa (half the weight, rounded down, at least w_min) when it does not.
 * Terms: V1 time warp, V2 load excess, V3 duration excess, V4 closure + fleet excess. */
static void adapt_weights(ref_instance* J, int64_t* wdep, const rsol* S, const ref_ls_options* opt) {
  int64_t t[6];
  sol_terms(J, S, t);
  const int viol[4] = {t[1] > 0, t[2] > 0, t[3] > 0, t[4] + t[5] > 0};
  int64_t w[4] = {J->w_tw, J->w_load, J->w_dur, *wdep};
  for (int i = 0; i < 4; ++i) {
    int64_t x = viol[i] ? 2 * w[i] : w[i] / 2;
    w[i] = mx(mn(x, opt->w_max[i]), opt->w_min[i]);
  }
  J->w_tw = (int32_t)w[0];
  J->w_load = (int32_t)w[1];
  J->w_dur = (int32_t)w[2];
  *wdep = w[3];
  J->w_depot = (int32_t)w[3];
}

static void ls_one(const ref_instance* I0, const int32_t* nbr, const int32_t* nbr_len, rsol* S,
                   const ref_ls_options* opt, int64_t wdep, ref_ls_stats* st) {
  memset(st, 0, sizeof(*st));
  /* the weights of this search (they change only with penalty_adapt) */
  ref_instance Jw = *I0;
  Jw.w_depot = (int32_t)wdep;
  ref_instance* I = &Jw;
  ref_move* sel = NULL;
  int64_t selcap = 0;
  const uint32_t all = (1u << 6) - 1;
  for (int64_t p = 0; opt->max_passes == 0 || p < opt->max_passes; ++p) {
    int32_t fam[6];
    int nf;
    uint32_t masks[6];
    if (opt->mode == 0) {
      nf = ref_family_order(I->has_tw, opt->seed, p, fam);
      for (int k = 0; k < nf; ++k) masks[k] = 1u << fam[k];
    } else {
      nf = 1;
      masks[0] = all;
    }
    st->passes += 1;
    int applied = 0;
    for (int k = 0; k < nf; ++k) {
      mvec M = {NULL, 0, 0};
      eval_all(I, nbr, nbr_len, S, masks[k], wdep, &M);
      st->evaluated += M.n;
      st->steps += 1;
      if (M.n + 1 > selcap) { selcap = M.n + 1; sel = (ref_move*)realloc(sel, sizeof(ref_move) * (size_t)selcap); }
      int64_t ns = select_moves(M.v, M.n, opt->leader_only, sel);
      if (ns) {
        apply_moves(I, S, sel, ns);
        applied = 1;
        st->moves_applied += ns;
        if (opt->penalty_adapt) adapt_weights(I, &wdep, S, opt);
      }
      free(M.v);
    }
    if (!applied) break;
  }
  free(sel);
  st->w_final[0] = I->w_tw;
  st->w_final[1] = I->w_load;
  st->w_final[2] = I->w_dur;
  st->w_final[3] = wdep;
}

int ref_local_search(const ref_instance* I, const int32_t* nbr, const int32_t* nbr_len, int32_t n_sol,
                     const int32_t* nodes, const int32_t* offs, const int32_t* start, const int32_t* end,
                     const int32_t* sol_offs, const ref_ls_options* opt, int32_t* o_nodes,
                     int32_t* o_offs, int32_t* o_start, int32_t* o_end, int32_t* o_sol_offs,
                     ref_ls_stats* stats) {
  /* with moving weights a search need not reach a fixed point: it runs to a depth */
  if (opt->penalty_adapt && opt->max_passes <= 0) return -1;
  rsol* S = (rsol*)calloc((size_t)(n_sol > 0 ? n_sol : 1), sizeof(rsol));
  int64_t ist[4];
  ref_instance_stats(I, ist);
#pragma omp parallel for schedule(dynamic, 1)
  for (int k = 0; k < n_sol; ++k) {
    int r0 = sol_offs[k], r1 = sol_offs[k + 1];
    int32_t* loffs = (int32_t*)malloc(sizeof(int32_t) * (size_t)(r1 - r0 + 1));
    for (int r = r0; r <= r1; ++r) loffs[r - r0] = offs[r] - offs[r0];
    S[k] = sol_load(I, r1 - r0, nodes + offs[r0], loffs, start + r0, end + r0);
    free(loffs);
    ls_one(I, nbr, nbr_len, &S[k], opt, ist[3], &stats[k]);
    int64_t terms[6];
    int32_t nr = S[k].nr;
    int32_t* tn = (int32_t*)malloc(sizeof(int32_t) * (size_t)(I->n_customers + 1));
    int32_t* to = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nr + 1));
    int32_t* ts = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nr + 1));
    int32_t* te = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nr + 1));
    sol_store(&S[k], NULL, tn, to, ts, te, 0);
    ref_instance Jw = *I; /* F under the weights the search ended with */
    Jw.w_tw = (int32_t)stats[k].w_final[0];
    Jw.w_load = (int32_t)stats[k].w_final[1];
    Jw.w_dur = (int32_t)stats[k].w_final[2];
    Jw.w_depot = (int32_t)stats[k].w_final[3];
    ref_cost(&Jw, nr, tn, to, ts, te, &stats[k].F, terms);
    free(tn); free(to); free(ts); free(te);
  }
  /* serial write-back in solution order */
  int32_t rr = 0, pp = 0;
  o_sol_offs[0] = 0;
  for (int k = 0; k < n_sol; ++k) {
    for (int r = 0; r < S[k].nr; ++r) {
      o_offs[rr] = pp;
      o_start[rr] = S[k].r[r].start;
      o_end[rr] = S[k].r[r].end;
      for (int z = 0; z < S[k].r[r].len; ++z) o_nodes[pp++] = S[k].r[r].x[z];
      ++rr;
    }
    o_sol_offs[k + 1] = rr;
    sol_free(&S[k]);
  }
  o_offs[rr] = pp;
  free(S);
  return 0;
}

/* Apply the moves with the given ids (route-disjoint) to a solution. */
int ref_apply_ids(const ref_instance* I, int32_t n_routes, const int32_t* nodes, const int32_t* offs,
                  const int32_t* start, const int32_t* end, const uint64_t* ids, int32_t n_ids,
                  int32_t* o_nroutes, int32_t* o_nodes, int32_t* o_offs, int32_t* o_start, int32_t* o_end) {
  rsol S = sol_load(I, n_routes, nodes, offs, start, end);
  ref_move* sel = (ref_move*)calloc((size_t)(n_ids > 0 ? n_ids : 1), sizeof(ref_move));
  for (int k = 0; k < n_ids; ++k) sel[k].id = ids[k];
  if (n_ids) apply_moves(I, &S, sel, n_ids);
  sol_store(&S, o_nroutes, o_nodes, o_offs, o_start, o_end, 0);
  free(sel);
  sol_free(&S);
  return 0;
}

/* Threads of the solution-parallel loop of ref_local_search (timing of the oracle
 * at one thread and at all host cores; the results do not depend on it). */
void ref_set_threads(int32_t n) { omp_set_num_threads(n > 0 ? n : 1); }
int32_t ref_get_threads(void) { return (int32_t)omp_get_max_threads(); }
