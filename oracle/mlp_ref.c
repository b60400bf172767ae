/*
 * mlp_ref.c -- plain CPU oracle of the learned move filter.
 * TEST INFRASTRUCTURE ONLY (see mdvrp_ref.h). Shares no code with the HIP path.
 *
 * The paper has no learned component; this follows the filter's own
 * definition: 32 integer features per anchor (u, v), each scaled by an fp32
 * reciprocal (one multiplication) and rounded to bf16 (round to nearest even);
 * an MLP 32 -> 256 -> 256 -> 1 with ReLU; BCE with logits; Adam.
 * The network arithmetic here is fp64. With round_act = 1 the weights, the
 * input and the two hidden activations are rounded to bf16 at the points
 * where the GPU path rounds them; with round_act = 0 the network is smooth
 * (used to check the backward pass against central finite differences).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "mdvrp_ref.h"

#define NT(I) ((int64_t)(I)->n_depots + (I)->n_customers)
#define H 256
#define F 32

static int64_t cc(const ref_instance* I, int a, int b) { return I->c[(int64_t)a * NT(I) + b]; }
static int64_t tt(const ref_instance* I, int a, int b) { return I->t[(int64_t)a * NT(I) + b]; }

/* fp32 -> bf16 with round to nearest even (NaN kept quiet). */
uint16_t ref_bf16(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}

float ref_bf16_to_f32(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}

/* ------------------------------------------------------------------ route facts for features */

typedef struct { int64_t load, dur, tw; } rfacts;

/* load, duration and time warp of a route: the evaluator's own route walk (one fold of
 * Vidal's concatenation for the whole oracle, pinned against departure-time enumeration) */
static rfacts route_facts(const ref_instance* I, int start, const int32_t* xs, int L, int end) {
  int64_t t[4];
  ref_route_terms(I, start, xs, L, end, t);
  rfacts o = {t[1], t[2], t[3]};
  return o;
}

/* Feature scales: mean nearest-neighbour distance (integer), capacity, depot
 * window length of depot 0 (time windows only). */
static void feature_scales(const ref_instance* I, const int32_t* nbr, const int32_t* nbr_len, float rcp[4]) {
  int64_t s = 0, n = 0;
  for (int i = 0; i < I->n_customers; ++i)
    if (nbr_len[i] > 0) {
      s += cc(I, I->n_depots + i, nbr[(int64_t)i * I->theta]);
      ++n;
    }
  int64_t dscale = n ? s / n : 1;
  if (dscale < 1) dscale = 1;
  int64_t hscale = I->has_tw ? (int64_t)I->l[0] - I->e[0] : 1;
  if (hscale < 1) hscale = 1;
  rcp[0] = 1.0f / (float)dscale;
  rcp[1] = 1.0f / (float)I->Q;
  rcp[2] = 1.0f / (float)hscale;
  rcp[3] = 1.0f / (float)I->n_depots;
}

static uint16_t feat(int64_t v, float rcp) {
  volatile float x = (float)v; /* one rounding int -> fp32 */
  volatile float y = x * rcp;  /* one rounding */
  return ref_bf16(y);
}

/* 32 bf16 features for every anchor (u, k-th entry of N(u)); out[(i*theta + k)*32 + f],
 * rows of missing entries are zero. */
int ref_filter_features(const ref_instance* I, const int32_t* nbr, const int32_t* nbr_len, int32_t n_routes,
                        const int32_t* nodes, const int32_t* offs, const int32_t* start, const int32_t* end,
                        uint16_t* out) {
  const int nd = I->n_depots, n = (int)NT(I), th = I->theta;
  float rcp[4];
  feature_scales(I, nbr, nbr_len, rcp);
  int32_t* rt = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* pos = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  rfacts* rf = (rfacts*)malloc(sizeof(rfacts) * (size_t)(n_routes > 0 ? n_routes : 1));
  for (int r = 0; r < n_routes; ++r) {
    const int L = offs[r + 1] - offs[r];
    for (int k = 0; k < L; ++k) { rt[nodes[offs[r] + k]] = r; pos[nodes[offs[r] + k]] = k + 1; }
    rf[r] = route_facts(I, start[r], nodes + offs[r], L, I->open_routes ? -1 : end[r]);
  }
  memset(out, 0, sizeof(uint16_t) * (size_t)I->n_customers * th * F);
  /* node at position p of route r: 0 = start depot, L+1 = end depot (or -1 when open) */
#define NODE_AT(r, p)                                                                                  \
  ((p) <= 0 ? start[r] : ((p) > offs[(r) + 1] - offs[r] ? (I->open_routes ? -1 : end[r]) : nodes[offs[r] + (p)-1]))
  for (int i = 0; i < I->n_customers; ++i) {
    const int u = nd + i;
    for (int k = 0; k < nbr_len[i]; ++k) {
      const int v = nbr[(int64_t)i * th + k];
      const int A = rt[u], B = rt[v];
      const int pu = pos[u], pv = pos[v];
      const int LA = offs[A + 1] - offs[A], LB = offs[B + 1] - offs[B];
      const int p_u = NODE_AT(A, pu - 1), s_u = NODE_AT(A, pu + 1);
      const int p_v = NODE_AT(B, pv - 1);
      const int pp_v = pv - 2 >= 0 ? NODE_AT(B, pv - 2) : p_v;
      const int64_t c_uv = cc(I, u, v), c_pu_u = cc(I, p_u, u);
      const int64_t c_u_su = s_u >= 0 ? cc(I, u, s_u) : 0;
      const int64_t c_pu_su = s_u >= 0 ? cc(I, p_u, s_u) : 0;
      const int64_t c_pv_v = cc(I, p_v, v), c_pv_u = cc(I, p_v, u);
      const int64_t c_pv_su = s_u >= 0 ? cc(I, p_v, s_u) : 0;
      int64_t iv[F];
      iv[0] = c_uv;
      iv[1] = c_pu_u;
      iv[2] = c_u_su;
      iv[3] = c_pu_su;
      iv[4] = c_pv_v;
      iv[5] = c_pv_u;
      iv[6] = c_pu_su - c_pu_u - c_u_su + c_pv_u + c_uv - c_pv_v;
      iv[7] = c_uv + c_pv_su - c_u_su - c_pv_v;
      iv[8] = cc(I, p_u, p_v) + c_pv_su + cc(I, pp_v, u) + c_uv - c_pu_u - c_u_su - cc(I, pp_v, p_v) - c_pv_v;
      iv[9] = rf[A].load - I->Q;
      iv[10] = rf[B].load - I->Q;
      iv[11] = I->q[u];
      iv[12] = I->q[v];
      iv[13] = I->Dmax >= 0 ? rf[A].dur - I->Dmax : 0;
      iv[14] = I->Dmax >= 0 ? rf[B].dur - I->Dmax : 0;
      iv[15] = rf[A].tw;
      iv[16] = rf[B].tw;
      if (I->has_tw) {
        const int64_t tuv = tt(I, u, v);
        iv[17] = (int64_t)I->l[u] - I->e[u];
        iv[18] = (int64_t)I->l[v] - I->e[v];
        iv[19] = I->e[u];
        iv[20] = I->e[v];
        iv[21] = I->e[v] - I->e[u] - I->s[u] - tuv > 0 ? I->e[v] - I->e[u] - I->s[u] - tuv : 0;
        iv[22] = I->e[u] + I->s[u] + tuv - I->l[v] > 0 ? I->e[u] + I->s[u] + tuv - I->l[v] : 0;
      } else {
        for (int z = 17; z <= 22; ++z) iv[z] = 0;
      }
      iv[23] = A == B;
      iv[24] = start[A] == start[B];
      iv[25] = start[A];
      iv[26] = start[B];
      iv[27] = LA;
      iv[28] = LB;
      iv[29] = pu;
      iv[30] = pv;
      iv[31] = k;
      uint16_t* o = out + ((int64_t)i * th + k) * F;
      for (int z = 0; z <= 8; ++z) o[z] = feat(iv[z], rcp[0]);
      for (int z = 9; z <= 12; ++z) o[z] = feat(iv[z], rcp[1]);
      for (int z = 13; z <= 22; ++z) o[z] = feat(iv[z], rcp[2]);
      o[23] = feat(iv[23], 1.0f);
      o[24] = feat(iv[24], 1.0f);
      o[25] = feat(iv[25], rcp[3]);
      o[26] = feat(iv[26], rcp[3]);
      o[27] = feat(iv[27], 1.0f / 32.0f);
      o[28] = feat(iv[28], 1.0f / 32.0f);
      o[29] = feat(iv[29], 1.0f / (float)LA);
      o[30] = feat(iv[30], 1.0f / (float)LB);
      o[31] = feat(iv[31], 1.0f / (float)th);
    }
  }
#undef NODE_AT
  free(rt);
  free(pos);
  free(rf);
  return 0;
}

/* ------------------------------------------------------------------ MLP */

/* parameter layout (fp32): W1[256][32], b1[256], W2[256][256], b2[256], w3[256], b3 */
enum { P_W1 = 0, P_B1 = P_W1 + H * F, P_W2 = P_B1 + H, P_B2 = P_W2 + H * H, P_W3 = P_B2 + H, P_B3 = P_W3 + H,
       P_N = P_B3 + 1 };

int ref_mlp_param_count(void) { return P_N; }

static double rnd(double x, int round_act) { return round_act ? ref_bf16_to_f32(ref_bf16((float)x)) : x; }

/* Forward of one sample; fills the hidden activations (after rounding when round_act). */
static double forward_one(const float* P, const uint16_t* x16, int round_act, double* h1, double* h2, double* z1,
                          double* z2) {
  double x[F];
  for (int i = 0; i < F; ++i) x[i] = ref_bf16_to_f32(x16[i]);
  for (int o = 0; o < H; ++o) {
    double s = 0;
    for (int i = 0; i < F; ++i) s += rnd(P[P_W1 + o * F + i], round_act) * x[i];
    s += P[P_B1 + o];
    z1[o] = s;
    h1[o] = rnd(s > 0 ? s : 0, round_act);
  }
  for (int o = 0; o < H; ++o) {
    double s = 0;
    for (int i = 0; i < H; ++i) s += rnd(P[P_W2 + o * H + i], round_act) * h1[i];
    s += P[P_B2 + o];
    z2[o] = s;
    h2[o] = rnd(s > 0 ? s : 0, round_act);
  }
  double z = P[P_B3];
  for (int o = 0; o < H; ++o) z += rnd(P[P_W3 + o], round_act) * h2[o];
  return z;
}

int ref_mlp_forward(const float* P, const uint16_t* x, int32_t n, int32_t round_act, double* logits) {
#pragma omp parallel for schedule(static)
  for (int p = 0; p < n; ++p) {
    double h1[H], h2[H], z1[H], z2[H];
    logits[p] = forward_one(P, x + (int64_t)p * F, round_act, h1, h2, z1, z2);
  }
  return 0;
}

/* Mean binary cross-entropy with logits; weights (nullable) scale each sample. */
double ref_bce(const double* z, const float* y, const float* w, int32_t n) {
  double s = 0, ws = 0;
  for (int p = 0; p < n; ++p) {
    const double wp = w ? w[p] : 1.0;
    const double l = (z[p] > 0 ? z[p] : 0) - z[p] * y[p] + log1p(exp(-fabs(z[p])));
    s += wp * l;
    ws += wp;
  }
  return ws > 0 ? s / ws : 0;
}

/* Gradient of sum_p dlogit[p] * logit_p with respect to every parameter. */
int ref_mlp_backward(const float* P, const uint16_t* x, int32_t n, const double* dlogits, int32_t round_act,
                     double* g) {
  memset(g, 0, sizeof(double) * P_N);
  for (int p = 0; p < n; ++p) {
    double h1[H], h2[H], z1[H], z2[H], d2[H], d1[H], xv[F];
    forward_one(P, x + (int64_t)p * F, round_act, h1, h2, z1, z2);
    for (int i = 0; i < F; ++i) xv[i] = ref_bf16_to_f32(x[(int64_t)p * F + i]);
    const double dz = dlogits[p];
    g[P_B3] += dz;
    for (int o = 0; o < H; ++o) {
      g[P_W3 + o] += dz * h2[o];
      d2[o] = z2[o] > 0 ? dz * rnd(P[P_W3 + o], round_act) : 0;
    }
    for (int o = 0; o < H; ++o) {
      g[P_B2 + o] += d2[o];
      for (int i = 0; i < H; ++i) g[P_W2 + o * H + i] += d2[o] * h1[i];
    }
    for (int i = 0; i < H; ++i) {
      double s = 0;
      for (int o = 0; o < H; ++o) s += d2[o] * rnd(P[P_W2 + o * H + i], round_act);
      d1[i] = z1[i] > 0 ? s : 0;
    }
    for (int o = 0; o < H; ++o) {
      g[P_B1 + o] += d1[o];
      for (int i = 0; i < F; ++i) g[P_W1 + o * F + i] += d1[o] * xv[i];
    }
  }
  return 0;
}

/* Adam (beta1 0.9, beta2 0.999, eps 1e-8) on fp32 parameters and moments. */
int ref_adam(float* P, float* m, float* v, const float* g, int32_t n, float lr, int32_t step) {
  const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
  const double c1 = 1.0 - pow(b1, step), c2 = 1.0 - pow(b2, step);
  for (int i = 0; i < n; ++i) {
    m[i] = (float)(b1 * m[i] + (1 - b1) * g[i]);
    v[i] = (float)(b2 * v[i] + (1 - b2) * (double)g[i] * g[i]);
    const double mh = m[i] / c1, vh = v[i] / c2;
    P[i] = (float)(P[i] - lr * mh / (sqrt(vh) + eps));
  }
  return 0;
}

/* The k entries with the largest scores per customer (ties -> lower customer id);
 * out[i*k + j], -1 padding. */
int ref_topk(const int32_t* nbr, const int32_t* nbr_len, int32_t n_customers, int32_t theta, const float* score,
             int32_t k, int32_t* out) {
  for (int i = 0; i < n_customers; ++i) {
    char used[256] = {0};
    for (int j = 0; j < k; ++j) {
      int best = -1;
      for (int q = 0; q < nbr_len[i] && q < 256; ++q) {
        if (used[q]) continue;
        if (best < 0) { best = q; continue; }
        const float a = score[(int64_t)i * theta + q], b = score[(int64_t)i * theta + best];
        const int va = nbr[(int64_t)i * theta + q], vb = nbr[(int64_t)i * theta + best];
        if (a > b || (a == b && va < vb)) best = q;
      }
      out[(int64_t)i * k + j] = best < 0 ? -1 : nbr[(int64_t)i * theta + best];
      if (best >= 0) used[best] = 1;
    }
  }
  return 0;
}
