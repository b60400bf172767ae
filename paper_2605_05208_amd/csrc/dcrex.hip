// dcrex.hip -- the data-parallel pieces of the diversity-controlled route-exchange
// crossover (Algorithm 3, Section 3.3) and its discounted UCB1 rule (Eq. 4):
//   * the four counts behind the score of every route pair (R_i of the offspring,
//     R_j of a parent): new arcs, missing, redundant and conflicting nodes;
//   * the random choice among the five lowest-scored pairs;
//   * UCB1 selection and update of a bandit's discounted statistics.
// The offspring may hold a customer in several routes (that is what the counts
// measure), so it is given as plain route lists, not as a batch unit.
//
// Counting plan: every occurrence of a customer y in the offspring is recorded in a
// per-node table (route, predecessor, successor; up to kOccMax per node); then each
// parent arc and customer learns how many offspring routes hold it and, when exactly
// one does, which. A pair (i, j) then needs one pass over R_j and one over R_i: an
// arc of R_j is new unless an offspring route other than R_i holds it, and so on.
#include "../../include/mdvrp.h"
#include "kernels.h"

namespace mdvrp {

constexpr int kDcrexBlock = 256;

struct OccTab {
  int32_t* n;      // [N] occurrences in the offspring
  int32_t* n_in;   // [N] occurrences in introduced routes
  int32_t* r_in;   // [N] an introduced route holding the node (meaningful when n_in == 1)
  int4* occ;       // [N * kOccMax] {route, predecessor, successor, 0}
  int32_t* err;    // [1] set when a node occurs more than kOccMax times
};

// Per parent position (arcs and customers of the parent in route order): how many
// offspring routes hold it, and one route that does.
struct ParentInfo {
  int2* arc;       // [p_len + np] {count, route} of the arc entering position k (the arc out of
                   // the departure depot for k = 0 of a route; the arc into the arrival depot last)
  int4* node;      // [p_len] {count, route, count in introduced routes, introduced route}
  int32_t* route_of;  // [N] parent route holding each customer (-1 for depots)
};

__global__ void k_fill_i32(int32_t* p, int n, int32_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Route of each flat position: route r owns positions offs[r] .. offs[r + 1] - 1.
__device__ __forceinline__ int route_of_pos(const int32_t* __restrict__ offs, int nr, int pos) {
  int lo = 0, hi = nr;  // offs[lo] <= pos < offs[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (ld(offs, mid) <= pos) lo = mid; else hi = mid;
  }
  return lo;
}

// Every occurrence of a customer in the offspring.
__global__ void k_dcrex_occ(int ns, int s_len, const int32_t* __restrict__ nodes, const int32_t* __restrict__ offs,
                            const int32_t* __restrict__ start, const int32_t* __restrict__ end,
                            const int32_t* __restrict__ intro, OccTab T) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= s_len) return;
  const int r = route_of_pos(offs, ns, p);
  const int a = ld(offs, r), b = ld(offs, r + 1);
  const int y = ld(nodes, p);
  const int pred = p > a ? ld(nodes, p - 1) : ld(start, r);
  const int succ = p + 1 < b ? ld(nodes, p + 1) : ld(end, r);
  const int k = atomicAdd(&T.n[y], 1);
  if (k < kOccMax) T.occ[(int64_t)y * kOccMax + k] = make_int4(r, pred, succ, 0);
  else atomicOr(T.err, 1);
  if (ld(intro, r)) {
    atomicAdd(&T.n_in[y], 1);
    T.r_in[y] = r;  // the one writer when n_in ends at 1
  }
}

// Parent arcs and customers against the offspring table.
__global__ void k_dcrex_parent(int np, int p_len, int n_depots, const int32_t* __restrict__ nodes,
                               const int32_t* __restrict__ offs, const int32_t* __restrict__ start,
                               const int32_t* __restrict__ end, OccTab T, ParentInfo P) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= p_len + np) return;
  // arcs are enumerated route by route: route r has (offs[r+1] - offs[r]) + 1 arc slots
  // (the last unused for an open route); arc slot k of the whole list belongs to route
  // r with offs[r] + r <= k < offs[r + 1] + r + 1
  int lo = 0, hi = np;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (ld(offs, mid) + mid <= k) lo = mid; else hi = mid;
  }
  const int r = lo;
  const int a0 = ld(offs, r), L = ld(offs, r + 1) - a0;
  const int q = k - (a0 + r);  // arc q of route r enters position q + 1 (q = L: the arrival depot)
  const int from = q == 0 ? ld(start, r) : ld(nodes, a0 + q - 1);
  const int to = q < L ? ld(nodes, a0 + q) : ld(end, r);
  int cnt = 0, rt = -1;
  if (to >= 0) {
    // an arc out of a customer: occurrences of `from` followed by `to`; out of a depot:
    // occurrences of `to` preceded by that depot (a depot only precedes position 1)
    const bool from_customer = from >= n_depots;
    const int y = from_customer ? from : to;
    const int ny = imin(T.n[y], kOccMax);
    for (int z = 0; z < ny; ++z) {
      const int4 o = T.occ[(int64_t)y * kOccMax + z];
      if (from_customer ? o.z == to : o.y == from) {
        ++cnt;
        rt = o.x;
      }
    }
  } else {
    cnt = -1;  // no arc (open route end)
  }
  P.arc[k] = make_int2(cnt, rt);
  if (q < L) {
    const int y = ld(nodes, a0 + q);
    P.route_of[y] = r;
    const int ny = T.n[y];
    const int rr = ny >= 1 ? T.occ[(int64_t)y * kOccMax].x : -1;
    P.node[a0 + q] = make_int4(ny, rr, T.n_in[y], T.r_in[y]);
  }
}

// One thread per pair (i, j), j the slow index.
__global__ void k_dcrex_pairs(int ns, int np, const int32_t* __restrict__ s_nodes, const int32_t* __restrict__ s_offs,
                              const int32_t* __restrict__ p_offs, OccTab T, ParentInfo P, int32_t* EI, int32_t* NR,
                              int32_t* NM, int32_t* NC) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)ns * np) return;
  const int j = (int)(t / ns), i = (int)(t - (int64_t)j * ns);
  const int pa = ld(p_offs, j), pb = ld(p_offs, j + 1);
  int ei = 0, nm = 0, nc = 0, nr = 0;
  // arcs of R_j: slots pa + j .. pb + j
  for (int k = pa + j; k <= pb + j; ++k) {
    const int2 a = P.arc[k];
    if (a.x < 0) continue;                          // the missing arc of an open route
    ei += (a.x == 0 || (a.x == 1 && a.y == i));     // held by no offspring route but R_i
  }
  for (int k = pa; k < pb; ++k) {
    const int4 v = P.node[k];
    nm += (v.x >= 2 || (v.x == 1 && v.y != i));
    nc += (v.z >= 2 || (v.z == 1 && v.w != i));
  }
  // customers of R_i that R_j does not bring back and that no other offspring route holds
  const int sa = ld(s_offs, i), sb = ld(s_offs, i + 1);
  for (int k = sa; k < sb; ++k) {
    const int y = ld(s_nodes, k);
    nr += (P.route_of[y] != j && T.n[y] == 1);
  }
  const int64_t o = (int64_t)i * np + j;
  EI[o] = ei;
  NR[o] = nr;
  NM[o] = nm;
  NC[o] = nc;
}

// The five lowest pairs by (score, i, j) -- score = -(EI - NR - NM - 10 NC) -- and one
// of them chosen by SplitMix64(seed) mod their number (Algorithm 3). out = {i, j, diversity
// increase EI + NR + NM, candidates}.
__global__ __launch_bounds__(kDcrexBlock) void k_dcrex_pick(int ns, int np, const int32_t* __restrict__ EI,
                                                            const int32_t* __restrict__ NR,
                                                            const int32_t* __restrict__ NM,
                                                            const int32_t* __restrict__ NC, uint64_t seed,
                                                            int32_t* out) {
  constexpr int K = 5;
  uint64_t best[K];
#pragma unroll
  for (int z = 0; z < K; ++z) best[z] = ~0ull;
  const int64_t n = (int64_t)ns * np;
  for (int64_t t = threadIdx.x; t < n; t += kDcrexBlock) {
    const int64_t score = -((int64_t)EI[t] - NR[t] - NM[t] - 10 * (int64_t)NC[t]);
    // (score, i, j) order = (score, flat index i * np + j): packed sortable key
    const uint64_t key = ((uint64_t)(score + (1ll << 31)) << 32) | (uint64_t)t;
    if (key < best[K - 1]) {
      best[K - 1] = key;
#pragma unroll
      for (int z = K - 1; z > 0; --z)
        if (best[z] < best[z - 1]) { const uint64_t x = best[z]; best[z] = best[z - 1]; best[z - 1] = x; }
    }
  }
  __shared__ uint64_t s_min[kDcrexBlock / 64];
  __shared__ uint64_t s_top[K];
  for (int z = 0; z < K; ++z) {
    uint64_t m = best[0];
    for (int o = 32; o > 0; o >>= 1) {
      const uint64_t g = __shfl_xor(m, o);
      m = g < m ? g : m;
    }
    if ((threadIdx.x & 63) == 0) s_min[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint64_t w = s_min[0];
      for (int v = 1; v < kDcrexBlock / 64; ++v) w = s_min[v] < w ? s_min[v] : w;
      s_top[z] = w;
    }
    __syncthreads();
    const uint64_t w = s_top[z];
    if (best[0] == w && w != ~0ull) {  // the owner pops its head (keys are unique)
#pragma unroll
      for (int y = 0; y < K - 1; ++y) best[y] = best[y + 1];
      best[K - 1] = ~0ull;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int cnt = (int)(n < K ? n : K);
    if (cnt == 0) {
      out[0] = -1; out[1] = -1; out[2] = 0; out[3] = 0;
      return;
    }
    uint64_t st = seed;
    const int pick = (int)(splitmix64_next(&st) % (uint64_t)cnt);
    const int64_t t = (int64_t)(s_top[pick] & 0xffffffffull);
    out[0] = (int32_t)(t / np);
    out[1] = (int32_t)(t - (t / np) * np);
    out[2] = EI[t] + NR[t] + NM[t];
    out[3] = cnt;
  }
}

// ---------------------------------------------------------------- discounted UCB1 (Eq. 4)

// ln x (x >= 1) and sqrt x by fixed operation sequences, each operation rounded on its
// own, so that the arm choice does not depend on a math library's last bit:
// ln x = k ln 2 + 2 atanh((m - 1)/(m + 1)) with m = x / 2^k in [1, 2), 40 series terms;
// sqrt by 8 Newton steps from 1.5 on x scaled into [1, 4) by powers of 4.
__device__ double ucb_ln(double x) {
#pragma clang fp contract(off)
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

__device__ double ucb_sqrt(double x) {
#pragma clang fp contract(off)
  if (!(x > 0.0)) return 0.0;
  double scale = 1.0;
  while (x >= 4.0) { x = x / 4.0; scale = scale * 2.0; }
  while (x < 1.0) { x = x * 4.0; scale = scale / 2.0; }
  double y = 1.5;
  for (int n = 0; n < 8; ++n) y = 0.5 * (y + x / y);
  return y * scale;
}

__global__ void k_ucb_select(int n_arms, const double* __restrict__ R, const double* __restrict__ N, int32_t* arm) {
#pragma clang fp contract(off)
  if (threadIdx.x != 0) return;
  for (int a = 0; a < n_arms; ++a)
    if (N[a] == 0.0) { *arm = a; return; }
  double tot = 0.0;
  for (int a = 0; a < n_arms; ++a) tot = tot + N[a];
  const double ln_tot = tot > 1.0 ? ucb_ln(tot) : 0.0;
  int best = 0;
  double bv = 0.0;
  for (int a = 0; a < n_arms; ++a) {
    const double v = R[a] / N[a] + ucb_sqrt(2.0 * ln_tot / N[a]);
    if (a == 0 || v > bv) { bv = v; best = a; }
  }
  *arm = best;
}

__global__ void k_ucb_update(int n_arms, double* R, double* N, const int32_t* __restrict__ arm,
                             const double* __restrict__ reward, double gamma) {
#pragma clang fp contract(off)
  const int a = threadIdx.x;
  if (a >= n_arms) return;
  double r = gamma * R[a], c = gamma * N[a];
  if (a == *arm) {
    r = r + *reward;
    c = c + 1.0;
  }
  R[a] = r;
  N[a] = c;
}

// ---------------------------------------------------------------- launchers

size_t dcrex_ws_bytes(int n_nodes, int ns, int np, int p_len) {
  (void)ns;
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  return al(4ull * n_nodes) * 3 + al(16ull * n_nodes * kOccMax) + al(4) + al(8ull * (p_len + np)) +
         al(16ull * (size_t)(p_len > 0 ? p_len : 1)) + al(4ull * n_nodes);
}

void launch_dcrex_counts(hipStream_t s, int n_nodes, int n_depots, int ns, int s_len, const int32_t* s_nodes,
                         const int32_t* s_offs, const int32_t* s_start, const int32_t* s_end, const int32_t* s_intro,
                         int np, int p_len, const int32_t* p_nodes, const int32_t* p_offs, const int32_t* p_start,
                         const int32_t* p_end, int32_t* EI, int32_t* NR, int32_t* NM, int32_t* NC, void* ws,
                         int32_t** err_out) {
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  char* w = (char*)ws;
  OccTab T;
  T.n = (int32_t*)w; w += al(4ull * n_nodes);
  T.n_in = (int32_t*)w; w += al(4ull * n_nodes);
  T.r_in = (int32_t*)w; w += al(4ull * n_nodes);
  T.occ = (int4*)w; w += al(16ull * n_nodes * kOccMax);
  T.err = (int32_t*)w; w += al(4);
  ParentInfo P;
  P.arc = (int2*)w; w += al(8ull * (p_len + np));
  P.node = (int4*)w; w += al(16ull * (size_t)(p_len > 0 ? p_len : 1));
  P.route_of = (int32_t*)w;
  const int b = 256;
  hipLaunchKernelGGL(k_fill_i32, dim3((n_nodes + b - 1) / b), dim3(b), 0, s, T.n, n_nodes, 0);
  hipLaunchKernelGGL(k_fill_i32, dim3((n_nodes + b - 1) / b), dim3(b), 0, s, T.n_in, n_nodes, 0);
  hipLaunchKernelGGL(k_fill_i32, dim3((n_nodes + b - 1) / b), dim3(b), 0, s, T.r_in, n_nodes, -1);
  hipLaunchKernelGGL(k_fill_i32, dim3((n_nodes + b - 1) / b), dim3(b), 0, s, P.route_of, n_nodes, -1);
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(1), 0, s, T.err, 1, 0);
  if (s_len > 0)
    hipLaunchKernelGGL(k_dcrex_occ, dim3((s_len + b - 1) / b), dim3(b), 0, s, ns, s_len, s_nodes, s_offs, s_start,
                       s_end, s_intro, T);
  if (np > 0)
    hipLaunchKernelGGL(k_dcrex_parent, dim3((p_len + np + b - 1) / b), dim3(b), 0, s, np, p_len, n_depots, p_nodes,
                       p_offs, p_start, p_end, T, P);
  const int64_t pairs = (int64_t)ns * np;
  if (pairs > 0)
    hipLaunchKernelGGL(k_dcrex_pairs, dim3((unsigned)((pairs + b - 1) / b)), dim3(b), 0, s, ns, np, s_nodes, s_offs,
                       p_offs, T, P, EI, NR, NM, NC);
  *err_out = T.err;
}

void launch_dcrex_pick(hipStream_t s, int ns, int np, const int32_t* EI, const int32_t* NR, const int32_t* NM,
                       const int32_t* NC, uint64_t seed, int32_t* out) {
  hipLaunchKernelGGL(k_dcrex_pick, dim3(1), dim3(kDcrexBlock), 0, s, ns, np, EI, NR, NM, NC, seed, out);
}

void launch_ucb_select(hipStream_t s, int n_arms, const double* R, const double* N, int32_t* arm) {
  hipLaunchKernelGGL(k_ucb_select, dim3(1), dim3(64), 0, s, n_arms, R, N, arm);
}

void launch_ucb_update(hipStream_t s, int n_arms, double* R, double* N, const int32_t* arm, const double* reward,
                       double gamma) {
  hipLaunchKernelGGL(k_ucb_update, dim3(1), dim3(((n_arms + 63) / 64) * 64), 0, s, n_arms, R, N, arm, reward, gamma);
}

}  // namespace mdvrp
