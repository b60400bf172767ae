// pop.hip -- population measures of Section 3.4 on the device: the distance
// between solutions (Eq. 7), the population distance (Eq. 6), the fitness-and-
// distance score chi (Eq. 5) and the reduction of a population to mu solutions.
//
// A solution's edge set is the set of directed arcs along its routes. Every
// customer x has at most one outgoing arc (to its successor, or to the arrival
// depot; none when it ends an open route), and every route has one arc out of
// its departure depot, into its first customer. So E is fully described per
// customer by two keys, {successor, departure depot if x is first else -1}, and
// |E_a & E_b| is the number of equal keys over the customers: one coalesced pass
// over two key arrays per pair of solutions.
#include "kernels.h"

namespace mdvrp {

constexpr int kPopBlock = 256;
constexpr int kReduceBlock = kPopMaxMembers;

__global__ void k_zero_i64(int64_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Keys of member i (unit list[i]) for every customer: keys[i * nc + (x - nd)].
template <class SEG, bool OPEN>
__global__ __launch_bounds__(kPopBlock) void k_arc_keys(const UnitDesc* __restrict__ units,
                                                       const int32_t* __restrict__ list, int nc, int2* keys,
                                                       int64_t* n_edges) {
  const int i = blockIdx.y;
  const UnitDesc& U = units[list[i]];
  const int cur = U.ctl->cur;
  const SEG* fw = (const SEG*)U.fw[cur];
  int cnt = 0;
  for (int k = blockIdx.x * kPopBlock + threadIdx.x; k < nc; k += gridDim.x * kPopBlock) {
    const int x = U.nd + k;
    const int slot = U.rt[x], p = U.pos[x];
    const int L = U.r_len[slot];
    int succ;
    if (p < L) succ = fw[U.apos[x] + 1].node;
    else succ = OPEN ? -1 : U.r_end[slot];
    const int head = p == 1 ? U.r_start[slot] : -1;
    keys[(int64_t)i * nc + k] = make_int2(succ, head);
    cnt += (succ >= 0) + (head >= 0);
  }
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
  if ((threadIdx.x & 63) == 0 && cnt) atomicAdd((unsigned long long*)&n_edges[i], (unsigned long long)cnt);
}

// One block per pair (i <= j) of members: common arcs, then Eq. 7.
__global__ __launch_bounds__(kPopBlock) void k_pair_distance(const int2* __restrict__ keys, int nc, int n,
                                                            const int64_t* __restrict__ n_edges, double* dist,
                                                            int64_t* common) {
#pragma clang fp contract(off)
  // pair index -> (i, j), i <= j, row-major over the upper triangle
  int b = blockIdx.x, i = 0;
  while (b >= n - i) { b -= n - i; ++i; }
  const int j = i + b;
  const int2* ki = keys + (int64_t)i * nc;
  const int2* kj = keys + (int64_t)j * nc;
  int cnt = 0;
  for (int k = threadIdx.x; k < nc; k += kPopBlock) {
    const int2 a = ki[k], c = kj[k];
    cnt += (a.x >= 0 && a.x == c.x) + (a.y >= 0 && a.y == c.y);
  }
  __shared__ int part[kPopBlock / 64];
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t c = 0;
    for (int w = 0; w < kPopBlock / 64; ++w) c += part[w];
    const int64_t m = n_edges[i] > n_edges[j] ? n_edges[i] : n_edges[j];
    // Eq. 7: the quotient, the difference and the product, each rounded once
    const double d = m > 0 ? 100.0 * (1.0 - (double)c / (double)m) : 0.0;
    dist[(int64_t)i * n + j] = d;
    dist[(int64_t)j * n + i] = d;
    if (common) {
      common[(int64_t)i * n + j] = c;
      common[(int64_t)j * n + i] = c;
    }
  }
}

// The reduction of a population of n members to mu (one block; n <= kReduceBlock): while
// more than mu remain, chi of Eq. 5 over the remaining members (population distance of
// Eq. 6 over the n_close nearest others), and the member of lowest chi leaves (ties: the
// higher index). Ranks count from 1; Rank_f orders objectives ascending, Rank_D population
// distances descending, ties in either by lower index.
__global__ __launch_bounds__(kReduceBlock) void k_pop_reduce(const double* __restrict__ dist,
                                                            const int64_t* __restrict__ f, int n, int mu, double xi,
                                                            int n_close, int32_t* keep, int32_t* order,
                                                            double* chi_out, double* dpop_out) {
  // every operation below rounds on its own (no fused multiply-add), as Eq. 5 and Eq. 6 are
  // evaluated everywhere they are compared
#pragma clang fp contract(off)
  __shared__ int alive[kReduceBlock];
  __shared__ double dpop[kReduceBlock];
  __shared__ double wchi[kReduceBlock / 64];
  __shared__ int widx[kReduceBlock / 64];
  __shared__ int s_m;
  const int i = threadIdx.x;
  const bool mine = i < n;
  if (mine) alive[i] = 1;
  if (i == 0) s_m = n;
  int64_t fi = mine ? f[i] : 0;
  __syncthreads();
  for (int round = 0;; ++round) {
    const int m = s_m;
    // Eq. 6: mean of the n_close smallest distances to the other remaining members,
    // summed in ascending order (ties: lower index first)
    double d_i = 0.0;
    if (mine && alive[i]) {
      double near[kPopMaxClose];
      int cnt = 0;
      for (int j = 0; j < n; ++j) {
        if (j == i || !alive[j]) continue;
        const double v = dist[(int64_t)i * n + j];
        if (cnt < n_close) {
          int p = cnt++;
          while (p > 0 && near[p - 1] > v) { near[p] = near[p - 1]; --p; }
          near[p] = v;
        } else if (v < near[n_close - 1]) {
          int p = n_close - 1;
          while (p > 0 && near[p - 1] > v) { near[p] = near[p - 1]; --p; }
          near[p] = v;
        }
      }
      double s = 0.0;
      for (int z = 0; z < cnt; ++z) s += near[z];
      d_i = cnt > 0 ? s / (double)cnt : 0.0;
      dpop[i] = d_i;
    }
    __syncthreads();
    double chi = 0.0;
    if (mine && alive[i]) {
      int rf = 1, rd = 1;
      for (int j = 0; j < n; ++j) {
        if (j == i || !alive[j]) continue;
        const int64_t fj = f[j];
        if (fj < fi || (fj == fi && j < i)) ++rf;
        const double dj = dpop[j];
        if (dj > d_i || (dj == d_i && j < i)) ++rd;
      }
      // Eq. 5
      const double a = (double)(m - rf) / (double)m;
      const double b = (double)(m - rd) / (double)m;
      chi = a + xi * b;
      if (round == 0) {
        if (chi_out) chi_out[i] = chi;
        if (dpop_out) dpop_out[i] = d_i;
      }
    }
    if (m <= mu) break;
    // lowest chi, ties to the higher index
    int idx = (mine && alive[i]) ? i : -1;
    double c = idx >= 0 ? chi : 0.0;
    for (int o = 32; o > 0; o >>= 1) {
      const double c2 = __shfl_xor(c, o);
      const int i2 = __shfl_xor(idx, o);
      if (i2 >= 0 && (idx < 0 || c2 < c || (c2 == c && i2 > idx))) { c = c2; idx = i2; }
    }
    if ((i & 63) == 0) { wchi[i >> 6] = c; widx[i >> 6] = idx; }
    __syncthreads();
    if (i == 0) {
      int w = -1;
      double wc = 0.0;
      for (int k = 0; k < kReduceBlock / 64; ++k) {
        const int ik = widx[k];
        if (ik >= 0 && (w < 0 || wchi[k] < wc || (wchi[k] == wc && ik > w))) { w = ik; wc = wchi[k]; }
      }
      alive[w] = 0;
      if (order) order[round] = w;
      s_m = m - 1;
    }
    __syncthreads();
  }
  if (mine) keep[i] = alive[i];
}

int pop_keys_blocks(int nc) { return (nc + kPopBlock - 1) / kPopBlock; }

void launch_pop_distance(const LaunchCtx& L, const int32_t* list, int n, int nc, int2* keys, int64_t* n_edges,
                         double* dist, int64_t* common) {
  const dim3 g(pop_keys_blocks(nc), n);
  hipLaunchKernelGGL(k_zero_i64, dim3((n + 255) / 256), dim3(256), 0, L.stream, n_edges, n);
  if (L.has_tw) {
    if (L.open) hipLaunchKernelGGL((k_arc_keys<SegTW, true>), g, dim3(kPopBlock), 0, L.stream, L.units, list, nc, keys, n_edges);
    else hipLaunchKernelGGL((k_arc_keys<SegTW, false>), g, dim3(kPopBlock), 0, L.stream, L.units, list, nc, keys, n_edges);
  } else {
    if (L.open) hipLaunchKernelGGL((k_arc_keys<SegNT, true>), g, dim3(kPopBlock), 0, L.stream, L.units, list, nc, keys, n_edges);
    else hipLaunchKernelGGL((k_arc_keys<SegNT, false>), g, dim3(kPopBlock), 0, L.stream, L.units, list, nc, keys, n_edges);
  }
  hipLaunchKernelGGL(k_pair_distance, dim3(n * (n + 1) / 2), dim3(kPopBlock), 0, L.stream, (const int2*)keys, nc, n,
                     (const int64_t*)n_edges, dist, common);
}

void launch_pop_reduce(hipStream_t s, const double* dist, const int64_t* f, int n, int mu, double xi, int n_close,
                       int32_t* keep, int32_t* order, double* chi, double* dpop) {
  hipLaunchKernelGGL(k_pop_reduce, dim3(1), dim3(kReduceBlock), 0, s, dist, f, n, mu, xi, n_close, keep, order, chi,
                     dpop);
}

}  // namespace mdvrp
