// prep.hip -- instance preprocessing (once per instance).
//
// * Matrix statistics: max/min c over u != v (Theta = 2 max c - min c, the
//   normaliser of Eq. A.1 used as the depot weight), sums of c and t (Gamma =
//   sum c / sum t, Eq. 3), symmetry and sign checks.
// * Granular lists (Section 3.2.3): arcs u -> v with e_u + s_u + t_uv > l_v
//   are pruned (time windows only), the theta customers with the smallest
//   eta_uv = c_uv + Gamma*(alpha*max(e_v - l_u - s_u - t_uv, 0) +
//   beta*max(l_u + s_u + t_uv - l_v, 0)), alpha = 1, beta = 10, are kept,
//   compared exactly as eta*den with Gamma = num/den; ties go to the lower id.
//   One 256-thread block per customer streams the row in chunks of 256 and
//   merges each chunk into a running sorted list with an LDS bitonic sort.
#include <algorithm>

#include "kernels.h"

namespace mdvrp {

constexpr int kStatsBlock = 256;
// partial layout per block: max c, min c, sum c, sum t, asym flag, negative flag, max t, max s (unused)
constexpr int kStatsFields = 8;

__global__ __launch_bounds__(kStatsBlock) void k_inst_stats(const int32_t* __restrict__ c,
                                                           const int32_t* __restrict__ t, int n,
                                                           int64_t* __restrict__ partial) {
  const int64_t total = (int64_t)n * n;
  int64_t mx = INT64_MIN, mn = INT64_MAX, sc = 0, st = 0, asym = 0, neg = 0, mt = INT64_MIN;
  for (int64_t i = (int64_t)blockIdx.x * kStatsBlock + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * kStatsBlock) {
    const int a = (int)(i / n), b = (int)(i - (int64_t)a * n);
    if (a == b) continue;
    const int64_t cv = c[i], tv = t[i];
    mx = cv > mx ? cv : mx;
    mn = cv < mn ? cv : mn;
    mt = tv > mt ? tv : mt;
    sc += cv;
    st += tv;
    if (cv < 0 || tv < 0) neg = 1;
    if (a < b) {
      const int64_t j = (int64_t)b * n + a;
      if (c[j] != cv || t[j] != tv) asym = 1;
    }
  }
  __shared__ int64_t sh[kStatsFields][kStatsBlock / 64];
  const int lane = __lane_id(), w = threadIdx.x >> 6;
  for (int off = 32; off > 0; off >>= 1) {
    const int64_t mx2 = __shfl_xor(mx, off), mn2 = __shfl_xor(mn, off), mt2 = __shfl_xor(mt, off);
    mx = mx2 > mx ? mx2 : mx;
    mn = mn2 < mn ? mn2 : mn;
    mt = mt2 > mt ? mt2 : mt;
    sc += __shfl_xor(sc, off);
    st += __shfl_xor(st, off);
    asym |= __shfl_xor(asym, off);
    neg |= __shfl_xor(neg, off);
  }
  if (lane == 0) {
    sh[0][w] = mx; sh[1][w] = mn; sh[2][w] = sc; sh[3][w] = st; sh[4][w] = asym; sh[5][w] = neg; sh[6][w] = mt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < kStatsBlock / 64; ++k) {
      sh[0][0] = sh[0][k] > sh[0][0] ? sh[0][k] : sh[0][0];
      sh[1][0] = sh[1][k] < sh[1][0] ? sh[1][k] : sh[1][0];
      sh[2][0] += sh[2][k];
      sh[3][0] += sh[3][k];
      sh[4][0] |= sh[4][k];
      sh[5][0] |= sh[5][k];
      sh[6][0] = sh[6][k] > sh[6][0] ? sh[6][k] : sh[6][0];
    }
    for (int f = 0; f < 7; ++f) partial[(int64_t)blockIdx.x * kStatsFields + f] = sh[f][0];
    partial[(int64_t)blockIdx.x * kStatsFields + 7] = 0;
  }
}

__global__ void k_inst_stats_final(const int64_t* __restrict__ partial, int nblocks, int64_t* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int64_t r[kStatsFields] = {INT64_MIN, INT64_MAX, 0, 0, 0, 0, INT64_MIN, 0};
  for (int b = 0; b < nblocks; ++b) {
    const int64_t* p = partial + (int64_t)b * kStatsFields;
    r[0] = p[0] > r[0] ? p[0] : r[0];
    r[1] = p[1] < r[1] ? p[1] : r[1];
    r[2] += p[2];
    r[3] += p[3];
    r[4] |= p[4];
    r[5] |= p[5];
    r[6] = p[6] > r[6] ? p[6] : r[6];
  }
  for (int f = 0; f < kStatsFields; ++f) out[f] = r[f];
}

int inst_stats_blocks(int n) {
  const int64_t total = (int64_t)n * n;
  int64_t b = (total + kStatsBlock * 16 - 1) / (kStatsBlock * 16);
  if (b < 1) b = 1;
  if (b > 4096) b = 4096;
  return (int)b;
}

void launch_inst_stats(hipStream_t s, const int32_t* c, const int32_t* t, int n, int64_t* partial, int nblocks) {
  hipLaunchKernelGGL(k_inst_stats, dim3(nblocks), dim3(kStatsBlock), 0, s, c, t, n, partial);
}

void launch_inst_stats_final(hipStream_t s, const int64_t* partial, int nblocks, int64_t* out) {
  hipLaunchKernelGGL(k_inst_stats_final, dim3(1), dim3(64), 0, s, partial, nblocks, out);
}

// ---------------------------------------------------------------------------- granular lists

constexpr int kNbrBlock = 256;
constexpr int kNbrKeep = 128;                    // maximum theta
constexpr int kNbrSort = 512;                    // kept list + one chunk, padded to a power of two

__device__ __forceinline__ bool pair_less(int64_t ka, int va, int64_t kb, int vb) {
  return ka < kb || (ka == kb && va < vb);
}

__global__ __launch_bounds__(kNbrBlock) void k_nbr_lists(const int32_t* __restrict__ c, const int32_t* __restrict__ t,
                                                        const int32_t* __restrict__ sv, const int32_t* __restrict__ ev,
                                                        const int32_t* __restrict__ lv, int nd, int nc, int theta,
                                                        int has_tw, int64_t gnum, int64_t gden,
                                                        int32_t* __restrict__ nbr, int32_t* __restrict__ nbr_len) {
  __shared__ int64_t key[kNbrSort];
  __shared__ int32_t vid[kNbrSort];
  const int i = blockIdx.x;
  const int n = nd + nc;
  const int u = nd + i;
  const int tid = threadIdx.x;
  for (int k = tid; k < kNbrSort; k += kNbrBlock) { key[k] = INT64_MAX; vid[k] = INT32_MAX; }
  __syncthreads();
  const int64_t eu = ev[u], lu = lv[u], su = sv[u];
  for (int base = 0; base < nc; base += kNbrBlock) {
    const int j = base + tid;
    int64_t kk = INT64_MAX;
    int vv = INT32_MAX;
    if (j < nc) {
      const int v = nd + j;
      if (v != u) {
        const int64_t cuv = c[(int64_t)u * n + v];
        if (has_tw) {
          const int64_t tuv = t[(int64_t)u * n + v];
          const int64_t evv = ev[v], lvv = lv[v];
          if (!(eu + su + tuv > lvv)) {
            const int64_t early = evv - lu - su - tuv > 0 ? evv - lu - su - tuv : 0;
            const int64_t late = lu + su + tuv - lvv > 0 ? lu + su + tuv - lvv : 0;
            kk = cuv * gden + gnum * (early + 10 * late);
            vv = v;
          }
        } else {
          kk = cuv;
          vv = v;
        }
      }
    }
    // skip the chunk when nothing beats the current theta-th entry
    const int64_t thk = key[theta - 1];
    const int thv = vid[theta - 1];
    const bool better = vv != INT32_MAX && pair_less(kk, vv, thk, thv);
    if (!__syncthreads_or(better)) continue;
    key[kNbrKeep + tid] = kk;
    vid[kNbrKeep + tid] = vv;
    for (int k = kNbrKeep + kNbrBlock + tid; k < kNbrSort; k += kNbrBlock) { key[k] = INT64_MAX; vid[k] = INT32_MAX; }
    for (int k = theta + tid; k < kNbrKeep; k += kNbrBlock) { key[k] = INT64_MAX; vid[k] = INT32_MAX; }
    __syncthreads();
    // bitonic sort of kNbrSort entries, two per thread per stage
    for (int size = 2; size <= kNbrSort; size <<= 1) {
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int x = tid; x < kNbrSort / 2; x += kNbrBlock) {
          const int lo = 2 * x - (x & (stride - 1));
          const int hi = lo + stride;
          const bool up = ((lo & size) == 0);
          const int64_t ka = key[lo], kb = key[hi];
          const int va = vid[lo], vb = vid[hi];
          const bool sw = up ? pair_less(kb, vb, ka, va) : pair_less(ka, va, kb, vb);
          if (sw) { key[lo] = kb; key[hi] = ka; vid[lo] = vb; vid[hi] = va; }
        }
        __syncthreads();
      }
    }
  }
  for (int k = tid; k < theta; k += kNbrBlock) nbr[(int64_t)i * theta + k] = vid[k] == INT32_MAX ? -1 : vid[k];
  if (tid == 0) {
    int cnt = 0;
    for (int k = 0; k < theta; ++k) cnt += vid[k] != INT32_MAX;
    nbr_len[i] = cnt;
  }
}

__global__ void k_node_attr(const int32_t* __restrict__ q, const int32_t* __restrict__ sv,
                            const int32_t* __restrict__ e, const int32_t* __restrict__ l, int n, int4* __restrict__ attr) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x < n) attr[x] = make_int4(q[x], sv[x], e[x], l[x]);
}

void launch_node_attr(hipStream_t s, const int32_t* q, const int32_t* sv, const int32_t* e, const int32_t* l, int n,
                      int4* attr) {
  hipLaunchKernelGGL(k_node_attr, dim3((n + 255) / 256), dim3(256), 0, s, q, sv, e, l, n, attr);
}

// Depot-arc table: out[(x - nd) * nd + d] = {c(d,x), t(d,x), c(x,d), t(x,d)} for every
// customer x and depot d (original node ids); one thread per entry, d fastest.
__global__ void k_depot_arcs(const int32_t* __restrict__ c, const int32_t* __restrict__ t, int nd, int nc,
                             int4* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nc * nd) return;
  const int64_t n = (int64_t)nd + nc;
  const int x = nd + (int)(i / nd), d = (int)(i % nd);
  out[i] = make_int4(c[d * n + x], t[d * n + x], c[x * n + d], t[x * n + d]);
}

void launch_depot_arcs(hipStream_t s, const int32_t* c, const int32_t* t, int nd, int nc, int4* out) {
  const int64_t m = (int64_t)nc * nd;
  if (m <= 0) return;
  hipLaunchKernelGGL(k_depot_arcs, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, c, t, nd, nc, out);
}

// {c(u, v), t(u, v)} of every list slot, kept beside the lists so that the evaluation
// reads the arc u -> v with the list entry instead of gathering it from the matrices
// (0 past the end of a list).
__global__ void k_nbr_arcs(const int32_t* __restrict__ c, const int32_t* __restrict__ t,
                           const int32_t* __restrict__ nbr, const int32_t* __restrict__ nbr_len, int nd, int nc,
                           int theta, int2* __restrict__ out) {
  const int64_t item = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= (int64_t)nc * theta) return;
  const int i = (int)(item / theta), k = (int)(item - (int64_t)i * theta);
  const int64_t n = (int64_t)nd + nc;
  int2 r = make_int2(0, 0);
  if (k < nbr_len[i]) {
    const int64_t a = (int64_t)(nd + i) * n + nbr[item];
    r = make_int2(c[a], t[a]);
  }
  out[item] = r;
}

void launch_nbr_arcs(hipStream_t s, const int32_t* c, const int32_t* t, const int32_t* nbr, const int32_t* nbr_len,
                     int nd, int nc, int theta, int2* out) {
  const int64_t items = (int64_t)nc * theta;
  hipLaunchKernelGGL(k_nbr_arcs, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, s, c, t, nbr, nbr_len, nd, nc,
                     theta, out);
}

void launch_nbr_lists(hipStream_t s, const int32_t* c, const int32_t* t, const int32_t* sv, const int32_t* ev,
                      const int32_t* lv, int nd, int nc, int theta, int has_tw, int64_t gnum, int64_t gden,
                      int32_t* nbr, int32_t* nbr_len) {
  hipLaunchKernelGGL(k_nbr_lists, dim3(nc), dim3(kNbrBlock), 0, s, c, t, sv, ev, lv, nd, nc, theta, has_tw, gnum,
                     gden, nbr, nbr_len);
}

}  // namespace mdvrp

namespace mdvrp {

// out[0] = sum over customers with a non-empty list of c(u, first list entry), out[1] = their count.
__global__ __launch_bounds__(1024) void k_nn_sum(const int32_t* __restrict__ c, const int32_t* __restrict__ nbr,
                                                 const int32_t* __restrict__ nbr_len, int nd, int nc, int theta,
                                                 int64_t* __restrict__ out) {
  __shared__ unsigned long long s_sum, s_cnt;
  if (threadIdx.x == 0) { s_sum = 0; s_cnt = 0; }
  __syncthreads();
  const int64_t n = (int64_t)nd + nc;
  unsigned long long sum = 0, cnt = 0;
  for (int i = threadIdx.x; i < nc; i += blockDim.x) {
    if (nbr_len[i] > 0) {
      sum += (unsigned long long)c[(int64_t)(nd + i) * n + nbr[(int64_t)i * theta]];
      cnt += 1;
    }
  }
  atomicAdd(&s_sum, sum);
  atomicAdd(&s_cnt, cnt);
  __syncthreads();
  if (threadIdx.x == 0) {
    out[0] = (int64_t)s_sum;
    out[1] = (int64_t)s_cnt;
  }
}

void launch_nn_sum(hipStream_t s, const int32_t* c, const int32_t* nbr, const int32_t* nbr_len, int nd, int nc,
                   int theta, int64_t* out) {
  hipLaunchKernelGGL(k_nn_sum, dim3(1), dim3(1024), 0, s, c, nbr, nbr_len, nd, nc, theta, out);
}

}  // namespace mdvrp

namespace mdvrp {

// ---------------------------------------------------------------------------- locality layout
//
// Evaluations read c(x, y) for nodes x, y that are close to each other (a customer, its
// route neighbours and its granular list). In the caller's numbering such reads land
// on unrelated cache lines of a large matrix. A copy of c (and t) in an order that
// keeps nearby nodes at nearby indices turns them into reads of a narrow band, shared
// by the anchors of one tile. The order is derived from c alone: three far-apart
// landmarks give each node three distances, whose interleaved (Morton) code is sorted.

constexpr int kLayoutBlock = 1024;

// argmax over x of f(x), ties to the lower x; one block.
template <class F>
__device__ int block_argmax(int n, F f, int64_t* best_val) {
  __shared__ int64_t sv[kLayoutBlock / 64];
  __shared__ int si[kLayoutBlock / 64];
  int64_t bv = -1;
  int bi = INT32_MAX;
  for (int x = threadIdx.x; x < n; x += kLayoutBlock) {
    const int64_t v = f(x);
    if (v > bv || (v == bv && x < bi)) { bv = v; bi = x; }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const int64_t v2 = __shfl_xor(bv, off);
    const int i2 = __shfl_xor(bi, off);
    if (v2 > bv || (v2 == bv && i2 < bi)) { bv = v2; bi = i2; }
  }
  __syncthreads();
  if (lane_id() == 0) { sv[threadIdx.x >> 6] = bv; si[threadIdx.x >> 6] = bi; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kLayoutBlock / 64; ++w)
      if (sv[w] > sv[0] || (sv[w] == sv[0] && si[w] < si[0])) { sv[0] = sv[w]; si[0] = si[w]; }
  }
  __syncthreads();
  if (best_val) *best_val = sv[0];
  return si[0];
}

// out: landmarks A, B, C and the largest distance from each.
__global__ __launch_bounds__(kLayoutBlock) void k_landmarks(const int32_t* __restrict__ c, int n, int64_t* out) {
  const int64_t N = n;
  int64_t mA, mB, mC;
  const int A = block_argmax(n, [&](int x) -> int64_t { return c[x]; }, nullptr);  // farthest from node 0
  const int B = block_argmax(n, [&](int x) -> int64_t { return c[A * N + x]; }, &mA);
  const int C = block_argmax(
      n, [&](int x) -> int64_t { return imin(c[A * N + x], c[B * N + x]); }, nullptr);
  block_argmax(n, [&](int x) -> int64_t { return c[B * N + x]; }, &mB);
  block_argmax(n, [&](int x) -> int64_t { return c[C * N + x]; }, &mC);
  if (threadIdx.x == 0) {
    out[0] = A; out[1] = B; out[2] = C;
    out[3] = mA > 0 ? mA : 1; out[4] = mB > 0 ? mB : 1; out[5] = mC > 0 ? mC : 1;
  }
}

__device__ __forceinline__ uint32_t spread3(uint32_t v) {  // 10 bits -> every third bit
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000ffu;
  v = (v | (v << 8)) & 0x0300f00fu;
  v = (v | (v << 4)) & 0x030c30c3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

// key[x] = Morton code of the node's three landmark distances (10 bits each) << 16 | x.
__global__ void k_layout_keys(const int32_t* __restrict__ c, int n, const int64_t* __restrict__ lm,
                              uint64_t* __restrict__ key) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  const int64_t N = n;
  uint32_t q[3];
  for (int j = 0; j < 3; ++j) q[j] = (uint32_t)((int64_t)c[lm[j] * N + x] * 1023 / lm[3 + j]);
  const uint32_t m = spread3(q[0]) | (spread3(q[1]) << 1) | (spread3(q[2]) << 2);
  key[x] = ((uint64_t)m << 16) | (uint32_t)x;
}

// pi[x] = rank of key[x] (keys are distinct); inv[pi[x]] = x.
__global__ __launch_bounds__(256) void k_layout_rank(const uint64_t* __restrict__ key, int n, int32_t* __restrict__ pi,
                                                     int32_t* __restrict__ inv) {
  __shared__ uint64_t sk[256];
  const int x = blockIdx.x * 256 + threadIdx.x;
  const uint64_t kx = x < n ? key[x] : ~0ull;
  int rank = 0;
  for (int base = 0; base < n; base += 256) {
    __syncthreads();
    sk[threadIdx.x] = base + threadIdx.x < n ? key[base + threadIdx.x] : ~0ull;
    __syncthreads();
    const int m = imin(256, n - base);
    for (int j = 0; j < m; ++j) rank += sk[j] < kx;
  }
  if (x < n) {
    pi[x] = rank;
    inv[rank] = x;
  }
}

// dst[r][s] = src[inv[r]][inv[s]]: rows written contiguously.
__global__ void k_layout_permute(const int32_t* __restrict__ src, int n, const int32_t* __restrict__ inv,
                                 int32_t* __restrict__ dst) {
  const int r = blockIdx.y;
  const int64_t N = n;
  const int32_t* row = src + inv[r] * N;
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += gridDim.x * blockDim.x) dst[r * N + s] = row[inv[s]];
}

// corder[k] = customer index (node - nd) of the k-th customer in layout order. One block.
__global__ __launch_bounds__(kLayoutBlock) void k_layout_customers(const int32_t* __restrict__ inv, int n, int nd,
                                                                   int32_t* __restrict__ corder) {
  __shared__ int sh[2 * (kLayoutBlock / 64) + 1];
  int carry = 0;
  for (int base = 0; base < n; base += kLayoutBlock) {
    const int r = base + threadIdx.x;
    const int x = r < n ? inv[r] : -1;
    const int is_c = x >= nd ? 1 : 0;
    int tot;
    const int ex = block_scan_excl<kLayoutBlock>(is_c, sh, &tot);
    if (is_c) corder[carry + ex] = x - nd;
    carry += tot;
  }
}

void launch_layout(hipStream_t s, const int32_t* c, const int32_t* t, int n, int nd, int64_t* lm, uint64_t* keys,
                   int32_t* pi, int32_t* inv, int32_t* corder, int32_t* cl, int32_t* tl) {
  hipLaunchKernelGGL(k_landmarks, dim3(1), dim3(kLayoutBlock), 0, s, c, n, lm);
  hipLaunchKernelGGL(k_layout_keys, dim3((n + 255) / 256), dim3(256), 0, s, c, n, (const int64_t*)lm, keys);
  hipLaunchKernelGGL(k_layout_rank, dim3((n + 255) / 256), dim3(256), 0, s, (const uint64_t*)keys, n, pi, inv);
  const dim3 grid((unsigned)std::min(8, (n + 255) / 256), (unsigned)n);
  hipLaunchKernelGGL(k_layout_permute, grid, dim3(256), 0, s, c, n, (const int32_t*)inv, cl);
  if (tl) hipLaunchKernelGGL(k_layout_permute, grid, dim3(256), 0, s, t, n, (const int32_t*)inv, tl);
  hipLaunchKernelGGL(k_layout_customers, dim3(1), dim3(kLayoutBlock), 0, s, (const int32_t*)inv, n, nd, corder);
}

}  // namespace mdvrp
