// mlp.hip -- learned move filter: anchor features, the scoring network on the
// matrix cores, per-customer top-k, and the network's training kernels.
//
// The paper prunes the neighbourhood with granular lists only (Section 3.2.3);
// this filter ranks each customer's granular list with a small network and
// evaluates the k best entries exactly, falling back to the full lists when the
// filtered neighbourhood has no improving move left.
//
// Network: 32 bf16 features -> 256 -> 256 -> 1 with ReLU. Operands are bf16,
// accumulation fp32 (MFMA 16x16x32), hidden activations are rounded to bf16
// between layers. The forward runs transposed (h^T = W x^T): a layer's output
// fragment (lane: one sample, four consecutive features) is, after bias, ReLU
// and rounding, exactly the B operand of the next layer, so activations stay
// in registers. W2 (128 KB in bf16) sits in LDS in fragment order, one 16-byte
// read per lane per MFMA, each read shared by T sample tiles.
//
// Parameter layout (fp32 master copy): W1[256][32], b1[256], W2[256][256],
// b2[256], w3[256], b3.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "eval_common.h"
#include "kernels.h"

namespace mdvrp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kH = 256, kF = 32;
constexpr int P_W1 = 0, P_B1 = P_W1 + kH * kF, P_W2 = P_B1 + kH, P_B2 = P_W2 + kH * kH, P_W3 = P_B2 + kH,
              P_B3 = P_W3 + kH, P_N = P_B3 + 1;

// fp32 -> bf16 bits, round to nearest even (quiet NaN kept).
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ __bf16 as_bf(uint16_t h) { return __builtin_bit_cast(__bf16, h); }

__device__ __forceinline__ f32x4 mfma(const bf16x8& a, const bf16x8& b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Orders this wave's LDS accesses (a lane reads what another lane wrote).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ uint4 pack8(const uint16_t* f) {
  uint4 w;
  w.x = (uint32_t)f[0] | ((uint32_t)f[1] << 16);
  w.y = (uint32_t)f[2] | ((uint32_t)f[3] << 16);
  w.z = (uint32_t)f[4] | ((uint32_t)f[5] << 16);
  w.w = (uint32_t)f[6] | ((uint32_t)f[7] << 16);
  return w;
}

// ---------------------------------------------------------------------------- weights in fragment order

// MFMA 16x16x32 operand layout: lane l holds A[l % 16][8 (l / 16) + e] and
// B[8 (l / 16) + e][l % 16], e = 0..7; the result D[4 (l / 16) + r][l % 16], r = 0..3.
// W1 fragment (ob, lane): W1[16 ob + lane % 16][8 (lane / 16) + e].
// W2 fragment (ob, j, lane): row 16 ob + lane % 16; columns 32 j + 4 (lane / 16) + e for
// e < 4 and 32 j + 16 + 4 (lane / 16) + e - 4 for e >= 4 -- the order in which layer 1's
// output fragments of blocks 2j and 2j+1 land in a lane.
// W2 backward fragment (nb, kb, lane): W2[32 kb + 8 (lane / 16) + e][16 nb + lane % 16], the
// B operand of the hidden-layer gradient (columns 16 nb .., inputs 32 kb ..).
__global__ void k_mlp_pack(const float* __restrict__ P, bf16x8* __restrict__ w1f, bf16x8* __restrict__ w2f,
                           bf16x8* __restrict__ w2b, float* __restrict__ w3b) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < 16 * 64) {
    const int ob = t / 64, lane = t % 64;
    bf16x8 v;
    for (int e = 0; e < 8; ++e) v[e] = as_bf(f2bf(P[P_W1 + (ob * 16 + lane % 16) * kF + 8 * (lane / 16) + e]));
    w1f[t] = v;
  }
  if (t < 16 * 8 * 64) {
    const int ob = t / 512, j = (t / 64) % 8, lane = t % 64;
    const int row = ob * 16 + lane % 16;
    bf16x8 v;
    for (int e = 0; e < 8; ++e) {
      const int col = e < 4 ? 32 * j + 4 * (lane / 16) + e : 32 * j + 16 + 4 * (lane / 16) + (e - 4);
      v[e] = as_bf(f2bf(P[P_W2 + row * kH + col]));
    }
    w2f[t] = v;
  }
  if (t < 16 * 8 * 64) {
    const int nb = t / 512, kb = (t / 64) % 8, lane = t % 64;
    bf16x8 v;
    for (int e = 0; e < 8; ++e) v[e] = as_bf(f2bf(P[P_W2 + (32 * kb + 8 * (lane / 16) + e) * kH + 16 * nb + lane % 16]));
    w2b[t] = v;
  }
  if (t < kH) w3b[t] = bf2f(f2bf(P[P_W3 + t]));
}

// ---------------------------------------------------------------------------- forward core

struct MlpSmem {
  bf16x8 w2f[16 * 8 * 64];  // 128 KB
  float b1[kH], b2[kH], w3[kH];
};

__device__ void mlp_stage(MlpSmem& S, const bf16x8* __restrict__ w2f, const float* __restrict__ P,
                          const float* __restrict__ w3b) {
  for (int t = threadIdx.x; t < 16 * 8 * 64; t += blockDim.x) S.w2f[t] = w2f[t];
  for (int t = threadIdx.x; t < kH; t += blockDim.x) {
    S.b1[t] = P[P_B1 + t];
    S.b2[t] = P[P_B2 + t];
    S.w3[t] = w3b[t];
  }
  __syncthreads();
}

// Writes four consecutive rounded activations of one sample (8-byte store).
__device__ __forceinline__ void put4(uint16_t* row, int f, const uint16_t h[4]) {
  uint2 w;
  w.x = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
  w.y = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
  *(uint2*)(row + f) = w;
}

// One wave, T tiles of 16 samples. xb[t] = this lane's B fragment of tile t (sample
// 16 t + lane % 16, features 8 (lane / 16) .. + 7). z[t] = logit of sample 16 t + lane % 16
// (the four lanes of a sample agree). With h1o / h2o the rounded activations of the
// 16 T samples are written row-major (256 bf16 per sample, row 16 t + lane % 16).
template <int T>
__device__ void mlp_tiles(const MlpSmem& S, const bf16x8* __restrict__ w1f, const bf16x8 (&xb)[T], float b3,
                          float (&z)[T], uint16_t* __restrict__ h1o, uint16_t* __restrict__ h2o) {
  const int lane = lane_id(), g = lane >> 4, col = lane & 15;
  bf16x8 hb[T][8];
#pragma unroll
  for (int ob = 0; ob < 16; ++ob) {
    const bf16x8 a = w1f[ob * 64 + lane];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      acc = mfma(a, xb[t], acc);
      uint16_t h[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float v = acc[r] + S.b1[ob * 16 + 4 * g + r];
        v = v > 0.f ? v : 0.f;
        h[r] = f2bf(v);
        hb[t][ob >> 1][(ob & 1) * 4 + r] = as_bf(h[r]);
      }
      if (h1o) put4(h1o + (16 * t + col) * kH, ob * 16 + 4 * g, h);
    }
  }
  float part[T];
#pragma unroll
  for (int t = 0; t < T; ++t) part[t] = 0.f;
#pragma unroll 1
  for (int ob = 0; ob < 16; ob += 2) {
    f32x4 acc[2][T];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int t = 0; t < T; ++t) acc[q][t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const bf16x8 a0 = S.w2f[(ob * 8 + j) * 64 + lane];
      const bf16x8 a1 = S.w2f[((ob + 1) * 8 + j) * 64 + lane];
#pragma unroll
      for (int t = 0; t < T; ++t) {
        acc[0][t] = mfma(a0, hb[t][j], acc[0][t]);
        acc[1][t] = mfma(a1, hb[t][j], acc[1][t]);
      }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int t = 0; t < T; ++t) {
        uint16_t h[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int f = (ob + q) * 16 + 4 * g + r;
          float v = acc[q][t][r] + S.b2[f];
          v = v > 0.f ? v : 0.f;
          h[r] = f2bf(v);
          part[t] += S.w3[f] * bf2f(h[r]);
        }
        if (h2o) put4(h2o + (16 * t + col) * kH, (ob + q) * 16 + 4 * g, h);
      }
  }
#pragma unroll
  for (int t = 0; t < T; ++t) {
    float p = part[t];
    p += __shfl_xor(p, 16);
    p += __shfl_xor(p, 32);
    z[t] = p + b3;
  }
}

// ---------------------------------------------------------------------------- features

// The 32 integer features of anchor (u, v), each scaled by one fp32 multiplication
// and rounded to bf16. Route facts come from the segment state of the current buffer.
template <class SEG, bool TW>
__device__ void pair_features(const UnitDesc& U, int cur, int u, int v, int rank, uint16_t (&out)[kF]) {
  const SEG* fw = (const SEG*)U.fw[cur];
  const int sa = U.rt[u], sb = U.rt[v];
  const int4 ma = U.r_meta[cur][sa], mb = U.r_meta[cur][sb];
  const int pu = U.pos[u], pv = U.pos[v];
  const int p_u = fw[ma.x + pu - 1].node;
  const int s_u = pu + 1 <= ma.y ? fw[ma.x + pu + 1].node : ma.w;  // ma.w = -1 for open routes
  const int p_v = fw[mb.x + pv - 1].node;
  const int pp_v = pv >= 2 ? fw[mb.x + pv - 2].node : p_v;
  const int c_uv = arc_c(U, u, v), c_pu_u = arc_c(U, p_u, u);
  const int c_u_su = s_u >= 0 ? arc_c(U, u, s_u) : 0;
  const int c_pu_su = s_u >= 0 ? arc_c(U, p_u, s_u) : 0;
  const int c_pv_v = arc_c(U, p_v, v), c_pv_u = arc_c(U, p_v, u);
  const int c_pv_su = s_u >= 0 ? arc_c(U, p_v, s_u) : 0;
  const int4 ta = U.r_tot[sa], tb = U.r_tot[sb];
  const int4 au = U.attr[u], av = U.attr[v];
  int iv[kF];
  iv[0] = c_uv;
  iv[1] = c_pu_u;
  iv[2] = c_u_su;
  iv[3] = c_pu_su;
  iv[4] = c_pv_v;
  iv[5] = c_pv_u;
  iv[6] = c_pu_su - c_pu_u - c_u_su + c_pv_u + c_uv - c_pv_v;  // relocate u before v
  iv[7] = c_uv + c_pv_su - c_u_su - c_pv_v;                     // 2-opt* joining u -> v
  iv[8] = arc_c(U, p_u, p_v) + c_pv_su + arc_c(U, pp_v, u) + c_uv - c_pu_u - c_u_su - arc_c(U, pp_v, p_v) -
          c_pv_v;                                               // swap u with p(v)
  iv[9] = ta.y - U.Q;
  iv[10] = tb.y - U.Q;
  iv[11] = au.x;
  iv[12] = av.x;
  iv[13] = U.Dmax >= 0 ? ta.z - U.Dmax : 0;
  iv[14] = U.Dmax >= 0 ? tb.z - U.Dmax : 0;
  iv[15] = TW ? ta.w : 0;
  iv[16] = TW ? tb.w : 0;
  if (TW) {
    const int tuv = arc_t(U, u, v);
    iv[17] = au.w - au.z;
    iv[18] = av.w - av.z;
    iv[19] = au.z;
    iv[20] = av.z;
    iv[21] = imax(av.z - au.z - au.y - tuv, 0);
    iv[22] = imax(au.z + au.y + tuv - av.w, 0);
  } else {
#pragma unroll
    for (int z = 17; z <= 22; ++z) iv[z] = 0;
  }
  iv[23] = sa == sb;
  iv[24] = ma.z == mb.z;
  iv[25] = ma.z;
  iv[26] = mb.z;
  iv[27] = ma.y;
  iv[28] = mb.y;
  iv[29] = pu;
  iv[30] = pv;
  iv[31] = rank;
  auto S = [](int x, float r) -> uint16_t { return f2bf(__fmul_rn((float)x, r)); };
#pragma unroll
  for (int z = 0; z <= 8; ++z) out[z] = S(iv[z], U.frcp[0]);
#pragma unroll
  for (int z = 9; z <= 12; ++z) out[z] = S(iv[z], U.frcp[1]);
#pragma unroll
  for (int z = 13; z <= 22; ++z) out[z] = S(iv[z], U.frcp[2]);
  out[23] = S(iv[23], 1.0f);
  out[24] = S(iv[24], 1.0f);
  out[25] = S(iv[25], U.frcp[3]);
  out[26] = S(iv[26], U.frcp[3]);
  out[27] = S(iv[27], 1.0f / 32.0f);
  out[28] = S(iv[28], 1.0f / 32.0f);
  out[29] = S(iv[29], __fdiv_rn(1.0f, (float)ma.y));
  out[30] = S(iv[30], __fdiv_rn(1.0f, (float)mb.y));
  out[31] = S(iv[31], __fdiv_rn(1.0f, (float)U.theta));
}

// Features of every anchor of every unit: out[(item_base + i * theta + k) * 32 + f];
// rows of missing list entries are zero.
template <class SEG, bool TW>
__global__ __launch_bounds__(256) void k_features(const UnitDesc* __restrict__ units,
                                                  const int32_t* __restrict__ tile_off, int n_units,
                                                  uint16_t* __restrict__ out) {
  const int tile = blockIdx.x;
  const int ui = unit_of_tile(tile_off, n_units, tile);
  const UnitDesc& U = units[ui];
  const int item = (tile - tile_off[ui]) * 256 + threadIdx.x;
  if (item >= U.nc * U.theta) return;
  uint16_t f[kF];
  const int i = item / U.theta, k = item - i * U.theta;
  const int v = U.nbr[item];
  if (k < U.nbr_len[i] && v >= 0) {
    pair_features<SEG, TW>(U, U.ctl->cur, U.nd + i, v, k, f);
  } else {
#pragma unroll
    for (int z = 0; z < kF; ++z) f[z] = 0;
  }
  uint4* o = (uint4*)(out + (U.item_base + item) * kF);
#pragma unroll
  for (int z = 0; z < 4; ++z) o[z] = pack8(f + 8 * z);
}

// ---------------------------------------------------------------------------- scoring + top-k
//
// Ranking is incremental at the level of anchors: every anchor's logit is cached
// (lcache[item_base + i * theta + k]); a ranking step recomputes only the anchors
// whose features may have changed -- the route of u or the route of v was rebuilt
// after the unit's last ranking (dirty tag above scored_epoch) -- and then redoes
// the top-k of the customers that own such an anchor from the cached logits.

constexpr int kScoreWaves = 8;
constexpr int kScoreT = 4;      // sample tiles per pass through W2 (one anchor per lane)
constexpr int kScoreStage = 2;  // tiles staged in LDS at a time

__global__ void k_queue_reset(int32_t* __restrict__ count) { *count = 0; }

// Unit of a batch-wide anchor index (binary search over the units' first anchors).
__device__ __forceinline__ int unit_of_anchor(const int64_t* __restrict__ off, int n_units, int64_t a) {
  int lo = 0, hi = n_units;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= a) lo = mid; else hi = mid;
  }
  return lo;
}

// Stale anchors of active filtered units: grid (anchor blocks, unit), one thread per
// anchor; an anchor is stale when the route of u or of v was rebuilt after the unit's
// last ranking. Marked anchors go to queue (one atomic per block); their customers
// are flagged in cmark.
__global__ __launch_bounds__(256) void k_anchor_mark(const UnitDesc* __restrict__ units,
                                                     const int64_t* __restrict__ anchor_off,
                                                     const int32_t* __restrict__ cust_off, int32_t* __restrict__ queue,
                                                     int32_t* __restrict__ count, uint8_t* __restrict__ cmark) {
  __shared__ int s_cnt[4], s_base;
  const int ui = blockIdx.y;
  const UnitDesc& U = units[ui];
  const UnitCtl* c = U.ctl;
  const int item = blockIdx.x * 256 + threadIdx.x;
  const int n_items = U.nc * U.theta;
  if (blockIdx.x * 256 >= n_items || !c->active || c->fmode != 1) return;  // uniform per block
  bool st = false;
  if (item < n_items) {
    const int i = item / U.theta, k = item - i * U.theta;
    if (k < U.nbr_len[i]) {
      const int se = c->scored_epoch;
      st = U.dirty[U.rt[U.nd + i]] > se || U.dirty[U.rt[U.nbr[item]]] > se;
      if (st) cmark[cust_off[ui] + i] = 1;
    }
  }
  const uint64_t m = __ballot(st);
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  if (lane == 0) s_cnt[wave] = __popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    const int tot = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
    s_base = tot ? atomicAdd(count, tot) : 0;
  }
  __syncthreads();
  if (st) {
    int at = s_base + __popcll(m & ((1ull << lane) - 1));
    for (int w = 0; w < wave; ++w) at += s_cnt[w];
    queue[at] = (int32_t)(anchor_off[ui] + item);
  }
}

// Logits of the queued anchors: each wavefront takes 64 anchors at a time (one per
// lane), builds their features, stages them in LDS as B fragments (32 anchors at a
// time), and runs the network on the matrix cores, 4 sample tiles per pass through
// the LDS copy of W2.
template <class SEG, bool TW>
__global__ __launch_bounds__(64 * kScoreWaves) void k_score_anchors(
    const UnitDesc* __restrict__ units, const int64_t* __restrict__ anchor_off, int n_units,
    const bf16x8* __restrict__ w1f, const bf16x8* __restrict__ w2f, const float* __restrict__ P,
    const float* __restrict__ w3b, const int32_t* __restrict__ queue, const int32_t* __restrict__ qcount,
    float* __restrict__ lcache) {
  static_assert(16 * kScoreT == 64 && kScoreT % kScoreStage == 0, "one anchor per lane");
  constexpr int SR = 16 * kScoreStage;  // staged rows
  __shared__ MlpSmem S;
  __shared__ __attribute__((aligned(16))) uint16_t xs[kScoreWaves][SR * kF];
  // without a queue every anchor of the batch is scored (missing list entries get zero
  // features; nothing reads their logits)
  const int n = queue ? *qcount : (int)anchor_off[n_units];
  if (n == 0) return;
  mlp_stage(S, w2f, P, w3b);
  const float b3 = P[P_B3];
  const int wave = threadIdx.x >> 6, lane = lane_id();
  constexpr int G = 16 * kScoreT;
  for (int g0 = (blockIdx.x * kScoreWaves + wave) * G; g0 < n; g0 += gridDim.x * kScoreWaves * G) {
    uint16_t f[kF];
    {
      const int q = g0 + lane;
      bool have = false;
      if (q < n) {
        const int64_t a = queue ? queue[q] : q;
        const int ui = unit_of_anchor(anchor_off, n_units, a);
        const UnitDesc& U = units[ui];
        const int item = (int)(a - anchor_off[ui]);
        const int i = item / U.theta, k = item - i * U.theta;
        if (k < U.nbr_len[i]) {  // queued anchors always are; in the all-anchors mode some are not
          pair_features<SEG, TW>(U, U.ctl->cur, U.nd + i, U.nbr[item], k, f);
          have = true;
        }
      }
      if (!have) {
#pragma unroll
        for (int z = 0; z < kF; ++z) f[z] = 0;
      }
    }
    bf16x8 xb[kScoreT];
#pragma unroll
    for (int h = 0; h < kScoreT / kScoreStage; ++h) {
      if (lane / SR == h) {
        uint4* row = (uint4*)&xs[wave][(lane % SR) * kF];
#pragma unroll
        for (int z = 0; z < 4; ++z) row[z] = pack8(f + 8 * z);
      }
      wave_lds_sync();
#pragma unroll
      for (int t = 0; t < kScoreStage; ++t)
        xb[h * kScoreStage + t] = *(const bf16x8*)&xs[wave][(16 * t + (lane & 15)) * kF + 8 * (lane >> 4)];
      wave_lds_sync();
    }
    float z[kScoreT];
    mlp_tiles<kScoreT>(S, w1f, xb, b3, z, nullptr, nullptr);
#pragma unroll
    for (int t = 0; t < kScoreT; ++t) {
      const int q = g0 + 16 * t + lane;
      if (lane < 16 && q < n) lcache[queue ? queue[q] : q] = z[t];
    }
  }
}

// Top-kc of every flagged customer (all = 1: every customer) from the cached logits
// (logit descending, customer id ascending; -1 padding); clears the flag. One
// wavefront per customer, lanes hold entries lane and lane + 64, kc rounds of a wave
// arg-max.
__global__ __launch_bounds__(256) void k_topk_marked(const UnitDesc* __restrict__ units,
                                                     const int32_t* __restrict__ cust_off, int n_units,
                                                     const float* __restrict__ lcache, uint8_t* __restrict__ cmark,
                                                     int all) {
  const int task = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = lane_id();
  if (task >= cust_off[n_units]) return;
  if (!all && !cmark[task]) return;
  const int ui = unit_of_tile(cust_off, n_units, task);
  const UnitDesc& U = units[ui];
  const int i = task - cust_off[ui];
  const int len = U.nbr_len[i];
  const int32_t* nb = U.nbr + (int64_t)i * U.theta;
  const float* lg = lcache + U.item_base + (int64_t)i * U.theta;
  float s0 = -INFINITY, s1 = -INFINITY;
  int v0 = INT32_MAX, v1 = INT32_MAX;
  if (lane < len) { s0 = lg[lane]; v0 = nb[lane]; }
  if (lane + 64 < len) { s1 = lg[lane + 64]; v1 = nb[lane + 64]; }
  int32_t* out = U.fcand + (int64_t)i * U.kc;
  for (int j = 0; j < U.kc; ++j) {
    float bs = s0;
    int bv = v0, src = lane, which = 0;
    if (s1 > bs || (s1 == bs && v1 < bv)) { bs = s1; bv = v1; which = 1; }
    for (int off = 32; off > 0; off >>= 1) {
      const float s2 = __shfl_xor(bs, off);
      const int v2 = __shfl_xor(bv, off);
      const int src2 = __shfl_xor(src, off);
      const int w2 = __shfl_xor(which, off);
      if (s2 > bs || (s2 == bs && v2 < bv)) { bs = s2; bv = v2; src = src2; which = w2; }
    }
    if (lane == 0) out[j] = bv == INT32_MAX ? -1 : bv;
    if (lane == src) {
      if (which == 0) { s0 = -INFINITY; v0 = INT32_MAX; }
      else { s1 = -INFINITY; v1 = INT32_MAX; }
    }
  }
  if (lane == 0) cmark[task] = 0;
}

// The heuristic filter: the first kc entries of each granular list (eta order).
__global__ void k_eta_lists(const UnitDesc* __restrict__ units, const int32_t* __restrict__ cust_off, int n_units) {
  const int task = blockIdx.x * blockDim.x + threadIdx.x;
  if (task >= cust_off[n_units]) return;
  const int ui = unit_of_tile(cust_off, n_units, task);
  const UnitDesc& U = units[ui];
  const int i = task - cust_off[ui];
  const int len = U.nbr_len[i];
  for (int j = 0; j < U.kc; ++j) U.fcand[(int64_t)i * U.kc + j] = j < len ? U.nbr[(int64_t)i * U.theta + j] : -1;
}

// ---------------------------------------------------------------------------- training forward

constexpr int kFwdT = 2;

// Forward over n samples x[n][32] (bf16): logits[n] and, when h1 / h2 are given, the
// rounded activations [n rounded up to 16 T][256] for the backward pass.
__global__ __launch_bounds__(256) void k_mlp_forward(const uint16_t* __restrict__ x, int n,
                                                     const bf16x8* __restrict__ w1f, const bf16x8* __restrict__ w2f,
                                                     const float* __restrict__ P, const float* __restrict__ w3b,
                                                     float* __restrict__ logits, uint16_t* __restrict__ h1,
                                                     uint16_t* __restrict__ h2) {
  __shared__ MlpSmem S;
  mlp_stage(S, w2f, P, w3b);
  const float b3 = P[P_B3];
  const int wave = threadIdx.x >> 6, lane = lane_id();
  const int groups = (n + 16 * kFwdT - 1) / (16 * kFwdT);
  for (int gi = blockIdx.x * 4 + wave; gi < groups; gi += gridDim.x * 4) {
    bf16x8 xb[kFwdT];
#pragma unroll
    for (int t = 0; t < kFwdT; ++t) {
      const int sample = (gi * kFwdT + t) * 16 + (lane & 15);
      if (sample < n) {
        xb[t] = *(const bf16x8*)&x[(int64_t)sample * kF + 8 * (lane >> 4)];
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) xb[t][e] = as_bf(0);
      }
    }
    float z[kFwdT];
    const int64_t row0 = (int64_t)gi * kFwdT * 16;
    mlp_tiles<kFwdT>(S, w1f, xb, b3, z, h1 ? h1 + row0 * kH : nullptr, h2 ? h2 + row0 * kH : nullptr);
#pragma unroll
    for (int t = 0; t < kFwdT; ++t) {
      const int sample = (gi * kFwdT + t) * 16 + (lane & 15);
      if (lane < 16 && sample < n) logits[sample] = z[t];
    }
  }
}

int mlp_row_pad() { return 16 * kFwdT; }

// ---------------------------------------------------------------------------- loss and backward

// wsum = sum of weights (n when weights is null). One block; the order of the sums is
// fixed by the block shape, so the result does not vary between runs.
__global__ void k_bce_prep(const float* __restrict__ w, int n, float* __restrict__ wsum) {
  __shared__ float sh[16];
  float s = 0.f;
  for (int p = threadIdx.x; p < n; p += blockDim.x) s += w ? w[p] : 1.f;
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (lane_id() == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.f;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += sh[k];
    *wsum = t;
  }
}

// Weighted mean BCE with logits: dz_p = w_p (sigmoid(z_p) - y_p) / sum w, and the block's
// share of the loss sum_p w_p l_p / sum w in part[blockIdx.x] (grid-stride over samples;
// 256 threads per block).
__global__ __launch_bounds__(256) void k_bce(const float* __restrict__ z, const float* __restrict__ y,
                                             const float* __restrict__ w, int n, const float* __restrict__ wsum,
                                             float* __restrict__ dz, float* __restrict__ part) {
  __shared__ float sh[4];
  const float ws = *wsum;
  const float inv = ws > 0.f ? 1.f / ws : 0.f;
  float l = 0.f;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
    const float wp = w ? w[p] : 1.f;
    const float zp = z[p];
    const float sg = 1.f / (1.f + expf(-zp));
    dz[p] = wp * (sg - y[p]) * inv;
    l += wp * ((zp > 0.f ? zp : 0.f) - zp * y[p] + log1pf(expf(-fabsf(zp)))) * inv;
  }
  for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off);
  if (lane_id() == 0) sh[threadIdx.x >> 6] = l;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// loss = sum of the nb block partials in a fixed order (one block of 1024 threads).
__global__ __launch_bounds__(1024) void k_bce_final(const float* __restrict__ part, int nb, float* __restrict__ loss) {
  __shared__ float sh[16];
  float s = 0.f;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) s += part[b];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (lane_id() == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.f;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += sh[k];
    *loss = t;
  }
}

__global__ void k_zero(float* __restrict__ g, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) g[i] = 0.f;
}

// Output layer, block share: part[blockIdx.x][0..255] = sum_p G2_p (the b2 gradient),
// [256..511] = sum_p dz_p h2_p (w3), [512] = sum_p dz_p (b3), over the block's samples;
// G2[p][o] = dz_p w3[o] [h2[p][o] > 0] rounded to bf16 (the layer-2 output gradient).
// Rows of kOutPart floats follow the parameter order b2, w3, b3.
constexpr int kOutPart = 2 * kH + 1;
__global__ __launch_bounds__(256) void k_back_out(const float* __restrict__ dz, const uint16_t* __restrict__ h2,
                                                  const float* __restrict__ w3b, int n, float* __restrict__ part,
                                                  uint16_t* __restrict__ G2) {
  const int o = threadIdx.x;
  float aw = 0.f, ab2 = 0.f, ab3 = 0.f;
  for (int p = blockIdx.x; p < n; p += gridDim.x) {
    const float d = dz[p];
    const float h = bf2f(h2[(int64_t)p * kH + o]);
    aw += d * h;
    ab3 += d;
    const float gv = h > 0.f ? d * w3b[o] : 0.f;
    ab2 += gv;
    G2[(int64_t)p * kH + o] = f2bf(gv);
  }
  float* row = part + (int64_t)blockIdx.x * kOutPart;
  row[o] = ab2;
  row[kH + o] = aw;
  if (o == 0) row[2 * kH] = ab3;
}

// G1 = (G2 W2) masked by [h1 > 0], rounded to bf16; one wave per 16 samples x 64 outputs
// (four 16 x 16 tiles sharing each A fragment). A(m, k) = G2[m][k] (row-major, 16-byte
// loads), B(k, n) = W2[k][n] (packed 16-byte fragments).
constexpr int kBhTiles = 4;
__global__ __launch_bounds__(256) void k_back_hidden(const uint16_t* __restrict__ G2, const bf16x8* __restrict__ w2b,
                                                     const uint16_t* __restrict__ h1, int n, uint16_t* __restrict__ G1) {
  const int wave = threadIdx.x >> 6, lane = lane_id(), g = lane >> 4;
  const int tm = (n + 15) / 16, tq = kH / (16 * kBhTiles);
  for (int t = blockIdx.x * 4 + wave; t < tm * tq; t += gridDim.x * 4) {
    const int m0 = (t / tq) * 16, nb0 = (t % tq) * kBhTiles;
    const int m = m0 + (lane & 15);
    f32x4 acc[kBhTiles];
#pragma unroll
    for (int q = 0; q < kBhTiles; ++q) acc[q] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int k0 = 0; k0 < kH; k0 += 32) {
      bf16x8 a;
      if (m < n) {
        a = *(const bf16x8*)&G2[(int64_t)m * kH + k0 + 8 * g];
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) a[e] = as_bf(0);
      }
#pragma unroll
      for (int q = 0; q < kBhTiles; ++q)  // W2[k0 + 8 g + e][16 (nb0 + q) + lane % 16], e = 0..7
        acc[q] = mfma(a, w2b[((nb0 + q) * 8 + k0 / 32) * 64 + lane], acc[q]);
    }
#pragma unroll
    for (int q = 0; q < kBhTiles; ++q) {
      const int nn = 16 * (nb0 + q) + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int mr = m0 + 4 * g + r;
        if (mr < n) {
          const int64_t at = (int64_t)mr * kH + nn;
          G1[at] = f2bf(bf2f(h1[at]) > 0.f ? acc[q][r] : 0.f);
        }
      }
    }
  }
}

// Block share of the column sums of bf16 rows of 256: part[blockIdx.x][o] = sum_p G[p][o].
__global__ __launch_bounds__(256) void k_colsum(const uint16_t* __restrict__ G, int n, float* __restrict__ part) {
  const int o = threadIdx.x;
  float acc = 0.f;
  for (int p = blockIdx.x; p < n; p += gridDim.x) acc += bf2f(G[(int64_t)p * kH + o]);
  part[(int64_t)blockIdx.x * kH + o] = acc;
}

constexpr int kSplitK = 1024;  // samples per chunk of the weight-gradient products
constexpr int kWgM = 64;       // output rows of one weight-gradient block (4 waves x 16)
constexpr int kWgLd = 40;      // LDS row length (bf16) of the transposed 32-sample slabs

// Position of sample s (0..31) in the LDS row of column c: the four 8-sample groups are
// permuted by bits 3-4 of c (XOR), so that the transposing 16-bit stores of the columns
// c8 .. c8 + 7 of different 8-column groups fall into different banks; a group stays
// contiguous and 16-byte aligned for the fragment reads.
__device__ __forceinline__ int wg_swz(int c, int s) { return s ^ (((c >> 3) & 3) << 3); }

// Weight gradient of one chunk of kSplitK samples: part[ch][M][N] = sum_p L[p][m] R[p][n]
// over the chunk's samples (both bf16, row-major with row lengths M and N; M a multiple
// of 64, N of 16). One block per (64 x 64 output tile, chunk): per step of 32 samples the
// block loads the 32 x 64 slabs of L and R with 16-byte row loads and stores them
// transposed in LDS (sample index contiguous), so that every MFMA operand fragment is one
// 16-byte LDS read; wave w computes rows 16 w .. 16 w + 15 of the tile against its (up
// to 64) columns. Every output element accumulates the chunk's samples 32 at a time in
// sample order, whatever the block shape, so the partial sums are deterministic.
__global__ __launch_bounds__(256) void k_wgrad(const uint16_t* __restrict__ Lm, int M, const uint16_t* __restrict__ Rm,
                                               int N, int n, float* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) uint16_t LT[kWgM * kWgLd];
  __shared__ __attribute__((aligned(16))) uint16_t RT[kWgM * kWgLd];
  const int tid = threadIdx.x, wave = tid >> 6, lane = lane_id(), g = lane >> 4;
  const int mb = M / kWgM, nb = (N + kWgM - 1) / kWgM;
  const int tile = blockIdx.x % (mb * nb), ch = blockIdx.x / (mb * nb);
  const int m0 = (tile / nb) * kWgM, n0 = (tile % nb) * kWgM;
  const int nw = min(kWgM, N - n0), tn = nw / 16;  // columns of this tile, in 16-column MFMA tiles
  const int p0 = ch * kSplitK, p1 = min(n, p0 + kSplitK);
  f32x4 acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = {0.f, 0.f, 0.f, 0.f};
  // slab loaders: thread t takes sample row t / 8 of the step and 8 consecutive columns;
  // the next step's rows are loaded while this step's MFMAs run
  const int row = tid >> 3, c8 = (tid & 7) * 8;
  auto load = [&](int k0, uint4& lv, uint4& rv) {
    const int p = k0 + row;
    lv = make_uint4(0, 0, 0, 0);
    rv = make_uint4(0, 0, 0, 0);
    if (p < p1) {
      lv = *(const uint4*)&Lm[(int64_t)p * M + m0 + c8];
      if (c8 < nw) rv = *(const uint4*)&Rm[(int64_t)p * N + n0 + c8];
    }
  };
  uint4 lv, rv;
  load(p0, lv, rv);
  for (int k0 = p0; k0 < p1; k0 += 32) {
    __syncthreads();  // the previous step's MFMAs have read the slabs
    const uint32_t lw[4] = {lv.x, lv.y, lv.z, lv.w}, rw[4] = {rv.x, rv.y, rv.z, rv.w};
    const int srow = wg_swz(c8, row);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      LT[(c8 + i) * kWgLd + srow] = (uint16_t)(lw[i >> 1] >> (16 * (i & 1)));
      RT[(c8 + i) * kWgLd + srow] = (uint16_t)(rw[i >> 1] >> (16 * (i & 1)));
    }
    load(k0 + 32, lv, rv);
    __syncthreads();
    const int ca = 16 * wave + (lane & 15);
    const bf16x8 a = *(const bf16x8*)&LT[ca * kWgLd + wg_swz(ca, 8 * g)];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (j >= tn) break;
      const int cb = 16 * j + (lane & 15);
      const bf16x8 bj = *(const bf16x8*)&RT[cb * kWgLd + wg_swz(cb, 8 * g)];
      acc[j] = mfma(a, bj, acc[j]);
    }
  }
  float* C = part + (int64_t)ch * M * N;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (j >= tn) break;
#pragma unroll
    for (int r = 0; r < 4; ++r) C[(m0 + 16 * wave + 4 * g + r) * N + n0 + 16 * j + (lane & 15)] = acc[j][r];
  }
}

// out[j] = sum over r of part[r][j], in the same order every run: 8 groups of rows
// (group k takes rows k, k + 8, ..., in order), then the 8 group sums in order. A block
// takes 32 columns (coalesced 128-byte row segments) with 8 threads per column.
constexpr int kRedCols = 32, kRedGroups = 8, kRedBatch = 16;
__global__ __launch_bounds__(kRedCols * kRedGroups) void k_reduce_rows(const float* __restrict__ part, int rows,
                                                                       int width, float* __restrict__ out) {
  __shared__ float sh[kRedGroups][kRedCols + 1];
  const int c = threadIdx.x % kRedCols, grp = threadIdx.x / kRedCols;
  const int j = blockIdx.x * kRedCols + c;
  float acc = 0.f;
  if (j < width) {
    // rows grp, grp + 8, ... added in order; loaded kRedBatch at a time so that the loads
    // overlap
    for (int r0 = grp; r0 < rows; r0 += kRedGroups * kRedBatch) {
      float v[kRedBatch];
#pragma unroll
      for (int u = 0; u < kRedBatch; ++u) {
        const int r = r0 + kRedGroups * u;
        v[u] = r < rows ? part[(int64_t)r * width + j] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < kRedBatch; ++u)
        if (r0 + kRedGroups * u < rows) acc += v[u];
    }
  }
  sh[grp][c] = acc;
  __syncthreads();
  if (grp == 0 && j < width) {
    float t = sh[0][c];
    for (int k = 1; k < kRedGroups; ++k) t += sh[k][c];
    out[j] = t;
  }
}

static void launch_reduce_rows(hipStream_t s, const float* part, int rows, int width, float* out) {
  hipLaunchKernelGGL(k_reduce_rows, dim3((width + kRedCols - 1) / kRedCols), dim3(kRedCols * kRedGroups), 0, s, part,
                     rows, width, out);
}

// Adam on the fp32 master parameters (bias-corrected moments).
__global__ void k_adam(float* __restrict__ P, float* __restrict__ m, float* __restrict__ v, const float* __restrict__ g,
                       int n, float lr, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  P[i] = P[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------------------- launchers

static int grid_for(int64_t work, int per_block, int cap) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(cap, (work + per_block - 1) / per_block));
}

void launch_mlp_pack(hipStream_t s, const MlpDev& M) {
  hipLaunchKernelGGL(k_mlp_pack, dim3((kH * kH + 255) / 256), dim3(256), 0, s, (const float*)M.P, (bf16x8*)M.w1f,
                     (bf16x8*)M.w2f, (bf16x8*)M.w2b, M.w3b);
}

void launch_mlp_zero(hipStream_t s, float* p, int n) {
  if (n > 0) hipLaunchKernelGGL(k_zero, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
}

template <class SEG, bool TW>
static void features_t(const LaunchCtx& L, uint16_t* out) {
  hipLaunchKernelGGL((k_features<SEG, TW>), dim3(L.tiles[0]), dim3(256), 0, L.stream, L.units, L.tile_off[0],
                     L.n_units, out);
}

void launch_features(const LaunchCtx& L, uint16_t* out) {
  if (L.tiles[0] <= 0) return;
  if (L.has_tw) features_t<SegTW, true>(L, out);
  else features_t<SegNT, false>(L, out);
}

template <class SEG, bool TW>
static void score_anchors_t(const LaunchCtx& L, const int64_t* anchor_off, const MlpDev& M, const FilterQueue& Q,
                            int64_t max_anchors) {
  const int blocks = grid_for(max_anchors, kScoreWaves * 16 * kScoreT, 256);
  hipLaunchKernelGGL((k_score_anchors<SEG, TW>), dim3(blocks), dim3(64 * kScoreWaves), 0, L.stream, L.units,
                     anchor_off, L.n_units, (const bf16x8*)M.w1f, (const bf16x8*)M.w2f, (const float*)M.P,
                     (const float*)M.w3b, Q.queue, Q.count, Q.lcache);
}

void launch_rank(const LaunchCtx& L, const int32_t* cust_off, int n_cust, const MlpDev& M, const FilterQueue& Q,
                 int all) {
  if (n_cust <= 0 || Q.n_anchors <= 0) return;
  if (!all) {
    // a fill kernel rather than a memset: the sequence may be captured in a graph
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(1), 0, L.stream, Q.count);
    hipLaunchKernelGGL(k_anchor_mark, dim3((unsigned)((Q.max_unit_anchors + 255) / 256), L.n_units), dim3(256), 0,
                       L.stream, L.units, Q.anchor_off, cust_off, Q.queue, Q.count, Q.cmark);
  }
  FilterQueue q = Q;
  if (all) q.queue = nullptr;
  if (L.has_tw) score_anchors_t<SegTW, true>(L, Q.anchor_off, M, q, Q.n_anchors);
  else score_anchors_t<SegNT, false>(L, Q.anchor_off, M, q, Q.n_anchors);
  hipLaunchKernelGGL(k_topk_marked, dim3((n_cust + 3) / 4), dim3(256), 0, L.stream, L.units, cust_off, L.n_units,
                     (const float*)Q.lcache, Q.cmark, all);
}

void launch_eta_lists(const LaunchCtx& L, const int32_t* cust_off, int n_tasks) {
  if (n_tasks <= 0) return;
  hipLaunchKernelGGL(k_eta_lists, dim3((n_tasks + 255) / 256), dim3(256), 0, L.stream, L.units, cust_off, L.n_units);
}

void launch_mlp_forward(hipStream_t s, const MlpDev& M, const uint16_t* x, int n, float* logits, uint16_t* h1,
                        uint16_t* h2) {
  if (n <= 0) return;
  const int groups = (n + 16 * kFwdT - 1) / (16 * kFwdT);
  hipLaunchKernelGGL(k_mlp_forward, dim3(grid_for(groups, 4, 1024)), dim3(256), 0, s, x, n, (const bf16x8*)M.w1f,
                     (const bf16x8*)M.w2f, (const float*)M.P, (const float*)M.w3b, logits, h1, h2);
}

int bce_blocks(int n, int max_blocks) { return grid_for(n, 256, max_blocks); }

void launch_bce(hipStream_t s, const float* z, const float* y, const float* w, int n, float* scratch, int nb,
                float* dz, float* loss) {
  hipLaunchKernelGGL(k_bce_prep, dim3(1), dim3(1024), 0, s, w, n, scratch);
  if (n > 0) hipLaunchKernelGGL(k_bce, dim3(nb), dim3(256), 0, s, z, y, w, n, (const float*)scratch, dz, scratch + 2);
  if (loss) hipLaunchKernelGGL(k_bce_final, dim3(1), dim3(1024), 0, s, (const float*)scratch + 2, n > 0 ? nb : 0, loss);
}

size_t mlp_grad_part_floats(int n) {
  const int64_t rows = grid_for(n, 1, 1024), chunks = (std::max(n, 1) + kSplitK - 1) / kSplitK;
  return (size_t)(rows * kOutPart + rows * kH + chunks * (int64_t)kH * (kH + kF));
}

// Gradient of sum_p dz_p logit_p written to g (every parameter); h1, h2 from the forward
// pass; G2, G1 scratch of [n][256] bf16 each; part: mlp_grad_part_floats(n) floats of
// per-block and per-chunk partial sums, reduced in a fixed order (the gradient does not
// vary between runs).
void launch_mlp_backward(hipStream_t s, const MlpDev& M, const uint16_t* x, int n, const float* dz, const uint16_t* h1,
                         const uint16_t* h2, float* g, uint16_t* G2, uint16_t* G1, float* part) {
  if (n <= 0) {
    launch_mlp_zero(s, g, P_N);
    return;
  }
  const int rows = grid_for(n, 1, 1024);
  const int chunks = (n + kSplitK - 1) / kSplitK;
  float* p_out = part;
  float* p_b1 = p_out + (int64_t)rows * kOutPart;
  float* p_w2 = p_b1 + (int64_t)rows * kH;
  float* p_w1 = p_w2 + (int64_t)chunks * kH * kH;
  hipLaunchKernelGGL(k_back_out, dim3(rows), dim3(kH), 0, s, dz, h2, (const float*)M.w3b, n, p_out, G2);
  launch_reduce_rows(s, (const float*)p_out, rows,
                     kOutPart, g + P_B2);
  // dW2[o2][o1] = sum_p G2[p][o2] h1[p][o1]
  static_assert(kH % kWgM == 0 && kH % 16 == 0 && kF % 16 == 0, "weight-gradient tiling");
  hipLaunchKernelGGL(k_wgrad, dim3((kH / kWgM) * ((kH + kWgM - 1) / kWgM) * chunks), dim3(256), 0, s,
                     (const uint16_t*)G2, kH, h1, kH, n, p_w2);
  launch_reduce_rows(s, (const float*)p_w2, chunks, kH * kH,
                     g + P_W2);
  const int64_t tiles = (int64_t)(n + 15) / 16 * (kH / (16 * kBhTiles));
  hipLaunchKernelGGL(k_back_hidden, dim3(grid_for(tiles, 4, 4096)), dim3(256), 0, s, (const uint16_t*)G2,
                     (const bf16x8*)M.w2b, h1, n, G1);
  hipLaunchKernelGGL(k_colsum, dim3(rows), dim3(kH), 0, s, (const uint16_t*)G1, n, p_b1);
  launch_reduce_rows(s, (const float*)p_b1, rows, kH, g + P_B1);
  // dW1[o1][i] = sum_p G1[p][o1] x[p][i]
  hipLaunchKernelGGL(k_wgrad, dim3((kH / kWgM) * ((kF + kWgM - 1) / kWgM) * chunks), dim3(256), 0, s,
                     (const uint16_t*)G1, kH, x, kF, n, p_w1);
  launch_reduce_rows(s, (const float*)p_w1, chunks, kH * kF,
                     g + P_W1);
}

void launch_adam(hipStream_t s, const MlpDev& M, const float* g, float lr, int step) {
  const double c1 = 1.0 - std::pow(0.9, step), c2 = 1.0 - std::pow(0.999, step);
  hipLaunchKernelGGL(k_adam, dim3((P_N + 255) / 256), dim3(256), 0, s, M.P, M.m, M.v, g, P_N, lr, (float)c1,
                     (float)c2);
}

int mlp_param_count() { return P_N; }

}  // namespace mdvrp
