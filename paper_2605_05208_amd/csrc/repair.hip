// repair.hip -- insertion of the customers missing from a partial solution
// (Section 3.3, after Algorithm 3): feasible / infeasible best insertion (FBI,
// IBI), feasible / infeasible regret insertion (FRI, IRI) and random insertion
// (RI).
//
// A unit loaded with a partial solution keeps its missing customers in a list
// (ascending ids). Each round inserts one customer per unit:
//   k_ins_eval   one block per (unit, missing customer still to place): the cost
//                change of inserting it at every position of every route, from
//                the prefix / suffix segments (fw[q] + x + bw[q+1]); the block
//                keeps the cheapest and the second cheapest admissible position;
//   k_ins_apply  one block per unit: picks the customer (the next in id order, or
//                the largest regret), and builds the new route (one wavefront) at
//                the end of the current position buffer -- or a new route at the
//                cheapest depot.
// Scratch of a unit (its follower-candidate arrays, unused outside an evaluation
// step): the missing list, per-customer records and flags.
#include "../../include/mdvrp.h"
#include "kernels.h"
#include "rebuild.h"

namespace mdvrp {

constexpr int kInsBlock = 256;
constexpr int kInsApplyBlock = 1024;

// Best two admissible positions of one missing customer.
struct InsRec {
  int64_t dF1, dF2;
  int64_t pos1;    // tie key of the best: predecessor customer, or N + first customer
  int32_t q1;      // absolute position of the predecessor of the best
  int32_t slot1;   // its route slot
  int32_t n_adm;   // admissible positions seen (counted up to 2)
  int32_t pad;
};

__device__ __forceinline__ int32_t* ins_list(const UnitDesc& U) { return (int32_t*)U.cand_key; }
__device__ __forceinline__ InsRec* ins_recs(const UnitDesc& U) { return (InsRec*)U.cand_id; }
__device__ __forceinline__ uint8_t* ins_done(const UnitDesc& U) { return U.cand_alive; }

__device__ __forceinline__ bool ins_less(int64_t f1, int64_t p1, int64_t f2, int64_t p2) {
  return f1 < f2 || (f1 == f2 && p1 < p2);
}

// Missing customers of each unit, ascending (one block per unit).
__global__ __launch_bounds__(kInsApplyBlock) void k_ins_begin(const UnitDesc* __restrict__ units) {
  const UnitDesc& U = units[blockIdx.x];
  __shared__ int sh[2 * (kInsApplyBlock / 64) + 1];
  int carry = 0;
  for (int base = 0; base < U.nc; base += kInsApplyBlock) {
    const int i = base + threadIdx.x;
    const int miss = i < U.nc && U.rt[U.nd + i] < 0 ? 1 : 0;
    int tot;
    const int ex = block_scan_excl<kInsApplyBlock>(miss, sh, &tot);
    if (miss) {
      ins_list(U)[carry + ex] = U.nd + i;
      ins_done(U)[carry + ex] = 0;
    }
    carry += tot;
  }
  if (threadIdx.x == 0) {
    U.ctl->n_unrouted = carry;
    U.ctl->n_inserted = 0;
    U.ctl->ins_evaluated = 0;
  }
}

// Cost change of inserting x after absolute position q of route slot s (route of L
// customers whose predecessor node is at position k of the route).
template <class SEG, bool TW, bool OPEN>
__device__ __forceinline__ void ins_cost(const UnitDesc& U, const SEG* fw, const SEG* bw, int q, int k, int L,
                                         int slot, int x, int64_t& dF, bool& feasible) {
  const SEG a = ld(fw, q);
  const SEG xs = node_seg<SEG>(U, x);
  const int32_t cax = arc_c(U, a.node, x), tax = arc_t(U, a.node, x);
  SEG nw = cat(a, cax, tax, xs);
  if (!OPEN || k < L) {
    const SEG b = ld(bw, q + 1);
    const int32_t cxb = arc_c(U, x, b.node), txb = arc_t(U, x, b.node);
    nw = cat(nw, cxb, txb, b);
  }
  const int4 tot = ld(U.r_tot, slot);
  const RouteTerms t = route_terms(U, nw);
  const int32_t lx0 = imax(tot.y - U.Q, 0);
  const int32_t dx0 = U.Dmax >= 0 ? imax(tot.z - U.Dmax, 0) : 0;
  const int32_t dTW = t.TW - tot.w, dLX = t.LX - lx0, dDX = t.DX - dx0;
  dF = delta_F(U, t.C - tot.x, dTW, dLX, dDX, 0);
  feasible = dTW == 0 && dLX == 0 && dDX == 0;
}

// One block per (unit, j): the j-th missing customer of the unit, when it is still to be
// placed and this round evaluates it (best insertion and the random operator: only the
// next one in id order; regret insertion: all of them).
template <class SEG, bool TW, bool OPEN>
__global__ __launch_bounds__(kInsBlock) void k_ins_eval(const UnitDesc* __restrict__ units, int op) {
  const UnitDesc& U = units[blockIdx.x];
  const UnitCtl* ctl = U.ctl;
  const int j = blockIdx.y;
  const int nu = ctl->n_unrouted, done = ctl->n_inserted;
  if (done >= nu || j >= nu) return;
  const bool regret = op == MDVRP_REPAIR_FRI || op == MDVRP_REPAIR_IRI;
  if (!regret && j != done) return;  // the list is taken in order: entry `done` is next
  if (ins_done(U)[j]) return;
  const bool feas_only = op == MDVRP_REPAIR_FBI || op == MDVRP_REPAIR_FRI;
  const int x = ins_list(U)[j];
  const int cur = ctl->cur;
  const SEG* fw = (const SEG*)U.fw[cur];
  const SEG* bw = (const SEG*)U.bw[cur];
  const int32_t* roff = U.r_off[cur];
  int64_t f1 = kNoMove, f2 = kNoMove, p1 = INT64_MAX;
  int q1 = -1, s1 = -1, adm = 0, ev = 0;
  // positions: after each routed customer a (items 0..nc-1), after the departure depot of
  // each live route slot (items nc..nc+R-1)
  for (int it = threadIdx.x; it < U.nc + U.R; it += kInsBlock) {
    int q, k, L, slot;
    int64_t pid;
    if (it < U.nc) {
      const int a = U.nd + it;
      slot = ld(U.rt, a);
      if (slot < 0) continue;
      k = ld(U.pos, a);
      L = ld(U.r_len, slot);
      q = ld(U.apos, a);
      pid = a;
    } else {
      slot = it - U.nc;
      L = ld(U.r_len, slot);
      if (L <= 0) continue;
      k = 0;
      q = ld(roff, slot);
      pid = (int64_t)U.n + ld(fw, q + 1).node;
    }
    int64_t dF;
    bool feas;
    ins_cost<SEG, TW, OPEN>(U, fw, bw, q, k, L, slot, x, dF, feas);
    ++ev;
    if (feas_only && !feas) continue;
    ++adm;
    if (ins_less(dF, pid, f1, p1)) {
      f2 = f1;
      f1 = dF; p1 = pid; q1 = q; s1 = slot;
    } else if (dF < f2) {
      f2 = dF;
    }
  }
  // block reduction of the best two
  __shared__ int64_t sf1[kInsBlock / 64], sf2[kInsBlock / 64], sp1[kInsBlock / 64];
  __shared__ int sq1[kInsBlock / 64], ss1[kInsBlock / 64], sadm[kInsBlock / 64], sev[kInsBlock / 64];
  for (int o = 32; o > 0; o >>= 1) {
    const int64_t g1 = __shfl_xor(f1, o), g2 = __shfl_xor(f2, o), gp = __shfl_xor(p1, o);
    const int gq = __shfl_xor(q1, o), gs = __shfl_xor(s1, o);
    adm += __shfl_xor(adm, o);
    ev += __shfl_xor(ev, o);
    if (ins_less(g1, gp, f1, p1)) {
      f2 = f1 < g2 ? f1 : g2;
      f1 = g1; p1 = gp; q1 = gq; s1 = gs;
    } else {
      f2 = g1 < f2 ? g1 : f2;
    }
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sf1[w] = f1; sf2[w] = f2; sp1[w] = p1; sq1[w] = q1; ss1[w] = s1; sadm[w] = adm; sev[w] = ev;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int v = 1; v < kInsBlock / 64; ++v) {
      if (ins_less(sf1[v], sp1[v], f1, p1)) {
        f2 = f1 < sf2[v] ? f1 : sf2[v];
        f1 = sf1[v]; p1 = sp1[v]; q1 = sq1[v]; s1 = ss1[v];
      } else {
        f2 = sf1[v] < f2 ? sf1[v] : f2;
      }
      adm += sadm[v];
      ev += sev[v];
    }
    InsRec r;
    r.dF1 = f1; r.dF2 = f2; r.pos1 = p1; r.q1 = q1; r.slot1 = s1; r.n_adm = adm; r.pad = 0;
    ins_recs(U)[j] = r;
    atomicAdd((unsigned long long*)&U.ctl->ins_evaluated, (unsigned long long)ev);
  }
}

// One block per unit: pick the customer to place, then build its new route. order
// receives the inserted customers of unit u from order_base[u] on.
template <class SEG, bool TW, bool OPEN>
__global__ __launch_bounds__(kInsApplyBlock) void k_ins_apply(const UnitDesc* __restrict__ units, int op,
                                                              uint64_t seed, int32_t* order,
                                                              const int32_t* __restrict__ order_base) {
  const UnitDesc& U = units[blockIdx.x];
  UnitCtl* ctl = U.ctl;
  const int nu = ctl->n_unrouted, done = ctl->n_inserted;
  if (done >= nu) return;
  const int tid = threadIdx.x;
  const int cur = ctl->cur;
  const SEG* fw = (const SEG*)U.fw[cur];
  __shared__ int sh[2 * (kInsApplyBlock / 64) + 1];
  __shared__ int s_j, s_slot, s_k, s_new, s_dep, s_found;
  __shared__ int64_t s_rg[kInsApplyBlock / 64];
  __shared__ int s_rj[kInsApplyBlock / 64];
  // ---- which customer
  if (op == MDVRP_REPAIR_FRI || op == MDVRP_REPAIR_IRI) {
    // largest regret (fewer than two admissible positions first), ties to the lower id
    int64_t best = -1;
    int bj = -1;
    for (int j = tid; j < nu; j += kInsApplyBlock) {
      if (ins_done(U)[j]) continue;
      const InsRec r = ins_recs(U)[j];
      const int64_t rg = r.n_adm >= 2 ? r.dF2 - r.dF1 : INT64_MAX;
      if (bj < 0 || rg > best) { best = rg; bj = j; }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const int64_t g = __shfl_xor(best, o);
      const int gj = __shfl_xor(bj, o);
      if (gj >= 0 && (bj < 0 || g > best || (g == best && gj < bj))) { best = g; bj = gj; }
    }
    if ((tid & 63) == 0) { s_rg[tid >> 6] = best; s_rj[tid >> 6] = bj; }
    __syncthreads();
    if (tid == 0) {
      for (int v = 1; v < kInsApplyBlock / 64; ++v) {
        const int gj = s_rj[v];
        if (gj >= 0 && (bj < 0 || s_rg[v] > best || (s_rg[v] == best && gj < bj))) { best = s_rg[v]; bj = gj; }
      }
      s_j = bj;
    }
  } else if (tid == 0) {
    s_j = done;
  }
  __syncthreads();
  const int j = s_j;
  const int x = ins_list(U)[j];
  // ---- where
  if (op == MDVRP_REPAIR_RI) {
    const int M = ctl->n_slots_alive;
    if (tid == 0) {
      s_new = M == 0;
      s_found = 0;
    }
    __syncthreads();
    if (M > 0) {
      uint64_t st = seed ^ (uint64_t)x;
      const uint64_t r1 = splitmix64_next(&st), r2 = splitmix64_next(&st);
      const int want = (int)(r1 % (uint64_t)M);  // route rank by first customer
      int carry = 0;
      for (int base = 0; base < U.nc; base += kInsApplyBlock) {
        const int i = base + tid;
        const int a = U.nd + i;
        const int head = i < U.nc && U.rt[a] >= 0 && U.pos[a] == 1 ? 1 : 0;
        int tot;
        const int ex = block_scan_excl<kInsApplyBlock>(head, sh, &tot);
        if (head && carry + ex == want) {
          const int slot = U.rt[a];
          const int L = U.r_len[slot];
          s_slot = slot;
          s_k = (int)(r2 % (uint64_t)(L + 1));
          s_found = 1;
        }
        carry += tot;
      }
      if (tid == 0) atomicAdd((unsigned long long*)&ctl->ins_evaluated, 1ull);
    }
    __syncthreads();
    if (M > 0 && !s_found) {  // cannot happen when the route table is consistent
      if (tid == 0) atomicOr(&ctl->err, 16);
      return;
    }
  } else {
    if (tid == 0) {
      const InsRec r = ins_recs(U)[j];
      s_new = r.n_adm == 0;
      s_slot = r.slot1;
      s_k = r.n_adm > 0 ? (r.pos1 < U.n ? U.pos[(int)r.pos1] : 0) : 0;
    }
    __syncthreads();
  }
  // ---- a new route: the cheapest depot (fleet term included, ties to the lower id) and
  // the lowest empty slot
  if (s_new) {
    if (tid < 64) {
      int64_t best = kNoMove;
      int bd = -1;
      for (int d = tid; d < U.nd; d += 64) {
        SEG r = cat(node_seg<SEG>(U, d), arc_c(U, d, x), arc_t(U, d, x), node_seg<SEG>(U, x));
        if (!OPEN) r = cat(r, arc_c(U, x, d), arc_t(U, x, d), node_seg<SEG>(U, d));
        const RouteTerms t = route_terms(U, r);
        const int n0 = U.ndep[d];
        const int dFX = imax(n0 + 1 - U.NV, 0) - imax(n0 - U.NV, 0);
        const int64_t f = delta_F(U, t.C, t.TW, t.LX, t.DX, dFX);
        if (bd < 0 || f < best) { best = f; bd = d; }
      }
      for (int o = 32; o > 0; o >>= 1) {
        const int64_t g = __shfl_xor(best, o);
        const int gd = __shfl_xor(bd, o);
        if (gd >= 0 && (bd < 0 || g < best || (g == best && gd < bd))) { best = g; bd = gd; }
      }
      if (tid == 0) s_dep = bd;
    }
    if (tid == 0) s_slot = -1;
    __syncthreads();
    // lowest empty slot
    for (int base = 0; base < U.R; base += kInsApplyBlock) {
      const int s = base + tid;
      const int empty = s < U.R && U.r_len[s] == 0 ? 1 : 0;
      int tot;
      const int ex = block_scan_excl<kInsApplyBlock>(empty, sh, &tot);
      if (empty && ex == 0 && s_slot < 0) s_slot = s;
      __syncthreads();
      if (s_slot >= 0) break;
    }
  }
  __syncthreads();
  const int slot = s_slot;
  const int top = ctl->arena_top;
  const int oldL = s_new ? 0 : U.r_len[slot];
  const int L = oldL + 1;
  if (slot < 0 || top + L + 2 > U.cap) {  // no empty slot or no room left in the buffer
    if (tid == 0) atomicOr(&ctl->err, 2);
    return;
  }
  const int start = s_new ? s_dep : U.r_start[slot];
  const int end = OPEN ? -1 : (s_new ? s_dep : U.r_end[slot]);
  const int old_off = s_new ? 0 : U.r_off[cur][slot];
  const int k = s_k;
  if (tid < 64) {
    auto nodeAt = [&](int p) -> int {
      if (s_new) return x;
      if (p <= k) return ld(fw, old_off + p).node;
      if (p == k + 1) return x;
      return ld(fw, old_off + p - 1).node;
    };
    build_route_wave<SEG, TW, OPEN>(U, cur, slot, top, L, start, end, nodeAt);
  }
  __syncthreads();
  if (tid == 0) {
    U.r_len[slot] = L;
    U.r_off[cur][slot] = top;
    U.r_meta[cur][slot] = make_int4(top, L, start, end);
    if (s_new) {
      U.r_start[slot] = start;
      U.r_end[slot] = end;
      U.ndep[start] += 1;
    }
    ctl->arena_top = top + L + 2;
    ins_done(U)[j] = 1;
    if (order) order[order_base[blockIdx.x] + done] = x;
    ctl->n_inserted = done + 1;
  }
  if (s_new) {  // the alive-slot list, in increasing order
    __syncthreads();
    int carry = 0;
    for (int base = 0; base < U.R; base += kInsApplyBlock) {
      const int s = base + tid;
      const int alive = s < U.R && U.r_len[s] > 0 ? 1 : 0;
      int tot;
      const int ex = block_scan_excl<kInsApplyBlock>(alive, sh, &tot);
      if (alive) U.slot_list[carry + ex] = s;
      carry += tot;
    }
    if (tid == 0) ctl->n_slots_alive = carry;
  }
}

__global__ void k_ins_export(const UnitDesc* __restrict__ units, int n_units, int64_t* out) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u < n_units) out[u] = units[u].ctl->ins_evaluated;
}

void launch_ins_export(const LaunchCtx& L, int64_t* out) {
  hipLaunchKernelGGL(k_ins_export, dim3((L.n_units + 255) / 256), dim3(256), 0, L.stream, L.units, L.n_units, out);
}

void launch_ins_begin(const LaunchCtx& L) {
  hipLaunchKernelGGL(k_ins_begin, dim3(L.n_units), dim3(kInsApplyBlock), 0, L.stream, L.units);
}

template <class SEG, bool TW, bool OPEN>
static void ins_round_t(const LaunchCtx& L, int op, uint64_t seed, int max_unrouted, int32_t* order,
                        const int32_t* order_base) {
  if (op != MDVRP_REPAIR_RI)
    hipLaunchKernelGGL((k_ins_eval<SEG, TW, OPEN>), dim3(L.n_units, max_unrouted), dim3(kInsBlock), 0, L.stream,
                       L.units, op);
  hipLaunchKernelGGL((k_ins_apply<SEG, TW, OPEN>), dim3(L.n_units), dim3(kInsApplyBlock), 0, L.stream, L.units, op,
                     seed, order, order_base);
}

void launch_ins_round(const LaunchCtx& L, int op, uint64_t seed, int max_unrouted, int32_t* order,
                      const int32_t* order_base) {
  if (L.has_tw) {
    if (L.open) ins_round_t<SegTW, true, true>(L, op, seed, max_unrouted, order, order_base);
    else ins_round_t<SegTW, true, false>(L, op, seed, max_unrouted, order, order_base);
  } else {
    if (L.open) ins_round_t<SegNT, false, true>(L, op, seed, max_unrouted, order, order_base);
    else ins_round_t<SegNT, false, false>(L, op, seed, max_unrouted, order, order_base);
  }
}

}  // namespace mdvrp
