// select.hip -- leader-follower multi-move selection and the apply plan (Section 3.2.5).
//
// The paper takes the leader (best move by F), then scans the followers
// (dD < 0, no penalty term changes) in ascending order and keeps each one that
// shares no route with a move already kept. With a strict total order on keys
// that greedy is the lexicographically first maximal independent set of the
// conflict graph, which iterated "locally dominant" rounds reach exactly: a
// move is taken when its key is the minimum among the live moves on every
// resource it touches; taken resources kill the other moves; repeat.
// Resources are route slots plus per-depot vehicle counts, so that the
// multi-move keeps F additive.
//
// One 1024-thread workgroup per unit. After selection the same workgroup
// turns each selected move into per-slot piece lists (the recipe of the
// evaluation) and lays out the rebuilt solution's offsets. In the local
// search it then rebuilds the new routes itself (one wavefront per route),
// which saves the separate apply launch and its round trips per step.
#include "kernels.h"
#include "rebuild.h"

namespace mdvrp {

constexpr int kSelBlock = 1024;
constexpr int kSelWaves = kSelBlock / 64;

__device__ __forceinline__ int block_scan(int v, int* sh, int* total) {
  return block_scan_excl<kSelBlock>(v, sh, total);
}

// resmin is only touched through device-scope atomics, so every access sees L2.
__device__ __forceinline__ uint64_t ld_min(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void reset_min(uint64_t* p) {
  __hip_atomic_store(p, ~0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int64_t unpack_dD(uint64_t key) { return (int64_t)(key >> 38) - (1ll << 25); }

// Units whose resources (route slots + depots) fit kLdsRes run the follower rounds
// with the per-resource minima in LDS, the candidates in registers when they fit
// kCandPerThread per thread; the others use the global-memory version (same rounds,
// same result). Units with more slots than that rename, in LDS, an alive route slot to
// its rank among the alive slots and depot d to n_alive + d (a bijection: the
// conflicts, and so the selection, are unchanged) when those fit.
constexpr int kLdsRes = 4096;
constexpr int kCandPerThread = 4;

struct SelLds {
  uint64_t rmin[kLdsRes];  // per resource: minimum key of the live candidates touching it
  uint8_t taken[kLdsRes];  // per resource: taken by a selected move of this step
};

// LDS name of resource r (a slot of an alive route, R + depot, or -1 = none). A slot
// that is not alive would be a broken invariant: it is reported (error bit 32) and
// dropped.
struct ResRename {
  const int32_t* rank;       // rank of each alive slot in the alive-slot list (null: no renaming)
  const int32_t* slot_list;  // the alive-slot list
  int R, n_alive;
  __device__ __forceinline__ int operator()(int r, UnitCtl* ctl) const {
    if (!rank || r < 0) return r < 0 ? -1 : r;
    if (r >= R) return n_alive + (r - R);
    const int x = rank[r];
    if (x >= 0 && x < n_alive && slot_list[x] == r) return x;
    atomicOr(&ctl->err, 32);
    return -1;
  }
  __device__ __forceinline__ int4 operator()(int4 r, UnitCtl* ctl) const {
    return make_int4((*this)(r.x, ctl), (*this)(r.y, ctl), (*this)(r.z, ctl), r.w);
  }
};

__device__ __forceinline__ bool lds_taken(const SelLds& S, const int4& r) {
  return (r.x >= 0 && S.taken[r.x]) || (r.y >= 0 && S.taken[r.y]) || (r.z >= 0 && S.taken[r.z]);
}

// Per-step data the selection keeps in LDS: the selected moves (the first kPlanLds;
// further ones go to the unit's global arrays), the objective delta, the vehicle
// counts per depot (kernels launched with DEPL), and in the fused step the recipes
// of the new routes of the first kPlanLds moves.
constexpr int kPlanLds = 256;
constexpr int kDepLds = 256;  // depot counts kept in LDS during the step when nd <= kDepLds

struct PlanLds {
  uint64_t id[kPlanLds];
  int64_t dF[kPlanLds];
  int32_t size[kPlanLds];  // positions the move's new routes take, then their exclusive offset
  int32_t ndep[kDepLds];   // vehicle counts per depot (DEPL kernels)
  unsigned long long F;
  RouteRec rr[2 * kPlanLds];  // fused step: new route w of move s is rr[2 s + w] (len < 0 = none)
};

template <bool APPLY, bool DEPL>
struct SelView {
  const UnitDesc& U;
  PlanLds& P;
  __device__ __forceinline__ bool in_lds(int s) const { return APPLY && s < kPlanLds; }
  __device__ __forceinline__ void put(int s, uint64_t id, int64_t dF) const {
    if (in_lds(s)) { P.id[s] = id; P.dF[s] = dF; }
    else { U.sel_id[s] = id; U.sel_dF[s] = dF; }
  }
  __device__ __forceinline__ uint64_t id(int s) const { return in_lds(s) ? P.id[s] : U.sel_id[s]; }
  __device__ __forceinline__ int64_t dF(int s) const { return in_lds(s) ? P.dF[s] : U.sel_dF[s]; }
  __device__ __forceinline__ int size(int s) const { return in_lds(s) ? P.size[s] : U.sel_size[s]; }
  __device__ __forceinline__ void set_size(int s, int v) const {
    if (in_lds(s)) P.size[s] = v;
    else U.sel_size[s] = v;
  }
  // DEPL (chosen per launch, so that no code path mixes the two address spaces): the
  // counts live in LDS for the step and are updated with LDS atomics through an
  // explicit LDS pointer; otherwise with device atomics on the unit's array
  __device__ __forceinline__ void dep_add(int d, int by) const {
    if constexpr (DEPL) {
      __attribute__((address_space(3))) int32_t* p = (__attribute__((address_space(3))) int32_t*)&P.ndep[d];
      __hip_atomic_fetch_add(p, by, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    } else {
      atomicAdd(&U.ndep[d], by);
    }
  }
};

// Locally dominant rounds with the candidates held in registers (thread t holds
// candidates t, t + kSelBlock, ...) and the per-resource minima in LDS.
template <bool APPLY, bool DEPL>
__device__ __forceinline__ void followers_lds(const SelView<APPLY, DEPL>& V, SelLds& S, const ResRename& rn, int n_cand,
                                              uint64_t lead_id, int* s_nsel, int* s_alive) {
  const UnitDesc& U = V.U;
  const int tid = threadIdx.x;
  uint64_t ck[kCandPerThread], ci[kCandPerThread];
  int4 cr[kCandPerThread];
  int st[kCandPerThread];  // 0 dead, 1 live, 2 selected this round
#pragma unroll
  for (int j = 0; j < kCandPerThread; ++j) {
    const int c = tid + j * kSelBlock;
    st[j] = 0;
    if (c < n_cand) {
      ck[j] = U.cand_key[c];
      ci[j] = U.cand_id[c];
      cr[j] = rn(U.cand_res[c], U.ctl);
      st[j] = (ci[j] != lead_id && !lds_taken(S, cr[j])) ? 1 : 0;
    }
  }
  for (int round = 0;; ++round) {
#pragma unroll
    for (int j = 0; j < kCandPerThread; ++j) {
      if (st[j] != 1) continue;
      const int4 r = cr[j];
      if (r.x >= 0) atomicMin((unsigned long long*)&S.rmin[r.x], (unsigned long long)ck[j]);
      if (r.y >= 0) atomicMin((unsigned long long*)&S.rmin[r.y], (unsigned long long)ck[j]);
      if (r.z >= 0) atomicMin((unsigned long long*)&S.rmin[r.z], (unsigned long long)ck[j]);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kCandPerThread; ++j) {
      if (st[j] != 1) continue;
      const int4 r = cr[j];
      const uint64_t k = ck[j];
      if ((r.x < 0 || S.rmin[r.x] == k) && (r.y < 0 || S.rmin[r.y] == k) && (r.z < 0 || S.rmin[r.z] == k)) {
        st[j] = 2;
        V.put(atomicAdd(s_nsel, 1), ci[j], unpack_dD(k));
      }
    }
    if (tid == 0) *s_alive = 0;
    __syncthreads();
    // the selected moves take their resources (no live move reads taken[] until the sync)
#pragma unroll
    for (int j = 0; j < kCandPerThread; ++j) {
      if (st[j] != 2) continue;
      const int4 r = cr[j];
      if (r.x >= 0) S.taken[r.x] = 1;
      if (r.y >= 0) S.taken[r.y] = 1;
      if (r.z >= 0) S.taken[r.z] = 1;
      st[j] = 0;
    }
    __syncthreads();
    int alive = 0;
#pragma unroll
    for (int j = 0; j < kCandPerThread; ++j) {
      if (st[j] != 1) continue;
      const int4 r = cr[j];
      if (lds_taken(S, r)) { st[j] = 0; continue; }
      if (r.x >= 0) S.rmin[r.x] = ~0ull;
      if (r.y >= 0) S.rmin[r.y] = ~0ull;
      if (r.z >= 0) S.rmin[r.z] = ~0ull;
      ++alive;
    }
    if (alive) atomicAdd(s_alive, alive);
    __syncthreads();
    if (*s_alive == 0) break;
    if (round > n_cand + 1) {  // every round takes the smallest live move
      if (tid == 0) atomicOr(&U.ctl->err, 16);
      break;
    }
  }
}

// The same rounds for more candidates than the registers hold: the per-resource minima
// and taken flags stay in LDS, the candidates are read from the unit's arrays every
// round (their resources renamed once, in place) and their state is kept in
// cand_alive (0 dead, 1 live, 2 selected this round). A move selected in a round
// takes its resources at once: the other moves of the round only compare minima.
template <bool APPLY, bool DEPL>
__device__ __forceinline__ void followers_lds_big(const SelView<APPLY, DEPL>& V, SelLds& S, const ResRename& rn,
                                                  int n_cand, uint64_t lead_id, int* s_nsel, int* s_alive) {
  const UnitDesc& U = V.U;
  const int tid = threadIdx.x;
  for (int c = tid; c < n_cand; c += kSelBlock) {
    const int4 r = rn(U.cand_res[c], U.ctl);
    if (rn.rank) U.cand_res[c] = r;
    U.cand_alive[c] = (U.cand_id[c] != lead_id && !lds_taken(S, r)) ? 1 : 0;
  }
  __syncthreads();
  for (int round = 0;; ++round) {
    for (int c = tid; c < n_cand; c += kSelBlock) {
      if (U.cand_alive[c] != 1) continue;
      const int4 r = U.cand_res[c];
      const unsigned long long k = U.cand_key[c];
      if (r.x >= 0) atomicMin((unsigned long long*)&S.rmin[r.x], k);
      if (r.y >= 0) atomicMin((unsigned long long*)&S.rmin[r.y], k);
      if (r.z >= 0) atomicMin((unsigned long long*)&S.rmin[r.z], k);
    }
    __syncthreads();
    for (int c = tid; c < n_cand; c += kSelBlock) {
      if (U.cand_alive[c] != 1) continue;
      const int4 r = U.cand_res[c];
      const uint64_t k = U.cand_key[c];
      if ((r.x < 0 || S.rmin[r.x] == k) && (r.y < 0 || S.rmin[r.y] == k) && (r.z < 0 || S.rmin[r.z] == k)) {
        U.cand_alive[c] = 2;
        V.put(atomicAdd(s_nsel, 1), U.cand_id[c], unpack_dD(k));
        if (r.x >= 0) S.taken[r.x] = 1;
        if (r.y >= 0) S.taken[r.y] = 1;
        if (r.z >= 0) S.taken[r.z] = 1;
      }
    }
    if (tid == 0) *s_alive = 0;
    __syncthreads();
    int alive = 0;
    for (int c = tid; c < n_cand; c += kSelBlock) {
      const uint8_t st = U.cand_alive[c];
      if (st == 0) continue;
      if (st == 2) { U.cand_alive[c] = 0; continue; }
      const int4 r = U.cand_res[c];
      if (lds_taken(S, r)) { U.cand_alive[c] = 0; continue; }
      if (r.x >= 0) S.rmin[r.x] = ~0ull;
      if (r.y >= 0) S.rmin[r.y] = ~0ull;
      if (r.z >= 0) S.rmin[r.z] = ~0ull;
      ++alive;
    }
    if (alive) atomicAdd(s_alive, alive);
    __syncthreads();
    if (*s_alive == 0) break;
    if (round > n_cand + 1) {  // every round takes the smallest live move
      if (tid == 0) atomicOr(&U.ctl->err, 16);
      break;
    }
  }
}

// Move s of the selection: per new route the pieces of the old routes it is made of
// (with the old routes' absolute offsets, so the rebuild can read them wherever the
// new routes go), its length, depots and slot. The recipe goes to LDS (fused step,
// s < kPlanLds) or to the unit's plan arrays; the route table entries are updated.
template <bool OPEN, bool APPLY, bool DEPL>
__device__ __forceinline__ void plan_move(const SelView<APPLY, DEPL>& V, int cur, uint64_t id, int64_t dF, int fresh_slot, int epoch, int s) {
  const UnitDesc& U = V.U;
  const int kind = (int)(id >> 56), var = (int)((id >> 48) & 0xff);
  const int a = (int)((id >> 24) & 0xffffff), b = (int)(id & 0xffffff);
  RouteCtx rc[2];
  Recipe R;
  rc[0] = route_ctx(U, cur, ld(U.rt, a));
  if (kind <= TWOOPT) {
    rc[1] = route_ctx(U, cur, ld(U.rt, b));
    build_pair(kind, var, rc[0], ld(U.pos, a), rc[1], ld(U.pos, b), rc[0].slot == rc[1].slot, /*sym=*/true, R);
  } else if (kind == DINS) {
    build_dins(rc[0], ld(U.pos, a), b, OPEN, R);
  } else {
    build_drep(rc[0], b, var, R);
  }
  // (loops over routes and pieces are unrolled with static indices: the recipe and the
  // route contexts stay in registers)
  V.dep_add(rc[0].start, -1);
  if (R.nold > 1) V.dep_add(rc[1].start, -1);
  const bool rec = V.in_lds(s);
  int size = 0;
  if (rec) V.P.rr[2 * s + 1].len = -1;
  else U.sel_slot[2 * s + 1] = -1;
#pragma unroll
  for (int w = 0; w < 2; ++w) {
    if (w >= R.nnew) break;
    const int slot = (R.fresh && w == 1) ? fresh_slot : rc[w].slot;
    const int np = R.np[w];
    int len = 0;
#pragma unroll
    for (int k = 0; k < kMaxPieces; ++k)
      if (k < np) len += R.pc[w][k].to - R.pc[w][k].from + 1;
    if (rec) {
      RouteRec& r = V.P.rr[2 * s + w];
      r.slot = slot; r.len = len; r.start = R.st[w]; r.end = R.en[w]; r.np = np;
#pragma unroll
      for (int k = 0; k < kMaxPieces; ++k) {
        if (k >= np) break;
        const Piece& p = R.pc[w][k];
        r.pc[k] = make_int4(p.src ? rc[1].off : rc[0].off, p.from, p.to, p.rev);
      }
      U.plan_n[slot] = -1;  // a relayout in this step leaves this route to the recorded build
    } else {
#pragma unroll
      for (int k = 0; k < kMaxPieces; ++k) {
        if (k >= np) break;
        const Piece& p = R.pc[w][k];
        U.plan_pc[(int64_t)slot * kMaxPieces + k] = make_int4(p.src ? rc[1].off : rc[0].off, p.from, p.to, p.rev);
      }
      U.plan_n[slot] = R.np[w];
      U.sel_slot[2 * s + w] = slot;
    }
    U.dirty[slot] = epoch;
    U.r_len[slot] = len;
    if (len > 0) {
      U.r_start[slot] = R.st[w];
      U.r_end[slot] = R.en[w];
      size += len + 2;
      V.dep_add(R.st[w], +1);
    }
    if (len > U.len_guard) atomicOr(&U.ctl->err, 4);
  }
  V.set_size(s, size);
  atomicAdd(&V.P.F, (unsigned long long)dF);
}

// Dynamic penalty coefficients (Section 3.2.1; kappa = 1/2, integer form) after a step
// that applied moves, from the unit's new solution: each weight is doubled when the
// solution violates its term (time warp; load excess; duration excess; closure or
// fleet excess) and halved, rounding down, when it does not, then clamped to its
// bounds. Called by the whole block after the new routes are built; the new weights go
// to the unit's entry of the device copy of the unit descriptors, which every later
// launch reads (this kernel reads none of them afterwards).
template <bool OPEN>
__device__ __forceinline__ void adapt_weights(const UnitDesc& U, const UnitCtl* ctl, UnitDesc* out,
                                              const AdaptBounds& b, int* s_viol) {
  const int tid = threadIdx.x;
  if (tid == 0) *s_viol = 0;
  __syncthreads();
  int v = 0;
  const int n_alive = ctl->n_slots_alive;
  for (int i = tid; i < n_alive; i += kSelBlock) {
    const int s = U.slot_list[i];
    const int4 t = U.r_tot[s];  // {C, Q, D, TW}
    if (t.w > 0) v |= 1;
    if (t.y > U.Q) v |= 2;
    if (U.Dmax >= 0 && t.z > U.Dmax) v |= 4;
    if (!OPEN && U.r_end[s] >= 0 && U.r_end[s] != U.r_start[s]) v |= 8;
  }
  for (int d = tid; d < U.nd; d += kSelBlock)
    if (U.ndep[d] > U.NV) v |= 8;
  if (v) atomicOr(s_viol, v);
  __syncthreads();
  if (tid == 0) {
    const int viol = *s_viol;
    const int64_t w[4] = {U.w_tw, U.w_load, U.w_dur, U.w_depot};
    int64_t nw[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t x = (viol >> k & 1) ? 2 * w[k] : w[k] / 2;
      nw[k] = x < b.lo[k] ? b.lo[k] : (x > b.hi[k] ? b.hi[k] : x);
    }
    out->w_tw = (int32_t)nw[0];
    out->w_load = (int32_t)nw[1];
    out->w_dur = (int32_t)nw[2];
    out->w_depot = nw[3];
  }
}

template <class SEG, bool TW, bool OPEN, bool APPLY, bool DEPL>
__global__ __launch_bounds__(kSelBlock) void k_select_plan(const UnitDesc* __restrict__ units, uint32_t cls_mask,
                                                           int leader_only, int scored, UnitDesc* adapt_units,
                                                           AdaptBounds adapt) {
  const UnitDesc& U = units[blockIdx.x];
  UnitCtl* ctl = U.ctl;
  __shared__ int64_t shF[kSelWaves];
  __shared__ uint64_t shI[kSelWaves];
  __shared__ int shT[kSelWaves];
  __shared__ int sh[2 * kSelWaves + 1];
  __shared__ MoveRec shRec[kSelWaves];
  __shared__ int s_nsel, s_alive, s_epoch, s_leader_wave, s_ndins, s_nbuild, s_alive_changed, s_viol;
  __shared__ SelLds S;
  __shared__ PlanLds P;
  if (!ctl->active) return;
  const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
  // every control field the step reads, loaded at once (the step is a chain of memory
  // round trips; these need not add to it)
  const int cur = ctl->cur, fmode = ctl->fmode, ftiles_ev = ctl->ftiles_eval, n_alive = ctl->n_slots_alive;
  const int epoch0 = ctl->epoch, n_cand0 = ctl->n_cand, top = ctl->arena_top;
  const SelView<APPLY, DEPL> V{U, P};
  if constexpr (DEPL)
    for (int d = tid; d < U.nd; d += kSelBlock) P.ndep[d] = U.ndep[d];

  // ---- leader: minimum (dF, id) over the block bests of the evaluated item classes
  int64_t bf = kNoMove;
  uint64_t bi = ~0ull;
  int bt = -1;
  for (int c = 0; c < 3; ++c) {
    if (!(cls_mask >> c & 1)) continue;
    // a filtered unit's pair tiles cover its candidate lists only; Depot-Replace tiles
    // cover the alive routes only
    int t_end = U.tile_base[c + 1];
    if (c == 0 && fmode == 1) t_end = U.tile_base[0] + ftiles_ev;
    if (c == 2) t_end = imin(t_end, U.tile_base[2] + (n_alive * U.nd + kTileSize - 1) / kTileSize);
    for (int t = U.tile_base[c] + tid; t < t_end; t += kSelBlock) {
      const int64_t f = U.wg_best[t].dF;
      const uint64_t i = U.wg_best[t].id;
      if (key_less(f, i, bf, bi)) { bf = f; bi = i; bt = t; }
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const int64_t f2 = __shfl_xor(bf, off);
    const uint64_t i2 = __shfl_xor(bi, off);
    const int t2 = __shfl_xor(bt, off);
    if (key_less(f2, i2, bf, bi)) { bf = f2; bi = i2; bt = t2; }
  }
  // each wavefront's best record goes to LDS with its key, so that the leader's record
  // needs no further load once the wavefronts are compared
  if (lane == 0) {
    shF[wave] = bf; shI[wave] = bi; shT[wave] = bt;
    if (bt >= 0) shRec[wave] = U.wg_best[bt];
  }
  __syncthreads();
  if (tid == 0) {
    int bw = 0;
    for (int w = 1; w < kSelWaves; ++w)
      if (key_less(shF[w], shI[w], shF[bw], shI[bw])) bw = w;
    s_leader_wave = bw;
    s_nsel = 0;
    s_ndins = 0;
    s_nbuild = 0;
    s_alive_changed = 0;
    P.F = 0;
    ctl->steps += 1;
    // the lists scored before this step's evaluation reflect every route up to this epoch
    if (scored && fmode == 1) ctl->scored_epoch = epoch0;
    if (shF[bw] < 0) {
      s_epoch = epoch0 + 1;
      ctl->epoch = s_epoch;
      ctl->leader = shRec[bw];
    } else {
      s_epoch = 0;
      ctl->n_sel = 0;
      ctl->n_cand = 0;
    }
  }
  __syncthreads();
  if (s_epoch == 0) return;  // no improving move: this step applies nothing
  const int epoch = s_epoch;
  const MoveRec lead = shRec[s_leader_wave];
  const int n_cand = imin(n_cand0, U.cand_cap);

  // resources in LDS: the slots themselves when they fit, else the renamed alive slots
  const bool rename = U.R + U.nd > kLdsRes;
  const int n_res = rename ? n_alive + U.nd : U.R + U.nd;
  const bool lds = !leader_only && n_res <= kLdsRes;
  const bool lds_regs = lds && n_cand <= kSelBlock * kCandPerThread;
  // ranks of the alive slots, in the resource minima's storage beyond the room of the
  // free-slot list the plan keeps there (as int32)
  int32_t* rank = rename ? (int32_t*)U.resmin + (U.R + U.nd) : nullptr;
  const ResRename rn{rank, U.slot_list, U.R, n_alive};
  if (lds) {
    for (int i = tid; i < n_res; i += kSelBlock) {
      S.rmin[i] = ~0ull;
      S.taken[i] = 0;
    }
    if (rename)
      for (int i = tid; i < n_alive; i += kSelBlock) rank[U.slot_list[i]] = i;
    __syncthreads();
  }
  if (tid == 0) {
    V.put(0, lead.id, lead.dF);
    s_nsel = 1;
    for (int k = 0; k < 3; ++k)
      if (lead.res[k] >= 0) {
        if (lds) {
          const int x = rn(lead.res[k], ctl);
          if (x >= 0) S.taken[x] = 1;
        } else {
          U.taken[lead.res[k]] = epoch;
        }
      }
  }
  __syncthreads();

  // ---- followers: locally dominant rounds
  if (lds_regs) {
    followers_lds(V, S, rn, n_cand, lead.id, &s_nsel, &s_alive);
  } else if (lds) {
    followers_lds_big(V, S, rn, n_cand, lead.id, &s_nsel, &s_alive);
  } else if (!leader_only) {
    for (int c = tid; c < n_cand; c += kSelBlock) {
      const int4 r = U.cand_res[c];
      bool live = U.cand_id[c] != lead.id;
      live = live && !(r.x >= 0 && U.taken[r.x] == epoch) && !(r.y >= 0 && U.taken[r.y] == epoch) &&
             !(r.z >= 0 && U.taken[r.z] == epoch);
      U.cand_alive[c] = live ? 1 : 0;
      if (live) {
        if (r.x >= 0) reset_min(&U.resmin[r.x]);
        if (r.y >= 0) reset_min(&U.resmin[r.y]);
        if (r.z >= 0) reset_min(&U.resmin[r.z]);
      }
    }
    __syncthreads();
    for (int round = 0;; ++round) {
      for (int c = tid; c < n_cand; c += kSelBlock) {
        if (U.cand_alive[c] != 1) continue;
        const int4 r = U.cand_res[c];
        const uint64_t k = U.cand_key[c];
        if (r.x >= 0) atomicMin((unsigned long long*)&U.resmin[r.x], (unsigned long long)k);
        if (r.y >= 0) atomicMin((unsigned long long*)&U.resmin[r.y], (unsigned long long)k);
        if (r.z >= 0) atomicMin((unsigned long long*)&U.resmin[r.z], (unsigned long long)k);
      }
      __syncthreads();
      for (int c = tid; c < n_cand; c += kSelBlock) {
        if (U.cand_alive[c] != 1) continue;
        const int4 r = U.cand_res[c];
        const uint64_t k = U.cand_key[c];
        const bool dom = (r.x < 0 || ld_min(&U.resmin[r.x]) == k) && (r.y < 0 || ld_min(&U.resmin[r.y]) == k) &&
                         (r.z < 0 || ld_min(&U.resmin[r.z]) == k);
        if (dom) {
          U.cand_alive[c] = 2;
          V.put(atomicAdd(&s_nsel, 1), U.cand_id[c], unpack_dD(k));
          if (r.x >= 0) U.taken[r.x] = epoch;
          if (r.y >= 0) U.taken[r.y] = epoch;
          if (r.z >= 0) U.taken[r.z] = epoch;
        }
      }
      if (tid == 0) s_alive = 0;
      __syncthreads();
      int alive = 0;
      for (int c = tid; c < n_cand; c += kSelBlock) {
        const uint8_t st = U.cand_alive[c];
        if (st == 0) continue;
        if (st == 2) { U.cand_alive[c] = 0; continue; }
        const int4 r = U.cand_res[c];
        if ((r.x >= 0 && U.taken[r.x] == epoch) || (r.y >= 0 && U.taken[r.y] == epoch) ||
            (r.z >= 0 && U.taken[r.z] == epoch)) {
          U.cand_alive[c] = 0;
          continue;
        }
        if (r.x >= 0) reset_min(&U.resmin[r.x]);
        if (r.y >= 0) reset_min(&U.resmin[r.y]);
        if (r.z >= 0) reset_min(&U.resmin[r.z]);
        ++alive;
      }
      if (alive) atomicAdd(&s_alive, alive);
      __syncthreads();
      if (s_alive == 0) break;
      // every round takes at least the smallest live move; a round count beyond
      // the candidate count means an invariant broke: stop and report it
      if (round > n_cand + 1) {
        if (tid == 0) atomicOr(&ctl->err, 16);
        break;
      }
    }
  }
  __syncthreads();
  const int n_sel = s_nsel;

  // ---- plan: free slots for Depot-Insert routes, taken in key order
  for (int s = tid; s < n_sel; s += kSelBlock)
    if ((V.id(s) >> 56) == DINS) atomicAdd(&s_ndins, 1);
  __syncthreads();
  const int n_dins = s_ndins;
  // free slot list (slots empty before this step) into resmin's storage as int32
  int32_t* free_list = (int32_t*)U.resmin;
  if (n_dins > 0) {
    int carry = 0;
    for (int base = 0; base < U.R; base += kSelBlock) {
      const int s = base + tid;
      const int f = (s < U.R && U.r_len[s] == 0) ? 1 : 0;
      int tot;
      const int ex = block_scan(f, sh, &tot);
      if (f && carry + ex < n_dins) free_list[carry + ex] = s;
      carry += tot;
    }
    if (carry < n_dins && tid == 0) atomicOr(&ctl->err, 2);
  }
  __syncthreads();
  for (int s = tid; s < n_sel; s += kSelBlock) {
    const uint64_t id = V.id(s);
    const int64_t dF = V.dF(s);
    int fresh = -1;
    if ((id >> 56) == DINS) {
      int rank = 0;
      for (int z = 0; z < n_sel; ++z) {
        const uint64_t iz = V.id(z);
        if ((iz >> 56) == DINS && key_less(V.dF(z), iz, dF, id)) ++rank;
      }
      fresh = rank < n_dins ? free_list[rank] : 0;
    }
    plan_move<OPEN, APPLY, DEPL>(V, cur, id, dF, fresh, epoch, s);
  }
  __syncthreads();
  if constexpr (DEPL)
    for (int d = tid; d < U.nd; d += kSelBlock) U.ndep[d] = P.ndep[d];

  // ---- where the new routes go: appended at the end of the current buffer when they
  // fit (the other routes stay where they are), else a relayout of every route into
  // the other buffer
  int total = 0;
  for (int base = 0; base < n_sel; base += kSelBlock) {
    const int k = base + tid;
    const int sz = k < n_sel ? V.size(k) : 0;
    int tot;
    const int ex = block_scan(sz, sh, &tot);
    if (k < n_sel) V.set_size(k, total + ex);  // exclusive offset of move k's routes
    total += tot;
  }
  __syncthreads();
  const bool in_place = (int64_t)top + total <= U.cap;
  int rb_alive = 0;  // alive routes after a relayout (the routes the rebuild visits)
  if (in_place) {
    for (int k = tid; k < n_sel; k += kSelBlock) {
      int at = top + V.size(k);
      for (int w = 0; w < 2; ++w) {
        int slot, len, st, en;
        if (V.in_lds(k)) {
          RouteRec& r = P.rr[2 * k + w];
          if (r.len < 0) continue;
          slot = r.slot; len = r.len; st = r.start; en = r.end;
          r.off = at;
        } else {
          slot = U.sel_slot[2 * k + w];
          if (slot < 0) continue;
          len = U.r_len[slot]; st = U.r_start[slot]; en = U.r_end[slot];
        }
        if (len > 0) {
          U.r_off[cur][slot] = at;
          U.r_meta[cur][slot] = make_int4(at, len, st, en);
          if (!V.in_lds(k)) U.build_list[atomicAdd(&s_nbuild, 1)] = slot;
          at += len + 2;
        } else {
          U.r_meta[cur][slot] = make_int4(0, 0, -1, -1);
          s_alive_changed = 1;
        }
      }
      if ((V.id(k) >> 56) == DINS) s_alive_changed = 1;  // a route in a slot that was empty
    }
    __syncthreads();
    if (s_alive_changed) {
      int alive_carry = 0;
      for (int base = 0; base < U.R; base += kSelBlock) {
        const int s = base + tid;
        const int alive = s < U.R && U.r_len[s] > 0 ? 1 : 0;
        int tot;
        const int ax = block_scan(alive, sh, &tot);
        if (alive) U.slot_list[alive_carry + ax] = s;
        alive_carry += tot;
      }
      if (tid == 0) ctl->n_slots_alive = alive_carry;
    }
    if (tid == 0) {
      ctl->arena_top = top + total;
      ctl->rebuild_mode = 0;
      ctl->n_build = s_nbuild;
    }
  } else {
    const int dst = cur ^ 1;
    int carry = 0, alive_carry = 0;  // (alive_carry ends equal in every thread)
    for (int base = 0; base < U.R; base += kSelBlock) {
      const int s = base + tid;
      const int len = s < U.R ? U.r_len[s] : 0;
      const int size = len > 0 ? len + 2 : 0;
      int tot, tot2;
      const int ex = block_scan(size, sh, &tot);
      const int ax = block_scan(len > 0 ? 1 : 0, sh, &tot2);
      if (s < U.R) {
        U.r_off[dst][s] = carry + ex;
        U.r_meta[dst][s] = make_int4(carry + ex, len, len > 0 ? U.r_start[s] : -1, len > 0 ? U.r_end[s] : -1);
        if (len > 0) U.slot_list[alive_carry + ax] = s;
      }
      carry += tot;
      alive_carry += tot2;
    }
    rb_alive = alive_carry;
    if (tid == 0) {
      if (carry > U.cap) atomicOr(&ctl->err, 2);
      ctl->n_slots_alive = alive_carry;
      ctl->cur = dst;
      ctl->arena_top = carry;
      ctl->rebuild_mode = 1;
      ctl->n_build = 0;
    }
  }
  if (tid == 0) {
    ctl->F += (int64_t)P.F;
    ctl->n_sel = n_sel;
    ctl->moves_applied += n_sel;
    ctl->pass_applied = 1;
    ctl->n_cand = 0;
  }
  if constexpr (APPLY) {
    __syncthreads();
    // the recorded routes (one wavefront each), then whatever the unit's plan arrays
    // hold: copies of untouched routes in a relayout, routes of moves beyond kPlanLds
    const int n_rec = 2 * imin(n_sel, kPlanLds);
    const int src = cur;  // the old routes live in the buffer that was current before this step
    const int dst = in_place ? cur : cur ^ 1;
    // routes of at most 32 positions (most of them): one per half-wavefront, two at a
    // time per wavefront; the longer ones: one per wavefront
    const int half = lane >> 5;
    for (int r = 2 * wave + half; r < n_rec; r += 2 * kSelWaves) {
      RouteRec rec = P.rr[r];
      if (rec.len <= 0 || (OPEN ? rec.len + 1 : rec.len + 2) > 32) continue;
      if (!in_place) rec.off = U.r_off[dst][rec.slot];
      build_recorded_route<SEG, TW, OPEN, 32>(U, rec, src, dst);
    }
    for (int r = wave; r < n_rec; r += kSelWaves) {
      RouteRec rec = P.rr[r];
      if (rec.len <= 0 || (OPEN ? rec.len + 1 : rec.len + 2) <= 32) continue;
      if (!in_place) rec.off = U.r_off[dst][rec.slot];
      build_recorded_route<SEG, TW, OPEN>(U, rec, src, dst);
    }
    // (mode, buffer, epoch and counts from this step's own values: no reload of the
    // control block)
    rebuild_items<SEG, TW, OPEN>(U, in_place, dst, epoch, in_place ? s_nbuild : rb_alive, wave, kSelWaves);
    if (adapt_units) {
      __syncthreads();
      adapt_weights<OPEN>(U, ctl, adapt_units + blockIdx.x, adapt, &s_viol);
    }
  }
}

template <class SEG, bool TW, bool OPEN, bool APPLY>
static void select_t(const LaunchCtx& L, uint32_t cls, int leader_only, int scored) {
  UnitDesc* au = APPLY ? L.adapt_units : nullptr;
  if (L.max_nd <= kDepLds)
    hipLaunchKernelGGL((k_select_plan<SEG, TW, OPEN, APPLY, true>), dim3(L.n_units), dim3(kSelBlock), 0, L.stream,
                       L.units, cls, leader_only, scored, au, L.adapt);
  else
    hipLaunchKernelGGL((k_select_plan<SEG, TW, OPEN, APPLY, false>), dim3(L.n_units), dim3(kSelBlock), 0, L.stream,
                       L.units, cls, leader_only, scored, au, L.adapt);
}

void launch_select(const LaunchCtx& L, uint32_t fam_mask, int leader_only, int scored, bool apply) {
  const uint32_t cls = eval_classes(L, fam_mask);
  if (!apply) {
    if (L.open) select_t<SegNT, false, true, false>(L, cls, leader_only, scored);
    else select_t<SegNT, false, false, false>(L, cls, leader_only, scored);
  } else if (L.has_tw) {
    if (L.open) select_t<SegTW, true, true, true>(L, cls, leader_only, scored);
    else select_t<SegTW, true, false, true>(L, cls, leader_only, scored);
  } else {
    if (L.open) select_t<SegNT, false, true, true>(L, cls, leader_only, scored);
    else select_t<SegNT, false, false, true>(L, cls, leader_only, scored);
  }
}

}  // namespace mdvrp
