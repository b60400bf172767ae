// eval.hip -- parallel evaluation of every move of the selected operator families.
//
// One thread per item: an anchor pair (u, v in N(u)) for Relocate / Swap /
// 2-opt* / 2-opt, or (customer, depot) for the depot operators (Section 3.2.2).
// Inter-route anchors go through the specialised prefix/suffix evaluator;
// intra-route anchors are packed into a block-level queue so that their
// (longer) evaluation occupies as few wavefronts as possible. Each block
// belongs to one unit and writes
//   * its best improving move by (dF, id) -> the step's leader candidate;
//   * the follower-eligible moves (dD < 0, no penalty term changes; Section
//     3.2.5), reduced per resource set inside the item, appended to the
//     unit's candidate list with one atomic per wavefront;
//   * the number of evaluated moves.
#include <type_traits>

#include "eval_common.h"
#include "kernels.h"

namespace mdvrp {

// Per-thread results. Follower candidates are reduced per resource set; an
// item has at most three distinct sets: {A, B} (or {A}), {A, B, depot of A},
// {A, B, depot of B}. Slot z holds the best (packed) key of set z.
struct ItemOut {
  int64_t bF;
  uint64_t bid;
  int32_t b_dD, b_elig;
  int32_t b_res0, b_res1, b_res2;
  uint64_t k0, k1, k2;
  uint64_t i0, i1, i2;
  uint64_t r0, r1, r2;  // resource sets, packed by pack_res
  int32_t evaluated;  // moves evaluated by this thread in this launch
  int32_t err;        // error bits, posted once by the block epilogue (no store inside the
                      // evaluation, so repeated matrix and segment loads can be merged)
};

__device__ __forceinline__ void item_init(ItemOut& o) {
  o.bF = kNoMove;
  o.bid = ~0ull;
  o.b_dD = 0; o.b_elig = 0; o.b_res0 = o.b_res1 = o.b_res2 = -1;
  o.k0 = o.k1 = o.k2 = ~0ull;
  o.evaluated = 0;
  o.err = 0;
}

// The (up to) three resources of a move in one word: 21 bits each, holding id + 1
// (0 = none); resource ids are below R + nd = N <= 65535. (Two registers per slot of
// the thread's follower bookkeeping instead of four.)
__device__ __forceinline__ uint64_t pack_res(const MoveEval& m) {
  return (uint64_t)(uint32_t)(m.res[0] + 1) | (uint64_t)(uint32_t)(m.res[1] + 1) << 21 |
         (uint64_t)(uint32_t)(m.res[2] + 1) << 42;
}
__device__ __forceinline__ int4 unpack_res(uint64_t p) {
  return make_int4((int)(p & 0x1fffff) - 1, (int)((p >> 21) & 0x1fffff) - 1, (int)((p >> 42) & 0x1fffff) - 1, 0);
}

__device__ __forceinline__ void item_take(const UnitDesc& U, ItemOut& o, const MoveEval& m, uint64_t id) {
  o.evaluated += 1;
  if (m.dF < 0 && key_less(m.dF, id, o.bF, o.bid)) {
    o.bF = m.dF;
    o.bid = id;
    o.b_dD = m.dD;
    o.b_elig = follower(m);
    o.b_res0 = m.res[0]; o.b_res1 = m.res[1]; o.b_res2 = m.res[2];
  }
  if (follower(m)) {
    const uint64_t key = pack_key(U, m.dD, id);
    const uint64_t r = pack_res(m);
    if (o.k0 == ~0ull || o.r0 == r) {
      if (key < o.k0) { o.k0 = key; o.i0 = id; o.r0 = r; }
    } else if (o.k1 == ~0ull || o.r1 == r) {
      if (key < o.k1) { o.k1 = key; o.i1 = id; o.r1 = r; }
    } else if (o.k2 == ~0ull || o.r2 == r) {
      if (key < o.k2) { o.k2 = key; o.i2 = id; o.r2 = r; }
    } else {
      o.err |= 8;
    }
  }
}

__device__ __forceinline__ void dense_put(const DenseOut& D, int unit, const MoveEval& m, uint64_t id) {
  const unsigned long long k = atomicAdd(D.count, 1ull);
  if ((int64_t)k >= D.cap) return;
  DenseRec r;
  r.dF = m.dF; r.dD = m.dD; r.dTW = m.dTW; r.dLX = m.dLX; r.dDX = m.dDX; r.dV4 = m.dV4;
  r.id = id; r.unit = unit;
  r.res[0] = m.res[0]; r.res[1] = m.res[1]; r.res[2] = m.res[2];
  D.rec[k] = r;
}

// Append an improving move to the compacted list (one atomic per wavefront: the
// compiler aggregates the same-address increments of the active lanes).
__device__ __forceinline__ void move_put(const MoveList& M, int unit, const MoveEval& m, uint64_t id) {
  const unsigned long long k = atomicAdd(M.count, 1ull);
  if ((int64_t)k >= M.cap) return;
  M.dF[k] = m.dF;
  M.dD[k] = m.dD;
  M.id[k] = id;
  M.kind[k] = (uint8_t)(id >> 56);
  M.variant[k] = (uint8_t)(id >> 48);
  M.changed[k] = (uint8_t)((m.dTW != 0) | (m.dLX != 0) << 1 | (m.dDX != 0) << 2 | (m.dV4 != 0) << 3);
  M.unit[k] = unit;
  M.a[k] = (int32_t)((id >> 24) & 0xffffff);
  M.b[k] = (int32_t)(id & 0xffffff);
  M.res[3 * k] = m.res[0];
  M.res[3 * k + 1] = m.res[1];
  M.res[3 * k + 2] = m.res[2];
}

// Result sink of the evaluators: leader/follower bookkeeping plus, by mode SM,
// nothing (0), the dense record of every evaluated move and / or the list of the
// improving ones (1), or the anchor's improving flag (2: label[item] = 1 when some
// move of the anchor has dF < 0).
template <int SM>
struct Sink {
  ItemOut* o;
  DenseOut d;
  int unit;
  int64_t item;
};

template <int SM>
__device__ __forceinline__ void take(const UnitDesc& U, Sink<SM>& s, const MoveEval& m, uint64_t id) {
  item_take(U, *s.o, m, id);
  if constexpr (SM == 1) {
    if (s.d.rec) dense_put(s.d, s.unit, m, id);
    if (s.d.ml.count && m.dF < 0) move_put(s.d.ml, s.unit, m, id);
  }
  if constexpr (SM == 2) {
    if (m.dF < 0) s.d.label[U.item_base + s.item] = 1;
  }
}

}  // namespace mdvrp

#include "eval_inter.h"
#include "eval_intra.h"

namespace mdvrp {

__device__ __forceinline__ void cand_put(const UnitDesc& U, int at, uint64_t k, uint64_t id, uint64_t r) {
  if (at < U.cand_cap) {
    U.cand_key[at] = k;
    U.cand_id[at] = id;
    U.cand_res[at] = unpack_res(r);
  } else {
    atomicOr(&U.ctl->err, 1);
  }
}

// Append this wave's follower candidates with one atomic per wavefront.
__device__ __forceinline__ void cand_flush(const UnitDesc& U, ItemOut& o) {
  const int lane = lane_id();
  const int n = (o.k0 != ~0ull) + (o.k1 != ~0ull) + (o.k2 != ~0ull);
  int incl = n;
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(incl, off);
    if (lane >= off) incl += y;
  }
  const int total = __shfl(incl, 63);
  if (total == 0) return;
  int base = 0;
  if (lane == 63) base = atomicAdd(&U.ctl->n_cand, total);
  base = __shfl(base, 63);
  int at = base + incl - n;
  if (o.k0 != ~0ull) cand_put(U, at++, o.k0, o.i0, o.r0);
  if (o.k1 != ~0ull) cand_put(U, at++, o.k1, o.i1, o.r1);
  if (o.k2 != ~0ull) cand_put(U, at++, o.k2, o.i2, o.r2);
  o.k0 = o.k1 = o.k2 = ~0ull;
}

// Block-level epilogue: candidate append, leader reduction, evaluated count.
template <int TPB>
__device__ __forceinline__ void item_flush(const UnitDesc& U, int wg_slot, ItemOut& o) {
  __shared__ int64_t sF[TPB / 64];
  __shared__ uint64_t sI[TPB / 64];
  __shared__ int sLane[TPB / 64];
  __shared__ unsigned long long sEval;
  const int lane = lane_id();
  const int wave = threadIdx.x >> 6;
  cand_flush(U, o);
  if (o.err) atomicOr(&U.ctl->err, o.err);
  if (threadIdx.x == 0) sEval = 0;
  int64_t f = o.bF;
  uint64_t id = o.bid;
  int src = threadIdx.x;
  for (int off = 32; off > 0; off >>= 1) {
    const int64_t f2 = __shfl_xor(f, off);
    const uint64_t i2 = __shfl_xor(id, off);
    const int s2 = __shfl_xor(src, off);
    if (key_less(f2, i2, f, id)) { f = f2; id = i2; src = s2; }
  }
  unsigned long long ev = (unsigned long long)o.evaluated;
  for (int off = 32; off > 0; off >>= 1) ev += __shfl_xor(ev, off);
  __syncthreads();
  if (lane == 0) {
    sF[wave] = f; sI[wave] = id; sLane[wave] = src;
    atomicAdd(&sEval, ev);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t bf = sF[0];
    uint64_t bi = sI[0];
    int bs = sLane[0];
    for (int w = 1; w < TPB / 64; ++w)
      if (key_less(sF[w], sI[w], bf, bi)) { bf = sF[w]; bi = sI[w]; bs = sLane[w]; }
    sLane[0] = bs;
    atomicAdd((unsigned long long*)&U.ctl->evaluated, sEval);
    atomicAdd((unsigned long long*)&U.ctl->last_eval, sEval);
  }
  __syncthreads();
  if ((int)threadIdx.x == sLane[0]) {
    MoveRec r;
    r.dF = o.bF;
    r.id = o.bid;
    r.dD = o.b_dD;
    r.elig = o.b_elig;
    r.res[0] = o.b_res0; r.res[1] = o.b_res1; r.res[2] = o.b_res2;
    r.pad = 0;
    U.wg_best[wg_slot] = r;
  }
}

// --------------------------------------------------------------------------- pair kinds

constexpr uint32_t kRelKinds = (1u << REL1) | (1u << REL2);
constexpr uint32_t kSwpKinds = (1u << SWP11) | (1u << SWP21) | (1u << SWP12) | (1u << SWP22);
constexpr uint32_t kX2Kinds = 1u << X2;
constexpr uint32_t k2optKinds = 1u << TWOOPT;

// Waves per SIMD the compiler must fit a pair kernel into (1: as many as its registers
// allow). The kernels wait on gathers most of their time, so a wave more per SIMD hides
// more of that wait. In 64-thread tiles the t-free Swap kernel needs 140 VGPRs and the
// time-window Relocate kernel 132 (3 waves each); held to 128 (4 waves) they keep a few
// values in scratch, and the searches are 1.7 % (without time windows) and 1.7-2.5 %
// (with) faster. (The time-window Swap kernel held to 4 waves spills far more and is
// 2.6 % slower; a fifth wave for Relocate or 2-opt* without time windows gained nothing.)
template <bool TW, uint32_t KM, int TPB, class AR>
constexpr int pair_min_waves() {
  if (TPB != 64) return 1;
  if (KM == kSwpKinds && !TW && AR::kTisC) return 4;
  if (KM == kRelKinds && TW) return 4;
  return 1;
}

// The same for the compact kernel of filtered searches, whose per-unit tile loop costs
// registers: its Swap kernel would need 169-170 VGPRs (2 waves per SIMD) and is held to
// 168 (3 waves; 2 values in scratch). Together with the changes of the same build the
// network-filtered search at k = 8 went from 1.96 to 1.84 s; holding the time-window
// Relocate kernel to 4 waves as well (23 values in scratch) gained nothing more.
template <bool TW, uint32_t KM, int TPB>
constexpr int compact_min_waves() {
  return (TPB <= 128 && KM == kSwpKinds) ? 3 : 1;
}

// One tile of pair anchors of unit ui (local tile lt of its item space: the filtered
// lists when the unit is in filtered mode, else the granular lists).
template <class SEG, bool TW, bool OPEN, int SM, class AR, int TPB>
__device__ __forceinline__ void pairs_tile(const UnitDesc& U, int ui, int lt, bool filt, uint32_t kind_mask,
                                           const DenseOut& dense) {
  constexpr int IPT = kTileSize / TPB;
  __shared__ int s_q[kTileSize];
  __shared__ int s_nq;
  const int th = filt ? U.kc : U.theta;
  const int32_t* lists = filt ? U.fcand : U.nbr;
  const int cur = U.ctl->cur;
  const SEG* fw = (const SEG*)U.fw[cur];
  const SEG* bw = (const SEG*)U.bw[cur];
  ItemOut o;
  item_init(o);
  Sink<SM> sk{&o, dense, ui, 0};
  AR ar;
  if constexpr (sizeof(AR) > 1) ar.bits = U.foot;
  if (threadIdx.x == 0) {
    s_nq = 0;
    // the selection scans the block bests of the tiles this evaluation covered; the lists
    // (and so their tile count) may be a caller's, valid for this evaluation only
    if (filt && lt == 0) U.ctl->ftiles_eval = U.ftiles;
  }
  __syncthreads();
  const uint32_t intra_kinds = kind_mask & ~(1u << X2);
  const uint32_t inter_kinds = kind_mask & ~(1u << TWOOPT);
#pragma unroll 1
  for (int r = 0; r < IPT; ++r) {
    // tiles walk the customers in layout order (neighbouring customers share cache lines)
    const int pos = lt * kTileSize + r * TPB + threadIdx.x;
    if (pos < U.nc * th) {
      const int ri = pos / th;
      const int k = pos - ri * th;
      const int i = U.corder ? ld(U.corder, ri) : ri;
      const int item = i * th + k;
      const int v = ld(lists, item);
      if ((filt || k < ld(U.nbr_len, i)) && v >= 0) {
        const int u = U.nd + i;
        const int sa = ld(U.rt, u), sb = ld(U.rt, v);
        if (sa != sb) {
          if (inter_kinds) {
            if constexpr (SM == 2) sk.item = item;
            const int4 ma = ld(U.r_meta[cur], sa), mb = ld(U.r_meta[cur], sb);
            InterCtx x;
            x.u = u; x.v = v; x.slotA = sa; x.slotB = sb;
            x.LA = ma.y; x.LB = mb.y;
            x.sA = ma.z; x.sB = mb.z;
            x.eA = ma.w; x.eB = mb.w;
            x.au = ld(U.apos, u); x.av = ld(U.apos, v);
            x.pu = x.au - ma.x; x.pv = x.av - mb.x;
            // the arc u -> v every pair move creates: with time windows, from the slot's
            // cache on the granular lists of instances in the locality layout (instead of a
            // gather through the layout's permutation; loaded with the other arcs, so that
            // it holds no register longer than they do); otherwise from the matrix: on the
            // filtered lists, on cache-resident matrices (where the gather is cheaper than
            // the extra load: 1.4 % on 8 x 1000), and without time windows (where the Swap
            // kernel, held to 128 VGPRs, would keep more values in scratch)
            x.uv_item = (TW && !filt && U.pi) ? item : -1;
            eval_inter<SEG, TW, OPEN>(U, fw, bw, ma.x, mb.x, x, inter_kinds, ar, sk);
          }
        } else if (intra_kinds) {
          s_q[atomicAdd(&s_nq, 1)] = item;
        }
      }
    }
    cand_flush(U, o);
  }
  __syncthreads();
  // intra-route anchors of the block, packed into as few wavefronts as possible
  const int nq = s_nq;
  for (int e0 = 0; e0 < nq; e0 += TPB) {
    const int e = e0 + threadIdx.x;
    if (e < nq) {
      const int it = s_q[e];
      const int i = it / th;
      const int u = U.nd + i, v = ld(lists, it);
      if constexpr (SM == 2) sk.item = it;
      const RouteCtx A = route_ctx(U, cur, ld(U.rt, u));
      eval_intra<SEG, TW, OPEN>(U, fw, bw, A, u, v, ld(U.pos, u), ld(U.pos, v), intra_kinds, ar, sk);
    }
    cand_flush(U, o);
  }
  item_flush<TPB>(U, U.tile_base[0] + lt, o);
}


// KM != 0 fixes the kind mask at compile time (one lean kernel per family);
// KM == 0 takes it from the argument. A tile is kTileSize items; a block of TPB
// threads covers it with kTileSize / TPB items per thread (the tile shape the
// autotuner picks; results do not depend on it). One block per tile of the
// granular lists.
template <class SEG, bool TW, bool OPEN, int SM, class AR, uint32_t KM, int TPB>
__global__ __launch_bounds__(TPB, (pair_min_waves<TW, KM, TPB, AR>())) void k_eval_pairs(const UnitDesc* __restrict__ units,
                                                   const int32_t* __restrict__ tile_off, int n_units, int per_unit,
                                                   uint32_t kind_arg, DenseOut dense,
                                                   const int32_t* __restrict__ act) {
  const uint32_t kind_mask = KM ? KM : kind_arg;
  // In a pass of the search (act) the first blocks take the active units' tiles, one
  // each, and the others have none; otherwise every block takes the tile of its index.
  const GridView gv = grid_view(act, n_units, 0, tile_off);
  const int t = block_tile(gv.T);
  if (t < 0) return;
  int ui, lt;
  map_tile(gv.off, gv.n, per_unit, gv.list, t, ui, lt);
  const UnitDesc& U = units[ui];
  if (!act && !U.ctl->active) return;  // every unit of the map is active
  // A unit in filtered mode has ftiles tiles: they are spread evenly over its full tile
  // range (every XCD gets its share); the other tiles have nothing to do. (A unit has at
  // most 65535 * 128 / 256 tiles, so the products fit 32 bits.)
  const bool filt = U.ctl->fmode == 1;
  if (filt) {
    const uint32_t full = (uint32_t)(U.tile_base[1] - U.tile_base[0]), ft = (uint32_t)U.ftiles;
    const int f = (int)((uint32_t)lt * ft / full);
    if (lt > 0 && f == (int)((uint32_t)(lt - 1) * ft / full)) return;
    lt = f;
  }
  pairs_tile<SEG, TW, OPEN, SM, AR, TPB>(U, ui, lt, filt, kind_mask, dense);
}

// The same evaluation on a compact grid of as many blocks per unit as its filtered
// lists have tiles (searches with a filter): a block of a unit in filtered mode
// takes one tile, a block of a unit evaluating its full lists loops over every
// blocks-per-unit-th tile.
template <class SEG, bool TW, bool OPEN, uint32_t KM, int TPB>
__global__ __launch_bounds__(TPB, (compact_min_waves<TW, KM, TPB>())) void k_eval_pairs_compact(const UnitDesc* __restrict__ units,
                                                           const int32_t* __restrict__ grid_off, int n_units,
                                                           int per_unit, uint32_t kind_arg,
                                                           const int32_t* __restrict__ act) {
  const uint32_t kind_mask = KM ? KM : kind_arg;
  const GridView gv = grid_view(act, n_units, 3, grid_off);
  const int t = block_tile(gv.T);
  if (t < 0) return;
  int ui, g;
  map_tile(gv.off, gv.n, per_unit, gv.list, t, ui, g);
  const UnitDesc& U = units[ui];
  if (!act && !U.ctl->active) return;
  const bool filt = U.ctl->fmode == 1;
  const int G = per_unit > 0 ? per_unit : grid_off[ui + 1] - grid_off[ui];
  const int T = filt ? U.ftiles : U.tile_base[1] - U.tile_base[0];
  for (int lt = g; lt < T; lt += G) {
    __syncthreads();
    pairs_tile<SEG, TW, OPEN, 0, ArcPlain, TPB>(U, ui, lt, filt, kind_mask, DenseOut{});
  }
}

// --------------------------------------------------------------------------- depot operators

// One tile of depot-operator items of unit ui: (customer, depot) pairs for
// Depot-Insert (which = 0), (alive route, depot) pairs for Depot-Replace (which = 1).
template <class SEG, bool TW, bool OPEN, int SM, class AR, int TPB>
__device__ __forceinline__ void depot_tile(const UnitDesc& U, int ui, int lt, int which, int n_drep,
                                           const DenseOut& dense) {
  constexpr int IPT = kTileSize / TPB;
  const int cur = U.ctl->cur;
  const SEG* fw = (const SEG*)U.fw[cur];
  const SEG* bw = (const SEG*)U.bw[cur];
  ItemOut o;
  item_init(o);
  Sink<SM> sk{&o, dense, ui, 0};
  AR ar;
  if constexpr (sizeof(AR) > 1) ar.bits = U.foot;
  MoveEval m;
#pragma unroll 1
  for (int r = 0; r < IPT; ++r) {
  const int item = lt * kTileSize + r * TPB + threadIdx.x;
  if (which == 0) {
    // Depot-Insert: one item per (customer u, depot d); cut after u when s(u) is a customer.
    if (item < U.nc * U.nd) {
      const int ri = item / U.nd;
      const int d = item - ri * U.nd;
      const int u = U.nd + (U.corder ? ld(U.corder, ri) : ri);
      const RouteCtx A = route_ctx(U, cur, ld(U.rt, u));
      const int pu = ld(U.pos, u);
      if (pu < A.L) {
        eval_dins<SEG, TW, OPEN>(U, fw, bw, A, pu, d, ar, m);
        take(U, sk, m, make_id(DINS, 0, u, d));
      }
    }
  } else if (item < n_drep) {
    // Depot-Replace: one item per (alive route, depot), the best surviving case.
    const int d = item % U.nd;
    const RouteCtx A = route_ctx(U, cur, ld(U.slot_list, item / U.nd));
    const int u = ld(fw, A.off + 1).node;
    bool have = false;
    MoveEval best;
    int bcase = 0;
    for (int cs = 0; cs < 3; ++cs) {
      if (OPEN && cs != 0) continue;
      const int ns = (cs == 0 || cs == 2) ? d : A.start;
      const int ne = (cs == 1 || cs == 2) ? d : A.end;
      if (ns == A.start && ne == A.end) continue;
      bool dup = false;
      for (int c2 = 0; c2 < cs; ++c2) {
        const int s2 = (c2 == 0 || c2 == 2) ? d : A.start;
        const int e2 = (c2 == 1 || c2 == 2) ? d : A.end;
        if (!(s2 == A.start && e2 == A.end) && s2 == ns && e2 == ne) dup = true;
      }
      if (dup) continue;
      eval_drep<SEG, TW, OPEN>(U, fw, bw, A, d, cs, ar, m);
      if (!have || m.dF < best.dF) { best = m; bcase = cs; have = true; }
    }
    if (have) take(U, sk, best, make_id(DREP, bcase, u, d));
  }
  cand_flush(U, o);
  }
  item_flush<TPB>(U, U.tile_base[1 + which] + lt, o);
}


// One block per tile of the class's full item space.
template <class SEG, bool TW, bool OPEN, int SM, class AR, int TPB>
__global__ __launch_bounds__(TPB) void k_eval_depot(const UnitDesc* __restrict__ units,
                                                   const int32_t* __restrict__ tile_off, int n_units, int per_unit,
                                                   int which, DenseOut dense, const int32_t* __restrict__ act) {
  const GridView gv = grid_view(act, n_units, 1 + which, tile_off);
  const int t = block_tile(gv.T);
  if (t < 0) return;
  int ui, lt;
  map_tile(gv.off, gv.n, per_unit, gv.list, t, ui, lt);
  const UnitDesc& U = units[ui];
  if (!act && !U.ctl->active) return;
  // Depot-Replace items cover the alive routes only; the tiles beyond them have
  // nothing to do (the selection reads as many tiles as the items need).
  const int n_drep = which == 1 ? U.ctl->n_slots_alive * U.nd : 0;
  if (which == 1 && lt * kTileSize >= n_drep) return;
  depot_tile<SEG, TW, OPEN, SM, AR, TPB>(U, ui, lt, which, n_drep, dense);
}

// Depot-Replace on a compact grid sized for the routes a solution is expected to hold;
// each block loops over every blocks-per-unit-th tile of the alive routes.
template <class SEG, bool TW, bool OPEN, int TPB>
__global__ __launch_bounds__(TPB) void k_eval_drep_compact(const UnitDesc* __restrict__ units,
                                                          const int32_t* __restrict__ grid_off, int n_units,
                                                          int per_unit, const int32_t* __restrict__ act) {
  const GridView gv = grid_view(act, n_units, 4, grid_off);
  const int t = block_tile(gv.T);
  if (t < 0) return;
  int ui, g;
  map_tile(gv.off, gv.n, per_unit, gv.list, t, ui, g);
  const UnitDesc& U = units[ui];
  if (!act && !U.ctl->active) return;
  const int G = per_unit > 0 ? per_unit : grid_off[ui + 1] - grid_off[ui];
  const int n_drep = U.ctl->n_slots_alive * U.nd;
  for (int lt = g; lt * kTileSize < n_drep; lt += G) {
    __syncthreads();
    depot_tile<SEG, TW, OPEN, 0, ArcPlain, TPB>(U, ui, lt, 1, n_drep, DenseOut{});
  }
}

// --------------------------------------------------------------------------- launchers

static uint32_t pair_kinds(uint32_t fam_mask, int has_tw) {
  uint32_t kinds = 0;
  if (fam_mask >> FAM_REL & 1) kinds |= (1u << REL1) | (1u << REL2);
  if (fam_mask >> FAM_SWP & 1) kinds |= (1u << SWP11) | (1u << SWP21) | (1u << SWP12) | (1u << SWP22);
  if (fam_mask >> FAM_X2 & 1) kinds |= 1u << X2;
  if (!has_tw && (fam_mask >> FAM_2OPT & 1)) kinds |= 1u << TWOOPT;
  return kinds;
}

uint32_t eval_classes(const LaunchCtx& L, uint32_t fam_mask) {
  uint32_t cls = 0;
  if (pair_kinds(fam_mask, L.has_tw) && L.tiles[0] > 0) cls |= 1u;
  if ((fam_mask >> FAM_DINS & 1) && L.tiles[1] > 0) cls |= 2u;
  if ((fam_mask >> FAM_DREP & 1) && L.tiles[2] > 0) cls |= 4u;
  return cls;
}

// Blocks of a launch over grid g with T tiles in all: one per tile of every unit (in a
// pass of the search the active units' tiles, fewer, take the first blocks).
static int grid_of(const LaunchCtx&, int, int T) { return T; }


template <class SEG, bool TW, bool OPEN, int SM, class AR, uint32_t KM, int TPB>
static void launch_pairs(const LaunchCtx& L, uint32_t kinds, const DenseOut& D) {
  if constexpr (SM == 0 && std::is_same<AR, ArcPlain>::value) {
    if (L.compact && L.tiles_f > 0) {
      hipLaunchKernelGGL((k_eval_pairs_compact<SEG, TW, OPEN, KM, TPB>), dim3(grid_of(L, 3, L.tiles_f)), dim3(TPB),
                         0, L.stream, L.units, L.tile_off_f, L.n_units, L.per_unit_f, kinds, L.act);
      return;
    }
  }
  hipLaunchKernelGGL((k_eval_pairs<SEG, TW, OPEN, SM, AR, KM, TPB>), dim3(grid_of(L, 0, L.tiles[0])), dim3(TPB), 0,
                     L.stream, L.units, L.tile_off[0], L.n_units, L.per_unit[0], kinds, D, L.act);
}

template <class SEG, bool TW, bool OPEN, int SM, class AR, int TPB>
static void launch_pair_kinds(const LaunchCtx& L, uint32_t kinds, const DenseOut& D) {
  if (kinds == kRelKinds) launch_pairs<SEG, TW, OPEN, SM, AR, kRelKinds, TPB>(L, kinds, D);
  else if (kinds == kSwpKinds) launch_pairs<SEG, TW, OPEN, SM, AR, kSwpKinds, TPB>(L, kinds, D);
  else if (kinds == kX2Kinds) launch_pairs<SEG, TW, OPEN, SM, AR, kX2Kinds, TPB>(L, kinds, D);
  else if (!TW && kinds == k2optKinds) launch_pairs<SEG, TW, OPEN, SM, AR, k2optKinds, TPB>(L, kinds, D);
  else launch_pairs<SEG, TW, OPEN, SM, AR, 0u, kTileSize>(L, kinds, D);
}

template <class SEG, bool TW, bool OPEN, int SM, class AR, int TPB>
static void launch_class_t(const LaunchCtx& L, uint32_t fam_mask, int cls, const DenseOut& D) {
  if (cls == 0) {
    const uint32_t kinds = pair_kinds(fam_mask, TW);
    if (!kinds || L.tiles[0] <= 0) return;
    // without time windows, batches whose travel times are their costs take the kernels
    // that read no t entries (fewer registers: a Swap tile fits 4 waves per SIMD)
    if constexpr (!TW && SM == 0 && std::is_same<AR, ArcPlain>::value) {
      if (L.t_is_c_all && !(L.compact && L.tiles_f > 0)) {
        launch_pair_kinds<SEG, TW, OPEN, SM, ArcPlainTC, TPB>(L, kinds, D);
        return;
      }
    }
    launch_pair_kinds<SEG, TW, OPEN, SM, AR, TPB>(L, kinds, D);
    return;
  }
  const int w = cls - 1;
  if (!(fam_mask >> (FAM_DINS + w) & 1) || L.tiles[1 + w] <= 0) return;
  if constexpr (SM == 0 && std::is_same<AR, ArcPlain>::value) {
    if (w == 1 && L.tiles_r > 0) {
      hipLaunchKernelGGL((k_eval_drep_compact<SEG, TW, OPEN, TPB>), dim3(grid_of(L, 4, L.tiles_r)), dim3(TPB), 0,
                         L.stream, L.units, L.tile_off_r, L.n_units, L.per_unit_r, L.act);
      return;
    }
  }
  hipLaunchKernelGGL((k_eval_depot<SEG, TW, OPEN, SM, AR, TPB>), dim3(grid_of(L, 1 + w, L.tiles[1 + w])), dim3(TPB), 0,
                     L.stream, L.units, L.tile_off[1 + w], L.n_units, L.per_unit[1 + w], w, D, L.act);
}

template <int SM, class AR, int TPB>
static void launch_class(const LaunchCtx& L, uint32_t fam_mask, int cls, const DenseOut& D) {
  if (L.has_tw) {
    if (L.open) launch_class_t<SegTW, true, true, SM, AR, TPB>(L, fam_mask, cls, D);
    else launch_class_t<SegTW, true, false, SM, AR, TPB>(L, fam_mask, cls, D);
  } else {
    if (L.open) launch_class_t<SegNT, false, true, SM, AR, TPB>(L, fam_mask, cls, D);
    else launch_class_t<SegNT, false, false, SM, AR, TPB>(L, fam_mask, cls, D);
  }
}

// Tile shapes of the search path (threads per block; a tile is always kTileSize items).
static const int kTileShapes[kNumTileShapes] = {256, 128, 64};

int tile_shape_threads(int shape) { return kTileShapes[shape < 0 || shape >= kNumTileShapes ? 0 : shape]; }

void launch_eval_class(const LaunchCtx& L, uint32_t fam_mask, int cls, const DenseOut* dense, int shape) {
  if (dense && dense->label) {
    if (cls == 0) launch_class<2, ArcPlain, kTileSize>(L, fam_mask, cls, *dense);
  } else if (dense) {
    launch_class<1, ArcPlain, kTileSize>(L, fam_mask, cls, *dense);
  } else if (shape == 1) {
    launch_class<0, ArcPlain, 128>(L, fam_mask, cls, DenseOut{});
  } else if (shape == 2) {
    launch_class<0, ArcPlain, 64>(L, fam_mask, cls, DenseOut{});
  } else {
    launch_class<0, ArcPlain, kTileSize>(L, fam_mask, cls, DenseOut{});
  }
}

void launch_eval_footprint(const LaunchCtx& L, uint32_t fam_mask, int cls) {
  launch_class<0, ArcFoot, kTileSize>(L, fam_mask, cls, DenseOut{});
}


}  // namespace mdvrp
