// eval.hip -- parallel evaluation of every move of the selected operator families.
//
// One thread per item: an anchor pair (u, v in N(u)) for Relocate / Swap /
// 2-opt* / 2-opt, or (customer, depot) for the depot operators (Section 3.2.2).
// Each block belongs to one unit and writes
//   * its best improving move by (dF, id) -> the step's leader candidate;
//   * the follower-eligible moves (dD < 0, no penalty term changes; Section
//     3.2.5), reduced per resource set inside the item, appended to the
//     unit's candidate list with one atomic per wavefront;
//   * the number of evaluated moves.
#include "eval_common.h"
#include "kernels.h"

namespace mdvrp {

constexpr int kEvalBlock = 256;

struct ItemOut {
  // leader candidate of this thread
  int64_t bF;
  uint64_t bid;
  MoveEval bm;
  // follower candidates, one per distinct resource set
  int nc;
  uint64_t ckey[3];
  uint64_t cid[3];
  int32_t cres[3][3];
  int64_t evaluated;
};

__device__ __forceinline__ void item_init(ItemOut& o) {
  o.bF = kNoMove;
  o.bid = ~0ull;
  o.nc = 0;
  o.evaluated = 0;
}

__device__ __forceinline__ void item_take(const UnitDesc& U, ItemOut& o, const MoveEval& m, uint64_t id) {
  o.evaluated += 1;
  if (m.dF < 0 && key_less(m.dF, id, o.bF, o.bid)) {
    o.bF = m.dF;
    o.bid = id;
    o.bm = m;
  }
  if (follower(m)) {
    const uint64_t key = pack_key(U, m.dD, id);
    for (int z = 0; z < o.nc; ++z) {
      if (o.cres[z][0] == m.res[0] && o.cres[z][1] == m.res[1] && o.cres[z][2] == m.res[2]) {
        if (key < o.ckey[z]) { o.ckey[z] = key; o.cid[z] = id; }
        return;
      }
    }
    if (o.nc < 3) {
      const int z = o.nc++;
      o.ckey[z] = key;
      o.cid[z] = id;
      o.cres[z][0] = m.res[0]; o.cres[z][1] = m.res[1]; o.cres[z][2] = m.res[2];
    } else {
      atomicOr(&U.ctl->err, 8);
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

// Block-level epilogue: leader reduction, candidate append, evaluated count.
__device__ void item_flush(const UnitDesc& U, int wg_slot, ItemOut& o) {
  __shared__ int64_t sF[kEvalBlock / 64];
  __shared__ uint64_t sI[kEvalBlock / 64];
  __shared__ int sLane[kEvalBlock / 64];
  __shared__ unsigned long long sEval;
  const int lane = lane_id();
  const int wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) sEval = 0;
  // wave-level argmin of (bF, bid)
  int64_t f = o.bF;
  uint64_t id = o.bid;
  int src = threadIdx.x;
  for (int off = 32; off > 0; off >>= 1) {
    const int64_t f2 = __shfl_xor(f, off);
    const uint64_t i2 = __shfl_xor(id, off);
    const int s2 = __shfl_xor(src, off);
    if (key_less(f2, i2, f, id)) { f = f2; id = i2; src = s2; }
  }
  // candidate append with one atomic per wave
  int n = o.nc;
  int incl = n;
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(incl, off);
    if (lane >= off) incl += y;
  }
  const int total = __shfl(incl, 63);
  int base = 0;
  if (lane == 63 && total > 0) base = atomicAdd(&U.ctl->n_cand, total);
  base = __shfl(base, 63);
  int at = base + incl - n;
  for (int z = 0; z < n; ++z, ++at) {
    if (at < U.cand_cap) {
      U.cand_key[at] = o.ckey[z];
      U.cand_id[at] = o.cid[z];
      U.cand_res[at] = make_int4(o.cres[z][0], o.cres[z][1], o.cres[z][2], 0);
    } else {
      atomicOr(&U.ctl->err, 1);
    }
  }
  // evaluated count
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
    for (int w = 1; w < kEvalBlock / 64; ++w)
      if (key_less(sF[w], sI[w], bf, bi)) { bf = sF[w]; bi = sI[w]; bs = sLane[w]; }
    sLane[0] = bs;
    sF[0] = bf;
    atomicAdd((unsigned long long*)&U.ctl->evaluated, sEval);
    atomicAdd((unsigned long long*)&U.ctl->last_eval, sEval);
  }
  __syncthreads();
  if ((int)threadIdx.x == sLane[0]) {
    MoveRec r;
    r.dF = o.bF;
    r.id = o.bid;
    if (o.bF != kNoMove) {
      r.dD = o.bm.dD;
      r.elig = follower(o.bm);
      r.res[0] = o.bm.res[0]; r.res[1] = o.bm.res[1]; r.res[2] = o.bm.res[2];
    } else {
      r.dD = 0; r.elig = 0; r.res[0] = r.res[1] = r.res[2] = -1;
    }
    r.pad = 0;
    U.wg_best[wg_slot] = r;
  }
}

// --------------------------------------------------------------------------- pair kinds

template <class SEG, bool TW, bool DENSE>
__global__ __launch_bounds__(kEvalBlock) void k_eval_pairs(const UnitDesc* __restrict__ units,
                                                          const int32_t* __restrict__ tile_off, int n_units,
                                                          uint32_t kind_mask, DenseOut dense) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int ui = unit_of_tile(tile_off, n_units, tile);
  const UnitDesc& U = units[ui];
  if (!U.ctl->active) return;
  const int lt = tile - tile_off[ui];
  const int item = lt * kEvalBlock + threadIdx.x;
  const int cur = U.ctl->cur;
  const SEG* fw = (const SEG*)U.fw[cur];
  const SEG* bw = (const SEG*)U.bw[cur];
  const bool sym = !TW;
  ItemOut o;
  item_init(o);
  if (item < U.nc * U.theta) {
    const int i = item / U.theta;
    const int k = item - i * U.theta;
    const int v = U.nbr[item];
    if (k < U.nbr_len[i] && v >= 0) {
      const int u = U.nd + i;
      RouteCtx rc[2];
      const int sa = U.rt[u], sb = U.rt[v];
      rc[0] = route_ctx(U, cur, sa);
      rc[1] = route_ctx(U, cur, sb);
      const int pu = U.pos[u], pv = U.pos[v];
      const bool intra = sa == sb;
      Recipe R;
      MoveEval m;
      for (int kind = REL1; kind <= TWOOPT; ++kind) {
        if (!(kind_mask >> kind & 1)) continue;
        for (int var = 0; var < 4; ++var) {
          if (!build_pair(kind, var, rc[0], pu, rc[1], pv, intra, sym, R)) continue;
          eval_recipe<SEG, TW>(U, fw, bw, rc, R, m);
          const uint64_t id = make_id(kind, var, u, v);
          item_take(U, o, m, id);
          if (DENSE) dense_put(dense, ui, m, id);
        }
      }
    }
  }
  item_flush(U, U.tile_base[0] + lt, o);
}

// --------------------------------------------------------------------------- depot operators

template <class SEG, bool TW, bool OPEN, bool DENSE>
__global__ __launch_bounds__(kEvalBlock) void k_eval_depot(const UnitDesc* __restrict__ units,
                                                          const int32_t* __restrict__ tile_off, int n_units,
                                                          int which, DenseOut dense) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int ui = unit_of_tile(tile_off, n_units, tile);
  const UnitDesc& U = units[ui];
  if (!U.ctl->active) return;
  const int lt = tile - tile_off[ui];
  const int item = lt * kEvalBlock + threadIdx.x;
  const int cur = U.ctl->cur;
  const SEG* fw = (const SEG*)U.fw[cur];
  const SEG* bw = (const SEG*)U.bw[cur];
  ItemOut o;
  item_init(o);
  if (item < U.nc * U.nd) {
    const int i = item / U.nd;
    const int d = item - i * U.nd;
    const int u = U.nd + i;
    RouteCtx rc[2];
    rc[0] = route_ctx(U, cur, U.rt[u]);
    const int pu = U.pos[u];
    Recipe R;
    MoveEval m;
    if (which == 0) {
      // Depot-Insert: cut after u when s(u) is a customer.
      if (pu < rc[0].L) {
        build_dins(rc[0], pu, d, OPEN, R);
        eval_recipe<SEG, TW>(U, fw, bw, rc, R, m);
        const uint64_t id = make_id(DINS, 0, u, d);
        item_take(U, o, m, id);
        if (DENSE) dense_put(dense, ui, m, id);
      }
    } else if (pu == 1) {
      // Depot-Replace on the route whose first customer is u: best surviving case.
      const RouteCtx& A = rc[0];
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
        build_drep(A, d, cs, R);
        eval_recipe<SEG, TW>(U, fw, bw, rc, R, m);
        if (!have || m.dF < best.dF) { best = m; bcase = cs; have = true; }
      }
      if (have) {
        const uint64_t id = make_id(DREP, bcase, u, d);
        item_take(U, o, best, id);
        if (DENSE) dense_put(dense, ui, best, id);
      }
    }
  }
  item_flush(U, U.tile_base[1 + which] + lt, o);
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

template <class SEG, bool TW, bool OPEN>
static void launch_eval_t(const LaunchCtx& L, uint32_t fam_mask, const DenseOut* dense) {
  const uint32_t kinds = pair_kinds(fam_mask, TW);
  DenseOut D = dense ? *dense : DenseOut{nullptr, nullptr, 0};
  if (kinds && L.tiles[0] > 0) {
    if (dense)
      hipLaunchKernelGGL((k_eval_pairs<SEG, TW, true>), dim3(L.tiles[0]), dim3(kEvalBlock), 0, L.stream, L.units,
                         L.tile_off[0], L.n_units, kinds, D);
    else
      hipLaunchKernelGGL((k_eval_pairs<SEG, TW, false>), dim3(L.tiles[0]), dim3(kEvalBlock), 0, L.stream, L.units,
                         L.tile_off[0], L.n_units, kinds, D);
  }
  for (int w = 0; w < 2; ++w) {
    if (!(fam_mask >> (FAM_DINS + w) & 1) || L.tiles[1 + w] <= 0) continue;
    if (dense)
      hipLaunchKernelGGL((k_eval_depot<SEG, TW, OPEN, true>), dim3(L.tiles[1 + w]), dim3(kEvalBlock), 0, L.stream,
                         L.units, L.tile_off[1 + w], L.n_units, w, D);
    else
      hipLaunchKernelGGL((k_eval_depot<SEG, TW, OPEN, false>), dim3(L.tiles[1 + w]), dim3(kEvalBlock), 0, L.stream,
                         L.units, L.tile_off[1 + w], L.n_units, w, D);
  }
}

void launch_eval(const LaunchCtx& L, uint32_t fam_mask, const DenseOut* dense) {
  if (L.has_tw) {
    if (L.open) launch_eval_t<SegTW, true, true>(L, fam_mask, dense);
    else launch_eval_t<SegTW, true, false>(L, fam_mask, dense);
  } else {
    if (L.open) launch_eval_t<SegNT, false, true>(L, fam_mask, dense);
    else launch_eval_t<SegNT, false, false>(L, fam_mask, dense);
  }
}

int eval_block_size() { return kEvalBlock; }

}  // namespace mdvrp
