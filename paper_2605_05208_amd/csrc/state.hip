// state.hip -- solution state: load, per-step rebuild, pass bookkeeping, cost, export.
//
// A route is (re)built by one wavefront: lanes own positions, the forward
// segments (start depot .. position) come from an inclusive wave scan of the
// concatenation operator and the backward segments (position .. end depot)
// from a reverse scan, 64 positions per chunk with a carried segment between
// chunks. Routes untouched by the step's moves are copied (coalesced) to
// their new offsets in the other buffer.
#include "eval_common.h"
#include "kernels.h"

namespace mdvrp {

constexpr int kRebuildBlock = 256;
constexpr int kUnitBlock = 1024;

template <class SEG> __device__ __forceinline__ void set_aux(SEG& s, int32_t v);
template <> __device__ __forceinline__ void set_aux<SegNT>(SegNT&, int32_t) {}
template <> __device__ __forceinline__ void set_aux<SegTW>(SegTW& s, int32_t v) { s.aux = v; }

// Build positions 0..P-1 of one route at flat offset `off` of buffer `dst`.
// nodeAt(p) returns the customer at position p (1..L).
template <class SEG, bool TW, bool OPEN, class NodeFn>
__device__ void build_route_wave(const UnitDesc& U, int dst, int slot, int L, int start, int end, NodeFn nodeAt) {
  const int lane = lane_id();
  const int P = OPEN ? L + 1 : L + 2;
  const int64_t off = U.r_off[dst][slot];
  SEG* fw = (SEG*)U.fw[dst];
  SEG* bw = (SEG*)U.bw[dst];
  auto node = [&](int p) -> int {
    if (p == 0) return start;
    if (p == L + 1) return end;
    return nodeAt(p);
  };
  // forward scan
  SEG carry;
  int32_t carry_c = 0, carry_t = 0;
  for (int base = 0; base < P; base += 64) {
    const int p = base + lane;
    const bool valid = p < P;
    const int x = valid ? node(p) : start;
    const int xn = (p + 1 < P) ? node(p + 1) : -1;
    const int32_t oc = xn >= 0 ? arc_c(U, x, xn) : 0;
    const int32_t ot = xn >= 0 ? arc_t(U, x, xn) : 0;
    SEG seg = node_seg<SEG>(U, x);
    set_aux(seg, ot);
    for (int o = 1; o < 64; o <<= 1) {
      const SEG l = shfl_up_seg(seg, o);
      const int32_t lc = __shfl_up(oc, o);
      const int32_t lt = __shfl_up(ot, o);
      if (lane >= o) seg = cat(l, lc, lt, seg);
    }
    if (base > 0) seg = cat(carry, carry_c, carry_t, seg);
    if (valid) {
      fw[off + p] = seg;
      if (p >= 1 && p <= L) {
        U.rt[x] = slot;
        U.pos[x] = p;
      }
      if (p == P - 1) {
        const RouteTerms t = route_terms(U, seg);
        U.r_tot[slot] = make_int4(seg.C, seg.Q, seg.D, seg_tw(seg));
        U.r_cost[slot] = t.cost;
      }
    }
    const int lv = imin(63, P - 1 - base);
    carry = shfl_seg(seg, lv);
    carry_c = __shfl(oc, lv);
    carry_t = __shfl(ot, lv);
  }
  // backward scan
  const int last_base = ((P - 1) / 64) * 64;
  for (int base = last_base; base >= 0; base -= 64) {
    const int p = base + lane;
    const bool valid = p < P;
    const int x = valid ? node(p) : start;
    const int xp = (valid && p >= 1) ? node(p - 1) : -1;
    const int32_t ic = xp >= 0 ? arc_c(U, xp, x) : 0;
    const int32_t it = xp >= 0 ? arc_t(U, xp, x) : 0;
    SEG seg = node_seg<SEG>(U, x);
    for (int o = 1; o < 64; o <<= 1) {
      const SEG r = shfl_down_seg(seg, o);
      const int32_t rc = __shfl_down(ic, o);
      const int32_t rt = __shfl_down(it, o);
      if (lane + o < 64 && p + o < P) seg = cat(seg, rc, rt, r);
    }
    if (base != last_base) seg = cat(seg, carry_c, carry_t, carry);
    seg.node = x;
    set_aux(seg, 0);
    if (valid) bw[off + p] = seg;
    carry = shfl_seg(seg, 0);
    carry_c = __shfl(ic, 0);
    carry_t = __shfl(it, 0);
  }
}

// --------------------------------------------------------------------------- per-step rebuild

template <class SEG, bool TW, bool OPEN>
__global__ __launch_bounds__(kRebuildBlock) void k_rebuild(const UnitDesc* __restrict__ units,
                                                          const int32_t* __restrict__ tile_off, int n_units) {
  const int tile = blockIdx.x;
  const int ui = unit_of_tile(tile_off, n_units, tile);
  const UnitDesc& U = units[ui];
  const UnitCtl* ctl = U.ctl;
  if (!ctl->active || ctl->n_sel == 0) return;
  const int lt = tile - tile_off[ui];
  const int ntiles = tile_off[ui + 1] - tile_off[ui];
  const int waves_per_block = kRebuildBlock / 64;
  const int w0 = lt * waves_per_block + (threadIdx.x >> 6);
  const int stride = ntiles * waves_per_block;
  // mode 0: the step's new routes were given fresh space at the end of the current
  // buffer; only they are built. mode 1: full relayout into the other buffer (the
  // current one after the flip): untouched routes are copied, new ones built.
  const bool in_place = ctl->rebuild_mode == 0;
  const int dst = ctl->cur, src = in_place ? dst : dst ^ 1;
  const int epoch = ctl->epoch;
  const int n_items = in_place ? ctl->n_build : ctl->n_slots_alive;
  const SEG* fws = (const SEG*)U.fw[src];
  const SEG* bws = (const SEG*)U.bw[src];
  SEG* fwd = (SEG*)U.fw[dst];
  SEG* bwd = (SEG*)U.bw[dst];
  const int lane = lane_id();
  for (int k = w0; k < n_items; k += stride) {
    const int slot = in_place ? U.build_list[k] : U.slot_list[k];
    const int L = U.r_len[slot];
    if (!in_place && U.dirty[slot] != epoch) {
      const int P = OPEN ? L + 1 : L + 2;
      const int64_t so = U.r_off[src][slot], d0 = U.r_off[dst][slot];
      for (int p = lane; p < P; p += 64) {
        fwd[d0 + p] = fws[so + p];
        bwd[d0 + p] = bws[so + p];
      }
      continue;
    }
    const int np = U.plan_n[slot];
    int4 pc[kMaxPieces];
    int po[kMaxPieces];
    for (int j = 0; j < np; ++j) {
      pc[j] = U.plan_pc[(int64_t)slot * kMaxPieces + j];
      po[j] = pc[j].x;
    }
    auto nodeAt = [&](int p) -> int {
      int q = p;
      for (int j = 0; j < np; ++j) {
        const int len = pc[j].z - pc[j].y + 1;
        if (q <= len) {
          const int at = pc[j].w ? pc[j].z - (q - 1) : pc[j].y + (q - 1);
          return fws[po[j] + at].node;
        }
        q -= len;
      }
      return -1;
    };
    build_route_wave<SEG, TW, OPEN>(U, dst, slot, L, U.r_start[slot], OPEN ? -1 : U.r_end[slot], nodeAt);
  }
}

// --------------------------------------------------------------------------- load

// Route table, depot counts and offsets from the caller's flat routes (one block per unit).
__global__ __launch_bounds__(kUnitBlock) void k_load_table(const UnitDesc* __restrict__ units,
                                                          const int32_t* __restrict__ offs,
                                                          const int32_t* __restrict__ starts,
                                                          const int32_t* __restrict__ ends,
                                                          const int32_t* __restrict__ unit_route_off, int open) {
  const UnitDesc& U = units[blockIdx.x];
  UnitCtl* ctl = U.ctl;
  __shared__ int sh[2 * (kUnitBlock / 64) + 1];
  const int tid = threadIdx.x;
  const int g0 = unit_route_off[blockIdx.x], g1 = unit_route_off[blockIdx.x + 1];
  for (int d = tid; d < U.nd; d += kUnitBlock) U.ndep[d] = 0;
  __syncthreads();
  int carry = 0, alive_carry = 0;
  for (int base = 0; base < U.R; base += kUnitBlock) {
    const int s = base + tid;
    int len = 0;
    if (s < U.R) {
      if (s < g1 - g0) {
        const int g = g0 + s;
        len = offs[g + 1] - offs[g];
        U.r_start[s] = starts[g];
        U.r_end[s] = open ? -1 : ends[g];
        if (len > 0) atomicAdd(&U.ndep[starts[g]], 1);
      }
      U.r_len[s] = len;
      U.dirty[s] = 0;
      U.plan_n[s] = 0;
    }
    int tot1, tot2;
    const int e1 = block_scan_excl<kUnitBlock>(len > 0 ? len + 2 : 0, sh, &tot1);
    const int e2 = block_scan_excl<kUnitBlock>(len > 0 ? 1 : 0, sh, &tot2);
    if (s < U.R) {
      U.r_off[0][s] = carry + e1;
      U.r_meta[0][s] = make_int4(carry + e1, len, len > 0 ? U.r_start[s] : -1, len > 0 ? U.r_end[s] : -1);
      if (len > 0) U.slot_list[alive_carry + e2] = s;
    }
    carry += tot1;
    alive_carry += tot2;
  }
  for (int x = tid; x < U.n; x += kUnitBlock) {
    U.rt[x] = -1;
    U.pos[x] = 0;
  }
  if (tid == 0) {
    if (carry > U.cap) atomicOr(&ctl->err, 2);
    ctl->n_slots_alive = alive_carry;
    ctl->cur = 0;
    ctl->active = 1;
    ctl->pass_applied = 0;
    ctl->n_sel = 0;
    ctl->n_cand = 0;
    ctl->err = 0;
    ctl->evaluated = 0;
    ctl->passes = 0;
    ctl->steps = 0;
    ctl->moves_applied = 0;
    ctl->last_eval = 0;
    ctl->fallbacks = 0;
    ctl->fmode = 0;
    ctl->scored_epoch = -1;
    ctl->arena_top = carry;
    ctl->rebuild_mode = 1;
    ctl->n_build = 0;
  }
}

template <class SEG, bool TW, bool OPEN>
__global__ __launch_bounds__(kRebuildBlock) void k_load_routes(const UnitDesc* __restrict__ units,
                                                              const int32_t* __restrict__ tile_off, int n_units,
                                                              const int32_t* __restrict__ nodes,
                                                              const int32_t* __restrict__ offs,
                                                              const int32_t* __restrict__ unit_route_off) {
  const int tile = blockIdx.x;
  const int ui = unit_of_tile(tile_off, n_units, tile);
  const UnitDesc& U = units[ui];
  const int lt = tile - tile_off[ui];
  const int ntiles = tile_off[ui + 1] - tile_off[ui];
  const int waves_per_block = kRebuildBlock / 64;
  const int stride = ntiles * waves_per_block;
  const int n_alive = U.ctl->n_slots_alive;
  const int g0 = unit_route_off[ui];
  for (int k = lt * waves_per_block + (threadIdx.x >> 6); k < n_alive; k += stride) {
    const int slot = U.slot_list[k];
    const int g = g0 + slot;
    const int base = offs[g];
    const int L = offs[g + 1] - base;
    auto nodeAt = [&](int p) -> int { return nodes[base + p - 1]; };
    build_route_wave<SEG, TW, OPEN>(U, 0, slot, L, U.r_start[slot], OPEN ? -1 : U.r_end[slot], nodeAt);
  }
}

// --------------------------------------------------------------------------- pass bookkeeping

__global__ void k_pass_begin(const UnitDesc* __restrict__ units, int n_units) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_units) return;
  UnitCtl* c = units[i].ctl;
  if (c->active) {
    c->pass_applied = 0;
    c->passes += 1;
  }
}

__global__ void k_pass_end(const UnitDesc* __restrict__ units, int n_units, int32_t* active_count) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < n_units; i += blockDim.x) {
    UnitCtl* c = units[i].ctl;
    if (c->active) {
      c->t_end = (int64_t)wall_clock64();
      if (c->fmode == 1) {
        // filtered optimum: the next pass evaluates the full lists
        if (!c->pass_applied) {
          c->fmode = 2;
          c->fallbacks += 1;
        }
      } else if (c->fmode == 2) {
        // a full pass that improved returns to the filtered lists; one that did not ends the search
        if (c->pass_applied) c->fmode = 1;
        else c->active = 0;
      } else if (!c->pass_applied) {
        c->active = 0;
      }
    }
    if (c->active) atomicAdd(&cnt, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) *active_count = cnt;
}

// --------------------------------------------------------------------------- cost and export

// F(S) from scratch: route costs + depot weight * (closure + fleet excess) (Eq. A.1).
__global__ __launch_bounds__(kUnitBlock) void k_cost(const UnitDesc* __restrict__ units, int64_t* F, int64_t* terms) {
  const UnitDesc& U = units[blockIdx.x];
  __shared__ unsigned long long acc[7];
  if (threadIdx.x < 7) acc[threadIdx.x] = 0;
  __syncthreads();
  unsigned long long cost = 0, D = 0, TW = 0, LX = 0, DX = 0, CL = 0, FX = 0;
  for (int s = threadIdx.x; s < U.R; s += kUnitBlock) {
    if (U.r_len[s] <= 0) continue;
    const int4 t = U.r_tot[s];
    cost += (unsigned long long)U.r_cost[s];
    D += (unsigned long long)(int64_t)t.x;
    TW += (unsigned long long)(int64_t)t.w;
    LX += (unsigned long long)(int64_t)imax(t.y - U.Q, 0);
    DX += (unsigned long long)(int64_t)(U.Dmax >= 0 ? imax(t.z - U.Dmax, 0) : 0);
    if (U.r_end[s] >= 0 && U.r_start[s] != U.r_end[s]) CL += 1;
  }
  for (int d = threadIdx.x; d < U.nd; d += kUnitBlock) FX += (unsigned long long)imax(U.ndep[d] - U.NV, 0);
  atomicAdd(&acc[0], cost); atomicAdd(&acc[1], D); atomicAdd(&acc[2], TW); atomicAdd(&acc[3], LX);
  atomicAdd(&acc[4], DX); atomicAdd(&acc[5], CL); atomicAdd(&acc[6], FX);
  __syncthreads();
  if (threadIdx.x == 0) {
    const int64_t f = (int64_t)acc[0] + U.w_depot * ((int64_t)acc[5] + (int64_t)acc[6]);
    U.ctl->F = f;
    if (F) F[blockIdx.x] = f;
    if (terms)
      for (int k = 0; k < 6; ++k) terms[blockIdx.x * 6 + k] = (int64_t)acc[1 + k];
  }
}

template <class SEG, bool OPEN>
__global__ __launch_bounds__(kUnitBlock) void k_export(const UnitDesc* __restrict__ units, int32_t* nodes,
                                                      int32_t* offs, int32_t* starts, int32_t* ends, int32_t* counts,
                                                      const int32_t* node_base, const int32_t* route_base) {
  const UnitDesc& U = units[blockIdx.x];
  const int cur = U.ctl->cur;
  const SEG* fw = (const SEG*)U.fw[cur];
  const int n_alive = U.ctl->n_slots_alive;
  // routes are exported in slot-list order
  __shared__ int sh[2 * (kUnitBlock / 64) + 1];
  int nb = node_base[blockIdx.x];
  const int rb = route_base[blockIdx.x];
  for (int base = 0; base < n_alive; base += kUnitBlock) {
    const int k = base + threadIdx.x;
    const int slot = k < n_alive ? U.slot_list[k] : 0;
    const int len = k < n_alive ? U.r_len[slot] : 0;
    int tot;
    const int ex = block_scan_excl<kUnitBlock>(len, sh, &tot);
    if (k < n_alive) {
      const int o = nb + ex;
      offs[rb + k] = o;
      starts[rb + k] = U.r_start[slot];
      ends[rb + k] = OPEN ? -1 : U.r_end[slot];
      const int64_t f0 = U.r_off[cur][slot];
      for (int p = 1; p <= len; ++p) nodes[o + p - 1] = fw[f0 + p].node;
    }
    nb += tot;
  }
  if (threadIdx.x == 0) {
    counts[blockIdx.x] = n_alive;
    offs[rb + n_alive] = nb;
  }
}

__global__ void k_sel_export(const UnitDesc* __restrict__ units, int n_units, uint64_t* ids, int64_t* dF,
                             int32_t* counts, int32_t cap) {
  const int u = blockIdx.x;
  if (u >= n_units) return;
  const UnitDesc& U = units[u];
  const int n = U.ctl->active ? U.ctl->n_sel : 0;
  for (int k = threadIdx.x; k < n && k < cap; k += blockDim.x) {
    ids[(int64_t)u * cap + k] = U.sel_id[k];
    dF[(int64_t)u * cap + k] = U.sel_dF[k];
  }
  if (threadIdx.x == 0) counts[u] = n;
}

__global__ void k_state_export(const UnitDesc* __restrict__ units, int n_units, int64_t* out) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n_units) return;
  const UnitCtl* c = units[u].ctl;
  int64_t* o = out + (int64_t)u * kStateWords;
  o[0] = c->F; o[1] = c->evaluated; o[2] = c->passes; o[3] = c->steps; o[4] = c->moves_applied;
  o[5] = c->err; o[6] = c->active; o[7] = c->n_sel; o[8] = c->fallbacks; o[9] = c->fmode;
  o[10] = c->t_start; o[11] = c->t_end;
}

// --------------------------------------------------------------------------- launchers

template <class SEG, bool TW, bool OPEN>
static void rebuild_t(const LaunchCtx& L) {
  hipLaunchKernelGGL((k_rebuild<SEG, TW, OPEN>), dim3(L.tiles[3]), dim3(kRebuildBlock), 0, L.stream, L.units,
                     L.tile_off[3], L.n_units);
}
void launch_rebuild(const LaunchCtx& L) {
  if (L.has_tw) { if (L.open) rebuild_t<SegTW, true, true>(L); else rebuild_t<SegTW, true, false>(L); }
  else { if (L.open) rebuild_t<SegNT, false, true>(L); else rebuild_t<SegNT, false, false>(L); }
}

template <class SEG, bool TW, bool OPEN>
static void load_t(const LaunchCtx& L, const int32_t* nodes, const int32_t* offs, const int32_t* uro) {
  hipLaunchKernelGGL((k_load_routes<SEG, TW, OPEN>), dim3(L.tiles[3]), dim3(kRebuildBlock), 0, L.stream, L.units,
                     L.tile_off[3], L.n_units, nodes, offs, uro);
}
void launch_load(const LaunchCtx& L, const int32_t* nodes, const int32_t* offs, const int32_t* starts,
                 const int32_t* ends, const int32_t* uro) {
  hipLaunchKernelGGL(k_load_table, dim3(L.n_units), dim3(kUnitBlock), 0, L.stream, L.units, offs, starts, ends, uro,
                     L.open);
  if (L.has_tw) { if (L.open) load_t<SegTW, true, true>(L, nodes, offs, uro); else load_t<SegTW, true, false>(L, nodes, offs, uro); }
  else { if (L.open) load_t<SegNT, false, true>(L, nodes, offs, uro); else load_t<SegNT, false, false>(L, nodes, offs, uro); }
  launch_cost(L, nullptr, nullptr);
}

void launch_pass_begin(const LaunchCtx& L) {
  hipLaunchKernelGGL(k_pass_begin, dim3((L.n_units + 255) / 256), dim3(256), 0, L.stream, L.units, L.n_units);
}
void launch_pass_end(const LaunchCtx& L) {
  hipLaunchKernelGGL(k_pass_end, dim3(1), dim3(1024), 0, L.stream, L.units, L.n_units, L.active_count);
}
void launch_cost(const LaunchCtx& L, int64_t* F, int64_t* terms) {
  hipLaunchKernelGGL(k_cost, dim3(L.n_units), dim3(kUnitBlock), 0, L.stream, L.units, F, terms);
}
void launch_export(const LaunchCtx& L, int32_t* nodes, int32_t* offs, int32_t* starts, int32_t* ends, int32_t* counts,
                   const int32_t* node_base, const int32_t* route_base) {
  if (L.has_tw) {
    if (L.open) hipLaunchKernelGGL((k_export<SegTW, true>), dim3(L.n_units), dim3(kUnitBlock), 0, L.stream, L.units, nodes, offs, starts, ends, counts, node_base, route_base);
    else hipLaunchKernelGGL((k_export<SegTW, false>), dim3(L.n_units), dim3(kUnitBlock), 0, L.stream, L.units, nodes, offs, starts, ends, counts, node_base, route_base);
  } else {
    if (L.open) hipLaunchKernelGGL((k_export<SegNT, true>), dim3(L.n_units), dim3(kUnitBlock), 0, L.stream, L.units, nodes, offs, starts, ends, counts, node_base, route_base);
    else hipLaunchKernelGGL((k_export<SegNT, false>), dim3(L.n_units), dim3(kUnitBlock), 0, L.stream, L.units, nodes, offs, starts, ends, counts, node_base, route_base);
  }
}
void launch_sel_export(const LaunchCtx& L, uint64_t* ids, int64_t* dF, int32_t* counts, int32_t cap) {
  hipLaunchKernelGGL(k_sel_export, dim3(L.n_units), dim3(256), 0, L.stream, L.units, L.n_units, ids, dF, counts, cap);
}
void launch_state_export(const LaunchCtx& L, int64_t* out) {
  hipLaunchKernelGGL(k_state_export, dim3((L.n_units + 255) / 256), dim3(256), 0, L.stream, L.units, L.n_units, out);
}

}  // namespace mdvrp
