// state.hip -- solution state: load, per-step rebuild, pass bookkeeping, cost, export.
//
// Routes are built by one wavefront each (rebuild.h); this file launches the
// per-step rebuild on its own grid (the apply call) and loads solutions.
#include "kernels.h"
#include "rebuild.h"

namespace mdvrp {

constexpr int kRebuildBlock = 256;
constexpr int kUnitBlock = 1024;

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
  rebuild_items<SEG, TW, OPEN>(U, ctl, lt * waves_per_block + (threadIdx.x >> 6), ntiles * waves_per_block);
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
    ctl->ftiles_eval = 0;
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
    build_route_wave<SEG, TW, OPEN>(U, 0, slot, U.r_off[0][slot], L, U.r_start[slot], OPEN ? -1 : U.r_end[slot], nodeAt);
  }
}

// --------------------------------------------------------------------------- pass bookkeeping

// Start of a pass: count it for every active unit, and (act != null) write the pass's
// active map: the active units in ascending order and the prefix offsets of their
// tiles in each grid (one block; units in chunks of its size).
struct ActSrc {
  const int32_t* off[kActGrids];  // per-unit prefix offsets of each grid over all units (null: no such grid)
};
__global__ __launch_bounds__(kUnitBlock) void k_pass_begin(const UnitDesc* __restrict__ units, int n_units,
                                                           ActSrc src, int32_t* __restrict__ act) {
  __shared__ int sh[2 * (kUnitBlock / 64) + 1];
  int base_n = 0, base[kActGrids];
  for (int g = 0; g < kActGrids; ++g) base[g] = 0;
  for (int i0 = 0; i0 < n_units; i0 += kUnitBlock) {
    const int i = i0 + (int)threadIdx.x;
    int a = 0;
    if (i < n_units) {
      UnitCtl* c = units[i].ctl;
      if (c->active) {
        c->pass_applied = 0;
        c->passes += 1;
        a = 1;
      }
    }
    if (!act) continue;  // uniform over the block
    int tot;
    const int pos = base_n + block_scan_excl<kUnitBlock>(a, sh, &tot);
    if (a) act[kActUnits + pos] = i;
    for (int g = 0; g < kActGrids; ++g) {
      const int cnt = (a && src.off[g]) ? src.off[g][i + 1] - src.off[g][i] : 0;
      int tg;
      const int o = base[g] + block_scan_excl<kUnitBlock>(cnt, sh, &tg);
      if (a) act[act_off_word(n_units, g) + pos] = o;
      base[g] += tg;
    }
    base_n += tot;
  }
  if (act && threadIdx.x == 0) {
    act[0] = base_n;
    for (int g = 0; g < kActGrids; ++g) {
      act[1 + g] = base[g];
      act[act_off_word(n_units, g) + base_n] = base[g];
    }
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

// F(S) from scratch (Eq. A.1 under the unit's current weights): the terms summed over
// the routes and depots, then weighted.
__global__ __launch_bounds__(kUnitBlock) void k_cost(const UnitDesc* __restrict__ units, int64_t* F, int64_t* terms) {
  const UnitDesc& U = units[blockIdx.x];
  __shared__ unsigned long long acc[7];
  if (threadIdx.x < 7) acc[threadIdx.x] = 0;
  __syncthreads();
  unsigned long long D = 0, TW = 0, LX = 0, DX = 0, CL = 0, FX = 0;
  for (int s = threadIdx.x; s < U.R; s += kUnitBlock) {
    if (U.r_len[s] <= 0) continue;
    const int4 t = U.r_tot[s];
    D += (unsigned long long)(int64_t)t.x;
    TW += (unsigned long long)(int64_t)t.w;
    LX += (unsigned long long)(int64_t)imax(t.y - U.Q, 0);
    DX += (unsigned long long)(int64_t)(U.Dmax >= 0 ? imax(t.z - U.Dmax, 0) : 0);
    if (U.r_end[s] >= 0 && U.r_start[s] != U.r_end[s]) CL += 1;
  }
  for (int d = threadIdx.x; d < U.nd; d += kUnitBlock) FX += (unsigned long long)imax(U.ndep[d] - U.NV, 0);
  atomicAdd(&acc[1], D); atomicAdd(&acc[2], TW); atomicAdd(&acc[3], LX);
  atomicAdd(&acc[4], DX); atomicAdd(&acc[5], CL); atomicAdd(&acc[6], FX);
  __syncthreads();
  if (threadIdx.x == 0) {
    const int64_t f = (int64_t)acc[1] + (int64_t)U.w_tw * (int64_t)acc[2] + (int64_t)U.w_load * (int64_t)acc[3] +
                      (int64_t)U.w_dur * (int64_t)acc[4] + U.w_depot * ((int64_t)acc[5] + (int64_t)acc[6]);
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
  o[12] = units[u].w_tw; o[13] = units[u].w_load; o[14] = units[u].w_dur; o[15] = units[u].w_depot;
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
  ActSrc src;
  src.off[0] = L.tile_off[0];
  src.off[1] = L.tile_off[1];
  src.off[2] = L.tile_off[2];
  src.off[3] = L.tiles_f > 0 ? L.tile_off_f : nullptr;
  src.off[4] = L.tiles_r > 0 ? L.tile_off_r : nullptr;
  hipLaunchKernelGGL(k_pass_begin, dim3(1), dim3(kUnitBlock), 0, L.stream, L.units, L.n_units, src, L.act);
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
__global__ static void k_evaluated_export(const UnitDesc* units, int n_units, int64_t* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_units) out[i] = units[i].ctl->last_eval;
}
void launch_evaluated_export(const LaunchCtx& L, int64_t* out) {
  hipLaunchKernelGGL(k_evaluated_export, dim3((L.n_units + 255) / 256), dim3(256), 0, L.stream, L.units, L.n_units,
                     out);
}
void launch_sel_export(const LaunchCtx& L, uint64_t* ids, int64_t* dF, int32_t* counts, int32_t cap) {
  hipLaunchKernelGGL(k_sel_export, dim3(L.n_units), dim3(256), 0, L.stream, L.units, L.n_units, ids, dF, counts, cap);
}
void launch_state_export(const LaunchCtx& L, int64_t* out) {
  hipLaunchKernelGGL(k_state_export, dim3((L.n_units + 255) / 256), dim3(256), 0, L.stream, L.units, L.n_units, out);
}

}  // namespace mdvrp
