// rebuild.h -- per-step rebuild of the routes a multi-move created.
//
// A route is (re)built by one wavefront: lanes own positions, the forward
// segments (start depot .. position) come from an inclusive wave scan of the
// concatenation operator and the backward segments (position .. end depot)
// from a reverse scan, 64 positions per chunk with a carried segment between
// chunks. In a full relayout the routes untouched by the step's moves are
// copied (coalesced) to their new offsets in the other buffer.
#pragma once
#include "eval_common.h"

namespace mdvrp {

template <class SEG> __device__ __forceinline__ void set_aux(SEG& s, int32_t v);
template <> __device__ __forceinline__ void set_aux<SegNT>(SegNT&, int32_t) {}
template <> __device__ __forceinline__ void set_aux<SegTW>(SegTW& s, int32_t v) { s.aux = v; }

// Build positions 0..P-1 of one route at flat offset `off` of buffer `dst`.
// nodeAt(p) returns the customer at position p (1..L). Each lane reads its own node
// once per chunk and gets its neighbours' by shuffles; a route of at most W
// positions (one chunk) reuses the forward pass's nodes, arcs and node segments in
// the backward pass.
// W = 64: the whole wavefront builds the route; W = 32: each half of the wavefront
// builds a route of its own (every shuffle stays within the half).
template <class SEG, bool TW, bool OPEN, int W = 64, class NodeFn>
__device__ __forceinline__ void build_route_wave(const UnitDesc& U, int dst, int slot, int64_t off, int L, int start, int end,
                                 NodeFn nodeAt) {
  const int lane = lane_id() & (W - 1);
  const int P = OPEN ? L + 1 : L + 2;
  SEG* fw = (SEG*)U.fw[dst];
  SEG* bw = (SEG*)U.bw[dst];
  auto node = [&](int p) -> int {
    if (p == 0) return start;
    if (p == L + 1) return end;
    return nodeAt(p);
  };
  const bool one_chunk = P <= W;
  int x1 = start;       // one chunk: this lane's node,
  int32_t c1 = 0, t1 = 0;  // the arc to the next position,
  SEG n1;               // and its node segment
  // forward scan
  SEG carry;
  int32_t carry_c = 0, carry_t = 0;
  for (int base = 0; base < P; base += W) {
    const int p = base + lane;
    const bool valid = p < P;
    const int x = valid ? node(p) : start;
    int xn = __shfl_down(x, 1, W);
    if (lane == W - 1) xn = p + 1 < P ? node(p + 1) : -1;
    if (p + 1 >= P) xn = -1;
    const int32_t oc = xn >= 0 ? arc_c(U, x, xn) : 0;
    const int32_t ot = xn >= 0 ? arc_t(U, x, xn) : 0;
    const SEG nseg = node_seg<SEG>(U, x);
    if (one_chunk) { x1 = x; c1 = oc; t1 = ot; n1 = nseg; }
    SEG seg = nseg;
    set_aux(seg, ot);
    for (int o = 1; o < W; o <<= 1) {
      const SEG l = shfl_up_seg<SEG, W>(seg, o);
      const int32_t lc = __shfl_up(oc, o, W);
      const int32_t lt = __shfl_up(ot, o, W);
      if (lane >= o) seg = cat(l, lc, lt, seg);
    }
    if (base > 0) seg = cat(carry, carry_c, carry_t, seg);
    if (valid) {
      fw[off + p] = seg;
      if (p >= 1 && p <= L) {
        U.rt[x] = slot;
        U.pos[x] = p;
        U.apos[x] = (int32_t)(off + p);
      }
      if (p == P - 1) U.r_tot[slot] = make_int4(seg.C, seg.Q, seg.D, seg_tw(seg));
    }
    const int lv = imin(W - 1, P - 1 - base);
    carry = shfl_seg<SEG, W>(seg, lv);
    carry_c = __shfl(oc, lv, W);
    carry_t = __shfl(ot, lv, W);
  }
  // time windows, one chunk: the segment of the customers alone (an inclusive scan that
  // starts at position 1), kept for Depot-Replace
  if constexpr (TW) {
    if (one_chunk && L >= 1 && L <= kCoreMaxL) {
      SEG seg = n1;
      for (int o = 1; o < W; o <<= 1) {
        const SEG l = shfl_up_seg<SEG, W>(seg, o);
        const int32_t lc = __shfl_up(c1, o, W);
        const int32_t lt = __shfl_up(t1, o, W);
        if (lane - o >= 1) seg = cat(l, lc, lt, seg);
      }
      if (lane == L) U.r_core[slot] = seg;
    }
  }
  // backward scan
  const int last_base = ((P - 1) / W) * W;
  for (int base = last_base; base >= 0; base -= W) {
    const int p = base + lane;
    const bool valid = p < P;
    int x;
    int32_t ic, it;
    SEG seg;
    if (one_chunk) {
      // the arc into position p is the forward arc out of position p - 1
      x = x1;
      ic = __shfl_up(c1, 1, W);
      it = __shfl_up(t1, 1, W);
      if (lane == 0) { ic = 0; it = 0; }
      seg = n1;
    } else {
      x = valid ? node(p) : start;
      int xp = __shfl_up(x, 1, W);
      if (lane == 0) xp = p >= 1 ? node(p - 1) : -1;
      if (!valid) xp = -1;
      ic = xp >= 0 ? arc_c(U, xp, x) : 0;
      it = xp >= 0 ? arc_t(U, xp, x) : 0;
      seg = node_seg<SEG>(U, x);
    }
    for (int o = 1; o < W; o <<= 1) {
      const SEG r = shfl_down_seg<SEG, W>(seg, o);
      const int32_t rc = __shfl_down(ic, o, W);
      const int32_t rt = __shfl_down(it, o, W);
      if (lane + o < W && p + o < P) seg = cat(seg, rc, rt, r);
    }
    if (base != last_base) seg = cat(seg, carry_c, carry_t, carry);
    seg.node = x;
    set_aux(seg, 0);
    if (valid) bw[off + p] = seg;
    carry = shfl_seg<SEG, W>(seg, 0);
    carry_c = __shfl(ic, 0, W);
    carry_t = __shfl(it, 0, W);
  }
}

// Customer at position p (1..L) of a route made of up to kMaxPieces pieces
// {old absolute offset, from, to, rev} of the old routes in fws (unrolled over the
// pieces so that they stay in registers).
template <class SEG>
__device__ __forceinline__ int piece_node(const SEG* fws, const int4 (&pc)[kMaxPieces], int np, int p) {
  int q = p, at = -1, base = 0;
#pragma unroll
  for (int j = 0; j < kMaxPieces; ++j) {
    if (j < np && at < 0) {
      const int len = pc[j].z - pc[j].y + 1;
      if (q <= len) {
        at = pc[j].w ? pc[j].z - (q - 1) : pc[j].y + (q - 1);
        base = pc[j].x;
      } else {
        q -= len;
      }
    }
  }
  return at < 0 ? -1 : ld(fws, base + at).node;
}

// Rebuild work of one step, spread over waves w0, w0 + stride, ...
// mode 0: the step's new routes were given fresh space at the end of the current
// buffer; only they are built. mode 1: full relayout into the other buffer (the
// current one after the flip): untouched routes are copied, new ones built.
// in_place: mode 0; dst: the buffer current after the step; n_items: routes to build
// (mode 0) or alive routes (mode 1).
template <class SEG, bool TW, bool OPEN>
__device__ __forceinline__ void rebuild_items(const UnitDesc& U, bool in_place, int dst, int epoch, int n_items,
                                              int w0, int stride) {
  const int src = in_place ? dst : dst ^ 1;
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
        const SEG f = fws[so + p];
        fwd[d0 + p] = f;
        bwd[d0 + p] = bws[so + p];
        if (p >= 1 && p <= L) U.apos[f.node] = (int32_t)(d0 + p);
      }
      continue;
    }
    const int np = U.plan_n[slot];
    if (np < 0) continue;  // recipe held in LDS by the fused step, which builds this route
    int4 pc[kMaxPieces];
#pragma unroll
    for (int j = 0; j < kMaxPieces; ++j)
      pc[j] = j < np ? U.plan_pc[(int64_t)slot * kMaxPieces + j] : make_int4(0, 0, -1, 0);
    auto nodeAt = [&](int p) -> int { return piece_node(fws, pc, np, p); };
    build_route_wave<SEG, TW, OPEN>(U, dst, slot, U.r_off[dst][slot], L, U.r_start[slot], OPEN ? -1 : U.r_end[slot],
                                    nodeAt);
  }
}

// The same, with the step's mode and counts read from the unit's control block.
template <class SEG, bool TW, bool OPEN>
__device__ __forceinline__ void rebuild_items(const UnitDesc& U, const UnitCtl* ctl, int w0, int stride) {
  const bool in_place = ctl->rebuild_mode == 0;
  rebuild_items<SEG, TW, OPEN>(U, in_place, ctl->cur, ctl->epoch, in_place ? ctl->n_build : ctl->n_slots_alive, w0,
                               stride);
}

// A new route of the step whose recipe is held in LDS (the fused select-and-apply
// step): its pieces {old absolute offset, from, to, rev} and where it goes.
struct RouteRec {
  int32_t slot, len, start, end;
  int32_t np, off, pad0, pad1;
  int4 pc[kMaxPieces];
};

// Build one recorded route (len > 0) at rec.off of buffer dst, reading its customers
// from the pieces of the old routes in buffer src.
template <class SEG, bool TW, bool OPEN, int W = 64>
__device__ __forceinline__ void build_recorded_route(const UnitDesc& U, const RouteRec& rec, int src, int dst) {
  const SEG* fws = (const SEG*)U.fw[src];
  const int np = rec.np;
  int4 pc[kMaxPieces];
#pragma unroll
  for (int j = 0; j < kMaxPieces; ++j) pc[j] = j < np ? rec.pc[j] : make_int4(0, 0, -1, 0);
  auto nodeAt = [&](int p) -> int { return piece_node(fws, pc, np, p); };
  build_route_wave<SEG, TW, OPEN, W>(U, dst, rec.slot, rec.off, rec.len, rec.start, OPEN ? -1 : rec.end, nodeAt);
}

}  // namespace mdvrp
