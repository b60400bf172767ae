// eval_common.h -- cost of a move recipe from prefix/suffix segments.
//
// The penalised delta of a move (Section 3.2.1, Eq. 2 / A.1 with fixed integer
// weights) is the cost of the new routes minus the cost of the replaced ones,
// plus the depot term for route closure and fleet excess. New routes are
// assembled from the current routes' prefix segments (start depot .. k),
// suffix segments (k .. end depot), single nodes and middle ranges.
#pragma once
#include "internal.h"

namespace mdvrp {

template <class SEG>
__device__ __forceinline__ SEG seg_at(const SEG* a, int64_t i) {
  return a[i];
}

__device__ __forceinline__ int node_at(const SegNT* fw, int64_t i) { return ld(fw, i).node; }
__device__ __forceinline__ int node_at(const SegTW* fw, int64_t i) { return ld(fw, i).node; }

// Middle range [from, to] of route cx (1 <= from < to <= L) as one segment.
// Without time windows the prefix sums are invertible; with time windows the
// range is folded position by position (the concatenation has no inverse).
template <class SEG, bool TW>
__device__ __forceinline__ SEG mid_range(const UnitDesc& U, const SEG* fw, const RouteCtx& cx, int from, int to,
                                         int rev);

template <>
__device__ __forceinline__ SegNT mid_range<SegNT, false>(const UnitDesc& U, const SegNT* fw, const RouteCtx& cx,
                                                        int from, int to, int rev) {
  const SegNT a = ld(fw, cx.off + from);
  const SegNT b = ld(fw, cx.off + to);
  const SegNT p = ld(fw, cx.off + from - 1);
  SegNT r;
  r.C = b.C - a.C;
  r.Q = b.Q - p.Q;
  r.D = b.D - a.D + service(U, a.node);
  r.node = rev ? a.node : b.node;
  return r;
}

template <>
__device__ __forceinline__ SegTW mid_range<SegTW, true>(const UnitDesc& U, const SegTW* fw, const RouteCtx& cx,
                                                       int from, int to, int rev) {
  (void)rev;  // reversal only exists without time windows
  SegTW prev = ld(fw, cx.off + from);
  SegTW acc = node_seg<SegTW>(U, prev.node);
  for (int k = from + 1; k <= to; ++k) {
    const SegTW cur = ld(fw, cx.off + k);
    acc = cat(acc, cur.C - prev.C, prev.aux, node_seg<SegTW>(U, cur.node));
    prev = cur;
  }
  return acc;
}

// Matrix access policies: the plain one reads c and t; the footprint one also
// marks every entry it reads in a bitmap (measurement of the distinct matrix
// bytes a launch needs).
// kTisC: the kernel is launched only for units whose travel times are the costs, so
// a t entry is never read (and never held beside its c entry).
struct ArcPlain {
  static constexpr bool kTisC = false;
  __device__ __forceinline__ void mark(const UnitDesc&, int, int) const {}
};
struct ArcPlainTC {
  static constexpr bool kTisC = true;
  __device__ __forceinline__ void mark(const UnitDesc&, int, int) const {}
};
struct ArcFoot {
  static constexpr bool kTisC = false;
  uint32_t* bits;
  __device__ __forceinline__ void mark(const UnitDesc& U, int a, int b) const {
    const uint64_t i = (uint64_t)a * U.n + b;
    atomicOr(&bits[i >> 5], 1u << (i & 31));
  }
};

// Total segment of a new route: start depot, pieces, end depot (-1 = open).
template <class SEG, bool TW, class AR = ArcPlain>
__device__ SEG eval_route(const UnitDesc& U, const SEG* fw, const SEG* bw, const RouteCtx* rc, int start, int end,
                          const Piece* pc, int np, const AR& ar = AR()) {
  SEG acc;
  int last;
  int k = 0;
  {
    const Piece& p0 = pc[0];
    const RouteCtx& c0 = rc[p0.src];
    if (!p0.rev && p0.from == 1 && start == c0.start) {
      if (np == 1 && p0.to == c0.L && end == c0.end) {
        return ld(fw, c0.off + (end >= 0 ? c0.L + 1 : c0.L));
      }
      acc = ld(fw, c0.off + p0.to);
      last = acc.node;
      k = 1;
    } else {
      acc = node_seg<SEG>(U, start);
      last = start;
    }
  }
  for (; k < np; ++k) {
    const Piece& p = pc[k];
    const RouteCtx& cx = rc[p.src];
    const int first = p.rev ? node_at(fw, cx.off + p.to) : node_at(fw, cx.off + p.from);
    ar.mark(U, last, first);
    const int32_t cab = arc_c(U, last, first);
    const int32_t tab = TW ? arc_t(U, last, first) : ((AR::kTisC || U.t_is_c) ? cab : arc_t(U, last, first));
    if (k == np - 1 && !p.rev && p.to == cx.L && end == cx.end) {
      return cat(acc, cab, tab, ld(bw, cx.off + p.from));
    }
    if (p.from == p.to) {
      acc = cat(acc, cab, tab, node_seg<SEG>(U, first));
      last = first;
    } else {
      const SEG m = mid_range<SEG, TW>(U, fw, cx, p.from, p.to, p.rev);
      acc = cat(acc, cab, tab, m);
      last = p.rev ? node_at(fw, cx.off + p.from) : node_at(fw, cx.off + p.to);
    }
  }
  if (end >= 0) {
    ar.mark(U, last, end);
    const int32_t cab = arc_c(U, last, end);
    const int32_t tab = (AR::kTisC || U.t_is_c) ? cab : arc_t(U, last, end);
    acc = cat(acc, cab, tab, node_seg<SEG>(U, end));
  }
  return acc;
}

struct MoveEval {
  int64_t dF;
  int32_t dD, dTW, dLX, dDX, dV4;
  int32_t res[3];
};

// Delta of a recipe against the routes it replaces.
template <class SEG, bool TW, class AR = ArcPlain>
__device__ __forceinline__ void eval_recipe(const UnitDesc& U, const SEG* fw, const SEG* bw, const RouteCtx* rc,
                                            const Recipe& R, MoveEval& o, const AR& ar = AR()) {
  int32_t dD = 0, dTW = 0, dLX = 0, dDX = 0, dCL = 0;
  int32_t dep[4], dd[4];
  int nd = 0;
  auto bump = [&](int d, int by) {
    for (int z = 0; z < nd; ++z)
      if (dep[z] == d) { dd[z] += by; return; }
    dep[nd] = d; dd[nd] = by; ++nd;
  };
  for (int k = 0; k < R.nold; ++k) {
    const RouteCtx& c = rc[k];
    const int4 tot = ld(U.r_tot, c.slot);
    dD -= tot.x;
    dTW -= tot.w;
    dLX -= imax(tot.y - U.Q, 0);
    dDX -= U.Dmax >= 0 ? imax(tot.z - U.Dmax, 0) : 0;
    if (c.end >= 0 && c.start != c.end) dCL -= 1;
    bump(c.start, -1);
  }
  for (int w = 0; w < R.nnew; ++w) {
    if (R.np[w] == 0) continue;  // an emptied route is deleted
    const SEG s = eval_route<SEG, TW, AR>(U, fw, bw, rc, R.st[w], R.en[w], R.pc[w], R.np[w], ar);
    const RouteTerms t = route_terms(U, s);
    dD += t.C;
    dTW += t.TW;
    dLX += t.LX;
    dDX += t.DX;
    if (R.en[w] >= 0 && R.st[w] != R.en[w]) dCL += 1;
    bump(R.st[w], +1);
  }
  int32_t dFX = 0;
  int nres = 0;
  o.res[0] = o.res[1] = o.res[2] = -1;
  for (int k = 0; k < R.nold; ++k) o.res[nres++] = rc[k].slot;
  for (int z = 0; z < nd; ++z) {
    if (dd[z] == 0) continue;
    const int32_t n0 = ld(U.ndep, dep[z]);
    dFX += imax(n0 + dd[z] - U.NV, 0) - imax(n0 - U.NV, 0);
    if (nres < 3) o.res[nres] = U.R + dep[z];
    ++nres;
  }
  o.dD = dD;
  o.dTW = dTW;
  o.dLX = dLX;
  o.dDX = dDX;
  o.dV4 = dCL + dFX;
  o.dF = delta_F(U, dD, dTW, dLX, dDX, dCL + dFX);
}

__device__ __forceinline__ bool follower(const MoveEval& m) {
  return m.dD < 0 && m.dTW == 0 && m.dLX == 0 && m.dDX == 0 && m.dV4 == 0;
}

__device__ __forceinline__ RouteCtx route_ctx(const UnitDesc& U, int cur, int slot) {
  const int4 m = ld(U.r_meta[cur], slot);
  RouteCtx c;
  c.slot = slot;
  c.off = m.x;
  c.L = m.y;
  c.start = m.z;
  c.end = m.w;
  return c;
}

// Packed follower key, order-isomorphic to (dF, id) within a unit for moves with
// dF = dD in (-2^25, 0): high bits dD biased, low 38 bits the id's rank.
__device__ __forceinline__ uint64_t pack_key(const UnitDesc& U, int32_t dD, uint64_t id) {
  const uint64_t kind = id >> 56, var = (id >> 48) & 0xff, a = (id >> 24) & 0xffffff, b = id & 0xffffff;
  const uint64_t n = (uint64_t)U.n;
  const uint64_t idc = ((kind * 4 + var) * n + a) * n + b;
  const uint64_t biased = (uint64_t)((int64_t)dD + (1ll << 25));
  return (biased << 38) | idc;
}

}  // namespace mdvrp
