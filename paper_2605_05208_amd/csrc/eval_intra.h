// eval_intra.h -- fixed-shape evaluation of intra-route pair moves and depot moves.
//
// An intra-route move rearranges one route A as
//   prefix(A, x) + up to three middle ranges of A (possibly reversed) + suffix(A, y)
// (Relocate inside a route, Swap inside a route, 2-opt; Section 3.2.2). The
// shape is the same for every kind, so the pieces are plain scalars and the
// evaluation is one straight-line routine (no per-piece arrays). Depot-Insert
// and Depot-Replace (Fig. 1) are prefix/suffix segments joined to a depot.
#pragma once
#include "eval_common.h"

namespace mdvrp {

struct Mid {
  int from, to, rev;  // empty when from > to
};

struct IntraShape {
  int x;          // prefix ends at position x (0 = start depot only)
  Mid m[3];
  int y;          // suffix starts at position y (L+1 = end depot; open routes: nothing)
};

__device__ __forceinline__ Mid mid(int from, int to, int rev) {
  Mid r;
  r.from = from; r.to = to; r.rev = rev;
  return r;
}

// Relocate inside A: block [xa, xb] (reversed when xrev) in front of position pv.
__device__ __forceinline__ IntraShape shape_rel(int xa, int xb, int xrev, int pv) {
  IntraShape s;
  if (pv < xa) {
    s.x = pv - 1; s.m[0] = mid(xa, xb, xrev); s.m[1] = mid(pv, xa - 1, 0); s.m[2] = mid(1, 0, 0); s.y = xb + 1;
  } else {
    s.x = xa - 1; s.m[0] = mid(xb + 1, pv - 1, 0); s.m[1] = mid(xa, xb, xrev); s.m[2] = mid(1, 0, 0); s.y = pv;
  }
  return s;
}

// Swap inside A: block X = [xa, xb] to Y's place, Y = [ya, yb] to X's place.
__device__ __forceinline__ IntraShape shape_swp(int xa, int xb, int xrev, int ya, int yb, int yrev) {
  IntraShape s;
  if (xa < ya) {
    s.x = xa - 1; s.m[0] = mid(ya, yb, yrev); s.m[1] = mid(xb + 1, ya - 1, 0); s.m[2] = mid(xa, xb, xrev);
    s.y = yb + 1;
  } else {
    s.x = ya - 1; s.m[0] = mid(xa, xb, xrev); s.m[1] = mid(yb + 1, xa - 1, 0); s.m[2] = mid(ya, yb, yrev);
    s.y = xb + 1;
  }
  return s;
}

template <class SEG, bool TW, bool OPEN, class AR>
__device__ __forceinline__ SEG eval_shape(const UnitDesc& U, const SEG* fw, const SEG* bw, const RouteCtx& A,
                                          const IntraShape& s, const AR& ar) {
  SEG acc = ld(fw, A.off + s.x);
  int last = acc.node;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const Mid& m = s.m[j];
    if (m.from > m.to) continue;
    const int first = node_at(fw, A.off + (m.rev ? m.to : m.from));
    ar.mark(U, last, first);
    const int32_t c = arc_c(U, last, first);
    const int32_t t = (AR::kTisC || U.t_is_c) ? c : arc_t(U, last, first);
    if (m.from == m.to) {
      acc = cat(acc, c, t, node_seg<SEG>(U, first));
    } else {
      acc = cat(acc, c, t, mid_range<SEG, TW>(U, fw, A, m.from, m.to, m.rev));
    }
    last = node_at(fw, A.off + (m.rev ? m.from : m.to));
  }
  const bool hasS = OPEN ? (s.y <= A.L) : true;
  if (hasS) {
    const SEG suf = ld(bw, A.off + s.y);
    ar.mark(U, last, suf.node);
    const int32_t c = arc_c(U, last, suf.node);
    const int32_t t = (AR::kTisC || U.t_is_c) ? c : arc_t(U, last, suf.node);
    acc = cat(acc, c, t, suf);
  }
  return acc;
}

// Delta of replacing route A by A' with the same depots (intra-route moves).
template <class SEG>
__device__ __forceinline__ void intra_delta(const UnitDesc& U, const RouteCtx& A, const SEG& Ap, MoveEval& m) {
  const int4 tot = ld(U.r_tot, A.slot);
  const RouteTerms t = route_terms(U, Ap);
  m.dD = t.C - tot.x;
  m.dTW = t.TW - tot.w;
  m.dLX = t.LX - imax(tot.y - U.Q, 0);
  m.dDX = t.DX - (U.Dmax >= 0 ? imax(tot.z - U.Dmax, 0) : 0);
  m.dV4 = 0;
  m.dF = delta_F(U, m.dD, m.dTW, m.dLX, m.dDX, 0);
  m.res[0] = A.slot;
  m.res[1] = -1;
  m.res[2] = -1;
}

// Every intra-route pair kind of kind_mask for anchor u (pu), v (pv) in route A.
template <class SEG, bool TW, bool OPEN, class AR, class SINK>
__device__ __forceinline__ void eval_intra(const UnitDesc& U, const SEG* fw, const SEG* bw, const RouteCtx& A,
                                           int u, int v, int pu, int pv, uint32_t kinds, const AR& ar, SINK& sk) {
  const bool sym = !TW;
  MoveEval m;
  auto run = [&](const IntraShape& s, uint64_t id) {
    const SEG Ap = eval_shape<SEG, TW, OPEN>(U, fw, bw, A, s, ar);
    intra_delta(U, A, Ap, m);
    take(U, sk, m, id);
  };
  if (kinds >> REL1 & 1) {
    if (pv != pu + 1) run(shape_rel(pu, pu, 0, pv), make_id(REL1, 0, u, v));
  }
  if (kinds >> REL2 & 1) {
    if (pu >= 2 && pv != pu - 1 && pv != pu + 1) run(shape_rel(pu - 1, pu, 0, pv), make_id(REL2, 0, u, v));
    if (sym && pu + 1 <= A.L && pv != pu + 1) run(shape_rel(pu, pu + 1, 1, pv), make_id(REL2, 1, u, v));
  }
  if (kinds >> SWP11 & 1) {
    if (pv >= 2 && pv - 1 != pu) run(shape_swp(pu, pu, 0, pv - 1, pv - 1, 0), make_id(SWP11, 0, u, v));
  }
  if (kinds >> SWP21 & 1) {
    if (pv >= 2) {
      const int ya = pv - 1;
      if (pu >= 2 && !(ya >= pu - 1 && ya <= pu) && !(pv >= pu - 1 && pv <= pu))
        run(shape_swp(pu - 1, pu, 0, ya, ya, 0), make_id(SWP21, 0, u, v));
      if (sym && pu + 1 <= A.L && !(ya >= pu && ya <= pu + 1) && !(pv >= pu && pv <= pu + 1))
        run(shape_swp(pu, pu + 1, 1, ya, ya, 0), make_id(SWP21, 1, u, v));
    }
  }
  if (kinds >> SWP12 & 1) {
    if (pv >= 3 && !(pu >= pv - 2 && pu <= pv - 1)) {
      run(shape_swp(pu, pu, 0, pv - 2, pv - 1, 0), make_id(SWP12, 0, u, v));
      if (sym) run(shape_swp(pu, pu, 0, pv - 2, pv - 1, 1), make_id(SWP12, 1, u, v));
    }
  }
  if (kinds >> SWP22 & 1) {
    if (pv >= 3) {
      const int ya = pv - 2, yb = pv - 1;
      for (int ox = 0; ox < (sym ? 2 : 1); ++ox) {
        const int xa = ox ? pu : pu - 1, xb = ox ? pu + 1 : pu;
        if (ox == 0 && pu < 2) continue;
        if (ox == 1 && pu + 1 > A.L) continue;
        if ((ya <= xb && xa <= yb) || (pv >= xa && pv <= xb)) continue;
        for (int oy = 0; oy < (sym ? 2 : 1); ++oy)
          run(shape_swp(xa, xb, ox, ya, yb, oy), make_id(SWP22, ox + 2 * oy, u, v));
      }
    }
  }
  if (sym && (kinds >> TWOOPT & 1)) {
    if (pu < pv - 1) {
      IntraShape s;
      s.x = pu; s.m[0] = mid(pu + 1, pv, 1); s.m[1] = mid(1, 0, 0); s.m[2] = mid(1, 0, 0); s.y = pv + 1;
      run(s, make_id(TWOOPT, 0, u, v));
    }
  }
}

// ----------------------------------------------------------------------------- depot operators

// Delta of a depot move replacing route A by one or two routes. Vehicle counts
// change by -1 at dm and +1 at dp (-1 = no change; dm != dp).
template <class SEG>
__device__ __forceinline__ void depot_delta(const UnitDesc& U, const RouteCtx& A, int n_new, const SEG& R1, int s1,
                                            int e1, const SEG& R2, int s2, int e2, int dm, int dp, MoveEval& m) {
  const int4 tot = ld(U.r_tot, A.slot);
  int32_t dD = -tot.x, dTW = -tot.w;
  int32_t dLX = -imax(tot.y - U.Q, 0);
  int32_t dDX = -(U.Dmax >= 0 ? imax(tot.z - U.Dmax, 0) : 0);
  int32_t dCL = -(A.end >= 0 && A.start != A.end);
  {
    const RouteTerms t = route_terms(U, R1);
    dD += t.C; dTW += t.TW; dLX += t.LX; dDX += t.DX;
    dCL += (e1 >= 0 && s1 != e1);
  }
  if (n_new == 2) {
    const RouteTerms t = route_terms(U, R2);
    dD += t.C; dTW += t.TW; dLX += t.LX; dDX += t.DX;
    dCL += (e2 >= 0 && s2 != e2);
  }
  int32_t dFX = 0;
  m.res[0] = A.slot;
  m.res[1] = -1;
  m.res[2] = -1;
  int nres = 1;
  if (dm >= 0) {
    const int32_t n0 = ld(U.ndep, dm);
    dFX += imax(n0 - 1 - U.NV, 0) - imax(n0 - U.NV, 0);
    m.res[nres++] = U.R + dm;
  }
  if (dp >= 0) {
    const int32_t n0 = ld(U.ndep, dp);
    dFX += imax(n0 + 1 - U.NV, 0) - imax(n0 - U.NV, 0);
    m.res[nres++] = U.R + dp;
  }
  m.dD = dD; m.dTW = dTW; m.dLX = dLX; m.dDX = dDX; m.dV4 = dCL + dFX;
  m.dF = delta_F(U, dD, dTW, dLX, dDX, dCL + dFX);
}

// Depot-Insert (Fig. 1a): cut after position pu of A, insert depot d between the parts.
template <class SEG, bool TW, bool OPEN, class AR>
__device__ __forceinline__ void eval_dins(const UnitDesc& U, const SEG* fw, const SEG* bw, const RouteCtx& A, int pu,
                                          int d, const AR& ar, MoveEval& m) {
  const SEG pre = ld(fw, A.off + pu);
  SEG R1 = pre;
  if (!OPEN) {
    if (!U.dep_arc) ar.mark(U, pre.node, d);
    const int4 a = dep_arcs(U, pre.node, d);
    R1 = cat(pre, a.z, a.w, node_seg<SEG>(U, d));
  }
  const SEG suf = ld(bw, A.off + pu + 1);
  if (!U.dep_arc) ar.mark(U, d, suf.node);
  const int4 a2 = dep_arcs(U, suf.node, d);
  const SEG R2 = cat(node_seg<SEG>(U, d), a2.x, a2.y, suf);
  depot_delta(U, A, 2, R1, A.start, OPEN ? -1 : d, R2, d, A.end, -1, d, m);
}

// Depot-Replace (Fig. 1b): case 0 departure depot, 1 arrival depot, 2 both.
template <class SEG, bool TW, bool OPEN, class AR>
__device__ __forceinline__ void eval_drep(const UnitDesc& U, const SEG* fw, const SEG* bw, const RouteCtx& A, int d,
                                          int cs, const AR& ar, MoveEval& m) {
  const int ns = (cs == 0 || cs == 2) ? d : A.start;
  const int ne = (cs == 1 || cs == 2) ? d : A.end;
  SEG R;
  if (cs == 0) {
    const SEG suf = ld(bw, A.off + 1);
    if (!U.dep_arc) ar.mark(U, d, suf.node);
    const int4 a = dep_arcs(U, suf.node, d);
    R = cat(node_seg<SEG>(U, d), a.x, a.y, suf);
  } else {
    const SEG pre = ld(fw, A.off + A.L);
    SEG body;
    int first;
    if (cs == 1) {
      body = pre;
    } else {
      first = ld(fw, A.off + 1).node;
      SEG core;
      if constexpr (TW) {
        core = A.L <= kCoreMaxL ? ld(U.r_core, A.slot)
                                : (A.L == 1 ? node_seg<SEG>(U, first) : mid_range<SEG, TW>(U, fw, A, 1, A.L, 0));
      } else {
        core = A.L == 1 ? node_seg<SEG>(U, first) : mid_range<SEG, TW>(U, fw, A, 1, A.L, 0);
      }
      if (!U.dep_arc) ar.mark(U, d, first);
      const int4 a = dep_arcs(U, first, d);
      body = cat(node_seg<SEG>(U, d), a.x, a.y, core);
    }
    if (!U.dep_arc) ar.mark(U, pre.node, d);
    const int4 a = dep_arcs(U, pre.node, d);
    R = cat(body, a.z, a.w, node_seg<SEG>(U, d));
  }
  const bool moves_start = cs != 1;
  depot_delta(U, A, 1, R, ns, ne, R, 0, 0, moves_start ? A.start : -1, moves_start ? d : -1, m);
}

}  // namespace mdvrp
