// eval_inter.h -- specialised evaluation of the inter-route pair kinds.
//
// For an anchor (u in route A at position pu, v in route B != A at position
// pv) every inter-route move is "prefix of one route + at most one moved block
// + suffix of a route" on each side, so it needs a handful of prefix/suffix
// segments around u and v that are loaded once and shared by all kinds:
//   A side: prefix to pp(u), p(u), u; suffix from s(u), ss(u)
//   B side: prefix to ppp(v), pp(v), p(v); suffix from v
// plus the few arcs the moves create. The recipes are the same as the generic
// evaluator's (Relocate / Swap / 2-opt*, Section 3.2.2) and produce identical
// integers.
#pragma once
#include "eval_common.h"

namespace mdvrp {

template <class SEG> struct Side {
  SEG s;      // segment
  int first;  // first node
  int last;   // last node
};

template <class SEG>
__device__ __forceinline__ Side<SEG> side(const SEG& s, int first, int last) {
  Side<SEG> r;
  r.s = s; r.first = first; r.last = last;
  return r;
}

template <class SEG>
__device__ __forceinline__ Side<SEG> join(const UnitDesc& U, const Side<SEG>& a, const Side<SEG>& b) {
  const int32_t c = arc_c(U, a.last, b.first);
  const int32_t t = U.t_is_c ? c : arc_t(U, a.last, b.first);
  return side(cat(a.s, c, t, b.s), a.first, b.last);
}

// Two-node block x -> y whose internal arc costs c_xy / t_xy are known.
template <class SEG>
__device__ __forceinline__ Side<SEG> block2(const UnitDesc& U, int x, int y, int32_t cxy, int32_t txy) {
  return side(cat(node_seg<SEG>(U, x), cxy, txy, node_seg<SEG>(U, y)), x, y);
}

template <class SEG>
__device__ __forceinline__ Side<SEG> single(const UnitDesc& U, int x) {
  return side(node_seg<SEG>(U, x), x, x);
}

// Travel time of the arc leaving position k (stored with time windows; derived
// from the duration prefix otherwise: D(k+1) - D(k) - s(next)).
__device__ __forceinline__ int32_t next_t(const UnitDesc& U, const SegTW& a, const SegTW& b) {
  (void)U; (void)b;
  return a.aux;
}
__device__ __forceinline__ int32_t next_t(const UnitDesc& U, const SegNT& a, const SegNT& b) {
  return b.D - a.D - service(U, b.node);
}

struct InterCtx {
  int u, v;
  int slotA, slotB, LA, LB, sA, sB, eA, eB, pu, pv;
  int au, av;  // absolute positions of u and v in the current buffer
};

template <class SEG, bool TW, bool OPEN, class AR, class OUT>
__device__ __forceinline__ void eval_inter(const UnitDesc& U, const SEG* fw, const SEG* bw, int offA, int offB,
                                           const InterCtx& x, uint32_t kinds, const AR& ar, OUT& o) {
  const bool sym = !TW;
  const int pu = x.pu, pv = x.pv, LA = x.LA;
  // ---------------------------------------------------------------- loads
  // Addressed by absolute position, so they do not wait for the route table; the
  // neighbours that may not exist are loaded at clamped in-buffer positions and
  // replaced below by the segment the position rules choose.
  (void)offA; (void)offB;
  const int au = x.au, av = x.av, last = U.cap - 1;
  const SEG fa0 = ld(fw, au);                  // prefix to u
  const SEG fa1 = ld(fw, au - 1);              // prefix to p(u)
  const SEG fa2l = ld(fw, imax(au - 2, 0));
  const SEG bau = ld(bw, au);                  // suffix from u
  const SEG ba1l = ld(bw, imin(au + 1, last));
  const SEG ba2l = sym ? ld(bw, imin(au + 2, last)) : bau;
  const SEG fb1 = ld(fw, av - 1);              // prefix to p(v)
  const SEG fb2l = ld(fw, imax(av - 2, 0));
  const SEG fb3l = ld(fw, imax(av - 3, 0));
  const SEG bb0 = ld(bw, av);                  // suffix from v
  const bool hasPPu = pu >= 2;
  const SEG fa2 = hasPPu ? fa2l : fa1;         // prefix to pp(u)
  const bool hasSA1 = OPEN ? (pu + 1 <= LA) : true;          // suffix from s(u) exists
  const SEG ba1 = hasSA1 ? ba1l : bau;
  const bool hasSu = pu + 1 <= LA;                           // s(u) is a customer
  const bool hasSA2 = OPEN ? (pu + 2 <= LA) : (pu + 2 <= LA + 1);
  const SEG ba2 = (sym && hasSA2) ? ba2l : bau;
  const bool hasPv = pv >= 2, hasPPv = pv >= 3;
  const SEG fb2 = hasPv ? fb2l : fb1;          // prefix to pp(v)
  const SEG fb3 = hasPPv ? fb3l : fb1;         // prefix to ppp(v)
  const int u = x.u, v = x.v;
  const int p_u = fa1.node, pp_u = fa2.node, s_u = hasSA1 ? ba1.node : -1, ss_u = hasSA2 ? ba2.node : -1;
  const int p_v = fb1.node, pp_v = fb2.node, ppp_v = fb3.node;
  // old route terms
  const int4 totA = ld(U.r_tot, x.slotA), totB = ld(U.r_tot, x.slotB);
  const int32_t lxAB = imax(totA.y - U.Q, 0) + imax(totB.y - U.Q, 0);
  const int32_t dxAB = U.Dmax >= 0 ? imax(totA.z - U.Dmax, 0) + imax(totB.z - U.Dmax, 0) : 0;
  const int32_t clAB = (x.eA >= 0 && x.sA != x.eA) + (x.eB >= 0 && x.sB != x.eB);
  // shared sides
  const Side<SEG> Pu1 = side(fa1, x.sA, p_u);   // A prefix up to p(u)
  const Side<SEG> Pu0 = side(fa0, x.sA, u);     // A prefix up to u
  const Side<SEG> Pu2 = side(fa2, x.sA, pp_u);  // A prefix up to pp(u)
  const Side<SEG> Su1 = side(ba1, s_u, x.eA);   // A suffix from s(u)
  const Side<SEG> Su2 = side(ba2, ss_u, x.eA);  // A suffix from ss(u)
  const Side<SEG> Pv1 = side(fb1, x.sB, p_v);
  const Side<SEG> Pv2 = side(fb2, x.sB, pp_v);
  const Side<SEG> Pv3 = side(fb3, x.sB, ppp_v);
  const Side<SEG> Sv0 = side(bb0, v, x.eB);
  // blocks
  const Side<SEG> Nu = single<SEG>(U, u);
  const Side<SEG> Npv = single<SEG>(U, p_v);
  const int32_t c_pu_u = fa0.C - fa1.C, t_pu_u = next_t(U, fa1, fa0);
  const Side<SEG> Xpu = block2<SEG>(U, p_u, u, c_pu_u, t_pu_u);             // (p(u), u)
  const int32_t c_pv2 = fb1.C - fb2.C, t_pv2 = next_t(U, fb2, fb1);
  const Side<SEG> Ypv = block2<SEG>(U, pp_v, p_v, c_pv2, t_pv2);           // (pp(v), p(v))

  // join with a matrix arc (marked for footprint measurements)
  auto J = [&](const Side<SEG>& a, const Side<SEG>& b) -> Side<SEG> {
    ar.mark(U, a.last, b.first);
    return join(U, a, b);
  };
  auto AC = [&](int a, int b) -> int32_t {
    ar.mark(U, a, b);
    return arc_c(U, a, b);
  };
  auto AT = [&](int a, int b) -> int32_t {
    ar.mark(U, a, b);
    return arc_t(U, a, b);
  };

  // move delta: new A' (may be empty), new B' (may be empty), end depots of the new routes
  auto finish = [&](uint64_t id, bool aEmpty, const SEG& Ap, int eAp, bool bEmpty, const SEG& Bp, int eBp) {
    MoveEval m;
    int32_t dD = -(totA.x + totB.x), dTW = -(totA.w + totB.w), dLX = -lxAB, dDX = -dxAB, dCL = -clAB;
    int dep = -1;
    if (!aEmpty) {
      const RouteTerms t = route_terms(U, Ap);
      dD += t.C; dTW += t.TW; dLX += t.LX; dDX += t.DX;
      dCL += (eAp >= 0 && x.sA != eAp);
    } else {
      dep = x.sA;
    }
    if (!bEmpty) {
      const RouteTerms t = route_terms(U, Bp);
      dD += t.C; dTW += t.TW; dLX += t.LX; dDX += t.DX;
      dCL += (eBp >= 0 && x.sB != eBp);
    } else {
      dep = x.sB;
    }
    int32_t dFX = 0;
    m.res[0] = x.slotA;
    m.res[1] = x.slotB;
    m.res[2] = -1;
    if (dep >= 0) {
      const int32_t n0 = ld(U.ndep, dep);
      dFX = imax(n0 - 1 - U.NV, 0) - imax(n0 - U.NV, 0);
      m.res[2] = U.R + dep;
    }
    m.dD = dD; m.dTW = dTW; m.dLX = dLX; m.dDX = dDX; m.dV4 = dCL + dFX;
    m.dF = delta_F(U, dD, dTW, dLX, dDX, dCL + dFX);
    take(U, o, m, id);
  };
  // A' = prefix + [block] + suffix (suffix may be absent on open routes)
  auto closeA = [&](const Side<SEG>& left, bool hasS, const Side<SEG>& S) -> SEG {
    return hasS ? J(left, S).s : left.s;
  };

  // ---------------------------------------------------------------- Relocate
  if (kinds >> REL1 & 1) {
    const bool aEmpty = LA == 1;
    SEG Ap = fa1;
    if (!aEmpty) Ap = closeA(Pu1, hasSA1, Su1);
    const SEG Bp = J(J(Pv1, Nu), Sv0).s;
    finish(make_id(REL1, 0, u, v), aEmpty, Ap, x.eA, false, Bp, x.eB);
  }
  if (kinds >> REL2 & 1) {
    if (hasPPu) {  // X = (p(u), u)
      const bool aEmpty = LA == 2;
      SEG Ap = fa2;
      if (!aEmpty) Ap = closeA(Pu2, hasSA1, Su1);
      const SEG Bp = J(J(Pv1, Xpu), Sv0).s;
      finish(make_id(REL2, 0, u, v), aEmpty, Ap, x.eA, false, Bp, x.eB);
    }
    if (sym && hasSu) {  // block (u, s(u)) placed as (s(u), u)
      const bool aEmpty = LA == 2;
      SEG Ap = fa1;
      if (!aEmpty) Ap = closeA(Pu1, hasSA2, Su2);
      const Side<SEG> Xsu = block2<SEG>(U, s_u, u, AC(s_u, u), AT(s_u, u));
      const SEG Bp = J(J(Pv1, Xsu), Sv0).s;
      finish(make_id(REL2, 1, u, v), aEmpty, Ap, x.eA, false, Bp, x.eB);
    }
  }
  // ---------------------------------------------------------------- Swap
  if (kinds >> SWP11 & 1) {
    if (hasPv) {
      const SEG Ap = closeA(J(Pu1, Npv), hasSA1, Su1);
      const SEG Bp = J(J(Pv2, Nu), Sv0).s;
      finish(make_id(SWP11, 0, u, v), false, Ap, x.eA, false, Bp, x.eB);
    }
  }
  if (kinds >> SWP21 & 1) {
    if (hasPv && hasPPu) {  // X = (p(u), u), Y = (p(v))
      const SEG Ap = closeA(J(Pu2, Npv), hasSA1, Su1);
      const SEG Bp = J(J(Pv2, Xpu), Sv0).s;
      finish(make_id(SWP21, 0, u, v), false, Ap, x.eA, false, Bp, x.eB);
    }
    if (sym && hasPv && hasSu) {  // X = (u, s(u)) placed as (s(u), u)
      const Side<SEG> Xsu = block2<SEG>(U, s_u, u, AC(s_u, u), AT(s_u, u));
      const SEG Ap = closeA(J(Pu1, Npv), hasSA2, Su2);
      const SEG Bp = J(J(Pv2, Xsu), Sv0).s;
      finish(make_id(SWP21, 1, u, v), false, Ap, x.eA, false, Bp, x.eB);
    }
  }
  if (kinds >> SWP12 & 1) {
    if (hasPPv) {
      const SEG Bp = J(J(Pv3, Nu), Sv0).s;
      {  // Y = (pp(v), p(v)) as is
        const SEG Ap = closeA(J(Pu1, Ypv), hasSA1, Su1);
        finish(make_id(SWP12, 0, u, v), false, Ap, x.eA, false, Bp, x.eB);
      }
      if (sym) {  // Y reversed: (p(v), pp(v))
        const Side<SEG> Yr = block2<SEG>(U, p_v, pp_v, c_pv2, AT(p_v, pp_v));
        const SEG Ap = closeA(J(Pu1, Yr), hasSA1, Su1);
        finish(make_id(SWP12, 1, u, v), false, Ap, x.eA, false, Bp, x.eB);
      }
    }
  }
  if (kinds >> SWP22 & 1) {
    if (hasPPv) {
      const Side<SEG> Yr = block2<SEG>(U, p_v, pp_v, c_pv2, sym ? AT(p_v, pp_v) : 0);
      if (hasPPu) {  // X = (p(u), u)
        const SEG Bp = J(J(Pv3, Xpu), Sv0).s;
        const SEG Ap = closeA(J(Pu2, Ypv), hasSA1, Su1);
        finish(make_id(SWP22, 0, u, v), false, Ap, x.eA, false, Bp, x.eB);
        if (sym) {
          const SEG Ap2 = closeA(J(Pu2, Yr), hasSA1, Su1);
          finish(make_id(SWP22, 2, u, v), false, Ap2, x.eA, false, Bp, x.eB);
        }
      }
      if (sym && hasSu) {  // X = (u, s(u)) placed as (s(u), u)
        const Side<SEG> Xsu = block2<SEG>(U, s_u, u, AC(s_u, u), AT(s_u, u));
        const SEG Bp = J(J(Pv3, Xsu), Sv0).s;
        const SEG Ap = closeA(J(Pu1, Ypv), hasSA2, Su2);
        finish(make_id(SWP22, 1, u, v), false, Ap, x.eA, false, Bp, x.eB);
        const SEG Ap2 = closeA(J(Pu1, Yr), hasSA2, Su2);
        finish(make_id(SWP22, 3, u, v), false, Ap2, x.eA, false, Bp, x.eB);
      }
    }
  }
  // ---------------------------------------------------------------- 2-opt*
  if (kinds >> X2 & 1) {
    // A' = A[..u] + B[v..] (ends at B's depot), B' = B[..p(v)] + A[s(u)..] (ends at A's depot)
    const SEG Ap = J(Pu0, Sv0).s;
    const bool bEmpty = (pv == 1) && (pu == LA);
    SEG Bp = fb1;
    if (!bEmpty) {
      if (pu == LA) {
        // B' = prefix of B to p(v), then A's end depot (closed) or nothing (open)
        if (!OPEN) Bp = J(Pv1, single<SEG>(U, x.eA)).s;
      } else {
        Bp = J(Pv1, Su1).s;
      }
    }
    finish(make_id(X2, 0, u, v), false, Ap, x.eB, bEmpty, Bp, x.eA);
  }
}

}  // namespace mdvrp
