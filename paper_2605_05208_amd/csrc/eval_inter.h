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
  int uv_item;  // list slot whose cache holds {c(u, v), t(u, v)}, or -1: read the matrix
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

  // Every arc the enabled kinds create between the two routes' neighbourhoods, loaded
  // up front and unconditionally (nodes that do not exist are replaced by u, whose
  // arcs are then not used), so that the gathers of one anchor overlap instead of
  // following the kinds' branches one after the other; each distinct arc is read once.
  auto CT = [&](int a, int b) -> int2 {
    ar.mark(U, a, b);
    const int32_t c = arc_c(U, a, b);
    return make_int2(c, (AR::kTisC || U.t_is_c) ? c : arc_t(U, a, b));
  };
  // An arc between the two neighbourhoods, wanted as a -> b with a on v's side: on a
  // symmetric instance it is read as b -> a, so that every such read of the anchors of
  // one u (adjacent lanes) comes from the rows of the few nodes around u, whose nearby
  // columns share cache lines.
  auto CTv = [&](int a_vside, int b_uside) -> int2 {
    return sym ? CT(b_uside, a_vside) : CT(a_vside, b_uside);
  };
  const bool fREL = kinds & ((1u << REL1) | (1u << REL2));
  const bool fSWP = kinds & ((1u << SWP11) | (1u << SWP21) | (1u << SWP12) | (1u << SWP22));
  const bool fX2 = kinds & (1u << X2);
  const int su = s_u >= 0 ? s_u : u, ssu = ss_u >= 0 ? ss_u : u;
  int2 k_u_v = make_int2(0, 0), k_pv_su = k_u_v, k_pu_su = k_u_v, k_pv_u = k_u_v, k_ppu_su = k_u_v,
       k_pv_pu = k_u_v, k_pu_ssu = k_u_v, k_pu_pv = k_u_v, k_ppv_u = k_u_v, k_ppu_pv = k_u_v, k_ppv_pu = k_u_v,
       k_pv_ssu = k_u_v, k_ppv_su = k_u_v, k_pppv_u = k_u_v, k_pu_ppv = k_u_v, k_pppv_pu = k_u_v,
       k_ppu_ppv = k_u_v, k_pppv_su = k_u_v, k_ppv_ssu = k_u_v;
  k_u_v = x.uv_item >= 0 ? ld(U.nbr_ct, (uint32_t)x.uv_item) : CT(u, v);
  k_pv_su = CTv(p_v, su);
  if (fREL) {
    k_pu_su = CT(p_u, su);
    k_pv_u = CTv(p_v, u);
    k_ppu_su = CT(pp_u, su);
    k_pv_pu = CTv(p_v, p_u);
    if (sym) k_pu_ssu = CT(p_u, ssu);
  }
  if (fSWP) {
    k_pu_pv = CT(p_u, p_v);
    k_ppv_u = CTv(pp_v, u);
    k_ppu_pv = CT(pp_u, p_v);
    k_ppv_pu = CTv(pp_v, p_u);
    k_pppv_u = CTv(ppp_v, u);
    k_pu_ppv = CT(p_u, pp_v);
    k_pppv_pu = CTv(ppp_v, p_u);
    k_ppu_ppv = CT(pp_u, pp_v);
    if (sym) {
      k_pv_ssu = CTv(p_v, ssu);
      k_ppv_su = CTv(pp_v, su);
      k_pppv_su = CTv(ppp_v, su);
      k_ppv_ssu = CTv(pp_v, ssu);
    }
  }
  (void)fX2;
  // join of two sides through a loaded arc
  auto J = [&](const Side<SEG>& a, const Side<SEG>& b, int2 ct) -> Side<SEG> {
    return side(cat(a.s, ct.x, ct.y, b.s), a.first, b.last);
  };
  // the block (s(u), u) of the reversed 2-node moves (symmetric instances only): its arc
  // is the route's own arc u -> s(u), read off the suffix segments
  auto Xsu_block = [&]() -> Side<SEG> {
    const int32_t c = bau.C - ba1.C;
    const int32_t t = bau.D - ba1.D - service(U, u);
    return block2<SEG>(U, s_u, u, c, t);
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
  auto closeA = [&](const Side<SEG>& left, bool hasS, const Side<SEG>& S, int2 ct) -> SEG {
    return hasS ? J(left, S, ct).s : left.s;
  };

  // ---------------------------------------------------------------- Relocate
  if (kinds >> REL1 & 1) {
    const bool aEmpty = LA == 1;
    SEG Ap = fa1;
    if (!aEmpty) Ap = closeA(Pu1, hasSA1, Su1, k_pu_su);
    const SEG Bp = J(J(Pv1, Nu, k_pv_u), Sv0, k_u_v).s;
    finish(make_id(REL1, 0, u, v), aEmpty, Ap, x.eA, false, Bp, x.eB);
  }
  if (kinds >> REL2 & 1) {
    if (hasPPu) {  // X = (p(u), u)
      const bool aEmpty = LA == 2;
      SEG Ap = fa2;
      if (!aEmpty) Ap = closeA(Pu2, hasSA1, Su1, k_ppu_su);
      const SEG Bp = J(J(Pv1, Xpu, k_pv_pu), Sv0, k_u_v).s;
      finish(make_id(REL2, 0, u, v), aEmpty, Ap, x.eA, false, Bp, x.eB);
    }
    if (sym && hasSu) {  // block (u, s(u)) placed as (s(u), u)
      const bool aEmpty = LA == 2;
      SEG Ap = fa1;
      if (!aEmpty) Ap = closeA(Pu1, hasSA2, Su2, k_pu_ssu);
      const SEG Bp = J(J(Pv1, Xsu_block(), k_pv_su), Sv0, k_u_v).s;
      finish(make_id(REL2, 1, u, v), aEmpty, Ap, x.eA, false, Bp, x.eB);
    }
  }
  // ---------------------------------------------------------------- Swap
  if (kinds >> SWP11 & 1) {
    if (hasPv) {
      const SEG Ap = closeA(J(Pu1, Npv, k_pu_pv), hasSA1, Su1, k_pv_su);
      const SEG Bp = J(J(Pv2, Nu, k_ppv_u), Sv0, k_u_v).s;
      finish(make_id(SWP11, 0, u, v), false, Ap, x.eA, false, Bp, x.eB);
    }
  }
  if (kinds >> SWP21 & 1) {
    if (hasPv && hasPPu) {  // X = (p(u), u), Y = (p(v))
      const SEG Ap = closeA(J(Pu2, Npv, k_ppu_pv), hasSA1, Su1, k_pv_su);
      const SEG Bp = J(J(Pv2, Xpu, k_ppv_pu), Sv0, k_u_v).s;
      finish(make_id(SWP21, 0, u, v), false, Ap, x.eA, false, Bp, x.eB);
    }
    if (sym && hasPv && hasSu) {  // X = (u, s(u)) placed as (s(u), u)
      const SEG Ap = closeA(J(Pu1, Npv, k_pu_pv), hasSA2, Su2, k_pv_ssu);
      const SEG Bp = J(J(Pv2, Xsu_block(), k_ppv_su), Sv0, k_u_v).s;
      finish(make_id(SWP21, 1, u, v), false, Ap, x.eA, false, Bp, x.eB);
    }
  }
  if (kinds >> SWP12 & 1) {
    if (hasPPv) {
      const SEG Bp = J(J(Pv3, Nu, k_pppv_u), Sv0, k_u_v).s;
      {  // Y = (pp(v), p(v)) as is
        const SEG Ap = closeA(J(Pu1, Ypv, k_pu_ppv), hasSA1, Su1, k_pv_su);
        finish(make_id(SWP12, 0, u, v), false, Ap, x.eA, false, Bp, x.eB);
      }
      if (sym) {  // Y reversed: (p(v), pp(v)); its arc is the route's own, symmetric
        const Side<SEG> Yr = block2<SEG>(U, p_v, pp_v, c_pv2, t_pv2);
        const SEG Ap = closeA(J(Pu1, Yr, k_pu_pv), hasSA1, Su1, k_ppv_su);
        finish(make_id(SWP12, 1, u, v), false, Ap, x.eA, false, Bp, x.eB);
      }
    }
  }
  if (kinds >> SWP22 & 1) {
    if (hasPPv) {
      const Side<SEG> Yr = block2<SEG>(U, p_v, pp_v, c_pv2, t_pv2);
      if (hasPPu) {  // X = (p(u), u)
        const SEG Bp = J(J(Pv3, Xpu, k_pppv_pu), Sv0, k_u_v).s;
        const SEG Ap = closeA(J(Pu2, Ypv, k_ppu_ppv), hasSA1, Su1, k_pv_su);
        finish(make_id(SWP22, 0, u, v), false, Ap, x.eA, false, Bp, x.eB);
        if (sym) {
          const SEG Ap2 = closeA(J(Pu2, Yr, k_ppu_pv), hasSA1, Su1, k_ppv_su);
          finish(make_id(SWP22, 2, u, v), false, Ap2, x.eA, false, Bp, x.eB);
        }
      }
      if (sym && hasSu) {  // X = (u, s(u)) placed as (s(u), u)
        const SEG Bp = J(J(Pv3, Xsu_block(), k_pppv_su), Sv0, k_u_v).s;
        const SEG Ap = closeA(J(Pu1, Ypv, k_pu_ppv), hasSA2, Su2, k_pv_ssu);
        finish(make_id(SWP22, 1, u, v), false, Ap, x.eA, false, Bp, x.eB);
        const SEG Ap2 = closeA(J(Pu1, Yr, k_pu_pv), hasSA2, Su2, k_ppv_ssu);
        finish(make_id(SWP22, 3, u, v), false, Ap2, x.eA, false, Bp, x.eB);
      }
    }
  }
  // ---------------------------------------------------------------- 2-opt*
  if (kinds >> X2 & 1) {
    // A' = A[..u] + B[v..] (ends at B's depot), B' = B[..p(v)] + A[s(u)..] (ends at A's depot)
    const SEG Ap = J(Pu0, Sv0, k_u_v).s;
    const bool bEmpty = (pv == 1) && (pu == LA);
    SEG Bp = fb1;
    if (!bEmpty) {
      if (pu == LA) {
        // B' = prefix of B to p(v), then A's end depot (closed) or nothing (open); the
        // suffix from s(u) of a closed route is that depot alone, s(u) = its node
        if (!OPEN) Bp = J(Pv1, single<SEG>(U, x.eA), k_pv_su).s;
      } else {
        Bp = J(Pv1, Su1, k_pv_su).s;
      }
    }
    finish(make_id(X2, 0, u, v), false, Ap, x.eB, bEmpty, Bp, x.eA);
  }
}

}  // namespace mdvrp
