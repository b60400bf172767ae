// internal.h -- device-side data layout and shared device code of libmdvrp.
//
// Solution state of one unit (= one solution of one instance) lives in HBM as
//   * node-indexed arrays rt[x] (route slot) and pos[x] (1..L in the route);
//   * a route table over slots 0..R-1 (R = number of customers, the most
//     non-empty routes a solution can have);
//   * a flat, route-major position array per buffer (double-buffered):
//     route r occupies positions off[r] .. off[r]+L+1 (0 = start depot,
//     1..L customers, L+1 = end depot; open routes leave L+1 unused).
//     Each position holds the forward segment fw (positions 0..k of its
//     route) and the backward segment bw (positions k..end), both in
//     array-of-structs form so that one random access touches one line.
// Segments follow the sequence-concatenation evaluation the paper adopts
// (Section 3.2.2): distance C and load Q are plain sums; with time windows,
// duration D, time warp TW, earliest start E and latest start L combine by
// Vidal's concatenation, which is associative, so prefixes are wave scans.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mdvrp {

constexpr int kMaxPieces = 5;
// Time-window routes of at most kCoreMaxL customers keep the segment of their customers
// (positions 1..L, no depots), which Depot-Replace needs for a new pair of depots.
constexpr int kCoreMaxL = 62;
constexpr int kTileSize = 256;  // items per evaluation tile (one block, one leader record)
constexpr int kPairKindSlots = 14;  // kind/variant slots of one (u, v) anchor
constexpr int64_t kNoMove = INT64_MAX;

enum Kind { REL1 = 0, REL2 = 1, SWP11 = 2, SWP21 = 3, SWP12 = 4, SWP22 = 5, X2 = 6, TWOOPT = 7,
            DINS = 8, DREP = 9 };
enum Family { FAM_REL = 0, FAM_SWP = 1, FAM_X2 = 2, FAM_2OPT = 3, FAM_DINS = 4, FAM_DREP = 5 };

// Segment without time windows: distance, load, duration (travel + service).
struct alignas(16) SegNT {
  int32_t C, Q, D, node;
};
// Segment with time windows; aux = travel time to the next position.
struct alignas(32) SegTW {
  int32_t C, Q, D, TW, E, L, node, aux;
};

// One move record: full key (dF, id), distance delta, follower flag, resources.
struct MoveRec {
  int64_t dF;
  uint64_t id;
  int32_t dD;
  int32_t elig;
  int32_t res[3];
  int32_t pad;
};

// Dense debug record (every evaluated move).
struct DenseRec {
  int64_t dF, dD, dTW, dLX, dDX, dV4;
  uint64_t id;
  int32_t unit;
  int32_t res[3];
};

// Per-unit control block.
struct UnitCtl {
  int32_t cur;           // buffer holding the current solution
  int32_t active;        // 0 once a pass applied nothing
  int32_t pass_applied;  // a step of this pass applied a move
  int32_t n_sel;         // moves selected in the current step
  int32_t n_cand;        // follower candidates appended by the evaluation
  int32_t epoch;         // step counter used to tag resources
  int32_t err;           // sticky error bits (1 = candidate overflow, 2 = slot overflow, 4 = length guard)
  int32_t n_slots_alive;
  int32_t fmode;         // pair neighbourhood: 0 full lists, 1 filtered lists, 2 full fallback pass
  int32_t scored_epoch;  // epoch up to which the filtered lists reflect the routes (-1 = none)
  int32_t arena_top;     // first free position of the current buffer (rebuilt routes are appended)
  int32_t rebuild_mode;  // latest step: 0 = rebuilt routes appended in place, 1 = full relayout
  int32_t n_build;       // routes to build in place (mode 0)
  int32_t ftiles_eval;   // pair tiles the latest evaluation in filtered mode covered (its lists' tiles)
  int32_t n_unrouted;    // repair: customers missing from the loaded partial solution
  int32_t n_inserted;    // repair: customers inserted so far
  int64_t F;             // running objective (sum of applied deltas)
  int64_t evaluated;
  int64_t passes, steps, moves_applied;
  int64_t last_eval;     // evaluated moves of the latest step
  int64_t fallbacks;     // full-list fallback passes of a filtered search
  int64_t t_start;       // device clock at the start of the latest search
  int64_t t_end;         // device clock at the end of this unit's latest pass
  int64_t ins_evaluated; // repair: insertion positions evaluated
  MoveRec leader;
};

// Bounds of the dynamic penalty weights (time window, load, duration, depot).
struct AdaptBounds {
  int32_t lo[4], hi[4];
};

struct UnitDesc {
  // instance
  const int32_t *c, *t, *q, *s, *e, *l;
  const int32_t *nbr, *nbr_len;
  const int2* nbr_ct;  // {c(u, v), t(u, v)} of every granular-list slot, beside the list (0 past a list's end)
  // locality layout (null when off): c and t reordered so that nearby nodes have nearby
  // indices (cl[pi[a] * n + pi[b]] = c(a, b)), and the customers in that order
  const int32_t *cl, *tl, *pi, *corder;
  const int4* attr;  // per node {q, s, e, l}
  const int4* dep_arc;  // per (customer, depot) {c(d,x), t(d,x), c(x,d), t(x,d)} at [(x - nd) * nd + d], or null
  int32_t nd, nc, n, theta;
  int32_t Q, NV, Dmax, w_tw, w_load, w_dur;
  int64_t w_depot;
  int32_t R, cap, t_is_c, pad0;
  // solution state
  int32_t *rt, *pos;
  int32_t* apos;  // absolute position of each customer in the current buffer (route offset + pos)
  int32_t *r_len, *r_start, *r_end;
  int32_t *r_off[2];
  int4* r_meta[2];  // per buffer and slot {offset, length, start depot, end depot}
  int4* r_tot;      // {C, Q, D, TW} of every route
  SegTW* r_core;    // time windows: segment of customers 1..L (routes with L <= kCoreMaxL)
  void* fw[2];
  void* bw[2];
  int32_t* ndep;
  UnitCtl* ctl;
  // step scratch
  uint64_t* cand_key;
  uint64_t* cand_id;
  int4* cand_res;
  uint8_t* cand_alive;
  int32_t cand_cap, len_guard;
  uint64_t* resmin;   // [R + nd]
  int32_t* taken;     // [R + nd] epoch tags
  int32_t* dirty;     // [R] epoch tags
  int32_t* plan_n;    // [R] number of pieces of a rebuilt route (0 = deleted)
  int4* plan_pc;      // [R * kMaxPieces] {old offset of the source route, from, to, rev}
  int32_t* slot_list; // [R] alive slots in increasing order
  int32_t* sel_size;  // [R + 1] per selected move: positions its new routes take (then their offsets)
  int32_t* sel_slot;  // [2 (R + 1)] per selected move: slots of its new routes (-1 = none)
  int32_t* build_list;  // [R] routes to build in place
  uint64_t* sel_id;   // [R]
  int64_t* sel_dF;    // [R]
  MoveRec* wg_best;   // [tiles of this unit]
  int32_t tile_base[4];  // first tile of each item class (pairs, dins, drep, end)
  int32_t key_shift;     // bit position of dD in the packed follower key
  int32_t pad1;
  uint32_t* foot;        // footprint bitmap of this unit's instance (measurement launches only)
  // learned move filter
  int32_t* fcand;        // [nc * kc] filtered candidate lists (-1 padding), null when not attached
  int32_t kc, ftiles;    // list length, pair tiles of the filtered item space
  int64_t item_base;     // first anchor of this unit in batch-wide per-anchor arrays
  float frcp[4];         // feature scales: distance, load, time, depot index
};

// ---------------------------------------------------------------------------- segment algebra

__device__ __forceinline__ int32_t imax(int32_t a, int32_t b) { return a > b ? a : b; }
__device__ __forceinline__ int32_t imin(int32_t a, int32_t b) { return a < b ? a : b; }

__device__ __forceinline__ SegNT cat(const SegNT& a, int32_t cab, int32_t tab, const SegNT& b) {
  SegNT r;
  r.C = a.C + cab + b.C;
  r.Q = a.Q + b.Q;
  r.D = a.D + tab + b.D;
  r.node = b.node;
  return r;
}

// Vidal's concatenation of two time-window segments joined by travel time tab.
__device__ __forceinline__ SegTW cat(const SegTW& a, int32_t cab, int32_t tab, const SegTW& b) {
  int32_t delta = a.D - a.TW + tab;
  int32_t wait = imax(b.E - delta - a.L, 0);
  int32_t warp = imax(a.E + delta - b.L, 0);
  SegTW r;
  r.C = a.C + cab + b.C;
  r.Q = a.Q + b.Q;
  r.D = a.D + b.D + tab + wait;
  r.TW = a.TW + b.TW + warp;
  r.E = imax(b.E - delta, a.E) - wait;
  r.L = imin(b.L - delta, a.L) + warp;
  r.node = b.node;
  r.aux = b.aux;
  return r;
}

// Loads of the hot per-unit and per-instance arrays: global address space and a 32-bit
// byte offset from a wave-uniform base, so each is one global load with an SGPR base
// and no 64-bit address arithmetic. Every such array is far below 4 GiB (segment
// buffers, route tables, lists, node attributes); the matrices use ld_mat.
#define MDVRP_GLOBAL __attribute__((address_space(1)))
// (The host pass only type-checks device code and cannot copy vector types out of
// address space 1, hence the plain form there.)
template <class T>
__device__ __forceinline__ T ld(const T* base, uint32_t i) {
#if defined(__HIP_DEVICE_COMPILE__)
  return *(const MDVRP_GLOBAL T*)((const MDVRP_GLOBAL char*)base + i * (uint32_t)sizeof(T));
#else
  return base[i];
#endif
}
// Matrix entry a * n + b: a 24-bit multiply-add (a, n < 2^16); a 32-bit byte offset from
// the (uniform) matrix base while n * n * 4 < 2^32, else a 64-bit address.
__device__ __forceinline__ int32_t ld_mat(const int32_t* m, uint32_t n, int a, int b) {
  const uint32_t i = __umul24((uint32_t)a, n) + (uint32_t)b;
  if (n <= 32767u) return ld(m, i);
  return ((const MDVRP_GLOBAL int32_t*)m)[i];
}

template <class SEG> __device__ __forceinline__ SEG node_seg(const UnitDesc& U, int x);
template <> __device__ __forceinline__ SegNT node_seg<SegNT>(const UnitDesc& U, int x) {
  const int4 a = ld(U.attr, x);
  SegNT r;
  r.C = 0; r.Q = a.x; r.D = a.y; r.node = x;
  return r;
}
template <> __device__ __forceinline__ SegTW node_seg<SegTW>(const UnitDesc& U, int x) {
  const int4 a = ld(U.attr, x);
  SegTW r;
  r.C = 0; r.Q = a.x; r.D = a.y; r.TW = 0; r.E = a.z; r.L = a.w; r.node = x; r.aux = 0;
  return r;
}
__device__ __forceinline__ int32_t service(const UnitDesc& U, int x) { return ld(U.attr, x).y; }

__device__ __forceinline__ int32_t seg_tw(const SegNT&) { return 0; }
__device__ __forceinline__ int32_t seg_tw(const SegTW& s) { return s.TW; }

__device__ __forceinline__ int32_t arc_c(const UnitDesc& U, int a, int b) {
  if (U.pi) return ld_mat(U.cl, U.n, ld(U.pi, a), ld(U.pi, b));
  return ld_mat(U.c, U.n, a, b);
}
__device__ __forceinline__ int32_t arc_t(const UnitDesc& U, int a, int b) {
  if (U.t_is_c) return arc_c(U, a, b);
  if (U.pi) return ld_mat(U.tl, U.n, ld(U.pi, a), ld(U.pi, b));
  return ld_mat(U.t, U.n, a, b);
}

// The arcs between customer x and depot d, {c(d,x), t(d,x), c(x,d), t(x,d)}: one
// 16-byte load from the instance's depot-arc table (contiguous over d for a given x),
// or the matrices when the instance has no table.
__device__ __forceinline__ int4 dep_arcs(const UnitDesc& U, int x, int d) {
  if (U.dep_arc) return ld(U.dep_arc, (uint32_t)((x - U.nd) * U.nd + d));
  const int32_t ci = arc_c(U, d, x), co = arc_c(U, x, d);
  return make_int4(ci, U.t_is_c ? ci : arc_t(U, d, x), co, U.t_is_c ? co : arc_t(U, x, d));
}

// Terms of Eq. A.1 of a complete route from its total segment.
struct RouteTerms {
  int32_t C, TW, LX, DX;
};
template <class SEG>
__device__ __forceinline__ RouteTerms route_terms(const UnitDesc& U, const SEG& s) {
  RouteTerms r;
  r.C = s.C;
  r.TW = seg_tw(s);
  r.LX = imax(s.Q - U.Q, 0);
  r.DX = U.Dmax >= 0 ? imax(s.D - U.Dmax, 0) : 0;
  return r;
}

// dF of a move from the int32 deltas of its cost terms. For given weights Eq. A.1 is
// linear in distance, time warp, load and duration excess and the depot term, so the
// difference of the route costs equals this combination exactly; the evaluators need
// no 64-bit per-route costs. (Every route term stays below 2^30, so the deltas fit int32.)
__device__ __forceinline__ int64_t delta_F(const UnitDesc& U, int32_t dC, int32_t dTW, int32_t dLX, int32_t dDX,
                                           int32_t dV4) {
  return (int64_t)dC + (int64_t)U.w_tw * dTW + (int64_t)U.w_load * dLX + (int64_t)U.w_dur * dDX +
         U.w_depot * (int64_t)dV4;
}

// ---------------------------------------------------------------------------- move recipes
//
// A move replaces one or two routes by one or two new routes, each described
// as start depot + up to five pieces (customer position ranges of the current
// routes, possibly reversed) + end depot. The same recipe drives the
// evaluation (cost of the new routes from segments) and the apply step
// (materialising the new routes).

struct Piece {
  int8_t src;   // which context route (0 = A, 1 = B)
  int8_t rev;
  int16_t pad;
  int32_t from, to;  // inclusive customer positions (1..L)
};

struct RouteCtx {
  int32_t slot, off, L, start, end;
};

struct Recipe {
  int32_t nnew;        // new routes (1 or 2)
  int32_t nold;        // old routes replaced (1 or 2), context order
  int32_t fresh;       // 1: new route 1 goes to a free slot (Depot-Insert)
  int32_t st[2], en[2];
  int32_t np[2];
  Piece pc[2][kMaxPieces];
};

__device__ __forceinline__ void rc_add(Recipe& R, int w, int src, int from, int to, int rev) {
  if (from > to) return;
  Piece p;
  p.src = (int8_t)src;
  p.rev = (int8_t)rev;
  p.pad = 0;
  p.from = from;
  p.to = to;
  // stores at static indices only, so that a recipe can live in registers
  const int k = R.np[w]++;
#pragma unroll
  for (int j = 0; j < kMaxPieces; ++j)
    if (j == k) R.pc[w][j] = p;
}

// Relocate: block [xa, xb] of A (placed reversed when xrev) goes in front of position pv of B.
__device__ __forceinline__ void rc_rel(Recipe& R, const RouteCtx& A, const RouteCtx& B, bool intra, int xa,
                                       int xb, int xrev, int pv) {
  R.np[0] = R.np[1] = 0;
  R.fresh = 0;
  R.st[0] = A.start; R.en[0] = A.end;
  if (!intra) {
    R.nnew = R.nold = 2;
    rc_add(R, 0, 0, 1, xa - 1, 0);
    rc_add(R, 0, 0, xb + 1, A.L, 0);
    R.st[1] = B.start; R.en[1] = B.end;
    rc_add(R, 1, 1, 1, pv - 1, 0);
    rc_add(R, 1, 0, xa, xb, xrev);
    rc_add(R, 1, 1, pv, B.L, 0);
  } else {
    R.nnew = R.nold = 1;
    if (pv < xa) {
      rc_add(R, 0, 0, 1, pv - 1, 0);
      rc_add(R, 0, 0, xa, xb, xrev);
      rc_add(R, 0, 0, pv, xa - 1, 0);
      rc_add(R, 0, 0, xb + 1, A.L, 0);
    } else {
      rc_add(R, 0, 0, 1, xa - 1, 0);
      rc_add(R, 0, 0, xb + 1, pv - 1, 0);
      rc_add(R, 0, 0, xa, xb, xrev);
      rc_add(R, 0, 0, pv, A.L, 0);
    }
  }
}

// Swap: block X = [xa, xb] of A goes to Y's place, block Y = [ya, yb] of B to X's place.
__device__ __forceinline__ void rc_swp(Recipe& R, const RouteCtx& A, const RouteCtx& B, bool intra, int xa,
                                       int xb, int xrev, int ya, int yb, int yrev) {
  R.np[0] = R.np[1] = 0;
  R.fresh = 0;
  R.st[0] = A.start; R.en[0] = A.end;
  if (!intra) {
    R.nnew = R.nold = 2;
    rc_add(R, 0, 0, 1, xa - 1, 0);
    rc_add(R, 0, 1, ya, yb, yrev);
    rc_add(R, 0, 0, xb + 1, A.L, 0);
    R.st[1] = B.start; R.en[1] = B.end;
    rc_add(R, 1, 1, 1, ya - 1, 0);
    rc_add(R, 1, 0, xa, xb, xrev);
    rc_add(R, 1, 1, yb + 1, B.L, 0);
  } else {
    R.nnew = R.nold = 1;
    if (xa < ya) {
      rc_add(R, 0, 0, 1, xa - 1, 0);
      rc_add(R, 0, 0, ya, yb, yrev);
      rc_add(R, 0, 0, xb + 1, ya - 1, 0);
      rc_add(R, 0, 0, xa, xb, xrev);
      rc_add(R, 0, 0, yb + 1, A.L, 0);
    } else {
      rc_add(R, 0, 0, 1, ya - 1, 0);
      rc_add(R, 0, 0, xa, xb, xrev);
      rc_add(R, 0, 0, yb + 1, xa - 1, 0);
      rc_add(R, 0, 0, ya, yb, yrev);
      rc_add(R, 0, 0, xb + 1, A.L, 0);
    }
  }
}

// X block of u for two-node kinds: o = 0 takes (p(u), u) as is; o = 1 takes (u, s(u))
// and places it as (s(u), u). Returns false when the block does not exist.
__device__ __forceinline__ bool x_block(const RouteCtx& A, int pu, int o, int& xa, int& xb, int& xrev) {
  if (o == 0) {
    if (pu < 2) return false;
    xa = pu - 1; xb = pu; xrev = 0;
  } else {
    if (pu + 1 > A.L) return false;
    xa = pu; xb = pu + 1; xrev = 1;
  }
  return true;
}

// Pair move anchored on u (position pu of A) and v (position pv of B); every pair
// move creates the arc u -> v (Section 3.2.2 operators on granular lists, Section 3.2.3).
__device__ __forceinline__ bool build_pair(int kind, int var, const RouteCtx& A, int pu, const RouteCtx& B,
                                           int pv, bool intra, bool sym, Recipe& R) {
  int xa, xb, xrev, ya, yb;
  switch (kind) {
    case REL1:
      if (var != 0) return false;
      if (intra && pv == pu + 1) return false;
      rc_rel(R, A, B, intra, pu, pu, 0, pv);
      return true;
    case REL2:
      if (var > 1 || (var == 1 && !sym)) return false;
      if (!x_block(A, pu, var, xa, xb, xrev)) return false;
      if (intra && ((pv >= xa && pv <= xb) || pv == pu + 1)) return false;
      rc_rel(R, A, B, intra, xa, xb, xrev, pv);
      return true;
    case SWP11:
      if (var != 0) return false;
      if (pv < 2 || (intra && pv - 1 == pu)) return false;
      rc_swp(R, A, B, intra, pu, pu, 0, pv - 1, pv - 1, 0);
      return true;
    case SWP21:
      if (var > 1 || (var == 1 && !sym)) return false;
      if (!x_block(A, pu, var, xa, xb, xrev)) return false;
      if (pv < 2) return false;
      ya = yb = pv - 1;
      if (intra && ((ya >= xa && ya <= xb) || (pv >= xa && pv <= xb))) return false;
      rc_swp(R, A, B, intra, xa, xb, xrev, ya, yb, 0);
      return true;
    case SWP12:
      if (var > 1 || (var == 1 && !sym)) return false;
      if (pv < 3) return false;
      ya = pv - 2; yb = pv - 1;
      if (intra && pu >= ya && pu <= yb) return false;
      rc_swp(R, A, B, intra, pu, pu, 0, ya, yb, var);
      return true;
    case SWP22: {
      if (var > 3) return false;
      int ox = var & 1, oy = var >> 1;
      if ((ox || oy) && !sym) return false;
      if (!x_block(A, pu, ox, xa, xb, xrev)) return false;
      if (pv < 3) return false;
      ya = pv - 2; yb = pv - 1;
      if (intra && ((ya <= xb && xa <= yb) || (pv >= xa && pv <= xb))) return false;
      rc_swp(R, A, B, intra, xa, xb, xrev, ya, yb, oy);
      return true;
    }
    case X2:
      // 2-opt*: A' = A[..u] + B[v..] ending at B's depot, B' = B[..p(v)] + A[s(u)..] ending at A's.
      if (var != 0 || intra) return false;
      R.nnew = R.nold = 2;
      R.fresh = 0;
      R.np[0] = R.np[1] = 0;
      R.st[0] = A.start; R.en[0] = B.end;
      rc_add(R, 0, 0, 1, pu, 0);
      rc_add(R, 0, 1, pv, B.L, 0);
      R.st[1] = B.start; R.en[1] = A.end;
      rc_add(R, 1, 1, 1, pv - 1, 0);
      rc_add(R, 1, 0, pu + 1, A.L, 0);
      return true;
    case TWOOPT:
      // 2-opt: reverse positions pu+1..pv of one route (creates u -> v and s(u) -> s(v)).
      if (var != 0 || !intra || !sym || !(pu < pv - 1)) return false;
      R.nnew = R.nold = 1;
      R.fresh = 0;
      R.np[0] = R.np[1] = 0;
      R.st[0] = A.start; R.en[0] = A.end;
      rc_add(R, 0, 0, 1, pu, 0);
      rc_add(R, 0, 0, pu + 1, pv, 1);
      rc_add(R, 0, 0, pv + 1, A.L, 0);
      return true;
    default:
      return false;
  }
}

// Depot-Insert (Fig. 1a): cut after position pu and insert depot d between the parts.
__device__ __forceinline__ void build_dins(const RouteCtx& A, int pu, int d, bool open, Recipe& R) {
  R.nnew = 2; R.nold = 1; R.fresh = 1;
  R.np[0] = R.np[1] = 0;
  R.st[0] = A.start; R.en[0] = open ? -1 : d;
  rc_add(R, 0, 0, 1, pu, 0);
  R.st[1] = d; R.en[1] = A.end;
  rc_add(R, 1, 0, pu + 1, A.L, 0);
}

// Depot-Replace (Fig. 1b): case 0 departure depot, 1 arrival depot, 2 both.
__device__ __forceinline__ void build_drep(const RouteCtx& A, int d, int cs, Recipe& R) {
  R.nnew = 1; R.nold = 1; R.fresh = 0;
  R.np[0] = R.np[1] = 0;
  R.st[0] = (cs == 0 || cs == 2) ? d : A.start;
  R.en[0] = (cs == 1 || cs == 2) ? d : A.end;
  rc_add(R, 0, 0, 1, A.L, 0);
}

__device__ __forceinline__ uint64_t make_id(int kind, int var, int a, int b) {
  return ((uint64_t)kind << 56) | ((uint64_t)var << 48) | ((uint64_t)a << 24) | (uint64_t)b;
}

// ---------------------------------------------------------------------------- wave helpers

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Segment shuffles within groups of W lanes (W = 64: the whole wavefront; W = 32: each
// half builds a route of its own).
template <class T, int W = 64> __device__ __forceinline__ T shfl_up_seg(const T& v, int off);
template <> __device__ __forceinline__ SegNT shfl_up_seg<SegNT, 64>(const SegNT& v, int off) {
  SegNT r;
  r.C = __shfl_up(v.C, off); r.Q = __shfl_up(v.Q, off); r.D = __shfl_up(v.D, off);
  r.node = __shfl_up(v.node, off);
  return r;
}
template <> __device__ __forceinline__ SegNT shfl_up_seg<SegNT, 32>(const SegNT& v, int off) {
  SegNT r;
  r.C = __shfl_up(v.C, off, 32); r.Q = __shfl_up(v.Q, off, 32); r.D = __shfl_up(v.D, off, 32);
  r.node = __shfl_up(v.node, off, 32);
  return r;
}
template <> __device__ __forceinline__ SegTW shfl_up_seg<SegTW, 64>(const SegTW& v, int off) {
  SegTW r;
  r.C = __shfl_up(v.C, off); r.Q = __shfl_up(v.Q, off); r.D = __shfl_up(v.D, off);
  r.TW = __shfl_up(v.TW, off); r.E = __shfl_up(v.E, off); r.L = __shfl_up(v.L, off);
  r.node = __shfl_up(v.node, off); r.aux = __shfl_up(v.aux, off);
  return r;
}
template <> __device__ __forceinline__ SegTW shfl_up_seg<SegTW, 32>(const SegTW& v, int off) {
  SegTW r;
  r.C = __shfl_up(v.C, off, 32); r.Q = __shfl_up(v.Q, off, 32); r.D = __shfl_up(v.D, off, 32);
  r.TW = __shfl_up(v.TW, off, 32); r.E = __shfl_up(v.E, off, 32); r.L = __shfl_up(v.L, off, 32);
  r.node = __shfl_up(v.node, off, 32); r.aux = __shfl_up(v.aux, off, 32);
  return r;
}
template <class T, int W = 64> __device__ __forceinline__ T shfl_down_seg(const T& v, int off);
template <> __device__ __forceinline__ SegNT shfl_down_seg<SegNT, 64>(const SegNT& v, int off) {
  SegNT r;
  r.C = __shfl_down(v.C, off); r.Q = __shfl_down(v.Q, off); r.D = __shfl_down(v.D, off);
  r.node = __shfl_down(v.node, off);
  return r;
}
template <> __device__ __forceinline__ SegNT shfl_down_seg<SegNT, 32>(const SegNT& v, int off) {
  SegNT r;
  r.C = __shfl_down(v.C, off, 32); r.Q = __shfl_down(v.Q, off, 32); r.D = __shfl_down(v.D, off, 32);
  r.node = __shfl_down(v.node, off, 32);
  return r;
}
template <> __device__ __forceinline__ SegTW shfl_down_seg<SegTW, 64>(const SegTW& v, int off) {
  SegTW r;
  r.C = __shfl_down(v.C, off); r.Q = __shfl_down(v.Q, off); r.D = __shfl_down(v.D, off);
  r.TW = __shfl_down(v.TW, off); r.E = __shfl_down(v.E, off); r.L = __shfl_down(v.L, off);
  r.node = __shfl_down(v.node, off); r.aux = __shfl_down(v.aux, off);
  return r;
}
template <> __device__ __forceinline__ SegTW shfl_down_seg<SegTW, 32>(const SegTW& v, int off) {
  SegTW r;
  r.C = __shfl_down(v.C, off, 32); r.Q = __shfl_down(v.Q, off, 32); r.D = __shfl_down(v.D, off, 32);
  r.TW = __shfl_down(v.TW, off, 32); r.E = __shfl_down(v.E, off, 32); r.L = __shfl_down(v.L, off, 32);
  r.node = __shfl_down(v.node, off, 32); r.aux = __shfl_down(v.aux, off, 32);
  return r;
}
template <class T, int W = 64> __device__ __forceinline__ T shfl_seg(const T& v, int src);
template <> __device__ __forceinline__ SegNT shfl_seg<SegNT, 64>(const SegNT& v, int src) {
  SegNT r;
  r.C = __shfl(v.C, src); r.Q = __shfl(v.Q, src); r.D = __shfl(v.D, src); r.node = __shfl(v.node, src);
  return r;
}
template <> __device__ __forceinline__ SegNT shfl_seg<SegNT, 32>(const SegNT& v, int src) {
  SegNT r;
  r.C = __shfl(v.C, src, 32); r.Q = __shfl(v.Q, src, 32); r.D = __shfl(v.D, src, 32);
  r.node = __shfl(v.node, src, 32);
  return r;
}
template <> __device__ __forceinline__ SegTW shfl_seg<SegTW, 64>(const SegTW& v, int src) {
  SegTW r;
  r.C = __shfl(v.C, src); r.Q = __shfl(v.Q, src); r.D = __shfl(v.D, src);
  r.TW = __shfl(v.TW, src); r.E = __shfl(v.E, src); r.L = __shfl(v.L, src);
  r.node = __shfl(v.node, src); r.aux = __shfl(v.aux, src);
  return r;
}
template <> __device__ __forceinline__ SegTW shfl_seg<SegTW, 32>(const SegTW& v, int src) {
  SegTW r;
  r.C = __shfl(v.C, src, 32); r.Q = __shfl(v.Q, src, 32); r.D = __shfl(v.D, src, 32);
  r.TW = __shfl(v.TW, src, 32); r.E = __shfl(v.E, src, 32); r.L = __shfl(v.L, src, 32);
  r.node = __shfl(v.node, src, 32); r.aux = __shfl(v.aux, src, 32);
  return r;
}

// Exclusive scan of one int per thread over a block of NT threads (NT multiple of
// 64, at most 4096); sh must hold 2*NT/64+1 ints. Returns the block total in *total.
template <int NT>
__device__ __forceinline__ int block_scan_excl(int v, int* sh, int* total) {
  constexpr int NW = NT / 64;
  const int lane = __lane_id(), wave = threadIdx.x >> 6;
  int incl = v;
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(incl, off);
    if (lane >= off) incl += y;
  }
  if (lane == 63) sh[wave] = incl;
  __syncthreads();
  if (wave == 0) {
    const int w = lane < NW ? sh[lane] : 0;
    int wi = w;
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(wi, off);
      if (lane >= off) wi += y;
    }
    if (lane < NW) sh[NW + lane] = wi - w;
    if (lane == NW - 1) sh[2 * NW] = wi;
  }
  __syncthreads();
  const int r = sh[NW + wave] + incl - v;
  *total = sh[2 * NW];
  __syncthreads();
  return r;
}

// SplitMix64 (Steele, Lea and Flood, 2014): the pass order of Algorithm 2 and the
// random insertion draw from it, on the host and on the device.
__host__ __device__ inline uint64_t splitmix64_next(uint64_t* st) {
  uint64_t z = (*st += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Lexicographic (dF, id) order of move keys.
__device__ __forceinline__ bool key_less(int64_t f1, uint64_t i1, int64_t f2, uint64_t i2) {
  return f1 < f2 || (f1 == f2 && i1 < i2);
}

// Active map of one pass of the local search, written by k_pass_begin: word 0 holds
// the number of active units n_act, words 1 .. kActGrids the active tile count of
// each grid, then n_units words the active units' indices in ascending order, then
// for each grid n_units + 1 prefix offsets of the active units' tile counts (the
// first n_act + 1 are valid). Grids: 0 pair tiles, 1 Depot-Insert tiles, 2
// Depot-Replace tiles, 3 blocks of the filtered pair grid, 4 blocks of the compact
// Depot-Replace grid.
constexpr int kActGrids = 5;
constexpr int kActUnits = 1 + kActGrids;  // first word of the unit list
__host__ __device__ constexpr int64_t act_map_words(int n_units) {
  return kActUnits + (int64_t)n_units + (int64_t)kActGrids * (n_units + 1);
}
__host__ __device__ constexpr int64_t act_off_word(int n_units, int g) {
  return kActUnits + (int64_t)n_units + (int64_t)g * (n_units + 1);
}

// The tile of this block among T tiles, for a grid of at least T blocks: the tiles are
// split into 8 contiguous ranges, one per XCD (blocks are dispatched round-robin over
// the 8 XCDs: block b runs on XCD b % 8); range x holds T / 8 tiles plus one for
// x < T % 8 and its tiles go to the blocks of XCD x in order. -1: the block has none
// (with exactly T blocks every block has one).
__device__ __forceinline__ int block_tile(int T) {
  const int b = (int)blockIdx.x, x = b & 7, k = b >> 3, per = T >> 3, rem = T & 7;
  const int len = per + (x < rem ? 1 : 0);
  return k < len ? x * per + (x < rem ? x : rem) + k : -1;
}

// Find the unit of a tile by binary search over per-unit tile offsets.
__device__ __forceinline__ int unit_of_tile(const int32_t* off, int n_units, int tile) {
  int lo = 0, hi = n_units;  // off[lo] <= tile < off[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (off[mid] <= tile) lo = mid; else hi = mid;
  }
  return lo;
}

// Unit and local tile of tile t of a grid whose n units have the tile offsets off
// (n + 1 prefix sums): with equal tile counts (per_unit > 0) tile t is local tile
// t / n of the (t % n)-th unit (an XCD then serves the same customers of every unit,
// whose matrix rows stay in its L2); otherwise the units' tiles follow one another.
// The k-th unit is list[k], or k itself without a list.
__device__ __forceinline__ void map_tile(const int32_t* __restrict__ off, int n, int per_unit,
                                         const int32_t* __restrict__ list, int t, int& ui, int& lt) {
  int k;
  if (per_unit > 0) {
    k = t % n;
    lt = t / n;
  } else {
    k = unit_of_tile(off, n, t);
    lt = t - off[k];
  }
  ui = list ? list[k] : k;
}

// The units, tile offsets and tile count of grid g of a launch: the active units of
// the pass when the launch has an active map, else every unit of the batch.
struct GridView {
  const int32_t* off;
  const int32_t* list;
  int n, T;
};
__device__ __forceinline__ GridView grid_view(const int32_t* __restrict__ act, int n_units, int g,
                                              const int32_t* __restrict__ all_off) {
  GridView v;
  if (act) {
    v.n = act[0];
    v.T = act[1 + g];
    v.off = act + act_off_word(n_units, g);
    v.list = v.n < n_units ? act + kActUnits : nullptr;
  } else {
    v.n = n_units;
    v.T = (int)gridDim.x;
    v.off = all_off;
    v.list = nullptr;
  }
  return v;
}

}  // namespace mdvrp
