"""Brute-force reference used to pin the oracle on tiny instances.

Independent of the oracle's C code: time warp and duration come from
enumerating every integer departure time, F(S) is recomputed over the whole
solution, and every neighbour is built with Python list surgery.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


# ----------------------------------------------------------------------------- routes

def schedule(inst, start, xs, end, tau):
    """Forward simulation departing the start depot at tau.

    Early arrival waits until e_k; late arrival warps back to l_k (cost = lateness).
    Returns (time warp, duration = elapsed + warp)."""
    T = tau + int(inst.s[start])
    warp = 0
    prev = start
    seq = list(xs) + ([end] if end >= 0 else [])
    for k in seq:
        A = T + int(inst.t[prev, k])
        if A < int(inst.e[k]):
            T = int(inst.e[k])
        elif A > int(inst.l[k]):
            warp += A - int(inst.l[k])
            T = int(inst.l[k])
        else:
            T = A
        T += int(inst.s[k])
        prev = k
    return warp, (T - tau) + warp


def tw_dur(inst, start, xs, end):
    """(time warp, duration): lexicographic minimum over integer departures in the depot window.

    Same simulation as schedule(), vectorised over every departure time."""
    if not inst.has_tw:
        prev, dur = start, int(inst.s[start])
        for k in list(xs) + ([end] if end >= 0 else []):
            dur += int(inst.t[prev, k]) + int(inst.s[k])
            prev = k
        return 0, dur
    tau = np.arange(int(inst.e[start]), int(inst.l[start]) + 1, dtype=np.int64)
    T = tau + int(inst.s[start])
    warp = np.zeros_like(tau)
    prev = start
    for k in list(xs) + ([end] if end >= 0 else []):
        A = T + int(inst.t[prev, k])
        ek, lk = int(inst.e[k]), int(inst.l[k])
        warp = warp + np.maximum(A - lk, 0)
        T = np.clip(A, ek, lk) + int(inst.s[k])
        prev = k
    dur = (T - tau) + warp
    order = np.lexsort((dur, warp))
    return int(warp[order[0]]), int(dur[order[0]])


_CACHE = {}
_TOKENS = iter(range(1 << 62))


def _token(inst):
    tok = getattr(inst, "_t0_token", None)
    if tok is None:
        tok = next(_TOKENS)
        inst._t0_token = tok
    return tok


def route_terms(inst, route):
    key = (_token(inst), route[0], tuple(route[1]), route[2])
    if key in _CACHE:
        return _CACHE[key]
    _CACHE[key] = v = _route_terms(inst, route)
    return v


def _route_terms(inst, route):
    a, xs, b = route
    if inst.open_routes:
        b = -1
    seq = [a] + list(xs) + ([b] if b >= 0 else [])
    dist = sum(int(inst.c[seq[k], seq[k + 1]]) for k in range(len(seq) - 1))
    load = sum(int(inst.q[x]) for x in xs)
    tw, dur = tw_dur(inst, a, xs, b)
    lx = max(load - inst.Q, 0)
    dx = max(dur - inst.Dmax, 0) if inst.Dmax >= 0 else 0
    return dict(dist=dist, load=load, tw=tw, dur=dur, lx=lx, dx=dx)


def theta_norm(inst):
    import numpy as np
    n = inst.N
    off = ~np.eye(n, dtype=bool)
    return 2 * int(inst.c[off].max()) - int(inst.c[off].min())


def w_depot(inst):
    return theta_norm(inst) if inst.w_depot < 0 else inst.w_depot


def F_terms(inst, routes):
    """Whole-solution F of Eq. A.1 with fixed weights; returns (F, dict of terms)."""
    D = TW = LX = DX = CL = 0
    cost = 0
    cnt = [0] * inst.n_depots
    for r in routes:
        a, xs, b = r
        if not xs:
            continue
        t = route_terms(inst, r)
        D += t["dist"]; TW += t["tw"]; LX += t["lx"]; DX += t["dx"]
        cost += t["dist"] + inst.w_tw * t["tw"] + inst.w_load * t["lx"] + inst.w_dur * t["dx"]
        if not inst.open_routes and a != b:
            CL += 1
        cnt[a] += 1
    FX = sum(max(n - inst.NV, 0) for n in cnt)
    return cost + w_depot(inst) * (CL + FX), dict(D=D, TW=TW, LX=LX, DX=DX, CL=CL, FX=FX)


# ----------------------------------------------------------------------------- granular lists

def neighbour_lists(inst):
    """theta customers per customer by eta (Eq. 3) with exact fractions; ties -> lower id."""
    nd, n = inst.n_depots, inst.N
    sc = sum(int(inst.c[a, b]) for a in range(n) for b in range(n) if a != b)
    st = sum(int(inst.t[a, b]) for a in range(n) for b in range(n) if a != b)
    gamma = Fraction(sc, st) if st else Fraction(1)
    out = {}
    for u in range(nd, n):
        cand = []
        for v in range(nd, n):
            if v == u:
                continue
            if inst.has_tw:
                tij = int(inst.t[u, v])
                if int(inst.e[u]) + int(inst.s[u]) + tij > int(inst.l[v]):
                    continue
                early = max(int(inst.e[v]) - int(inst.l[u]) - int(inst.s[u]) - tij, 0)
                late = max(int(inst.l[u]) + int(inst.s[u]) + tij - int(inst.l[v]), 0)
                eta = int(inst.c[u, v]) + gamma * (1 * early + 10 * late)
            else:
                eta = Fraction(int(inst.c[u, v]))
            cand.append((eta, v))
        cand.sort()
        out[u] = [v for _, v in cand[:inst.theta]]
    return out


# ----------------------------------------------------------------------------- neighbourhood

KIND = dict(REL1=0, REL2=1, SWP11=2, SWP21=3, SWP12=4, SWP22=5, X2=6, TWOOPT=7, DINS=8, DREP=9)


def mk_id(kind, var, a, b):
    return (int(kind) << 56) | (int(var) << 48) | (int(a) << 24) | int(b)


def _expand(tokens, table):
    out = []
    for t in tokens:
        out.extend(table[t] if isinstance(t, str) else [t])
    return out


def pair_moves(inst, routes, u, v):
    """All (kind, variant) -> list of (old route index -> new route) for anchor (u, v).

    Built with marker substitution on Python lists: the moved blocks are
    replaced by markers, then the markers are expanded to the other block."""
    sym = not inst.has_tw
    loc = {}
    for ri, (a, xs, b) in enumerate(routes):
        for k, x in enumerate(xs):
            loc[x] = (ri, k)
    ra, i = loc[u]
    rb, j = loc[v]
    A = routes[ra][1]
    B = routes[rb][1]
    intra = ra == rb
    res = {}

    def blocks_u():  # orientation -> (indices in A, placement)
        bl = {}
        if i >= 1:
            bl[0] = ([i - 1, i], [A[i - 1], A[i]])
        if sym and i + 1 < len(A):
            bl[1] = ([i, i + 1], [A[i + 1], A[i]])
        return bl

    def rel(xidx, xplace):
        if intra:
            if v in [A[k] for k in xidx]:
                return None
            toks = [x for k, x in enumerate(A) if k not in xidx]
            p = toks.index(v)
            new = toks[:p] + xplace + toks[p:]
            if new == A:
                return None
            return {ra: (routes[ra][0], new, routes[ra][2])}
        na = [x for k, x in enumerate(A) if k not in xidx]
        p = B.index(v)
        nb = B[:p] + xplace + B[p:]
        return {ra: (routes[ra][0], na, routes[ra][2]), rb: (routes[rb][0], nb, routes[rb][2])}

    def swp(xidx, xplace, yidx, yplace):
        if intra:
            if set(xidx) & set(yidx) or A.index(v) in xidx:
                return None
            toks = []
            for k, x in enumerate(A):
                if k == xidx[0]:
                    toks.append("X")
                elif k == yidx[0]:
                    toks.append("Y")
                elif k in xidx or k in yidx:
                    continue
                else:
                    toks.append(x)
            new = _expand(toks, {"X": yplace, "Y": xplace})
            return {ra: (routes[ra][0], new, routes[ra][2])}
        ta = ["X" if k == xidx[0] else x for k, x in enumerate(A) if k == xidx[0] or k not in xidx]
        tb = ["Y" if k == yidx[0] else x for k, x in enumerate(B) if k == yidx[0] or k not in yidx]
        return {ra: (routes[ra][0], _expand(ta, {"X": yplace}), routes[ra][2]),
                rb: (routes[rb][0], _expand(tb, {"Y": xplace}), routes[rb][2])}

    # Relocate of one node
    m = rel([i], [u])
    if m is not None:
        res[(KIND["REL1"], 0)] = m
    # Relocate of two nodes
    for o, (xi, xp) in blocks_u().items():
        m = rel(xi, xp)
        if m is not None:
            res[(KIND["REL2"], o)] = m
    # Swaps; Y blocks end immediately before v
    ys1 = ([j - 1], [B[j - 1]]) if j >= 1 else None
    ys2 = {}
    if j >= 2:
        ys2[0] = ([j - 2, j - 1], [B[j - 2], B[j - 1]])
        if sym:
            ys2[1] = ([j - 2, j - 1], [B[j - 1], B[j - 2]])
    if ys1 is not None and B[j - 1] != u:
        m = swp([i], [u], ys1[0], ys1[1])
        if m is not None:
            res[(KIND["SWP11"], 0)] = m
    for o, (xi, xp) in blocks_u().items():
        if ys1 is not None:
            m = swp(xi, xp, ys1[0], ys1[1])
            if m is not None:
                res[(KIND["SWP21"], o)] = m
        for oy, (yi, yp) in ys2.items():
            m = swp(xi, xp, yi, yp)
            if m is not None:
                res[(KIND["SWP22"], o + 2 * oy)] = m
    for oy, (yi, yp) in ys2.items():
        if intra and i in yi:
            continue
        m = swp([i], [u], yi, yp)
        if m is not None:
            res[(KIND["SWP12"], oy)] = m
    # 2-opt*
    if not intra:
        a_s, _, a_e = routes[ra]
        b_s, _, b_e = routes[rb]
        res[(KIND["X2"], 0)] = {ra: (a_s, A[:i + 1] + B[j:], b_e), rb: (b_s, B[:j] + A[i + 1:], a_e)}
    # 2-opt
    if intra and sym and i < j - 1:
        new = A[:i + 1] + list(reversed(A[i + 1:j + 1])) + A[j + 1:]
        res[(KIND["TWOOPT"], 0)] = {ra: (routes[ra][0], new, routes[ra][2])}
    return res


def family_of_kind(k):
    return {0: 0, 1: 0, 2: 1, 3: 1, 4: 1, 5: 1, 6: 2, 7: 3, 8: 4, 9: 5}[k]


def apply_change(routes, change, extra=()):
    out = []
    for ri, r in enumerate(routes):
        if ri in change:
            if change[ri] is not None and change[ri][1]:
                out.append(change[ri])
        else:
            out.append(r)
    out.extend(r for r in extra if r[1])
    return out


def all_neighbours(inst, routes, fam_mask=0x3F, nbrs=None):
    """id -> neighbour routes for every move of the families in fam_mask."""
    nd = inst.n_depots
    nbrs = nbrs if nbrs is not None else neighbour_lists(inst)
    out = {}
    open_r = inst.open_routes
    for u in range(nd, inst.N):
        for v in nbrs[u]:
            for (kind, var), ch in pair_moves(inst, routes, u, v).items():
                if not fam_mask >> family_of_kind(kind) & 1:
                    continue
                out[mk_id(kind, var, u, v)] = apply_change(routes, ch)
    if fam_mask >> 4 & 1:
        for ri, (a, xs, b) in enumerate(routes):
            for k in range(len(xs) - 1):
                for d in range(nd):
                    r1 = (a, xs[:k + 1], -1 if open_r else d)
                    r2 = (d, xs[k + 1:], b)
                    out[mk_id(8, 0, xs[k], d)] = apply_change(routes, {ri: r1}, [r2])
    return out


def drep_candidates(inst, routes):
    """(route index, depot) -> list of (case, new route) after dropping identities and duplicates."""
    out = {}
    for ri, (a, xs, b) in enumerate(routes):
        for d in range(inst.n_depots):
            seen = []
            cases = []
            for cs in range(3):
                if inst.open_routes and cs != 0:
                    continue
                ns = d if cs in (0, 2) else a
                ne = d if cs in (1, 2) else b
                if (ns, ne) == (a, b) or (ns, ne) in seen:
                    continue
                seen.append((ns, ne))
                cases.append((cs, (ns, xs, ne)))
            if cases:
                out[(ri, d)] = cases
    return out


def greedy(moves, leader_only=False):
    """Leader + conflict-free followers in ascending (dF, id) order (Section 3.2.5)."""
    order = sorted(range(len(moves)), key=lambda k: (int(moves[k]["dF"]), int(moves[k]["id"])))
    if not order or int(moves[order[0]]["dF"]) >= 0:
        return []
    sel = [order[0]]
    if leader_only:
        return sel
    used = set(int(r) for r in moves[order[0]]["res"] if r != -1)
    for k in order[1:]:
        m = moves[k]
        if not (m["dD"] < 0 and m["dTW"] == 0 and m["dLX"] == 0 and m["dDX"] == 0 and m["dV4"] == 0):
            continue
        rs = set(int(r) for r in m["res"] if r != -1)
        if rs & used:
            continue
        sel.append(k)
        used |= rs
    return sel
