"""Seeded synthetic instances and start solutions for the MDVRP local-search path.

This module only synthesises inputs. It holds none of the method's arithmetic
(no route cost, no time warp, no move evaluation): both the HIP path and the
CPU oracle consume what it produces.

Instances follow the problem statement of the paper (Section 1): depots take
ids [0, n_depots), customers take [n_depots, N); c and t are symmetric integer
matrices, q is the demand, s the service time, [e, l] the time window, Q the
vehicle capacity, NV the fleet per depot and Dmax the route-duration limit.

Distances and times are int32 fixed point: c = t = floor(scale * Euclid + 1/2)
with scale = 10 (tenths of a coordinate unit). The paper's benchmark files are
not available; the workloads below are stand-ins with the shapes of its suites
(see the workload table in the design notes).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BIG_HORIZON = 1_000_000_000  # window end used when an instance has no time windows


@dataclass
class Instance:
    n_depots: int
    n_customers: int
    c: np.ndarray  # (N, N) int32, row-major
    t: np.ndarray  # (N, N) int32 (may be the same object as c)
    q: np.ndarray  # (N,) int32
    s: np.ndarray  # (N,) int32
    e: np.ndarray  # (N,) int32
    l: np.ndarray  # (N,) int32
    Q: int
    NV: int
    Dmax: int  # < 0: no duration limit
    open_routes: int
    has_tw: int
    theta: int
    w_tw: int = 0
    w_load: int = 10
    w_dur: int = 0
    w_depot: int = -1  # < 0: use 2*max c - min c
    name: str = ""
    seed: int = 0
    coords: np.ndarray | None = field(default=None, repr=False)

    @property
    def N(self) -> int:
        return self.n_depots + self.n_customers


@dataclass
class Solution:
    """Routes as (start depot, [customers...], end depot or -1 when open)."""
    routes: list

    def flat(self):
        """Flat arrays: nodes, offsets[R+1], start[R], end[R]."""
        nodes, offs, st, en = [], [0], [], []
        for (a, xs, b) in self.routes:
            nodes.extend(xs)
            offs.append(len(nodes))
            st.append(a)
            en.append(b)
        return (np.asarray(nodes, np.int32), np.asarray(offs, np.int32),
                np.asarray(st, np.int32), np.asarray(en, np.int32))


def canonical(routes):
    """Routes sorted by (start depot, first customer); used to compare solutions."""
    return sorted(((int(a), tuple(int(x) for x in xs), int(b)) for (a, xs, b) in routes),
                  key=lambda r: (r[0], r[1][0] if r[1] else -1, r[1], r[2]))


def solutions_from_flat(nodes, offs, st, en, sol_offs):
    out = []
    for k in range(len(sol_offs) - 1):
        rs = []
        for r in range(int(sol_offs[k]), int(sol_offs[k + 1])):
            rs.append((int(st[r]), [int(x) for x in nodes[offs[r]:offs[r + 1]]], int(en[r])))
        out.append(Solution(rs))
    return out


def batch_flat(solutions):
    """Concatenate solutions: nodes, route offsets, starts, ends, solution route offsets."""
    nodes, offs, st, en, so = [], [0], [], [], [0]
    for sol in solutions:
        for (a, xs, b) in sol.routes:
            nodes.extend(xs)
            offs.append(len(nodes))
            st.append(a)
            en.append(b)
        so.append(len(st))
    return (np.asarray(nodes, np.int32), np.asarray(offs, np.int32), np.asarray(st, np.int32),
            np.asarray(en, np.int32), np.asarray(so, np.int32))


# ----------------------------------------------------------------------------- distances

def _dist_matrix(xy: np.ndarray, scale: int) -> np.ndarray:
    """floor(scale*sqrt(dx^2+dy^2) + 0.5) in int32, computed in row blocks."""
    n = xy.shape[0]
    out = np.empty((n, n), dtype=np.int32)
    xyf = xy.astype(np.float64)
    blk = max(1, min(n, 2_000_000 // max(n, 1)))
    for i0 in range(0, n, blk):
        d = xyf[i0:i0 + blk, None, :] - xyf[None, :, :]
        dd = np.sqrt((d * d).sum(-1)) * scale
        out[i0:i0 + blk] = np.floor(dd + 0.5).astype(np.int32)
    return out


def _nearest_depot(c: np.ndarray, nd: int) -> np.ndarray:
    """Per customer the nearest depot (ties -> lower depot id)."""
    dc = c[nd:, :nd]
    return np.argmin(dc, axis=1).astype(np.int64)  # argmin returns the first minimum


# ----------------------------------------------------------------------------- windows

def _reference_routes(c, t, s, q, nd, Q, Dmax):
    """A simple reference plan, used to centre time windows.

    Nearest-depot assignment, a nearest-neighbour tour per depot, and a greedy
    split whenever the next customer would exceed Q or the route could not
    return to its depot by Dmax. Each route departs at time 0. Returns the
    routes and the arrival time at every customer."""
    n = c.shape[0]
    assign = _nearest_depot(c, nd)
    arr = np.zeros(n, dtype=np.int64)
    routes = []
    for d in range(nd):
        custs = [int(x) + nd for x in np.nonzero(assign == d)[0]]
        left = set(custs)
        order = []
        cur = d
        while left:
            cand = np.fromiter(left, dtype=np.int64)
            row = c[cur, cand]
            m = row.min()
            nxt = int(cand[row == m].min())
            order.append(nxt)
            left.remove(nxt)
            cur = nxt
        time, load, prev, route = 0, 0, d, []
        for x in order:
            a = time + int(t[prev, x])
            fin = a + int(s[x])
            if prev != d and (load + int(q[x]) > Q or fin + int(t[x, d]) > Dmax):
                routes.append((d, route, d))
                time, load, prev, route = 0, 0, d, []
                a = int(t[d, x])
                fin = a + int(s[x])
            arr[x] = a
            route.append(x)
            time, load, prev = fin, load + int(q[x]), x
        if route:
            routes.append((d, route, d))
    return routes, arr


def reference_plan(inst: "Instance"):
    """The reference plan the windows of a time-window instance were centred on."""
    routes, _ = _reference_routes(inst.c, inst.t, inst.s, inst.q, inst.n_depots, inst.Q, inst.Dmax)
    return routes


# ----------------------------------------------------------------------------- configs

def _make(nd, nc, xy, scale, q, s, e, l, **kw) -> Instance:
    c = _dist_matrix(xy, scale)
    return Instance(n_depots=nd, n_customers=nc, c=c, t=c, q=q.astype(np.int32), s=s.astype(np.int32),
                    e=e.astype(np.int32), l=l.astype(np.int32), coords=xy, **kw)


def config1(seed: int = 101) -> Instance:
    """MDVRP, 4 depots + 100 customers on [0,1000]^2, full neighbourhood (theta = 99)."""
    rng = np.random.default_rng(seed)
    nd, nc = 4, 100
    xy = rng.integers(0, 1001, size=(nd + nc, 2))
    q = np.concatenate([np.zeros(nd, np.int64), rng.integers(1, 26, nc)])
    n = nd + nc
    return _make(nd, nc, xy, 10, q, np.zeros(n), np.zeros(n), np.full(n, BIG_HORIZON),
                 Q=200, NV=4, Dmax=-1, open_routes=0, has_tw=0, theta=99,
                 w_tw=0, w_load=10, w_dur=0, w_depot=-1, name="mdvrp-4x100", seed=seed)


def _tw_instance(rng, nd, nc, box, cluster_sigma, n_clusters, q_hi, Q, s_srv, horizon, theta,
                 name, seed, NV=None, uniform=False):
    dep = rng.integers(0, box + 1, size=(nd, 2))
    if uniform:
        cus = rng.integers(0, box + 1, size=(nc, 2))
    else:
        centres = rng.uniform(0.15 * box, 0.85 * box, size=(n_clusters, 2))
        sizes = [nc // n_clusters + (1 if i < nc % n_clusters else 0) for i in range(n_clusters)]
        parts = [rng.normal(centres[i], cluster_sigma, size=(sizes[i], 2)) for i in range(n_clusters)]
        cus = np.floor(np.clip(np.concatenate(parts), 0, box) + 0.5).astype(np.int64)
    xy = np.concatenate([dep, cus]).astype(np.int64)
    n = nd + nc
    q = np.concatenate([np.zeros(nd, np.int64), rng.integers(1, q_hi + 1, nc)])
    s = np.concatenate([np.zeros(nd, np.int64), np.full(nc, s_srv)])
    width = rng.integers(100, 601, nc)
    c = _dist_matrix(xy, 10)
    if NV is None:
        NV = int(math.ceil(1.5 * q.sum() / (Q * nd)))
    _, arr = _reference_routes(c, c, s, q, nd, Q, horizon)
    e = np.zeros(n, np.int64)
    l = np.full(n, horizon, np.int64)
    a = arr[nd:]
    e[nd:] = np.maximum(0, a - width // 2)
    l[nd:] = np.minimum(e[nd:] + width, horizon)
    return Instance(n_depots=nd, n_customers=nc, c=c, t=c, q=q.astype(np.int32), s=s.astype(np.int32),
                    e=e.astype(np.int32), l=l.astype(np.int32), Q=Q, NV=NV, Dmax=horizon,
                    open_routes=0, has_tw=1, theta=theta, w_tw=20, w_load=10, w_dur=5, w_depot=-1,
                    name=name, seed=seed, coords=xy)


def config2(seed: int = 202) -> Instance:
    """MDVRPTW, 8 depots + 1000 customers in 8 Gaussian clusters (sigma 50), theta = 50."""
    rng = np.random.default_rng(seed)
    return _tw_instance(rng, 8, 1000, 1000, 50.0, 8, 30, 200, 90, 10_000, 50,
                        "mdvrptw-8x1000", seed)


def config3(seed: int = 303, open_routes: int = 0) -> Instance:
    """Large MDVRP / MDOVRP: 20 depots + 10000 customers on [0,10000]^2, theta = 50."""
    rng = np.random.default_rng(seed)
    nd, nc = 20, 10_000
    xy = rng.integers(0, 10_001, size=(nd + nc, 2))
    q = np.concatenate([np.zeros(nd, np.int64), rng.integers(1, 26, nc)])
    n = nd + nc
    return _make(nd, nc, xy, 10, q, np.zeros(n), np.zeros(n), np.full(n, BIG_HORIZON),
                 Q=300, NV=25, Dmax=-1, open_routes=open_routes, has_tw=0, theta=50,
                 w_tw=0, w_load=10, w_dur=0, w_depot=-1,
                 name="mdovrp-20x10000" if open_routes else "mdvrp-20x10000", seed=seed)


def config4_instance(i: int) -> Instance:
    """One of the 256 uneven MDVRPTW instances (seed 40000 + i)."""
    seed = 40_000 + i
    rng = np.random.default_rng(seed)
    nc = int(round(math.exp(rng.uniform(math.log(100), math.log(5000)))))
    nd = int(rng.integers(2, 21))
    return _tw_instance(rng, nd, nc, 1000, 50.0, 8, 30, 200, 90, 10_000, 50,
                        f"uneven-{i}", seed)


def config5(seed: int = 505) -> Instance:
    """Config-3 shape with time windows: 20 + 10000, horizon = Dmax = 100000, theta = 50."""
    rng = np.random.default_rng(seed)
    return _tw_instance(rng, 20, 10_000, 10_000, 0.0, 1, 25, 300, 90, 100_000, 50,
                        "mdvrptw-20x10000", seed, NV=25, uniform=True)


def tiny(seed: int, has_tw: int = 0, open_routes: int = 0, nd: int | None = None,
         nc: int | None = None, theta: int | None = None, Dmax: int = -1) -> Instance:
    """Small random instance for brute-force checks (<= 3 depots, <= 8 customers)."""
    rng = np.random.default_rng(seed)
    nd = int(rng.integers(1, 4)) if nd is None else nd
    nc = int(rng.integers(2, 9)) if nc is None else nc
    n = nd + nc
    xy = rng.integers(0, 21, size=(n, 2))
    c = _dist_matrix(xy, 1)
    q = np.concatenate([np.zeros(nd, np.int64), rng.integers(1, 10, nc)])
    Q = int(rng.integers(8, 30))
    if has_tw:
        horizon = 200
        s = np.concatenate([np.zeros(nd, np.int64), rng.integers(0, 6, nc)])
        e = np.zeros(n, np.int64)
        l = np.full(n, horizon, np.int64)
        e[nd:] = rng.integers(0, 150, nc)
        l[nd:] = np.minimum(e[nd:] + rng.integers(5, 80, nc), horizon)
        w = dict(w_tw=int(rng.integers(1, 6)), w_load=int(rng.integers(1, 6)), w_dur=int(rng.integers(1, 4)))
        Dm = Dmax if Dmax >= 0 else int(rng.integers(60, 200))
    else:
        s = np.zeros(n, np.int64)
        e = np.zeros(n, np.int64)
        l = np.full(n, BIG_HORIZON, np.int64)
        w = dict(w_tw=0, w_load=int(rng.integers(1, 6)), w_dur=int(rng.integers(1, 4)) if Dmax >= 0 else 0)
        Dm = Dmax
    th = nc - 1 if theta is None else theta
    return Instance(n_depots=nd, n_customers=nc, c=c, t=c, q=q.astype(np.int32), s=s.astype(np.int32),
                    e=e.astype(np.int32), l=l.astype(np.int32), Q=Q, NV=int(rng.integers(1, 3)),
                    Dmax=Dm, open_routes=open_routes, has_tw=has_tw, theta=th, w_depot=-1,
                    name=f"tiny-{seed}", seed=seed, coords=xy, **w)


def with_separate_times(inst: Instance, seed: int, c_jitter: int = 3, t_extra: int = 6) -> Instance:
    """A copy of a time-window instance whose distance matrix c is made asymmetric
    (each off-diagonal entry raised by U{0..c_jitter-1}) and whose travel times are a
    separate, asymmetric matrix t = c + U{0..t_extra-1} per arc; the diagonals stay 0.
    The distance-time ratio Gamma of the granular lists is then not 1."""
    assert inst.has_tw, "asymmetric matrices need time windows"
    rng = np.random.default_rng(seed)
    n = inst.N
    c = inst.c.astype(np.int64) + rng.integers(0, c_jitter, (n, n))
    t = c + rng.integers(0, t_extra, (n, n))
    np.fill_diagonal(c, 0)
    np.fill_diagonal(t, 0)
    out = Instance(**{**inst.__dict__})
    out.c = np.ascontiguousarray(c, np.int32)
    out.t = np.ascontiguousarray(t, np.int32)
    out.name = inst.name + "-ct"
    return out


# ----------------------------------------------------------------------------- start solutions

def start_solution(inst: Instance, sol_seed: int) -> Solution:
    """Nearest-depot assignment, per-depot shuffle, greedy split on capacity Q."""
    rng = np.random.default_rng(sol_seed)
    nd = inst.n_depots
    assign = _nearest_depot(inst.c, nd)
    routes = []
    for d in range(nd):
        custs = np.nonzero(assign == d)[0] + nd
        if len(custs) == 0:
            continue
        perm = rng.permutation(custs)
        cur, load = [], 0
        for x in perm:
            qx = int(inst.q[x])
            if cur and load + qx > inst.Q:
                routes.append((d, cur, -1 if inst.open_routes else d))
                cur, load = [], 0
            cur.append(int(x))
            load += qx
        if cur:
            routes.append((d, cur, -1 if inst.open_routes else d))
    return Solution(routes)


def random_solution(inst: Instance, sol_seed: int, max_routes: int | None = None) -> Solution:
    """Arbitrary routes with random (possibly different) start/end depots, for checks."""
    rng = np.random.default_rng(sol_seed)
    nd, nc = inst.n_depots, inst.n_customers
    perm = rng.permutation(np.arange(nd, nd + nc))
    m = int(rng.integers(1, min(nc, max_routes or nc) + 1))
    cuts = np.sort(rng.choice(np.arange(1, nc), size=m - 1, replace=False)) if m > 1 else []
    parts = np.split(perm, cuts)
    routes = []
    for p in parts:
        a = int(rng.integers(0, nd))
        b = -1 if inst.open_routes else int(rng.integers(0, nd))
        routes.append((a, [int(x) for x in p], b))
    return Solution(routes)


def seeds_for(instance_seed: int, n: int):
    """Solution k of an instance with seed s uses seed s*1000 + k."""
    return [instance_seed * 1000 + k for k in range(n)]
