"""Python access to the plain CPU oracle (libmdvrp_ref.so).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg. The product package never imports this module.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmdvrp_ref.so")
SOURCES = ["mdvrp_ref.c", "mlp_ref.c", "pop_ref.c", "repair_ref.c", "dcrex_ref.c"]

FAM_REL, FAM_SWP, FAM_X2, FAM_2OPT, FAM_DINS, FAM_DREP = range(6)
ALL_FAMILIES = (1 << 6) - 1
KIND_NAMES = ["REL1", "REL2", "SWP11", "SWP21", "SWP12", "SWP22", "X2", "2OPT", "DINS", "DREP"]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    cmd = ["gcc", "-O2", "-std=gnu11", "-Wall", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC", "-o", LIB_PATH] \
        + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    return LIB_PATH


class RefInstance(C.Structure):
    _fields_ = [("n_depots", C.c_int32), ("n_customers", C.c_int32),
                ("c", C.c_void_p), ("t", C.c_void_p), ("q", C.c_void_p), ("s", C.c_void_p),
                ("e", C.c_void_p), ("l", C.c_void_p),
                ("Q", C.c_int32), ("NV", C.c_int32), ("Dmax", C.c_int32),
                ("open_routes", C.c_int32), ("has_tw", C.c_int32), ("theta", C.c_int32),
                ("w_tw", C.c_int32), ("w_load", C.c_int32), ("w_dur", C.c_int32), ("w_depot", C.c_int32)]


class RefMove(C.Structure):
    _fields_ = [("dF", C.c_int64), ("dD", C.c_int64), ("dTW", C.c_int64), ("dLX", C.c_int64),
                ("dDX", C.c_int64), ("dV4", C.c_int64), ("id", C.c_uint64), ("res", C.c_int32 * 3)]


MOVE_DTYPE = np.dtype([("dF", np.int64), ("dD", np.int64), ("dTW", np.int64), ("dLX", np.int64),
                       ("dDX", np.int64), ("dV4", np.int64), ("id", np.uint64), ("res", np.int32, (3,)),
                       ("_pad", np.int32)])
assert MOVE_DTYPE.itemsize == C.sizeof(RefMove)


class RefLsOptions(C.Structure):
    _fields_ = [("mode", C.c_int32), ("leader_only", C.c_int32), ("max_passes", C.c_int32),
                ("penalty_adapt", C.c_int32), ("seed", C.c_uint64),
                ("w_min", C.c_int32 * 4), ("w_max", C.c_int32 * 4)]


class RefLsStats(C.Structure):
    _fields_ = [("passes", C.c_int64), ("steps", C.c_int64), ("moves_applied", C.c_int64),
                ("evaluated", C.c_int64), ("F", C.c_int64), ("w_final", C.c_int64 * 4)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        p = C.c_void_p
        L.ref_instance_stats.argtypes = [p, p]
        L.ref_neighbours.argtypes = [p, p, p]
        L.ref_cost.argtypes = [p, C.c_int32, p, p, p, p, p, p]
        L.ref_eval.argtypes = [p, p, p, C.c_int32, p, p, p, p, C.c_uint32, p, C.c_int64, p]
        L.ref_step.argtypes = [p, p, p, C.c_int32, p, p, p, p, C.c_uint32, C.c_int32,
                               p, p, p, p, p, p, p, p, p]
        L.ref_local_search.argtypes = [p, p, p, C.c_int32, p, p, p, p, p, p, p, p, p, p, p, p]
        L.ref_apply_ids.argtypes = [p, C.c_int32, p, p, p, p, p, C.c_int32, p, p, p, p, p]
        L.ref_filter_features.argtypes = [p, p, p, C.c_int32, p, p, p, p, p]
        L.ref_mlp_param_count.restype = C.c_int32
        L.ref_mlp_forward.argtypes = [p, p, C.c_int32, C.c_int32, p]
        L.ref_mlp_backward.argtypes = [p, p, C.c_int32, p, C.c_int32, p]
        L.ref_bce.argtypes = [p, p, p, C.c_int32]
        L.ref_bce.restype = C.c_double
        L.ref_adam.argtypes = [p, p, p, p, C.c_int32, C.c_float, C.c_int32]
        L.ref_topk.argtypes = [p, p, C.c_int32, C.c_int32, p, C.c_int32, p]
        L.ref_bf16.argtypes = [C.c_float]
        L.ref_bf16.restype = C.c_uint16
        L.ref_route_terms.argtypes = [p, C.c_int32, p, C.c_int32, C.c_int32, p]
        L.ref_splitmix64.argtypes = [p]
        L.ref_splitmix64.restype = C.c_uint64
        L.ref_family_order.argtypes = [C.c_int32, C.c_uint64, C.c_int64, p]
        L.ref_family_order.restype = C.c_int32
        L.ref_population_distance.argtypes = [C.c_void_p, C.c_int32] + [p] * 8
        L.ref_population_reduce.argtypes = [C.c_int32, p, p, C.c_int32, C.c_double, C.c_int32, p, p, p, p]
        L.ref_repair.argtypes = [p, C.c_int32, p, p, p, p, C.c_int32, C.c_uint64] + [p] * 8
        L.ref_dcrex_counts.argtypes = [C.c_int32] + [p] * 5 + [C.c_int32] + [p] * 8
        L.ref_ucb_select.argtypes = [C.c_int32, p, p]
        L.ref_ucb_select.restype = C.c_int32
        L.ref_ucb_update.argtypes = [C.c_int32, p, p, C.c_int32, C.c_double, C.c_double]
        L.ref_ucb_ln.argtypes = [C.c_double]
        L.ref_ucb_ln.restype = C.c_double
        L.ref_ucb_sqrt.argtypes = [C.c_double]
        L.ref_ucb_sqrt.restype = C.c_double
        L.ref_set_threads.argtypes = [C.c_int32]
        L.ref_get_threads.restype = C.c_int32
        _lib = L
    return _lib


def set_threads(n: int) -> int:
    """OpenMP threads of the oracle's solution-parallel local search; returns the previous count."""
    old = int(lib().ref_get_threads())
    lib().ref_set_threads(int(n))
    return old


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class Ref:
    """Oracle bound to one instance (keeps the numpy buffers alive)."""

    def __init__(self, inst):
        self.inst = inst
        self._keep = [np.ascontiguousarray(x, dtype=np.int32) for x in
                      (inst.c, inst.t, inst.q, inst.s, inst.e, inst.l)]
        c, t, q, s, e, l = self._keep
        self.desc = RefInstance(inst.n_depots, inst.n_customers, _ptr(c).value, _ptr(t).value,
                                _ptr(q).value, _ptr(s).value, _ptr(e).value, _ptr(l).value,
                                inst.Q, inst.NV, inst.Dmax, inst.open_routes, inst.has_tw, inst.theta,
                                inst.w_tw, inst.w_load, inst.w_dur, inst.w_depot)
        self._nbr = None

    @property
    def dref(self):
        return C.byref(self.desc)

    def stats(self):
        out = np.zeros(4, np.int64)
        lib().ref_instance_stats(self.dref, _ptr(out))
        return dict(Theta=int(out[0]), gamma_num=int(out[1]), gamma_den=int(out[2]), w_depot=int(out[3]))

    def neighbours(self):
        if self._nbr is None:
            nc, th = self.inst.n_customers, self.inst.theta
            nbr = np.full(nc * th, -1, np.int32)
            ln = np.zeros(nc, np.int32)
            rc = lib().ref_neighbours(self.dref, _ptr(nbr), _ptr(ln))
            assert rc == 0
            self._nbr = (nbr, ln)
        return self._nbr

    def route_terms(self, start, xs, end):
        """(distance, load, duration, time warp) of one route walked node by node."""
        xs = np.ascontiguousarray(xs if len(xs) else [0], np.int32)
        out = np.zeros(4, np.int64)
        lib().ref_route_terms(self.dref, int(start), _ptr(xs), len(xs), int(end), _ptr(out))
        return tuple(int(x) for x in out)

    def cost(self, sol):
        nodes, offs, st, en = sol.flat()
        F = np.zeros(1, np.int64)
        terms = np.zeros(6, np.int64)
        lib().ref_cost(self.dref, len(st), _ptr(nodes), _ptr(offs), _ptr(st), _ptr(en), _ptr(F), _ptr(terms))
        return int(F[0]), terms

    def _lists(self, lists):
        """(descriptor, nbr, nbr_len) for the granular lists, or for caller lists
        (nbr [n_customers * stride], nbr_len, stride) evaluated in their place."""
        if lists is None:
            nbr, ln = self.neighbours()
            return self.dref, nbr, ln
        nbr, ln, stride = lists
        d = RefInstance(*[getattr(self.desc, f) for f, _ in RefInstance._fields_])
        d.theta = int(stride)
        self._keep_lists = (d, np.ascontiguousarray(nbr, np.int32), np.ascontiguousarray(ln, np.int32))
        return C.byref(d), self._keep_lists[1], self._keep_lists[2]

    def eval(self, sol, fam_mask=ALL_FAMILIES, lists=None):
        dref, nbr, ln = self._lists(lists)
        nodes, offs, st, en = sol.flat()
        cnt = np.zeros(1, np.int64)
        cap = 1 << 16
        while True:
            out = np.zeros(cap, MOVE_DTYPE)
            rc = lib().ref_eval(dref, _ptr(nbr), _ptr(ln), len(st), _ptr(nodes), _ptr(offs), _ptr(st),
                                _ptr(en), fam_mask, _ptr(out), cap, _ptr(cnt))
            if rc == -3:
                cap = int(cnt[0])
                continue
            assert rc == 0, rc
            return out[:int(cnt[0])]

    def step(self, sol, fam_mask, leader_only=0, lists=None):
        from paper_2605_05208_amd.gen import Solution
        dref, nbr, ln = self._lists(lists)
        nodes, offs, st, en = sol.flat()
        nc = self.inst.n_customers
        o_nr = np.zeros(1, np.int32)
        o_nodes = np.zeros(nc + 1, np.int32)
        o_offs = np.zeros(nc + 2, np.int32)
        o_st = np.zeros(nc + 1, np.int32)
        o_en = np.zeros(nc + 1, np.int32)
        sel_ids = np.zeros(nc + 1, np.uint64)
        sel_dF = np.zeros(nc + 1, np.int64)
        n_sel = np.zeros(1, np.int32)
        n_eval = np.zeros(1, np.int64)
        lib().ref_step(dref, _ptr(nbr), _ptr(ln), len(st), _ptr(nodes), _ptr(offs), _ptr(st), _ptr(en),
                       fam_mask, leader_only, _ptr(o_nr), _ptr(o_nodes), _ptr(o_offs), _ptr(o_st), _ptr(o_en),
                       _ptr(sel_ids), _ptr(sel_dF), _ptr(n_sel), _ptr(n_eval))
        nr = int(o_nr[0])
        routes = [(int(o_st[r]), [int(x) for x in o_nodes[o_offs[r]:o_offs[r + 1]]], int(o_en[r])) for r in range(nr)]
        k = int(n_sel[0])
        return Solution(routes), sel_ids[:k].copy(), sel_dF[:k].copy(), int(n_eval[0])

    def apply_ids(self, sol, ids):
        from paper_2605_05208_amd.gen import Solution
        nodes, offs, st, en = sol.flat()
        ids = np.ascontiguousarray(ids, dtype=np.uint64)
        nc = self.inst.n_customers
        o_nr = np.zeros(1, np.int32)
        o_nodes = np.zeros(nc + 1, np.int32)
        o_offs = np.zeros(nc + 2, np.int32)
        o_st = np.zeros(nc + 1, np.int32)
        o_en = np.zeros(nc + 1, np.int32)
        lib().ref_apply_ids(self.dref, len(st), _ptr(nodes), _ptr(offs), _ptr(st), _ptr(en), _ptr(ids), len(ids),
                            _ptr(o_nr), _ptr(o_nodes), _ptr(o_offs), _ptr(o_st), _ptr(o_en))
        nr = int(o_nr[0])
        return Solution([(int(o_st[r]), [int(x) for x in o_nodes[o_offs[r]:o_offs[r + 1]]], int(o_en[r]))
                         for r in range(nr)])

    def local_search(self, sols, mode=0, seed=0, max_passes=0, leader_only=0, adapt=None):
        """adapt = (w_min, w_max), each 4 weights (time window, load, duration, depot): dynamic
        penalty coefficients (Section 3.2.1) within those bounds; None = fixed weights."""
        from paper_2605_05208_amd.gen import batch_flat, solutions_from_flat
        nbr, ln = self.neighbours()
        nodes, offs, st, en, so = batch_flat(sols)
        n = len(sols)
        nc = self.inst.n_customers
        o_nodes = np.zeros(n * nc + 1, np.int32)
        o_offs = np.zeros(n * nc + 2, np.int32)
        o_st = np.zeros(n * nc + 1, np.int32)
        o_en = np.zeros(n * nc + 1, np.int32)
        o_so = np.zeros(n + 1, np.int32)
        stats = (RefLsStats * n)()
        opt = RefLsOptions(mode, leader_only, max_passes, 0, seed)
        if adapt is not None:
            opt.penalty_adapt = 1
            opt.w_min = (C.c_int32 * 4)(*[int(x) for x in adapt[0]])
            opt.w_max = (C.c_int32 * 4)(*[int(x) for x in adapt[1]])
        rc = lib().ref_local_search(self.dref, _ptr(nbr), _ptr(ln), n, _ptr(nodes), _ptr(offs), _ptr(st),
                                    _ptr(en), _ptr(so), C.byref(opt), _ptr(o_nodes), _ptr(o_offs), _ptr(o_st),
                                    _ptr(o_en), _ptr(o_so), stats)
        if rc != 0:
            raise ValueError(f"oracle local search refused its options ({rc})")
        out = solutions_from_flat(o_nodes, o_offs, o_st, o_en, o_so)
        st_list = [dict(passes=s.passes, steps=s.steps, moves_applied=s.moves_applied, evaluated=s.evaluated, F=s.F,
                        w_final=[int(x) for x in s.w_final]) for s in stats]
        return out, st_list


    def population_distance(self, sols):
        """Eq. 7 between every pair of solutions: (dist [n][n] fp64, common arcs [n][n], |E| [n])."""
        from paper_2605_05208_amd.gen import batch_flat
        nodes, offs, st, en, so = batch_flat(sols)
        n = len(sols)
        dist = np.zeros((n, n), np.float64)
        common = np.zeros((n, n), np.int64)
        ne = np.zeros(n, np.int64)
        rc = lib().ref_population_distance(self.dref, n, _ptr(nodes), _ptr(offs), _ptr(st), _ptr(en), _ptr(so),
                                           _ptr(dist), _ptr(common), _ptr(ne))
        assert rc == 0, rc
        return dist, common, ne

    def repair(self, sol, op, seed=0):
        """Insert the customers missing from sol with operator op (0 FBI, 1 IBI, 2 FRI, 3 IRI,
        4 RI): (complete solution, insertion order, positions evaluated)."""
        from paper_2605_05208_amd.gen import Solution
        nc = self.inst.n_customers
        if sol.routes:
            nodes, offs, st, en = sol.flat()
        else:
            nodes, offs, st, en = (np.zeros(1, np.int32), np.zeros(1, np.int32), np.zeros(1, np.int32),
                                   np.zeros(1, np.int32))
        nr = len(sol.routes)
        o_nr = np.zeros(1, np.int32)
        o_nodes = np.zeros(nc + 1, np.int32)
        o_offs = np.zeros(nc + 2, np.int32)
        o_st = np.zeros(nc + 1, np.int32)
        o_en = np.zeros(nc + 1, np.int32)
        order = np.zeros(nc + 1, np.int32)
        n_order = np.zeros(1, np.int32)
        n_eval = np.zeros(1, np.int64)
        rc = lib().ref_repair(self.dref, nr, _ptr(nodes), _ptr(offs), _ptr(st), _ptr(en), int(op), int(seed),
                              _ptr(o_nr), _ptr(o_nodes), _ptr(o_offs), _ptr(o_st), _ptr(o_en), _ptr(order),
                              _ptr(n_order), _ptr(n_eval))
        assert rc == 0, rc
        m = int(o_nr[0])
        out = Solution([(int(o_st[r]), [int(v) for v in o_nodes[o_offs[r]:o_offs[r + 1]]], int(o_en[r]))
                        for r in range(m)])
        return out, [int(v) for v in order[:int(n_order[0])]], int(n_eval[0])

    def features(self, sol):
        nbr, ln = self.neighbours()
        nodes, offs, st, en = sol.flat()
        out = np.zeros(self.inst.n_customers * self.inst.theta * 32, np.uint16)
        lib().ref_filter_features(self.dref, _ptr(nbr), _ptr(ln), len(st), _ptr(nodes), _ptr(offs), _ptr(st),
                                  _ptr(en), _ptr(out))
        return out.reshape(self.inst.n_customers * self.inst.theta, 32)


N_PARAMS = 74497


def population_reduce(dist, f, mu, xi=0.7, n_close=5):
    """Reduce a population to mu solutions by chi (Eq. 5-6): (keep [n], removal order,
    chi over all n, population distance over all n)."""
    dist = np.ascontiguousarray(dist, np.float64)
    f = np.ascontiguousarray(f, np.int64)
    n = len(f)
    keep = np.zeros(n, np.int32)
    order = np.zeros(max(n - mu, 1), np.int32)
    chi = np.zeros(n, np.float64)
    dpop = np.zeros(n, np.float64)
    rc = lib().ref_population_reduce(n, _ptr(dist), _ptr(f), int(mu), float(xi), int(n_close), _ptr(keep),
                                     _ptr(order), _ptr(chi), _ptr(dpop))
    assert rc == 0, rc
    return keep, order[:max(n - mu, 0)], chi, dpop


def _flat_routes(routes):
    nodes, offs, st, en = [], [0], [], []
    for a, xs, b in routes:
        nodes.extend(xs)
        offs.append(len(nodes))
        st.append(a)
        en.append(b)
    z = lambda v: np.asarray(v if len(v) else [0], np.int32)  # noqa: E731
    return z(nodes), np.asarray(offs, np.int32), z(st), z(en)


def dcrex_counts(offspring, intro, parent):
    """Route-pair counts of the crossover (Algorithm 3): offspring and parent are lists of
    (start, customers, end) routes (the offspring may hold a customer twice), intro the
    offspring routes introduced from parents. Returns EI, NR, NM, NC as [ns][np] arrays."""
    ns, np_ = len(offspring), len(parent)
    sn, so, ss, se = _flat_routes(offspring)
    pn, po, ps, pe = _flat_routes(parent)
    it = np.ascontiguousarray(intro if len(intro) else [0], np.int32)
    out = [np.zeros((max(ns, 1), max(np_, 1)), np.int32) for _ in range(4)]
    lib().ref_dcrex_counts(ns, _ptr(sn), _ptr(so), _ptr(ss), _ptr(se), _ptr(it), np_, _ptr(pn), _ptr(po),
                           _ptr(ps), _ptr(pe), *[_ptr(o) for o in out])
    return [o[:ns, :np_] for o in out]


def dcrex_score(ei, nr, nm, nc):
    """Score of a route pair (Algorithm 3): lower is better."""
    return -(ei - nr - nm - 10 * nc)


def dcrex_dsigma(ei, nr, nm):
    """Diversity increase of an exchange (Algorithm 3)."""
    return ei + nr + nm


def dcrex_pick(ei, nr, nm, nc, seed):
    """Algorithm 3's choice: among the min(5, #pairs) pairs of lowest (score, i, j), the one
    at index SplitMix64(seed) mod their number: (i, j, diversity increase, candidates)."""
    ns, np_ = ei.shape
    if ns * np_ == 0:
        return [-1, -1, 0, 0]
    score = dcrex_score(ei.astype(np.int64), nr, nm, nc)
    flat = np.arange(ns * np_)
    order = np.lexsort((flat, score.ravel()))  # score ascending, then i * np + j
    cnt = min(5, ns * np_)
    t = int(order[splitmix64(seed, 1)[0] % cnt])
    i, j = divmod(t, np_)
    return [i, j, int(dcrex_dsigma(ei[i, j], nr[i, j], nm[i, j])), cnt]


def ucb_select(R, N):
    R = np.ascontiguousarray(R, np.float64)
    N = np.ascontiguousarray(N, np.float64)
    return int(lib().ref_ucb_select(len(R), _ptr(R), _ptr(N)))


def ucb_update(R, N, arm, reward, gamma=0.99):
    """In place on float64 arrays R, N."""
    lib().ref_ucb_update(len(R), _ptr(R), _ptr(N), int(arm), float(reward), float(gamma))


def ucb_ln(x):
    return float(lib().ref_ucb_ln(float(x)))


def ucb_sqrt(x):
    return float(lib().ref_ucb_sqrt(float(x)))


def mlp_forward(params, x, round_act=1):
    params = np.ascontiguousarray(params, np.float32)
    x = np.ascontiguousarray(x, np.uint16)
    out = np.zeros(len(x), np.float64)
    lib().ref_mlp_forward(_ptr(params), _ptr(x), len(x), round_act, _ptr(out))
    return out


def mlp_backward(params, x, dlogits, round_act=1):
    params = np.ascontiguousarray(params, np.float32)
    x = np.ascontiguousarray(x, np.uint16)
    d = np.ascontiguousarray(dlogits, np.float64)
    g = np.zeros(N_PARAMS, np.float64)
    lib().ref_mlp_backward(_ptr(params), _ptr(x), len(x), _ptr(d), round_act, _ptr(g))
    return g


def bce(logits, labels, weights=None):
    z = np.ascontiguousarray(logits, np.float64)
    y = np.ascontiguousarray(labels, np.float32)
    w = None if weights is None else np.ascontiguousarray(weights, np.float32)
    return lib().ref_bce(_ptr(z), _ptr(y), None if w is None else _ptr(w), len(z))


def adam(params, m, v, grads, lr, step):
    for a in (params, m, v):
        assert a.dtype == np.float32 and a.flags.c_contiguous
    g = np.ascontiguousarray(grads, np.float32)
    lib().ref_adam(_ptr(params), _ptr(m), _ptr(v), _ptr(g), len(params), lr, step)


def topk(nbr, nbr_len, n_customers, theta, score, k):
    out = np.zeros(n_customers * k, np.int32)
    lib().ref_topk(_ptr(np.ascontiguousarray(nbr, np.int32)), _ptr(np.ascontiguousarray(nbr_len, np.int32)),
                   n_customers, theta, _ptr(np.ascontiguousarray(score, np.float32)), k, _ptr(out))
    return out.reshape(n_customers, k)


def bf16(x):
    return np.array([lib().ref_bf16(float(v)) for v in np.ravel(x)], np.uint16)


def family_order(has_tw: int, seed: int, p: int):
    fam = np.zeros(6, np.int32)
    n = lib().ref_family_order(has_tw, seed, p, _ptr(fam))
    return [int(x) for x in fam[:n]]


def splitmix64(state: int, n: int):
    """The first n outputs of SplitMix64 started from state."""
    st = np.array([state], np.uint64)
    return [int(lib().ref_splitmix64(_ptr(st))) for _ in range(n)]
