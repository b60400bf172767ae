"""Pins of the oracle's repair insertions (Section 3.3, after Algorithm 3):
hand-computed best insertions (tests/golden/hand_cases.json, with citations),
and properties every operator must have, checked with an independent
computation of each position's cost from whole-solution costs (best insertion
and the regret order). No GPU."""
import json
import os

import numpy as np
import pytest

from oracle import Ref
from paper_2605_05208_amd import gen
from paper_2605_05208_amd.gen import Instance, Solution, canonical

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_cases.json")))
OPS = {"FBI": 0, "IBI": 1, "FRI": 2, "IRI": 3, "RI": 4}


def _instance(case):
    xy = np.asarray(case["xy"], np.int64)
    n = len(xy)
    d = xy[:, None, :] - xy[None, :, :]
    c = np.floor(np.sqrt((d * d).sum(-1)) * 10 + 0.5).astype(np.int32)
    z = np.zeros(n, np.int32)
    nd = case["n_depots"]
    return Instance(n_depots=nd, n_customers=n - nd, c=c, t=c, q=np.asarray(case["q"], np.int32), s=z, e=z,
                    l=np.full(n, gen.BIG_HORIZON, np.int32), Q=case["Q"], NV=case.get("NV", 4), Dmax=-1,
                    open_routes=case.get("open_routes", 0), has_tw=0, theta=n - nd - 1, w_tw=0,
                    w_load=case.get("w_load", 10), w_dur=0, w_depot=-1)


def _sol(routes):
    return Solution([(a, list(xs), b) for a, xs, b in routes])


@pytest.mark.parametrize("case", GOLDEN["repair"], ids=lambda c: c["note"][:40])
def test_repair_worked_examples(case):
    inst = _instance(case)
    out, order, _ = Ref(inst).repair(_sol(case["routes"]), OPS[case["op"]])
    assert order == case["order"]
    assert canonical(out.routes) == canonical([tuple(r) for r in case["expect"]])


def _positions(sol):
    for r, (a, xs, b) in enumerate(sol.routes):
        for k in range(len(xs) + 1):
            yield r, k


def _with(sol, r, k, x):
    routes = [list(t) for t in sol.routes]
    a, xs, b = routes[r]
    routes[r] = (a, list(xs[:k]) + [x] + list(xs[k:]), b)
    return Solution([tuple(t) for t in routes])


def _partial(inst, seed, drop):
    rng = np.random.default_rng(seed)
    full = gen.random_solution(inst, seed)
    gone = set(rng.choice(np.arange(inst.n_depots, inst.N), size=drop, replace=False).tolist())
    routes = [(a, [x for x in xs if x not in gone], b) for a, xs, b in full.routes]
    return Solution([r for r in routes if r[1]]), sorted(gone)


@pytest.mark.parametrize("tw,open_r", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("op", ["FBI", "IBI", "FRI", "IRI", "RI"])
def test_repair_properties(tw, open_r, op):
    inst = gen.tiny(5200 + 10 * tw + open_r, has_tw=tw, open_routes=open_r, nc=12)
    ref = Ref(inst)
    for seed in range(4):
        part, gone = _partial(inst, seed, 4)
        out, order, nev = ref.repair(part, OPS[op], seed=seed)
        # every customer once, the inserted ones exactly the missing ones
        seen = sorted(x for _, xs, _ in out.routes for x in xs)
        assert seen == list(range(inst.n_depots, inst.N))
        assert sorted(order) == gone
        if op in ("FBI", "IBI", "RI"):
            assert order == gone  # ascending ids
        n_routes_in = len(part.routes)
        if op in ("IBI", "IRI", "RI") and n_routes_in > 0:
            assert len(out.routes) == n_routes_in  # infeasible and random insertions open no route
        assert nev > 0


@pytest.mark.parametrize("op", ["FBI", "IBI"])
def test_best_insertion_is_the_cheapest_position(op):
    """The first inserted customer goes to the cheapest (feasible) position, the cost of a
    position being F(S with x inserted) - F(S), both from whole-solution costs; with no
    feasible position FBI opens a route at the cheapest depot."""
    for seed in range(6):
        inst = gen.tiny(5300 + seed, nc=10)
        if seed % 2:  # tight capacity: few or no feasible positions
            inst.Q = int(inst.q.max()) + 1
        ref = Ref(inst)
        part, gone = _partial(inst, seed, 1)
        x = gone[0]
        F0, t0 = ref.cost(part)
        best = None
        for r, k in _positions(part):
            S = _with(part, r, k, x)
            F1, t1 = ref.cost(S)
            feasible = t1[1] == t0[1] and t1[2] == t0[2] and t1[3] == t0[3]
            if op == "FBI" and not feasible:
                continue
            xs = part.routes[r][1]
            posid = xs[k - 1] if k > 0 else inst.N + xs[0]
            key = (F1 - F0, posid)
            if best is None or key < best[0]:
                best = (key, S)
        out, order, _ = ref.repair(part, OPS[op])
        if best is not None:
            assert canonical(out.routes) == canonical(best[1].routes)
        else:
            assert op == "FBI" and len(out.routes) == len(part.routes) + 1
            new = [r for r in out.routes if r[1] == [x]]
            assert len(new) == 1


def test_regret_takes_the_largest_regret_first():
    """FRI / IRI with two missing customers: the first one inserted has the larger gap between
    its two cheapest admissible positions (computed here from whole-solution costs)."""
    for seed in range(8):
        inst = gen.tiny(5400 + seed, nc=10)
        ref = Ref(inst)
        part, gone = _partial(inst, seed, 2)
        F0, _ = ref.cost(part)
        regrets = {}
        for x in gone:
            costs = sorted(((ref.cost(_with(part, r, k, x))[0] - F0), r, k) for r, k in _positions(part))
            regrets[x] = costs[1][0] - costs[0][0] if len(costs) >= 2 else float("inf")
        first = max(gone, key=lambda x: (regrets[x], -x))
        _, order, _ = ref.repair(part, OPS["IRI"])
        assert order[0] == first


def test_repair_of_an_empty_solution_opens_routes():
    inst = gen.tiny(5500, nc=6)
    for op in OPS.values():
        out, order, _ = Ref(inst).repair(Solution([]), op, seed=3)
        assert sorted(order) == list(range(inst.n_depots, inst.N))
        assert sorted(x for _, xs, _ in out.routes for x in xs) == list(range(inst.n_depots, inst.N))


def test_random_insertion_depends_on_the_seed_only():
    inst = gen.tiny(5600, nc=12)
    part, _ = _partial(inst, 1, 5)
    a = Ref(inst).repair(part, OPS["RI"], seed=11)[0]
    b = Ref(inst).repair(part, OPS["RI"], seed=11)[0]
    c = [Ref(inst).repair(part, OPS["RI"], seed=s)[0] for s in range(12, 20)]
    assert canonical(a.routes) == canonical(b.routes)
    assert any(canonical(x.routes) != canonical(a.routes) for x in c)
