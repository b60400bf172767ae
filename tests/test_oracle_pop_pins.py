"""Pins of the oracle's population measures (Section 3.4, Eq. 5-7) against
hand-computed worked examples (tests/golden/hand_cases.json, each with its
citation), properties the definitions fix, and an independent set-based count
of common arcs on small random solutions. No GPU."""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import Ref
from paper_2605_05208_amd import gen
from paper_2605_05208_amd.gen import Instance, Solution

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_cases.json")))


def _line_instance(nd, nc, open_routes):
    n = nd + nc
    xy = np.stack([np.arange(n) * 7 % 13, np.arange(n) * 5 % 11], 1).astype(np.int64)
    d = xy[:, None, :] - xy[None, :, :]
    c = np.floor(np.sqrt((d * d).sum(-1)) * 10 + 0.5).astype(np.int32)
    z = np.zeros(n, np.int32)
    return Instance(n_depots=nd, n_customers=nc, c=c, t=c, q=z + np.r_[np.zeros(nd), np.ones(nc)].astype(np.int32),
                    s=z, e=z, l=np.full(n, gen.BIG_HORIZON, np.int32), Q=100, NV=4, Dmax=-1,
                    open_routes=open_routes, has_tw=0, theta=nc - 1, w_tw=0, w_load=10, w_dur=0, w_depot=-1)


def _sol(routes):
    return Solution([(a, list(xs), b) for a, xs, b in routes])


@pytest.mark.parametrize("case", GOLDEN["population_distance"], ids=lambda c: c["note"][:40])
def test_distance_worked_examples(case):
    inst = _line_instance(case["n_depots"], case["n_customers"], case["open_routes"])
    d, common, ne = Ref(inst).population_distance([_sol(case["a"]), _sol(case["b"])])
    assert ne.tolist() == case["edges"]
    assert common[0, 1] == common[1, 0] == case["common"]
    assert abs(d[0, 1] - case["dist"]) < 1e-12 and d[0, 1] == d[1, 0]
    assert d[0, 0] == d[1, 1] == 0.0


@pytest.mark.parametrize("case", GOLDEN["population_reduce"], ids=lambda c: c["note"][:40])
def test_reduce_worked_examples(case):
    keep, order, chi, dpop = oracle.population_reduce(np.array(case["dist"], np.float64), case["f"], case["mu"],
                                                      case["xi"], case["n_close"])
    assert np.allclose(dpop, case["dpop"], rtol=0, atol=1e-12)
    assert np.allclose(chi, case["chi"], rtol=0, atol=1e-12)
    assert order.tolist() == case["order"]
    assert keep.tolist() == case["keep"]


def _arcs(sol):
    """The directed arcs of a solution's routes, written out independently."""
    out = set()
    for start, xs, end in sol.routes:
        path = [start] + list(xs) + ([end] if end >= 0 else [])
        out |= {(a, b) for a, b in zip(path[:-1], path[1:])}
    return out


@pytest.mark.parametrize("tw,open_r", [(0, 0), (1, 0), (0, 1)])
def test_distance_against_arc_sets(tw, open_r):
    inst = gen.tiny(4100 + 10 * tw + open_r, has_tw=tw, open_routes=open_r)
    sols = [gen.random_solution(inst, k) for k in range(5)] + [gen.start_solution(inst, 9)]
    sols.append(sols[2])  # a duplicate solution
    d, common, ne = Ref(inst).population_distance(sols)
    arcs = [_arcs(s) for s in sols]
    for i, a in enumerate(arcs):
        closed = sum(1 for r in sols[i].routes if r[2] >= 0)
        assert ne[i] == len(a) == inst.n_customers + closed
        for j, b in enumerate(arcs):
            assert common[i, j] == len(a & b)
            exp = 100.0 * (1.0 - len(a & b) / max(len(a), len(b)))
            assert d[i, j] == exp
    assert np.all(d >= 0) and np.all(d <= 100) and np.array_equal(d, d.T)
    assert d[2, 6] == 0.0 and np.all(np.diag(d) == 0)


def test_reduce_properties():
    """Survivor count, removal order a permutation of the leavers, and with xi = 0 the
    survivors are the mu best objectives."""
    rng = np.random.default_rng(3)
    n, mu = 30, 20
    a = rng.random((n, n)) * 100
    dist = np.triu(a, 1) + np.triu(a, 1).T
    f = rng.integers(0, 1000, n)
    keep, order, chi, dpop = oracle.population_reduce(dist, f, mu, 0.7, 5)
    assert keep.sum() == mu and len(order) == n - mu
    assert sorted(order.tolist()) == sorted(np.nonzero(keep == 0)[0].tolist())
    for i in range(n):  # Eq. 6 over all n: the mean of the five smallest distances to the others
        others = np.sort(np.delete(dist[i], i))
        assert abs(dpop[i] - others[:5].mean()) < 1e-9
    keep0, _, _, _ = oracle.population_reduce(dist, f, mu, 0.0, 5)
    best = np.lexsort((np.arange(n), f))[:mu]
    assert sorted(np.nonzero(keep0)[0].tolist()) == sorted(best.tolist())
