"""Crossover pieces (Section 3.3, Algorithm 3 and Eq. 4) on the GPU against the
oracle: route-pair counts exactly (the hand-computed example, offspring that hold
customers twice, open routes, the 20 x 10000 scale), the choice among the five
lowest-scored pairs, and a sequence of discounted UCB1 choices and updates bit
for bit."""
import json
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2605_05208_amd import gen, mdvrp

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_cases.json")))


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _check(nd, n, off, intro, par, tag):
    got = [x.cpu().numpy() for x in mdvrp.dcrex_counts(nd, n, off, intro, par)]
    exp = oracle.dcrex_counts(off, intro, par)
    for g, e, name in zip(got, exp, ("EI", "NR", "NM", "NC")):
        assert np.array_equal(g, e), f"{tag}: {name}"
    return got


@pytest.mark.parametrize("case", GOLDEN["dcrex"]["cases"], ids=lambda c: str(c["intro"]))
def test_counts_worked_example(case):
    off = [tuple(r) for r in GOLDEN["dcrex"]["offspring"]]
    par = [tuple(r) for r in GOLDEN["dcrex"]["parent"]]
    ei, nr, nm, nc = _check(1, 5, off, case["intro"], par, "worked example")
    assert ei.tolist() == case["EI"] and nc.tolist() == case["NC"]


def _offspring(inst, rng, t, extra):
    s1, s2, p = (gen.random_solution(inst, 3 * t + k) for k in range(3))
    pick = rng.choice(len(s2.routes), size=min(extra, len(s2.routes)), replace=False)
    off = list(s1.routes) + [s2.routes[k] for k in pick]
    intro = [0] * len(s1.routes) + [1] * len(pick)
    return off, intro, list(p.routes)


@pytest.mark.parametrize("tw,open_r", [(0, 0), (1, 0), (0, 1)])
def test_counts_tiny(tw, open_r):
    rng = np.random.default_rng(11 + tw + 2 * open_r)
    for t in range(8):
        inst = gen.tiny(8300 + 10 * tw + open_r + 100 * t, has_tw=tw, open_routes=open_r, nc=12)
        off, intro, par = _offspring(inst, rng, t, 1 + t % 3)
        _check(inst.n_depots, inst.N, off, intro, par, f"tiny {t}")


def test_counts_and_pick_config2():
    """Offspring = one start solution plus 12 routes of another (customers held twice)."""
    inst = gen.config2()
    rng = np.random.default_rng(5)
    a, b, p = (gen.start_solution(inst, inst.seed * 1000 + k) for k in range(3))
    pick = rng.choice(len(b.routes), size=12, replace=False)
    off = list(a.routes) + [b.routes[k] for k in pick]
    intro = [0] * len(a.routes) + [1] * 12
    log("dcrex config2", len(off), len(p.routes))
    got = _check(inst.n_depots, inst.N, off, intro, list(p.routes), "config2")
    counts = mdvrp.dcrex_counts(inst.n_depots, inst.N, off, intro, list(p.routes))
    for seed in range(10):
        assert mdvrp.dcrex_pick(counts, seed) == oracle.dcrex_pick(*got, seed), seed


def test_counts_config3_scale():
    """20 x 10000: every route of one start solution against every route of another;
    checked on a grid of pairs against the definitions written with sets (the oracle's
    scan is quadratic in the number of routes)."""
    inst = gen.config3()
    a, p = (gen.start_solution(inst, inst.seed * 1000 + k) for k in range(2))
    log("dcrex config3", len(a.routes), len(p.routes))
    ei, nr, nm, nc = (x.cpu().numpy() for x in mdvrp.dcrex_counts(inst.n_depots, inst.N, list(a.routes),
                                                                    [0] * len(a.routes), list(p.routes)))

    def arcs(route):
        s, xs, e = route
        path = [s] + list(xs) + ([e] if e >= 0 else [])
        return set(zip(path[:-1], path[1:]))

    owner = {}
    for i, r in enumerate(a.routes):
        for arc in arcs(r):
            owner.setdefault(arc, set()).add(i)
    held = {x: i for i, r in enumerate(a.routes) for x in r[1]}
    for i in range(0, len(a.routes), 53):
        Ri = set(a.routes[i][1])
        for j in range(0, len(p.routes), 29):
            Rj = p.routes[j]
            assert ei[i, j] == sum(1 for arc in arcs(Rj) if not (owner.get(arc, set()) - {i}))
            assert nm[i, j] == sum(1 for x in Rj[1] if held[x] != i)
            assert nr[i, j] == len(Ri - set(Rj[1]))
            assert nc[i, j] == 0


def test_pick_edge_cases():
    t = __import__("torch")
    z = t.zeros((0, 3), dtype=t.int32, device="cuda")
    assert mdvrp.dcrex_pick([z, z, z, z], 1) == [-1, -1, 0, 0]
    one = [t.tensor([[v]], dtype=t.int32, device="cuda") for v in (3, 2, 1, 0)]
    assert mdvrp.dcrex_pick(one, 9) == [0, 0, 6, 1]


def test_ucb_sequence_bit_for_bit():
    t = __import__("torch")
    for n_arms, gamma in ((20, 0.99), (5, 0.99), (3, 0.9)):
        R = t.zeros(n_arms, dtype=t.float64, device="cuda")
        N = t.zeros(n_arms, dtype=t.float64, device="cuda")
        Rr = np.zeros(n_arms)
        Nr = np.zeros(n_arms)
        rng = np.random.default_rng(n_arms)
        means = rng.random(n_arms) * 10
        for k in range(300):
            arm = mdvrp.ucb_select(R, N)
            a = int(arm.cpu().numpy()[0])
            assert a == oracle.ucb_select(Rr, Nr), (n_arms, k)
            reward = float(means[a] + rng.standard_normal())
            mdvrp.ucb_update(R, N, arm, t.tensor([reward], dtype=t.float64, device="cuda"), gamma)
            oracle.ucb_update(Rr, Nr, a, reward, gamma)
        assert np.array_equal(R.cpu().numpy().view(np.int64), Rr.view(np.int64))
        assert np.array_equal(N.cpu().numpy().view(np.int64), Nr.view(np.int64))


def test_route_lists_are_checked_on_the_host():
    off = [(0, [1, 2], 0)]
    for bad_par in ([(0, [1, 1], 0)], [(0, [1], 0), (0, [1], 0)], [(3, [1], 0)], [(0, [9], 0)]):
        with pytest.raises(mdvrp.MdvrpError) as e:
            mdvrp.dcrex_counts(1, 5, off, [0], bad_par)
        assert e.value.status == mdvrp.EINVAL
    with pytest.raises(mdvrp.MdvrpError) as e:  # more than 8 copies of customer 1
        mdvrp.dcrex_counts(1, 5, [(0, [1], 0)] * 9, [1] * 9, [(0, [1], 0)])
    assert e.value.status == mdvrp.ENOSPC
