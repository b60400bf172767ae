"""Repair insertions (Section 3.3, after Algorithm 3) on the GPU against the
oracle: for every operator (FBI, IBI, FRI, IRI, RI) the completed solutions, the
order in which customers were inserted, the number of positions evaluated and
F are compared exactly."""
import sys

import numpy as np
import pytest

from oracle import Ref
from paper_2605_05208_amd import gen, mdvrp
from paper_2605_05208_amd.gen import Solution, canonical

pytestmark = pytest.mark.gpu

OPS = [mdvrp.REPAIR_FBI, mdvrp.REPAIR_IBI, mdvrp.REPAIR_FRI, mdvrp.REPAIR_IRI, mdvrp.REPAIR_RI]


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _partial(inst, seed, drop, base=None):
    rng = np.random.default_rng(seed)
    full = base if base is not None else gen.random_solution(inst, seed)
    gone = set(rng.choice(np.arange(inst.n_depots, inst.N), size=drop, replace=False).tolist())
    routes = [(a, [x for x in xs if x not in gone], b) for a, xs, b in full.routes]
    return Solution([r for r in routes if r[1]])


def _compare(insts, parts, op, seed, tag):
    dev = [mdvrp.Instance(i) for i in insts]
    unit_inst = [k for k, ps in enumerate(parts) for _ in ps]
    B = mdvrp.Batch(dev, unit_inst)
    flat = [p for ps in parts for p in ps]
    B.load_partial(flat)
    order, nev = B.repair(op, seed=seed)
    got = B.export()
    F, _ = B.cost()
    u = 0
    for k, inst in enumerate(insts):
        ref = Ref(inst)
        for p in parts[k]:
            out, rorder, rnev = ref.repair(p, op, seed=seed)
            tagu = f"{tag} op {op} inst {k} unit {u}"
            assert order[u] == rorder, tagu
            assert canonical(got[u].routes) == canonical(out.routes), tagu
            assert nev[u] == rnev, f"{tagu}: evaluated {nev[u]} vs {rnev}"
            assert int(F[u]) == ref.cost(out)[0], tagu
            u += 1
    return B


@pytest.mark.parametrize("tw,open_r", [(0, 0), (0, 1), (1, 0), (1, 1)])
@pytest.mark.parametrize("op", OPS)
def test_repair_tiny_multi_instance(tw, open_r, op):
    insts, parts = [], []
    for k in range(10):
        inst = gen.tiny(7000 + 100 * tw + 10 * open_r + k, has_tw=tw, open_routes=open_r, nc=9 + k % 4)
        if k % 3 == 1:
            inst.Q = int(inst.q.max()) + 2  # tight: FBI / FRI open routes
        insts.append(inst)
        drop = 1 + k % 5
        parts.append([_partial(inst, 3 * k + 1, drop), _partial(inst, 3 * k + 2, min(inst.n_customers, drop + 3))])
    log("repair tiny", tw, open_r, op)
    _compare(insts, parts, op, seed=17 + op, tag=f"tiny tw={tw} open={open_r}")


@pytest.mark.parametrize("op", OPS)
def test_repair_config2(op):
    """MDVRPTW 8 x 1000: two start solutions with 40 and 25 customers removed."""
    inst = gen.config2()
    parts = [[_partial(inst, 10 + j, n, gen.start_solution(inst, inst.seed * 1000 + j)) for j, n in ((0, 40), (1, 25))]]
    log("repair config2", op)
    _compare([inst], parts, op, seed=5, tag="config2")


def test_repair_config3_open_then_search():
    """MDOVRP 20 x 10000 (400 MB matrix): 30 customers removed, infeasible regret insertion;
    the completed batch then runs a pass of the local search like any other."""
    inst = gen.config3(open_routes=1)
    part = _partial(inst, 99, 30, gen.start_solution(inst, inst.seed * 1000))
    log("repair config3 open")
    B = _compare([inst], [[part]], mdvrp.REPAIR_IRI, seed=1, tag="config3 open")
    st = B.local_search_to_optimum(seed=3, max_passes=1)
    assert st[0]["err"] == 0 and st[0]["moves_applied"] > 0


def test_search_after_repair_matches_the_oracle():
    insts = [gen.tiny(7500 + k, has_tw=1, nc=10) for k in range(6)]
    parts = [[_partial(i, k, 3)] for k, i in enumerate(insts)]
    dev = [mdvrp.Instance(i) for i in insts]
    B = mdvrp.Batch(dev, list(range(len(insts))))
    B.load_partial([p[0] for p in parts])
    B.repair(mdvrp.REPAIR_FRI)
    st = B.local_search_to_optimum(seed=8)
    got = B.export()
    for k, inst in enumerate(insts):
        ref = Ref(inst)
        full, _, _ = ref.repair(parts[k][0], mdvrp.REPAIR_FRI)
        out, rst = ref.local_search([full], seed=8)
        assert canonical(got[k].routes) == canonical(out[0].routes)
        for key in ("F", "passes", "steps", "moves_applied", "evaluated"):
            assert st[k][key] == rst[0][key], key


def test_partial_batches_are_checked():
    inst = gen.tiny(7600, nc=8)
    B = mdvrp.Batch([mdvrp.Instance(inst)], [0])
    B.load_partial([_partial(inst, 1, 3)])
    with pytest.raises(mdvrp.MdvrpError) as e:  # evaluation needs every customer routed
        B.local_search_to_optimum()
    assert e.value.status == mdvrp.ESTATE
    with pytest.raises(mdvrp.MdvrpError) as e:
        B.repair(7)
    assert e.value.status == mdvrp.EINVAL
    with pytest.raises(mdvrp.MdvrpError) as e:  # a customer twice
        B.load_partial([Solution([(0, [inst.n_depots, inst.n_depots], 0)])])
    assert e.value.status == mdvrp.EINVAL
    # nothing missing: repair leaves the solution as it is
    full = gen.random_solution(inst, 2)
    B.load_partial([full])
    order, nev = B.repair(mdvrp.REPAIR_FBI)
    assert order == [[]] and nev == [0]
    assert canonical(B.export()[0].routes) == canonical(full.routes)
    # everything missing: routes are opened from nothing
    B.load_partial([Solution([])])
    order, _ = B.repair(mdvrp.REPAIR_IBI)
    out, rorder, _ = Ref(inst).repair(Solution([]), mdvrp.REPAIR_IBI)
    assert order == [rorder] and canonical(B.export()[0].routes) == canonical(out.routes)
