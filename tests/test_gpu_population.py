"""Population measures of Section 3.4 on the GPU against the oracle: the
distance between solutions (Eq. 7; common arc counts and edge-set sizes exactly,
the fp64 distance bit for bit, both sides rounding the quotient, the difference
and the product once each in that order), and the reduction to mu members by
the score of Eq. 5 (survivors, removal order, scores and population distances
bit for bit)."""
import json
import os
import sys

import numpy as np
import pytest

import oracle
from oracle import Ref
from paper_2605_05208_amd import gen, mdvrp

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_cases.json")))


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def torch():
    import torch as t
    return t


def _batch(inst, sols, extra_inst=None):
    insts = [inst] + ([extra_inst] if extra_inst is not None else [])
    dev = [mdvrp.Instance(i) for i in insts]
    unit_inst = [0] * len(sols) + ([1] if extra_inst is not None else [])
    B = mdvrp.Batch(dev, unit_inst)
    flat = list(sols) + ([gen.start_solution(extra_inst, 1)] if extra_inst is not None else [])
    B.load(flat)
    return dev, B


def _check_distance(B, units, sols, inst, tag):
    d, c, ne = (x.cpu().numpy() for x in B.population_distance(units))
    rd, rc, rne = Ref(inst).population_distance(sols)
    assert np.array_equal(ne, rne), tag
    assert np.array_equal(c, rc), tag
    assert np.array_equal(d.view(np.int64), rd.view(np.int64)), tag  # bit for bit


@pytest.mark.parametrize("tw,open_r", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_distance_tiny(tw, open_r):
    inst = gen.tiny(6100 + 10 * tw + open_r, has_tw=tw, open_routes=open_r)
    sols = [gen.random_solution(inst, k) for k in range(9)] + [gen.start_solution(inst, 3)]
    sols.append(sols[4])  # a duplicate: distance 0
    log("population tiny", tw, open_r)
    dev, B = _batch(inst, sols, extra_inst=gen.tiny(6199, has_tw=tw, open_routes=open_r))
    units = list(range(len(sols)))
    _check_distance(B, units, sols, inst, f"tiny tw={tw} open={open_r}")
    # a permuted subset of the members
    sub = [7, 2, 10, 0, 5]
    _check_distance(B, sub, [sols[k] for k in sub], inst, "subset")


def test_distance_and_reduce_config2_after_search():
    """64 MDVRPTW solutions after 6 passes of the local search (close to each other):
    distances, then the reduction to mu = 20 with xi = 0.7 and 5 nearest (Table 1)."""
    t = torch()
    inst = gen.config2()
    sols = [gen.start_solution(inst, inst.seed * 1000 + k) for k in range(64)]
    log("population config2")
    dev, B = _batch(inst, sols)
    B.local_search_to_optimum(seed=1, max_passes=6)
    cur = B.export()
    units = list(range(64))
    _check_distance(B, units, cur, inst, "config2")
    d, _, _ = B.population_distance(units)
    F, _ = B.cost()
    f = t.from_numpy(np.ascontiguousarray(F)).to("cuda")
    keep, order, chi, dpop = (x.cpu().numpy() for x in mdvrp.population_reduce(d, f, 20, 0.7, 5))
    rkeep, rorder, rchi, rdpop = oracle.population_reduce(d.cpu().numpy(), F, 20, 0.7, 5)
    assert np.array_equal(keep, rkeep) and np.array_equal(order, rorder)
    assert np.array_equal(chi.view(np.int64), rchi.view(np.int64))
    assert np.array_equal(dpop.view(np.int64), rdpop.view(np.int64))
    assert keep.sum() == 20


@pytest.mark.parametrize("case", GOLDEN["population_reduce"], ids=lambda c: c["note"][:40])
def test_reduce_worked_examples(case):
    t = torch()
    d = t.tensor(case["dist"], dtype=t.float64, device="cuda")
    f = t.tensor(case["f"], dtype=t.int64, device="cuda")
    keep, order, chi, dpop = (x.cpu().numpy() for x in mdvrp.population_reduce(d, f, case["mu"], case["xi"],
                                                                                 case["n_close"]))
    assert keep.tolist() == case["keep"] and order.tolist() == case["order"]
    assert np.allclose(chi, case["chi"], rtol=0, atol=1e-12)
    assert np.allclose(dpop, case["dpop"], rtol=0, atol=1e-12)


@pytest.mark.parametrize("n,mu,n_close", [(1, 1, 5), (6, 10, 5), (40, 20, 16), (300, 100, 5), (1024, 1012, 3)])
def test_reduce_sizes_against_the_oracle(n, mu, n_close):
    """Random symmetric matrices with repeated values (ties) and repeated objectives,
    from one member to the largest population of a call."""
    t = torch()
    rng = np.random.default_rng(n * 31 + mu)
    a = rng.integers(0, 12, (n, n)).astype(np.float64) * 7.5
    dist = np.triu(a, 1) + np.triu(a, 1).T
    f = rng.integers(0, max(2, n // 3), n).astype(np.int64)
    log("reduce", n, mu, n_close)
    out = mdvrp.population_reduce(t.from_numpy(dist).to("cuda"), t.from_numpy(f).to("cuda"), mu, 0.7, n_close)
    keep, order, chi, dpop = (x.cpu().numpy() for x in out)
    rkeep, rorder, rchi, rdpop = oracle.population_reduce(dist, f, mu, 0.7, n_close)
    assert np.array_equal(keep, rkeep) and np.array_equal(order, rorder)
    assert np.array_equal(chi.view(np.int64), rchi.view(np.int64))
    assert np.array_equal(dpop.view(np.int64), rdpop.view(np.int64))


def test_member_lists_are_checked_on_the_host():
    inst = gen.tiny(6300)
    sols = [gen.random_solution(inst, k) for k in range(3)]
    dev, B = _batch(inst, sols, extra_inst=gen.tiny(6301))
    for units in ([0, 0], [0, 3], [0, 7], [], [-1]):  # repeat, other instance, out of range, empty
        with pytest.raises(mdvrp.MdvrpError) as e:
            B.population_distance(units)
        assert e.value.status == mdvrp.EINVAL
    t = torch()
    d = t.zeros((3, 3), dtype=t.float64, device="cuda")
    f = t.zeros(3, dtype=t.int64, device="cuda")
    for mu, n_close in ((0, 5), (2, 0), (2, 17)):
        with pytest.raises(mdvrp.MdvrpError) as e:
            mdvrp.population_reduce(d, f, mu, 0.7, n_close)
        assert e.value.status == mdvrp.EINVAL
