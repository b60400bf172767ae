"""Edge cases of the HIP path against the oracle, exact integers throughout.

* instances with a single customer (empty granular lists, one one-customer
  route; 1-3 depots, with and without time windows, closed and open routes);
* the largest granular lists the library accepts (theta = 128) on medium
  instances, with and without time windows;
* a search that starts at a local optimum (one pass, nothing applied);
* one batch that mixes all of these with ordinary units;
* long routes (up to about 80 customers), whose rebuild in the fused step takes a
  whole wavefront and, beyond 62 customers, more than one 64-position chunk, beside
  short routes built two per wavefront.
"""
import numpy as np
import pytest

from oracle import ALL_FAMILIES, Ref
from paper_2605_05208_amd import gen
from paper_2605_05208_amd.gen import canonical
from test_gpu_parity import _ls_compare, compare_dense, dense_cap_for, log, make_batch

pytestmark = pytest.mark.gpu


def _one_customer(nd, tw, open_r):
    return gen.tiny(77_000 + 10 * nd + 2 * tw + open_r, has_tw=tw, open_routes=open_r, nd=nd, nc=1, theta=1)


def _theta128_tw():
    return gen._tw_instance(np.random.default_rng(7), 4, 400, 1000, 50.0, 4, 30, 200, 90, 10_000, 128,
                            "mdvrptw-4x400-theta128", 7)


def _theta128_plain():
    rng = np.random.default_rng(8)
    nd, nc = 3, 300
    xy = rng.integers(0, 1001, size=(nd + nc, 2))
    q = np.concatenate([np.zeros(nd, np.int64), rng.integers(1, 26, nc)])
    n = nd + nc
    return gen._make(nd, nc, xy, 10, q, np.zeros(n), np.zeros(n), np.full(n, gen.BIG_HORIZON), Q=200, NV=6,
                     Dmax=-1, open_routes=0, has_tw=0, theta=128, w_tw=0, w_load=10, w_dur=0, w_depot=-1,
                     name="mdvrp-3x300-theta128", seed=8)


def _dense_compare(insts, sols, fam, tag):
    dev, B, flat = make_batch(insts, sols)
    got = B.eval_neighbourhood(fam, dense_cap=dense_cap_for([insts[k] for k in B.unit_inst]))
    u = 0
    for k, inst in enumerate(insts):
        ref = Ref(inst)
        for sol in sols[k]:
            compare_dense(got[got["unit"] == u], ref.eval(sol, fam), inst.n_customers, f"{tag} inst {k} unit {u}")
            u += 1


@pytest.mark.parametrize("tw,open_r", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_one_customer_instances(tw, open_r):
    insts = [_one_customer(nd, tw, open_r) for nd in (1, 2, 3)]
    sols = [[gen.random_solution(i, 3), gen.start_solution(i, 4)] for i in insts]
    log("one customer", tw, open_r)
    for fam in [ALL_FAMILIES, 1, 2, 4, 8, 16, 32]:
        _dense_compare(insts, sols, fam, f"one customer tw={tw} open={open_r} fam {fam}")
    _ls_compare(insts, sols, 0, 11, tag=f"one customer tw={tw} open={open_r}")
    _ls_compare(insts, sols, 1, 11, tag=f"one customer union tw={tw} open={open_r}")


@pytest.mark.parametrize("which", ["tw", "plain"])
def test_maximum_theta(which):
    inst = _theta128_tw() if which == "tw" else _theta128_plain()
    assert inst.theta == 128 and inst.n_customers > 129
    sols = [gen.start_solution(inst, 7000 + k) for k in range(2)]
    log("theta 128", which)
    _dense_compare([inst], [sols], ALL_FAMILIES, f"theta 128 {which}")
    _ls_compare([inst], [sols], 0, 2, tag=f"theta 128 {which}")


def test_search_started_at_a_local_optimum():
    inst = gen.config1()
    sols = [gen.start_solution(inst, inst.seed * 1000 + k) for k in range(3)]
    log("restart at optimum")
    dev, B, flat = make_batch([inst], [sols])
    B.local_search_to_optimum(seed=9)
    opt = B.export()
    F1, _ = B.cost()
    dev2, B2, _ = make_batch([inst], [opt])
    st = B2.local_search_to_optimum(seed=9)
    F2, _ = B2.cost()
    assert np.array_equal(F1, F2)
    for u, s in enumerate(st):
        assert s["moves_applied"] == 0 and s["passes"] == 1, (u, s)
        assert canonical(B2.export()[u].routes) == canonical(opt[u].routes)
    _ls_compare([inst], [opt], 0, 9, tag="restart at optimum")


def test_batch_mixing_edge_cases_with_ordinary_units():
    insts = [_one_customer(2, 1, 0), _theta128_tw(), gen.tiny(31_337, has_tw=1), _one_customer(3, 1, 0)]
    sols = [[gen.start_solution(insts[0], 1)],
            [gen.start_solution(insts[1], 7100)],
            [gen.random_solution(insts[2], 5), gen.start_solution(insts[2], 6)],
            [gen.random_solution(insts[3], 2)]]
    log("mixed edge batch")
    _dense_compare(insts, sols, ALL_FAMILIES, "mixed edge batch")
    _ls_compare(insts, sols, 0, 13, tag="mixed edge batch")


@pytest.mark.parametrize("tw,open_r", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_many_depots(tw, open_r):
    """64 depots (the depot operators read the instance's depot-arc table) and 65 (they
    read the matrices), in one batch."""
    insts = [gen.tiny(88_100 + 10 * nd + 2 * tw + open_r, has_tw=tw, open_routes=open_r, nd=nd, nc=8)
             for nd in (64, 65)]
    sols = [[gen.random_solution(i, 3), gen.start_solution(i, 4)] for i in insts]
    log("many depots", tw, open_r)
    for fam in [ALL_FAMILIES, 16, 32]:
        _dense_compare(insts, sols, fam, f"many depots tw={tw} open={open_r} fam {fam}")
    _ls_compare(insts, sols, 0, 17, tag=f"many depots tw={tw} open={open_r}")


def _long_routes(tw, open_r):
    """Two depots, capacity so large that the start solution has one route per depot."""
    rng = np.random.default_rng(61 + 2 * tw + open_r)
    if tw:
        inst = gen._tw_instance(rng, 2, 130, 1000, 60.0, 3, 30, 10**6, 10, 200_000, 16,
                                "mdvrptw-2x130-long", 61, NV=3)
    else:
        nd, nc = 2, 160
        xy = rng.integers(0, 1001, size=(nd + nc, 2))
        q = np.concatenate([np.zeros(nd, np.int64), rng.integers(1, 26, nc)])
        n = nd + nc
        inst = gen._make(nd, nc, xy, 10, q, np.zeros(n), np.zeros(n), np.full(n, gen.BIG_HORIZON), Q=10**6,
                         NV=3, Dmax=-1, open_routes=0, has_tw=0, theta=16, w_tw=0, w_load=10, w_dur=0,
                         w_depot=-1, name="mdvrp-2x160-long", seed=62)
    inst.open_routes = open_r
    return inst


@pytest.mark.parametrize("tw,open_r", [(0, 0), (0, 1), (1, 0)])
def test_long_routes_in_the_fused_step(tw, open_r):
    inst = _long_routes(tw, open_r)
    sols = [gen.start_solution(inst, 5), gen.start_solution(inst, 6)]
    assert max(len(r[1]) for s in sols for r in s.routes) > 62
    log("long routes", tw, open_r)
    _ls_compare([inst], [sols], 0, 77, max_passes=6, tag=f"long tw={tw} open={open_r}")
