"""Dynamic penalty coefficients (Section 3.2.1; kappa = 1/2 of Table 1) on the GPU
against the oracle: after every step that applied moves each of the four weights
doubles when the new solution violates its term and halves (rounding down)
otherwise, within the caller's bounds. Whole trajectories are compared exactly:
final routes, F under the final weights, passes, steps, moves, evaluated moves
and the final weights themselves."""
import sys

import numpy as np
import pytest

from oracle import Ref
from paper_2605_05208_amd import gen, mdvrp
from paper_2605_05208_amd.gen import canonical

pytestmark = pytest.mark.gpu

LO = [1, 1, 1, 1]
HI = [1 << 12, 1 << 12, 1 << 12, 1 << 16]


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _tiny_group(tw, open_r, n_inst=16, base=0):
    insts = []
    for k in range(n_inst):
        seed = 95_000 + base + 100 * tw + 10 * open_r + k
        theta = None if k % 3 else 3
        Dmax = 40 if (k % 4 == 1 and not tw) else -1
        insts.append(gen.tiny(seed, has_tw=tw, open_routes=open_r, theta=theta, Dmax=Dmax))
    sols = [[gen.random_solution(i, 11 * k + 1), gen.start_solution(i, 11 * k + 2)] for k, i in enumerate(insts)]
    return insts, sols


def _compare(insts, sols, mode=0, seed=1, adapt=(LO, HI), graph=False, max_passes=40, tag=""):
    dev = [mdvrp.Instance(i) for i in insts]
    unit_inst = [k for k, s in enumerate(sols) for _ in s]
    B = mdvrp.Batch(dev, unit_inst)
    flat = [s for ss in sols for s in ss]
    B.load(flat)
    st = B.local_search_to_optimum(mode=mode, seed=seed, max_passes=max_passes, adapt=adapt, graph=graph)
    got = B.export()
    Fg, _ = B.cost()
    u = 0
    moved = 0
    for k, inst in enumerate(insts):
        out, rst = Ref(inst).local_search(sols[k], mode=mode, seed=seed, max_passes=max_passes, adapt=adapt)
        for j in range(len(sols[k])):
            g, r = st[u], rst[j]
            tagu = f"{tag} inst {k} unit {u}"
            assert canonical(got[u].routes) == canonical(out[j].routes), tagu
            assert g["w_final"] == r["w_final"], f"{tagu}: weights {g['w_final']} vs {r['w_final']}"
            assert int(Fg[u]) == r["F"] == g["F"], tagu
            for key in ("passes", "steps", "moves_applied", "evaluated"):
                assert g[key] == r[key], f"{tagu}: {key} {g[key]} vs {r[key]}"
            assert g["err"] == 0
            w0 = [inst.w_tw, inst.w_load, inst.w_dur]
            moved += int(g["w_final"][:3] != w0)
            u += 1
    return B, flat, st, moved


@pytest.mark.parametrize("tw,open_r", [(0, 0), (0, 1), (1, 0), (1, 1)])
@pytest.mark.parametrize("mode", [0, 1])
def test_adaptive_search_tiny_multi_instance(tw, open_r, mode):
    insts, sols = _tiny_group(tw, open_r, base=10 * mode)
    log("adaptive tiny", tw, open_r, mode)
    _, _, _, moved = _compare(insts, sols, mode=mode, seed=31, tag=f"tiny tw={tw} open={open_r} mode={mode}")
    assert moved > 0, "no weight changed: the test would not see the update rule"


def test_adaptive_search_config1():
    inst = gen.config1()
    log("adaptive config1")
    sols = [gen.start_solution(inst, inst.seed * 1000 + k) for k in range(3)]
    _compare([inst], [sols], seed=7, tag="config1")


def test_adaptive_search_config2_two_solutions():
    inst = gen.config2()
    log("adaptive config2")
    sols = [gen.start_solution(inst, inst.seed * 1000 + k) for k in range(2)]
    _compare([inst], [sols], seed=2, max_passes=12, adapt=([1, 1, 1, 1], [1 << 10, 1 << 10, 1 << 10, 1 << 20]),
             tag="config2")


def test_adaptive_search_depth_limit_and_graph():
    """A short depth (max_passes) and passes replayed from captured graphs."""
    insts, sols = _tiny_group(1, 0, n_inst=8, base=500)
    log("adaptive depth + graph")
    _compare(insts, sols, seed=3, max_passes=3, tag="depth 3")
    _compare(insts, sols, seed=3, max_passes=25, graph=True, tag="graph")


def test_fixed_bounds_equal_the_fixed_weight_search():
    """w_min = w_max = the instance's weights: nothing can move, so the adaptive search
    is the fixed-weight one."""
    inst = gen.config1()
    sols = [gen.start_solution(inst, inst.seed * 1000 + k) for k in range(2)]
    dev = mdvrp.Instance(inst)
    w = [inst.w_tw, inst.w_load, inst.w_dur, dev.info()["w_depot"]]
    B = mdvrp.Batch([dev], [0, 0])
    B.load(sols)
    a = B.local_search_to_optimum(seed=9, max_passes=1000, adapt=(w, w))
    ea = [canonical(s.routes) for s in B.export()]
    B.load(sols)
    b = B.local_search_to_optimum(seed=9)
    eb = [canonical(s.routes) for s in B.export()]
    assert ea == eb
    for x, y in zip(a, b):
        assert x["w_final"] == w and y["passes"] < 1000
        for key in ("F", "passes", "steps", "moves_applied", "evaluated"):
            assert x[key] == y[key], key


def test_load_resets_the_weights():
    """After an adaptive search the batch keeps the final weights (F is under them);
    loading solutions returns every unit to its instance's weights."""
    inst = gen.tiny(777, has_tw=1)
    sols = [gen.random_solution(inst, 5), gen.random_solution(inst, 6)]
    dev = mdvrp.Instance(inst)
    B = mdvrp.Batch([dev], [0, 0])
    B.load(sols)
    st = B.local_search_to_optimum(seed=4, max_passes=30, adapt=(LO, HI))
    state = B.state()
    for k in range(2):
        assert list(state[k, 12:16]) == st[k]["w_final"]
    B.load(sols)
    state = B.state()
    w0 = [inst.w_tw, inst.w_load, inst.w_dur, dev.info()["w_depot"]]
    F, _ = B.cost()
    ref = Ref(inst)
    for k in range(2):
        assert list(state[k, 12:16]) == w0
        assert int(F[k]) == ref.cost(sols[k])[0]


def test_bounds_are_checked_on_the_host():
    inst = gen.tiny(778)
    B = mdvrp.Batch([mdvrp.Instance(inst)], [0])
    B.load([gen.start_solution(inst, 1)])
    bad = [(([2, 1, 1, 1], [1, 8, 8, 8]), 10), (([-1, 1, 1, 1], [8, 8, 8, 8]), 10),
           (([1, 1, 1, 1], [8, 8, 8, (1 << 30) + 1]), 10), (([1, 1, 1, 1], [8, 8, 8, 8]), 0)]
    for bounds, depth in bad:  # depth 0: no depth, which a search with moving weights needs
        with pytest.raises(mdvrp.MdvrpError) as e:
            B.local_search_to_optimum(max_passes=depth, adapt=bounds)
        assert e.value.status == mdvrp.EINVAL
    assert np.all(B.state()[:, 5] == 0)
