"""Batching: uneven multi-instance batches and graph-captured local-search passes.

A batch holds units (instance, solution) of instances of different sizes; one
launch per kernel class serves all of them. Results must not depend on the
batch composition (bit-exact against the oracle per unit), and a pass replayed
from a captured HIP graph must give exactly what the eager launches give, on
every replay, with eager work and synchronisations between the replays.
"""
import sys

import numpy as np
import pytest

from oracle import ALL_FAMILIES, Ref
from paper_2605_05208_amd import gen, mdvrp
from paper_2605_05208_amd.gen import canonical

pytestmark = pytest.mark.gpu

# the smallest instances of the 256-instance uneven set (customer counts 100..125)
SMALL_UNEVEN = [236, 160, 196, 17, 37, 199]


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_batch(insts, sols_per_inst):
    dev = [mdvrp.Instance(i) for i in insts]
    unit_inst = [k for k, s in enumerate(sols_per_inst) for _ in s]
    B = mdvrp.Batch(dev, unit_inst)
    flat = [s for ss in sols_per_inst for s in ss]
    B.load(flat)
    return dev, B, flat


def _uneven(ids):
    return [gen.config4_instance(i) for i in ids]


def test_uneven_batch_dense_evaluation_matches_oracle():
    insts = _uneven(SMALL_UNEVEN) + [gen.config2()]
    groups = [[gen.start_solution(I, I.seed * 1000)] for I in insts]
    dev, B, flat = make_batch(insts, groups)
    cap = sum(I.n_customers * I.theta * 14 + 2 * I.n_customers * I.n_depots for I in insts) + 1024
    got = B.eval_neighbourhood(ALL_FAMILIES, dense_cap=cap)
    for u, I in enumerate(insts):
        exp = Ref(I).eval(flat[u], ALL_FAMILIES)
        g = got[got["unit"] == u]
        log(f"unit {u}: {I.name} {len(g)} moves")
        assert len(g) == len(exp)
        g = g[np.argsort(g["id"], kind="stable")]
        e = exp[np.argsort(exp["id"], kind="stable")]
        assert np.array_equal(g["id"], e["id"])
        for f in ("dF", "dD", "dTW", "dLX", "dDX", "dV4"):
            assert np.array_equal(g[f], e[f]), f"unit {u} field {f}"


def test_uneven_batch_local_search_matches_oracle():
    insts = _uneven(SMALL_UNEVEN)
    groups = [[gen.start_solution(I, I.seed * 1000 + j) for j in range(2)] for I in insts]
    dev, B, flat = make_batch(insts, groups)
    st = B.local_search_to_optimum(seed=7, graph=True)
    out = B.export()
    unit_inst = [k for k, s in enumerate(groups) for _ in s]
    for k, I in enumerate(insts):
        sols, rst = Ref(I).local_search(groups[k], seed=7)
        for j in range(2):
            u = unit_inst.index(k) + j
            assert canonical(out[u].routes) == canonical(sols[j].routes), f"{I.name} solution {j}"
            for key in ("passes", "steps", "moves_applied", "evaluated", "F"):
                assert st[u][key] == rst[j][key], f"{I.name} solution {j}: {key}"
            assert st[u]["converged"] == 1 and st[u]["device_ms"] > 0


def _eager_vs_graph(B, sols, reps=3, **kw):
    B.load(sols)
    ref = B.local_search_to_optimum(**kw)
    ref_sol = [canonical(s.routes) for s in B.export()]
    for r in range(reps):
        B.load(sols)
        st = B.local_search_to_optimum(graph=True, **kw)
        got = [canonical(s.routes) for s in B.export()]
        assert got == ref_sol, f"replay {r}: solutions differ from the eager run"
        for a, b in zip(st, ref):
            for key in ("passes", "steps", "moves_applied", "evaluated", "F", "fallback_passes", "converged"):
                assert a[key] == b[key], f"replay {r}: {key}"
        # eager work and a synchronisation between the replays
        B.load(sols)
        B.eval_neighbourhood(ALL_FAMILIES)
        B.cost()


@pytest.mark.parametrize("tw,open_r", [(0, 0), (0, 1), (1, 0), (1, 1)])
@pytest.mark.parametrize("mode", [0, 1])
def test_graph_passes_equal_eager_passes_tiny(tw, open_r, mode):
    insts = [gen.tiny(72_000 + 10 * tw + open_r + k, has_tw=tw, open_routes=open_r, nc=30 + 7 * k) for k in range(3)]
    groups = [[gen.start_solution(I, I.seed * 1000 + j) for j in range(2)] for I in insts]
    dev, B, flat = make_batch(insts, groups)
    _eager_vs_graph(B, flat, mode=mode, seed=3)


def test_graph_passes_on_a_side_stream_config2():
    import torch
    I = gen.config2()
    sols = [gen.start_solution(I, I.seed * 1000 + j) for j in range(8)]
    dev, B, flat = make_batch([I], [sols])
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        _eager_vs_graph(B, flat, seed=1, reps=2, poll_every=4)
    torch.cuda.synchronize()


def test_graph_passes_with_the_learned_filter():
    I = gen.config2()
    sols = [gen.start_solution(I, I.seed * 1000 + j) for j in range(4)]
    dev, B, flat = make_batch([I], [sols])
    B.filter_attach(8)
    rng = np.random.default_rng(3)
    from paper_2605_05208_amd import filter_train as ft
    M = mdvrp.Mlp(ft.init_params(1))
    for rescore in (mdvrp.RESCORE_STEP, mdvrp.RESCORE_PASS):
        _eager_vs_graph(B, flat, seed=2, reps=2, filter=mdvrp.FILTER_MLP, mlp=M, rescore=rescore)
    del rng


# ----------------------------------------------------------------------------- tile shapes and autotuner

def _ls_fingerprint(B, sols, **kw):
    B.load(sols)
    st = B.local_search_to_optimum(**kw)
    return [canonical(s.routes) for s in B.export()], [(s["passes"], s["steps"], s["moves_applied"], s["evaluated"],
                                                         s["F"]) for s in st]


@pytest.mark.parametrize("tw,open_r", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_tile_shapes_give_identical_searches(tw, open_r):
    insts = [gen.tiny(73_000 + 10 * tw + open_r + k, has_tw=tw, open_routes=open_r, nc=40 + 9 * k) for k in range(3)]
    groups = [[gen.start_solution(I, I.seed * 1000 + j) for j in range(2)] for I in insts]
    dev, B, flat = make_batch(insts, groups)
    ref = _ls_fingerprint(B, flat, seed=5)
    ref_union = _ls_fingerprint(B, flat, seed=5, mode=1)
    for threads in (128, 64):
        B.set_tile_shapes([threads] * 6)
        assert _ls_fingerprint(B, flat, seed=5) == ref, f"{threads} threads per block"
        assert _ls_fingerprint(B, flat, seed=5, graph=True) == ref, f"{threads} threads per block, graph"
    B.set_tile_shapes([256, 128, 64, 128, 64, 256])
    assert _ls_fingerprint(B, flat, seed=5) == ref
    assert _ls_fingerprint(B, flat, seed=5, mode=1) == ref_union


def test_autotune_on_config2_keeps_results_and_counters():
    I = gen.config2()
    sols = [gen.start_solution(I, I.seed * 1000 + j) for j in range(8)]
    dev, B, flat = make_batch([I], [sols])
    ref = _ls_fingerprint(B, flat, seed=1, poll_every=4)
    B.load(flat)
    before = B.state()[:, 1].copy()
    shapes = B.autotune(reps=2)
    log("  tuned threads per block", shapes)
    assert all(x in (256, 128, 64) for x in shapes)
    assert np.array_equal(B.state()[:, 1], before), "autotuning changed the evaluation counters"
    assert _ls_fingerprint(B, flat, seed=1, poll_every=4) == ref
    assert _ls_fingerprint(B, flat, seed=1, poll_every=4, graph=True) == ref


# ----------------------------------------------------------------------------- matrix layout

@pytest.mark.parametrize("which", ["tiny_nt", "tiny_tw_open", "config2"])
def test_ordered_layout_gives_identical_results(which):
    """The locality-ordered copy of the matrices changes where the kernels read, never what."""
    if which == "config2":
        insts = [gen.config2()]
        groups = [[gen.start_solution(insts[0], insts[0].seed * 1000 + j) for j in range(4)]]
    else:
        tw, o = (0, 0) if which == "tiny_nt" else (1, 1)
        insts = [gen.tiny(74_000 + k, has_tw=tw, open_routes=o, nc=30 + 11 * k) for k in range(3)]
        groups = [[gen.start_solution(I, I.seed * 1000 + j) for j in range(2)] for I in insts]
    flat = [s for g in groups for s in g]
    unit_inst = [k for k, g in enumerate(groups) for _ in g]
    res = {}
    for layout in (mdvrp.LAYOUT_GIVEN, mdvrp.LAYOUT_ORDERED):
        dev = [mdvrp.Instance(I, layout=layout) for I in insts]
        B = mdvrp.Batch(dev, unit_inst)
        B.load(flat)
        cap = sum(I.n_customers * I.theta * 14 + 2 * I.n_customers * I.n_depots for I in insts) * 2 + 1024
        d = B.eval_neighbourhood(ALL_FAMILIES, dense_cap=cap)
        d = d[np.lexsort((d["id"], d["unit"]))]
        res[layout] = (d, _ls_fingerprint(B, flat, seed=4), B.features())
    (d0, f0, x0), (d1, f1, x1) = res[mdvrp.LAYOUT_GIVEN], res[mdvrp.LAYOUT_ORDERED]
    assert np.array_equal(d0["id"], d1["id"]) and np.array_equal(d0["dF"], d1["dF"])
    assert f0 == f1
    assert np.array_equal(x0, x1)


@pytest.mark.parametrize("graph,open_r", [(False, 0), (True, 1)])
def test_results_do_not_depend_on_the_poll_interval(graph, open_r):
    """The host reads the active-unit count of one poll interval while the next one
    runs; the extra passes after convergence must change nothing."""
    insts = [gen.tiny(76_000 + k, has_tw=1, open_routes=open_r, nc=35 + 8 * k) for k in range(2)]
    groups = [[gen.start_solution(I, I.seed * 1000 + j) for j in range(2)] for I in insts]
    dev, B, flat = make_batch(insts, groups)
    ref = None
    for poll in (1, 2, 5, 11):
        got = _ls_fingerprint(B, flat, seed=9, poll_every=poll, graph=graph)
        if ref is None:
            ref = got
        assert got == ref, f"poll_every={poll}"
