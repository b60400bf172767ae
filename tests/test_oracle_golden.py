"""Worked examples of the paper's definitions, stored as text fixtures in
tests/golden/hand_cases.json (each with its citation), checked against the CPU
oracle. No GPU."""
import json
import os

import numpy as np
import pytest

from oracle import KIND_NAMES, Ref
from paper_2605_05208_amd import gen
from paper_2605_05208_amd.gen import Instance, Solution

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_cases.json")))


def _instance(case, **kw):
    xy = np.asarray(case["xy"], np.int64)
    n = len(xy)
    d = xy[:, None, :] - xy[None, :, :]
    c = np.floor(np.sqrt((d * d).sum(-1)) * 10 + 0.5).astype(np.int32)
    z = np.zeros(n, np.int32)
    nd = case["n_depots"]
    args = dict(n_depots=nd, n_customers=n - nd, c=c, t=c, q=np.asarray(case["q"], np.int32), s=z, e=z,
                l=np.full(n, gen.BIG_HORIZON, np.int32), Q=case["Q"], NV=case.get("NV", 4), Dmax=-1,
                open_routes=0, has_tw=0, theta=n - nd - 1, w_tw=0, w_load=case.get("w_load", 10), w_dur=0,
                w_depot=-1)
    args.update(kw)
    return Instance(**args)


def _routes(case):
    return Solution([(a, list(xs), b) for a, xs, b in case["routes"]])


@pytest.mark.parametrize("case", GOLDEN["cost"], ids=lambda c: c["note"][:30])
def test_cost_worked_example(case):
    F, terms = Ref(_instance(case)).cost(_routes(case))
    assert terms.tolist() == case["terms"]
    assert F == case["F"]


@pytest.mark.parametrize("case", GOLDEN["time_warp"], ids=lambda c: c["note"][:30])
def test_time_warp_worked_example(case):
    """One open route from depot 0 through the windowed nodes; F with w_tw = 1
    reads off the time warp, with w_dur = 1 and Dmax = 0 the duration."""
    win, travel = case["windows"], case["travel"]
    n = len(win)
    c = np.zeros((n, n), np.int32)
    for k, tk in enumerate(travel):
        c[k, k + 1] = c[k + 1, k] = tk
    e = np.array([a for a, _ in win], np.int32)
    l = np.array([b for _, b in win], np.int32)
    base = dict(n_depots=1, n_customers=n - 1, c=c, t=c, q=np.zeros(n, np.int32), s=np.zeros(n, np.int32),
                e=e, l=l, Q=10, NV=9, Dmax=0, open_routes=1, has_tw=1, theta=1, w_load=0, w_depot=0)
    sol = Solution([(0, list(range(1, n)), -1)])
    _, t_tw = Ref(Instance(**base, w_tw=1, w_dur=0)).cost(sol)
    _, t_dur = Ref(Instance(**base, w_tw=0, w_dur=1)).cost(sol)
    assert int(t_tw[1]) == case["TW"]
    assert int(t_dur[3]) == case["D"]


@pytest.mark.parametrize("case", GOLDEN["depot_moves"], ids=lambda c: c["cite"][:20])
def test_depot_operator_worked_example(case):
    inst = _instance(case)
    ref = Ref(inst)
    sol = _routes(case)
    assert ref.cost(sol)[0] == case["F"]
    moves = ref.eval(sol, (1 << 4) | (1 << 5))
    got = {}
    for m in moves:
        i = int(m["id"])
        got[(KIND_NAMES[i >> 56], (i >> 48) & 0xFF, (i >> 24) & 0xFFFFFF, i & 0xFFFFFF)] = m
    want = {(w["kind"], w["variant"], w["a"], w["b"]): w for w in case["moves"]}
    assert set(got) == set(want), (sorted(got), sorted(want))
    for key, w in want.items():
        m = got[key]
        assert (int(m["dF"]), int(m["dD"]), int(m["dV4"])) == (w["dF"], w["dD"], w["dV4"]), key


def _ff_instance(case):
    n = len(case["q"])
    return Instance(n_depots=case["n_depots"], n_customers=n - case["n_depots"],
                    c=np.asarray(case["c"], np.int32), t=np.asarray(case["t"], np.int32),
                    q=np.asarray(case["q"], np.int32), s=np.asarray(case["s"], np.int32),
                    e=np.asarray(case["e"], np.int32), l=np.asarray(case["l"], np.int32), Q=case["Q"], NV=4,
                    Dmax=case["Dmax"], open_routes=0, has_tw=1, theta=case["theta"], w_tw=1, w_load=1, w_dur=1,
                    w_depot=-1)


def _bf16_value(iv, rcp):
    """bf16 (nearest even) of fp32(iv) * fp32 rcp, as a float: the filter's scaling rule."""
    import struct
    x = np.float32(np.float32(iv) * np.float32(rcp))
    u = struct.unpack("<I", struct.pack("<f", float(x)))[0]
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return struct.unpack("<f", struct.pack("<I", u << 16))[0]


@pytest.mark.parametrize("case", GOLDEN["filter_features"], ids=lambda c: c["cite"][:20])
def test_filter_features_time_windows_worked_example(case):
    """Time-window features (13..22) of hand-computed anchors, with travel times t != c,
    service times and a duration limit; also the route facts and lists they rest on."""
    import struct
    inst = _ff_instance(case)
    ref = Ref(inst)
    st = ref.stats()
    assert (st["gamma_num"], st["gamma_den"]) == tuple(case["gamma"])
    nbr, ln = ref.neighbours()
    th = inst.theta
    for i, want in enumerate(case["lists"]):
        assert list(nbr[i * th:i * th + ln[i]]) == want, i
    sol = _routes(case)
    for rf in case["route_facts"]:
        a, xs, b = case["routes"][rf["route"]]
        dist, load, dur, tw = ref.route_terms(a, xs, b)
        assert (tw, dur) == (rf["tw"], rf["dur"]), rf["note"]
    fx = ref.features(sol)
    sc = case["scales"]
    rcp = [np.float32(1) / np.float32(sc["dist"]), np.float32(1) / np.float32(sc["load"]),
           np.float32(1) / np.float32(sc["time"]), np.float32(1) / np.float32(sc["depots"])]
    routes = case["routes"]
    for an in case["anchors"]:
        u, k, ints = an["u"], an["k"], an["ints"]
        row = fx[(u - inst.n_depots) * th + k]
        got = [struct.unpack("<f", struct.pack("<I", int(b) << 16))[0] for b in row]
        LA = next(len(xs) for _, xs, _ in routes if u in xs)
        LB = next(len(xs) for _, xs, _ in routes if an["v"] in xs)
        scale = [rcp[0]] * 9 + [rcp[1]] * 4 + [rcp[2]] * 10 + [1, 1, rcp[3], rcp[3], 1 / 32, 1 / 32,
                                                                 np.float32(1) / np.float32(LA),
                                                                 np.float32(1) / np.float32(LB),
                                                                 np.float32(1) / np.float32(th)]
        for f in range(32):
            assert got[f] == _bf16_value(ints[f], scale[f]), (u, f, got[f], ints[f])
    # customer 3 has no list: its rows are zero, as is the missing second entry of 1 and 2
    for i in range(inst.n_customers):
        for kk in range(ln[i], th):
            assert not fx[i * th + kk].any()


@pytest.mark.parametrize("case", GOLDEN["penalty_adapt"], ids=lambda c: c["note"][:30])
def test_dynamic_penalty_worked_example(case):
    """Dynamic penalty coefficients (Section 3.2.1, kappa = 0.5 of Table 1): final weights and
    objective of a local search whose one accepted step is computed by hand."""
    c = np.asarray(case["c"], np.int32)
    n = len(c)
    z = np.zeros(n, np.int32)
    inst = Instance(n_depots=case["n_depots"], n_customers=n - case["n_depots"], c=c, t=c,
                    q=np.asarray(case["q"], np.int32), s=z, e=z, l=np.full(n, gen.BIG_HORIZON, np.int32),
                    Q=case["Q"], NV=case["NV"], Dmax=-1, open_routes=0, has_tw=0, theta=n - 2,
                    **case["weights"])
    sol = _routes(case)
    for seed in range(4):  # the family order does not matter here
        out, st = Ref(inst).local_search([sol], seed=seed, max_passes=50, adapt=(case["w_min"], case["w_max"]))
        assert st[0]["w_final"] == case["w_final"]
        assert st[0]["F"] == case["F"]
        assert len(out[0].routes) == 1 and sorted(out[0].routes[0][1]) == [1, 2]
        _, terms = Ref(inst).cost(out[0])
        assert int(terms[0]) == case["D"]
