"""Pins of the oracle's crossover pieces (Section 3.3, Algorithm 3 and Eq. 4):
hand-computed route-pair counts and scores, the score and diversity arithmetic
of the paper's worked example (Appendix, Fig. A.1), the counts against an
independent set-based computation, and the discounted UCB1 rule worked by hand
with its logarithm and square root against the math library. No GPU."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2605_05208_amd import gen

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_cases.json")))
D = GOLDEN["dcrex"]


@pytest.mark.parametrize("case", D["cases"], ids=lambda c: str(c["intro"]))
def test_counts_worked_example(case):
    ei, nr, nm, nc = oracle.dcrex_counts([tuple(r) for r in D["offspring"]], case["intro"],
                                         [tuple(r) for r in D["parent"]])
    assert ei.tolist() == case["EI"] and nr.tolist() == case["NR"]
    assert nm.tolist() == case["NM"] and nc.tolist() == case["NC"]
    assert oracle.dcrex_score(ei, nr, nm, nc).tolist() == case["score"]
    assert oracle.dcrex_dsigma(ei, nr, nm).tolist() == case["dsigma"]


@pytest.mark.parametrize("ex", D["example"], ids=lambda e: str(e["score"]))
def test_paper_worked_example_arithmetic(ex):
    assert oracle.dcrex_score(ex["EI"], ex["NR"], ex["NM"], ex["NC"]) == ex["score"]
    assert oracle.dcrex_dsigma(ex["EI"], ex["NR"], ex["NM"]) == ex["dsigma"]


def _arcs(route):
    a, xs, b = route
    path = [a] + list(xs) + ([b] if b >= 0 else [])
    return set(zip(path[:-1], path[1:]))


@pytest.mark.parametrize("open_r", [0, 1])
def test_counts_against_sets(open_r):
    """Offspring built from two solutions' routes, so that customers repeat."""
    rng = np.random.default_rng(7 + open_r)
    for t in range(6):
        inst = gen.tiny(8100 + 10 * open_r + t, open_routes=open_r, nc=12)
        s1, s2, p = (gen.random_solution(inst, 3 * t + k) for k in range(3))
        off = list(s1.routes) + [s2.routes[k] for k in rng.choice(len(s2.routes), size=min(2, len(s2.routes)),
                                                                  replace=False)]
        intro = [0] * len(s1.routes) + [1] * (len(off) - len(s1.routes))
        ei, nr, nm, nc = oracle.dcrex_counts(off, intro, list(p.routes))
        for i, Ri in enumerate(off):
            others = [off[r] for r in range(len(off)) if r != i]
            held = set(x for r in others for x in r[1])
            held_intro = set(x for r in range(len(off)) if r != i and intro[r] for x in off[r][1])
            arcs_other = set().union(*[_arcs(r) for r in others]) if others else set()
            for j, Rj in enumerate(p.routes):
                assert ei[i, j] == len(_arcs(Rj) - arcs_other)
                assert nm[i, j] == len(set(Rj[1]) & held)
                assert nc[i, j] == len(set(Rj[1]) & held_intro)
                assert nr[i, j] == len(set(Ri[1]) - set(Rj[1]) - held)


def test_ucb_worked_example():
    u = D["ucb"]
    R = np.zeros(4)
    N = np.zeros(4)
    for arm, reward in u["plays"]:
        oracle.ucb_update(R, N, arm, reward, u["gamma"])
    assert np.allclose(N[:3], u["N"], rtol=0, atol=1e-12) and N[3] == 0
    assert np.allclose(R[:3], u["R"], rtol=0, atol=1e-12) and R[3] == 0
    assert oracle.ucb_select(R, N) == 3  # never played
    assert oracle.ucb_select(R[:3], N[:3]) == u["next_of_three"]


def test_ucb_prefers_the_arm_of_higher_mean_once_counts_are_large():
    R = np.zeros(3)
    N = np.zeros(3)
    for k in range(600):
        arm = oracle.ucb_select(R, N)
        oracle.ucb_update(R, N, arm, [0.1, 1.0, 0.3][arm], 0.99)
    # the best arm holds most of the discounted count (sum of counts tends to 1/(1-gamma))
    assert N[1] > N[0] and N[1] > N[2]
    assert abs(N.sum() - (1 - 0.99 ** 600) / 0.01) < 1e-9


def test_ln_and_sqrt_against_the_math_library():
    for x in [1.0, 1.0000001, 1.5, 2.0, 3.99, 10.0, 99.3, 1e6, 123456.789, 2.0 ** 40 + 3]:
        assert abs(oracle.ucb_ln(x) - math.log(x)) <= 4e-16 * max(1.0, math.log(x))
    for x in [1e-9, 0.25, 0.5, 1.0, 2.0, 3.0, 1e6, 7.777e15]:
        assert abs(oracle.ucb_sqrt(x) - math.sqrt(x)) <= 2.3e-16 * math.sqrt(x)
    assert oracle.ucb_sqrt(0.0) == 0.0
