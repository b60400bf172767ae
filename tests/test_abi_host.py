"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, and its host-side validation rejects bad input with EINVAL."""
import os
import re

import numpy as np
import pytest

from paper_2605_05208_amd import gen, mdvrp
from paper_2605_05208_amd.gen import Solution

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            names |= set(re.findall(r"\b(mdvrp_[a-z0-9_]+)\s*\(", txt))
    return names


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(mdvrp.LIB_PATH):
        from paper_2605_05208_amd import build
        build.build()
    return mdvrp.lib()


def test_every_declared_symbol_is_exported(L):
    declared = _declared()
    assert declared, "no declarations found"
    for name in sorted(declared):
        assert hasattr(L, name), name
    assert set(mdvrp.EXPORTED) == declared


def test_status_strings(L):
    for s in (0, -1, -2, -3, -4, -5):
        assert L.mdvrp_status_string(s)


def test_family_order_matches_oracle(L):
    from oracle import family_order as ref_order
    for p in range(40):
        for tw in (0, 1):
            assert mdvrp.family_order(tw, 987654321, p) == ref_order(tw, 987654321, p)


def test_validate_instance_host(L):
    I = gen.tiny(5)
    assert mdvrp.validate_instance_host(I) == 0
    bad = [dict(Q=0), dict(NV=-1), dict(theta=0), dict(theta=200), dict(w_load=-1), dict(n_depots=0),
           dict(has_tw=2), dict(open_routes=5)]
    for b in bad:
        J = gen.Instance(**{**I.__dict__, **b})
        assert mdvrp.validate_instance_host(J) == mdvrp.EINVAL, b
    e = I.e.copy(); l = I.l.copy()
    e[I.n_depots] = 10; l[I.n_depots] = 5
    assert mdvrp.validate_instance_host(gen.Instance(**{**I.__dict__, "e": e, "l": l})) == mdvrp.EINVAL
    q = I.q.copy(); q[0] = 3
    assert mdvrp.validate_instance_host(gen.Instance(**{**I.__dict__, "q": q})) == mdvrp.EINVAL
    q = I.q.copy(); q[-1] = -1
    assert mdvrp.validate_instance_host(gen.Instance(**{**I.__dict__, "q": q})) == mdvrp.EINVAL
    # route loads and load deltas are int32: the total demand must stay below 2^30
    q = I.q.copy(); q[I.n_depots:] = (1 << 30) // (len(q) - I.n_depots) + 1
    assert mdvrp.validate_instance_host(gen.Instance(**{**I.__dict__, "q": q})) == mdvrp.ERANGE


def test_validate_solutions_host(L):
    I = gen.tiny(6, nd=2, nc=6)
    good = gen.start_solution(I, 1)
    assert mdvrp.validate_solutions_host([I], [0], [good]) == 0
    assert mdvrp.validate_solutions_host([I, I], [0, 1], [good, good]) == 0
    r = good.routes
    cases = {
        "missing customer": Solution([(r[0][0], r[0][1][1:], r[0][2])] + r[1:]) if len(r[0][1]) > 1 else None,
        "duplicate": Solution(r + [(0, [r[0][1][0]], 0)]),
        "empty route": Solution(r + [(0, [], 0)]),
        "start not a depot": Solution([(I.n_depots, r[0][1], r[0][2])] + r[1:]),
        "end not a depot": Solution([(r[0][0], r[0][1], I.N + 3)] + r[1:]),
        "depot as customer": Solution([(r[0][0], r[0][1] + [0], r[0][2])] + r[1:]),
    }
    for name, sol in cases.items():
        if sol is None:
            continue
        assert mdvrp.validate_solutions_host([I], [0], [sol]) == mdvrp.EINVAL, name
    assert "unit 0" in L.mdvrp_last_error().decode()
    # an open instance ignores the end depots
    Io = gen.Instance(**{**I.__dict__, "open_routes": 1})
    assert mdvrp.validate_solutions_host([Io], [0], [cases["end not a depot"]]) == 0
    # bad instance index
    assert mdvrp.validate_solutions_host([I], [1], [good]) == mdvrp.EINVAL


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    monkeypatch.setattr(mdvrp, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(mdvrp, "_lib", None)
    with pytest.raises(RuntimeError):
        mdvrp.lib()


def test_header_has_no_torch_types():
    txt = open(os.path.join(ROOT, "include", "mdvrp.h")).read()
    assert "torch" not in txt.lower() and "at::" not in txt
    assert np is not None
