"""Parity with the oracle at the full sizes of the large workloads and on inputs
that earlier tests did not reach (exact integers throughout):

* the 20 + 10 000 time-window instance (400 MB matrix, horizon 100 000): the
  dense move table of every family, then a pass of family steps;
* the 20 + 10 000 open-route instance: a pass of family steps;
* searches of up to ten passes on instances above 4 096 nodes, where the
  selection keeps its per-resource minima in global memory instead of LDS;
* separate, asymmetric c and t (Gamma != 1) with 64 and 65 depots and with the
  locality layout of the matrices; separate symmetric t without time windows (the
  kernels that read t, beside the t-free ones);
* routes beyond the int32-safe length are refused at load time.
"""
import numpy as np
import pytest

from oracle import ALL_FAMILIES, Ref
from paper_2605_05208_amd import gen, mdvrp
from paper_2605_05208_amd.gen import canonical
from test_gpu_parity import _ls_compare, _step_compare, compare_dense, dense_cap_for, log, make_batch

pytestmark = pytest.mark.gpu

TW_FAMS = [1, 2, 4, 16, 32]
ALL_PLAIN = [1, 2, 4, 8, 16, 32]


def test_config5_dense_table():
    inst = gen.config5()
    sol = gen.start_solution(inst, inst.seed * 1000)
    log("config5 dense")
    dev, B, flat = make_batch([inst], [[sol]])
    got = B.eval_neighbourhood(ALL_FAMILIES, dense_cap=dense_cap_for([inst]))
    compare_dense(got, Ref(inst).eval(sol, ALL_FAMILIES), inst.n_customers, "config5")


def test_config5_first_pass_of_steps():
    inst = gen.config5()
    sols = [gen.start_solution(inst, inst.seed * 1000 + k) for k in range(2)]
    log("config5 steps")
    dev, B, flat = make_batch([inst], [sols])
    ref = Ref(inst)
    cur = flat
    for fam in TW_FAMS:
        cur = _step_compare(B, [ref, ref], cur, fam, 0, f"config5 fam {fam}")


def test_config3_open_first_pass_of_steps():
    inst = gen.config3(open_routes=1)
    sols = [gen.start_solution(inst, inst.seed * 1000 + k) for k in range(2)]
    log("config3 open steps")
    dev, B, flat = make_batch([inst], [sols])
    ref = Ref(inst)
    cur = flat
    for fam in ALL_PLAIN:
        cur = _step_compare(B, [ref, ref], cur, fam, 0, f"config3 open fam {fam}")


def test_search_above_4096_nodes_uneven_instance():
    """Instance 182 of the uneven batch (4 970 customers, 12 depots): ten passes of the
    search (Algorithm 2) on two solutions, trajectories and solutions exact."""
    inst = gen.config4_instance(182)
    assert inst.N > 4096
    sols = [gen.start_solution(inst, inst.seed * 1000 + k) for k in range(2)]
    log("ls uneven-182 10 passes")
    _ls_compare([inst], [sols], 0, 21, max_passes=10, tag="uneven-182")


def test_search_above_4096_nodes_config5():
    inst = gen.config5()
    sols = [gen.start_solution(inst, inst.seed * 1000 + 3)]
    log("ls config5 6 passes")
    _ls_compare([inst], [sols], 0, 5, max_passes=6, tag="config5")


def _tw_medium(seed, nd, nc):
    return gen._tw_instance(np.random.default_rng(seed), nd, nc, 1000, 50.0, 4, 30, 200, 90, 10_000, 20,
                            f"mdvrptw-{nd}x{nc}", seed)


def _make_batch_layout(insts, sols_per_inst, layout):
    dev = [mdvrp.Instance(i, layout=layout) for i in insts]
    unit_inst = [k for k, s in enumerate(sols_per_inst) for _ in s]
    B = mdvrp.Batch(dev, unit_inst)
    flat = [s for ss in sols_per_inst for s in ss]
    B.load(flat)
    return dev, B, flat


@pytest.mark.parametrize("layout", [mdvrp.LAYOUT_GIVEN, mdvrp.LAYOUT_ORDERED])
@pytest.mark.parametrize("open_r", [0, 1])
def test_separate_asymmetric_times(layout, open_r):
    """c asymmetric and t a separate asymmetric matrix (Gamma != 1): granular lists, the
    dense move tables, and whole searches; instances with 64 depots (depot-arc table), 65
    depots (matrix reads) and 8 depots."""
    insts = []
    for j, nd in enumerate((64, 65)):
        base = gen.tiny(91_000 + 10 * nd + open_r, has_tw=1, open_routes=open_r, nd=nd, nc=9)
        insts.append(gen.with_separate_times(base, 5 + j))
    med = _tw_medium(93_000 + open_r, 8, 300)
    med.open_routes = open_r
    insts.append(gen.with_separate_times(med, 9))
    sols = [[gen.random_solution(i, 3), gen.start_solution(i, 4)] for i in insts]
    log("separate times", layout, open_r)
    dev, B, flat = _make_batch_layout(insts, sols, layout)
    for d, inst in zip(dev, insts):
        ref = Ref(inst)
        nbr, ln = d.lists()
        rn, rl = ref.neighbours()
        assert np.array_equal(ln, rl) and np.array_equal(nbr, rn)
        info, st = d.info(), ref.stats()
        assert (info["gamma_num"], info["gamma_den"]) == (st["gamma_num"], st["gamma_den"])
        assert st["gamma_num"] != st["gamma_den"]
    for fam in [ALL_FAMILIES] + TW_FAMS:
        got = B.eval_neighbourhood(fam, dense_cap=dense_cap_for([insts[k] for k in B.unit_inst]))
        u = 0
        for k, inst in enumerate(insts):
            ref = Ref(inst)
            for sol in sols[k]:
                compare_dense(got[got["unit"] == u], ref.eval(sol, fam), inst.n_customers, f"inst {k} unit {u}")
                u += 1
    # whole searches, same layout
    dev, B, flat = _make_batch_layout(insts, sols, layout)
    st = B.local_search_to_optimum(seed=23)
    got = B.export()
    u = 0
    for k, inst in enumerate(insts):
        out, rst = Ref(inst).local_search(sols[k], seed=23)
        for j in range(len(sols[k])):
            assert canonical(got[u].routes) == canonical(out[j].routes), (k, j)
            for key in ("F", "passes", "steps", "moves_applied", "evaluated"):
                assert st[u][key] == rst[j][key], (k, j, key)
            u += 1


def _with_symmetric_times(inst, seed, dmax_frac):
    """A copy of an instance without time windows whose travel times are a separate,
    symmetric matrix t = c + a symmetric per-arc offset, with a duration limit that
    binds (so that t enters F through the duration excess)."""
    rng = np.random.default_rng(seed)
    n = inst.N
    off = rng.integers(0, 40, (n, n))
    off = np.triu(off, 1)
    off = off + off.T
    out = gen.Instance(**{**inst.__dict__})
    out.t = np.ascontiguousarray(inst.c.astype(np.int64) + off, np.int32)
    out.Dmax = int(dmax_frac * np.sort(out.t[:inst.n_depots].ravel())[-1])
    out.w_dur = 5
    out.name = inst.name + "-t"
    return out


@pytest.mark.parametrize("layout", [mdvrp.LAYOUT_GIVEN, mdvrp.LAYOUT_ORDERED])
def test_separate_symmetric_times_without_windows(layout):
    """Without time windows the batches whose travel times are their costs take kernels
    that never read t; an instance with a separate t matrix (symmetric, as required, and
    a binding duration limit) takes the kernels that do, alone and in a batch beside an
    instance with t = c: dense move tables and whole searches against the oracle."""
    a = _with_symmetric_times(gen.config1(), 7, 3.0)
    b = _with_symmetric_times(gen.tiny(97_000, has_tw=0, nd=3, nc=12), 8, 2.0)
    c = gen.config1(111)
    for insts in ([a], [a, b, c]):
        sols = [[gen.random_solution(i, 3), gen.start_solution(i, 4)] for i in insts]
        log("separate symmetric times", layout, len(insts))
        dev, B, flat = _make_batch_layout(insts, sols, layout)
        for fam in [ALL_FAMILIES] + ALL_PLAIN:
            got = B.eval_neighbourhood(fam, dense_cap=dense_cap_for([insts[k] for k in B.unit_inst]))
            u = 0
            for k, inst in enumerate(insts):
                ref = Ref(inst)
                for sol in sols[k]:
                    compare_dense(got[got["unit"] == u], ref.eval(sol, fam), inst.n_customers, f"inst {k} unit {u}")
                    u += 1
        dev, B, flat = _make_batch_layout(insts, sols, layout)
        st = B.local_search_to_optimum(seed=29)
        got = B.export()
        u = 0
        for k, inst in enumerate(insts):
            out, rst = Ref(inst).local_search(sols[k], seed=29)
            for j in range(len(sols[k])):
                assert canonical(got[u].routes) == canonical(out[j].routes), (k, j)
                for key in ("F", "passes", "steps", "moves_applied", "evaluated"):
                    assert st[u][key] == rst[j][key], (k, j, key)
                u += 1


def test_route_beyond_the_int32_safe_length_is_refused():
    """A depot window of 1.5e8 leaves room for 5 customers per route in int32 segment sums:
    a 6-customer route is refused with ERANGE before any launch; 5 are accepted."""
    inst = gen.tiny(95_001, has_tw=1, nd=1, nc=8)
    inst.l = inst.l.copy()
    inst.l[0] = 150_000_000
    d = mdvrp.Instance(inst)
    guard = d.info()["len_guard"]
    assert guard == 5
    B = mdvrp.Batch([d], [0])
    cust = list(range(1, 9))
    with pytest.raises(mdvrp.MdvrpError) as ei:
        B.load([gen.Solution([(0, cust[:6], 0), (0, cust[6:], 0)])])
    assert ei.value.status == mdvrp.ERANGE
    B.load([gen.Solution([(0, cust[:5], 0), (0, cust[5:], 0)])])
    F, _ = B.cost()
    assert int(F[0]) == Ref(inst).cost(gen.Solution([(0, cust[:5], 0), (0, cust[5:], 0)]))[0]
