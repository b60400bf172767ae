"""Parity of the learned move filter's HIP path with the CPU oracle.

Features and labels are integers or bit patterns: compared exactly. The
network runs bf16 x bf16 -> fp32 on the matrix cores against the oracle's
fp64 arithmetic on the same bf16-rounded operands: logits within 1e-2,
gradients within 2e-2 relative Frobenius error per tensor. Candidate lists
are compared exactly against the oracle's top-k of the GPU's own logits, and
the filtered evaluation and the filtered local search against the oracle run
over the same lists.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import ALL_FAMILIES, Ref
from paper_2605_05208_amd import gen, mdvrp
from paper_2605_05208_amd.gen import canonical

pytestmark = pytest.mark.gpu

H, F = 256, 32
P_W1, P_B1 = 0, H * F
P_W2 = P_B1 + H
P_B2 = P_W2 + H * H
P_W3 = P_B2 + H
P_B3 = P_W3 + H
TENSORS = {"W1": (P_W1, P_B1), "b1": (P_B1, P_W2), "W2": (P_W2, P_B2), "b2": (P_B2, P_W3), "w3": (P_W3, P_B3),
           "b3": (P_B3, P_B3 + 1)}
PAIR_KINDS = 8  # kinds 0..7 are anchored on (u, v)


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def torch():
    import torch as t
    return t


def he_params(seed, out_scale=0.2):
    """He-initialised hidden layers with small random biases; the output layer is
    scaled so that logits on real features stay within about +-10, the range of a
    trained filter's logits, where the 1e-2 logit tolerance applies."""
    rng = np.random.default_rng(seed)
    P = np.zeros(oracle.N_PARAMS, np.float32)
    P[P_W1:P_B1] = rng.standard_normal(H * F) * np.sqrt(2.0 / F)
    P[P_B1:P_W2] = rng.standard_normal(H) * 0.1
    P[P_W2:P_B2] = rng.standard_normal(H * H) * np.sqrt(2.0 / H)
    P[P_B2:P_W3] = rng.standard_normal(H) * 0.1
    P[P_W3:P_B3] = rng.standard_normal(H) * np.sqrt(1.0 / H) * out_scale
    P[P_B3] = 0.05
    return P


def make_batch(insts, sols_per_inst):
    dev = [mdvrp.Instance(i) for i in insts]
    unit_inst = [k for k, s in enumerate(sols_per_inst) for _ in s]
    B = mdvrp.Batch(dev, unit_inst)
    flat = [s for ss in sols_per_inst for s in ss]
    B.load(flat)
    return dev, B, flat


def unit_slices(insts, unit_inst):
    out, at = [], 0
    for k in unit_inst:
        n = insts[k].n_customers * insts[k].theta
        out.append(slice(at, at + n))
        at += n
    return out


def _tiny(tw, o):
    # a batch mixes instances of one kind: several sizes, theta = 3 and full lists, a duration limit
    return [gen.tiny(70_000 + 100 * tw + 10 * o + k, has_tw=tw, open_routes=o, theta=(3 if k % 2 else None),
                     Dmax=(40 if (k == 1 and not tw) else -1)) for k in range(4)]


def _feature_cases():
    return {"tiny": _tiny(0, 0), "tiny_open": _tiny(0, 1), "tiny_tw": _tiny(1, 0), "tiny_tw_open": _tiny(1, 1),
            "config1": [gen.config1()], "config2": [gen.config2()], "config3_open": [gen.config3(open_routes=1)]}


TINY = ["tiny", "tiny_open", "tiny_tw", "tiny_tw_open"]


# ----------------------------------------------------------------------------- features

@pytest.mark.parametrize("which", TINY + ["config1", "config2", "config3_open"])
def test_features_bit_exact(which):
    insts = _feature_cases()[which]
    log("features", which)
    groups = []
    for I in insts:
        n = 2 if I.n_customers < 2000 else 1
        groups.append([gen.start_solution(I, I.seed * 1000 + k) for k in range(n)])
    dev, B, flat = make_batch(insts, groups)
    unit_inst = [k for k, s in enumerate(groups) for _ in s]
    sl = unit_slices(insts, unit_inst)
    for phase in range(2):
        got = B.features()
        sols = B.export()
        for u, k in enumerate(unit_inst):
            exp = Ref(insts[k]).features(sols[u])
            g = got[sl[u]]
            bad = np.nonzero((g != exp).any(1))[0]
            assert len(bad) == 0, (f"{which} unit {u} phase {phase}: anchor {bad[0]}: "
                                   f"{g[bad[0]].tolist()} vs {exp[bad[0]].tolist()}")
        # a second state: after two passes of the local search
        B.local_search_to_optimum(seed=3, max_passes=2)


# ----------------------------------------------------------------------------- network

def test_forward_matches_oracle_on_features_and_random_inputs():
    t = torch()
    P = he_params(1)
    M = mdvrp.Mlp(P)
    insts = [gen.config1()]
    dev, B, flat = make_batch(insts, [[gen.start_solution(insts[0], 101_000)]])
    xf = B.features()
    rng = np.random.default_rng(2)
    xr = oracle.bf16(rng.standard_normal(3001 * F)).reshape(3001, F)
    for name, x in (("features", xf), ("random", xr)):
        log("forward", name, x.shape)
        xd = t.from_numpy(x.view(np.int16)).to("cuda")
        z = M.forward(xd).cpu().numpy()
        ref = oracle.mlp_forward(P, x, round_act=1)
        err = np.abs(z - ref).max()
        log(f"  |logit| <= {np.abs(ref).max():.2f}, max |dlogit| {err:.2e}")
        assert err <= 1e-2
    # n not a multiple of the tile, and n = 1
    for n in (1, 17, 33):
        xd = t.from_numpy(xr[:n].view(np.int16)).to("cuda")
        z = M.forward(xd).cpu().numpy()
        assert np.abs(z - oracle.mlp_forward(P, xr[:n], round_act=1)).max() <= 1e-2


def _rel_fro(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("n", [37, 2500])
def test_backward_matches_oracle(n):
    t = torch()
    P = he_params(3)
    M = mdvrp.Mlp(P)
    rng = np.random.default_rng(4 + n)
    x = oracle.bf16(rng.standard_normal(n * F)).reshape(n, F)
    y = (rng.random(n) < 0.3).astype(np.float32)
    xd = t.from_numpy(x.view(np.int16)).to("cuda")
    z = M.forward(xd, keep=True)
    yd = t.from_numpy(y).to("cuda")
    dz, loss = M.bce(z, yd)
    g = M.backward(xd, dz).cpu().numpy().astype(np.float64)
    zh = z.cpu().numpy()
    dzh = dz.cpu().numpy().astype(np.float64)
    # loss and its gradient against the oracle and the closed form of the BCE derivative
    assert abs(float(loss.cpu().numpy()[0]) - oracle.bce(zh, y)) <= 1e-5 * max(1.0, oracle.bce(zh, y))
    assert np.allclose(dzh, (1 / (1 + np.exp(-zh.astype(np.float64))) - y) / n, rtol=1e-5, atol=1e-9)
    ref = oracle.mlp_backward(P, x, dzh, round_act=1)
    for name, (a, b) in TENSORS.items():
        e = _rel_fro(g[a:b], ref[a:b])
        log(f"  grad {name}: rel Frobenius {e:.2e}")
        assert e <= 2e-2, name


def test_adam_matches_oracle():
    t = torch()
    P = he_params(5)
    M = mdvrp.Mlp(P)
    rng = np.random.default_rng(6)
    Pr = P.copy()
    m = np.zeros_like(P)
    v = np.zeros_like(P)
    for step in range(1, 4):
        g = (rng.standard_normal(P.size) * 10.0 ** rng.integers(-4, 1, P.size)).astype(np.float32)
        M.adam(t.from_numpy(g).to("cuda"), 1e-3, step)
        oracle.adam(Pr, m, v, g, 1e-3, step)
    got = M.get_params()
    assert np.allclose(got, Pr, rtol=1e-5, atol=1e-7)


def test_train_step_is_forward_bce_backward_adam_and_learns():
    """The fused step equals the separate calls, and the loss falls on a learnable labelling."""
    t = torch()
    P = he_params(7)
    n = 4096
    rng = np.random.default_rng(8)
    xf = rng.standard_normal((n, F)).astype(np.float32)
    x = oracle.bf16(xf.ravel()).reshape(n, F)
    y = (xf[:, 0] + 0.5 * xf[:, 3] > 0.2).astype(np.float32)
    w = np.where(y > 0, 2.0, 1.0).astype(np.float32)
    xd, yd, wd = (t.from_numpy(a).to("cuda") for a in (x.view(np.int16), y, w))
    A = mdvrp.Mlp(P)
    Bn = mdvrp.Mlp(P)
    z1, loss1, g1 = A.train_step(xd, yd, wd, 1e-3, 1)
    z2 = Bn.forward(xd, keep=True)
    dz, loss2 = Bn.bce(z2, yd, wd)
    g2 = Bn.backward(xd, dz)
    Bn.adam(g2, 1e-3, 1)
    t.cuda.synchronize()
    # the same kernels in the same fixed reduction order: bit-identical results
    assert t.equal(z1, z2)
    assert t.equal(loss1, loss2)
    assert t.equal(g1, g2)
    assert np.array_equal(A.get_params(), Bn.get_params())
    first = float(loss1.cpu().numpy()[0])
    last = first
    for step in range(2, 150):
        _, loss, _ = A.train_step(xd, yd, wd, 3e-3, step)
        last = float(loss.cpu().numpy()[0])
    log("  loss", first, "->", last)
    assert last < 0.5 * first


def test_training_is_deterministic():
    """Loss, gradients and trained weights are bit-identical across runs: every reduction
    over samples (loss, biases, weight-gradient chunks) is summed in a fixed order."""
    t = torch()
    P = he_params(11)
    n = 5000  # five weight-gradient chunks, several samples per output-layer block
    rng = np.random.default_rng(12)
    x = oracle.bf16(rng.standard_normal(n * F)).reshape(n, F)
    y = (rng.random(n) < 0.25).astype(np.float32)
    w = np.where(y > 0, 3.0, 1.0).astype(np.float32)
    xd, yd, wd = (t.from_numpy(a).to("cuda") for a in (x.view(np.int16), y, w))
    runs = []
    for _ in range(3):
        M = mdvrp.Mlp(P)
        out = []
        for step in range(1, 6):
            z, loss, g = M.train_step(xd, yd, wd, 2e-3, step)
            out.append((loss.cpu().numpy().copy(), g.cpu().numpy().copy()))
        runs.append((out, M.get_params()))
    for out, params in runs[1:]:
        assert np.array_equal(params, runs[0][1])
        for (l0, g0), (l1, g1) in zip(runs[0][0], out):
            assert np.array_equal(l0, l1) and np.array_equal(g0, g1)


# ----------------------------------------------------------------------------- scoring, top-k, labels

@pytest.mark.parametrize("which", TINY + ["config2"])
def test_score_topk(which):
    insts = _feature_cases()[which]
    groups = [[gen.start_solution(I, I.seed * 1000 + k) for k in range(2)] for I in insts]
    dev, B, flat = make_batch(insts, groups)
    unit_inst = [k for k, s in enumerate(groups) for _ in s]
    sl = unit_slices(insts, unit_inst)
    kc = min(8, min(I.theta for I in insts))
    B.filter_attach(kc)
    P = he_params(9)
    M = mdvrp.Mlp(P)
    lg = B.score_topk(M)
    cand = B.filter_lists()
    feats = B.features()
    for u, k in enumerate(unit_inst):
        I = insts[k]
        ref = Ref(I)
        nbr, ln = ref.neighbours()
        valid = (np.arange(I.theta)[None, :] < ln[:, None]).ravel()
        z = lg[sl[u]]
        zr = oracle.mlp_forward(P, feats[sl[u]], round_act=1)
        log(f"  unit {u}: |logit| <= {np.abs(zr[valid]).max():.2f}, max |dlogit| {np.abs(z[valid] - zr[valid]).max():.2e}")
        assert np.abs(z[valid] - zr[valid]).max() <= 1e-2, f"unit {u}"
        exp = oracle.topk(nbr, ln, I.n_customers, I.theta, np.where(valid, z, 0).astype(np.float32), kc)
        assert np.array_equal(cand[u], exp), f"unit {u}: top-{kc} lists"


@pytest.mark.parametrize("which", TINY + ["config1", "config2"])
def test_labels_match_oracle_dense_evaluation(which):
    insts = _feature_cases()[which]
    groups = [[gen.start_solution(I, I.seed * 1000 + 5)] for I in insts]
    dev, B, flat = make_batch(insts, groups)
    sl = unit_slices(insts, list(range(len(insts))))
    lab = B.labels()
    for u, I in enumerate(insts):
        ref = Ref(I)
        nbr, ln = ref.neighbours()
        moves = ref.eval(flat[u], ALL_FAMILIES)
        kind = (moves["id"] >> np.uint64(56)).astype(np.int64)
        a = ((moves["id"] >> np.uint64(24)) & np.uint64(0xFFFFFF)).astype(np.int64)
        b = (moves["id"] & np.uint64(0xFFFFFF)).astype(np.int64)
        exp = np.zeros(I.n_customers * I.theta, np.uint8)
        rows = nbr.reshape(I.n_customers, I.theta)
        for aa, bb in zip(a[(kind < PAIR_KINDS) & (moves["dF"] < 0)], b[(kind < PAIR_KINDS) & (moves["dF"] < 0)]):
            i = aa - I.n_depots
            r = int(np.nonzero(rows[i, :ln[i]] == bb)[0][0])
            exp[i * I.theta + r] = 1
        assert np.array_equal(lab[sl[u]], exp), f"{which} unit {u}: {int(lab[sl[u]].sum())} vs {int(exp.sum())}"


# ----------------------------------------------------------------------------- filtered evaluation and search

def _lists_for_oracle(c):
    ln = (c >= 0).sum(1).astype(np.int32)
    return c.ravel().astype(np.int32), ln, c.shape[1]


def _compare_dense(got, exp, tag):
    assert len(got) == len(exp), f"{tag}: {len(got)} vs {len(exp)} evaluated"
    g = got[np.argsort(got["id"], kind="stable")]
    e = exp[np.argsort(exp["id"], kind="stable")]
    assert np.array_equal(g["id"], e["id"]), tag
    for f in ("dF", "dD", "dTW", "dLX", "dDX", "dV4"):
        assert np.array_equal(g[f], e[f]), f"{tag}: {f}"


@pytest.mark.parametrize("which", TINY + ["config1", "config2"])
@pytest.mark.parametrize("lists", ["eta", "mlp"])
def test_filtered_dense_evaluation(which, lists):
    insts = _feature_cases()[which]
    groups = [[gen.start_solution(I, I.seed * 1000 + 7)] for I in insts]
    dev, B, flat = make_batch(insts, groups)
    kc = min(8, min(I.theta for I in insts))
    B.filter_attach(kc)
    if lists == "mlp":
        B.score_topk(mdvrp.Mlp(he_params(10)), want_logits=False)
    cand = B.filter_lists()
    cap = sum(I.n_customers * kc * 14 + 2 * I.n_customers * I.n_depots for I in insts) + 1024
    got = B.eval_neighbourhood(ALL_FAMILIES, dense_cap=cap, filtered=True)
    for u, I in enumerate(insts):
        exp = Ref(I).eval(flat[u], ALL_FAMILIES, lists=_lists_for_oracle(cand[u]))
        _compare_dense(got[got["unit"] == u], exp, f"{which}/{lists} unit {u}")


def ref_filtered_ls(I, sol, kc, seed, mode=0):
    """The filtered search of the library restated over the oracle's steps, with
    the first kc entries of every granular list as the filtered lists."""
    ref = Ref(I)
    nbr, ln = ref.neighbours()
    rows = nbr.reshape(I.n_customers, I.theta)
    c = np.where(np.arange(kc)[None, :] < np.minimum(ln, kc)[:, None], rows[:, :kc], -1)
    flists = _lists_for_oracle(c)
    fmode, p, steps, evaluated, fallbacks = 1, 0, 0, 0, 0
    while True:
        fams = oracle.family_order(I.has_tw, seed, p) if mode == 0 else None
        masks = [1 << f for f in fams] if mode == 0 else [ALL_FAMILIES]
        applied = False
        for m in masks:
            sol, sel, _, n_ev = ref.step(sol, m, lists=flists if fmode == 1 else None)
            steps += 1
            evaluated += n_ev
            applied = applied or len(sel) > 0
        p += 1
        if fmode == 1:
            if not applied:
                fmode, fallbacks = 2, fallbacks + 1
        elif applied:
            fmode = 1
        else:
            break
    return sol, dict(passes=p, steps=steps, evaluated=evaluated, fallback_passes=fallbacks, F=ref.cost(sol)[0])


@pytest.mark.parametrize("tw,open_r", [(0, 0), (0, 1), (1, 0), (1, 1)])
@pytest.mark.parametrize("mode", [0, 1])
def test_eta_filtered_local_search_matches_oracle(tw, open_r, mode):
    insts = [gen.tiny(71_000 + 10 * tw + open_r + k, has_tw=tw, open_routes=open_r, nc=40 + 5 * k)
             for k in range(4)]
    groups = [[gen.start_solution(I, I.seed * 1000 + j) for j in range(2)] for I in insts]
    dev, B, flat = make_batch(insts, groups)
    kc = 4
    B.filter_attach(kc)
    st = B.local_search_to_optimum(mode=mode, seed=11, filter=mdvrp.FILTER_LISTS)
    out = B.export()
    unit_inst = [k for k, s in enumerate(groups) for _ in s]
    for u, k in enumerate(unit_inst):
        sol, rs = ref_filtered_ls(insts[k], flat[u], kc, 11, mode)
        assert canonical(out[u].routes) == canonical(sol.routes), f"unit {u}"
        for key in ("passes", "steps", "evaluated", "fallback_passes", "F"):
            assert st[u][key] == rs[key], f"unit {u}: {key} {st[u][key]} vs {rs[key]}"
        assert st[u]["converged"] == 1


@pytest.mark.parametrize("which", TINY + ["config1", "config2"])
def test_mlp_filtered_local_search_reaches_a_full_local_optimum(which):
    insts = _feature_cases()[which]
    n = 2 if which != "config2" else 4
    groups = [[gen.start_solution(I, I.seed * 1000 + j) for j in range(n)] for I in insts]
    dev, B, flat = make_batch(insts, groups)
    kc = min(8, min(I.theta for I in insts))
    B.filter_attach(kc)
    M = mdvrp.Mlp(he_params(12))
    st = B.local_search_to_optimum(seed=5, filter=mdvrp.FILTER_MLP, mlp=M, poll_every=2)
    out = B.export()
    unit_inst = [k for k, s in enumerate(groups) for _ in s]
    for u, k in enumerate(unit_inst):
        ref = Ref(insts[k])
        assert st[u]["converged"] == 1 and st[u]["err"] == 0
        assert st[u]["fallback_passes"] >= 1
        assert ref.cost(out[u])[0] == st[u]["F"]
        moves = ref.eval(out[u], ALL_FAMILIES)
        assert len(moves) == 0 or moves["dF"].min() >= 0, f"unit {u}: improving move left"
    log("  filtered F", [s["F"] for s in st], "evaluated", [s["evaluated"] for s in st])


# ----------------------------------------------------------------------------- what the trained network gains

def test_trained_filter_gains_over_full_evaluation():
    """Train on logs of full-list searches of the 1000-customer instance (GPU kernels end
    to end), then search held-out uneven instances: the filtered search must reach a
    certified local optimum of the full neighbourhood, evaluate far fewer moves than the
    full search, and rank the improving anchors of mid-search states better than an
    untrained network does."""
    from paper_2605_05208_amd import filter_train as ft
    I2 = gen.config2()
    dev2, TB, flat2 = make_batch([I2], [[gen.start_solution(I2, I2.seed * 1000 + j) for j in range(8)]])
    x, y, w, snaps = ft.log_states(TB, flat2, chunk=2, max_chunks=30)
    trained = mdvrp.Mlp(ft.init_params(0))
    losses, _ = ft.train(trained, x, y, w, epochs=4, lr=1e-3)
    log(f"  {x.shape[0]} samples from {snaps} snapshots, loss {losses[0]:.3f} -> {losses[-1]:.3f}")
    assert losses[-1] < losses[0]
    untrained = mdvrp.Mlp(ft.init_params(0))
    insts = [gen.config4_instance(i) for i in (3, 11, 29)]
    groups = [[gen.start_solution(I, I.seed * 1000 + j) for j in range(2)] for I in insts]
    dev, B, flat = make_batch(insts, groups)
    B.filter_attach(8)
    full = B.local_search_to_optimum(seed=3)
    B.load(flat)
    filt = B.local_search_to_optimum(seed=3, filter=mdvrp.FILTER_MLP, mlp=trained, rescore=4)
    out = B.export()
    unit_inst = [k for k, s in enumerate(groups) for _ in s]
    for u, k in enumerate(unit_inst):
        ref = Ref(insts[k])
        moves = ref.eval(out[u], ALL_FAMILIES)
        assert len(moves) == 0 or moves["dF"].min() >= 0, f"unit {u}: improving move left"
        assert ref.cost(out[u])[0] == filt[u]["F"]
    ev_full = sum(s["evaluated"] for s in full)
    ev_filt = sum(s["evaluated"] for s in filt)
    F_full = np.mean([s["F"] for s in full])
    F_filt = np.mean([s["F"] for s in filt])
    log(f"  evaluated {ev_filt} vs {ev_full} full; mean F {F_filt:.0f} vs {F_full:.0f} full")
    assert ev_filt * 2 < ev_full
    # ranking quality at a mid-search state of the held-out instances
    B.load(flat)
    B.local_search_to_optimum(seed=3, max_passes=6)
    r_trained, n_pos = ft.recall_at_k(B, trained, 8)
    r_untrained, _ = ft.recall_at_k(B, untrained, 8)
    log(f"  recall@8 of the {n_pos} improving anchors: trained {r_trained:.3f}, untrained {r_untrained:.3f}")
    assert r_trained > r_untrained
