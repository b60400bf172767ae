#!/usr/bin/env python3
"""Benchmark: penalised move evaluations per second, time to local optimum, and
the learned filter against full evaluation.

One step = load the 16 seeded start solutions of the 20-depot / 10000-customer
MDVRP instance (400 MB distance matrix; inputs already resident in HBM) into the
segment state and run the multi-move local search of every solution to its
local optimum (evaluation of every operator family, leader-follower selection,
apply, repeat until a full pass applies nothing). The line reports whole-job
move evaluations per second, the time per step (time to the local optimum), the
roofline of the dominant kernel (HIP events on the library's stream; compulsory
bytes per launch) and the CPU oracle timed on a bounded sample of the same
workload at one thread and at all host cores.

Sub-objects: `open` (the same instance with open routes, MDOVRP), `small` (the
8-depot / 1000-customer MDVRPTW population of 64 solutions), `filter` (on the
20 x 10000 MDVRPTW instance with 16 solutions: the search over the full granular
lists against the searches over k-entry lists ranked by the trained network and
by the eta order, at k = 8 and at k = 4: GPU time, the gap of the local-optimum
cost per seed, and the cost terms of each optimum) and `batch` (256 uneven
instances in one batch).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PROFILE_EVERY = 8
HBM_PEAK_GBS = 8000.0


def workload(name):
    from paper_2605_05208_amd import gen
    if name == "config2":
        inst, n = gen.config2(), 64
    elif name == "config1":
        inst, n = gen.config1(), 1
    elif name == "config3":
        inst, n = gen.config3(), 16
    elif name == "config3_open":
        inst, n = gen.config3(open_routes=1), 16
    elif name == "config5":
        inst, n = gen.config5(), 16
    else:
        raise SystemExit(f"unknown workload {name}")
    sols = [gen.start_solution(inst, inst.seed * 1000 + k) for k in range(n)]
    return inst, sols


PAIR_KERNEL_SOURCES = ("eval.hip", "eval_common.h", "eval_inter.h", "eval_intra.h", "internal.h")
PAIR_PROFILES = {"config2": "k_eval_pairs_mdvrptw-8x1000_64sol.md", "config5": "k_eval_pairs_mdvrptw-20x10000_16sol.md",
                 "config3": "k_eval_pairs_mdvrp-20x10000_16sol.md"}


def measured_traffic(workload):
    """HBM bytes per pair-evaluation launch from the committed counter summary of the workload
    (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy), or None when there is none or the
    kernel sources changed since the counters were taken."""
    import hashlib
    if workload not in PAIR_PROFILES:
        return None
    try:
        text = open(os.path.join(ROOT, "profiles", PAIR_PROFILES[workload])).read()
    except OSError:
        return None
    h = hashlib.sha256()
    for f in PAIR_KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2605_05208_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    vals = dict(line.split(":", 1) for line in text.splitlines()
                if line.startswith(("traffic_bytes_per_launch:", "kernel-source-sha256:")))
    if vals.get("kernel-source-sha256", "").split()[:1] != [h.hexdigest()]:
        return None
    return int(vals["traffic_bytes_per_launch"])


def instance_bytes(inst):
    """Compulsory bytes of one pair-evaluation launch that the units of one instance
    share, read once per launch: granular lists (entries, lengths, and, for time-window
    instances in the locality layout, the {c, t} of the arc u -> v kept beside every
    slot) and node attributes. The matrix entries are
    counted the same way, once per instance: 4 bytes per distinct entry the launch
    reads (mdvrp_eval_footprint)."""
    nc, n, th = inst.n_customers, inst.N, inst.theta
    attrs = 16 if inst.has_tw else 8
    # read with time windows and the locality layout only
    slot_arcs = nc * th * 8 if inst.has_tw and inst.N * inst.N * 4 > (64 << 20) else 0
    return (nc * th * 4 + nc * 4 + slot_arcs) + attrs * n


def unit_bytes(inst, n_routes):
    """Compulsory bytes of one pair-evaluation launch for one unit's own state: node
    state (rt, pos), both segment arrays over the used positions, the route table,
    and the block-best records written."""
    nc, n, th = inst.n_customers, inst.N, inst.theta
    seg = 32 if inst.has_tw else 16
    tiles = (nc * th + 255) // 256
    return 8 * n + 2 * (nc + 2 * n_routes) * seg + 40 * n_routes + 40 * tiles


def pair_families(inst):
    from paper_2605_05208_amd import mdvrp
    f = [mdvrp.FAM_RELOCATE, mdvrp.FAM_SWAP, mdvrp.FAM_2OPT_STAR]
    if not inst.has_tw:
        f.append(mdvrp.FAM_2OPT)
    return f


def algorithmic_bytes(B, inst, sols):
    """Mean compulsory bytes per pair-evaluation launch on the given states: what the
    units of the instance share, once (lists, node attributes, 4 bytes per distinct
    matrix entry read; c = t), plus each unit's own state."""
    out = []
    for fam in pair_families(inst):
        distinct = sum(B.eval_footprint(fam))
        per_matrix_entry = 4 if inst.t is inst.c else 8
        own = sum(unit_bytes(inst, len(s.routes)) for s in sols)
        out.append(instance_bytes(inst) + own + per_matrix_entry * distinct)
    return float(np.mean(out))


def host_facts():
    """Host cores usable by this process and the CPU model (from /proc/cpuinfo)."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    limit = int(os.environ.get("OMP_NUM_THREADS", usable) or usable)
    return dict(nproc=usable, omp_threads=min(usable, limit), cpu_model=model)


def cpu_baseline(inst, sols, seed, passes=1):
    """The oracle's local search (every move of a family evaluated by recomputing the
    changed routes from scratch) over `passes` passes from the start solutions: one
    solution on one thread, and one solution per thread on every usable core."""
    import oracle
    from oracle import Ref
    host = host_facts()
    ref = Ref(inst)
    ref.neighbours()
    out = {}
    old = oracle.set_threads(1)
    try:
        for name, threads in (("one_thread", 1), ("all_cores", host["omp_threads"])):
            oracle.set_threads(threads)
            sample = sols[:min(threads, len(sols))]
            t0 = time.perf_counter()
            _, st = ref.local_search(sample, seed=seed, max_passes=passes)
            dt = time.perf_counter() - t0
            ev = sum(s["evaluated"] for s in st)
            out[name] = dict(value=ev / dt, threads=threads, solutions=len(sample), evaluated=ev,
                             seconds=round(dt, 2))
    finally:
        oracle.set_threads(old)
    a = out["all_cores"]
    return dict(value=a["value"], unit="move-evals/s", cores=a["threads"], kind="oracle",
                sample=f"{a['solutions']} of the {len(sols)} start solutions, {passes} pass(es) of the local search "
                       f"(Algorithm 2) each, one solution per thread: {a['evaluated']} evaluated moves in "
                       f"{a['seconds']} s",
                one_thread=out["one_thread"], host=host)


def ls_run(B, sols, **kw):
    """Local search of the batch from `sols`; returns (seconds, stats, profile)."""
    import torch
    B.load(sols)
    if kw.pop("eta", False):
        B.eta_lists()
    torch.cuda.synchronize()
    B.profile_enable(1 << 5)  # HIP events around the re-ranking launches only
    t0 = time.perf_counter()
    st = B.local_search_to_optimum(seed=1, poll_every=4, **kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = B.profile_read()
    B.profile_enable(0)
    assert all(s["converged"] and s["err"] == 0 for s in st)
    _, terms = B.cost()
    return dt, st, prof, terms


TERM_NAMES = ("D", "TW", "LX", "DX", "CL", "FX")


def term_means(terms):
    """Mean over units of each term of Eq. A.1 (distance, time warp, load, duration,
    closure and fleet excess) at the local optima."""
    return {k: float(np.mean(terms[:, j])) for j, k in enumerate(TERM_NAMES)}


def filter_study(n_sol=16, ks=(8, 4), epochs=6, rescore=32):
    """Full vs filtered local search on the 20 x 10000 MDVRPTW instance, for each list
    length in ks (8 is the configured top-8; 4 is shorter)."""
    import torch

    from paper_2605_05208_amd import filter_train as ft
    from paper_2605_05208_amd import gen, mdvrp
    t0 = time.perf_counter()
    insts = ft.training_instances(8)
    dev = [mdvrp.Instance(i) for i in insts]
    unit_inst = [0] * 16 + list(range(1, len(insts)))
    sols = [gen.start_solution(insts[0], insts[0].seed * 1000 + j) for j in range(16)]
    sols += [gen.start_solution(insts[j], insts[j].seed * 1000) for j in range(1, len(insts))]
    TB = mdvrp.Batch(dev, unit_inst)
    x, y, w, snaps = ft.log_states(TB, sols, chunk=2, max_chunks=40)
    torch.cuda.synchronize()
    t_log = time.perf_counter() - t0
    M = mdvrp.Mlp(None)
    M.set_params(ft.init_params(0))
    losses, t_train = ft.train(M, x, y, w, epochs=epochs, lr=1e-3)
    del TB, dev

    I5 = gen.config5()
    D5 = mdvrp.Instance(I5)
    s5 = [gen.start_solution(I5, I5.seed * 1000 + j) for j in range(n_sol)]
    B5 = mdvrp.Batch([D5], [0] * n_sol)
    B5.load(s5)
    shapes = B5.autotune(reps=2)
    full_dt, full_st, _, full_terms = ls_run(B5, s5)
    full_F = np.array([s["F"] for s in full_st], np.float64)
    out = dict(workload=f"{I5.name}: {n_sol} solutions, local search to a local optimum of the full neighbourhood",
               rescore_every_passes=rescore, full_ms=round(full_dt * 1e3, 1), full_F_mean=float(full_F.mean()),
               full_terms=term_means(full_terms), tile_threads_per_family=shapes,
               full_evaluated=int(sum(s["evaluated"] for s in full_st)),
               full_passes_max=int(max(s["passes"] for s in full_st)),
               train=dict(samples=int(x.shape[0]), positives=int(y.sum().item()), snapshots=snaps,
                          log_s=round(t_log, 2), train_s=round(t_train, 2), epochs=epochs,
                          loss_first=round(losses[0], 4), loss_last=round(losses[-1], 4)))
    for k in ks:
        Bk = mdvrp.Batch([D5], [0] * n_sol)
        Bk.filter_attach(k)
        Bk.load(s5)
        Bk.set_tile_shapes(shapes)
        res = {}
        for name, kw in (("mlp", dict(filter=mdvrp.FILTER_MLP, mlp=M, rescore=rescore)),
                         ("eta", dict(filter=mdvrp.FILTER_LISTS, eta=True))):
            dt, st, prof, terms = ls_run(Bk, s5, **kw)
            F = np.array([s["F"] for s in st], np.float64)
            gap = (F - full_F) / full_F
            res[name] = dict(ms=round(dt * 1e3, 1), speedup=round(full_dt / dt, 3), gap_mean=float(gap.mean()),
                             gap_max=float(gap.max()), F_mean=float(F.mean()), terms=term_means(terms),
                             evaluated=int(sum(s["evaluated"] for s in st)),
                             passes_max=int(max(s["passes"] for s in st)),
                             fallback_passes_max=int(max(s["fallback_passes"] for s in st)),
                             score_ms=round(prof["filter_score"][1], 1))
        out[f"k{k}"] = res
        del Bk
    return out


def batch_study(n_inst=256, graph=True):
    """All 256 uneven MDVRPTW instances (one seeded solution each) in one batch, every pass
    of the local search replayed from a captured HIP graph. Per-instance time is the
    device clock from the start of the search to the end of the instance's last pass."""
    import concurrent.futures as cf

    import torch

    from paper_2605_05208_amd import gen, mdvrp
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=8) as ex:
        insts = list(ex.map(gen.config4_instance, range(n_inst)))
    t_gen = time.perf_counter() - t0
    dev = [mdvrp.Instance(I) for I in insts]
    B = mdvrp.Batch(dev, list(range(n_inst)))
    sols = [gen.start_solution(I, I.seed * 1000) for I in insts]
    B.load(sols)
    shapes = B.autotune(reps=2)
    runs = []
    for _ in range(2):  # the first run captures the graphs
        B.load(sols)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st = B.local_search_to_optimum(seed=1, poll_every=4, graph=graph)
        torch.cuda.synchronize()
        runs.append((time.perf_counter() - t1, st))
    dt, st = runs[-1]
    assert all(s["converged"] and s["err"] == 0 for s in st)
    per = np.array([s["device_ms"] for s in st])
    ev = sum(s["evaluated"] for s in st)
    nc = np.array([I.n_customers for I in insts])
    # the critical path: the unit that finishes last, searched alone in a batch of its own
    # (no batch of any design can finish before its own pass chain does)
    last = int(per.argmax())
    B1 = mdvrp.Batch([dev[last]], [0])
    B1.load([sols[last]])
    B1.set_tile_shapes(shapes)
    B1.local_search_to_optimum(seed=1, poll_every=4, graph=graph)  # capture
    B1.load([sols[last]])
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    st1 = B1.local_search_to_optimum(seed=1, poll_every=4, graph=graph)
    torch.cuda.synchronize()
    alone_s = time.perf_counter() - t2
    assert st1[0]["passes"] == st[last]["passes"]
    lanes = batch_lanes(dev, sols, shapes, nc, [s["F"] for s in st], graph)
    return dict(workload=f"{n_inst} uneven MDVRPTW instances (100..5000 customers, 2..20 depots), one solution each, "
                         "one batch, local search to optimum" + (", passes replayed from HIP graphs" if graph else ""),
                customers=int(nc.sum()), seconds=round(dt, 3), instances_per_s=round(n_inst / dt, 2),
                move_evals_per_s=round(ev / dt, 1), per_instance_ms_p50=round(float(np.percentile(per, 50)), 2),
                per_instance_ms_p99=round(float(np.percentile(per, 99)), 2),
                per_instance_ms_max=round(float(per.max()), 2),
                passes_max=int(max(s["passes"] for s in st)), first_run_s=round(runs[0][0], 3),
                last_unit=dict(customers=int(nc[last]), passes=int(st[last]["passes"]),
                               in_batch_ms=round(float(per[last]), 2), alone_ms=round(alone_s * 1e3, 2)),
                tile_threads_per_family=shapes, lanes=lanes,
                generate_s=round(t_gen, 1))


def batch_lanes(dev, sols, shapes, nc, ref_F, graph, k_big=16):
    """The same instances as two batches searched at once on two streams: the k_big
    largest in one, the rest in the other (each host thread drives one batch). The
    large instances' long pass chains then no longer wait for the small instances'
    passes, which is what a persistent work queue would buy."""
    import threading

    import torch

    from paper_2605_05208_amd import mdvrp
    order = np.argsort(-np.asarray(nc), kind="stable")
    groups = [sorted(order[:k_big].tolist()), sorted(order[k_big:].tolist())]
    batches = []
    for g in groups:
        Bg = mdvrp.Batch(dev, g)
        Bg.set_tile_shapes(shapes)
        batches.append(Bg)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    res = {}

    def run(k):
        with torch.cuda.stream(streams[k]):
            res[k] = batches[k].local_search_to_optimum(seed=1, poll_every=4, graph=graph)
            torch.cuda.current_stream().synchronize()

    dt = None
    for _ in range(2):  # the first run captures the graphs
        for k in range(2):
            with torch.cuda.stream(streams[k]):
                batches[k].load([sols[i] for i in groups[k]])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        threads = [threading.Thread(target=run, args=(k,)) for k in range(2)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    per = np.zeros(len(nc))
    F = [0] * len(nc)
    for k in range(2):
        for i, s in zip(groups[k], res[k]):
            assert s["converged"] and s["err"] == 0
            per[i] = s["device_ms"]
            F[i] = s["F"]
    assert F == list(ref_F), "two concurrent batches must reach the single batch's optima"
    n = len(nc)
    return dict(design=f"two concurrent batches on two streams: the {k_big} largest instances and the other {n - k_big}",
                seconds=round(dt, 3), instances_per_s=round(n / dt, 2),
                per_instance_ms_p50=round(float(np.percentile(per, 50)), 2),
                per_instance_ms_p99=round(float(np.percentile(per, 99)), 2))


def _event_ms(fn, reps=1):
    """Mean milliseconds of fn() between two HIP events on the current stream (the stream
    the library launches on)."""
    import torch
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = None
    e0.record(s)
    for _ in range(reps):
        out = fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps, out


def rows_study(seed=1):
    """The rows beyond the local search itself, each timed on the GPU: dynamic penalty
    coefficients (Section 3.2.1), repair insertions (Section 3.3), population distance
    and reduction (Section 3.4), DCREX route-pair counts and UCB1 (Algorithm 3, Eq. 4)."""
    import torch

    from paper_2605_05208_amd import gen, mdvrp
    out = {}
    # ---- dynamic penalty coefficients: 64 MDVRPTW solutions, depth delta = 500 (Table 1)
    I2 = gen.config2()
    s2 = [gen.start_solution(I2, I2.seed * 1000 + k) for k in range(64)]
    B2 = mdvrp.Batch([mdvrp.Instance(I2)], [0] * 64)
    B2.load(s2)
    B2.autotune(reps=2)
    adapt = ([1, 1, 1, 1], [1 << 12, 1 << 12, 1 << 12, 1 << 20])
    B2.load(s2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = B2.local_search_to_optimum(seed=seed, poll_every=4, max_passes=500, adapt=adapt)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ev = sum(x["evaluated"] for x in st)
    w = np.array([x["w_final"] for x in st])
    out["penalty_adapt"] = dict(workload=f"{I2.name}: 64 solutions, local search of depth 500 with dynamic penalty "
                                         "coefficients (kappa = 1/2)", ms=round(dt * 1e3, 1),
                                move_evals_per_s=round(ev / dt, 1), passes_max=int(max(x["passes"] for x in st)),
                                moves_applied=int(sum(x["moves_applied"] for x in st)),
                                final_weights_median=[int(v) for v in np.median(w, axis=0)])
    # ---- population: the 64 local optima of the fixed-weight search, reduced to mu = 20
    B2.load(s2)
    B2.local_search_to_optimum(seed=seed, poll_every=4)
    units = list(range(64))
    d, _, _ = B2.population_distance(units)
    ms_d, (d, _, _) = _event_ms(lambda: B2.population_distance(units), reps=5)
    F, _ = B2.cost()
    f = torch.from_numpy(np.ascontiguousarray(F)).to("cuda")
    ms_r, _ = _event_ms(lambda: mdvrp.population_reduce(d, f, 20, 0.7, 5), reps=5)
    dd = d.cpu().numpy()
    out["population"] = dict(workload=f"{I2.name}: 64 local optima, distance of every pair (Eq. 7), reduction to "
                                      "mu = 20 by chi (Eq. 5-6, xi = 0.7)", distance_ms=round(ms_d, 3),
                             pairs=64 * 65 // 2, reduce_ms=round(ms_r, 3),
                             mean_distance=round(float(dd[np.triu_indices(64, 1)].mean()), 3))
    del B2
    # ---- repair and DCREX at the 20 x 10000 scale
    I3 = gen.config3()
    D3 = mdvrp.Instance(I3)
    s3 = [gen.start_solution(I3, I3.seed * 1000 + k) for k in range(16)]
    rng = np.random.default_rng(seed)
    parts = []
    for k, sol in enumerate(s3):
        gone = set(rng.choice(np.arange(I3.n_depots, I3.N), size=200, replace=False).tolist())
        routes = [(a, [x for x in xs if x not in gone], b) for a, xs, b in sol.routes]
        parts.append(gen.Solution([r for r in routes if r[1]]))
    B3 = mdvrp.Batch([D3], [0] * 16)
    rep = {}
    for name, op in (("FBI", mdvrp.REPAIR_FBI), ("IBI", mdvrp.REPAIR_IBI), ("FRI", mdvrp.REPAIR_FRI),
                     ("IRI", mdvrp.REPAIR_IRI), ("RI", mdvrp.REPAIR_RI)):
        B3.load_partial(parts)
        torch.cuda.synchronize()
        ms, (_, nev) = _event_ms(lambda: B3.repair(op, seed=seed))
        rep[name] = dict(ms=round(ms, 2), positions_evaluated=int(sum(nev)),
                         positions_per_s=round(sum(nev) / (ms / 1e3), 1))
    out["repair"] = dict(workload=f"{I3.name}: 16 start solutions with 200 customers removed from each", **rep)
    a, b, p = s3[0], s3[1], s3[2]
    pick = rng.choice(len(b.routes), size=20, replace=False)
    off = list(a.routes) + [b.routes[k] for k in pick]
    intro = [0] * len(a.routes) + [1] * 20
    mdvrp.dcrex_counts(I3.n_depots, I3.N, off, intro, list(p.routes))
    ms_c, counts = _event_ms(lambda: mdvrp.dcrex_counts(I3.n_depots, I3.N, off, intro, list(p.routes)), reps=3)
    out["dcrex"] = dict(workload=f"{I3.name}: offspring of {len(off)} routes (20 introduced) against a parent of "
                                 f"{len(p.routes)} routes", pairs=len(off) * len(p.routes),
                        counts_ms_incl_host_checks=round(ms_c, 3), pick=mdvrp.dcrex_pick(counts, seed))
    return out


MLP_FWD_FLOP = 2 * (32 * 256 + 256 * 256 + 256)  # per scored anchor / forward sample
MFMA_BF16_PEAK_TFLOPS = 2500.0


def mlp_probe(n_sol=16, reps=5, n_train=65536):
    """Scoring every list of the 20 x 10000 MDVRPTW batch and training steps, timed with
    HIP events on the library's stream (MFMA-bound kernels of the filter)."""
    import torch

    from paper_2605_05208_amd import filter_train as ft
    from paper_2605_05208_amd import gen, mdvrp
    I5 = gen.config5()
    B5 = mdvrp.Batch([mdvrp.Instance(I5)], [0] * n_sol)
    B5.filter_attach(8)
    B5.load([gen.start_solution(I5, I5.seed * 1000 + j) for j in range(n_sol)])
    M = mdvrp.Mlp(ft.init_params(0))
    B5.score_topk(M, want_logits=False)
    torch.cuda.synchronize()
    B5.profile_enable(1 << 5)
    for _ in range(reps):
        B5.score_topk(M, want_logits=False)
    n_l, ms = B5.profile_read()["filter_score"]
    B5.profile_enable(0)
    anchors = B5.anchor_count()
    score_s = ms / n_l / 1e3
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    x = (torch.randint(0, 1 << 14, (n_train, 32), dtype=torch.int16, device="cuda", generator=g) & 0x3FFF) - 0x2000
    y = (torch.rand(n_train, device="cuda", generator=g) < 0.3).float()
    M.train_step(x, y, None, 1e-3, 1)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for k in range(reps):
        M.train_step(x, y, None, 1e-3, k + 2)
    e1.record(s)
    torch.cuda.synchronize()
    train_s = e0.elapsed_time(e1) / reps / 1e3
    score_tf = anchors * MLP_FWD_FLOP / score_s / 1e12
    train_tf = n_train * 3 * MLP_FWD_FLOP / train_s / 1e12
    return dict(anchors=anchors, score_ms=round(score_s * 1e3, 3), score_tflops=round(score_tf, 1),
                score_frac=round(score_tf / MFMA_BF16_PEAK_TFLOPS, 4), train_samples=n_train,
                train_step_ms=round(train_s * 1e3, 3), train_tflops=round(train_tf, 1),
                train_frac=round(train_tf / MFMA_BF16_PEAK_TFLOPS, 4))


def calibrate_copy(nbytes=1 << 30, reps=5):
    """A plain device-to-device copy of known size (reference for the HBM byte counters)."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "reps": reps}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="config3")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-passes", type=int, default=1, help="search passes of the CPU oracle leg (0 = skip)")
    ap.add_argument("--no-extra", action="store_true", help="skip the open-route and small-instance searches")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--no-filter", action="store_true", help="skip the learned-filter comparison")
    ap.add_argument("--no-batch", action="store_true", help="skip the 256-instance uneven batch")
    ap.add_argument("--no-rows", action="store_true",
                    help="skip the adaptive-penalty, population, repair and crossover measurements")
    ap.add_argument("--rows-only", action="store_true", help="only run those measurements")
    ap.add_argument("--no-tune", action="store_true", help="keep the default tile shapes (no autotuning)")
    ap.add_argument("--calibrate-copy", action="store_true", help="only run a plain 1 GiB copy (counter reference)")
    ap.add_argument("--mlp-probe", action="store_true", help="only time the filter's scoring and training kernels")
    ap.add_argument("--filter-only", action="store_true", help="only run the learned-filter comparison")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the local search of a population is data parallel over "
              "solutions, and this implementation runs on a single MI355X; a population would shard by solutions, one process per GPU.",
              file=sys.stderr)
        return 2

    if args.calibrate_copy:
        calibrate_copy()
        return 0
    if args.mlp_probe:
        print(json.dumps(mlp_probe()), flush=True)
        return 0
    if args.filter_only:
        print(json.dumps(filter_study()), flush=True)
        return 0
    if args.rows_only:
        print(json.dumps(rows_study(args.seed)), flush=True)
        return 0

    from paper_2605_05208_amd import mdvrp  # noqa: F401  (fails loudly without the library)

    head = search_bench(args.workload, args.steps, args.warmup, args.seed, tune=not args.no_tune,
                        roofline=not args.no_roofline)
    inst, sols, stats, dt = head.pop("_inst"), head.pop("_sols"), head.pop("_stats"), head.pop("_dt")
    subs = {}
    if not args.no_extra:
        for key, name in (("open", "config3_open"), ("small", "config2")):
            if name != args.workload:
                r = search_bench(name, 2, 1, args.seed, tune=not args.no_tune, roofline=False)
                for k in ("_inst", "_sols", "_stats", "_dt"):
                    r.pop(k)
                subs[key] = r

    cpu = None
    if args.cpu_passes > 0:
        cpu = cpu_baseline(inst, sols, args.seed, passes=args.cpu_passes)
    filt = None if args.no_filter else filter_study()
    batch = None if args.no_batch else batch_study()
    rows = None if args.no_rows else rows_study(args.seed)

    line = {
        "metric": "penalised move evals/s + time to local optimum",
        "value": head["move_evals_per_s"],
        "unit": "move-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": head["config"],
        "time_to_local_optimum_ms": head["time_to_local_optimum_ms"],
        "evaluated_per_step": head["evaluated_per_step"],
        "passes_max": head["passes_max"],
        "moves_applied_per_step": head["moves_applied_per_step"],
        "F_mean": head["F_mean"],
        "eval_pairs_ms_per_step_est": head["eval_pairs_ms_per_step_est"],
        "tile_threads_per_family": head["tile_threads_per_family"],
        "roofline": head["roofline"],
        "cpu_baseline": cpu,
        **subs,
        "filter": filt,
        "batch": batch,
        "rows": rows,
    }
    print(json.dumps(line), flush=True)
    return 0


def search_bench(name, steps, warmup, seed, tune=True, roofline=True):
    """Time `steps` local searches to the local optimum of workload `name` (start
    solutions reloaded from HBM each step) after `warmup` untimed ones."""
    import torch

    from paper_2605_05208_amd import mdvrp
    from paper_2605_05208_amd.gen import batch_flat

    inst, sols = workload(name)
    dev = mdvrp.Instance(inst)
    B = mdvrp.Batch([dev], [0] * len(sols))
    nodes, offs, st, en, so = batch_flat(sols)
    d_in = [torch.from_numpy(x).to("cuda") for x in (nodes, offs, st, en, so)]
    n_routes, n_nodes = len(st), len(nodes)

    B.load_device(*d_in, n_routes, n_nodes)
    shapes = B.autotune(reps=3) if tune else None

    def step():
        B.load_device(*d_in, n_routes, n_nodes)
        return B.local_search_to_optimum(seed=seed, poll_every=4)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    # HIP events around every 8th launch of the dominant kernel class (pair evaluation):
    # each timed launch delays the next one by a few microseconds, so sampling keeps
    # the timed region close to an untimed run while still averaging over all passes
    B.profile_sampling(PROFILE_EVERY)
    B.profile_enable(1)
    t0 = time.perf_counter()
    stats = None
    for _ in range(steps):
        stats = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = B.profile_read()
    B.profile_enable(0)
    dt = t1 - t0
    evaluated = sum(s["evaluated"] for s in stats)
    assert all(s["converged"] and s["err"] == 0 for s in stats), "a unit did not converge"

    roof = None
    if roofline:
        final = B.export()
        b_final = algorithmic_bytes(B, inst, final)
        B.load_device(*d_in, n_routes, n_nodes)
        b_start = algorithmic_bytes(B, inst, sols)
        b_alg = 0.5 * (b_final + b_start)
        n_l, ms_l = prof["eval_pairs"]
        avg_s = ms_l / max(n_l, 1) / 1e3
        achieved = b_alg / avg_s / 1e9
        traffic = measured_traffic(name)
        roof = dict(bound="hbm", achieved=round(achieved, 2), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 5), traffic=traffic, kernel="k_eval_pairs",
                    bytes_per_launch=int(b_alg), bytes_start=int(b_start), bytes_final=int(b_final),
                    timed_launches=n_l, timed_every=PROFILE_EVERY, avg_launch_us=round(avg_s * 1e6, 2))
    F = [int(s["F"]) for s in stats]
    return {
        "config": {
            "workload": f"{inst.name}: {len(sols)} seeded start solutions, multi-move local search to a local "
                        "optimum (all operator families, leader-follower selection)",
            "depots": inst.n_depots, "customers": inst.n_customers, "solutions": len(sols),
            "theta": inst.theta, "time_windows": bool(inst.has_tw), "open_routes": bool(inst.open_routes),
        },
        "move_evals_per_s": round(evaluated * steps / dt, 1),
        "steps": steps,
        "time_to_local_optimum_ms": round(dt / steps * 1e3, 3),
        "evaluated_per_step": evaluated,
        "passes_max": int(max(s["passes"] for s in stats)),
        "moves_applied_per_step": int(sum(s["moves_applied"] for s in stats)),
        "F_mean": float(np.mean(F)),
        # sampled launches scaled by the sampling period
        "eval_pairs_ms_per_step_est": round(prof["eval_pairs"][1] * PROFILE_EVERY / steps, 3),
        "tile_threads_per_family": shapes,
        "roofline": roof,
        "_inst": inst, "_sols": sols, "_stats": stats, "_dt": dt,
    }


if __name__ == "__main__":
    sys.exit(main())
