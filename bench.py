#!/usr/bin/env python3
"""Benchmark: penalised move evaluations per second, time to local optimum, and
the learned filter against full evaluation.

One step = load 64 seeded start solutions of the 8-depot / 1000-customer
MDVRPTW instance (already resident in HBM) into the segment state and run the
multi-move local search of every solution to its local optimum (evaluation of
every operator family, leader-follower selection, apply, repeat until a full
pass applies nothing). The line reports whole-job move evaluations per second,
the time per step, the roofline of the dominant kernel (HIP events on the
library's stream; compulsory bytes per launch, see the design notes) and the
CPU oracle timed on a bounded sample of the same workload.

The `filter` object compares, on the 20-depot / 10000-customer MDVRPTW
instance with 16 solutions, the local search over the full granular lists
with the searches over 4-entry lists ranked by the trained network (stale lists
re-ranked every 32 passes) and by the eta order: GPU time, and the gap of the
local-optimum cost per seed. The
network is trained first, on the GPU, from logs of full-list searches of the
1000-customer instance and of uneven instances (not timed in the comparison).
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
PAIR_PROFILES = {"config2": "k_eval_pairs_mdvrptw-8x1000_64sol.md", "config5": "k_eval_pairs_mdvrptw-20x10000_16sol.md"}


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


def non_matrix_bytes(inst, n_routes):
    """Compulsory bytes of one pair-evaluation launch for one unit, matrix excluded:
    granular lists, node state (rt, pos), node attributes, both segment arrays over
    the used positions, the route table, and the block-best records written."""
    nc, n, th = inst.n_customers, inst.N, inst.theta
    seg = 32 if inst.has_tw else 16
    attrs = 16 if inst.has_tw else 8
    tiles = (nc * th + 255) // 256
    return (nc * th * 4 + nc * 4) + 8 * n + attrs * n + 2 * (nc + 2 * n_routes) * seg + 40 * n_routes + 40 * tiles


def pair_families(inst):
    from paper_2605_05208_amd import mdvrp
    f = [mdvrp.FAM_RELOCATE, mdvrp.FAM_SWAP, mdvrp.FAM_2OPT_STAR]
    if not inst.has_tw:
        f.append(mdvrp.FAM_2OPT)
    return f


def algorithmic_bytes(B, inst, sols):
    """Mean compulsory bytes per pair-evaluation launch on the given states:
    per unit non-matrix bytes + 4 bytes per distinct matrix entry read (c = t)."""
    out = []
    for fam in pair_families(inst):
        distinct = sum(B.eval_footprint(fam))
        per_matrix_entry = 4 if inst.t is inst.c else 8
        nm = sum(non_matrix_bytes(inst, len(s.routes)) for s in sols)
        out.append(nm + per_matrix_entry * distinct)
    return float(np.mean(out))


def cpu_baseline(inst, sols, n_sample, seed):
    from oracle import Ref
    ref = Ref(inst)
    ref.neighbours()
    sample = sols[:n_sample]
    t0 = time.perf_counter()
    _, st = ref.local_search(sample, seed=seed)
    dt = time.perf_counter() - t0
    ev = sum(s["evaluated"] for s in st)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    cores = max(1, min(len(sample), threads, os.cpu_count() or 1))
    return dict(value=ev / dt, unit="move-evals/s", cores=cores, kind="oracle",
                sample=f"{len(sample)} of the {len(sols)} solutions, local search to optimum, "
                       f"{ev} evaluated moves in {dt:.1f} s", seconds=round(dt, 2))


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
    return dt, st, prof


def filter_study(n_sol=16, k=4, epochs=6, rescore=32):
    """Full vs filtered local search on the 20 x 10000 MDVRPTW instance."""
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
    s5 = [gen.start_solution(I5, I5.seed * 1000 + j) for j in range(n_sol)]
    B5 = mdvrp.Batch([mdvrp.Instance(I5)], [0] * n_sol)
    B5.filter_attach(k)
    B5.load(s5)
    shapes = B5.autotune(reps=2)
    runs = {}
    for name, kw in (("full", {}), ("eta", dict(filter=mdvrp.FILTER_LISTS, eta=True)),
                     ("mlp", dict(filter=mdvrp.FILTER_MLP, mlp=M, rescore=rescore))):
        dt, st, prof = ls_run(B5, s5, **kw)
        runs[name] = (dt, np.array([s["F"] for s in st], np.float64), st, prof)
    full_dt, full_F = runs["full"][0], runs["full"][1]
    out = dict(workload=f"{I5.name}: {n_sol} solutions, local search to a local optimum of the full neighbourhood",
               k=k, rescore_every_passes=rescore, full_ms=round(full_dt * 1e3, 1), full_F_mean=float(full_F.mean()),
               tile_threads_per_family=shapes,
               full_evaluated=int(sum(s["evaluated"] for s in runs["full"][2])),
               full_passes_max=int(max(s["passes"] for s in runs["full"][2])),
               train=dict(samples=int(x.shape[0]), positives=int(y.sum().item()), snapshots=snaps,
                          log_s=round(t_log, 2), train_s=round(t_train, 2), epochs=epochs,
                          loss_first=round(losses[0], 4), loss_last=round(losses[-1], 4)))
    for name in ("mlp", "eta"):
        dt, F, st, prof = runs[name]
        gap = (F - full_F) / full_F
        out[name] = dict(ms=round(dt * 1e3, 1), speedup=round(full_dt / dt, 3), gap_mean=float(gap.mean()),
                         gap_max=float(gap.max()), F_mean=float(F.mean()),
                         evaluated=int(sum(s["evaluated"] for s in st)),
                         passes_max=int(max(s["passes"] for s in st)),
                         fallback_passes_max=int(max(s["fallback_passes"] for s in st)),
                         score_ms=round(prof["filter_score"][1], 1))
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
    return dict(workload=f"{n_inst} uneven MDVRPTW instances (100..5000 customers, 2..20 depots), one solution each, "
                         "one batch, local search to optimum" + (", passes replayed from HIP graphs" if graph else ""),
                customers=int(nc.sum()), seconds=round(dt, 3), instances_per_s=round(n_inst / dt, 2),
                move_evals_per_s=round(ev / dt, 1), per_instance_ms_p50=round(float(np.percentile(per, 50)), 2),
                per_instance_ms_p99=round(float(np.percentile(per, 99)), 2),
                per_instance_ms_max=round(float(per.max()), 2),
                passes_max=int(max(s["passes"] for s in st)), first_run_s=round(runs[0][0], 3),
                tile_threads_per_family=shapes,
                generate_s=round(t_gen, 1))


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
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="config2")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-sample", type=int, default=8, help="solutions for the CPU oracle leg (0 = skip)")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--no-filter", action="store_true", help="skip the learned-filter comparison")
    ap.add_argument("--no-batch", action="store_true", help="skip the 256-instance uneven batch")
    ap.add_argument("--no-tune", action="store_true", help="keep the default tile shapes (no autotuning)")
    ap.add_argument("--calibrate-copy", action="store_true", help="only run a plain 1 GiB copy (counter reference)")
    ap.add_argument("--mlp-probe", action="store_true", help="only time the filter's scoring and training kernels")
    ap.add_argument("--filter-only", action="store_true", help="only run the learned-filter comparison")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the local search of a population is data parallel over "
              "solutions, and this build runs on a single MI355X (see the design notes for how it shards).",
              file=sys.stderr)
        return 2

    import torch

    if args.calibrate_copy:
        calibrate_copy()
        return 0
    if args.mlp_probe:
        print(json.dumps(mlp_probe()), flush=True)
        return 0
    if args.filter_only:
        print(json.dumps(filter_study()), flush=True)
        return 0

    from paper_2605_05208_amd import mdvrp
    from paper_2605_05208_amd.gen import batch_flat

    inst, sols = workload(args.workload)
    dev = mdvrp.Instance(inst)
    B = mdvrp.Batch([dev], [0] * len(sols))
    nodes, offs, st, en, so = batch_flat(sols)
    d_in = [torch.from_numpy(x).to("cuda") for x in (nodes, offs, st, en, so)]
    n_routes, n_nodes = len(st), len(nodes)

    B.load_device(*d_in, n_routes, n_nodes)
    shapes = B.autotune(reps=3) if not args.no_tune else None

    def step():
        B.load_device(*d_in, n_routes, n_nodes)
        return B.local_search_to_optimum(seed=args.seed, poll_every=4)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # HIP events around every 8th launch of the dominant kernel class (pair evaluation):
    # each timed launch delays the next one by a few microseconds, so sampling keeps
    # the timed region close to an untimed run while still averaging over all passes
    B.profile_sampling(PROFILE_EVERY)
    B.profile_enable(1)
    t0 = time.perf_counter()
    stats = None
    for _ in range(args.steps):
        stats = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = B.profile_read()
    B.profile_enable(0)
    dt = t1 - t0
    evaluated = sum(s["evaluated"] for s in stats)
    assert all(s["converged"] and s["err"] == 0 for s in stats), "a unit did not converge"
    value = evaluated * args.steps / dt

    roof = None
    if not args.no_roofline:
        final = B.export()
        b_final = algorithmic_bytes(B, inst, final)
        B.load_device(*d_in, n_routes, n_nodes)
        b_start = algorithmic_bytes(B, inst, sols)
        b_alg = 0.5 * (b_final + b_start)
        n_l, ms_l = prof["eval_pairs"]
        avg_s = ms_l / max(n_l, 1) / 1e3
        achieved = b_alg / avg_s / 1e9
        traffic = measured_traffic(args.workload)
        roof = dict(bound="hbm", achieved=round(achieved, 2), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 5), traffic=traffic, kernel="k_eval_pairs",
                    bytes_per_launch=int(b_alg), timed_launches=n_l, timed_every=PROFILE_EVERY,
                    avg_launch_us=round(avg_s * 1e6, 2))

    cpu = None
    if args.cpu_sample > 0:
        cpu = cpu_baseline(inst, sols, args.cpu_sample, args.seed)
    filt = None if args.no_filter else filter_study()
    batch = None if args.no_batch else batch_study()

    F = [int(s["F"]) for s in stats]
    line = {
        "metric": "penalised move evals/s + time to local optimum",
        "value": round(value, 1),
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
        "config": {
            "workload": f"{inst.name}: {len(sols)} seeded start solutions, multi-move local search to a local "
                        "optimum (all operator families, leader-follower selection)",
            "depots": inst.n_depots, "customers": inst.n_customers, "solutions": len(sols),
            "theta": inst.theta, "time_windows": bool(inst.has_tw), "open_routes": bool(inst.open_routes),
        },
        "time_to_local_optimum_ms": round(dt / args.steps * 1e3, 3),
        "evaluated_per_step": evaluated,
        "passes_max": int(max(s["passes"] for s in stats)),
        "moves_applied_per_step": int(sum(s["moves_applied"] for s in stats)),
        "F_mean": float(np.mean(F)),
        # sampled launches scaled by the sampling period
        "eval_pairs_ms_per_step_est": round(prof["eval_pairs"][1] * PROFILE_EVERY / args.steps, 3),
        "tile_threads_per_family": shapes,
        "roofline": roof,
        "cpu_baseline": cpu,
        "filter": filt,
        "batch": batch,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
