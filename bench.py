#!/usr/bin/env python3
"""Benchmark: penalised move evaluations per second and time to local optimum.

One step = load 64 seeded start solutions of the 8-depot / 1000-customer
MDVRPTW instance (already resident in HBM) into the segment state and run the
multi-move local search of every solution to its local optimum (evaluation of
every operator family, leader-follower selection, apply, repeat until a full
pass applies nothing). The line reports whole-job move evaluations per second,
the time per step, the roofline of the dominant kernel (HIP events on the
library's stream; compulsory bytes per launch, see the design notes) and the
CPU oracle timed on a bounded sample of the same workload.
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
    else:
        raise SystemExit(f"unknown workload {name}")
    sols = [gen.start_solution(inst, inst.seed * 1000 + k) for k in range(n)]
    return inst, sols


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="config2")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-sample", type=int, default=8, help="solutions for the CPU oracle leg (0 = skip)")
    ap.add_argument("--no-roofline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the local search of a population is data parallel over "
              "solutions, and this build runs on a single MI355X (see the design notes for how it shards).",
              file=sys.stderr)
        return 2

    import torch

    from paper_2605_05208_amd import mdvrp
    from paper_2605_05208_amd.gen import batch_flat

    inst, sols = workload(args.workload)
    dev = mdvrp.Instance(inst)
    B = mdvrp.Batch([dev], [0] * len(sols))
    nodes, offs, st, en, so = batch_flat(sols)
    d_in = [torch.from_numpy(x).to("cuda") for x in (nodes, offs, st, en, so)]
    n_routes, n_nodes = len(st), len(nodes)

    def step():
        B.load_device(*d_in, n_routes, n_nodes)
        return B.local_search_to_optimum(seed=args.seed, poll_every=4)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    B.profile_enable(1)  # time the dominant kernel class (pair evaluation) only
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
        roof = dict(bound="hbm", achieved=round(achieved, 2), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 5), traffic=None, kernel="k_eval_pairs",
                    bytes_per_launch=int(b_alg), launches=n_l, avg_launch_us=round(avg_s * 1e6, 2))

    cpu = None
    if args.cpu_sample > 0:
        cpu = cpu_baseline(inst, sols, args.cpu_sample, args.seed)

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
        "eval_pairs_ms_per_step": round(prof["eval_pairs"][1] / args.steps, 3),
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
