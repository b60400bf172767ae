"""Training data and training loop of the learned move filter.

The logs come from the method itself: full-list local searches are run in
chunks of a few passes; after each chunk the features of every anchor
(u, v in N(u)) of the current solutions and its label (some pair move anchored
at (u, v) improves F) are taken from the library (`mdvrp_filter_features`,
`mdvrp_filter_labels`). Positives are all kept; negatives are sub-sampled to
about `neg_ratio` per positive and weighted by the inverse of their keep rate,
so the weighted loss is the loss over all anchors. Training runs the library's
BF16-MFMA forward / backward kernels and Adam (`mdvrp_mlp_train_step`).

Device tensors come from PyTorch (memory only); every feature, label,
forward, backward and optimiser step runs in the library's kernels.
"""
from __future__ import annotations

import time

import numpy as np

from . import gen, mdvrp


def _torch():
    import torch
    return torch


def valid_anchors(batch: mdvrp.Batch):
    """Device bool mask over the batch's anchors: list entry k < nbr_len of its customer."""
    torch = _torch()
    parts = []
    for k in batch.unit_inst:
        inst = batch.instances[k]
        _, ln = inst.lists()
        th = inst.inst.theta
        parts.append(np.arange(th)[None, :] < ln[:, None])
    return torch.from_numpy(np.concatenate([p.ravel() for p in parts])).to("cuda")


def log_states(batch: mdvrp.Batch, solutions, seed=1, chunk=2, max_chunks=40, neg_ratio=4.0, rng_seed=0,
               max_samples=None, pos_budget=None, search=None):
    """Run the full-list local search of `solutions` in chunks of `chunk` passes and log
    (features, label, weight) of sub-sampled anchors after every chunk (the start state
    included). With pos_budget, at most that many positives are kept per snapshot, with
    weight 1, so that the early states, where most anchors improve, do not dominate the
    logs; negatives are weighted by the inverse of their keep rate, which restores each
    snapshot's ratio of negatives to kept positives. `search` (keyword arguments of the
    local search) selects the trajectory, e.g. a filtered search; the labels always
    come from the full lists. Returns device tensors x [n][32] (int16 bf16 bits), y [n],
    w [n] and the number of snapshots."""
    torch = _torch()
    g = torch.Generator(device="cuda")
    g.manual_seed(rng_seed)
    valid = valid_anchors(batch)
    batch.load(solutions)
    xs, ys, ws = [], [], []
    total = 0
    snaps = 0
    for c in range(max_chunks + 1):
        feats = batch.features(as_numpy=False)
        lab = batch.labels(as_numpy=False)
        pos = valid & (lab == 1)
        neg = valid & (lab == 0)
        n_pos, n_neg = int(pos.sum()), int(neg.sum())
        pp = 1.0 if not pos_budget or n_pos <= pos_budget else pos_budget / n_pos
        kept_pos = n_pos * pp
        p = 1.0 if n_neg == 0 else min(1.0, neg_ratio * max(kept_pos, 1) / n_neg)
        r = torch.rand(neg.shape, device="cuda", generator=g)
        keep = (pos & (r < pp)) | (neg & (r < p))
        idx = torch.nonzero(keep).squeeze(1)
        xs.append(feats[idx])
        ys.append(lab[idx].float())
        ws.append(torch.where(pos[idx], torch.ones_like(idx, dtype=torch.float32),
                              torch.full_like(idx, pp / p, dtype=torch.float32)))
        total += len(idx)
        snaps += 1
        if max_samples and total >= max_samples:
            break
        st = batch.local_search_to_optimum(seed=seed + c, max_passes=chunk, **(search or {}))
        if all(s["converged"] for s in st) or n_pos == 0:
            break
    return torch.cat(xs), torch.cat(ys), torch.cat(ws), snaps


def train(mlp: mdvrp.Mlp, x, y, w, epochs=4, batch_size=65536, lr=1e-3, seed=0, log=None):
    """Mini-batch Adam on the library's train step; returns per-epoch mean losses and seconds."""
    torch = _torch()
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    n = x.shape[0]
    step = getattr(mlp, "_adam_step", 0)
    losses = []
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.randperm(n, device="cuda", generator=g)
        acc = torch.zeros(1, dtype=torch.float32, device="cuda")
        nb = 0
        for a in range(0, n - batch_size // 4, batch_size):
            idx = perm[a:a + batch_size]
            step += 1
            _, loss, _ = mlp.train_step(x[idx].contiguous(), y[idx].contiguous(), w[idx].contiguous(), lr, step)
            acc += loss
            nb += 1
        losses.append(float(acc.item()) / max(nb, 1))
        if log:
            log(f"epoch {ep}: loss {losses[-1]:.4f}")
    torch.cuda.synchronize()
    mlp._adam_step = step
    return losses, time.perf_counter() - t0


def recall_at_k(batch: mdvrp.Batch, mlp: mdvrp.Mlp | None, k: int):
    """Share of the improving anchors of the batch's current solutions that fall in the
    k-entry lists (network ranking when mlp is given, else the first k of each list)."""
    torch = _torch()
    lab = batch.labels(as_numpy=False).bool()
    if mlp is not None:
        batch.score_topk(mlp, want_logits=False)
    else:
        batch.eta_lists()
    lists = batch.filter_lists()
    hit, tot = 0, 0
    at = 0
    for u, kk in enumerate(batch.unit_inst):
        inst = batch.instances[kk]
        nbr, ln = inst.lists()
        th = inst.inst.theta
        nc = inst.inst.n_customers
        lu = lab[at:at + nc * th].cpu().numpy().reshape(nc, th)
        at += nc * th
        rows = nbr.reshape(nc, th)
        good = [set(rows[i, :ln[i]][lu[i, :ln[i]]].tolist()) for i in range(nc)]
        tot += sum(len(s) for s in good)
        hit += sum(len(good[i] & set(lists[u][i].tolist())) for i in range(nc))
    return hit / max(tot, 1), tot


def init_params(seed=0):
    """He-initialised hidden layers, zero biases, a small output layer."""
    rng = np.random.default_rng(seed)
    H, F = 256, 32
    P = np.zeros(mdvrp.MLP_PARAMS, np.float32)
    P[0:H * F] = rng.standard_normal(H * F) * np.sqrt(2.0 / F)
    w2 = H * F + H
    P[w2:w2 + H * H] = rng.standard_normal(H * H) * np.sqrt(2.0 / H)
    w3 = w2 + H * H + H
    P[w3:w3 + H] = rng.standard_normal(H) * np.sqrt(1.0 / H)
    return P


def training_instances(n_config4=8):
    """Instances whose full runs provide the logs: config 2 and a spread of config-4 sizes."""
    insts = [gen.config2()]
    insts += [gen.config4_instance(i) for i in range(n_config4)]
    return insts
