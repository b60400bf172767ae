"""The allocation-free training step (mdvrp_mlp_train_step_static) against the
workspace form (mdvrp_mlp_train_step): the same kernels in the same fixed
reduction order, so logits, loss, gradients and the updated parameters must be
bit-identical, on two calls in a row (the second with fewer samples, so stale
scratch from the first call must not leak into it), plus the size limit."""
import numpy as np
import pytest

import oracle
from paper_2605_05208_amd import mdvrp

pytestmark = pytest.mark.gpu

H, F = 256, 32


def _params(seed):
    rng = np.random.default_rng(seed)
    P = np.zeros(oracle.N_PARAMS, np.float32)
    P[:H * F] = rng.standard_normal(H * F) * np.sqrt(2.0 / F)
    P[H * F:H * F + H] = rng.standard_normal(H) * 0.1
    o = H * F + H
    P[o:o + H * H] = rng.standard_normal(H * H) * np.sqrt(2.0 / H)
    P[o + H * H:o + H * H + H] = rng.standard_normal(H) * 0.1
    P[o + H * H + H:o + H * H + 2 * H] = rng.standard_normal(H) * np.sqrt(1.0 / H) * 0.2
    P[-1] = 0.05
    return P


def _batch(t, n, seed):
    rng = np.random.default_rng(seed)
    x = oracle.bf16(rng.standard_normal(n * F)).reshape(n, F)
    y = (rng.random(n) < 0.3).astype(np.float32)
    w = np.where(y > 0, 2.0, 1.0).astype(np.float32)
    return tuple(t.from_numpy(a).to("cuda") for a in (x.view(np.int16), y, w))


def test_static_train_step_equals_workspace_form():
    import torch as t
    P = _params(21)
    A = mdvrp.Mlp(P)   # workspace form
    B = mdvrp.Mlp(P)   # allocation-free form
    print("static train step: n = 4096 then 1500", flush=True)
    for step, (n, seed, w_on) in enumerate([(4096, 1, True), (1500, 2, False)], start=1):
        xd, yd, wd = _batch(t, n, seed)
        w = wd if w_on else None
        za, la, ga = A.train_step(xd, yd, w, 2e-3, step)
        zb, lb, gb = B.train_step_static(xd, yd, w, 2e-3, step)
        t.cuda.synchronize()
        assert t.equal(za, zb), step
        assert t.equal(la, lb), step
        assert t.equal(ga, gb), step
        assert np.array_equal(A.get_params(), B.get_params()), step
        assert np.isfinite(float(lb.cpu().numpy()[0]))


def test_static_train_step_rejects_more_samples_than_its_limit():
    import torch as t
    M = mdvrp.Mlp(_params(22))
    n = mdvrp.TRAIN_STATIC_MAX_N + 1
    xd, yd, wd = _batch(t, n, 3)
    with pytest.raises(mdvrp.MdvrpError) as e:
        M.train_step_static(xd, yd, wd, 1e-3, 1)
    assert e.value.status == mdvrp.EINVAL
