"""Pins of the learned-filter oracle (CPU): closed forms, finite differences,
hand-computed features. The paper has no learned component; these pin the
filter's own definition."""
import math
import struct

import numpy as np
import pytest

import oracle
from oracle import Ref
from paper_2605_05208_amd import gen
from paper_2605_05208_amd.gen import Instance, Solution

H, F = 256, 32
P_W1, P_B1 = 0, H * F
P_W2 = P_B1 + H
P_B2 = P_W2 + H * H
P_W3 = P_B2 + H
P_B3 = P_W3 + H


def bf16_bits(x):
    return oracle.bf16([x])[0]


def f32_of_bits(b):
    return struct.unpack("<f", struct.pack("<I", int(b) << 16))[0]


def test_bf16_rounding_cases():
    assert bf16_bits(1.0) == 0x3F80
    assert bf16_bits(-2.0) == 0xC000
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties to even -> 1.0
    assert bf16_bits(1.0 + 2 ** -8) == 0x3F80
    # 1 + 3*2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6: ties to even -> 1 + 2^-6
    assert f32_of_bits(bf16_bits(1.0 + 3 * 2 ** -8)) == 1.0 + 2 ** -6
    # just above halfway rounds up
    assert f32_of_bits(bf16_bits(1.0 + 2 ** -8 + 2 ** -20)) == 1.0 + 2 ** -7
    for v in (0.0, 3.0, -0.5, 1024.0, 2.0 ** -100):
        assert f32_of_bits(bf16_bits(v)) == v


def _params_hand():
    P = np.zeros(oracle.N_PARAMS, np.float32)
    P[P_W1 + 0 * F + 0] = 1.0   # h1[0] = relu(x0)
    P[P_W1 + 1 * F + 1] = 1.0   # h1[1] = relu(x1)
    P[P_W2 + 0 * H + 0] = 1.0   # h2[0] = relu(h1[0])
    P[P_W2 + 1 * H + 1] = 2.0   # h2[1] = relu(2 h1[1])
    P[P_W3 + 0] = 1.0
    P[P_W3 + 1] = 1.0
    P[P_B3] = -0.5
    return P


def test_forward_closed_form():
    """logit = x0 + 2 x1 - 0.5 for x0, x1 > 0; negative parts cut by ReLU."""
    P = _params_hand()
    x = np.zeros((3, F), np.uint16)
    x[0, 0], x[0, 1] = bf16_bits(1.5), bf16_bits(0.25)
    x[1, 0], x[1, 1] = bf16_bits(-3.0), bf16_bits(2.0)
    x[2, 0], x[2, 1] = bf16_bits(0.0), bf16_bits(-1.0)
    z = oracle.mlp_forward(P, x, round_act=1)
    assert z.tolist() == [1.5 + 0.5 - 0.5, 0 + 4.0 - 0.5, -0.5]
    z0 = oracle.mlp_forward(P, x, round_act=0)
    assert np.allclose(z0, z)


def test_bce_closed_form():
    assert math.isclose(oracle.bce([0.0], [1.0]), math.log(2), rel_tol=1e-12)
    assert math.isclose(oracle.bce([0.0, 0.0], [0.0, 1.0]), math.log(2), rel_tol=1e-12)
    z = 3.0
    assert math.isclose(oracle.bce([z], [0.0]), math.log1p(math.exp(z)), rel_tol=1e-12)
    assert math.isclose(oracle.bce([z], [1.0]), math.log1p(math.exp(-z)), rel_tol=1e-12)
    # weights: only the weighted sample counts
    assert math.isclose(oracle.bce([z, 0.0], [1.0, 1.0], [1.0, 0.0]), math.log1p(math.exp(-z)), rel_tol=1e-12)


def test_adam_first_step_closed_form():
    P = np.ones(5, np.float32)
    m = np.zeros(5, np.float32)
    v = np.zeros(5, np.float32)
    g = np.array([0.5, -2.0, 1e-3, 0.0, 7.0], np.float32)
    oracle.adam(P, m, v, g, 0.01, 1)
    # bias-corrected first step: theta -= lr * g / (|g| + eps)
    exp = 1.0 - 0.01 * g / (np.abs(g) + 1e-8)
    assert np.allclose(P, exp, rtol=0, atol=1e-6)


def _random_params(seed, scale=0.2):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(oracle.N_PARAMS) * scale).astype(np.float32)


def _random_x(seed, n):
    rng = np.random.default_rng(seed)
    return oracle.bf16(rng.standard_normal(n * F)).reshape(n, F)


def test_backward_matches_central_differences():
    """The fp64 backward of the smooth network matches central finite differences."""
    P = _random_params(1)
    x = _random_x(2, 6)
    y = np.array([1, 0, 1, 1, 0, 0], np.float32)

    def loss(p):
        return oracle.bce(oracle.mlp_forward(p.astype(np.float32), x, round_act=0), y)

    z = oracle.mlp_forward(P, x, round_act=0)
    dl = (1 / (1 + np.exp(-z)) - y) / len(y)
    g = oracle.mlp_backward(P, x, dl, round_act=0)
    rng = np.random.default_rng(3)
    idx = np.concatenate([rng.choice(np.arange(P_W1, P_B1), 40, replace=False),
                          rng.choice(np.arange(P_B1, P_W2), 20, replace=False),
                          rng.choice(np.arange(P_W2, P_B2), 60, replace=False),
                          rng.choice(np.arange(P_B2, P_W3), 20, replace=False),
                          rng.choice(np.arange(P_W3, P_B3), 20, replace=False), [P_B3]])
    num, den = 0.0, 0.0
    for i in idx:
        h = 1e-3 * max(1.0, abs(float(P[i])))
        # central difference in fp64 on a parameter copy held in fp64 via two fp32 evaluations
        Pp = P.astype(np.float64).copy()
        Pm = P.astype(np.float64).copy()
        Pp[i] += h
        Pm[i] -= h
        # the oracle takes fp32 parameters: step sizes are exact in fp32 here
        fd = (loss(Pp) - loss(Pm)) / ((np.float32(Pp[i]) - np.float32(Pm[i])))
        num += (fd - g[i]) ** 2
        den += g[i] ** 2
    assert math.sqrt(num / den) <= 1e-4


def test_topk_matches_stable_sort():
    rng = np.random.default_rng(5)
    nc, th, k = 30, 12, 5
    nbr = rng.permuted(np.tile(np.arange(100, 100 + th), (nc, 1)), axis=1).astype(np.int32)
    ln = rng.integers(3, th + 1, nc).astype(np.int32)
    score = rng.integers(-3, 3, (nc, th)).astype(np.float32)  # many ties
    out = oracle.topk(nbr.ravel(), ln, nc, th, score.ravel(), k)
    for i in range(nc):
        cand = sorted(range(ln[i]), key=lambda q: (-score[i, q], nbr[i, q]))[:k]
        exp = [int(nbr[i, q]) for q in cand] + [-1] * (k - len(cand))
        assert out[i].tolist() == exp


def test_features_hand_example():
    """Depot 0 at (0,0); customers 1 (3,4), 2 (6,8), 3 (0,5) at scale 10; routes (0,1,2,0) and (0,3,0).
    Anchor u = 1, v = 3 (other route): every integer feature by hand."""
    xy = np.array([(0, 0), (3, 4), (6, 8), (0, 5)], np.int64)
    d = xy[:, None, :] - xy[None, :, :]
    c = np.floor(np.sqrt((d * d).sum(-1)) * 10 + 0.5).astype(np.int32)
    n = 4
    I = Instance(n_depots=1, n_customers=3, c=c, t=c, q=np.array([0, 5, 7, 4], np.int32), s=np.zeros(n, np.int32),
                 e=np.zeros(n, np.int32), l=np.full(n, gen.BIG_HORIZON, np.int32), Q=10, NV=2, Dmax=-1,
                 open_routes=0, has_tw=0, theta=2, w_load=10)
    ref = Ref(I)
    nbr, ln = ref.neighbours()
    sol = Solution([(0, [1, 2], 0), (0, [3], 0)])
    fx = ref.features(sol)
    # N(1) by distance: c(1,3) = round(10*sqrt(9+1)) = 32, c(1,2) = 50 -> [3, 2]
    assert list(nbr[0:2]) == [3, 2]
    row = fx[0]  # u = 1, k = 0 -> v = 3
    # nearest-neighbour distances: c(1,3)=32, c(2,1)=50, c(3,1)=32 -> mean 114 // 3 = 38
    dscale = np.float32(1.0) / np.float32(38)
    vals = [f32_of_bits(b) for b in row]

    def S(iv, r):
        return f32_of_bits(bf16_bits(float(np.float32(iv) * r)))

    c01, c12, c20, c03, c13, c23 = 50, 50, 100, 50, 32, 67
    assert c[0, 1] == c01 and c[1, 2] == c12 and c[2, 0] == c20 and c[0, 3] == c03 and c[1, 3] == c13
    ints = {0: c13, 1: c01, 2: c12, 3: c[0, 2], 4: c03, 5: c[0, 1],
            6: c[0, 2] - c01 - c12 + c[0, 1] + c13 - c03,
            7: c13 + c[0, 2] - c12 - c03,
            8: c[0, 0] + c[0, 2] + c[0, 1] + c13 - c01 - c12 - c[0, 0] - c03}
    for f, iv in ints.items():
        assert vals[f] == S(iv, dscale), f
    rq = np.float32(1.0) / np.float32(10)
    assert vals[9] == S(12 - 10, rq) and vals[10] == S(4 - 10, rq)
    assert vals[11] == S(5, rq) and vals[12] == S(4, rq)
    assert all(vals[f] == 0.0 for f in range(13, 23))
    assert vals[23] == 0.0 and vals[24] == 1.0 and vals[25] == 0.0 and vals[26] == 0.0
    assert vals[27] == S(2, np.float32(1 / 32)) and vals[28] == S(1, np.float32(1 / 32))
    assert vals[29] == S(1, np.float32(1) / np.float32(2)) and vals[30] == 1.0 and vals[31] == 0.0


def test_adam_second_step_by_hand():
    """Two Adam steps on one parameter (beta 0.9 / 0.999, eps 1e-8, lr 0.1), gradients 0.5 then
    -0.25. Step 1: m = 0.05, v = 2.5e-4, m^ = 0.5, v^ = 0.25, theta = 1 - 0.1 * 0.5 / 0.5 = 0.9.
    Step 2: m = 0.9 * 0.05 - 0.1 * 0.25 = 0.02, v = 0.999 * 2.5e-4 + 0.001 * 0.0625 = 3.1225e-4,
    m^ = 0.02 / 0.19, v^ = 3.1225e-4 / 0.001999, theta = 0.9 - 0.1 * m^ / sqrt(v^) = 0.8733663.
    (Swapped betas would give 0.8679139; no bias correction 0.7868.)"""
    P = np.ones(1, np.float32)
    m = np.zeros(1, np.float32)
    v = np.zeros(1, np.float32)
    oracle.adam(P, m, v, np.array([0.5], np.float32), 0.1, 1)
    assert abs(float(P[0]) - 0.9) <= 1e-6
    oracle.adam(P, m, v, np.array([-0.25], np.float32), 0.1, 2)
    assert abs(float(m[0]) - 0.02) <= 1e-8 and abs(float(v[0]) - 3.1225e-4) <= 1e-10
    assert abs(float(P[0]) - 0.8733663) <= 1e-6
