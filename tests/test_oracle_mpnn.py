"""Pins of the learned-initialiser oracle: finite-difference gradients (every parameter
tensor), the adjoint identity of the mean aggregation, a regular-graph closed form, labels
against a direct count, and a decreasing loss under Adam."""
import numpy as np
import pytest

import oracle
from oracle import mpnn
from paper_2509_18612_amd import synth


def small_batch():
    return synth.block_diagonal([synth.barabasi_albert(40, 2, 1), synth.erdos_renyi(30, 0.15, 2),
                                 synth.star(8), synth.edgeless(3)])


def test_mean_aggregate_adjoint():
    g = small_batch()
    rng = np.random.default_rng(0)
    H = rng.normal(size=(g.n, 5))
    G = rng.normal(size=(g.n, 5))
    lhs = np.sum(mpnn.mean_aggregate(g, H) * G)
    rhs = np.sum(H * mpnn.mean_aggregate_T(g, G))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_features_and_labels_by_hand():
    g = synth.star(5)  # centre 0 with 4 leaves
    f = mpnn.features(g)
    dbar = 8 / 5
    assert np.allclose(f[0], [4 / dbar, 1 / dbar, np.log(5) - np.log1p(dbar)])
    assert np.allclose(f[1], [1 / dbar, 4 / dbar, np.log(2) - np.log1p(dbar)])
    z = np.array([1, 0, 0, 1, 0])
    t = mpnn.labels(g, z)
    assert np.allclose(t, [3 / 4, 1, 1, 0, 1])
    # a best vector of the star cuts every edge: every label is 1
    best, zb = oracle.brute_force(g)
    assert np.allclose(mpnn.labels(g, zb), 1.0)


def test_regular_graph_closed_form():
    g = synth.random_regular3(40, 3)
    p = mpnn.init_params(1)
    y = mpnn.forward(g, p)
    q = {k: mpnn.bf16(v).astype(np.float64) for k, v in p.items()}
    h = np.array([1.0, 1.0, 0.0])  # d = m = dbar, log terms cancel
    for k in (1, 2, 3):
        h = np.maximum(h @ q[f"ws{k}"] + h @ q[f"wn{k}"] + q[f"b{k}"], 0.0)  # mean of equal rows
    want = 1 / (1 + np.exp(-(h @ q["wo"] + q["bo"][0])))
    assert np.allclose(y, want, rtol=1e-12)


def test_gradients_match_finite_differences():
    g = small_batch()
    p = mpnn.init_params(3)
    for k in p:  # non-zero biases so every path is exercised
        if k.startswith("b"):
            p[k] = np.random.default_rng(4).uniform(-0.2, 0.2, p[k].shape).astype(np.float32)
    t = np.random.default_rng(5).uniform(0, 1, g.n)
    L, grads = mpnn.loss_and_grads(g, p, t)
    # finite differences with respect to the bfloat16-rounded weights used by forward():
    # perturb in float64 through a forward that skips the rounding
    q = {k: mpnn.bf16(v).astype(np.float64) for k, v in p.items()}

    def loss64(qq):
        h = mpnn.features(g)
        for k in (1, 2, 3):
            a = mpnn.mean_aggregate(g, h)
            h = np.maximum(h @ qq[f"ws{k}"] + a @ qq[f"wn{k}"] + qq[f"b{k}"], 0.0)
        y = 1 / (1 + np.exp(-(h @ qq["wo"] + qq["bo"][0])))
        return np.mean((y - t) ** 2)

    assert loss64(q) == pytest.approx(L, rel=1e-12)
    rng = np.random.default_rng(6)
    eps = 1e-6
    for name, _ in mpnn.SHAPES:
        flat = q[name].reshape(-1)
        for idx in rng.choice(flat.size, min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + eps
            lp = loss64(q)
            flat[idx] = old - eps
            lm = loss64(q)
            flat[idx] = old
            fd = (lp - lm) / (2 * eps)
            an = grads[name].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (name, idx, fd, an)


def test_adam_decreases_loss():
    g = small_batch()
    best, z, _, _ = oracle.deco(synth.barabasi_albert(60, 3, 2), B=16, K=4, rounds=1, evo_rounds=0, Tq=40, Tl=20)
    t = np.random.default_rng(1).uniform(0.3, 1.0, g.n)
    p = mpnn.init_params(0)
    st = {}
    L0 = mpnn.loss_and_grads(g, p, t)[0]
    for _ in range(60):
        L, gr = mpnn.loss_and_grads(g, p, t)
        p = mpnn.adam(p, gr, st, lr=3e-3)
    assert mpnn.loss_and_grads(g, p, t)[0] < 0.7 * L0
