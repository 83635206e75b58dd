"""GPU kernels of the learned starting-magnitude network against the FP64 oracle, its
training on the GPU, and the measured effect of the learned start (steps to a target cut
against the importance-based start, paired by seed: reported, parity unpinned)."""
import numpy as np
import pytest

import oracle
from oracle import mpnn as ompnn
from paper_2509_18612_amd import deco, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)


def batch():
    return synth.block_diagonal([synth.barabasi_albert(300, 3, 1), synth.erdos_renyi(200, 0.03, 2),
                                 synth.star(12), synth.edgeless(4), synth.barabasi_albert(500, 2, 3)])


def random_params(seed):
    p = ompnn.init_params(seed)
    rng = np.random.default_rng(seed + 100)
    for k in p:
        if k.startswith("b"):
            p[k] = rng.uniform(-0.1, 0.1, p[k].shape).astype(np.float32)
    return p


def test_forward_matches_oracle():
    g = batch()
    p = random_params(1)
    net = deco.Mpnn(deco.pack_mpnn(p))
    y = net.forward(deco.Graph(g)).cpu().numpy().astype(np.float64)
    want = ompnn.forward(g, p)
    assert np.abs(y - want).max() <= 2e-6


def test_loss_and_gradients_match_oracle():
    g = batch()
    p = random_params(2)
    t = np.random.default_rng(3).uniform(0, 1, g.n)
    net = deco.Mpnn(deco.pack_mpnn(p))
    L = net.loss_grad(deco.Graph(g), torch.from_numpy(t.astype(np.float32)).cuda())
    Lw, gw = ompnn.loss_and_grads(g, p, t.astype(np.float32).astype(np.float64))
    assert L == pytest.approx(Lw, rel=1e-5)
    got = deco.unpack_mpnn(net.grads.cpu().numpy())
    for k, v in gw.items():
        a, b = got[k].reshape(-1), np.asarray(v, np.float64).reshape(-1)
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        cos = a @ b / max(np.linalg.norm(a) * np.linalg.norm(b), 1e-30)
        assert rel < 1e-3 and cos > 0.99999, (k, rel, cos)


def test_labels_match_oracle():
    g = synth.with_rademacher_weights(synth.erdos_renyi(300, 0.05, 4), 5)
    g = synth.with_weights(g, np.abs(g.w[g.col_idx > np.repeat(np.arange(g.n), np.diff(g.row_ptr))]) + 1)
    z = np.random.default_rng(1).integers(0, 2, g.n).astype(np.uint8)
    net = deco.Mpnn()
    t = net.labels(deco.Graph(g), z).cpu().numpy()
    assert np.allclose(t, ompnn.labels(g, z), atol=1e-7)


def test_adam_matches_oracle_step():
    g = batch()
    p = random_params(5)
    t = np.random.default_rng(6).uniform(0, 1, g.n).astype(np.float32)
    net = deco.Mpnn(deco.pack_mpnn(p))
    G = deco.Graph(g)
    tt = torch.from_numpy(t).cuda()
    st = {}
    q = p
    for _ in range(3):
        net.loss_grad(G, tt)
        net.adam(lr=1e-2)
        _, gr = ompnn.loss_and_grads(g, q, t.astype(np.float64))
        q = ompnn.adam(q, gr, st, lr=1e-2)
    got = net.params.cpu().numpy()
    assert np.abs(got - deco.pack_mpnn(q)).max() <= 1e-4


def train(net, graphs, steps, lr=3e-3):
    losses = []
    for it in range(steps):
        G, t = graphs[it % len(graphs)]
        losses.append(net.loss_grad(G, t))
        net.adam(lr)
    return losses


def test_training_on_deco_labels_decreases_loss_and_learned_start():
    rng = np.random.default_rng(0)
    graphs = []
    for i in range(6):
        parts = [synth.barabasi_albert(int(rng.integers(500, 2000)), int(rng.integers(2, 7)), 100 + 4 * i + j)
                 for j in range(4)]
        bd = synth.block_diagonal(parts)
        G = deco.Graph(bd)
        r = deco.solve(G, B=64, K=8, l_max=2, rounds=2, evo_rounds=1, T_q=300, T_l=100, seed=i)
        net0 = deco.Mpnn()
        graphs.append((G, net0.labels(G, r["z"])))
    net = deco.Mpnn(deco.pack_mpnn(ompnn.init_params(0)))
    losses = train(net, graphs, 240)
    first, last = np.mean(losses[:12]), np.mean(losses[-12:])
    print(f"training loss {first:.4f} -> {last:.4f}")
    assert last < first
    # the learned start: mean = y_v * IDI sign, here without noise and scale 1
    g = synth.barabasi_albert(3000, 4, 77)
    G = deco.Graph(g)
    y = net.forward(G)
    h = deco.Handle(G, B=32, seed=9)
    h.start(deco.INIT_LEARNED, magnitude=y, scale=1.0, sigma2=0.0, batch=2)
    x = h.read_x().cpu().numpy().astype(np.float64)
    want = oracle.init_idi(g, 32, 9, 2) * y.cpu().numpy().astype(np.float64)[:, None]
    assert np.abs(x - want).max() <= 1e-7
    h.destroy()


def test_learned_start_gain_steps_to_target():
    """The learned-start protocol of paper_2509_18612_amd.learned at a test's size: train on DECO
    labels of 40 BA graphs, evaluate 8 held-out BA(5000) graphs (paired seeds, steps of the
    unlifted batch to 0.995 of the best of a long unlifted batch). The full-size protocol
    (2,000 training graphs, 200 BA(20000) + 200 ER(5000, 0.002) graphs) measured no gain over
    the importance-based start (paper_2509_18612_amd/data/mpnn_ba_report.json), so the
    criterion asserted here is non-regression: on average the learned start needs at most 10%
    more steps than IDI, and both reach the target on every graph. Parity unpinned (no closed
    form or published number for the gain)."""
    from paper_2509_18612_amd import learned
    graphs = [synth.barabasi_albert(n, m, 700 + i) for i, (n, m, _) in enumerate(learned.training_specs(40, 3))]
    batches = learned.label_batches(graphs, 10, seed=11)
    net = deco.Mpnn(learned.glorot_params(3))
    losses = learned.train(net, batches, 5, 2e-3, log=lambda _: None)
    assert losses[-1] < losses[0]
    rng = np.random.default_rng(4)
    held = [synth.barabasi_albert(5000, int(rng.integers(2, 7)), 9000 + k) for k in range(8)]
    rows = learned.evaluate(net, held, 8, 128, 600, 10 ** -1.5, 77, log=lambda _: None)
    summ = learned.summarise(rows, 600)
    b = summ["batch"]
    print("learned start, 8 BA(5000):", b)
    assert b["learned_fewer"] + b["learned_more"] + b["ties"] == b["graphs"] == 8
    assert b["reached_idi"] == 8 and b["reached_learned"] == 8
    assert b["steps_saved_when_both_reach"]["mean"] >= -0.1 * b["median_steps_idi"]
