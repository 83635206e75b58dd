"""The allocation-free forward pass of the learned-start network (deco_mpnn_forward_static,
activations in the library's static scratch array) against the workspace variant
(deco_mpnn_forward) and the FP64 oracle: two calls in a row, the second on a smaller
graph, then the largest supported size and the first size past it."""
import numpy as np
import pytest

from oracle import mpnn as ompnn
from paper_2509_18612_amd import deco, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

MAX_NODES = 31_774  # 1,056 bytes per node in the 32 MiB scratch array


def params(seed):
    p = ompnn.init_params(seed)
    rng = np.random.default_rng(seed + 100)
    for k in p:
        if k.startswith("b"):
            p[k] = rng.uniform(-0.1, 0.1, p[k].shape).astype(np.float32)
    return p


def test_static_forward_equals_workspace_forward_on_two_calls():
    p = params(7)
    net = deco.Mpnn(deco.pack_mpnn(p))
    big = synth.block_diagonal([synth.barabasi_albert(600, 3, 1), synth.erdos_renyi(300, 0.03, 2), synth.star(9),
                                synth.edgeless(3)])
    small = synth.barabasi_albert(120, 2, 5)
    for g in (big, small):
        G = deco.Graph(g)
        print(f"static forward n={g.n} graphs={G.struct.num_graphs}", flush=True)
        ys = net.forward_static(G).cpu().numpy()
        yw = net.forward(G).cpu().numpy()
        assert np.array_equal(ys, yw)
        assert np.abs(ys.astype(np.float64) - ompnn.forward(g, p)).max() <= 2e-6


def test_static_forward_size_limit():
    p = params(8)
    net = deco.Mpnn(deco.pack_mpnn(p))
    g = synth.barabasi_albert(MAX_NODES, 2, 9)
    G = deco.Graph(g)
    print(f"static forward n={g.n} (largest supported)", flush=True)
    ys = net.forward_static(G).cpu().numpy()
    assert np.array_equal(ys, net.forward(G).cpu().numpy())
    over = deco.Graph(synth.edgeless(MAX_NODES + 1))
    with pytest.raises(deco.DecoError) as e:
        net.forward_static(over)
    assert e.value.status == deco.E_UNSUPPORTED
