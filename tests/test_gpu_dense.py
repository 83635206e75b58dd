"""GPU parity of the dense (bfloat16 MFMA) path against the CPU oracle.

The oracle steps the CSR form of the same graph; the dense path's float32 accumulation
order differs, so iterates are compared to one bfloat16 ulp of the oracle's emulation plus
the float32 summation bound; cuts of the GPU's own sign vectors are compared bit for bit.
"""
import numpy as np
import pytest

import oracle
from paper_2509_18612_amd import deco, synth

from gpu_util import bf16_ulp, oracle_cuts, step_bound, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)


def dense_bf16(g):
    W = np.zeros((g.n, g.n), np.float32)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr.astype(np.int64)))
    W[rows, g.col_idx] = 1.0 if g.w is None else g.w
    return torch.from_numpy(W).to(torch.bfloat16).cuda()


@pytest.mark.parametrize("n,p,B,weights", [(256, 0.5, 128, None), (384, 0.2, 256, "pm1"), (512, 0.05, 128, "int")])
def test_dense_teacher_forced_parity(n, p, B, weights):
    g = synth.erdos_renyi(n, p, n)
    if weights == "pm1":
        g = synth.with_rademacher_weights(g, 2)
    elif weights == "int":
        g = synth.with_weights(g, np.random.default_rng(1).integers(1, 4, g.nnz // 2).astype(np.float32))
    h = deco.DenseHandle(dense_bf16(g), B=B, eta=0.05, seed=3)
    h.start(deco.INIT_UNIFORM, batch=1)
    x0 = to_np(h.read_x()).astype(np.float64)
    assert np.array_equal(x0, oracle.to_bf16(oracle.init_uniform(n, B, 3, 1).astype(np.float32)).astype(np.float64))
    tr = h.set_trace(16)
    xs = [x0]
    for _ in range(12):
        h.step(1)
        xs.append(to_np(h.read_x()).astype(np.float64))
    h.round_score()
    trn = tr.cpu().numpy()
    best = np.full(B, -np.inf)
    bstep = np.full(B, -1)
    for t in range(13):
        cuts = oracle_cuts(g, xs[t], B, 1, False)[0][0]
        assert np.array_equal(trn[t][0], cuts), f"cut mismatch at step {t}"
        imp = cuts > best
        best[imp] = cuts[imp]
        bstep[imp] = t
        if t < 12:
            want = oracle.step(g, xs[t], 0.05)
            emu = oracle.to_bf16(want.astype(np.float32)).astype(np.float64)
            tol = bf16_ulp(emu) + step_bound(g, xs[t], np.full(B, 0.05), -0.5, oracle.CUT_FORM)
            assert np.all(np.abs(xs[t + 1] - emu) <= tol)
    bc, bs, bb = h.best()
    assert np.array_equal(bc[0], best) and np.array_equal(bs[0], bstep)
    assert np.array_equal(oracle.cut_batch(g, deco.bits_to_z(bb, B))[0], best)
    h.destroy()


def test_dense_and_sparse_paths_agree():
    g = synth.erdos_renyi(256, 0.3, 5)
    B = 128
    x0 = torch.from_numpy(synth.uniform_batch(g.n, B, 2)).to(torch.bfloat16).cuda()
    hd = deco.DenseHandle(dense_bf16(g), B=B, eta=0.1)
    hs = deco.Handle(deco.Graph(g), B=B, x_dtype=deco.BF16, eta=0.1)
    for h in (hd, hs):
        h.start(deco.INIT_USER, x0=x0)
    for _ in range(5):
        cd, bd = hd.round_score()
        cs, bs = hs.round_score()
        assert torch.equal(cd, cs) and torch.equal(bd, bs)
        xd = to_np(hd.read_x()).astype(np.float64)
        hd.step(1)
        hs.step(1)
        ad = to_np(hd.read_x()).astype(np.float64)
        as_ = to_np(hs.read_x()).astype(np.float64)
        tol = 2 * bf16_ulp(np.maximum(np.abs(ad), np.abs(as_))) + step_bound(g, xd, np.full(B, 0.1), -0.5, 0)
        assert np.all(np.abs(ad - as_) <= tol)
        hs.start(deco.INIT_USER, x0=torch.from_numpy(ad.astype(np.float32)).to(torch.bfloat16).cuda())
        hd.start(deco.INIT_USER, x0=torch.from_numpy(ad.astype(np.float32)).to(torch.bfloat16).cuda())
    hd.destroy()
    hs.destroy()


def test_dense_rejects_unsupported_and_invalid():
    W = torch.zeros((200, 200), dtype=torch.bfloat16, device="cuda")
    with pytest.raises(deco.DecoError) as e:
        deco.DenseHandle(W, B=128)
    assert e.value.status == deco.E_UNSUPPORTED
    W = torch.zeros((128, 128), dtype=torch.bfloat16, device="cuda")
    W[0, 1] = 1.0  # not symmetric
    with pytest.raises(deco.DecoError) as e:
        deco.DenseHandle(W, B=128)
    assert e.value.status == deco.E_INVAL
    W[1, 0] = 1.0
    W[5, 5] = 1.0  # diagonal
    with pytest.raises(deco.DecoError) as e:
        deco.DenseHandle(W, B=128)
    assert e.value.status == deco.E_INVAL


def test_dense_rejects_weights_without_an_exact_score():
    """The exact score needs integer weights whose |w| sums stay within 2^24 per row."""
    W = torch.zeros((128, 128), dtype=torch.bfloat16, device="cuda")
    W[0, 1] = W[1, 0] = 0.5
    with pytest.raises(deco.DecoError) as e:
        deco.DenseHandle(W, B=128)
    assert e.value.status == deco.E_UNSUPPORTED
    W = torch.full((128, 128), 2.0 ** 18, dtype=torch.bfloat16, device="cuda")
    W.fill_diagonal_(0.0)  # 127 x 2^18 > 2^24 per row
    with pytest.raises(deco.DecoError) as e:
        deco.DenseHandle(W, B=128)
    assert e.value.status == deco.E_UNSUPPORTED
    W = torch.full((128, 128), 2.0 ** 17, dtype=torch.bfloat16, device="cuda")
    W.fill_diagonal_(0.0)  # 127 x 2^17 < 2^24: accepted
    deco.DenseHandle(W, B=128).destroy()


def test_dense_er8192_large_integer_weights_exact_cuts():
    """ER(8192, 0.5) with integer weights of magnitude up to 2048 (k 2^j, k <= 8, exact in
    bfloat16; row sums of |w| about 4e6, within 2^24), B = 512 on the MFMA path: the cuts of 64
    sampled initialisations equal the oracle's eq. (1) cuts of the GPU's own sign vectors, bit
    for bit, at three iterates. Each column sum reaches ~1e10, far past float32's exact
    integers, so the double column sums are what keeps them exact."""
    g = synth.erdos_renyi(8192, 0.5, 0)
    rng = np.random.default_rng(4)
    m = g.nnz // 2
    w = (rng.integers(1, 9, m) * 2.0 ** rng.integers(0, 9, m) * rng.choice([-1.0, 1.0], m)).astype(np.float32)
    g = synth.with_weights(g, w)
    h = deco.DenseHandle(dense_bf16(g), B=512, eta=0.001, seed=1)
    h.start(deco.INIT_UNIFORM, batch=0)
    tr = h.set_trace(4)
    xs = [to_np(h.read_x())]
    for _ in range(2):
        h.step(1)
        xs.append(to_np(h.read_x()))
    h.round_score()
    cols = np.random.default_rng(3).choice(512, 64, replace=False)
    trn = tr.cpu().numpy()
    for t in range(3):
        z = oracle.round_signs(np.ascontiguousarray(xs[t][:, cols].astype(np.float64)), 64)
        assert np.array_equal(trn[t][0][cols], oracle.cut_batch(g, z)[0]), f"cut at step {t}"
    h.destroy()


def test_dense_er8192_half_B512_sampled():
    """ER(8192, 0.5), unit weights, B = 512 on the MFMA path: sampled rows against the oracle
    (star subgraphs) and exact cuts of 64 sampled initialisations, for two steps."""
    from test_gpu_full_size import check_rows
    g = synth.erdos_renyi(8192, 0.5, 0)
    h = deco.DenseHandle(dense_bf16(g), B=512, eta=0.01, seed=1)
    h.start(deco.INIT_UNIFORM, batch=0)
    tr = h.set_trace(4)
    xs = [to_np(h.read_x()).astype(np.float64)]
    for _ in range(2):
        h.step(1)
        xs.append(to_np(h.read_x()).astype(np.float64))
    rows = np.random.default_rng(2).integers(0, g.n, 64)
    cols = np.random.default_rng(3).choice(512, 64, replace=False)
    trn = tr.cpu().numpy()
    for t in range(2):
        check_rows(g, xs[t][:, cols], xs[t + 1][:, cols], rows, 0.01, deco.BF16)
        z = oracle.round_signs(np.ascontiguousarray(xs[t][:, cols]), 64)
        assert np.array_equal(trn[t][0][cols], oracle.cut_batch(g, z)[0])
    h.destroy()
