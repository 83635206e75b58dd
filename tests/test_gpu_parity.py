"""GPU parity of the fused step kernel against the CPU oracle (through the C ABI).

Floating point: teacher forcing. For every step t the oracle's FP64 step from the GPU's
own X_t must agree with the GPU's X_{t+1} to 1e-5 (the per-step bound for float32
iterates), or to the float32 summation bound where a high-degree row makes that larger
(Higham's gamma_k bound, reported). Cuts: the GPU's cut of its own sign vector equals
the oracle's eq. (1) cut of that vector bit for bit. Running best: equal to the oracle's
bookkeeping over the GPU's cut sequence. BF16 storage: within one bfloat16 ulp of the
oracle's emulation (exact step, rounded to float32 then to bfloat16).
"""
import numpy as np
import pytest

import oracle
from paper_2509_18612_amd import deco, synth

from gpu_util import U32, bf16_ulp, oracle_cuts, run_teacher_forced, step_bound, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)


def cw_of(form):
    return -0.5 if form == deco.GRAD_CUT else -1.0


def check_run(g, B, steps, l=1, lifted=False, form=deco.GRAD_CUT, dtype=deco.F32, eta=0.1, x0=None, seed=3,
              schedule_tune=False, eta_per_init=None, schedule=None, l_active=None):
    r = run_teacher_forced(g, B, steps, l, lifted, form, dtype, eta, x0, seed, schedule_tune, eta_per_init,
                           schedule=schedule, l_active=l_active)
    xs = r["xs"]
    C = l * B
    eta_cols = (np.full(C, eta) if eta_per_init is None
                else np.tile(np.asarray(eta_per_init, np.float32).astype(np.float64), l))
    worst = 0.0
    widened = 0
    G = 1 if g.graph_row_offset is None else len(g.graph_row_offset) - 1
    gbest = np.full((G, B), -np.inf)
    gstep = np.full((G, B), -1)
    for t in range(steps + 1):
        cuts, z = oracle_cuts(g, xs[t], B, l, lifted)
        # exact cut of the GPU's own sign vector, per graph and initialisation
        assert np.array_equal(r["trace"][t], cuts), f"cut mismatch at step {t}"
        imp = cuts > gbest
        gbest[imp] = cuts[imp]
        gstep[imp] = t
        if t == steps:
            break
        want = oracle.step(g, xs[t], eta_cols, form)
        if dtype == deco.BF16:
            emu = oracle.to_bf16(want.astype(np.float32)).astype(np.float64)
            tol = bf16_ulp(emu) + step_bound(g, xs[t], eta_cols, cw_of(form), form)
            diff = np.abs(xs[t + 1] - emu)
        else:
            bound = step_bound(g, xs[t], eta_cols, cw_of(form), form)
            tol = np.maximum(1e-5, bound)
            widened += int((bound > 1e-5).sum())
            diff = np.abs(xs[t + 1] - want)
        worst = max(worst, float(diff.max()))
        bad = diff > tol
        assert not bad.any(), f"step {t}: {bad.sum()} elements off, max {diff.max():.3e}"
    # final iterate scored by round_score, then the running best
    assert np.array_equal(r["cut_T"], oracle_cuts(g, xs[steps], B, l, lifted)[0])
    bc, bs, bb = r["best"]
    assert np.array_equal(bc, gbest)
    assert np.array_equal(bs, gstep)
    zb = deco.bits_to_z(bb, B)
    for gi in range(G):
        for b in range(B):
            zt = oracle.round_signs(xs[gstep[gi, b]], B, l, lifted)
            r0 = 0 if g.graph_row_offset is None else g.graph_row_offset[gi]
            r1 = g.n if g.graph_row_offset is None else g.graph_row_offset[gi + 1]
            assert np.array_equal(zb[r0:r1, b], zt[r0:r1, b])
    # the best vector's cut, recomputed from its bits
    assert np.array_equal(oracle.cut_batch(g, zb), bc)
    r["handle"].destroy()
    return worst, widened, r["schedule"]


CASES = {
    "er_unit_B16": (lambda: synth.erdos_renyi(500, 0.05, 1), 16, {}),
    "ba_hubs_B64": (lambda: synth.barabasi_albert(600, 3, 2), 64, {}),
    "er_pm1_B24_tiles": (lambda: synth.with_rademacher_weights(synth.erdos_renyi(400, 0.1, 3), 4), 24, {}),
    "laplacian_B16": (lambda: synth.erdos_renyi(400, 0.05, 6), 16, dict(form=deco.GRAD_LAPLACIAN, eta=0.01)),
    "lifted_l2_B16": (lambda: synth.erdos_renyi(400, 0.06, 7), 16, dict(l=2, lifted=True)),
    "lifted_l3_B8": (lambda: synth.barabasi_albert(300, 4, 8), 8, dict(l=3, lifted=True)),
    "lifted_l4_B32": (lambda: synth.erdos_renyi(300, 0.05, 9), 32, dict(l=4, lifted=True)),
    "lifted_l5_B8": (lambda: synth.barabasi_albert(300, 4, 16), 8, dict(l=5, lifted=True)),
    "lifted_l6_B24": (lambda: synth.erdos_renyi(250, 0.06, 18), 24, dict(l=6, lifted=True)),
    "lifted_l7_B2": (lambda: synth.barabasi_albert(250, 3, 19), 2, dict(l=7, lifted=True)),
    "lifted_l8_B16": (lambda: synth.erdos_renyi(300, 0.05, 17), 16, dict(l=8, lifted=True)),
    # members with fewer active components than l (their other components are exactly 0 and
    # are not gathered); the active count changes inside a lane's initialisations
    "lifted_l4_active_B32": (lambda: synth.barabasi_albert(400, 3, 20), 32,
                             dict(l=4, lifted=True, l_active=np.array([1 + (b // 3) % 4 for b in range(32)],
                                                                      np.int32))),
    "lifted_l8_active_B16": (lambda: synth.erdos_renyi(300, 0.05, 21), 16,
                             dict(l=8, lifted=True, l_active=np.array([1 + (5 * b) % 8 for b in range(16)],
                                                                      np.int32))),
    # more than 8 components: iterates as an unlifted batch over the l B columns, scores from
    # the float32 component sums
    "lifted_l12_B8": (lambda: synth.barabasi_albert(300, 3, 22), 8, dict(l=12, lifted=True)),
    "lifted_l16_active_B16": (lambda: synth.erdos_renyi(250, 0.06, 23), 16,
                              dict(l=16, lifted=True, l_active=np.array([1 + (7 * b) % 16 for b in range(16)],
                                                                        np.int32))),
    # l = n (the largest lift of Table 2)
    "lifted_l_eq_n_B8": (lambda: synth.erdos_renyi(48, 0.2, 24), 8, dict(l=48, lifted=True)),
    "B1": (lambda: synth.erdos_renyi(200, 0.05, 10), 1, {}),
    "B2": (lambda: synth.erdos_renyi(200, 0.05, 11), 2, {}),
    "B4_lifted": (lambda: synth.erdos_renyi(200, 0.05, 12), 4, dict(l=2, lifted=True)),
    "B256_wide": (lambda: synth.barabasi_albert(400, 4, 13), 256, {}),
    "unlifted_as_l1_lifted": (lambda: synth.erdos_renyi(300, 0.05, 14), 16, dict(l=1, lifted=True)),
    "per_init_eta": (lambda: synth.erdos_renyi(300, 0.06, 15), 16,
                     dict(eta_per_init=np.geomspace(1e-3, 0.3, 16).astype(np.float32))),
}


def _intw_graph():
    g = synth.erdos_renyi(300, 0.08, 5)
    m = g.nnz // 2
    return synth.with_weights(g, np.random.default_rng(1).integers(1, 5, m).astype(np.float32))


CASES["er_intw_B8"] = (_intw_graph, 8, {})


def _realw_graph():
    g = synth.erdos_renyi(300, 0.06, 25)
    m = g.nnz // 2
    return synth.with_weights(g, np.random.default_rng(4).uniform(0.1, 2.0, m).astype(np.float32))


# lifted rows under the other weight modes (float32 runs them 2 values per lane)
CASES["lifted_l3_pm1_B16"] = (lambda: synth.with_rademacher_weights(synth.erdos_renyi(350, 0.06, 26), 6), 16,
                              dict(l=3, lifted=True))
CASES["lifted_l2_intw_B32"] = (_intw_graph, 32, dict(l=2, lifted=True))


@pytest.mark.parametrize("name", sorted(CASES))
def test_fp32_teacher_forced_parity(name):
    make, B, kw = CASES[name]
    g = make()
    worst, widened, sched = check_run(g, B, 50, **kw)
    print(f"{name}: max |dX| = {worst:.2e}, rows on the gamma_k bound: {widened}, schedule: {sched}")


@pytest.mark.parametrize("name", ["er_unit_B16", "ba_hubs_B64", "lifted_l2_B16", "er_pm1_B24_tiles",
                                  "laplacian_B16", "lifted_l8_B16", "lifted_l4_active_B32", "lifted_l12_B8"])
def test_bf16_teacher_forced_parity(name):
    make, B, kw = CASES[name]
    g = make()
    worst, _, sched = check_run(g, B, 50, dtype=deco.BF16, **kw)
    print(f"{name} bf16: max |dX| = {worst:.2e}, schedule: {sched}")


LANES4 = {
    "ba_B256": (lambda: synth.barabasi_albert(600, 3, 2), 256, (64, 1 << 30, 0, 4096, 256, 4), {}),
    "er_pm1_B64": (lambda: synth.with_rademacher_weights(synth.erdos_renyi(400, 0.1, 3), 4), 64,
                   (16, 1 << 30, 1, 4096, 512, 4), {}),
    "lifted_l1_B64": (lambda: synth.erdos_renyi(300, 0.05, 14), 64, (16, 1 << 30, 0, 4096, 256, 4),
                      dict(l=1, lifted=True)),
    "laplacian_B64": (lambda: synth.erdos_renyi(400, 0.05, 6), 64, (16, 1 << 30, 0, 4096, 256, 4),
                      dict(form=deco.GRAD_LAPLACIAN, eta=0.01)),
}


# float32 rows of 2 to 4 components run 2 values per lane by default; 4 values per lane
# (lane_elems = 4) is the alternative the autotuner also tries. A batch whose members all have
# one active component runs the 4-value kernels on the same tile with half the lanes.
F32_LIFTED_LANES = {
    "l2_B64_four": (lambda: synth.barabasi_albert(500, 3, 30), 64, 2, (8, 1 << 30, 1, 4096, 256, 4), None),
    "l3_B16_four": (lambda: synth.erdos_renyi(400, 0.05, 31), 16, 3, (4, 1 << 30, 0, 4096, 512, 4), None),
    "l4_B32_four": (lambda: synth.barabasi_albert(400, 4, 32), 32, 4, (8, 1 << 30, 0, 4096, 128, 4), None),
    "l4_B32_two_wide": (lambda: synth.barabasi_albert(400, 4, 33), 32, 4, (16, 1 << 30, 0, 4096, 128, 0), None),
    "l4_B32_two_active1": (lambda: synth.erdos_renyi(400, 0.05, 34), 32, 4, None, np.ones(32, np.int32)),
    "l3_B64_two_active_mix": (lambda: synth.barabasi_albert(500, 3, 35), 64, 3, (16, 1 << 30, 1, 4096, 256, 0),
                              np.array([1 + (b % 3) for b in range(64)], np.int32)),
}


@pytest.mark.parametrize("name", sorted(F32_LIFTED_LANES))
def test_f32_lifted_lane_width_parity(name):
    """Lifted float32 rows under both lane widths: teacher-forced parity with the oracle,
    exact cuts and the running best."""
    make, B, l, sched, la = F32_LIFTED_LANES[name]
    g = make()
    worst, _, s = check_run(g, B, 20, l=l, lifted=True, schedule=sched, l_active=la)
    assert ("vec=4" if name.split("_")[2] == "four" else "vec=2") in s
    print(f"{name}: max |dX| = {worst:.2e}, schedule: {s}")


# bfloat16 rows of 2 to 8 components with 2 values per lane (lane_elems = 2, 4-byte loads;
# the autotuner's alternative to the native 4); one-component members and momentum run the
# 4-value kernels on the same tile.
BF16_LIFTED_PAIRS = {
    "l2_B64": (lambda: synth.barabasi_albert(500, 3, 40), 64, 2, (16, 1 << 30, 1, 4096, 256, 2), None),
    "l3_B16_pm1": (lambda: synth.with_rademacher_weights(synth.erdos_renyi(400, 0.05, 41), 5), 16, 3,
                   (8, 1 << 30, 0, 4096, 512, 2), None),
    "l4_B32": (lambda: synth.barabasi_albert(400, 4, 42), 32, 4, (16, 1 << 30, 0, 4096, 128, 2), None),
    "l4_B32_active1": (lambda: synth.erdos_renyi(400, 0.05, 43), 32, 4, (16, 1 << 30, 0, 4096, 128, 2),
                       np.ones(32, np.int32)),
    "l4_B64_active_mix": (lambda: synth.barabasi_albert(500, 3, 44), 64, 4, (32, 1 << 30, 1, 4096, 256, 2),
                          np.array([1 + (b % 4) for b in range(64)], np.int32)),
    "l2_B32_intw": (_intw_graph, 32, 2, (16, 1 << 30, 0, 4096, 256, 2), None),
    "l6_B24": (lambda: synth.erdos_renyi(250, 0.06, 45), 24, 6, (4, 1 << 30, 0, 4096, 256, 2), None),
    "l8_B16_active_mix": (lambda: synth.barabasi_albert(300, 3, 46), 16, 8, (8, 1 << 30, 0, 4096, 256, 2),
                          np.array([1 + (5 * b) % 8 for b in range(16)], np.int32)),
}


@pytest.mark.parametrize("name", sorted(BF16_LIFTED_PAIRS))
def test_bf16_lifted_pair_lane_parity(name):
    """Lifted bfloat16 rows, 2 values per lane: teacher-forced parity with the oracle (one
    bfloat16 ulp plus the float32 step bound), exact cuts and the running best."""
    make, B, l, sched, la = BF16_LIFTED_PAIRS[name]
    g = make()
    worst, _, s = check_run(g, B, 20, l=l, lifted=True, dtype=deco.BF16, schedule=sched, l_active=la)
    assert "vec=2" in s
    print(f"{name} bf16 2-lane: max |dX| = {worst:.2e}, schedule: {s}")


@pytest.mark.parametrize("name", sorted(LANES4))
def test_bf16_four_lane_schedule_parity(name):
    """Unlifted bfloat16 rows with 4 values per lane (8-byte loads, one row team per wave at
    B = 256): the same teacher-forced parity, exact cuts and running best."""
    make, B, sched, kw = LANES4[name]
    g = make()
    worst, _, s = check_run(g, B, 15, dtype=deco.BF16, schedule=sched, **kw)
    assert "vec=4" in s
    print(f"{name} bf16 4-lane: max |dX| = {worst:.2e}, schedule: {s}")


def test_float_weights_cut_within_bound():
    g = synth.erdos_renyi(300, 0.06, 21)
    m = g.nnz // 2
    g = synth.with_weights(g, np.random.default_rng(3).uniform(0.1, 2.0, m).astype(np.float32))
    r = run_teacher_forced(g, 16, 10)
    for t, X in enumerate(r["xs"]):
        cuts, _ = oracle_cuts(g, X, 16, 1, False)
        # real weights: float32 partials of at most 2048 terms per lane and item (the
        # staging limit), then double: |error| <= 1/2 sum|w| * 2048 * 2^-24
        tol = 0.5 * np.abs(g.w.astype(np.float64)).sum() * 2048 * 2.0 ** -24
        assert np.all(np.abs(r["trace"][t] - cuts) <= tol)
        want = oracle.step(g, X, 0.1) if t < 10 else None
        if want is not None:
            assert np.abs(r["xs"][t + 1] - want).max() <= 1e-5
    r["handle"].destroy()


@pytest.mark.parametrize("dtype,l,sched", [(deco.F32, 4, None), (deco.F32, 2, (4, 1 << 30, 0, 4096, 256, 4)),
                                           (deco.BF16, 3, (8, 1 << 30, 0, 4096, 256, 2))])
def test_lifted_float_weights_cut_within_bound(dtype, l, sched):
    """Lifted rows with real weights (float32 on its default 2-value lanes and on 4-value
    lanes; bfloat16 on 2-value lanes): cuts within the bound of float32 partials, steps within
    1e-5 of the oracle's (bfloat16: one ulp more)."""
    g = _realw_graph()
    B = 16
    r = run_teacher_forced(g, B, 10, l=l, lifted=True, dtype=dtype, schedule=sched)
    want_vec = "vec=4" if sched is not None and sched[5] == 4 else "vec=2"
    assert want_vec in r["handle"].schedule()
    tol = 0.5 * np.abs(g.w.astype(np.float64)).sum() * 2048 * 2.0 ** -24
    for t, X in enumerate(r["xs"]):
        cuts, _ = oracle_cuts(g, X, B, l, True)
        assert np.all(np.abs(r["trace"][t] - cuts) <= tol), f"cut at step {t}"
        if t < 10:
            want = oracle.step(g, X, 0.1)
            if dtype == deco.BF16:
                emu = oracle.to_bf16(want.astype(np.float32)).astype(np.float64)
                assert np.all(np.abs(r["xs"][t + 1] - emu) <= bf16_ulp(emu) + 1e-5), f"step {t}"
            else:
                assert np.abs(r["xs"][t + 1] - want).max() <= 1e-5, f"step {t}"
    r["handle"].destroy()


def test_multi_graph_batch_parity():
    gs = [synth.erdos_renyi(150, 0.1, 1), synth.barabasi_albert(220, 3, 2), synth.cycle(9), synth.star(40),
          synth.erdos_renyi(90, 0.2, 3)]
    bd = synth.block_diagonal(gs)
    worst, _, sched = check_run(bd, 8, 25)
    print(f"multi-graph: {worst:.2e} {sched}")


def test_autotuned_schedule_keeps_parity():
    g = synth.barabasi_albert(3000, 4, 5)
    worst, _, sched = check_run(g, 64, 8, schedule_tune=True)
    print(f"autotuned: {sched}, {worst:.2e}")


def test_negated_start_gives_bitwise_negated_trajectory():
    g = synth.barabasi_albert(500, 3, 1)
    x0 = synth.uniform_batch(g.n, 32, 9)
    a = run_teacher_forced(g, 32, 15, x0=x0)
    b = run_teacher_forced(g, 32, 15, x0=-x0)
    for xa, xb in zip(a["xs"], b["xs"]):
        assert np.array_equal(xa, -xb)
    if not any(np.any(x == 0) for x in a["xs"]):
        assert np.array_equal(a["trace"], b["trace"])
    a["handle"].destroy()
    b["handle"].destroy()


def test_lifted_columns_equal_unlifted_runs_bitwise():
    """Under one schedule (same lane width and teams, same item cuts, so the same summation
    order) each component of a lifted run evolves exactly as an unlifted run of those
    columns. Lifted float32 rows take the 4-value lanes of the unlifted kernels here
    (lane_elems = 4): their default 2-value lanes put twice the lanes on a tile, so a
    workgroup has half the row teams, the item's slots split at other points and the partial
    sums of a split row add in another order; those are held to the oracle's step bound
    (test_f32_lifted_lane_width_parity)."""
    g = synth.erdos_renyi(400, 0.05, 2)
    B, l = 16, 3
    x0 = synth.uniform_batch(g.n, l * B, 4)
    sched = (4, 1 << 30, 0, 4096, 512)
    lifted = run_teacher_forced(g, B, 10, l=l, lifted=True, x0=x0, schedule=sched + (4,))
    assert "vec=4" in lifted["handle"].schedule()
    for i in range(l):
        un = run_teacher_forced(g, B, 10, x0=np.ascontiguousarray(x0[:, i * B:(i + 1) * B]), schedule=sched)
        for xl, xu in zip(lifted["xs"], un["xs"]):
            assert np.array_equal(xl[:, i * B:(i + 1) * B], xu)
        un["handle"].destroy()
    lifted["handle"].destroy()


def test_determinism_bitwise():
    g = synth.barabasi_albert(2000, 3, 3)
    a = run_teacher_forced(g, 64, 12)
    b = run_teacher_forced(g, 64, 12)
    for xa, xb in zip(a["xs"], b["xs"]):
        assert np.array_equal(xa, xb)
    assert np.array_equal(a["trace"], b["trace"])
    for u, v in zip(a["best"], b["best"]):
        assert np.array_equal(u, v)
    a["handle"].destroy()
    b["handle"].destroy()


def test_score_every_and_graph_replay():
    g = synth.erdos_renyi(600, 0.03, 5)
    B = 32
    G = deco.Graph(g)
    h = deco.Handle(G, B=B, eta=0.1, score_every=5, seed=2)
    x0 = torch.from_numpy(synth.uniform_batch(g.n, B, 1)).cuda()
    h.start(deco.INIT_USER, x0=x0)
    tr = h.set_trace(64)
    xs = [to_np(h.read_x()).astype(np.float64)]
    for _ in range(20):
        h.step(1)
        xs.append(to_np(h.read_x()).astype(np.float64))
    trn = tr.cpu().numpy()
    for t in range(20):
        if t % 5 == 0:
            assert np.array_equal(trn[t], oracle_cuts(g, xs[t], B, 1, False)[0])
        else:
            assert np.all(np.isnan(trn[t]))
    # the same 20 steps replayed through a captured graph give the same iterate
    h2 = deco.Handle(G, B=B, eta=0.1, score_every=5, seed=2)
    h2.start(deco.INIT_USER, x0=x0)
    h2.step(10, use_graph=True)
    h2.step(10, use_graph=True)
    assert h2.current_step() == 20
    assert np.array_equal(to_np(h2.read_x()).astype(np.float64), xs[20])
    b1 = h.best()
    b2 = h2.best()
    for u, v in zip(b1, b2):
        assert np.array_equal(u, v)
    # replays of one graph, with eager work between them, agree with eager steps
    h3 = deco.Handle(G, B=B, eta=0.1, score_every=5, seed=2)
    h3.start(deco.INIT_USER, x0=x0)
    for _ in range(4):
        h3.step(5, use_graph=True)
        h3.synchronize()
        _ = torch.ones(1000, device="cuda").sum().item()
    assert np.array_equal(to_np(h3.read_x()).astype(np.float64), xs[20])
    for hh in (h, h2, h3):
        hh.destroy()


def test_start_kinds_match_oracle():
    g = synth.barabasi_albert(700, 3, 4)
    B = 32
    seed = 77
    G = deco.Graph(g)
    h = deco.Handle(G, B=B, seed=seed)
    h.start(deco.INIT_UNIFORM, batch=3)
    x = to_np(h.read_x()).astype(np.float64)
    assert np.array_equal(x, oracle.init_uniform(g.n, B, seed, 3))
    # IDI signs: with no noise the start is h / scale exactly
    h.start(deco.INIT_IDI, scale=1.0, sigma2=0.0, beta=0.2, batch=5)
    x = to_np(h.read_x()).astype(np.float64)
    assert np.array_equal(x, oracle.init_idi(g, B, seed, 5, 0.2))
    # DUI and the Gaussian exploration around a mean: within float rounding
    h.start(deco.INIT_DUI, scale=1.0, sigma2=0.0, batch=6)
    x = to_np(h.read_x()).astype(np.float64)
    assert np.abs(x - oracle.init_dui(g, B, seed, 6)).max() <= 2 ** -23
    h.start(deco.INIT_IDI, scale=1e4, sigma2=0.8, beta=0.2, batch=7)
    x = to_np(h.read_x()).astype(np.float64)
    want = oracle.init_gauss(oracle.init_idi(g, B, seed, 7, 0.2), 0.8, 1e4, seed, 7)
    assert np.all(np.abs(x - want) <= 2 * np.spacing(np.abs(want).astype(np.float32)).astype(np.float64))
    z = torch.from_numpy((np.arange(g.n) % 3 == 0).astype(np.uint8)).cuda()
    h.start(deco.INIT_MEAN, mean_z=z, scale=2.0, sigma2=0.5, batch=8)
    x = to_np(h.read_x()).astype(np.float64)
    M = np.repeat(np.where(z.cpu().numpy() == 1, 1.0, -1.0)[:, None], B, 1)
    want = oracle.init_gauss(M, 0.5, 2.0, seed, 8)
    assert np.all(np.abs(x - want) <= 2 * np.spacing(np.abs(want).astype(np.float32)).astype(np.float64))
    h.destroy()


def test_idi_per_graph_statistics_in_a_batch():
    gs = [synth.star(30), synth.barabasi_albert(200, 2, 1), synth.erdos_renyi(100, 0.1, 2)]
    bd = synth.block_diagonal(gs)
    G = deco.Graph(bd)
    h = deco.Handle(G, B=16, seed=5)
    h.start(deco.INIT_IDI, scale=1.0, sigma2=0.0, batch=1)
    x = to_np(h.read_x()).astype(np.float64)
    assert np.array_equal(x, oracle.init_idi(bd, 16, 5, 1))
    star = x[:30]
    assert np.all(star[1:] == -star[0:1])
    h.destroy()


@pytest.mark.parametrize("B", [1, 8])
def test_lifted_side_uses_float32_sum_in_component_order(B):
    """l = 8, float32: a vertex whose components are (0.1, 0.2, 0.3, -0.6, 0, 0, 0, 0) sums
    to exactly 0 in component order (side 1, the lifted tie), although the exact sum is
    negative; joined by one edge to a vertex at -0.5 everywhere, every initialisation cuts
    the edge. B = 1 runs one-element lanes, B = 8 four-element lanes."""
    l = 8
    g = synth.from_edges(2, np.array([0]), np.array([1]))
    comp = np.array([0.1, 0.2, 0.3, -0.6, 0, 0, 0, 0], np.float32)
    x0 = np.empty((2, l * B), np.float32)
    for i in range(l):
        x0[0, i * B:(i + 1) * B] = comp[i]
        x0[1, i * B:(i + 1) * B] = -0.5
    h = deco.Handle(deco.Graph(g), B=B, l=l, lifted=True, seed=1)
    h.start(deco.INIT_USER, x0=torch.from_numpy(x0).cuda())
    cut, bits = h.round_score()
    cut = cut.cpu().numpy()
    z = deco.bits_to_z(bits.cpu().numpy(), B)
    assert z[0].tolist() == [1] * B and z[1].tolist() == [0] * B
    assert np.array_equal(cut, np.ones((1, B)))
    assert np.array_equal(cut[0], oracle_cuts(g, x0.astype(np.float64), B, l, True)[0][0])
    h.destroy()


@pytest.mark.parametrize("l", [4, 8])
def test_inactive_lift_components_stay_zero(l):
    g = synth.erdos_renyi(300, 0.05, 3)
    B = 16
    G = deco.Graph(g)
    h = deco.Handle(G, B=B, l=l, lifted=True, seed=1)
    la = np.array([1 + b % l for b in range(B)], np.int32)
    z = torch.ones(g.n, dtype=torch.uint8, device="cuda")
    h.start(deco.INIT_MEAN, mean_z=z, scale=1e4, sigma2=0.8, batch=2, l_active=la)
    h.step(25)
    x = to_np(h.read_x())
    for b in range(B):
        for i in range(l):
            col = x[:, i * B + b]
            if i >= la[b]:
                assert np.all(col == 0.0)
            else:
                assert np.any(col != 0.0)
    h.destroy()


@pytest.mark.parametrize("l,dtype", [(4, deco.BF16), (4, deco.F32), (2, deco.BF16), (8, deco.BF16)])
def test_active_component_gathers_equal_full_gathers(l, dtype):
    """A start that names each initialisation's active components (the step kernel then
    gathers only those) gives the same iterates, cuts, running best and best bits, bit for
    bit, as the same start without them (every component gathered), on the bench's lane
    layout (B = 256) and with active counts that change inside a lane."""
    g = synth.barabasi_albert(2000, 4, 31)
    B = 256
    G = deco.Graph(g)
    la = np.array([1 + ((b // 32) + (b % 3)) % l for b in range(B)], np.int32)
    rng = np.random.default_rng(5)
    x0 = rng.uniform(-1, 1, (g.n, l * B)).astype(np.float32)
    for b in range(B):
        x0[:, la[b] * B + b::B] = 0.0
    tdt = torch.float32 if dtype == deco.F32 else torch.bfloat16
    X0 = torch.from_numpy(x0).to(tdt).cuda()
    runs = []
    for active in (la, None):
        h = deco.Handle(G, B=B, l=l, lifted=True, x_dtype=dtype, eta=0.05, seed=2)
        h.start(deco.INIT_USER, x0=X0, l_active=active)
        tr = h.set_trace(31)
        xs = []
        for _ in range(3):
            h.step(10, use_graph=True)
            xs.append(h.read_x().clone())
        cut, bits = h.round_score()
        bc, bs, bb = h.best()
        runs.append((xs, tr.cpu().numpy(), cut.cpu().numpy(), bits.cpu().numpy(), bc, bs, bb))
        h.destroy()
    (xa, ta, ca, ba, bca, bsa, bba), (xf, tf, cf, bf, bcf, bsf, bbf) = runs
    for u, v in zip(xa, xf):
        assert torch.equal(u.view(torch.int16) if dtype == deco.BF16 else u.view(torch.int32),
                           v.view(torch.int16) if dtype == deco.BF16 else v.view(torch.int32))
    for u, v in [(ta, tf), (ca, cf), (ba, bf), (bca, bcf), (bsa, bsf), (bba, bbf)]:
        assert np.array_equal(u, v)
    # and the inactive components are still exactly 0
    x = to_np(xa[-1])
    for b in range(B):
        assert np.all(x[:, la[b] * B + b::B] == 0.0)


def test_philox_device_matches_host_and_oracle():
    out = deco.philox_device(5, 7, 11, 0x1234_5678_9ABC, 257)
    for i in [0, 1, 100, 256]:
        ctr = [i, 5, 7, 11]
        key = [0x5678_9ABC, 0x1234]
        assert list(out[i]) == list(oracle.philox(ctr, key)) == list(deco.philox(ctr, key))


# ------------------------------------------------------------------ edge cases
def test_tiny_and_empty_graphs():
    for g in [synth.edgeless(1), synth.edgeless(7), synth.path(2)]:
        r = run_teacher_forced(g, 8, 3)
        for t, X in enumerate(r["xs"]):
            assert np.array_equal(r["trace"][t], oracle_cuts(g, X, 8, 1, False)[0])
        if g.nnz == 0:
            assert np.array_equal(r["xs"][0], r["xs"][-1])  # no neighbours: the cut-form gradient is zero
        r["handle"].destroy()


def test_invalid_inputs_are_rejected_before_any_launch():
    g = synth.cycle(8)
    bad = synth.CSR(g.n, g.row_ptr.copy(), g.col_idx.copy())
    bad.col_idx[1] = 5  # row 0 -> 5 has no mirror entry
    with pytest.raises(deco.DecoError) as e:
        deco.Handle(deco.Graph(bad), B=8)
    assert e.value.status == deco.E_INVAL
    bad2 = synth.CSR(g.n, g.row_ptr.copy(), g.col_idx.copy())
    bad2.col_idx[0] = 0  # self loop
    with pytest.raises(deco.DecoError) as e:
        deco.Handle(deco.Graph(bad2), B=8)
    assert e.value.status == deco.E_INVAL
    bad3 = synth.CSR(g.n, g.row_ptr.copy(), g.col_idx.copy(), np.ones(g.nnz, np.float32))
    bad3.w[3] = np.nan
    with pytest.raises(deco.DecoError) as e:
        deco.Handle(deco.Graph(bad3), B=8)
    assert e.value.status in (deco.E_NONFINITE, deco.E_INVAL)
    bad4 = synth.CSR(g.n, g.row_ptr.copy(), g.col_idx.copy())
    bad4.row_ptr[-1] = g.nnz - 1  # row_ptr end does not match nnz
    with pytest.raises(deco.DecoError) as e:
        deco.Handle(deco.Graph(bad4), B=8)
    assert e.value.status == deco.E_INVAL
    h = deco.Handle(deco.Graph(g), B=8)
    x0 = torch.zeros((g.n, 8), device="cuda")
    x0[2, 3] = float("nan")
    with pytest.raises(deco.DecoError) as e:
        h.start(deco.INIT_USER, x0=x0)
    assert e.value.status == deco.E_NONFINITE
    with pytest.raises(deco.DecoError) as e:
        h.start(deco.INIT_MEAN)  # no mean vector
    assert e.value.status == deco.E_INVAL
    with pytest.raises(deco.DecoError):
        deco.Handle(deco.Graph(g), B=3)
    h.destroy()


def test_workspace_too_small():
    import ctypes as ct
    g = synth.erdos_renyi(100, 0.1, 1)
    G = deco.Graph(g)
    p = deco.deco_params(16, 1, 0, 0, 0, 1, 0.1, 0)
    nb = ct.c_size_t(0)
    assert deco.lib().deco_workspace_size(ct.byref(G.struct), ct.byref(p), ct.byref(nb)) == 0
    X = torch.zeros((g.n, 16), device="cuda")
    ws = torch.zeros(nb.value, dtype=torch.uint8, device="cuda")
    h = ct.c_void_p()
    st = deco.lib().deco_init(ct.byref(h), ct.byref(G.struct), ct.byref(p), X.data_ptr(), ws.data_ptr(),
                              nb.value - 1, None)
    assert st == deco.E_NOMEM and not h.value


@pytest.mark.parametrize("lifted,l", [(False, 1), (True, 2), (True, 10)])
def test_step_calls_split_and_replayed_agree_bitwise(lifted, l):
    """A step's cuts are completed by the next launch and every call ends with a drain: the
    same 12 steps (scored every step) taken as one call, as 12 calls and as two graph replays
    give the same iterates, traces, running best (cuts, steps, bits) and round score; reading
    the best twice gives the same result."""
    gs = [synth.barabasi_albert(700, 3, 11), synth.erdos_renyi(300, 0.05, 12)]
    g = synth.block_diagonal(gs)
    G = deco.Graph(g)
    B = 32
    x0 = torch.from_numpy(synth.uniform_batch(g.n, l * B, 4)).to(torch.bfloat16).cuda()
    runs = []
    for mode in ("one", "each", "graph"):
        h = deco.Handle(G, B=B, l=l, lifted=lifted, x_dtype=deco.BF16, eta=0.05, seed=3)
        h.start(deco.INIT_USER, x0=x0)
        tr = h.set_trace(16)
        if mode == "one":
            h.step(12)
        elif mode == "each":
            for _ in range(12):
                h.step(1)
        else:
            h.step(6, use_graph=True)
            h.step(6, use_graph=True)
        cut_T, bits_T = h.round_score()
        best = h.best()
        again = h.best()
        for u, v in zip(best, again):
            assert np.array_equal(u, v)
        runs.append((to_np(h.read_x()), tr.cpu().numpy(), best, to_np(cut_T), to_np(bits_T)))
        h.destroy()
    ref = runs[0]
    assert np.array_equal(ref[1][12], oracle_cuts(g, ref[0].astype(np.float64), B, l, lifted)[0])
    for other in runs[1:]:
        assert np.array_equal(ref[0], other[0])
        assert np.array_equal(ref[1][:13], other[1][:13])
        for u, v in zip(ref[2], other[2]):
            assert np.array_equal(u, v)
        assert np.array_equal(ref[3], other[3]) and np.array_equal(ref[4], other[4])


@pytest.mark.parametrize("dtype,l", [(deco.F32, 1), (deco.BF16, 1), (deco.F32, 2), (deco.F32, 6)])
def test_momentum_teacher_forced_parity(dtype, l):
    """Heavy-ball momentum (deco_set_momentum): from the GPU's own X_t and V_t, the oracle's
    momentum step gives X_t+1 and V_t+1 (float32: V within 2e-5 relative, X within the step
    bound; bfloat16 X within one ulp more); cuts stay exact; a new start begins at rest."""
    g = synth.barabasi_albert(900, 3, 21)
    B, mu, eta = 32, 0.9, 0.02
    G = deco.Graph(g)
    h = deco.Handle(G, B=B, l=l, lifted=l > 1, x_dtype=dtype, eta=eta, seed=5)
    vel = h.set_momentum(mu)
    tdt = torch.float32 if dtype == deco.F32 else torch.bfloat16
    x0 = torch.from_numpy(synth.uniform_batch(g.n, l * B, 6)).to(tdt).cuda()
    h.start(deco.INIT_USER, x0=x0)
    tr = h.set_trace(16)
    X = to_np(h.read_x()).astype(np.float64)
    V = vel.cpu().numpy().astype(np.float64)
    assert not V.any()
    for t in range(8):
        h.step(1)
        Xg = to_np(h.read_x()).astype(np.float64)
        Vg = vel.cpu().numpy().astype(np.float64)
        Xw, Vw = oracle.step_momentum(g, X, V, eta, mu)
        assert np.all(np.abs(Vg - Vw) <= 2e-5 * np.maximum(1.0, np.abs(Vw))), t
        tol = eta * 2e-5 * np.maximum(1.0, np.abs(Vw)) + 4 * U32
        if dtype == deco.BF16:
            emu = oracle.to_bf16(np.clip(X + eta * Vg, -1, 1).astype(np.float32)).astype(np.float64)
            assert np.all(np.abs(Xg - emu) <= bf16_ulp(emu) + tol), t
        else:
            assert np.all(np.abs(Xg - Xw) <= tol), t
        assert np.array_equal(tr.cpu().numpy()[t], oracle_cuts(g, X, B, l, l > 1)[0])
        X, V = Xg, Vg
    h.start(deco.INIT_USER, x0=x0)
    assert not vel.cpu().numpy().any()
    h.destroy()


def test_momentum_zero_equals_plain_steps():
    """mu = 0 with a velocity buffer gives the plain steps bit for bit (float32 rows)."""
    g = synth.erdos_renyi(500, 0.04, 9)
    G = deco.Graph(g)
    x0 = torch.from_numpy(synth.uniform_batch(g.n, 16, 3)).cuda()
    out = []
    for mu in (None, 0.0):
        h = deco.Handle(G, B=16, eta=0.1, seed=1)
        if mu is not None:
            h.set_momentum(mu)
        h.start(deco.INIT_USER, x0=x0)
        h.step(6)
        out.append(to_np(h.read_x()))
        h.destroy()
    assert np.array_equal(out[0], out[1])


def test_momentum_with_captured_graphs_and_errors():
    """Turning momentum on after step graphs were captured re-captures them (the replayed
    steps use the velocity), turning it off restores plain steps; a non-finite coefficient is
    rejected before any launch."""
    g = synth.erdos_renyi(400, 0.05, 13)
    G = deco.Graph(g)
    x0 = torch.from_numpy(synth.uniform_batch(g.n, 16, 7)).cuda()
    ref = deco.Handle(G, B=16, eta=0.05, seed=1)
    ref.start(deco.INIT_USER, x0=x0)
    ref.step(4)
    ref.set_momentum(0.8)
    ref.step(4)
    ref.set_momentum(None)
    ref.step(4)
    h = deco.Handle(G, B=16, eta=0.05, seed=1)
    h.start(deco.INIT_USER, x0=x0)
    h.step(4, use_graph=True)
    h.set_momentum(0.8)
    h.step(4, use_graph=True)
    h.set_momentum(None)
    h.step(4, use_graph=True)
    assert np.array_equal(to_np(ref.read_x()), to_np(h.read_x()))
    for u, v in zip(ref.best(), h.best()):
        assert np.array_equal(u, v)
    with pytest.raises(deco.DecoError):
        h.set_momentum(float("nan"))
    ref.destroy()
    h.destroy()


# Resident schedule: every step of a call in one launch, each workgroup holding a tile of
# columns of one graph's rows in LDS (set_schedule resident_cols).
def resident(bt):
    return (64, 1 << 30, 0, 128, 2048, 0, bt)


RESIDENT = {
    "er_unit_B16_bt16": ("er_unit_B16", 16, deco.F32),
    "er_unit_B16_bt1": ("er_unit_B16", 1, deco.F32),
    "ba_hubs_B64_bt8": ("ba_hubs_B64", 8, deco.F32),
    "ba_hubs_B64_bt16_bf16": ("ba_hubs_B64", 16, deco.BF16),
    "er_pm1_B24_bt8": ("er_pm1_B24_tiles", 8, deco.F32),
    "er_pm1_B24_bt4_bf16": ("er_pm1_B24_tiles", 4, deco.BF16),
    "laplacian_B16_bt4": ("laplacian_B16", 4, deco.F32),
    "lifted_l1_B16_bt16": ("unlifted_as_l1_lifted", 16, deco.F32),
    "intw_B8_bt8": ("er_intw_B8", 8, deco.F32),
    "per_init_eta_bt2": ("per_init_eta", 2, deco.F32),
    "B1_bt1": ("B1", 1, deco.F32),
    "B2_bt2_bf16": ("B2", 2, deco.BF16),
    # one- and two-column tiles (per-lane boolean flags) under every weight mode, both
    # rounding rules and the Laplacian form
    "laplacian_B16_bt1": ("laplacian_B16", 1, deco.F32),
    "laplacian_B16_bt2_bf16": ("laplacian_B16", 2, deco.BF16),
    "intw_B8_bt2": ("er_intw_B8", 2, deco.F32),
    "intw_B8_bt1_bf16": ("er_intw_B8", 1, deco.BF16),
    "er_pm1_B24_bt1": ("er_pm1_B24_tiles", 1, deco.F32),
    "er_pm1_B24_bt2_bf16": ("er_pm1_B24_tiles", 2, deco.BF16),
    "lifted_l1_B16_bt1": ("unlifted_as_l1_lifted", 1, deco.F32),
    "lifted_l1_B16_bt2_bf16": ("unlifted_as_l1_lifted", 2, deco.BF16),
    "ba_hubs_B64_bt1_bf16": ("ba_hubs_B64", 1, deco.BF16),
}


@pytest.mark.parametrize("name", sorted(RESIDENT))
def test_resident_teacher_forced_parity(name):
    """The resident kernel, one step per call: teacher-forced iterates (float32: 1e-5 or the
    summation bound; bfloat16: one ulp plus the bound), exact cuts of every iterate, the
    running best and its bits, against the oracle."""
    case, bt, dtype = RESIDENT[name]
    make, B, kw = CASES[case]
    g = make()
    worst, _, s = check_run(g, B, 30, dtype=dtype, schedule=resident(bt), **kw)
    assert s.startswith(f"resident cols={bt}")
    print(f"{name}: max |dX| = {worst:.2e}, schedule: {s}")


def test_resident_multi_graph_batch_and_real_weights():
    """Resident steps on a block-diagonal batch (a workgroup per graph and tile; the largest
    graphs first) and on real weights (double cut partials: within the float32-to-double
    bound of the step kernel, here much tighter)."""
    gs = [synth.erdos_renyi(150, 0.1, 1), synth.barabasi_albert(220, 3, 2), synth.cycle(9), synth.star(40),
          synth.erdos_renyi(90, 0.2, 3), synth.edgeless(5)]
    bd = synth.block_diagonal(gs)
    worst, _, s = check_run(bd, 8, 25, schedule=resident(8))
    assert s.startswith("resident cols=8")
    g = synth.erdos_renyi(300, 0.06, 21)
    m = g.nnz // 2
    g = synth.with_weights(g, np.random.default_rng(3).uniform(0.1, 2.0, m).astype(np.float32))
    for bt in (16, 2, 1):
        _real_weights_resident(g, bt)


def _real_weights_resident(g, bt):
    r = run_teacher_forced(g, 16, 10, schedule=resident(bt))
    assert r["handle"].schedule().startswith(f"resident cols={bt}")
    for t, X in enumerate(r["xs"]):
        cuts, _ = oracle_cuts(g, X, 16, 1, False)
        if t < 10:
            # scored by the resident kernel (double partials)
            tol = np.abs(g.w.astype(np.float64)).sum() * 2.0 ** -40
        else:
            # the last iterate is scored by the step kernel's score pass (float32 partials)
            tol = 0.5 * np.abs(g.w.astype(np.float64)).sum() * 2048 * 2.0 ** -24
        assert np.all(np.abs(r["trace"][t] - cuts) <= tol), f"cut at step {t}"
        if t < 10:
            assert np.abs(r["xs"][t + 1] - oracle.step(g, X, 0.1)).max() <= 1e-5
    r["handle"].destroy()


@pytest.mark.parametrize("bt,dtype", [(16, deco.BF16), (1, deco.F32), (4, deco.F32)])
def test_resident_one_launch_equals_step_calls(bt, dtype):
    """Many steps in one resident launch give bit for bit the iterates, traces, running best
    (cuts, steps, bits) and round score of one launch per step and of graph replays (odd and
    even step counts, so the final iterate lands in either buffer)."""
    gs = [synth.barabasi_albert(700, 3, 11), synth.erdos_renyi(300, 0.05, 12)]
    g = synth.block_diagonal(gs)
    G = deco.Graph(g)
    B = 32
    tdt = torch.float32 if dtype == deco.F32 else torch.bfloat16
    x0 = torch.from_numpy(synth.uniform_batch(g.n, B, 4)).to(tdt).cuda()
    runs = []
    for mode in ("one", "each", "graph"):
        h = deco.Handle(G, B=B, x_dtype=dtype, eta=0.05, seed=3)
        h.set_schedule(*resident(bt))
        h.start(deco.INIT_USER, x0=x0)
        tr = h.set_trace(24)
        if mode == "one":
            h.step(13)
            h.step(8)
        elif mode == "each":
            for _ in range(21):
                h.step(1)
        else:
            h.step(13, use_graph=True)
            h.step(8, use_graph=True)
        cut_T, bits_T = h.round_score()
        best = h.best()
        runs.append((to_np(h.read_x()), tr.cpu().numpy(), best, to_np(cut_T), to_np(bits_T)))
        h.destroy()
    ref = runs[0]
    assert np.array_equal(ref[1][21], oracle_cuts(g, ref[0].astype(np.float64), B, 1, False)[0])
    zb = deco.bits_to_z(ref[2][2], B)
    assert np.array_equal(oracle.cut_batch(g, zb), ref[2][0])
    for other in runs[1:]:
        assert np.array_equal(ref[0], other[0])
        assert np.array_equal(ref[1][:22], other[1][:22])
        for u, v in zip(ref[2], other[2]):
            assert np.array_equal(u, v)
        assert np.array_equal(ref[3], other[3]) and np.array_equal(ref[4], other[4])


def test_resident_rejects_tiles_that_do_not_fit():
    g = synth.barabasi_albert(3000, 3, 5)
    h = deco.Handle(deco.Graph(g), B=32, x_dtype=deco.F32, eta=0.05)
    with pytest.raises(deco.DecoError) as e:
        h.set_schedule(*resident(16))  # 2 x 3000 x 16 x 4 bytes does not fit
    assert e.value.status == deco.E_UNSUPPORTED
    with pytest.raises(deco.DecoError):
        h.set_schedule(*resident(3))  # not a power of two
    h.set_schedule(*resident(2))
    h.destroy()
    hl = deco.Handle(deco.Graph(g), B=8, l=2, lifted=True, eta=0.05)
    with pytest.raises(deco.DecoError) as e:
        hl.set_schedule(*resident(1))  # lifted l > 1 keeps the step kernel
    assert e.value.status == deco.E_UNSUPPORTED
    hl.destroy()
