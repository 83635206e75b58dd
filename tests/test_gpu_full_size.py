"""GPU parity at the full sizes of the workloads (same launch path as bench.py).

The oracle cannot step a million-row batch quickly, so iterates are checked on sampled
rows: the oracle steps a star subgraph made of each sampled row and its neighbours, which
gives exactly that row's result. Cuts are checked on every graph and initialisation (the
oracle's eq. (1) scorer is fast enough), bit for bit.
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


def star_rows(g, rows):
    """Block-diagonal union of stars (row v and its neighbours, edges v-u with w_vu)."""
    rp = g.row_ptr.astype(np.int64)
    us, vs, ws, offs = [], [], [], [0]
    src_rows = []
    base = 0
    for v in rows:
        nb = g.col_idx[rp[v]:rp[v + 1]].astype(np.int64)
        k = len(nb)
        us.append(np.full(k, base))
        vs.append(base + 1 + np.arange(k))
        if g.w is not None:
            ws.append(g.w[rp[v]:rp[v + 1]])
        src_rows.append(np.concatenate([[v], nb]))
        base += 1 + k
        offs.append(base)
    u = np.concatenate(us) if us else np.zeros(0, np.int64)
    w = np.concatenate(ws) if ws else None
    mini = synth.from_edges(base, u, np.concatenate(vs), w)
    return mini, np.concatenate(src_rows), np.array(offs[:-1])


def block_of(g, i):
    """Graph i of a block-diagonal batch as a graph of its own (rows renumbered from 0)."""
    o = g.graph_row_offset
    r0, r1 = int(o[i]), int(o[i + 1])
    rp = g.row_ptr[r0:r1 + 1].astype(np.int64)
    ci = g.col_idx[rp[0]:rp[-1]].astype(np.int64) - r0
    w = None if g.w is None else g.w[rp[0]:rp[-1]]
    return synth.CSR(n=r1 - r0, row_ptr=(rp - rp[0]).astype(np.int32), col_idx=ci.astype(np.int32), w=w)


def step_tol(g, X_t, want, eta, dtype, form=deco.GRAD_CUT):
    """Per-element tolerance of one step (the float32 summation bound of Higham, Sec. 3.1,
    gamma_k sum|w x_u| per row, plus the update's roundings; one bfloat16 ulp on top for
    bfloat16 storage) and the value the GPU must be compared with (the exact step, or its
    float32 -> bfloat16 rounding)."""
    cw = -0.5 if form == deco.GRAD_CUT else -1.0
    bound = step_bound(g, X_t, eta, cw, form)
    if dtype == deco.BF16:
        emu = oracle.to_bf16(want.astype(np.float32)).astype(np.float64)
        return emu, bf16_ulp(emu) + bound
    return want, np.maximum(1e-5, bound)


def check_rows(g, X_t, X_next, rows, eta, dtype, form=deco.GRAD_CUT):
    """Rows of X_next against the oracle's step of their star subgraphs (each row's result is
    exact there). Returns the largest deviation and, per checked element, whether the step
    moved it by more than its tolerance (where a skipped update would be caught)."""
    mini, src, centre = star_rows(g, rows)
    Xs = X_t[src]
    want = oracle.step(mini, Xs, eta, form)
    cmp, tol = step_tol(mini, Xs, want, eta, dtype, form)
    cmp, tol = cmp[centre], tol[centre]
    got = X_next[rows]
    d = np.abs(got - cmp)
    assert np.all(d <= tol), f"max deviation {d.max():.3e}, {(d > tol).sum()} elements off"
    moved = np.abs(want[centre] - X_t[rows]) > tol
    return float(d.max()), moved


def run_steps(G, g, B, l, lifted, dtype, steps, eta, kind=deco.INIT_IDI, seed=1):
    h = deco.Handle(G, B=B, l=l, lifted=lifted, x_dtype=dtype, eta=eta, seed=seed)
    h.start(kind, scale=1e4, sigma2=0.8, batch=0)
    tr = h.set_trace(steps + 1)
    xs = [to_np(h.read_x()).astype(np.float64)]
    for _ in range(steps):
        h.step(1, use_graph=True)
        xs.append(to_np(h.read_x()).astype(np.float64))
    h.round_score()  # scores X_steps into the trace
    return h, xs, tr.cpu().numpy()


def test_er800_uniform_start_200_steps():
    """ER(800, 0.06) seed 0, B = 16 uniform starts in [-1, 1], eta = 0.1, 200 steps, every
    iterate rounded and scored: teacher-forced float32 parity on the first 50 steps (1e-5),
    bit-exact cuts on all 201 iterates, running best equal to the oracle's bookkeeping."""
    g = synth.erdos_renyi(800, 0.06, 0)
    G = deco.Graph(g)
    B, T = 16, 200
    h = deco.Handle(G, B=B, eta=0.1, seed=0)
    h.start(deco.INIT_UNIFORM, batch=0)
    x0 = to_np(h.read_x()).astype(np.float64)
    assert np.array_equal(x0, oracle.init_uniform(g.n, B, 0, 0))
    tr = h.set_trace(T + 1)
    xs = [x0]
    for t in range(T):
        h.step(1)
        xs.append(to_np(h.read_x()).astype(np.float64))
    h.round_score()
    trn = tr.cpu().numpy()
    best = np.full(B, -np.inf)
    step = np.full(B, -1)
    worst = 0.0
    for t in range(T + 1):
        cuts = oracle_cuts(g, xs[t], B, 1, False)[0][0]
        assert np.array_equal(trn[t][0], cuts)
        imp = cuts > best
        best[imp] = cuts[imp]
        step[imp] = t
        if t < 50:
            d = np.abs(xs[t + 1] - oracle.step(g, xs[t], 0.1)).max()
            worst = max(worst, d)
            assert d <= 1e-5
    bc, bs, bb = h.best()
    assert np.array_equal(bc[0], best) and np.array_equal(bs[0], step)
    assert np.array_equal(oracle.cut_batch(g, deco.bits_to_z(bb, B))[0], best)
    print(f"ER800: max per-step error {worst:.2e}, best cut {best.max():.0f}")
    h.destroy()


@pytest.mark.parametrize("dtype,l", [(deco.F32, 1), (deco.BF16, 1), (deco.F32, 4), (deco.BF16, 2), (deco.BF16, 8),
                                     (deco.BF16, 12)])
def test_ba10k_B256_full_rows(dtype, l):
    """BA(10^4, 4), B = 256 (the bench's graph and batch), uniform starts in [-1, 1], eta =
    0.05, 12 teacher-forced steps on every row and column: each element within the float32
    summation bound of its row (1e-5 at least; plus one bfloat16 ulp for bfloat16 storage),
    exact cuts of every iterate. The starts make the check able to fail: a step leaves most
    entries of low-degree rows (d <= 8) unclipped and moves them by eta/2 |sum_u x_u|, far
    above the tolerance, so a kernel that dropped their update would be off on most of them
    (the test asserts that more than 30% of those entries move by more than the tolerance
    in the oracle's own step; the share is printed)."""
    g = synth.barabasi_albert(10_000, 4, 0)
    G = deco.Graph(g)
    B, T, eta = 256, 12, 0.05
    h = deco.Handle(G, B=B, l=l, lifted=l > 1, x_dtype=dtype, eta=eta, seed=1)
    h.start(deco.INIT_UNIFORM, batch=0)
    tr = h.set_trace(T + 1)
    low = g.degrees() <= 8
    x = to_np(h.read_x()).astype(np.float64)
    moved_low = total_low = 0
    for t in range(T):
        h.step(1, use_graph=True)
        xn = to_np(h.read_x()).astype(np.float64)
        want = oracle.step(g, x, eta)
        cmp, tol = step_tol(g, x, want, eta, dtype)
        d = np.abs(xn - cmp)
        assert np.all(d <= tol), f"step {t}: {(d > tol).sum()} elements off, max {d.max():.3e}"
        assert np.array_equal(tr.cpu().numpy()[t], oracle_cuts(g, x, B, l, l > 1)[0]), f"cut at step {t}"
        mv = np.abs(want - x) > tol
        moved_low += int(mv[low].sum())
        total_low += int(mv[low].size)
        x = xn
    h.round_score()
    trn = tr.cpu().numpy()
    assert np.array_equal(trn[T], oracle_cuts(g, x, B, l, l > 1)[0])
    assert moved_low > 0.3 * total_low, (moved_low, total_low)
    print(f"BA10k dtype={dtype} l={l}: {moved_low / total_low:.1%} of low-degree entries moved beyond tolerance")
    h.destroy()


@pytest.mark.parametrize("dtype", [deco.F32, deco.BF16])
def test_ba10k_B256_resident_full_rows(dtype):
    """The bench's unlifted batch on the resident schedule the solver tunes to (one column per
    workgroup; the graph's 89,968 slots split evenly over 1024 threads, so hub rows span many
    threads' shares and are finished from their partial sums): 12 teacher-forced steps, one
    launch each, every row and column within the per-row float32 summation bound (plus one
    bfloat16 ulp), exact cuts of every iterate, and more than 30% of the entries of degree <= 8
    rows moving by more than the tolerance in the oracle's step (so a dropped update fails);
    then 12 steps in one launch equal, bit for bit, to the same 12 steps one launch each."""
    g = synth.barabasi_albert(10_000, 4, 0)
    G = deco.Graph(g)
    B, T, eta = 256, 12, 0.05
    h = deco.Handle(G, B=B, x_dtype=dtype, eta=eta, seed=1)
    h.set_schedule(64, 1 << 30, 0, 128, 2048, 0, 1)
    assert h.schedule().startswith("resident cols=1")
    h.start(deco.INIT_UNIFORM, batch=0)
    tr = h.set_trace(2 * T + 1)
    low = g.degrees() <= 8
    x = to_np(h.read_x()).astype(np.float64)
    moved_low = total_low = 0
    for t in range(T):
        h.step(1, use_graph=True)
        xn = to_np(h.read_x()).astype(np.float64)
        want = oracle.step(g, x, eta)
        cmp, tol = step_tol(g, x, want, eta, dtype)
        d = np.abs(xn - cmp)
        assert np.all(d <= tol), f"step {t}: {(d > tol).sum()} elements off, max {d.max():.3e}"
        assert np.array_equal(tr.cpu().numpy()[t], oracle_cuts(g, x, B, 1, False)[0]), f"cut at step {t}"
        mv = np.abs(want - x) > tol
        moved_low += int(mv[low].sum())
        total_low += int(mv[low].size)
        x = xn
    assert moved_low > 0.3 * total_low, (moved_low, total_low)
    x_mid = h.read_x().clone()
    h.step(T)
    one = to_np(h.read_x())
    h2 = deco.Handle(G, B=B, x_dtype=dtype, eta=eta, seed=1)
    h2.set_schedule(64, 1 << 30, 0, 128, 2048, 0, 1)
    h2.start(deco.INIT_USER, x0=x_mid)
    tr2 = h2.set_trace(T + 1)
    for _ in range(T):
        h2.step(1)
    assert np.array_equal(one, to_np(h2.read_x()))
    assert np.array_equal(tr.cpu().numpy()[T:2 * T], tr2.cpu().numpy()[:T])
    print(f"BA10k resident dtype={dtype}: {moved_low / total_low:.1%} of low-degree entries moved beyond tolerance")
    h.destroy()
    h2.destroy()


def test_ba10k_B256_cuts_every_step():
    """Exact cuts of every iterate of the bench's lifted shape (l = 4, bfloat16) from an IDI
    start, the start the solver uses."""
    g = synth.barabasi_albert(10_000, 4, 0)
    G = deco.Graph(g)
    h, xs, tr = run_steps(G, g, 256, 4, True, deco.BF16, 6, eta=0.05)
    for t in range(7):
        assert np.array_equal(tr[t], oracle_cuts(g, xs[t], 256, 4, True)[0])
    h.destroy()


def test_uneven_512_graph_batch():
    """512 graphs (half ER(n~U{200..1200}, 0.15), half BA(n~U{100..2000}, m~U{2..6})) in one
    launch per step, B = 64, bfloat16 storage, autotuned schedule, uniform starts, eta =
    0.02, 10 steps: exact cuts of all 512 x 64 (graph, initialisation) pairs at every
    iterate; every row of 32 whole graphs (16 ER, 16 BA) and 4 sampled rows of every other
    graph against the oracle's step within the per-row float32 bound plus one bfloat16 ulp.
    A step moves more than 30% of the checked entries, and of those of degree <= 8 rows, by
    more than the tolerance (asserted; the shares are printed), so a dropped update fails."""
    g = synth.uneven_batch(512, 7)
    G = deco.Graph(g)
    B, T, eta = 64, 10, 0.02
    h = deco.Handle(G, B=B, x_dtype=deco.BF16, eta=eta, seed=1)
    h.autotune(3)
    h.start(deco.INIT_UNIFORM, batch=0)
    tr = h.set_trace(T + 1)
    goff = g.graph_row_offset
    whole = list(range(0, 32))  # graphs 0..31: even ER, odd BA
    blocks = [block_of(g, i) for i in whole]
    rng = np.random.default_rng(0)
    rows = np.concatenate([rng.integers(goff[i], goff[i + 1], 4) for i in range(32, 512)])
    deg = g.degrees()
    x = to_np(h.read_x()).astype(np.float64)
    moved = checked = moved_low = checked_low = 0
    for t in range(T):
        h.step(1, use_graph=True)
        xn = to_np(h.read_x()).astype(np.float64)
        assert np.array_equal(tr.cpu().numpy()[t], oracle_cuts(g, x, B, 1, False)[0])
        for i, bg in zip(whole, blocks):
            r0, r1 = goff[i], goff[i + 1]
            want = oracle.step(bg, x[r0:r1], eta)
            cmp, tol = step_tol(bg, x[r0:r1], want, eta, deco.BF16)
            d = np.abs(xn[r0:r1] - cmp)
            assert np.all(d <= tol), f"step {t} graph {i}: {(d > tol).sum()} off, max {d.max():.3e}"
            mv = np.abs(want - x[r0:r1]) > tol
            moved += int(mv.sum())
            checked += mv.size
            lowr = deg[r0:r1] <= 8
            moved_low += int(mv[lowr].sum())
            checked_low += int(mv[lowr].size)
        _, mv = check_rows(g, x, xn, rows, eta, deco.BF16)
        moved += int(mv.sum())
        checked += mv.size
        x = xn
    h.round_score()
    assert np.array_equal(tr.cpu().numpy()[T], oracle_cuts(g, x, B, 1, False)[0])
    bc, bs, bb = h.best()
    assert np.array_equal(oracle.cut_batch(g, deco.bits_to_z(bb, B)), bc)
    assert moved > 0.3 * checked and moved_low > 0.3 * checked_low, (moved, checked, moved_low, checked_low)
    print(f"uneven batch: n={g.n} nnz={g.nnz}; schedule {h.schedule()}; {moved / checked:.1%} of checked "
          f"entries moved beyond tolerance ({moved_low / max(checked_low, 1):.1%} on degree <= 8 rows)")
    h.destroy()


def test_regular3_million_pm1_B128():
    """Random 3-regular n = 1e6 with +-1 weights, B = 128, bfloat16, autotuned schedule,
    uniform starts, eta = 0.1, 10 steps: exact cuts for all 128 initialisations at every
    iterate and 4000 sampled rows per step within the per-row bound plus one bfloat16 ulp;
    more than 30% of the sampled entries move by more than the tolerance (asserted)."""
    g = synth.with_rademacher_weights(synth.random_regular3(1_000_000, 0), 3)
    G = deco.Graph(g)
    B, T, eta = 128, 10, 0.1
    h = deco.Handle(G, B=B, x_dtype=deco.BF16, eta=eta, seed=1)
    h.autotune(3)
    h.start(deco.INIT_UNIFORM, batch=0)
    tr = h.set_trace(T + 1)
    rng = np.random.default_rng(1)
    moved = checked = 0
    x_dev = h.read_x().clone()
    for t in range(T):
        h.step(1, use_graph=True)
        xn_dev = h.read_x().clone()
        rows = rng.integers(0, g.n, 4000)
        mini, src, centre = star_rows(g, rows)
        xs = to_np(x_dev[torch.from_numpy(src).cuda()]).astype(np.float64)
        got = to_np(xn_dev[torch.from_numpy(rows).cuda()]).astype(np.float64)
        want = oracle.step(mini, xs, eta)
        cmp, tol = step_tol(mini, xs, want, eta, deco.BF16)
        d = np.abs(got - cmp[centre])
        assert np.all(d <= tol[centre]), f"step {t}: max deviation {d.max():.3e}"
        mv = np.abs(want[centre] - xs[centre]) > tol[centre]
        moved += int(mv.sum())
        checked += mv.size
        x_host = to_np(x_dev).astype(np.float64)
        assert np.array_equal(tr.cpu().numpy()[t], oracle_cuts(g, x_host, B, 1, False)[0])
        del x_host
        x_dev = xn_dev
    assert moved > 0.3 * checked, (moved, checked)
    print(f"3-regular: schedule {h.schedule()}; {moved / checked:.1%} of sampled entries moved beyond tolerance")
    h.destroy()


@pytest.mark.parametrize("l_max", [4, 8, 12])
def test_solve_small_graph_bounded_by_brute_force(l_max):
    g = synth.erdos_renyi(18, 0.4, 3)
    opt = oracle.brute_force(g)[0]
    r = deco.solve(deco.Graph(g), B=32, K=8, l_max=l_max, rounds=3, evo_rounds=2, T_q=100, T_l=50, seed=3)
    assert 1 <= r["l_best"] <= l_max
    assert r["best_cut"][0] == oracle.cut(g, r["z"]) <= opt
    assert r["best_cut"][0] >= 0.9 * opt
    assert np.all(np.diff(r["round_best"][:, 0]) >= 0)


@pytest.mark.parametrize("dtype", [deco.F32, deco.BF16])
def test_solve_ba10k_exact_result_and_beats_greedy(dtype):
    g = synth.barabasi_albert(10_000, 4, 0)
    r = deco.solve(deco.Graph(g), B=256, K=8, l_max=4, rounds=3, evo_rounds=2, T_q=300, T_l=150, x_dtype=dtype,
                   seed=1)
    assert r["best_cut"][0] == oracle.cut(g, r["z"])  # the reported cut is the exact cut of the vector
    gb, _ = oracle.greedy(g, orders=2, seed=1)
    assert r["best_cut"][0] > gb
    print(f"BA10k solve dtype={dtype}: {r['best_cut'][0]:.0f} (greedy {gb:.0f}) in {r['seconds']:.2f}s, "
          f"genes {r['eq_best']:.2f} {r['el_best']:.2f} {r['l_best']}")


def test_solver_object_continues_and_multi_graph():
    gs = [synth.erdos_renyi(300, 0.1, i) for i in range(3)] + [synth.barabasi_albert(500, 3, 9)]
    bd = synth.block_diagonal(gs)
    s = deco.Solver(deco.Graph(bd), B=64, K=8, l_max=2, evo_rounds=1, T_q=100, T_l=50, seed=4)
    r1 = s.run(2)
    r2 = s.run(2)
    assert r2["steps_done"] == 2 * r1["steps_done"]
    assert np.all(r2["best_cut"] >= r1["best_cut"])
    for i, gi in enumerate(gs):
        o = bd.graph_row_offset
        assert r2["best_cut"][i] == oracle.cut(gi, r2["z"][o[i]:o[i + 1]])
    s.destroy()


def test_rows_beyond_24_bits_use_one_element_lanes():
    """A cycle of n = 2^24 + 3 rows, B = 8, bfloat16: lanes of several elements address rows
    with 24-bit offsets, so a graph this large runs on one-element lanes (64-bit addresses).
    One step: sampled rows (including the last ones) against the oracle, exact cut of X_0 for
    every initialisation."""
    n = (1 << 24) + 3
    g = synth.cycle(n)
    G = deco.Graph(g)
    h = deco.Handle(G, B=8, x_dtype=deco.BF16, eta=0.1, seed=2)
    assert "vec=1" in h.schedule()
    h.start(deco.INIT_UNIFORM, batch=0)
    tr = h.set_trace(2)
    x0_dev = h.read_x().clone()
    h.step(1)
    x1_dev = h.read_x()
    rng = np.random.default_rng(5)
    rows = np.concatenate([rng.integers(0, n, 2000), np.arange(n - 8, n), np.arange((1 << 24) - 4, (1 << 24) + 3)])
    mini, src, centre = star_rows(g, rows)
    idx = torch.from_numpy(src).cuda()
    xs = to_np(x0_dev[idx]).astype(np.float64)
    got = to_np(x1_dev[torch.from_numpy(rows).cuda()]).astype(np.float64)
    want = oracle.step(mini, xs, 0.1)[centre]
    emu = oracle.to_bf16(want.astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(got - emu) <= bf16_ulp(emu) + 1e-5)
    x0 = to_np(x0_dev).astype(np.float64)
    assert np.array_equal(tr.cpu().numpy()[0], oracle_cuts(g, x0, 8, 1, False)[0])
    h.destroy()


def test_zero_step_keeps_columns_still():
    """A column with step size 0 keeps its iterate bit for bit while the others move (what the
    step-count search relies on to stop a member)."""
    g = synth.barabasi_albert(3000, 3, 4)
    G = deco.Graph(g)
    h = deco.Handle(G, B=32, x_dtype=deco.BF16, eta=0.05, seed=2)
    eta = np.full(32, 0.05, np.float32)
    eta[8:16] = 0.0
    h.set_eta(eta)
    h.start(deco.INIT_IDI, scale=1e4, sigma2=0.8)
    x0 = to_np(h.read_x())
    h.step(25, use_graph=True)
    x1 = to_np(h.read_x())
    assert np.array_equal(x0[:, 8:16], x1[:, 8:16])
    assert not np.array_equal(x0[:, :8], x1[:, :8])
    h.destroy()


@pytest.mark.parametrize("T_l_min", [0, 15])
def test_solve_with_step_count_search(T_l_min):
    """pDECO with the step-count half of the search (T_k in [T_min, T_q] per member, and the
    lifted count in [T_l_min, T_l] when T_l_min > 0): the returned cut is the exact cut of the
    returned vector and the final counts are in range."""
    g = synth.barabasi_albert(2000, 3, 6)
    r = deco.solve(deco.Graph(g), B=32, K=4, l_max=2, rounds=3, evo_rounds=2, T_q=160, T_l=40, x_dtype=deco.BF16,
                   seed=5, T_min=60, T_l_min=T_l_min)
    assert r["best_cut"][0] == oracle.cut(g, r["z"])
    assert 60 <= r["T_best"] <= 160
    tl_lo = T_l_min if T_l_min else 40
    assert tl_lo <= r["T_l_best"] <= 40
    assert 3 * (60 + tl_lo) <= r["steps_done"] <= 3 * (160 + 40)
    gb, _ = oracle.greedy(g, orders=2, seed=1)
    assert r["best_cut"][0] > 0.95 * gb


def test_solver_stops_inside_a_batch_at_the_target():
    """With check_every, a run with a target stops at the first check where every graph's best
    reached it (here inside the first unlifted batch), and still returns the exact cut of its
    vector; without it the run finishes its round."""
    g = synth.barabasi_albert(2000, 3, 8)
    G = deco.Graph(g)
    r0 = deco.solve(G, B=64, K=8, l_max=2, rounds=2, evo_rounds=1, T_q=400, T_l=100, seed=2)
    target = 0.98 * r0["best_cut"][0]
    r = deco.solve(G, B=64, K=8, l_max=2, rounds=3, evo_rounds=1, T_q=400, T_l=100, seed=2, target_cut=[target],
                   check_every=10)
    assert r["rounds_done"] == 1 and r["steps_done"] < 400 and r["steps_done"] % 10 == 0
    assert r["best_cut"][0] >= target
    assert r["best_cut"][0] == oracle.cut(g, r["z"])
    full = deco.solve(G, B=64, K=8, l_max=2, rounds=3, evo_rounds=1, T_q=400, T_l=100, seed=2, target_cut=[target])
    assert full["rounds_done"] == 1 and full["steps_done"] == 500


@pytest.mark.parametrize("mode,steps", [(deco.SOLVE_UNLIFTED, 2 * 100), (deco.SOLVE_LIFTED, 2 * 50)])
def test_solve_unlifted_only_and_lifted_only(mode, steps):
    """pQUCO-only and pLUCO-only runs (the two formulations with the search, without the
    alternation): each round runs one batch of its kind; the returned cut is exact."""
    g = synth.barabasi_albert(1500, 3, 11)
    r = deco.solve(deco.Graph(g), B=48, K=6, l_max=2, rounds=2, evo_rounds=1, T_q=100, T_l=50, seed=4, mode=mode)
    assert r["steps_done"] == steps
    assert r["best_cut"][0] == oracle.cut(g, r["z"])
    gb, _ = oracle.greedy(g, orders=2, seed=1)
    assert r["best_cut"][0] > 0.9 * gb


def test_uneven_512_graph_batch_resident():
    """The 512-graph uneven batch on the resident schedule (16 columns of a graph per
    workgroup, all steps of a call in one launch), bfloat16, uniform starts, eta = 0.02: 10
    teacher-forced steps with exact cuts of all 512 x 64 pairs at every iterate and every row
    of 16 whole graphs against the oracle's step (per-row float32 bound plus one bfloat16
    ulp), the best bits' cuts, and then 10 steps in one launch equal to 10 launches of one
    step, bit for bit."""
    g = synth.uneven_batch(512, 7)
    G = deco.Graph(g)
    B, T, eta = 64, 10, 0.02
    h = deco.Handle(G, B=B, x_dtype=deco.BF16, eta=eta, seed=1)
    h.set_schedule(64, 1 << 30, 0, 128, 2048, 0, 16)
    h.start(deco.INIT_UNIFORM, batch=0)
    tr = h.set_trace(T + 1)
    goff = g.graph_row_offset
    blocks = [block_of(g, i) for i in range(16)]
    x = to_np(h.read_x()).astype(np.float64)
    moved = checked = 0
    for t in range(T):
        h.step(1, use_graph=True)
        xn = to_np(h.read_x()).astype(np.float64)
        assert np.array_equal(tr.cpu().numpy()[t], oracle_cuts(g, x, B, 1, False)[0])
        for i, bg in enumerate(blocks):
            r0, r1 = goff[i], goff[i + 1]
            want = oracle.step(bg, x[r0:r1], eta)
            cmp, tol = step_tol(bg, x[r0:r1], want, eta, deco.BF16)
            d = np.abs(xn[r0:r1] - cmp)
            assert np.all(d <= tol), f"step {t} graph {i}: {(d > tol).sum()} off, max {d.max():.3e}"
            mv = np.abs(want - x[r0:r1]) > tol
            moved += int(mv.sum())
            checked += mv.size
        x = xn
    h.round_score()
    bc, bs, bb = h.best()
    assert np.array_equal(oracle.cut_batch(g, deco.bits_to_z(bb, B)), bc)
    assert moved > 0.3 * checked
    # one launch for 10 more steps equals 10 launches of one step
    x_mid = h.read_x().clone()
    h.step(10)
    one = to_np(h.read_x())
    h2 = deco.Handle(G, B=B, x_dtype=deco.BF16, eta=eta, seed=1)
    h2.set_schedule(64, 1 << 30, 0, 128, 2048, 0, 16)
    h2.start(deco.INIT_USER, x0=x_mid)
    for _ in range(10):
        h2.step(1)
    assert np.array_equal(one, to_np(h2.read_x()))
    print(f"uneven batch resident: {h.schedule()}")
    h.destroy()
    h2.destroy()
