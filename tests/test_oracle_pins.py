"""Pins of the CPU oracle against facts the paper and the mathematics fix.

Every check here uses an independent route to the expected value (brute force, dense
linear algebra, closed forms, published known-answer vectors, hand-worked examples), so
a dropped term, a wrong sign or index, or a transposed operand in the oracle fails one
of them. No GPU is involved.
"""
import itertools
import math
import os

import numpy as np
import scipy.sparse
import scipy.sparse.csgraph
import pytest

import oracle
from paper_2509_18612_amd import synth


# ------------------------------------------------------------------ helpers (independent)
def dense_w(g):
    W = np.zeros((g.n, g.n))
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr.astype(np.int64)))
    W[rows, g.col_idx] = 1.0 if g.w is None else g.w
    return W


def all_pm1(n):
    return np.array(list(itertools.product([-1.0, 1.0], repeat=n)))


def load_golden(golden_dir, name):
    path = os.path.join(golden_dir, name)
    g = synth.from_edge_file(path)
    meta = {}
    with open(path) as f:
        for ln in f:
            if ln.startswith("# max_cut"):
                meta["max_cut"] = float(ln.split()[2])
            if ln.startswith("# important"):
                meta["important"] = [int(t) for t in ln.split()[2:]]
    return g, meta


def small_graphs():
    out = [synth.erdos_renyi(9, 0.5, 3), synth.erdos_renyi(11, 0.35, 4), synth.barabasi_albert(10, 2, 5),
           synth.cycle(7), synth.complete(6)]
    wg = synth.erdos_renyi(10, 0.5, 6)
    out.append(synth.with_rademacher_weights(wg, 7))
    rng = np.random.default_rng(8)
    m = wg.nnz // 2
    out.append(synth.with_weights(wg, rng.integers(1, 5, m).astype(np.float32)))
    out.append(synth.with_weights(wg, rng.uniform(0.1, 2.0, m).astype(np.float32)))
    return out


# ------------------------------------------------------------------ CSR + degrees
def test_csr_check_accepts_generators_and_rejects_defects():
    for g in small_graphs() + [synth.barabasi_albert(300, 3, 1), synth.random_regular3(100, 2)]:
        assert oracle.check_csr(g) == 0
    g = synth.cycle(6)
    bad = synth.CSR(g.n, g.row_ptr.copy(), g.col_idx.copy())
    bad.col_idx[0] = 0  # self loop at row 0
    assert oracle.check_csr(bad) == 3
    bad = synth.CSR(g.n, g.row_ptr.copy(), g.col_idx.copy())
    bad.col_idx[0] = 17
    assert oracle.check_csr(bad) == 2
    bad = synth.CSR(g.n, g.row_ptr.copy(), g.col_idx.copy())
    bad.col_idx[[0, 1]] = bad.col_idx[[1, 0]]
    assert oracle.check_csr(bad) == 4
    bad = synth.CSR(g.n, g.row_ptr.copy(), g.col_idx.copy(), np.ones(g.nnz, np.float32))
    bad.w[0] = 2.0
    assert oracle.check_csr(bad) == 5
    bad = synth.CSR(g.n, g.row_ptr.copy(), g.col_idx.copy())
    bad.col_idx[1] = 3  # row 0 now points at 3 but row 3 does not point back
    assert oracle.check_csr(bad) == 5


def test_degrees_match_dense_row_sums():
    for g in small_graphs():
        d, dw, delta = oracle.degrees(g)
        W = dense_w(g)
        assert np.array_equal(d, (W != 0).sum(1))
        assert np.allclose(dw, W.sum(1), rtol=0, atol=1e-12)
        assert delta == d.max()


# ------------------------------------------------------------------ P1/P2/P6: exact cut
@pytest.mark.parametrize("gi", range(8))
def test_cut_equals_three_independent_formulas_on_every_vector(gi):
    """eq. (1) (oracle) == 1/4 (1'W1 - x'Wx) == z'Lz (eq. (5)) == edge count over unordered
    pairs, for every z in {0,1}^n."""
    g = small_graphs()[gi]
    W = dense_w(g)
    L = np.diag(W.sum(1)) - W
    X = all_pm1(g.n)
    Z = (X > 0).astype(np.uint8)
    cuts = oracle.cut_batch(g, Z.T.copy())[0]
    F = 0.25 * (W.sum() - np.einsum("ki,ij,kj->k", X, W, X))
    zLz = np.einsum("ki,ij,kj->k", Z.astype(float), L, Z.astype(float))
    iu = np.triu_indices(g.n, 1)
    pair = np.array([(W[iu] * (z[iu[0]] != z[iu[1]])).sum() for z in Z])
    assert np.allclose(cuts, F, atol=1e-9)
    assert np.allclose(cuts, zLz, atol=1e-9)
    assert np.allclose(cuts, pair, atol=1e-9)
    # x'Lx = 4 Cut on the +-1 vertices (the relaxed objective at the boundary)
    xLx = np.einsum("ki,ij,kj->k", X, L, X)
    assert np.allclose(xLx, 4 * cuts, atol=1e-9)


@pytest.mark.parametrize("gi", range(8))
def test_brute_force_is_the_maximum_over_all_vectors(gi):
    g = small_graphs()[gi]
    X = all_pm1(g.n)
    Z = (X > 0).astype(np.uint8)
    cuts = oracle.cut_batch(g, Z.T.copy())[0]
    best, z = oracle.brute_force(g)
    assert best == pytest.approx(cuts.max(), abs=1e-9)
    assert oracle.cut(g, z) == pytest.approx(best, abs=1e-9)


def test_closed_form_maximum_cuts():
    for n in range(2, 11):
        assert oracle.brute_force(synth.complete(n))[0] == (n * n) // 4
    for n in range(3, 13):
        assert oracle.brute_force(synth.cycle(n))[0] == (n if n % 2 == 0 else n - 1)
    for n in range(2, 12):
        assert oracle.brute_force(synth.star(n))[0] == n - 1
        assert oracle.brute_force(synth.path(n))[0] == n - 1
    for a, b in [(1, 1), (2, 3), (3, 4), (4, 5)]:
        assert oracle.brute_force(synth.complete_bipartite(a, b))[0] == a * b
    for r, c in [(2, 2), (3, 3), (3, 4)]:
        g = synth.grid(r, c)
        assert oracle.brute_force(g)[0] == g.nnz // 2
    assert oracle.brute_force(synth.edgeless(5))[0] == 0
    assert oracle.cut(synth.edgeless(5), np.ones(5, np.uint8)) == 0


@pytest.mark.parametrize("name", ["petersen.txt", "cube_q3.txt"])
def test_golden_textbook_max_cuts(golden_dir, name):
    g, meta = load_golden(golden_dir, name)
    assert oracle.check_csr(g) == 0
    assert oracle.brute_force(g)[0] == meta["max_cut"]


def test_cut_per_graph_in_block_diagonal_batch():
    gs = [synth.erdos_renyi(8, 0.5, 1), synth.cycle(5), synth.star(6)]
    bd = synth.block_diagonal(gs)
    rng = np.random.default_rng(0)
    Z = rng.integers(0, 2, (bd.n, 4)).astype(np.uint8)
    got = oracle.cut_batch(bd, Z)
    for gi, g in enumerate(gs):
        r0, r1 = bd.graph_row_offset[gi], bd.graph_row_offset[gi + 1]
        assert np.array_equal(got[gi], oracle.cut_batch(g, Z[r0:r1].copy())[0])


# ------------------------------------------------------------------ P4: gradients
@pytest.mark.parametrize("gi", [0, 2, 5, 7])
def test_gradient_matches_finite_differences(gi):
    g = small_graphs()[gi]
    W = dense_w(g)
    L = np.diag(W.sum(1)) - W
    rng = np.random.default_rng(gi)
    x = rng.uniform(-1, 1, g.n)
    h = 1e-6

    def F(y):  # cut-form objective, equal to the cut on {-1,1}^n
        return 0.25 * (W.sum() - y @ W @ y)

    def f(y):  # eq. (QUCO)
        return y @ L @ y

    fd_F = np.array([(F(x + h * e) - F(x - h * e)) / (2 * h) for e in np.eye(g.n)])
    fd_f = np.array([(f(x + h * e) - f(x - h * e)) / (2 * h) for e in np.eye(g.n)])
    g_cut = oracle.grad(g, x[:, None], oracle.CUT_FORM)[:, 0]
    g_lap = oracle.grad(g, x[:, None], oracle.LAPLACIAN_FORM)[:, 0]
    assert np.allclose(g_cut, fd_F, rtol=1e-6, atol=1e-7)
    # eq. (6) prints g = L x, which is half the gradient of x'Lx
    assert np.allclose(g_lap, 0.5 * fd_f, rtol=1e-6, atol=1e-7)


# ------------------------------------------------------------------ P3: fixed points
@pytest.mark.parametrize("gi", [0, 1, 2, 5, 6])
@pytest.mark.parametrize("eta", [1e-3, 0.1, 2.0])
def test_cut_form_boundary_fixed_points_are_one_flip_local_optima(gi, eta):
    g = small_graphs()[gi]
    X = all_pm1(g.n)
    Z = (X > 0).astype(np.uint8)
    base = oracle.cut_batch(g, Z.T.copy())[0]
    Xn = oracle.step(g, X.T.copy(), eta, oracle.CUT_FORM).T
    fixed = np.all(Xn == X, axis=1)
    # local optimality by single flips, scored with the exact cut
    local = np.ones(len(X), bool)
    for v in range(g.n):
        Zf = Z.copy()
        Zf[:, v] ^= 1
        local &= oracle.cut_batch(g, Zf.T.copy())[0] <= base
    assert np.array_equal(fixed, local)


@pytest.mark.parametrize("gi", [0, 2, 3, 4, 6])
def test_laplacian_form_every_boundary_point_is_fixed(gi):
    """With non-negative weights x_v (Lx)_v >= 0 on {-1,1}^n, so Proj keeps every vertex
    (Definition of MaxCut fixed points, Sec. 3.1); the null-space points c e_n are stationary
    (Lemma 2)."""
    g = small_graphs()[gi]
    X = all_pm1(g.n)
    Xn = oracle.step(g, X.T.copy(), 0.37, oracle.LAPLACIAN_FORM).T
    assert np.array_equal(Xn, X)
    for c in [-0.5, 0.0, 0.25]:  # dyadic: d_v * c and the neighbour sum are both exact
        x = np.full((g.n, 1), c)
        assert np.array_equal(oracle.step(g, x, 0.5, oracle.LAPLACIAN_FORM), x)
        assert np.array_equal(oracle.grad(g, x, oracle.LAPLACIAN_FORM), np.zeros_like(x))
    x = np.full((g.n, 1), -0.7)
    assert np.allclose(oracle.grad(g, x, oracle.LAPLACIAN_FORM), 0.0, atol=1e-14)


def test_laplacian_form_saturation_is_absorbing():
    g = synth.erdos_renyi(12, 0.4, 2)
    rng = np.random.default_rng(1)
    X = rng.uniform(-1, 1, (g.n, 16))
    X[0, :8] = 1.0
    X[0, 8:] = -1.0
    for _ in range(5):
        X = oracle.step(g, X, 0.3, oracle.LAPLACIAN_FORM)
        assert np.all(X[0, :8] == 1.0) and np.all(X[0, 8:] == -1.0)


@pytest.mark.parametrize("l", [3, 8])
def test_theorem1_lifted_boundary_points_fixed_and_zero_cut_iff_constant_rounding(l):
    # the zero-cut side of the statement needs a connected graph (an isolated vertex can
    # round apart from the rest without cutting an edge)
    g = synth.barabasi_albert(7, 2, 11)
    A = scipy.sparse.csr_matrix((np.ones(g.nnz), g.col_idx, g.row_ptr), shape=(g.n, g.n))
    assert scipy.sparse.csgraph.connected_components(A)[0] == 1
    rng = np.random.default_rng(3)
    Xs = np.where(rng.random((g.n, l * 64)) < 0.5, -1.0, 1.0)
    Xn = oracle.step(g, Xs, 0.2, oracle.LAPLACIAN_FORM)
    assert np.array_equal(Xn, Xs)
    z = oracle.round_signs(Xs, 64, l, lifted=True)
    cuts = oracle.cut_batch(g, z)[0]
    constant = np.all(z == z[0:1], axis=0)
    assert np.array_equal(cuts == 0, constant)
    assert 0 < constant.sum() < constant.size  # both sides of the equivalence occur
    # X = e_n c' gives a zero cut for every c in {-1,1}^l
    for c in itertools.product([-1.0, 1.0], repeat=l):
        X = np.tile(np.repeat(np.array(c), 1)[None, :], (g.n, 1))
        zc = oracle.round_signs(X, 1, l, lifted=True)
        assert oracle.cut(g, zc[:, 0]) == 0


# ------------------------------------------------------------------ P5: linear regime
@pytest.mark.parametrize("form", [oracle.CUT_FORM, oracle.LAPLACIAN_FORM])
def test_linear_regime_matches_eigendecomposition(form):
    g = synth.erdos_renyi(60, 0.1, 5)
    W = dense_w(g)
    M = -0.5 * W if form == oracle.CUT_FORM else np.diag(W.sum(1)) - W
    lam, V = np.linalg.eigh(M)
    rng = np.random.default_rng(9)
    X0 = rng.uniform(-1, 1, (g.n, 5)) * 1e-6
    eta, T = 0.01, 40
    X = X0.copy()
    for _ in range(T):
        X = oracle.step(g, X, eta, form)
    assert np.abs(X).max() < 1  # no clipping happened
    closed = V @ np.diag((1 + eta * lam) ** T) @ V.T @ X0
    assert np.allclose(X, closed, rtol=1e-9, atol=1e-18)


# ------------------------------------------------------------------ P7/P8: symmetry, lifted
def test_negated_start_gives_negated_trajectory_and_equal_cuts():
    g = synth.barabasi_albert(40, 3, 4)
    X = synth.uniform_batch(g.n, 8, 5).astype(np.float64)
    Y = -X
    for _ in range(20):
        X = oracle.step(g, X, 0.1)
        Y = oracle.step(g, Y, 0.1)
        assert np.array_equal(Y, -X)
    assert not np.any(X == 0)
    zx = oracle.round_signs(X, 8)
    zy = oracle.round_signs(Y, 8)
    assert np.array_equal(zy, 1 - zx)
    assert np.array_equal(oracle.cut_batch(g, zx), oracle.cut_batch(g, zy))


def test_lifted_columns_evolve_as_unlifted_runs():
    g = synth.erdos_renyi(30, 0.2, 8)
    B, l = 4, 3
    X = synth.uniform_batch(g.n, l * B, 1).astype(np.float64)
    eta = np.tile(np.array([0.05, 0.1, 0.2, 0.3]), l)
    Xl = oracle.step(g, X, eta)
    for c in range(l * B):
        assert np.array_equal(Xl[:, c:c + 1], oracle.step(g, X[:, c:c + 1], eta[c]))


def test_lifted_rounding_rule_and_tie():
    X = np.array([[0.5, -0.5, 0.1, 0.2],   # v0: b0 sum 0.0 -> 1 (>=); b1: sum 0.3... see below
                  [-0.25, 0.0, -0.2, 0.0]])
    # l = 2, B = 2: init b has components X[:, b] and X[:, 2 + b]
    z = oracle.round_signs(X, 2, 2, lifted=True)
    assert z.tolist() == [[1, 0], [0, 1]]   # v0: 0.6, -0.3 ; v1: -0.45, 0.0 (tie -> 1)
    zu = oracle.round_signs(np.array([[0.0], [-0.0], [1e-30]]), 1)
    assert zu[:, 0].tolist() == [0, 0, 1]   # unlifted eq. (5) is strict


def test_lifted_side_is_taken_on_the_float32_sum_in_component_order():
    """Hand-worked, l = 8: the float32 values of (0.1, 0.2, 0.3, -0.6, 0, 0, 0, 0) add up to
    exactly 0 from the first component on (0.1f + 0.2f rounds to 0.3f, + 0.3f gives 0.6f),
    so the side is 1 (the lifted rule's tie); their exact sum is -2^-27 and the reversed
    float32 sum is negative too, so a double-precision or reordered sum gives side 0."""
    comp = np.array([0.1, 0.2, 0.3, -0.6, 0, 0, 0, 0], np.float32).astype(np.float64)
    assert comp.sum() < 0 and math.fsum(comp[::-1]) == -2.0 ** -27
    z = oracle.round_signs(comp[None, :], 1, 8, lifted=True)
    assert z.tolist() == [[1]]
    z = oracle.round_signs(comp[None, ::-1].copy(), 1, 8, lifted=True)
    assert z.tolist() == [[0]]
    assert oracle.round_signs(comp[None, :], 1, 8, lifted=True, sum_f32=False).tolist() == [[0]]


def test_running_best_strict_improvement_keeps_earliest_step():
    g = synth.cycle(6)
    best = np.full(2, -np.inf)
    step = np.full(2, -1, np.int64)
    zb = np.zeros((6, 2), np.uint8)
    z1 = np.array([[1, 0], [0, 0], [1, 0], [0, 0], [1, 0], [0, 0]], np.uint8)
    z2 = np.array([[0, 0], [1, 0], [0, 0], [1, 0], [0, 0], [1, 0]], np.uint8)
    c1 = oracle.cut_batch(g, z1)[0]
    oracle.best_update(0, c1, z1, best, step, zb)
    c2 = oracle.cut_batch(g, z2)[0]
    oracle.best_update(1, c2, z2, best, step, zb)
    assert best.tolist() == [6.0, 0.0] and step.tolist() == [0, 0]
    assert np.array_equal(zb[:, 0], z1[:, 0])


# ------------------------------------------------------------------ Philox
def test_philox_published_known_answer_vectors(golden_dir):
    n = 0
    with open(os.path.join(golden_dir, "philox4x32_10_kat.txt")) as f:
        for ln in f:
            if ln.startswith("#") or not ln.strip():
                continue
            t = [int(x, 16) for x in ln.split()]
            out = oracle.philox(t[0:4], t[4:6])
            assert [int(x) for x in out] == t[6:10]
            n += 1
    assert n == 3


def test_uniform_init_grid_and_range():
    X = oracle.init_uniform(200, 16, seed=5)
    assert X.min() >= -1.0 and X.max() <= 1.0 - 2.0 ** -23
    assert np.all((X + 1.0) * 2 ** 23 == np.round((X + 1.0) * 2 ** 23))
    assert abs(X.mean()) < 0.02 and abs(X.var() - 1 / 3) < 0.02
    assert np.array_equal(X, oracle.init_uniform(200, 16, seed=5))
    assert not np.array_equal(X, oracle.init_uniform(200, 16, seed=6))
    assert not np.array_equal(X, oracle.init_uniform(200, 16, seed=5, batch=1))


# ------------------------------------------------------------------ P13/P14: DUI, IDI
def test_dui_support_zero_at_max_degree_and_variance():
    g = synth.barabasi_albert(2000, 2, 3)
    d = g.degrees()
    delta = d.max()
    H = oracle.init_dui(g, 64, seed=1)
    half = 1 - d / delta
    assert np.all(np.abs(H) <= half[:, None] + 1e-15)
    assert np.all(H[d == delta] == 0)
    sel = d == d.min()
    emp = H[sel].var()
    assert abs(emp - half[sel][0] ** 2 / 3) < 0.02


def test_idi_threshold_population_statistics():
    g = synth.barabasi_albert(500, 3, 2)
    d = g.degrees().astype(float)
    assert oracle.idi_threshold(g, 0.2) == pytest.approx(d.mean() + 0.2 * d.std(ddof=0), rel=1e-12)


def test_idi_hand_worked_example(golden_dir):
    g, meta = load_golden(golden_dir, "idi_hand6.txt")
    d = g.degrees()
    thr = oracle.idi_threshold(g, 0.2)
    assert list(np.nonzero(d > thr)[0]) == meta["important"]
    H = oracle.init_idi(g, 4096, seed=3)
    assert set(np.unique(H)) <= {-1.0, 1.0}
    same = H[0] == H[1]
    # hubs on the same side: every leaf joins the other side, and the start is optimal
    assert np.all(H[2:, same] == -H[0:1, same])
    z = (H[:, same] > 0).astype(np.uint8)
    assert oracle.brute_force(g)[0] == 8
    assert np.all(oracle.cut_batch(g, z)[0] == 8)
    # hubs apart: every leaf ties and flips a fair coin
    frac = (H[2:, ~same] > 0).mean()
    assert 0.45 < frac < 0.55
    # the hub signs themselves are fair
    assert 0.45 < (H[0] > 0).mean() < 0.55


def test_idi_star_and_regular_special_cases():
    g = synth.star(30)
    H = oracle.init_idi(g, 32, seed=1)
    assert np.all(H[1:] == -H[0:1])          # leaves opposite the important centre
    z = (H > 0).astype(np.uint8)
    assert np.all(oracle.cut_batch(g, z)[0] == 29)
    r = synth.random_regular3(50, 1)         # sigma = 0: nobody is important, all tie
    Hr = oracle.init_idi(r, 256, seed=2)
    assert set(np.unique(Hr)) == {-1.0, 1.0}
    assert 0.45 < (Hr > 0).mean() < 0.55


def test_gauss_start_moments_and_scaling():
    M = np.ones((400, 64))
    X = oracle.init_gauss(M, 0.8, 1.0, seed=4)
    eps = X - 1.0
    eps = eps[np.abs(X) < 1]                 # values not clipped
    X2 = oracle.init_gauss(np.zeros((400, 64)), 0.8, 1e4, seed=4)
    assert np.abs(X2).max() < 1e-3
    assert abs(X2.std() * 1e4 - math.sqrt(0.8)) < 0.03
    assert abs(X2.mean() * 1e4) < 0.03


# ------------------------------------------------------------------ P15: search
def test_evo_next_ranks_keeps_top_half_and_bounds():
    fit = np.array([5.0, 9.0, 9.0, 1.0, 7.0, 3.0, 8.0, 2.0])
    eq = np.linspace(-4, -1, 8)
    el = np.linspace(-1, -4, 8)
    lk = np.array([1, 2, 3, 4, 1, 2, 3, 4], np.int32)
    a, b, c = oracle.evo_next(fit, eq, el, lk, seed=1, rnd=0)
    order = [1, 2, 6, 4]  # descending fitness, ties to the lower index
    assert np.array_equal(a[:4], eq[order]) and np.array_equal(b[:4], el[order])
    assert np.array_equal(c[:4], lk[order])
    assert np.all((a >= -4) & (a <= -1) & (b >= -4) & (b <= -1))
    assert np.all((c >= 1) & (c <= 4))
    for j in range(4):  # bottom member j+4 perturbs ranked member j
        assert abs(a[4 + j] - a[j]) <= 0.2 * 6 and abs(int(c[4 + j]) - int(c[j])) <= 1
    a2, b2, c2 = oracle.evo_next(fit, eq, el, lk, seed=1, rnd=0)
    assert np.array_equal(a, a2) and np.array_equal(b, b2) and np.array_equal(c, c2)


def load_evo_hand(golden_dir):
    vals = {}
    with open(os.path.join(golden_dir, "evo_hand.txt")) as f:
        for ln in f:
            if ln.startswith("#") or not ln.strip():
                continue
            k, *v = ln.split()
            vals[k] = v
    return vals


def test_evo_init_hand_worked_member(golden_dir):
    """One member of the initial population worked out by hand from its Philox words
    (tests/golden/evo_hand.txt): e = -4 + 3 u24, l = 1 + r mod lmax, T = T_lo + r mod range."""
    h = load_evo_hand(golden_dir)
    k = int(h["init_member"][0])
    eq, el, lk, tq, tl = oracle.evo_init(3, int(h["init_seed"][0]), 4, (3000, 10000), (100, 500))
    num, den = (int(x) for x in h["init_eq_num"])
    assert eq[k] == num / den
    num, den = (int(x) for x in h["init_el_num"])
    assert el[k] == num / den
    assert lk[k] == int(h["init_l"][0]) and tq[k] == int(h["init_tq"][0]) and tl[k] == int(h["init_tl"][0])


def test_evo_init_bounds_uniformity_and_determinism():
    """Sec. 4.3 draws the initial combinations uniformly from the bounds: exponents on
    [-4, -1), l on {1..lmax}, counts on their ranges; members differ; same seed, same draw."""
    K = 4000
    eq, el, lk, tq, tl = oracle.evo_init(K, 3, 4, (3000, 10000), (100, 500))
    for e in (eq, el):
        assert np.all((e >= -4.0) & (e < -1.0))
        assert abs(e.mean() + 2.5) < 0.05 and abs(e.std() - 3 / math.sqrt(12)) < 0.03
        hist = np.histogram(e, bins=6, range=(-4, -1))[0]
        assert np.all(np.abs(hist - K / 6) < 5 * math.sqrt(K / 6))
    assert np.corrcoef(eq, el)[0, 1] ** 2 < 0.01          # the two exponents draw apart
    counts = np.bincount(lk, minlength=5)[1:]
    assert counts.min() > 0.2 * K and counts.max() < 0.3 * K and lk.min() == 1 and lk.max() == 4
    assert tq.min() >= 3000 and tq.max() <= 10000 and abs(tq.mean() - 6500) < 120
    assert tl.min() >= 100 and tl.max() <= 500 and abs(tl.mean() - 300) < 8
    again = oracle.evo_init(K, 3, 4, (3000, 10000), (100, 500))
    for x, y in zip((eq, el, lk, tq, tl), again):
        assert np.array_equal(x, y)
    other = oracle.evo_init(K, 4, 4, (3000, 10000), (100, 500))
    assert not np.array_equal(eq, other[0])
    fixed = oracle.evo_init(8, 3, 1, (400, 400), (200, 200))  # one-point ranges
    assert np.all(fixed[2] == 1) and np.all(fixed[3] == 400) and np.all(fixed[4] == 200)


def test_evo_round_hand_worked_k6(golden_dir):
    """A whole evolution round for K = 6 worked out by hand (tests/golden/evo_hand.txt):
    ranking with ties to the lower index, the kept half in rank order, slot K/2 + j from
    ranked member j, Box-Muller perturbation of both exponents with clipping to [-4, -1], l
    moved by U{-1,0,1} and clipped, and T' = floor(T0 (1 + 0.2 (2 eps' - 1))) clipped to
    [3000, 10000] (one child clipped at each end)."""
    h = load_evo_hand(golden_dir)
    fit = np.array([float(x) for x in h["evo_fitness"]])
    T = np.array([int(x) for x in h["evo_T"]], np.int32)
    got = oracle.evo_next_steps(fit, T, 3000, 10000, 7, 0, 0)
    assert np.array_equal(got, [int(x) for x in h["evo_T_out"]])
    eq = np.array([float(x) for x in h["evo_eq"]])
    el = np.array([float(x) for x in h["evo_el"]])
    lk = np.array([int(x) for x in h["evo_l"]], np.int32)
    a, b, c = oracle.evo_next(fit, eq, el, lk, 7, 0, lmax=4)
    assert np.allclose(a, [float(x) for x in h["evo_eq_out"]], rtol=0, atol=1e-12)
    assert np.allclose(b, [float(x) for x in h["evo_el_out"]], rtol=0, atol=1e-12)
    assert np.array_equal(c, [int(x) for x in h["evo_l_out"]])


def test_gauss_start_box_muller_hand_value(golden_dir):
    """One Gaussian draw worked out by hand from its Philox words (cos branch, u1 offset by
    one grid step so that it is never 0): X = (0 + sqrt(1) eps) / 4 at seed 12."""
    h = load_evo_hand(golden_dir)
    X = oracle.init_gauss(np.zeros((1, 1)), 1.0, 4.0, int(h["gauss_seed"][0]), 0)
    assert abs(X[0, 0] * 4.0 - float(h["gauss_eps"][0])) <= 1e-13


def test_step_count_perturbation_formula():
    for T0 in [3000, 5000, 9999]:
        for e in [0.0, 0.25, 0.5, 0.999]:
            want = math.floor(T0 * (1 + 0.2 * (2 * e - 1)))
            assert oracle.perturb_T(T0, e, 3000, 10000) == min(max(want, 3000), 10000)


# ------------------------------------------------------------------ batches and DECO
def test_run_batch_best_equals_cut_of_best_vector_and_bounded_by_optimum():
    g = synth.erdos_renyi(16, 0.4, 21)
    opt = oracle.brute_force(g)[0]
    X0 = oracle.init_uniform(g.n, 32, seed=3)
    _, best, bstep, zb = oracle.run_batch(g, X0, 32, 1, False, 0.1, 50)
    assert np.array_equal(best, oracle.cut_batch(g, zb)[0])
    assert np.all(best <= opt) and np.all(bstep >= 0) and best.max() >= 0.9 * opt


def test_deco_result_is_consistent_and_beats_greedy_bound():
    g = synth.erdos_renyi(18, 0.35, 2)
    opt = oracle.brute_force(g)[0]
    best, z, trace, _ = oracle.deco(g, B=32, K=8, lmax=4, rounds=3, evo_rounds=2, Tq=60, Tl=30, seed=1)
    assert best == oracle.cut(g, z)
    assert best <= opt and np.all(np.diff(trace) >= 0)
    gb, gz = oracle.greedy(g, orders=4, seed=1)
    assert gb == oracle.cut(g, gz) and gb >= (g.nnz // 2) / 2  # greedy's 1/2 guarantee
    assert best >= gb


def test_deco_deterministic_in_seed():
    g = synth.barabasi_albert(60, 2, 5)
    r1 = oracle.deco(g, B=16, K=4, rounds=2, evo_rounds=1, Tq=30, Tl=20, seed=7)
    r2 = oracle.deco(g, B=16, K=4, rounds=2, evo_rounds=1, Tq=30, Tl=20, seed=7)
    assert r1[0] == r2[0] and np.array_equal(r1[1], r2[1])


def test_deco_draws_its_population_and_searches_step_counts():
    """Without explicit genes the loop starts from the drawn population (with evo_rounds = 0
    the genes come back unchanged), and with both counts searched the final counts stay in
    their ranges; the result is the exact cut of its vector and never beats brute force."""
    g = synth.erdos_renyi(16, 0.4, 9)
    opt = oracle.brute_force(g)[0]
    best, z, _, genes = oracle.deco(g, B=16, K=4, lmax=3, rounds=1, evo_rounds=0, Tq=30, Tl=20, seed=11)
    want = oracle.evo_init(4, 11, 3, (30, 30), (20, 20))
    for x, y in zip(genes, want):
        assert np.array_equal(x, y)
    best, z, _, (eq, el, lk, tq, tl) = oracle.deco(g, B=16, K=4, lmax=3, rounds=3, evo_rounds=2, Tq=40, Tl=30,
                                                  seed=11, Tq_min=10, Tl_min=5)
    assert best == oracle.cut(g, z) <= opt
    assert np.all((tq >= 10) & (tq <= 40)) and np.all((tl >= 5) & (tl <= 30))
    assert np.all(tq == tq[0]) and np.all(lk == lk[0])  # the best genes everywhere after the search


def test_run_batch_member_counts_stop_columns():
    """A column whose count is reached keeps its iterate (a step of size 0) while the batch
    runs on: equal to running that column alone for its own count."""
    g = synth.erdos_renyi(20, 0.3, 4)
    X0 = oracle.init_uniform(g.n, 4, seed=5)
    Tb = np.array([3, 7, 0, 7])
    X, best, _, _ = oracle.run_batch(g, X0, 4, 1, False, 0.1, 7, T_b=Tb)
    for b in range(4):
        Xb, bb, _, _ = oracle.run_batch(g, X0[:, b:b + 1], 1, 1, False, 0.1, int(Tb[b]))
        assert np.array_equal(X[:, b], Xb[:, 0]) and best[b] == bb[0]


def test_bf16_rounding_emulation():
    x = np.array([1.0, 1.00390625, 1.005859375, -2.5, 3.0e-39, 65504.0], np.float32)
    y = oracle.to_bf16(x)
    assert y[0] == 1.0
    assert y[1] == 1.0                   # 1 + 2^-8 is a tie between 1 and 1+2^-7: to even (1)
    assert y[2] == np.float32(1.0078125)  # 1 + 1.5*2^-8 rounds up
    assert y[3] == -2.5
    bits = y.view(np.uint32)
    assert np.all(bits & 0xFFFF == 0)


def test_momentum_step_pins():
    """Heavy-ball momentum step (reading of Sec. 4.2 / Sec. 5): mu = 0 is the plain step; a
    single edge worked by hand; two steps from V = 0 unroll to mu G0 + G1; the box holds."""
    import oracle
    from paper_2509_18612_amd import synth
    g = synth.erdos_renyi(60, 0.1, 4)
    rng = np.random.default_rng(8)
    X = rng.uniform(-1, 1, (g.n, 5))
    V = rng.uniform(-2, 2, (g.n, 5))
    Xm, Vm = oracle.step_momentum(g, X, V, 0.07, 0.0)
    assert np.allclose(Xm, oracle.step(g, X, 0.07), rtol=0, atol=1e-15)
    # one edge 0-1, cut form G = -1/2 W X: G0 = -x1/2, G1 = -x0/2 (worked by hand)
    e = synth.from_edges(2, np.array([0]), np.array([1]))
    Xe = np.array([[0.2], [-0.4]])
    Ve = np.array([[0.1], [-0.3]])
    Xn, Vn = oracle.step_momentum(e, Xe, Ve, 0.5, 0.9)
    assert np.allclose(Vn, [[0.29], [-0.37]], rtol=0, atol=1e-15)   # 0.09 + 0.2, -0.27 - 0.1
    assert np.allclose(Xn, [[0.345], [-0.585]], rtol=0, atol=1e-15)  # 0.2 + 0.145, -0.4 - 0.185
    # two steps from V = 0: V2 = mu G(X0) + G(X1)
    X0 = rng.uniform(-0.3, 0.3, (g.n, 3))
    X1, V1 = oracle.step_momentum(g, X0, np.zeros_like(X0), 0.01, 0.9)
    X2, V2 = oracle.step_momentum(g, X1, V1, 0.01, 0.9)
    assert np.allclose(V2, 0.9 * oracle.grad(g, X0) + oracle.grad(g, X1), rtol=0, atol=1e-13)
    assert np.allclose(X2, np.clip(X1 + 0.01 * V2, -1, 1), rtol=0, atol=1e-15)
    # a large step lands on the box
    Xb, _ = oracle.step_momentum(g, X, V, 50.0, 0.9)
    assert np.all(np.abs(Xb) <= 1.0) and np.any(np.abs(Xb) == 1.0)
