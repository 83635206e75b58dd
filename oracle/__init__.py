"""CPU FP64 oracle of the DECO batched projected-gradient MaxCut method.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package; the GPU library never does, and the two share no code.
The arithmetic lives in ``deco_oracle.c`` (plain C loops, double precision) and, for the
learned initialiser, in ``mpnn.py`` (numpy, float64). This wrapper only marshals numpy
arrays. See the header of ``deco_oracle.c`` for the readings of the paper it takes.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "deco_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_BUILD, "libdeco_oracle.so")
_lib = None

CUT_FORM = 0
LAPLACIAN_FORM = 1


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, single thread)."""
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
                               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _L():
    global _lib
    if _lib is None:
        _lib = ct.CDLL(build())
        _declare(_lib)
    return _lib


P = ct.c_void_p
I64 = ct.c_int64
I32 = ct.c_int32
U64 = ct.c_uint64
U32 = ct.c_uint32
D = ct.c_double


def _declare(L):
    L.orc_csr_check.argtypes = [I64, P, P, P]
    L.orc_csr_check.restype = ct.c_int
    L.orc_degrees.argtypes = [I64, P, P, P, P]
    L.orc_degrees.restype = I64
    L.orc_step.argtypes = [I64, P, P, P, I64, P, P, P, ct.c_int]
    L.orc_grad.argtypes = [I64, P, P, P, I64, P, P, ct.c_int]
    L.orc_round.argtypes = [I64, I64, I64, ct.c_int, ct.c_int, P, P]
    L.orc_cut_batch.argtypes = [I64, I64, P, P, P, I64, P, P]
    L.orc_best_update.argtypes = [I64, I64, I64, P, P, P, P, P]
    L.orc_philox.argtypes = [P, P, P]
    L.orc_init_uniform.argtypes = [I64, I64, U64, U32, P]
    L.orc_init_dui.argtypes = [I64, P, I64, U64, U32, P]
    L.orc_idi_threshold.argtypes = [I64, P, D]
    L.orc_idi_threshold.restype = D
    L.orc_init_idi.argtypes = [I64, I64, P, P, P, I64, D, U64, U32, P]
    L.orc_init_gauss.argtypes = [I64, I64, P, D, D, U64, U32, P]
    L.orc_evo_next.argtypes = [I64, P, P, P, P, D, D, I32, U64, U32, P, P, P]
    L.orc_evo_next_steps.argtypes = [I64, P, P, I64, I64, U64, U32, U32, P]
    L.orc_evo_init.argtypes = [I64, D, D, I32, I64, I64, I64, I64, U64, P, P, P, P, P]
    L.orc_perturb_T.argtypes = [I64, D, I64, I64]
    L.orc_perturb_T.restype = I64
    L.orc_run_batch.argtypes = [I64, P, P, P, I64, I64, ct.c_int, ct.c_int, P, I64, P, I64, P, P, P, P]
    L.orc_deco.argtypes = [I64, P, P, P, I64, I64, I32, I64, I64, I64, I64, I64, I64, ct.c_int, D, D, D, U64,
                           P, P, P, P, P, P, P]
    L.orc_deco.restype = D
    L.orc_brute_force.argtypes = [I64, P, P, P, P]
    L.orc_brute_force.restype = D
    L.orc_greedy.argtypes = [I64, P, P, P, I64, U64, P]
    L.orc_greedy.restype = D


def _p(a):
    return None if a is None else a.ctypes.data_as(ct.c_void_p)


class Graph:
    """The oracle's own copy of a CSR graph (int64 row_ptr, int32 col, float64 weights)."""

    def __init__(self, csr):
        self.n = int(csr.n)
        self.rp = np.ascontiguousarray(csr.row_ptr, dtype=np.int64)
        self.col = np.ascontiguousarray(csr.col_idx, dtype=np.int32)
        self.w = None if csr.w is None else np.ascontiguousarray(csr.w, dtype=np.float64)
        off = getattr(csr, "graph_row_offset", None)
        self.goff = (np.array([0, self.n], np.int64) if off is None
                     else np.asarray(off, dtype=np.int64))

    @property
    def nnz(self):
        return int(self.col.shape[0])

    @property
    def num_graphs(self):
        return int(self.goff.shape[0] - 1)


def _g(g):
    return g if isinstance(g, Graph) else Graph(g)


def check_csr(g) -> int:
    g = _g(g)
    return int(_L().orc_csr_check(g.n, _p(g.rp), _p(g.col), _p(g.w)))


def degrees(g):
    g = _g(g)
    d = np.zeros(g.n, np.int64)
    dw = np.zeros(g.n, np.float64)
    delta = _L().orc_degrees(g.n, _p(g.rp), _p(g.w), _p(d), _p(dw))
    return d, dw, int(delta)


def _eta_cols(eta, C):
    e = np.asarray(eta, dtype=np.float64)
    if e.ndim == 0:
        e = np.full(C, float(e))
    return np.ascontiguousarray(e)


def step(g, X, eta, form=CUT_FORM) -> np.ndarray:
    """One projected step X -> Proj(X + eta*G); eta scalar or per column."""
    g = _g(g)
    X = np.ascontiguousarray(X, dtype=np.float64)
    C = X.shape[1]
    Xn = np.empty_like(X)
    e = _eta_cols(eta, C)
    _L().orc_step(g.n, _p(g.rp), _p(g.col), _p(g.w), C, _p(X), _p(Xn), _p(e), form)
    return Xn


def step_momentum(g, X, V, eta, mu, form=CUT_FORM):
    """One projected step with heavy-ball momentum (Sec. 4.2 says PGA runs with momentum in
    practice and Sec. 5 uses 0.9, without the update rule; the reading taken is the
    heavy-ball form): V' = mu V + G(X), X' = Proj(X + eta V'). Returns (X', V')."""
    G = grad(g, X, form)
    Vn = float(mu) * np.asarray(V, dtype=np.float64) + G
    e = _eta_cols(eta, Vn.shape[1])
    Xn = np.clip(np.asarray(X, dtype=np.float64) + e[None, :] * Vn, -1.0, 1.0)
    return Xn, Vn


def grad(g, X, form=CUT_FORM) -> np.ndarray:
    g = _g(g)
    X = np.ascontiguousarray(X, dtype=np.float64)
    G = np.empty_like(X)
    _L().orc_grad(g.n, _p(g.rp), _p(g.col), _p(g.w), X.shape[1], _p(X), _p(G), form)
    return G


def round_signs(X, B, l=1, lifted=False, sum_f32=True) -> np.ndarray:
    """z (n x B uint8) from X (n x l*B) by eq. (5) (unlifted) or the lifted rule."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    n = X.shape[0]
    assert X.shape[1] == l * B
    z = np.empty((n, B), np.uint8)
    _L().orc_round(n, B, l, int(bool(lifted)), int(bool(sum_f32)), _p(X), _p(z))
    return z


def cut_batch(g, z) -> np.ndarray:
    """Cut of every column of z (n x B) per graph: returns (num_graphs, B) float64."""
    g = _g(g)
    z = np.ascontiguousarray(z, dtype=np.uint8)
    if z.ndim == 1:
        z = z[:, None]
    B = z.shape[1]
    out = np.zeros((g.num_graphs, B), np.float64)
    for gi in range(g.num_graphs):
        row = np.zeros(B, np.float64)
        _L().orc_cut_batch(int(g.goff[gi]), int(g.goff[gi + 1]), _p(g.rp), _p(g.col), _p(g.w), B,
                           _p(z), _p(row))
        out[gi] = row
    return out


def cut(g, z) -> float:
    return float(cut_batch(g, np.asarray(z, np.uint8).reshape(-1, 1))[0, 0])


def best_update(t, cut_t, z, best, best_step, z_best):
    n, B = z.shape
    _L().orc_best_update(n, B, t, _p(np.ascontiguousarray(cut_t, np.float64)),
                         _p(np.ascontiguousarray(z, np.uint8)), _p(best), _p(best_step), _p(z_best))


def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    _L().orc_philox(_p(c), _p(k), _p(out))
    return out


def init_uniform(n, C, seed, batch=0) -> np.ndarray:
    X = np.empty((n, C), np.float64)
    _L().orc_init_uniform(n, C, seed, batch, _p(X))
    return X


def init_dui(g, C, seed, batch=0) -> np.ndarray:
    g = _g(g)
    H = np.empty((g.n, C), np.float64)
    _L().orc_init_dui(g.n, _p(g.rp), C, seed, batch, _p(H))
    return H


def idi_threshold(g, beta=0.2) -> float:
    g = _g(g)
    return float(_L().orc_idi_threshold(g.n, _p(g.rp), beta))


def init_idi(g, C, seed, batch=0, beta=0.2) -> np.ndarray:
    """IDI sign matrix (n x C, entries +-1), each graph of a batch on its own statistics."""
    g = _g(g)
    H = np.zeros((g.n, C), np.float64)
    for gi in range(g.num_graphs):
        _L().orc_init_idi(int(g.goff[gi]), int(g.goff[gi + 1]), _p(g.rp), _p(g.col), _p(g.w), C,
                          beta, seed, batch, _p(H))
    return H


def init_gauss(M, s2, scale, seed, batch=0) -> np.ndarray:
    M = np.ascontiguousarray(M, dtype=np.float64)
    n, C = M.shape
    X = np.empty_like(M)
    _L().orc_init_gauss(n, C, _p(M), s2, scale, seed, batch, _p(X))
    return X


def evo_next(fitness, eq, el, l, seed, rnd, lo=-4.0, hi=-1.0, lmax=4):
    K = len(fitness)
    f = np.ascontiguousarray(fitness, np.float64)
    a = np.ascontiguousarray(eq, np.float64)
    b = np.ascontiguousarray(el, np.float64)
    c = np.ascontiguousarray(l, np.int32)
    ao, bo, co = np.zeros(K), np.zeros(K), np.zeros(K, np.int32)
    _L().orc_evo_next(K, _p(f), _p(a), _p(b), _p(c), lo, hi, lmax, seed, rnd, _p(ao), _p(bo), _p(co))
    return ao, bo, co


def evo_next_steps(fitness, T, Tl, Tu, seed, rnd, gene=0):
    """Step counts after one evolution round (Sec. 4.3), paired with evo_next's ranking;
    gene 0 is the unlifted count, 1 the lifted one (separate draws)."""
    K = len(fitness)
    f = np.ascontiguousarray(fitness, np.float64)
    t = np.ascontiguousarray(T, np.int32)
    out = np.zeros(K, np.int32)
    _L().orc_evo_next_steps(K, _p(f), _p(t), Tl, Tu, seed, rnd, gene, _p(out))
    return out


def evo_init(K, seed, lmax=4, Tq=(1, 1), Tl=(1, 1), lo=-4.0, hi=-1.0):
    """Initial population of the search (Sec. 4.3): per member e_q, e_l ~ U[lo, hi),
    l ~ U{1..lmax}, T_q ~ U{Tq[0]..Tq[1]}, T_l ~ U{Tl[0]..Tl[1]}. Returns (eq, el, l, tq, tl)."""
    eq, el = np.zeros(K), np.zeros(K)
    l, tq, tl = np.zeros(K, np.int32), np.zeros(K, np.int32), np.zeros(K, np.int32)
    _L().orc_evo_init(K, lo, hi, lmax, int(Tq[0]), int(Tq[1]), int(Tl[0]), int(Tl[1]), seed, _p(eq), _p(el),
                      _p(l), _p(tq), _p(tl))
    return eq, el, l, tq, tl


def perturb_T(T0, eps_u, Tl, Tu) -> int:
    return int(_L().orc_perturb_T(T0, eps_u, Tl, Tu))


def run_batch(g, X, B, l, lifted, eta_b, T, form=CUT_FORM, score_every=1, T_b=None):
    """Alg. 1 (l = 1, unlifted) or Alg. 2 (lifted): returns (X_T, best, best_step, z_best).
    T_b: optional per-initialisation step counts (columns past their count keep still)."""
    g = _g(g)
    X = np.array(X, dtype=np.float64, order="C", copy=True)
    best = np.full(B, -np.inf)
    bstep = np.full(B, -1, np.int64)
    zb = np.zeros((g.n, B), np.uint8)
    e = _eta_cols(eta_b, B)
    tb = None if T_b is None else np.ascontiguousarray(T_b, np.int64)
    _L().orc_run_batch(g.n, _p(g.rp), _p(g.col), _p(g.w), B, l, int(bool(lifted)), form, _p(e), T, _p(tb),
                       score_every, _p(X), _p(best), _p(bstep), _p(zb))
    return X, best, bstep, zb


def deco(g, B=64, K=8, lmax=4, rounds=4, evo_rounds=2, Tq=200, Tl=100, form=CUT_FORM, beta=0.2,
         s2=0.8, scale=1e4, seed=0, eq=None, el=None, l=None, Tq_min=0, Tl_min=0):
    """pDECO (Alg. 3) with the column-group population; returns (best_cut, z, trace, genes).
    The initial genes are drawn by evo_init (Sec. 4.3) unless eq / el / l are given; the step
    counts are searched in [Tq_min, Tq] and [Tl_min, Tl] when the minimum is positive."""
    g = _g(g)
    assert B % K == 0
    d_eq, d_el, d_l, d_tq, d_tl = evo_init(K, seed, lmax, (Tq_min if Tq_min > 0 else Tq, Tq),
                                           (Tl_min if Tl_min > 0 else Tl, Tl))
    eq = d_eq if eq is None else np.array(eq, np.float64)
    el = d_el if el is None else np.array(el, np.float64)
    lk = d_l if l is None else np.array(l, np.int32)
    tq, tl = d_tq.copy(), d_tl.copy()
    trace = np.zeros(rounds)
    z = np.zeros(g.n, np.uint8)
    best = _L().orc_deco(g.n, _p(g.rp), _p(g.col), _p(g.w), B, K, lmax, rounds, evo_rounds, Tq, Tl, Tq_min,
                         Tl_min, form, beta, s2, scale, seed, _p(eq), _p(el), _p(lk), _p(tq), _p(tl), _p(trace),
                         _p(z))
    return float(best), z, trace, (eq, el, lk, tq, tl)


def brute_force(g):
    g = _g(g)
    z = np.zeros(max(g.n, 1), np.uint8)
    best = _L().orc_brute_force(g.n, _p(g.rp), _p(g.col), _p(g.w), _p(z))
    return float(best), z[:g.n]


def greedy(g, orders=8, seed=0):
    g = _g(g)
    z = np.zeros(max(g.n, 1), np.uint8)
    best = _L().orc_greedy(g.n, _p(g.rp), _p(g.col), _p(g.w), orders, seed, _p(z))
    return float(best), z[:g.n]


# ----------------------------------------------------------------------------------------
# Storage-precision emulation (float32 -> bfloat16 by round-to-nearest-even on the bits).
# ----------------------------------------------------------------------------------------
def to_bf16(x) -> np.ndarray:
    """Round float32 values to bfloat16 (RNE), returned widened back to float32."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32)
    nan = np.isnan(f)
    if nan.any():
        out = out.copy()
        out[nan] = np.float32(np.nan)
    return out
