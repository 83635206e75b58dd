"""Seeded synthetic inputs: graphs in symmetric CSR form and random starting batches.

This module is shared by the GPU library's tests and benchmark and by the CPU oracle's
tests. It holds none of the method's arithmetic: it only draws graphs of the families the
paper evaluates on (Erdos-Renyi, Sec. 5 datasets; Barabasi-Albert and random regular graphs
as further synthetic families) and packs them as CSR.

CSR convention (both directions stored, rows sorted by column, no self-loops):
    row_ptr  int32[n+1]
    col_idx  int32[nnz]
    w        float32[nnz] or None (unit weights)
Every generator is deterministic in its integer seed (numpy PCG64).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


@dataclass
class CSR:
    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    w: Optional[np.ndarray] = None
    # Block-diagonal batches: graph g owns rows [graph_row_offset[g], graph_row_offset[g+1]).
    graph_row_offset: Optional[np.ndarray] = None
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    @property
    def num_graphs(self) -> int:
        return 1 if self.graph_row_offset is None else int(self.graph_row_offset.shape[0] - 1)

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))


def from_edges(n: int, u: np.ndarray, v: np.ndarray, w: Optional[np.ndarray] = None,
               name: str = "") -> CSR:
    """Undirected edge list (each edge once, u != v, no duplicates) -> symmetric sorted CSR."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    src = np.concatenate([u, v])
    dst = np.concatenate([v, u])
    order = np.lexsort((dst, src))
    src = src[order]
    dst = dst[order]
    counts = np.bincount(src, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("graph too large for int32 CSR")
    ww = None
    if w is not None:
        w = np.asarray(w, dtype=np.float32)
        ww = np.concatenate([w, w])[order].astype(np.float32)
    return CSR(n=n, row_ptr=row_ptr.astype(np.int32), col_idx=dst.astype(np.int32), w=ww, name=name)


def erdos_renyi(n: int, p: float, seed: int) -> CSR:
    """G(n, p): every unordered pair is an edge independently with probability p."""
    rng = np.random.Generator(np.random.PCG64(seed))
    us, vs = [], []
    chunk = max(1, min(n, (1 << 24) // max(n, 1)))
    for r0 in range(0, n, chunk):
        r1 = min(n, r0 + chunk)
        draw = rng.random((r1 - r0, n), dtype=np.float32) < np.float32(p)
        rows, cols = np.nonzero(draw)
        rows = rows + r0
        keep = cols > rows
        us.append(rows[keep])
        vs.append(cols[keep])
    u = np.concatenate(us) if us else np.zeros(0, np.int64)
    v = np.concatenate(vs) if vs else np.zeros(0, np.int64)
    return from_edges(n, u, v, name=f"ER({n},{p})")


def barabasi_albert(n: int, m: int, seed: int) -> CSR:
    """Preferential attachment: a star K_{1,m} on nodes 0..m, then every new node attaches
    to m distinct existing nodes chosen with probability proportional to their degree."""
    if m < 1 or n <= m:
        raise ValueError("need 1 <= m < n")
    rng = np.random.Generator(np.random.PCG64(seed))
    eu = np.empty(m * (n - m), dtype=np.int64)
    ev = np.empty(m * (n - m), dtype=np.int64)
    ne = 0
    # 'ends' lists every edge endpoint, so a uniform pick from it is degree-proportional.
    ends = np.empty(2 * m * (n - m), dtype=np.int64)
    ne_ends = 0
    for leaf in range(1, m + 1):
        eu[ne], ev[ne] = 0, leaf
        ne += 1
        ends[ne_ends], ends[ne_ends + 1] = 0, leaf
        ne_ends += 2
    for new in range(m + 1, n):
        chosen = set()
        while len(chosen) < m:
            picks = ends[rng.integers(0, ne_ends, size=2 * m)]
            for t in picks:
                if len(chosen) < m:
                    chosen.add(int(t))
        for t in sorted(chosen):
            eu[ne], ev[ne] = t, new
            ne += 1
            ends[ne_ends], ends[ne_ends + 1] = t, new
            ne_ends += 2
    return from_edges(n, eu[:ne], ev[:ne], name=f"BA({n},{m})")


def random_regular3(n: int, seed: int, max_tries: int = 1000) -> CSR:
    """Uniform random 3-regular graph by the pairing (configuration) model: pair the 3n
    points by a uniform perfect matching; restart when a loop or a multi-edge appears."""
    if (3 * n) % 2 or n < 4:
        raise ValueError("3-regular needs even n >= 4")
    rng = np.random.Generator(np.random.PCG64(seed))
    for _ in range(max_tries):
        pts = rng.permutation(3 * n)
        a = pts[0::2] // 3
        b = pts[1::2] // 3
        if np.any(a == b):
            continue
        lo = np.minimum(a, b)
        hi = np.maximum(a, b)
        key = lo.astype(np.int64) * n + hi
        if np.unique(key).shape[0] != key.shape[0]:
            continue
        return from_edges(n, lo, hi, name=f"3reg({n})")
    raise RuntimeError("pairing model did not produce a simple graph")


def with_rademacher_weights(g: CSR, seed: int) -> CSR:
    """Give every undirected edge an independent weight in {-1, +1} (probability 1/2 each),
    stored identically in both directions."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = g.n
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(g.row_ptr.astype(np.int64)))
    cols = g.col_idx.astype(np.int64)
    upper = cols > rows
    m = int(upper.sum())
    s = np.where(rng.random(m) < 0.5, -1.0, 1.0).astype(np.float32)
    return from_edges(n, rows[upper], cols[upper], s, name=g.name + "+pm1")


def with_weights(g: CSR, values: np.ndarray) -> CSR:
    """Attach per-undirected-edge weights (ordered like the upper-triangle entries in CSR order)."""
    n = g.n
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(g.row_ptr.astype(np.int64)))
    cols = g.col_idx.astype(np.int64)
    upper = cols > rows
    return from_edges(n, rows[upper], cols[upper], np.asarray(values, np.float32), name=g.name + "+w")


def block_diagonal(graphs: List[CSR]) -> CSR:
    """Concatenate graphs into one block-diagonal CSR with graph_row_offset."""
    offs = np.zeros(len(graphs) + 1, dtype=np.int64)
    for i, g in enumerate(graphs):
        offs[i + 1] = offs[i] + g.n
    nnz_offs = np.zeros(len(graphs) + 1, dtype=np.int64)
    for i, g in enumerate(graphs):
        nnz_offs[i + 1] = nnz_offs[i] + g.nnz
    if nnz_offs[-1] >= 2**31 or offs[-1] >= 2**31:
        raise ValueError("batch too large for int32 CSR")
    row_ptr = np.concatenate([g.row_ptr[:-1].astype(np.int64) + nnz_offs[i] for i, g in enumerate(graphs)]
                             + [np.array([nnz_offs[-1]])])
    col_idx = np.concatenate([g.col_idx.astype(np.int64) + offs[i] for i, g in enumerate(graphs)])
    weighted = any(g.w is not None for g in graphs)
    w = None
    if weighted:
        w = np.concatenate([g.w if g.w is not None else np.ones(g.nnz, np.float32) for g in graphs])
    return CSR(n=int(offs[-1]), row_ptr=row_ptr.astype(np.int32), col_idx=col_idx.astype(np.int32),
               w=w, graph_row_offset=offs.astype(np.int32), name=f"batch[{len(graphs)}]")


def uneven_batch(num_graphs: int, seed: int) -> CSR:
    """Half Erdos-Renyi graphs with n ~ U{200..1200}, p = 0.15 and half Barabasi-Albert graphs
    with n ~ U{100..2000}, m ~ U{2..6}, interleaved, all independently drawn."""
    rng = np.random.Generator(np.random.PCG64(seed))
    graphs = []
    for g in range(num_graphs):
        if g % 2 == 0:
            n = int(rng.integers(200, 1201))
            graphs.append(erdos_renyi(n, 0.15, seed * 100003 + g))
        else:
            n = int(rng.integers(100, 2001))
            m = int(rng.integers(2, 7))
            graphs.append(barabasi_albert(n, m, seed * 100003 + g))
    return block_diagonal(graphs)


def uniform_batch(n: int, C: int, seed: int, dtype=np.float32) -> np.ndarray:
    """n x C matrix with entries uniform in [-1, 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return (rng.random((n, C), dtype=np.float64) * 2.0 - 1.0).astype(dtype)


def small_batch(n: int, C: int, seed: int, scale: float = 1e-4) -> np.ndarray:
    """n x C matrix with small entries, uniform in [-scale, scale)."""
    return (uniform_batch(n, C, seed, np.float64) * scale).astype(np.float32)


def random_signs(n: int, C: int, seed: int) -> np.ndarray:
    """n x C matrix of independent +-1 entries (float32)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.where(rng.random((n, C)) < 0.5, -1.0, 1.0).astype(np.float32)


# Small named graphs with textbook maximum cuts (used as fixtures).
def complete(n: int) -> CSR:
    u, v = np.triu_indices(n, 1)
    return from_edges(n, u, v, name=f"K{n}")


def cycle(n: int) -> CSR:
    u = np.arange(n)
    v = (u + 1) % n
    lo, hi = np.minimum(u, v), np.maximum(u, v)
    return from_edges(n, lo, hi, name=f"C{n}")


def path(n: int) -> CSR:
    u = np.arange(n - 1)
    return from_edges(n, u, u + 1, name=f"P{n}")


def star(n: int) -> CSR:
    return from_edges(n, np.zeros(n - 1, np.int64), np.arange(1, n), name=f"S{n}")


def complete_bipartite(a: int, b: int) -> CSR:
    u = np.repeat(np.arange(a), b)
    v = np.tile(np.arange(a, a + b), a)
    return from_edges(a + b, u, v, name=f"K{a},{b}")


def grid(r: int, c: int) -> CSR:
    idx = np.arange(r * c).reshape(r, c)
    u = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    v = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    return from_edges(r * c, u, v, name=f"grid{r}x{c}")


def edgeless(n: int) -> CSR:
    return from_edges(n, np.zeros(0, np.int64), np.zeros(0, np.int64), name=f"E{n}")


def from_edge_file(path_: str) -> CSR:
    """Read 'n m' then m lines 'u v [w]' (0-based, each undirected edge once)."""
    with open(path_) as f:
        lines = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    n, m = int(lines[0][0]), int(lines[0][1])
    body = lines[1:1 + m]
    u = np.array([int(t[0]) for t in body], np.int64)
    v = np.array([int(t[1]) for t in body], np.int64)
    w = None
    if body and len(body[0]) > 2:
        w = np.array([float(t[2]) for t in body], np.float32)
    lo, hi = np.minimum(u, v), np.maximum(u, v)
    return from_edges(n, lo, hi, w, name=path_)
