"""FP64 oracle of the learned starting-point proposer (a 3-layer message-passing network).

TEST INFRASTRUCTURE ONLY (see the package docstring). The paper's method is training-free
(abstract); this network is an extension that proposes per-node starting magnitudes. It
is written here plainly in float64 numpy so that the GPU forward/backward kernels can be
checked against it.

Network (per graph of a block-diagonal batch):
  features f_v = [d_v / dbar, m_v / dbar, log(1 + d_v) - log(1 + dbar)]
      d_v = degree (count), m_v = mean degree of v's neighbours (0 for an isolated node),
      dbar = mean degree of v's graph
  layer k = 1..3:  h_v <- relu(W_s^k h_v + W_n^k a_v + b^k),  a_v = mean_{u in N(v)} h_u
      (a_v = 0 for an isolated node); dims 3 -> 64 -> 64 -> 64
  head:            y_v = sigmoid(w_o . h_v + b_o)
  label:           t_v = (sum_u w_vu 1{z*_u != z*_v}) / d_w(v), the fraction of v's weight
                   cut by a best vector z* (0 for an isolated node)
  loss:            L = mean_v (y_v - t_v)^2
Weights are stored as float32 masters; the forward pass uses them rounded to bfloat16
(the GPU stores them so), with float64 arithmetic here.
Pins: finite-difference gradients, and on a regular graph every node has the same
features, so every output equals the closed form of one node's forward pass.
"""
from __future__ import annotations

import numpy as np

HID = 64
IN = 3
SHAPES = [("ws1", (IN, HID)), ("wn1", (IN, HID)), ("b1", (HID,)),
          ("ws2", (HID, HID)), ("wn2", (HID, HID)), ("b2", (HID,)),
          ("ws3", (HID, HID)), ("wn3", (HID, HID)), ("b3", (HID,)),
          ("wo", (HID,)), ("bo", (1,))]


def init_params(seed: int) -> dict:
    """Glorot-uniform weights, zero biases (float32 masters)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in SHAPES:
        if name.startswith("b"):
            p[name] = np.zeros(shp, np.float32)
        else:
            fan_in = shp[0]
            fan_out = shp[1] if len(shp) > 1 else 1
            lim = np.sqrt(6.0 / (fan_in + fan_out))
            p[name] = rng.uniform(-lim, lim, shp).astype(np.float32)
    return p


def bf16(x):
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).reshape(f.shape)


def _graph_arrays(csr):
    n = csr.n
    rp = csr.row_ptr.astype(np.int64)
    d = np.diff(rp).astype(np.float64)
    rows = np.repeat(np.arange(n), np.diff(rp))
    cols = csr.col_idx.astype(np.int64)
    w = np.ones(len(cols)) if csr.w is None else csr.w.astype(np.float64)
    goff = np.array([0, n]) if csr.graph_row_offset is None else csr.graph_row_offset.astype(np.int64)
    return n, d, rows, cols, w, goff


def features(csr) -> np.ndarray:
    n, d, rows, cols, _, goff = _graph_arrays(csr)
    nbr_sum = np.zeros(n)
    np.add.at(nbr_sum, rows, d[cols])
    m = np.where(d > 0, nbr_sum / np.maximum(d, 1), 0.0)
    f = np.zeros((n, 3))
    for g in range(len(goff) - 1):
        r0, r1 = goff[g], goff[g + 1]
        dbar = d[r0:r1].mean()
        dbar = dbar if dbar > 0 else 1.0
        f[r0:r1, 0] = d[r0:r1] / dbar
        f[r0:r1, 1] = m[r0:r1] / dbar
        f[r0:r1, 2] = np.log1p(d[r0:r1]) - np.log1p(dbar)
    return f


def mean_aggregate(csr, H) -> np.ndarray:
    n, d, rows, cols, _, _ = _graph_arrays(csr)
    A = np.zeros_like(H)
    np.add.at(A, rows, H[cols])
    return np.where(d[:, None] > 0, A / np.maximum(d, 1)[:, None], 0.0)


def mean_aggregate_T(csr, G) -> np.ndarray:
    """Adjoint of mean_aggregate: dH_u = sum_{v in N(u)} G_v / d_v."""
    n, d, rows, cols, _, _ = _graph_arrays(csr)
    Gs = np.where(d[:, None] > 0, G / np.maximum(d, 1)[:, None], 0.0)
    out = np.zeros_like(G)
    np.add.at(out, cols, Gs[rows])
    return out


def labels(csr, z) -> np.ndarray:
    n, d, rows, cols, w, _ = _graph_arrays(csr)
    z = np.asarray(z).astype(np.int64)
    cut = np.zeros(n)
    np.add.at(cut, rows, w * (z[rows] != z[cols]))
    dw = np.zeros(n)
    np.add.at(dw, rows, w)
    return np.where(dw != 0, cut / np.where(dw != 0, dw, 1.0), 0.0)


def forward(csr, params, F=None, keep=False):
    q = {k: bf16(v).astype(np.float64) for k, v in params.items()}
    h = features(csr) if F is None else F
    cache = []
    for k in (1, 2, 3):
        a = mean_aggregate(csr, h)
        pre = h @ q[f"ws{k}"] + a @ q[f"wn{k}"] + q[f"b{k}"]
        cache.append((h, a, pre))
        h = np.maximum(pre, 0.0)
    z = h @ q["wo"] + q["bo"][0]
    y = 1.0 / (1.0 + np.exp(-z))
    if keep:
        return y, (cache, h, y, q)
    return y


def loss_and_grads(csr, params, t):
    """L = mean (y - t)^2 and dL/d(each weight), float64 (gradients with respect to the
    bfloat16-rounded weights the forward pass uses)."""
    y, (cache, h3, _, q) = forward(csr, params, keep=True)
    n = len(y)
    L = float(np.mean((y - t) ** 2))
    dy = 2.0 * (y - t) / n
    dz = dy * y * (1.0 - y)
    g = {"wo": h3.T @ dz, "bo": np.array([dz.sum()])}
    dh = np.outer(dz, q["wo"])
    for k in (3, 2, 1):
        h, a, pre = cache[k - 1]
        dpre = dh * (pre > 0)
        g[f"ws{k}"] = h.T @ dpre
        g[f"wn{k}"] = a.T @ dpre
        g[f"b{k}"] = dpre.sum(0)
        dh = dpre @ q[f"ws{k}"].T + mean_aggregate_T(csr, dpre @ q[f"wn{k}"].T)
    return L, g


def adam(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step on the float32 masters (Kingma and Ba, 2015)."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    out = {}
    for k, v in params.items():
        m = state.setdefault("m_" + k, np.zeros_like(v, np.float64))
        s = state.setdefault("v_" + k, np.zeros_like(v, np.float64))
        m[...] = b1 * m + (1 - b1) * grads[k]
        s[...] = b2 * s + (1 - b2) * grads[k] ** 2
        mh = m / (1 - b1 ** t)
        sh = s / (1 - b2 ** t)
        out[k] = (v - lr * mh / (np.sqrt(sh) + eps)).astype(np.float32)
    return out
