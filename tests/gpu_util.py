"""Shared helpers of the GPU parity tests: run the library step by step and replay the
same steps on the oracle from the GPU's own iterates (teacher forcing)."""
import numpy as np

import oracle
from paper_2509_18612_amd import deco

U32 = 2.0 ** -24


def to_np(t):
    import torch
    if t.dtype == torch.bfloat16:
        return t.float().cpu().numpy()
    return t.cpu().numpy()


def step_bound(g, X, eta, cw, form):
    """Per-element bound on |float32 step - exact step|: the float32 sum of d_v products
    (Higham, Accuracy and Stability of Numerical Algorithms, Sec. 3.1: gamma_k sum|w x|),
    scaled by eta*|cW|, plus the roundings of the update itself."""
    import scipy.sparse as sps
    n, C = X.shape
    d = np.diff(g.row_ptr.astype(np.int64))
    w = np.ones(g.nnz) if g.w is None else np.abs(g.w.astype(np.float64))
    Wabs = sps.csr_matrix((w, g.col_idx.astype(np.int64), g.row_ptr.astype(np.int64)), shape=(n, n))
    absum = np.asarray(Wabs @ np.abs(X))
    k = np.maximum(d, 1)[:, None]
    gamma = k * U32 / (1 - k * U32)
    b = np.abs(eta) * abs(cw) * gamma * absum
    if form == oracle.LAPLACIAN_FORM:
        dw = np.asarray(Wabs.sum(axis=1)).reshape(-1)
        b += np.abs(eta) * (dw[:, None] * np.abs(X)) * 4 * U32
    return b + 4 * U32


def bf16_ulp(x):
    a = np.abs(np.asarray(x, np.float64))
    a = np.maximum(a, 2.0 ** -126)
    return 2.0 ** (np.floor(np.log2(a)) - 7)


def run_teacher_forced(g, B, steps, l=1, lifted=False, form=deco.GRAD_CUT, dtype=deco.F32, eta=0.1, x0=None,
                       seed=3, schedule_tune=False, eta_per_init=None, schedule=None, l_active=None):
    """Returns per-step records: list of (X_t, X_{t+1}) as float64 arrays (GPU values),
    plus the handle's trace of cuts and its final best state. schedule: optional
    set_schedule arguments."""
    import torch
    G = deco.Graph(g)
    h = deco.Handle(G, B=B, l=l, lifted=lifted, grad_form=form, x_dtype=dtype, eta=eta, seed=seed)
    if schedule_tune:
        h.autotune(3)
    if schedule is not None:
        h.set_schedule(*schedule)
    if eta_per_init is not None:
        h.set_eta(eta_per_init)
    C = l * B
    if x0 is None:
        x0 = np.asarray(np.random.default_rng(seed).uniform(-1, 1, (g.n, C)), np.float32)
    tdt = torch.float32 if dtype == deco.F32 else torch.bfloat16
    h.start(deco.INIT_USER, x0=torch.from_numpy(np.asarray(x0, np.float32)).to(tdt).cuda(), l_active=l_active)
    trace = h.set_trace(steps + 1)
    xs = [to_np(h.read_x()).astype(np.float64)]
    for _ in range(steps):
        h.step(1)
        xs.append(to_np(h.read_x()).astype(np.float64))
    cut_T, bits_T = h.round_score()
    best = h.best()
    tr = trace.cpu().numpy()
    out = dict(xs=xs, trace=tr, best=best, cut_T=to_np(cut_T), bits_T=to_np(bits_T), handle=h,
               schedule=h.schedule())
    return out


def oracle_cuts(g, X, B, l, lifted):
    z = oracle.round_signs(X, B, l, lifted, sum_f32=True)
    return oracle.cut_batch(g, z), z
