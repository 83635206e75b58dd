"""Python binding of libdeco.so (include/deco.h), same names as the C ABI.

Argument marshalling only: every step of the method runs in the library's HIP kernels.
PyTorch provides device memory (tensors) and streams. If the library is missing this
module raises; there is no fallback path.
"""
from __future__ import annotations

import ctypes as ct
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# DECO_LIBRARY may name another build of the same sources (e.g. other compile options).
LIB_PATH = os.environ.get("DECO_LIBRARY", os.path.join(_HERE, "libdeco.so"))

OK, E_INVAL, E_NOMEM, E_DEVICE, E_STATE, E_NONFINITE, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
SOLVE_DECO, SOLVE_UNLIFTED, SOLVE_LIFTED = 0, 1, 2
GRAD_CUT, GRAD_LAPLACIAN = 0, 1
F32, BF16 = 0, 1
INIT_USER, INIT_UNIFORM, INIT_DUI, INIT_IDI, INIT_MEAN, INIT_LEARNED = 0, 1, 2, 3, 4, 5


class DecoError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


class deco_graph(ct.Structure):
    _fields_ = [("n", ct.c_int64), ("nnz", ct.c_int64), ("row_ptr", ct.c_void_p), ("col_idx", ct.c_void_p),
                ("w", ct.c_void_p), ("num_graphs", ct.c_int32), ("graph_row_offset", ct.c_void_p)]


class deco_params(ct.Structure):
    _fields_ = [("B", ct.c_int32), ("l", ct.c_int32), ("lifted", ct.c_int32), ("grad_form", ct.c_int32),
                ("x_dtype", ct.c_int32), ("score_every", ct.c_int32), ("eta", ct.c_float), ("seed", ct.c_uint64)]


class deco_start_args(ct.Structure):
    _fields_ = [("kind", ct.c_int32), ("x0", ct.c_void_p), ("mean_z", ct.c_void_p), ("scale", ct.c_double),
                ("sigma2", ct.c_double), ("beta", ct.c_double), ("batch", ct.c_uint32),
                ("l_active", ct.c_void_p), ("magnitude", ct.c_void_p)]


class deco_solve_params(ct.Structure):
    _fields_ = [("B", ct.c_int32), ("K", ct.c_int32), ("l_max", ct.c_int32), ("rounds", ct.c_int32),
                ("evo_rounds", ct.c_int32), ("T_q", ct.c_int32), ("T_l", ct.c_int32), ("grad_form", ct.c_int32),
                ("x_dtype", ct.c_int32), ("init_kind", ct.c_int32), ("beta", ct.c_double),
                ("sigma2", ct.c_double), ("scale", ct.c_double), ("time_budget_s", ct.c_double),
                ("seed", ct.c_uint64), ("eq0", ct.c_void_p), ("el0", ct.c_void_p), ("l0", ct.c_void_p),
                ("target_cut", ct.c_void_p), ("use_graph", ct.c_int32), ("autotune", ct.c_int32),
                ("T_min", ct.c_int32), ("T_l_min", ct.c_int32), ("magnitude", ct.c_void_p),
                ("check_every", ct.c_int32), ("mode", ct.c_int32)]


class deco_schedule(ct.Structure):
    _fields_ = [("lanes_per_row", ct.c_int32), ("long_row", ct.c_int32),
                ("xcd_mode", ct.c_int32), ("blocks_per_xcd", ct.c_int32), ("nnz_per_item", ct.c_int32),
                ("lane_elems", ct.c_int32), ("resident_cols", ct.c_int32)]


class deco_solve_report(ct.Structure):
    _fields_ = [("rounds_done", ct.c_int32), ("steps_done", ct.c_int64), ("edge_updates", ct.c_double),
                ("seconds", ct.c_double), ("eq_best", ct.c_double), ("el_best", ct.c_double),
                ("l_best", ct.c_int32), ("T_best", ct.c_int32), ("T_l_best", ct.c_int32)]


EXPORTS = ["deco_status_string", "deco_workspace_size", "deco_init", "deco_start", "deco_set_eta",
           "deco_set_momentum", "deco_step",
           "deco_round_score", "deco_best", "deco_read_x", "deco_set_trace", "deco_current_step",
           "deco_autotune", "deco_schedule_string", "deco_destroy", "deco_solve", "deco_evo_next",
           "deco_evo_next_steps", "deco_evo_init",
           "deco_philox", "deco_philox_device", "deco_solver_create", "deco_solver_run",
           "deco_solver_set_target", "deco_solver_destroy", "deco_set_schedule", "deco_dense_workspace_size",
           "deco_dense_init", "deco_mpnn_num_params", "deco_mpnn_workspace_size", "deco_mpnn_forward",
           "deco_mpnn_loss_grad", "deco_mpnn_adam", "deco_mpnn_labels", "deco_mpnn_forward_static"]

_lib = None


def lib():
    """Load libdeco.so (raises if it has not been built: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2509_18612_amd.build.build()")
        L = ct.CDLL(LIB_PATH)
        P, I32, I64, U32, U64, D = ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_uint32, ct.c_uint64, ct.c_double
        L.deco_status_string.argtypes = [I32]
        L.deco_status_string.restype = ct.c_char_p
        L.deco_workspace_size.argtypes = [P, P, ct.POINTER(ct.c_size_t)]
        L.deco_init.argtypes = [ct.POINTER(P), P, P, P, P, ct.c_size_t, P]
        L.deco_start.argtypes = [P, P]
        L.deco_set_eta.argtypes = [P, P]
        L.deco_set_momentum.argtypes = [P, ct.c_float, P]
        L.deco_step.argtypes = [P, I32, I32]
        L.deco_round_score.argtypes = [P, P, P]
        L.deco_best.argtypes = [P, P, P, P]
        L.deco_read_x.argtypes = [P, P]
        L.deco_set_trace.argtypes = [P, P, I32]
        L.deco_current_step.argtypes = [P]
        L.deco_current_step.restype = I64
        L.deco_autotune.argtypes = [P, I32]
        L.deco_schedule_string.argtypes = [P, ct.c_char_p, I32]
        L.deco_destroy.argtypes = [P]
        L.deco_destroy.restype = None
        L.deco_solve.argtypes = [P, P, P, P, P, P, P, P]
        L.deco_set_schedule.argtypes = [P, P]
        L.deco_mpnn_num_params.argtypes = []
        L.deco_mpnn_workspace_size.argtypes = [P, ct.POINTER(ct.c_size_t)]
        L.deco_mpnn_forward.argtypes = [P, P, P, P, ct.c_size_t, P]
        L.deco_mpnn_forward_static.argtypes = [P, P, P, P]
        L.deco_mpnn_loss_grad.argtypes = [P, P, P, P, ct.POINTER(D), P, ct.c_size_t, P]
        L.deco_mpnn_adam.argtypes = [P, P, P, P, I32, ct.c_float, P]
        L.deco_mpnn_labels.argtypes = [P, P, P, P]
        L.deco_dense_workspace_size.argtypes = [I64, P, ct.POINTER(ct.c_size_t)]
        L.deco_dense_init.argtypes = [ct.POINTER(P), I64, P, P, P, P, ct.c_size_t, P]
        L.deco_solver_create.argtypes = [ct.POINTER(P), P, P, P]
        L.deco_solver_run.argtypes = [P, I32, P, P, P, P, P]
        L.deco_solver_set_target.argtypes = [P, P]
        L.deco_solver_destroy.argtypes = [P]
        L.deco_solver_destroy.restype = None
        L.deco_evo_next.argtypes = [I32, P, P, P, P, D, D, I32, U64, U32, P, P, P]
        L.deco_evo_next_steps.argtypes = [I32, P, P, I32, I32, U64, U32, U32, P]
        L.deco_evo_init.argtypes = [I32, D, D, I32, I32, I32, I32, I32, U64, P, P, P, P, P]
        L.deco_philox.argtypes = [P, P, P]
        L.deco_philox.restype = None
        L.deco_philox_device.argtypes = [U32, U32, U32, U64, I32, P, P]
        for name in EXPORTS:
            f = getattr(L, name)
            if f.restype is ct.c_int:  # default: statuses are int32
                f.restype = I32
        _lib = L
    return _lib


def status_string(s: int) -> str:
    return lib().deco_status_string(int(s)).decode()


def _check(st: int, where: str):
    if st != OK:
        raise DecoError(st, where)


def _ptr(a) -> Optional[int]:
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


# ------------------------------------------------------------------------ graphs
class Graph:
    """Device copy (torch tensors) of a symmetric CSR graph or block-diagonal batch."""

    def __init__(self, csr, device="cuda"):
        import torch
        self.csr = csr
        self.n = int(csr.n)
        self.nnz = int(csr.nnz)
        self.row_ptr = torch.from_numpy(np.ascontiguousarray(csr.row_ptr, np.int32)).to(device)
        self.col_idx = torch.from_numpy(np.ascontiguousarray(csr.col_idx, np.int32)).to(device)
        self.w = None if csr.w is None else torch.from_numpy(np.ascontiguousarray(csr.w, np.float32)).to(device)
        off = csr.graph_row_offset
        self.num_graphs = 1 if off is None else int(len(off) - 1)
        self.goff = None if off is None else torch.from_numpy(np.ascontiguousarray(off, np.int32)).to(device)
        self.struct = deco_graph(self.n, self.nnz, self.row_ptr.data_ptr(),
                                 self.col_idx.data_ptr() if self.nnz else self.row_ptr.data_ptr(),
                                 None if self.w is None else self.w.data_ptr(), self.num_graphs,
                                 None if self.goff is None else self.goff.data_ptr())


def bits_to_z(bits: np.ndarray, B: int) -> np.ndarray:
    """Packed cut bits (n x ceil(B/8) bytes) -> n x B bytes in {0,1}."""
    bits = np.asarray(bits, np.uint8)
    n = bits.shape[0] if bits.ndim == 2 else bits.size // ((B + 7) // 8)
    bits = bits.reshape(n, (B + 7) // 8)
    z = np.unpackbits(bits, axis=1, bitorder="little")[:, :B]
    return np.ascontiguousarray(z)


def z_to_bits(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, np.uint8)
    return np.packbits(z, axis=1, bitorder="little")


# ------------------------------------------------------------------------ handle
class Handle:
    """One bound batch: graph + X (n x l*B) + workspace + stream."""

    def __init__(self, graph: Graph, B: int, l: int = 1, lifted: bool = False, grad_form: int = GRAD_CUT,
                 x_dtype: int = F32, eta: float = 0.1, score_every: int = 1, seed: int = 0, stream=None):
        import torch
        self.torch = torch
        self.graph = graph
        self.B, self.l, self.lifted = int(B), int(l), bool(lifted)
        self.C = self.l * self.B
        self.x_dtype = x_dtype
        self.params = deco_params(self.B, self.l, int(self.lifted), grad_form, x_dtype, score_every, eta, seed)
        nbytes = ct.c_size_t(0)
        _check(lib().deco_workspace_size(ct.byref(graph.struct), ct.byref(self.params), ct.byref(nbytes)),
               "deco_workspace_size")
        self.ws_bytes = int(nbytes.value)
        self.stream = stream if stream is not None else torch.cuda.Stream()
        tdt = torch.float32 if x_dtype == F32 else torch.bfloat16
        self.X = torch.empty((graph.n, self.C), dtype=tdt, device="cuda")
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device="cuda")
        self.nby = (self.B + 7) // 8
        self.G = graph.num_graphs
        torch.cuda.synchronize()
        h = ct.c_void_p()
        _check(lib().deco_init(ct.byref(h), ct.byref(graph.struct), ct.byref(self.params), self.X.data_ptr(),
                               self.ws.data_ptr(), self.ws_bytes, ct.c_void_p(self.stream.cuda_stream)),
               "deco_init")
        self.h = h

    # -- lifecycle
    def destroy(self):
        if getattr(self, "h", None):
            lib().deco_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def synchronize(self):
        self.stream.synchronize()

    # -- API
    def start(self, kind=INIT_UNIFORM, x0=None, mean_z=None, scale=1.0, sigma2=0.0, beta=0.2, batch=0,
              l_active: Optional[Sequence[int]] = None, magnitude=None):
        keep = []
        if x0 is not None:
            x0 = x0.contiguous()
            keep.append(x0)
        if mean_z is not None:
            mean_z = mean_z.contiguous()
            keep.append(mean_z)
        la = None
        if l_active is not None:
            la = np.ascontiguousarray(l_active, np.int32)
        if magnitude is not None:
            magnitude = magnitude.contiguous()
            keep.append(magnitude)
        a = deco_start_args(kind, _ptr(x0), _ptr(mean_z), float(scale), float(sigma2), float(beta), int(batch),
                            _ptr(la), _ptr(magnitude))
        self.torch.cuda.current_stream().synchronize()
        _check(lib().deco_start(self.h, ct.byref(a)), "deco_start")
        self._keep = keep

    def set_eta(self, eta):
        e = np.ascontiguousarray(np.broadcast_to(np.asarray(eta, np.float32), (self.B,)), np.float32)
        _check(lib().deco_set_eta(self.h, e.ctypes.data), "deco_set_eta")

    def set_momentum(self, mu: float):
        """Heavy-ball momentum (deco_set_momentum); the velocity buffer (float32, the shape of
        X) is allocated here and returned. mu = None turns it off."""
        torch = self.torch
        if mu is None:
            _check(lib().deco_set_momentum(self.h, 0.0, None), "deco_set_momentum")
            self._vel = None
            return None
        self._vel = torch.zeros((self.graph.n, self.C), dtype=torch.float32, device="cuda")
        _check(lib().deco_set_momentum(self.h, float(mu), self._vel.data_ptr()), "deco_set_momentum")
        return self._vel

    def step(self, steps: int, use_graph: bool = False):
        _check(lib().deco_step(self.h, int(steps), int(bool(use_graph))), "deco_step")

    def round_score(self):
        """Score the current iterate; returns (cuts [G,B] float64, bits [n, nby] uint8) device tensors."""
        torch = self.torch
        cut = torch.empty((self.G, self.B), dtype=torch.float64, device="cuda")
        bits = torch.empty((self.graph.n, self.nby), dtype=torch.uint8, device="cuda")
        _check(lib().deco_round_score(self.h, cut.data_ptr(), bits.data_ptr()), "deco_round_score")
        self.synchronize()
        return cut, bits

    def best(self):
        """(best cut [G,B], best step [G,B], best bits [n, nby]) as numpy arrays (synchronises)."""
        bc = np.zeros((self.G, self.B), np.float64)
        bs = np.zeros((self.G, self.B), np.int32)
        bb = np.zeros((self.graph.n, self.nby), np.uint8)
        _check(lib().deco_best(self.h, bc.ctypes.data, bs.ctypes.data, bb.ctypes.data), "deco_best")
        return bc, bs, bb

    def read_x(self):
        out = self.torch.empty_like(self.X)
        _check(lib().deco_read_x(self.h, out.data_ptr()), "deco_read_x")
        self.synchronize()
        return out

    def set_trace(self, capacity: int):
        if capacity <= 0:
            self.trace = None
            _check(lib().deco_set_trace(self.h, None, 0), "deco_set_trace")
            return None
        self.trace = self.torch.full((capacity, self.G, self.B), float("nan"), dtype=self.torch.float64,
                                     device="cuda")
        self.torch.cuda.current_stream().synchronize()
        _check(lib().deco_set_trace(self.h, self.trace.data_ptr(), int(capacity)), "deco_set_trace")
        return self.trace

    def current_step(self) -> int:
        return int(lib().deco_current_step(self.h))

    def autotune(self, steps: int = 10):
        _check(lib().deco_autotune(self.h, int(steps)), "deco_autotune")

    def set_schedule(self, lanes_per_row, long_row=64, xcd_mode=0, blocks_per_xcd=128, nnz_per_item=2048,
                     lane_elems=0, resident_cols=0):
        q = deco_schedule(lanes_per_row, long_row, xcd_mode, blocks_per_xcd, nnz_per_item, lane_elems,
                          resident_cols)
        _check(lib().deco_set_schedule(self.h, ct.byref(q)), "deco_set_schedule")

    def schedule(self) -> str:
        buf = ct.create_string_buffer(512)
        _check(lib().deco_schedule_string(self.h, buf, 512), "deco_schedule_string")
        return buf.value.decode()


class DenseHandle(Handle):
    """Dense-matrix batch: W is a device bfloat16 n x n tensor (symmetric, zero diagonal)."""

    def __init__(self, W, B: int, grad_form: int = GRAD_CUT, eta: float = 0.1, score_every: int = 1, seed: int = 0,
                 stream=None):
        import torch
        self.torch = torch
        n = int(W.shape[0])
        self.W = W.contiguous()
        self.graph = type("DenseGraph", (), {"n": n, "num_graphs": 1})()
        self.B, self.l, self.lifted, self.C = int(B), 1, False, int(B)
        self.x_dtype = BF16
        self.params = deco_params(self.B, 1, 0, grad_form, BF16, score_every, eta, seed)
        nbytes = ct.c_size_t(0)
        _check(lib().deco_dense_workspace_size(n, ct.byref(self.params), ct.byref(nbytes)), "deco_dense_workspace_size")
        self.ws_bytes = int(nbytes.value)
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.X = torch.empty((n, self.C), dtype=torch.bfloat16, device="cuda")
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device="cuda")
        self.nby = (self.B + 7) // 8
        self.G = 1
        torch.cuda.synchronize()
        h = ct.c_void_p()
        _check(lib().deco_dense_init(ct.byref(h), n, self.W.data_ptr(), ct.byref(self.params), self.X.data_ptr(),
                                     self.ws.data_ptr(), self.ws_bytes, ct.c_void_p(self.stream.cuda_stream)),
               "deco_dense_init")
        self.h = h


class Mpnn:
    """Learned starting magnitudes: parameters and Adam moments on the device, forward /
    loss-gradient / Adam / label kernels of the library (deco_mpnn_*)."""

    def __init__(self, params=None, stream=None):
        import torch
        self.torch = torch
        self.count = int(lib().deco_mpnn_num_params())
        if params is None:
            params = torch.zeros(self.count, dtype=torch.float32)
        self.params = torch.as_tensor(params, dtype=torch.float32).reshape(-1).cuda().contiguous()
        assert self.params.numel() == self.count
        self.grads = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = 0
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self._ws = None

    def _workspace(self, graph: Graph):
        nb = ct.c_size_t(0)
        _check(lib().deco_mpnn_workspace_size(ct.byref(graph.struct), ct.byref(nb)), "deco_mpnn_workspace_size")
        if self._ws is None or self._ws.numel() < nb.value:
            self._ws = self.torch.empty(int(nb.value), dtype=self.torch.uint8, device="cuda")
        return self._ws

    def forward(self, graph: Graph):
        ws = self._workspace(graph)
        y = self.torch.empty(graph.n, dtype=self.torch.float32, device="cuda")
        self.torch.cuda.current_stream().synchronize()
        _check(lib().deco_mpnn_forward(ct.byref(graph.struct), self.params.data_ptr(), y.data_ptr(), ws.data_ptr(),
                                       ws.numel(), ct.c_void_p(self.stream.cuda_stream)), "deco_mpnn_forward")
        self.stream.synchronize()
        return y

    def forward_static(self, graph: Graph):
        """forward() through deco_mpnn_forward_static: activations in the library's static
        scratch array, no workspace."""
        y = self.torch.empty(graph.n, dtype=self.torch.float32, device="cuda")
        self.torch.cuda.current_stream().synchronize()
        _check(lib().deco_mpnn_forward_static(ct.byref(graph.struct), self.params.data_ptr(), y.data_ptr(),
                                              ct.c_void_p(self.stream.cuda_stream)), "deco_mpnn_forward_static")
        self.stream.synchronize()
        return y

    def loss_grad(self, graph: Graph, target):
        ws = self._workspace(graph)
        target = target.contiguous()
        loss = ct.c_double(0.0)
        self.torch.cuda.current_stream().synchronize()
        _check(lib().deco_mpnn_loss_grad(ct.byref(graph.struct), self.params.data_ptr(), target.data_ptr(),
                                         self.grads.data_ptr(), ct.byref(loss), ws.data_ptr(), ws.numel(),
                                         ct.c_void_p(self.stream.cuda_stream)), "deco_mpnn_loss_grad")
        return float(loss.value)

    def adam(self, lr=1e-3):
        self.t += 1
        _check(lib().deco_mpnn_adam(self.params.data_ptr(), self.grads.data_ptr(), self.m.data_ptr(),
                                    self.v.data_ptr(), self.t, lr, ct.c_void_p(self.stream.cuda_stream)),
               "deco_mpnn_adam")
        self.stream.synchronize()

    def labels(self, graph: Graph, z):
        z = self.torch.as_tensor(np.ascontiguousarray(z, np.uint8)).cuda()
        t = self.torch.empty(graph.n, dtype=self.torch.float32, device="cuda")
        self.torch.cuda.current_stream().synchronize()
        _check(lib().deco_mpnn_labels(ct.byref(graph.struct), z.data_ptr(), t.data_ptr(),
                                      ct.c_void_p(self.stream.cuda_stream)), "deco_mpnn_labels")
        self.stream.synchronize()
        return t


def pack_mpnn(params: dict) -> np.ndarray:
    """Pack a name -> array dict (ws1, wn1, b1, ..., wo, bo) in the library's order."""
    order = ["ws1", "wn1", "b1", "ws2", "wn2", "b2", "ws3", "wn3", "b3", "wo", "bo"]
    return np.concatenate([np.asarray(params[k], np.float32).reshape(-1) for k in order])


def unpack_mpnn(vec) -> dict:
    shapes = [("ws1", (3, 64)), ("wn1", (3, 64)), ("b1", (64,)), ("ws2", (64, 64)), ("wn2", (64, 64)),
              ("b2", (64,)), ("ws3", (64, 64)), ("wn3", (64, 64)), ("b3", (64,)), ("wo", (64,)), ("bo", (1,))]
    vec = np.asarray(vec, np.float64).reshape(-1)
    out, o = {}, 0
    for k, shp in shapes:
        size = int(np.prod(shp))
        out[k] = vec[o:o + size].reshape(shp)
        o += size
    return out


# ------------------------------------------------------------------------ solve
def solve(graph: Graph, B=256, K=8, l_max=4, rounds=4, evo_rounds=2, T_q=500, T_l=200, grad_form=GRAD_CUT,
          x_dtype=F32, init_kind=INIT_IDI, beta=0.2, sigma2=0.8, scale=1e4, time_budget_s=0.0, seed=0,
          eq0=None, el0=None, l0=None, target_cut=None, use_graph=True, autotune=False, stream=None, T_min=0,
          T_l_min=0, magnitude=None, check_every=0, mode=0):
    """Full pDECO with the evolutionary search; returns a dict of host results. T_min > 0
    also searches the unlifted step count per member in [T_min, T_q], T_l_min > 0 the lifted
    one in [T_l_min, T_l]. magnitude: device float32 [n] for init_kind=INIT_LEARNED."""
    import torch
    stream = stream if stream is not None else torch.cuda.Stream()
    keep = []

    def arr(a, dt):
        if a is None:
            return None
        x = np.ascontiguousarray(a, dt)
        keep.append(x)
        return x.ctypes.data

    p = deco_solve_params(B, K, l_max, rounds, evo_rounds, T_q, T_l, grad_form, x_dtype, init_kind, beta, sigma2,
                          scale, time_budget_s, seed, arr(eq0, np.float64), arr(el0, np.float64),
                          arr(l0, np.int32), arr(target_cut, np.float64), int(bool(use_graph)),
                          int(bool(autotune)), int(T_min), int(T_l_min),
                          None if magnitude is None else magnitude.data_ptr(), int(check_every), int(mode))
    G = graph.num_graphs
    best = np.zeros(G, np.float64)
    z = np.zeros(graph.n, np.uint8)
    rt = np.zeros(rounds, np.float64)
    rb = np.zeros((rounds, G), np.float64)
    rep = deco_solve_report()
    torch.cuda.synchronize()
    _check(lib().deco_solve(ct.byref(graph.struct), ct.byref(p), ct.c_void_p(stream.cuda_stream), best.ctypes.data,
                            z.ctypes.data, rt.ctypes.data, rb.ctypes.data, ct.byref(rep)), "deco_solve")
    r = rep.rounds_done
    return {"best_cut": best, "z": z, "round_time": rt[:r], "round_best": rb[:r], "rounds_done": r,
            "steps_done": rep.steps_done, "edge_updates": rep.edge_updates, "seconds": rep.seconds,
            "eq_best": rep.eq_best, "el_best": rep.el_best, "l_best": rep.l_best, "T_best": rep.T_best,
            "T_l_best": rep.T_l_best}


class Solver:
    """Persistent pDECO solver (deco_solver_*): run() continues from the current state."""

    def __init__(self, graph: Graph, B=256, K=8, l_max=4, evo_rounds=2, T_q=500, T_l=200, grad_form=GRAD_CUT,
                 x_dtype=F32, init_kind=INIT_IDI, beta=0.2, sigma2=0.8, scale=1e4, time_budget_s=0.0, seed=0,
                 eq0=None, el0=None, l0=None, target_cut=None, use_graph=True, autotune=False, stream=None,
                 T_min=0, T_l_min=0, magnitude=None, check_every=0, mode=0):
        import torch
        self.graph = graph
        # LEARNED starts read the device magnitudes at every run: keep the tensor alive
        self._magnitude = None if magnitude is None else magnitude.contiguous()
        self.stream = stream if stream is not None else torch.cuda.Stream()
        keep = []

        def arr(a, dt):
            if a is None:
                return None
            x = np.ascontiguousarray(a, dt)
            keep.append(x)
            return x.ctypes.data

        p = deco_solve_params(B, K, l_max, 1, evo_rounds, T_q, T_l, grad_form, x_dtype, init_kind, beta, sigma2,
                              scale, time_budget_s, seed, arr(eq0, np.float64), arr(el0, np.float64),
                              arr(l0, np.int32), arr(target_cut, np.float64), int(bool(use_graph)),
                              int(bool(autotune)), int(T_min), int(T_l_min),
                              None if self._magnitude is None else self._magnitude.data_ptr(), int(check_every),
                              int(mode))
        torch.cuda.synchronize()
        h = ct.c_void_p()
        _check(lib().deco_solver_create(ct.byref(h), ct.byref(graph.struct), ct.byref(p),
                                        ct.c_void_p(self.stream.cuda_stream)), "deco_solver_create")
        self.h = h
        self.G = graph.num_graphs

    def run(self, rounds: int):
        G = self.G
        best = np.zeros(G, np.float64)
        z = np.zeros(self.graph.n, np.uint8)
        rt = np.zeros(max(rounds, 1), np.float64)
        rb = np.zeros((max(rounds, 1), G), np.float64)
        rep = deco_solve_report()
        _check(lib().deco_solver_run(self.h, int(rounds), best.ctypes.data, z.ctypes.data, rt.ctypes.data,
                                     rb.ctypes.data, ct.byref(rep)), "deco_solver_run")
        r = rep.rounds_done
        return {"best_cut": best, "z": z, "round_time": rt[:r], "round_best": rb[:r], "rounds_done": r,
                "steps_done": rep.steps_done, "edge_updates": rep.edge_updates, "seconds": rep.seconds,
                "eq_best": rep.eq_best, "el_best": rep.el_best, "l_best": rep.l_best, "T_best": rep.T_best,
                "T_l_best": rep.T_l_best}

    def set_target(self, target_cut):
        t = None if target_cut is None else np.ascontiguousarray(target_cut, np.float64)
        _check(lib().deco_solver_set_target(self.h, None if t is None else t.ctypes.data), "deco_solver_set_target")
        self._t = t

    def destroy(self):
        if getattr(self, "h", None):
            lib().deco_solver_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


# ------------------------------------------------------------------------ host utilities
def evo_next(fitness, eq, el, l, seed, rnd, lo=-4.0, hi=-1.0, lmax=4):
    K = len(fitness)
    f = np.ascontiguousarray(fitness, np.float64)
    a = np.ascontiguousarray(eq, np.float64)
    b = np.ascontiguousarray(el, np.float64)
    c = np.ascontiguousarray(l, np.int32)
    ao, bo, co = np.zeros(K), np.zeros(K), np.zeros(K, np.int32)
    _check(lib().deco_evo_next(K, f.ctypes.data, a.ctypes.data, b.ctypes.data, c.ctypes.data, lo, hi, lmax, seed,
                               rnd, ao.ctypes.data, bo.ctypes.data, co.ctypes.data), "deco_evo_next")
    return ao, bo, co


def evo_next_steps(fitness, T, T_lo, T_hi, seed, rnd, gene=0):
    K = len(fitness)
    f = np.ascontiguousarray(fitness, np.float64)
    t = np.ascontiguousarray(T, np.int32)
    out = np.zeros(K, np.int32)
    _check(lib().deco_evo_next_steps(K, f.ctypes.data, t.ctypes.data, T_lo, T_hi, seed, rnd, gene, out.ctypes.data),
           "deco_evo_next_steps")
    return out


def evo_init(K, seed, lmax=4, Tq=(1, 1), Tl=(1, 1), lo=-4.0, hi=-1.0):
    """Initial population of the search (deco_evo_init): returns (eq, el, l, tq, tl)."""
    eq, el = np.zeros(K), np.zeros(K)
    l, tq, tl = np.zeros(K, np.int32), np.zeros(K, np.int32), np.zeros(K, np.int32)
    _check(lib().deco_evo_init(K, lo, hi, lmax, int(Tq[0]), int(Tq[1]), int(Tl[0]), int(Tl[1]), seed,
                               eq.ctypes.data, el.ctypes.data, l.ctypes.data, tq.ctypes.data, tl.ctypes.data),
           "deco_evo_init")
    return eq, el, l, tq, tl


def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().deco_philox(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def philox_device(c1, c2, c3, seed, count):
    import torch
    out = torch.zeros(count * 4, dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream()
    _check(lib().deco_philox_device(c1, c2, c3, seed, count, out.data_ptr(), ct.c_void_p(s.cuda_stream)),
           "deco_philox_device")
    s.synchronize()
    return out.cpu().numpy().view(np.uint32).reshape(count, 4)
