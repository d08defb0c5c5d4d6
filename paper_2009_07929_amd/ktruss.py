"""Thin Python binding of the C-ABI in include/ktruss.h (ctypes).

Argument marshalling only: every step of the K-truss path runs in the HIP
library.  Device buffers are torch tensors on the current HIP device (torch is
used for device memory and streams); the calls take the same names as the C
functions.  If libktruss.so cannot be loaded the import fails loudly — there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

# status codes (include/ktruss.h)
OK, E_INVALID, E_OVERFLOW, E_CAPACITY, E_HIP, E_NOMEM = 0, -1, -2, -3, -4, -5
SCHED_PLAIN, SCHED_HEURISTIC, SCHED_LEARNED, SCHED_FORCE_WAVE, SCHED_FORCE_HUB, SCHED_COARSE = 0, 1, 2, 3, 4, 5

_lib = None


class KtrussError(RuntimeError):
    def __init__(self, code, message):
        super().__init__("%s (%d): %s" % (_strerror(code), code, message))
        self.code = code


class ktruss_tuning(ctypes.Structure):
    _fields_ = [("wave_min_work", ctypes.c_int32), ("hub_min_work", ctypes.c_int32),
                ("hub_chunk_work", ctypes.c_int32), ("rounds_per_sync", ctypes.c_int32),
                ("learned_hub_min", ctypes.c_float), ("hub_chunk_tasks", ctypes.c_int32),
                ("plain_max_work", ctypes.c_int32), ("incremental", ctypes.c_int32), ("peel_ratio", ctypes.c_float)]


MLP_IN, MLP_HIDDEN, MLP_PARAMS = 5, 64, 4609


class ktruss_graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("schedule", ctypes.c_int32), ("m", ctypes.c_int64),
                ("rowptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("work", ctypes.c_void_p),
                ("work_bytes", ctypes.c_int64), ("mlp_params", ctypes.c_void_p), ("tuning", ktruss_tuning)]


def library_path() -> str:
    return _build.LIB


def load():
    """Load libktruss.so (building it with hipcc only if it does not exist yet)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_build.LIB):
        _build.build_library(force=False)
    lib = ctypes.CDLL(_build.LIB)
    i32, i64, p = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    G = ctypes.POINTER(ktruss_graph)
    sig = {
        "ktruss_strerror": ([i32], ctypes.c_char_p),
        "ktruss_last_error_message": ([], ctypes.c_char_p),
        "ktruss_last_hip_error": ([], i32),
        "ktruss_version": ([], i32),
        "ktruss_build_csr": ([p, p, i64, i32, i32, p, p, i64, p, p], i32),
        "ktruss_workspace_bytes": ([i32, i64, i32], i64),
        "ktruss_validate": ([G, p], i32),
        "ktruss_support": ([G, p, p, p], i32),
        "ktruss_prune": ([G, i32, p, p, p, p], i32),
        "ktruss_run": ([G, i32, p, p, p, p], i32),
        "ktruss_run_noalloc": ([i32, i64, p, p, i32, i32, p, p, p, p], i32),
        "ktruss_decompose": ([G, p, p, p], i32),
        "ktruss_set_schedule": ([G, i32, p, ctypes.POINTER(ktruss_tuning)], i32),
        "ktruss_profile_enable": ([i32], i32),
        "ktruss_profile_read": ([i32, p, p, p, p], i32),
        "ktruss_profile_stats": ([p, i32], i32),
        "ktruss_batch_workspace_bytes": ([i32, i64, i64, i32], i64),
        "ktruss_butterfly_workspace_bytes": ([i32, i32, i64], i64),
        "ktruss_butterflies": ([ctypes.POINTER(ktruss_bipartite), p, p, p], i32),
        "ktruss_run_batched": ([ctypes.POINTER(ktruss_batch), p, p, p, p, p], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _strerror(code):
    try:
        return load().ktruss_strerror(code).decode()
    except Exception:
        return "status"


def _check(rc):
    if rc != OK:
        raise KtrussError(rc, load().ktruss_last_error_message().decode())
    return rc


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def ktruss_build_csr(src, dst, n: int, order: int = 1):
    """Host CSR builder: (rowptr int32[n+1], col int32[m], new_to_old int32[n]) as NumPy arrays."""
    src = np.ascontiguousarray(src, np.int32)
    dst = np.ascontiguousarray(dst, np.int32)
    if src.shape != dst.shape:
        raise ValueError("src and dst differ in length")
    rowptr = np.empty(n + 1, np.int32)
    col = np.empty(max(len(src), 1), np.int32)
    n2o = np.empty(max(n, 1), np.int32)
    m = ctypes.c_int64()
    _check(load().ktruss_build_csr(_ptr(src), _ptr(dst), len(src), n, order, _ptr(rowptr), _ptr(col),
                                   len(col), _ptr(n2o), ctypes.byref(m)))
    return rowptr, col[: m.value].copy(), n2o[:n].copy()


def build_csrs(pairs, order: int = 1, threads: int = 16):
    """ktruss_build_csr over many graphs [(n, src, dst), ...] on a thread pool
    (the C builder runs outside the interpreter lock).  Returns [(rowptr, col)]."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(lambda g: ktruss_build_csr(g[1], g[2], g[0], order)[:2], pairs))


def ktruss_workspace_bytes(n: int, m: int, flags: int = 0) -> int:
    r = load().ktruss_workspace_bytes(n, m, flags)
    if r < 0:
        _check(int(r))
    return int(r)


class Graph:
    """A device-resident CSR graph with its workspace (owns the torch tensors)."""

    def __init__(self, rowptr, col, device="cuda", schedule=SCHED_PLAIN):
        import torch
        rowptr = torch.as_tensor(np.ascontiguousarray(rowptr, np.int32) if isinstance(rowptr, np.ndarray) else rowptr)
        col = torch.as_tensor(np.ascontiguousarray(col, np.int32) if isinstance(col, np.ndarray) else col)
        self.n = int(rowptr.numel()) - 1
        self.m = int(col.numel())
        self.rowptr = rowptr.to(device=device, dtype=torch.int32).contiguous()
        self.col = (col if self.m else torch.zeros(1, dtype=torch.int32)).to(device=device, dtype=torch.int32).contiguous()
        nbytes = ktruss_workspace_bytes(self.n, self.m)
        self.work = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.mlp_params = None
        self.c = ktruss_graph()
        self.c.n = self.n
        self.c.m = self.m
        self.c.schedule = schedule
        self.c.rowptr = self.rowptr.data_ptr()
        self.c.col = self.col.data_ptr()
        self.c.work = self.work.data_ptr()
        self.c.work_bytes = nbytes
        self.c.mlp_params = None

    @property
    def device(self):
        return self.rowptr.device


def ktruss_set_schedule(g: Graph, mode: int, mlp_params=None, tuning: ktruss_tuning | None = None):
    g.mlp_params = mlp_params
    _check(load().ktruss_set_schedule(ctypes.byref(g.c), mode, _ptr(mlp_params),
                                      ctypes.byref(tuning) if tuning is not None else None))


def ktruss_validate(g: Graph, stream=None):
    _check(load().ktruss_validate(ctypes.byref(g.c), _stream(stream)))


def ktruss_support(g: Graph, alive=None, support=None, stream=None):
    """One support evaluation on the alive subgraph; returns support int32[m] (device)."""
    import torch
    if support is None:
        support = torch.empty(max(g.m, 1), dtype=torch.int32, device=g.device)
    _check(load().ktruss_support(ctypes.byref(g.c), _ptr(alive), _ptr(support), _stream(stream)))
    return support[: g.m]


def ktruss_prune(g: Graph, K: int, support, alive, removed=None, stream=None):
    """alive &= support >= K-2 in place; `removed` (int64[1] device tensor) gets the count."""
    _check(load().ktruss_prune(ctypes.byref(g.c), K, _ptr(support), _ptr(alive), _ptr(removed), _stream(stream)))
    return alive


def ktruss_profile_enable(on: bool = True):
    _check(load().ktruss_profile_enable(1 if on else 0))


PROFILE_PASS, PROFILE_THREAD, PROFILE_WAVE, PROFILE_HUB, PROFILE_HIT_SUM, PROFILE_ROW = 0, 1, 2, 3, 4, 5


def ktruss_profile_read(kind: int = PROFILE_PASS):
    """(launches, total_ms, tasks, compulsory_bytes) of the timed support launches of `kind`."""
    launches, edges, nbytes = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    ms = ctypes.c_double()
    _check(load().ktruss_profile_read(kind, ctypes.byref(launches), ctypes.byref(ms), ctypes.byref(edges),
                                      ctypes.byref(nbytes)))
    return launches.value, ms.value, edges.value, nbytes.value


PASS_STATS = ("edges", "tail", "rowk", "support", "hub_tasks", "hub_tail", "hub_words", "hub_staged")


def ktruss_profile_stats():
    """Pass statistics summed over the profiled passes, as a dict keyed by PASS_STATS."""
    out = (ctypes.c_int64 * len(PASS_STATS))()
    _check(load().ktruss_profile_stats(out, len(PASS_STATS)))
    return dict(zip(PASS_STATS, (int(v) for v in out)))


def ktruss_run(g: Graph, K: int, mask=None, support=None, stream=None):
    """Full fixpoint.  Returns (mask uint8[m], support int32[m], rounds)."""
    import torch
    if mask is None:
        mask = torch.empty(max(g.m, 1), dtype=torch.uint8, device=g.device)
    if support is None:
        support = torch.empty(max(g.m, 1), dtype=torch.int32, device=g.device)
    rounds = ctypes.c_int32()
    _check(load().ktruss_run(ctypes.byref(g.c), K, _ptr(mask), _ptr(support), ctypes.byref(rounds),
                             _stream(stream)))
    return mask[: g.m], support[: g.m], rounds.value


def ktruss_decompose(g: Graph, trussness=None, stream=None):
    """Trussness of every edge.  Returns (trussness int32[m], k_max)."""
    import torch
    if trussness is None:
        trussness = torch.empty(max(g.m, 1), dtype=torch.int32, device=g.device)
    k_max = ctypes.c_int32()
    _check(load().ktruss_decompose(ctypes.byref(g.c), _ptr(trussness), ctypes.byref(k_max), _stream(stream)))
    return trussness[: g.m], k_max.value


# ------------------------------------------------------------------ batched form

class ktruss_batch(ctypes.Structure):
    _fields_ = [("G", ctypes.c_int32), ("schedule", ctypes.c_int32), ("n_total", ctypes.c_int64),
                ("m_total", ctypes.c_int64), ("vert_off", ctypes.c_void_p), ("rowptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("work", ctypes.c_void_p), ("work_bytes", ctypes.c_int64),
                ("tuning", ktruss_tuning)]


class ktruss_bipartite(ctypes.Structure):
    _fields_ = [("nu", ctypes.c_int32), ("nv", ctypes.c_int32), ("m", ctypes.c_int64),
                ("rowptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("work", ctypes.c_void_p),
                ("work_bytes", ctypes.c_int64)]


def ktruss_butterfly_workspace_bytes(nu: int, nv: int, m: int) -> int:
    r = load().ktruss_butterfly_workspace_bytes(nu, nv, m)
    if r < 0:
        _check(int(r))
    return int(r)


def ktruss_butterflies(nu: int, nv: int, rowptr, col, device="cuda", count=None, stream=None, work=None):
    """Butterflies of the bipartite graph with CSR rows over U (columns in [0, nv)):
    (count int64[m] device tensor per edge, total).  work: a device uint8 tensor of
    at least ktruss_butterfly_workspace_bytes + 256 bytes, or None (allocated here)."""
    import torch
    rp = torch.as_tensor(np.ascontiguousarray(rowptr, np.int32) if isinstance(rowptr, np.ndarray) else rowptr)
    cl = torch.as_tensor(np.ascontiguousarray(col, np.int32) if isinstance(col, np.ndarray) else col)
    m = int(cl.numel())
    rp = rp.to(device=device, dtype=torch.int32).contiguous()
    cl = (cl if m else torch.zeros(1, dtype=torch.int32)).to(device=device, dtype=torch.int32).contiguous()
    nbytes = ktruss_butterfly_workspace_bytes(nu, nv, m)
    if work is None:
        work = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    elif work.numel() < nbytes + 256:
        raise ValueError("butterfly workspace too small")
    base = (work.data_ptr() + 255) & ~255
    if count is None:
        count = torch.empty(max(m, 1), dtype=torch.int64, device=device)
    g = ktruss_bipartite()
    g.nu, g.nv, g.m = nu, nv, m
    g.rowptr, g.col = rp.data_ptr(), cl.data_ptr()
    g.work, g.work_bytes = base, int(nbytes)
    total = ctypes.c_int64()
    _check(load().ktruss_butterflies(ctypes.byref(g), _ptr(count), ctypes.byref(total), _stream(stream)))
    return count[:m], total.value


def ktruss_batch_workspace_bytes(G: int, n_total: int, m_total: int, flags: int = 0) -> int:
    r = load().ktruss_batch_workspace_bytes(G, n_total, m_total, flags)
    if r < 0:
        _check(int(r))
    return int(r)


def union_csr(graphs):
    """Concatenate per-graph CSRs [(rowptr, col), ...] into the union CSR.

    Returns (vert_off int32[G+1], rowptr int32[n_total+1], col int32[m_total])."""
    ns = [len(rp) - 1 for rp, _ in graphs]
    ms = [len(c) for _, c in graphs]
    vert_off = np.zeros(len(graphs) + 1, np.int64)
    vert_off[1:] = np.cumsum(ns)
    edge_off = np.zeros(len(graphs) + 1, np.int64)
    edge_off[1:] = np.cumsum(ms)
    if vert_off[-1] > 2**31 - 2 or edge_off[-1] > 2**31 - 2:
        raise ValueError("batch too large for int32 offsets")
    rowptr = np.empty(vert_off[-1] + 1, np.int32)
    col = np.empty(edge_off[-1], np.int32)
    for g, (rp, c) in enumerate(graphs):
        v0, v1, e0, e1 = vert_off[g], vert_off[g + 1], edge_off[g], edge_off[g + 1]
        np.add(rp[:-1], np.int32(e0), out=rowptr[v0:v1], casting="unsafe")
        np.add(c, np.int32(v0), out=col[e0:e1], casting="unsafe")
    rowptr[-1] = edge_off[-1]
    return vert_off.astype(np.int32), rowptr, col


class Batch:
    """Device-resident union CSR of many graphs plus its workspace."""

    def __init__(self, graphs=None, device="cuda", schedule=SCHED_PLAIN, vert_off=None, rowptr=None, col=None):
        import torch
        if graphs is not None:
            vert_off, rowptr, col = union_csr(graphs)
        self.G = len(vert_off) - 1
        self.n_total = len(rowptr) - 1
        self.m_total = len(col)
        self.vert_off = torch.from_numpy(np.ascontiguousarray(vert_off, np.int32)).to(device)
        self.rowptr = torch.from_numpy(np.ascontiguousarray(rowptr, np.int32)).to(device)
        self.col = torch.from_numpy(np.ascontiguousarray(col if len(col) else np.zeros(1), np.int32)).to(device)
        nbytes = ktruss_batch_workspace_bytes(self.G, self.n_total, self.m_total)
        self.work = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.c = ktruss_batch()
        self.c.G = self.G
        self.c.schedule = schedule
        self.c.n_total = self.n_total
        self.c.m_total = self.m_total
        self.c.vert_off = self.vert_off.data_ptr()
        self.c.rowptr = self.rowptr.data_ptr()
        self.c.col = self.col.data_ptr()
        self.c.work = self.work.data_ptr()
        self.c.work_bytes = nbytes

    @property
    def device(self):
        return self.rowptr.device

    def edge_offsets(self):
        """Edge offset of every graph in the union CSR (host int64[G+1])."""
        vo = self.vert_off.cpu().numpy().astype(np.int64)
        return self.rowptr.cpu().numpy().astype(np.int64)[vo]


def ktruss_run_batched(b: Batch, K, mask=None, support=None, rounds=None, stream=None):
    """Every graph's K-truss (K per graph).  Returns (mask, support, rounds) device tensors."""
    import torch
    K = torch.as_tensor(np.ascontiguousarray(K, np.int32) if not isinstance(K, torch.Tensor) else K)
    K = K.to(device=b.device, dtype=torch.int32).contiguous()
    if mask is None:
        mask = torch.empty(max(b.m_total, 1), dtype=torch.uint8, device=b.device)
    if support is None:
        support = torch.empty(max(b.m_total, 1), dtype=torch.int32, device=b.device)
    if rounds is None:
        rounds = torch.empty(max(b.G, 1), dtype=torch.int32, device=b.device)
    _check(load().ktruss_run_batched(ctypes.byref(b.c), _ptr(K), _ptr(mask), _ptr(support), _ptr(rounds),
                                     _stream(stream)))
    return mask[: b.m_total], support[: b.m_total], rounds[: b.G]


# -------------------------------------------------------------------- cost model

def _cost_model_sigs(lib):
    i32, i64, p, f32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_float
    G = ctypes.POINTER(ktruss_graph)
    for name, args, res in (
            ("ktruss_collect_row_costs", [G, i32, i32, p, p, i32, ctypes.POINTER(ctypes.c_int32), p], i32),
            ("ktruss_mlp_workspace_bytes", [i32], i64),
            ("ktruss_mlp_forward", [p, p, i32, p, p], i32),
            ("ktruss_mlp_loss_grad", [p, p, p, i32, p, p, p, i64, p], i32),
            ("ktruss_mlp_adam", [p, p, p, p, i32, f32, f32, f32, f32, p], i32)):
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res


def ktruss_collect_row_costs(g: Graph, K: int, capacity: int, stream=None, variant: int = 0):
    """Per-row cost samples of a timed run with every task on one variant (0 hub, 1 wavefront):
    (features float[count,5], log2(1 + wave-cycles) float[count])."""
    import torch
    lib = load()
    _cost_model_sigs(lib)
    X = torch.empty(max(capacity, 1) * MLP_IN, dtype=torch.float32, device=g.device)
    Y = torch.empty(max(capacity, 1), dtype=torch.float32, device=g.device)
    count = ctypes.c_int32()
    _check(lib.ktruss_collect_row_costs(ctypes.byref(g.c), K, variant, _ptr(X), _ptr(Y), capacity,
                                        ctypes.byref(count), _stream(stream)))
    c = count.value
    return X[: c * MLP_IN].view(c, MLP_IN), Y[:c]


def ktruss_mlp_forward(params, X, stream=None):
    import torch
    lib = load()
    _cost_model_sigs(lib)
    rows = X.shape[0]
    Y = torch.empty(max(rows, 1), dtype=torch.float32, device=X.device)
    _check(lib.ktruss_mlp_forward(_ptr(params), _ptr(X), rows, _ptr(Y), _stream(stream)))
    return Y[:rows]


def ktruss_mlp_loss_grad(params, X, T, work=None, stream=None):
    """(loss tensor[1], grad tensor[4609]) of mean squared error on device."""
    import torch
    lib = load()
    _cost_model_sigs(lib)
    rows = X.shape[0]
    nbytes = int(lib.ktruss_mlp_workspace_bytes(rows))
    if work is None or work.numel() < nbytes:
        work = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=X.device)
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=X.device)
    _check(lib.ktruss_mlp_loss_grad(_ptr(params), _ptr(X), _ptr(T), rows, _ptr(loss), _ptr(grad), _ptr(work),
                                    work.numel(), _stream(stream)))
    return loss, grad


def ktruss_mlp_adam(params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    lib = load()
    _cost_model_sigs(lib)
    _check(lib.ktruss_mlp_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), step, lr, beta1, beta2, eps,
                               _stream(stream)))
