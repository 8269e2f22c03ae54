"""gf2pls: PLS decomposition and RREF of dense GF(2) matrices on MI355X (gfx950).

Thin ctypes binding over ``libgf2pls.so`` (see ``include/gf2pls.h``).  Every
step of the method runs in the library's HIP kernels; PyTorch only provides
device memory and the stream.  There is no CPU fallback: if the library is
missing, importing the binding raises.

Matrices are ``torch.int64`` CUDA tensors of shape ``(m, stride)`` holding the
bit-packed rows (column j of row i is bit j % 64 of word j // 64, LSB first).
"""
from __future__ import annotations

import ctypes
import os

import torch

from .build import LIB as _LIB_PATH

__all__ = ["Sched", "Mat", "get_lib", "default_sched", "pls", "pls_noalloc", "rref", "solve", "kernel_basis", "m4ri", "rref_mp", "addmul", "to_device",
           "to_host", "workspace", "Batch", "SCHUR_XOR", "SCHUR_MFMA", "SCHUR_FP4", "GF2Error"]

SCHUR_XOR = 0
SCHUR_MFMA = 1
SCHUR_FP4 = 2


class GF2Error(RuntimeError):
    pass


class Mat(ctypes.Structure):
    _fields_ = [("words", ctypes.c_void_p), ("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("stride", ctypes.c_int64)]


class Sched(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("tables", ctypes.c_int32), ("cutoff", ctypes.c_int32),
                ("schur", ctypes.c_int32)]

    def astuple(self):
        return (self.k, self.tables, self.cutoff, self.schur)

    def __repr__(self):
        return f"Sched(k={self.k}, tables={self.tables}, cutoff={self.cutoff}, schur={self.schur})"


class BatchItem(ctypes.Structure):
    _fields_ = [("words", ctypes.c_void_p), ("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("stride", ctypes.c_int64), ("P", ctypes.c_void_p), ("Q", ctypes.c_void_p)]


class MlpNet(ctypes.Structure):
    _fields_ = [("params", ctypes.c_void_p), ("S", ctypes.c_int32)]


class ProfStats(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("total_ops", ctypes.c_double)]


class ProfLaunch(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double), ("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("k", ctypes.c_int64)]


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is not built; run python -m paper_1006_1744_amd.build")
    L = ctypes.CDLL(_LIB_PATH)
    vp, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_size_t
    L.gf2_ctx_create.argtypes = [ctypes.POINTER(vp), i32]
    L.gf2_ctx_create.restype = i32
    L.gf2_ctx_destroy.argtypes = [vp]
    L.gf2_ctx_destroy.restype = None
    L.gf2_status_str.argtypes = [i32]
    L.gf2_status_str.restype = ctypes.c_char_p
    L.gf2_default_sched.argtypes = [ctypes.POINTER(Sched)]
    L.gf2_default_sched.restype = None
    L.gf2_sched_valid.argtypes = [ctypes.POINTER(Sched)]
    L.gf2_sched_valid.restype = i32
    L.gf2_pls_workspace_bytes.argtypes = [i64, i64, ctypes.POINTER(Sched)]
    L.gf2_pls_workspace_bytes.restype = sz
    L.gf2_pls.argtypes = [vp, Mat, vp, vp, vp, ctypes.POINTER(Sched), vp, sz, vp]
    L.gf2_pls.restype = i32
    L.gf2_pls_noalloc.argtypes = [vp, Mat, vp, vp, vp, ctypes.POINTER(Sched), vp]
    L.gf2_pls_noalloc.restype = i32
    L.gf2_pls_noalloc_max_bytes.argtypes = []
    L.gf2_pls_noalloc_max_bytes.restype = sz
    L.gf2_pls_unpack.argtypes = [vp, Mat, vp, vp, Mat, Mat, vp]
    L.gf2_pls_unpack.restype = i32
    L.gf2_rref_workspace_bytes.argtypes = [i64, i64]
    L.gf2_rref_workspace_bytes.restype = sz
    L.gf2_rref.argtypes = [vp, Mat, vp, vp, Mat, ctypes.POINTER(Sched), vp, sz, vp]
    L.gf2_rref.restype = i32
    L.gf2_m4ri_workspace_bytes.argtypes = [i64, i64]
    L.gf2_m4ri_workspace_bytes.restype = sz
    L.gf2_m4ri.argtypes = [vp, Mat, vp, vp, ctypes.POINTER(Sched), vp, sz, vp]
    L.gf2_m4ri.restype = i32
    L.gf2_rref_mp_workspace_bytes.argtypes = [i64, i64, ctypes.POINTER(Sched)]
    L.gf2_rref_mp_workspace_bytes.restype = sz
    L.gf2_rref_mp.argtypes = [vp, Mat, vp, vp, ctypes.c_float, ctypes.POINTER(ctypes.c_int32),
                              ctypes.POINTER(Sched), vp, sz, vp]
    L.gf2_rref_mp.restype = i32
    L.gf2_solve_workspace_bytes.argtypes = [i64, i64, i64]
    L.gf2_solve_workspace_bytes.restype = sz
    L.gf2_solve.argtypes = [vp, Mat, vp, vp, vp, Mat, Mat, vp, ctypes.POINTER(Sched), vp, sz, vp]
    L.gf2_solve.restype = i32
    L.gf2_kernel_basis_workspace_bytes.argtypes = [i64, i64]
    L.gf2_kernel_basis_workspace_bytes.restype = sz
    L.gf2_kernel_basis.argtypes = [vp, Mat, vp, vp, Mat, ctypes.POINTER(Sched), vp, sz, vp]
    L.gf2_kernel_basis.restype = i32
    L.gf2_pls_batched_workspace_bytes.argtypes = [i64]
    L.gf2_pls_batched_workspace_bytes.restype = sz
    L.gf2_pls_batched.argtypes = [vp, vp, i64, vp, vp, ctypes.POINTER(Sched), vp, sz, vp]
    L.gf2_pls_batched.restype = i32
    L.gf2_sched_candidates.argtypes = [i64, i64, i32, ctypes.POINTER(Sched), i32]
    L.gf2_sched_candidates.restype = i32
    L.gf2_autotune_workspace_bytes.argtypes = [i64, i64, ctypes.POINTER(Sched), i32]
    L.gf2_autotune_workspace_bytes.restype = sz
    L.gf2_autotune.argtypes = [vp, Mat, Mat, ctypes.POINTER(Sched), i32, i32,
                               ctypes.POINTER(ctypes.c_float), ctypes.POINTER(Sched), vp, sz, vp]
    L.gf2_autotune.restype = i32
    L.gf2_autotune_batched.argtypes = [vp, vp, vp, i64, vp, ctypes.POINTER(Sched), i32, i32,
                                       ctypes.POINTER(ctypes.c_float), ctypes.POINTER(Sched), vp,
                                       sz, vp]
    L.gf2_autotune_batched.restype = i32
    fp = ctypes.c_float
    L.gf2_mlp_param_count.argtypes = [i32]
    L.gf2_mlp_param_count.restype = i64
    L.gf2_mlp_init.argtypes = [vp, MlpNet, ctypes.c_uint64, vp]
    L.gf2_mlp_init.restype = i32
    L.gf2_mlp_forward.argtypes = [vp, MlpNet, vp, i64, vp, vp]
    L.gf2_mlp_forward.restype = i32
    L.gf2_mlp_grad_workspace_bytes.argtypes = [i32, i64]
    L.gf2_mlp_grad_workspace_bytes.restype = sz
    L.gf2_mlp_grad.argtypes = [vp, MlpNet, vp, vp, vp, i64, fp, vp, vp, sz, vp]
    L.gf2_mlp_grad.restype = i32
    L.gf2_mlp_adam.argtypes = [vp, MlpNet, vp, vp, vp, fp, fp, fp, fp, i32, vp]
    L.gf2_mlp_adam.restype = i32
    L.gf2_costmodel_predict.argtypes = [vp, MlpNet, vp, i64, vp, vp, vp]
    L.gf2_costmodel_predict.restype = i32
    L.gf2_features.argtypes = [vp, vp, i64, vp, vp, vp]
    L.gf2_features.restype = i32
    L.gf2_ctx_set_learned_workspace_bytes.argtypes = []
    L.gf2_ctx_set_learned_workspace_bytes.restype = sz
    L.gf2_ctx_set_learned.argtypes = [vp, MlpNet, vp, fp, fp, fp, vp, sz, vp]
    L.gf2_ctx_set_learned.restype = i32
    L.gf2_ctx_learned_sched.argtypes = [vp, i64, i64, ctypes.POINTER(Sched)]
    L.gf2_ctx_learned_sched.restype = i32
    L.gf2_addmul_workspace_bytes.argtypes = [i64, i64, i64]
    L.gf2_addmul_workspace_bytes.restype = sz
    L.gf2_addmul.argtypes = [vp, Mat, Mat, Mat, i32, vp, sz, vp]
    L.gf2_addmul.restype = i32
    L.gf2_prof_enable.argtypes = [vp, vp, i64]
    L.gf2_prof_enable.restype = i32
    L.gf2_prof_read.argtypes = [vp, ctypes.POINTER(ProfStats)]
    L.gf2_prof_read.restype = i32
    L.gf2_prof_read_launches.argtypes = [vp, ctypes.POINTER(ProfLaunch), i64,
                                         ctypes.POINTER(ctypes.c_int64)]
    L.gf2_prof_read_launches.restype = i32
    return L


_lib_handle = None
_ctx = {}


def get_lib():
    """The loaded libgf2pls (raises ImportError if it has not been built)."""
    global _lib_handle
    if _lib_handle is None:
        _lib_handle = _load()
    return _lib_handle


def __getattr__(name):
    if name == "lib":
        return get_lib()
    raise AttributeError(name)


def ctx(device: int | None = None):
    dev = torch.cuda.current_device() if device is None else device
    if dev not in _ctx:
        h = ctypes.c_void_p()
        _check(get_lib().gf2_ctx_create(ctypes.byref(h), dev))
        _ctx[dev] = h
    return _ctx[dev]


def _check(rc: int):
    if rc != 0:
        raise GF2Error(f"gf2 error {rc}: {get_lib().gf2_status_str(rc).decode()}")


def default_sched() -> Sched:
    s = Sched()
    get_lib().gf2_default_sched(ctypes.byref(s))
    return s


def sched(k=8, tables=8, cutoff=2048, schur=SCHUR_FP4) -> Sched:
    return Sched(k, tables, cutoff, schur)


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _mat(t: torch.Tensor, m: int, n: int) -> Mat:
    if t.dtype != torch.int64 or not t.is_cuda or t.dim() != 2 or not t.is_contiguous():
        raise ValueError("matrix must be a contiguous 2-D int64 CUDA tensor")
    if t.shape[0] != m:
        raise ValueError("row count mismatch")
    return Mat(t.data_ptr(), m, n, t.shape[1])


def workspace(nbytes: int, device=None) -> torch.Tensor:
    """Caller-owned workspace (256-byte aligned by the caching allocator)."""
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8,
                       device=device if device is not None else "cuda")


def to_device(a, device="cuda") -> torch.Tensor:
    """numpy uint64 (m, stride) -> int64 CUDA tensor with the same bits."""
    import numpy as np
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).to(device)


def to_host(t: torch.Tensor):
    import numpy as np
    return t.cpu().numpy().view(np.uint64)


def pls_workspace_bytes(m: int, n: int, s: Sched | None = None) -> int:
    return int(get_lib().gf2_pls_workspace_bytes(m, n, ctypes.byref(s) if s is not None else None))


def pls(A: torch.Tensor, m: int, n: int, s: Sched | None = None, ws: torch.Tensor | None = None,
        P: torch.Tensor | None = None, Q: torch.Tensor | None = None,
        rank: torch.Tensor | None = None, stream=None):
    """In-place PLS of A.  Returns (P, Q, rank) int32 CUDA tensors (asynchronous)."""
    dev = A.device
    nb = pls_workspace_bytes(m, n, s)
    if nb == 0:
        raise GF2Error("invalid size or schedule")
    if ws is None or ws.numel() < nb:
        ws = workspace(nb, dev)
    P = torch.empty(max(m, 1), dtype=torch.int32, device=dev) if P is None else P
    Q = torch.empty(max(n, 1), dtype=torch.int32, device=dev) if Q is None else Q
    rank = torch.empty(1, dtype=torch.int32, device=dev) if rank is None else rank
    _check(get_lib().gf2_pls(ctx(dev.index), _mat(A, m, n), P.data_ptr(), Q.data_ptr(), rank.data_ptr(),
                       ctypes.byref(s) if s is not None else None, ws.data_ptr(), ws.numel(),
                       _stream(stream)))
    return P[:m], Q[:n], rank


def pls_noalloc(A: torch.Tensor, m: int, n: int, s: Sched | None = None,
                P: torch.Tensor | None = None, Q: torch.Tensor | None = None,
                rank: torch.Tensor | None = None, stream=None):
    """gf2_pls_noalloc: in-place PLS of A using the library's fixed per-device
    scratch instead of a workspace.  P, Q and rank must be passed in by callers
    that cannot allocate; returns (P, Q, rank)."""
    dev = A.device
    P = torch.empty(max(m, 1), dtype=torch.int32, device=dev) if P is None else P
    Q = torch.empty(max(n, 1), dtype=torch.int32, device=dev) if Q is None else Q
    rank = torch.empty(1, dtype=torch.int32, device=dev) if rank is None else rank
    _check(get_lib().gf2_pls_noalloc(ctx(dev.index), _mat(A, m, n), P.data_ptr(), Q.data_ptr(),
                                     rank.data_ptr(), ctypes.byref(s) if s is not None else None,
                                     _stream(stream)))
    return P[:m], Q[:n], rank


class Batch:
    """Descriptors for gf2_pls_batched over a list of device matrices.

    mats[j] is an int64 CUDA tensor (m_j, stride_j) factored in place; the
    descriptors, P/Q buffers, ranks and workspace are allocated here once, so
    that ``run`` enqueues kernels only (and can be captured into a graph).
    """

    def __init__(self, mats, shapes, device=None):
        if len(mats) != len(shapes):
            raise ValueError("one shape per matrix")
        dev = torch.device(device) if device is not None else (
            mats[0].device if mats else torch.device("cuda"))
        self.device = dev
        self.count = len(mats)
        self.shapes = [(int(m), int(n)) for m, n in shapes]
        self.p_off, self.q_off = [], []
        pm = pn = 0
        for m, n in self.shapes:
            self.p_off.append(pm)
            self.q_off.append(pn)
            pm += m
            pn += n
        self.P = torch.empty(max(pm, 1), dtype=torch.int32, device=dev)
        self.Q = torch.empty(max(pn, 1), dtype=torch.int32, device=dev)
        arr = (BatchItem * max(self.count, 1))()
        for j, (t, (m, n)) in enumerate(zip(mats, self.shapes)):
            if t.dtype != torch.int64 or not t.is_cuda or t.dim() != 2 or not t.is_contiguous():
                raise ValueError("matrix must be a contiguous 2-D int64 CUDA tensor")
            if t.shape[0] != m:
                raise ValueError("row count mismatch")
            arr[j] = BatchItem(t.data_ptr(), m, n, t.shape[1],
                               self.P.data_ptr() + 4 * self.p_off[j],
                               self.Q.data_ptr() + 4 * self.q_off[j])
        raw = bytes(arr)
        self.items = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(dev)
        self.ranks = torch.empty(max(self.count, 1), dtype=torch.int32, device=dev)
        nb = int(get_lib().gf2_pls_batched_workspace_bytes(self.count))
        self.ws = workspace(nb, dev)
        self.per_item = None
        self.mats = list(mats)

    def set_scheds(self, scheds):
        """Per-matrix schedules (Sched or (k, tables, cutoff, schur) tuples); None clears."""
        if scheds is None:
            self.per_item = None
            return
        rows = [x.astuple() if isinstance(x, Sched) else tuple(x) for x in scheds]
        if len(rows) != self.count:
            raise ValueError("one schedule per matrix")
        self.per_item = torch.tensor(rows, dtype=torch.int32).to(self.device)

    def run(self, s: Sched | None = None, stream=None):
        """Enqueue the batched decomposition (asynchronous)."""
        per = self.per_item.data_ptr() if self.per_item is not None else None
        _check(get_lib().gf2_pls_batched(ctx(self.device.index), self.items.data_ptr(), self.count,
                                         self.ranks.data_ptr(), per,
                                         ctypes.byref(s) if s is not None else None,
                                         self.ws.data_ptr(), self.ws.numel(), _stream(stream)))
        return self.ranks[:self.count]

    def pq(self, j: int):
        m, n = self.shapes[j]
        return (self.P[self.p_off[j]:self.p_off[j] + m], self.Q[self.q_off[j]:self.q_off[j] + n])


def sched_candidates(m: int, n: int, batched: bool = False) -> list:
    """The deduplicated candidate schedules for an m x n problem (host list)."""
    L = get_lib()
    cnt = L.gf2_sched_candidates(m, n, int(batched), None, 0)
    if cnt < 0:
        raise GF2Error(f"gf2 error {cnt}")
    arr = (Sched * max(cnt, 1))()
    L.gf2_sched_candidates(m, n, int(batched), arr, cnt)
    return [Sched(*arr[i].astuple()) for i in range(cnt)]


def autotune(A_trial: torch.Tensor, m: int, n: int, cands=None, reps: int = 2,
             A_work: torch.Tensor | None = None, stream=None):
    """Time every candidate schedule on A_trial (left unchanged); returns
    (best Sched, list of fastest times in ms, one per candidate)."""
    cands = sched_candidates(m, n) if cands is None else list(cands)
    dev = A_trial.device
    A_work = torch.empty_like(A_trial) if A_work is None else A_work
    arr = (Sched * max(len(cands), 1))(*[Sched(*c.astuple()) for c in cands])
    ms = (ctypes.c_float * max(len(cands), 1))()
    best = Sched()
    nb = int(get_lib().gf2_autotune_workspace_bytes(m, n, arr, len(cands)))
    ws = workspace(nb, dev)
    _check(get_lib().gf2_autotune(ctx(dev.index), _mat(A_trial, m, n), _mat(A_work, m, n), arr,
                                  len(cands), reps, ms, ctypes.byref(best), ws.data_ptr(),
                                  ws.numel(), _stream(stream)))
    return Sched(*best.astuple()), [float(ms[i]) for i in range(len(cands))]


def autotune_batched(trial: "Batch", work: "Batch", cands=None, reps: int = 2, stream=None):
    """Time every candidate (k, tables) on the batch `trial` (restored into the
    same-shaped batch `work` before each run); returns (best, times in ms)."""
    cands = sched_candidates(64, 64, batched=True) if cands is None else list(cands)
    arr = (Sched * max(len(cands), 1))(*[Sched(*c.astuple()) for c in cands])
    ms = (ctypes.c_float * max(len(cands), 1))()
    best = Sched()
    _check(get_lib().gf2_autotune_batched(ctx(work.device.index), trial.items.data_ptr(),
                                          work.items.data_ptr(), work.count, work.ranks.data_ptr(),
                                          arr, len(cands), reps, ms, ctypes.byref(best),
                                          work.ws.data_ptr(), work.ws.numel(), _stream(stream)))
    return Sched(*best.astuple()), [float(ms[i]) for i in range(len(cands))]


# ------------------------------------------------------------- cost model
def mlp_param_count(S: int) -> int:
    n = int(get_lib().gf2_mlp_param_count(S))
    if n < 0:
        raise GF2Error(f"gf2 error {n}")
    return n


def _f32(t: torch.Tensor, name: str):
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
    return t.data_ptr()


def mlp_init(params: torch.Tensor, S: int, seed: int, stream=None):
    _check(get_lib().gf2_mlp_init(ctx(params.device.index), MlpNet(_f32(params, "params"), S),
                                  seed, _stream(stream)))
    return params


def mlp_forward(params: torch.Tensor, S: int, feats: torch.Tensor, stream=None) -> torch.Tensor:
    N = feats.shape[0]
    out = torch.empty((N, S), dtype=torch.float32, device=params.device)
    _check(get_lib().gf2_mlp_forward(ctx(params.device.index), MlpNet(_f32(params, "params"), S),
                                     _f32(feats, "feats"), N, out.data_ptr(), _stream(stream)))
    return out


def mlp_grad(params: torch.Tensor, S: int, feats: torch.Tensor, target: torch.Tensor,
             mask: torch.Tensor, inv_count: float, ws: torch.Tensor | None = None,
             out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Gradient of the masked squared error (P values), then the loss."""
    N = feats.shape[0]
    dev = params.device
    nb = int(get_lib().gf2_mlp_grad_workspace_bytes(S, N))
    if ws is None or ws.numel() < nb:
        ws = workspace(nb, dev)
    out = torch.empty(mlp_param_count(S) + 1, dtype=torch.float32, device=dev) if out is None else out
    _check(get_lib().gf2_mlp_grad(ctx(dev.index), MlpNet(_f32(params, "params"), S),
                                  _f32(feats, "feats"), _f32(target, "target"), _f32(mask, "mask"),
                                  N, float(inv_count), out.data_ptr(), ws.data_ptr(), ws.numel(),
                                  _stream(stream)))
    return out


def mlp_adam(params: torch.Tensor, S: int, grad: torch.Tensor, m1: torch.Tensor, m2: torch.Tensor,
             lr: float, step: int, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
             stream=None):
    _check(get_lib().gf2_mlp_adam(ctx(params.device.index), MlpNet(_f32(params, "params"), S),
                                  _f32(grad, "grad"), _f32(m1, "m1"), _f32(m2, "m2"), lr, beta1,
                                  beta2, eps, step, _stream(stream)))


def costmodel_predict(params: torch.Tensor, S: int, feats: torch.Tensor, table: torch.Tensor,
                      stream=None) -> torch.Tensor:
    """Per problem, the table row (k, tables, cutoff, schur) of the smallest
    predicted log time; table is an int32 CUDA tensor (S, 4)."""
    N = feats.shape[0]
    if table.dtype != torch.int32 or tuple(table.shape) != (S, 4):
        raise ValueError("table must be an int32 (S, 4) tensor")
    out = torch.empty((max(N, 1), 4), dtype=torch.int32, device=params.device)
    _check(get_lib().gf2_costmodel_predict(ctx(params.device.index),
                                           MlpNet(_f32(params, "params"), S), _f32(feats, "feats"),
                                           N, table.data_ptr(), out.data_ptr(), _stream(stream)))
    return out[:N]


def items_of(mats, shapes, device=None) -> torch.Tensor:
    """Device descriptor array (gf2_batch_item[]) for int64 CUDA matrices (P, Q
    unset): the argument of gf2_features."""
    arr = (BatchItem * max(len(mats), 1))()
    for j, (t, (m, n)) in enumerate(zip(mats, shapes)):
        if t.dtype != torch.int64 or not t.is_cuda or t.dim() != 2 or not t.is_contiguous():
            raise ValueError("matrix must be a contiguous 2-D int64 CUDA tensor")
        arr[j] = BatchItem(t.data_ptr(), m, n, t.shape[1], None, None)
    dev = mats[0].device if mats else torch.device(device or "cuda")
    return torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8).to(dev)


def features(items: torch.Tensor, count: int, r_hint: torch.Tensor | None = None,
             stream=None) -> torch.Tensor:
    """Cost-model features of `count` matrices computed on the device from the
    matrices themselves (gf2_features): float32 CUDA (count, 4)."""
    out = torch.empty((max(count, 1), 4), dtype=torch.float32, device=items.device)
    _check(get_lib().gf2_features(ctx(items.device.index), items.data_ptr(), count,
                                  r_hint.data_ptr() if r_hint is not None else None,
                                  out.data_ptr(), _stream(stream)))
    return out[:count]


def set_learned(params: torch.Tensor | None, S: int = 0, table: torch.Tensor | None = None,
                log2_lo: float = 6.0, log2_hi: float = 16.0, log2_mn_hi: float = 31.0, device=None,
                stream=None):
    """Install (or with params None remove) the learned choice gf2_pls uses when
    it is given no schedule (gf2_ctx_set_learned).  Waits on the stream."""
    dev = torch.cuda.current_device() if device is None else device
    L = get_lib()
    if params is None:
        _check(L.gf2_ctx_set_learned(ctx(dev), MlpNet(None, 0), None, 0.0, 0.0, 0.0, None, 0,
                                     _stream(stream)))
        return
    if table is None or table.dtype != torch.int32 or tuple(table.shape) != (S, 4):
        raise ValueError("table must be an int32 (S, 4) tensor")
    ws = workspace(int(L.gf2_ctx_set_learned_workspace_bytes()), params.device)
    _check(L.gf2_ctx_set_learned(ctx(dev), MlpNet(_f32(params, "params"), S), table.data_ptr(),
                                 float(log2_lo), float(log2_hi), float(log2_mn_hi), ws.data_ptr(),
                                 ws.numel(), _stream(stream)))


def learned_sched(m: int, n: int, device=None):
    """(schedule a call without one would use for m x n, True if it is learned)."""
    dev = torch.cuda.current_device() if device is None else device
    out = Sched()
    rc = get_lib().gf2_ctx_learned_sched(ctx(dev), m, n, ctypes.byref(out))
    if rc < 0:
        _check(rc)
    return Sched(*out.astuple()), rc == 1


def pls_unpack(A_pls: torch.Tensor, m: int, n: int, Q: torch.Tensor, rank: torch.Tensor,
               stream=None):
    """Explicit (L, S) from a PLS result: L m x min(m,n), S min(m,n) x n (int64 CUDA
    tensors, packed rows); only the first rank columns of L and rows of S count."""
    dev = A_pls.device
    rmax = min(m, n)
    L = torch.zeros((max(m, 1), max((rmax + 63) // 64, 1)), dtype=torch.int64, device=dev)[:m]
    S = torch.zeros((max(rmax, 1), max((n + 63) // 64, 1)), dtype=torch.int64, device=dev)[:rmax]
    _check(get_lib().gf2_pls_unpack(ctx(dev.index), _mat(A_pls, m, n), Q.data_ptr(), rank.data_ptr(),
                                    _mat(L, m, rmax), _mat(S, rmax, n), _stream(stream)))
    return L, S


def rref_workspace_bytes(m: int, n: int) -> int:
    return int(get_lib().gf2_rref_workspace_bytes(m, n))


def rref(A_pls: torch.Tensor, m: int, n: int, Q: torch.Tensor, rank: torch.Tensor,
         R: torch.Tensor | None = None, ws: torch.Tensor | None = None, s: Sched | None = None,
         stream=None):
    """RREF of the original matrix from its PLS; returns R (m, stride) int64.
    The triangular solve's products use s.schur (None: the default schedule)."""
    dev = A_pls.device
    R = torch.empty_like(A_pls) if R is None else R
    nb = rref_workspace_bytes(m, n)
    if ws is None or ws.numel() < nb:
        ws = workspace(nb, dev)
    _check(get_lib().gf2_rref(ctx(dev.index), _mat(A_pls, m, n), Q.data_ptr(), rank.data_ptr(),
                              _mat(R, m, n), ctypes.byref(s) if s is not None else None,
                              ws.data_ptr(), ws.numel(), _stream(stream)))
    return R


def m4ri(A: torch.Tensor, m: int, n: int, s: Sched | None = None, Q: torch.Tensor | None = None,
         rank: torch.Tensor | None = None, ws: torch.Tensor | None = None, stream=None):
    """M4RI (gf2_m4ri): A is replaced by its RREF.  Returns (Q, rank) int32 CUDA
    tensors (pivot columns first), asynchronous."""
    dev = A.device
    Q = torch.empty(max(n, 1), dtype=torch.int32, device=dev) if Q is None else Q
    rank = torch.empty(1, dtype=torch.int32, device=dev) if rank is None else rank
    nb = int(get_lib().gf2_m4ri_workspace_bytes(m, n))
    if ws is None or ws.numel() < nb:
        ws = workspace(nb, dev)
    _check(get_lib().gf2_m4ri(ctx(dev.index), _mat(A, m, n), Q.data_ptr(), rank.data_ptr(),
                              ctypes.byref(s) if s is not None else None, ws.data_ptr(), ws.numel(),
                              _stream(stream)))
    return Q[:n], rank


def rref_mp(A: torch.Tensor, m: int, n: int, threshold: float = 0.15, s: Sched | None = None,
            Q: torch.Tensor | None = None, rank: torch.Tensor | None = None,
            ws: torch.Tensor | None = None, stream=None):
    """The M+P hybrid (gf2_rref_mp): A is replaced by its RREF.  Returns (Q, rank,
    switch panel or -1).  Waits on the stream (density checks)."""
    dev = A.device
    Q = torch.empty(max(n, 1), dtype=torch.int32, device=dev) if Q is None else Q
    rank = torch.empty(1, dtype=torch.int32, device=dev) if rank is None else rank
    nb = int(get_lib().gf2_rref_mp_workspace_bytes(m, n, ctypes.byref(s) if s is not None else None))
    if nb == 0:
        raise GF2Error("invalid size or schedule")
    if ws is None or ws.numel() < nb:
        ws = workspace(nb, dev)
    sw = ctypes.c_int32(-2)
    _check(get_lib().gf2_rref_mp(ctx(dev.index), _mat(A, m, n), Q.data_ptr(), rank.data_ptr(),
                                 float(threshold), ctypes.byref(sw),
                                 ctypes.byref(s) if s is not None else None, ws.data_ptr(),
                                 ws.numel(), _stream(stream)))
    return Q[:n], rank, int(sw.value)


def solve(A_pls: torch.Tensor, m: int, n: int, P: torch.Tensor, Q: torch.Tensor,
          rank: torch.Tensor, B: torch.Tensor, nrhs: int, X: torch.Tensor | None = None,
          bad: torch.Tensor | None = None, ws: torch.Tensor | None = None, s: Sched | None = None,
          stream=None):
    """Solve A X = B from A's PLS (gf2_solve).  B: (m, stride) int64 CUDA tensor of
    nrhs packed columns.  Returns (X (n, ceil(nrhs/64)) int64, bad int64 bit mask of
    the inconsistent right-hand sides), asynchronous."""
    dev = A_pls.device
    nrw = max((nrhs + 63) // 64, 1)
    X = torch.empty((max(n, 1), nrw), dtype=torch.int64, device=dev)[:n] if X is None else X
    bad = torch.empty(nrw, dtype=torch.int64, device=dev) if bad is None else bad
    nb = int(get_lib().gf2_solve_workspace_bytes(m, n, nrhs))
    if ws is None or ws.numel() < nb:
        ws = workspace(nb, dev)
    _check(get_lib().gf2_solve(ctx(dev.index), _mat(A_pls, m, n), P.data_ptr(), Q.data_ptr(),
                               rank.data_ptr(), _mat(B, m, nrhs), _mat(X, n, nrhs), bad.data_ptr(),
                               ctypes.byref(s) if s is not None else None, ws.data_ptr(),
                               ws.numel(), _stream(stream)))
    return X, bad


def kernel_basis(A_pls: torch.Tensor, m: int, n: int, Q: torch.Tensor, rank: torch.Tensor,
                 K: torch.Tensor | None = None, ws: torch.Tensor | None = None,
                 s: Sched | None = None, stream=None) -> torch.Tensor:
    """Null-space basis from A's PLS (gf2_kernel_basis): (n, ceil(n/64)) int64 whose
    first n - rank rows are the basis vectors, the rest zero."""
    dev = A_pls.device
    nw = max((n + 63) // 64, 1)
    K = torch.empty((max(n, 1), nw), dtype=torch.int64, device=dev)[:n] if K is None else K
    nb = int(get_lib().gf2_kernel_basis_workspace_bytes(m, n))
    if ws is None or ws.numel() < nb:
        ws = workspace(nb, dev)
    _check(get_lib().gf2_kernel_basis(ctx(dev.index), _mat(A_pls, m, n), Q.data_ptr(),
                                      rank.data_ptr(), _mat(K, n, n),
                                      ctypes.byref(s) if s is not None else None, ws.data_ptr(),
                                      ws.numel(), _stream(stream)))
    return K


def addmul(C: torch.Tensor, A: torch.Tensor, B: torch.Tensor, m: int, k: int, n: int,
           variant: int = SCHUR_FP4, ws: torch.Tensor | None = None, stream=None):
    """C <- C + A * B over GF(2) (A m x k, B k x n, C m x n)."""
    dev = C.device
    nb = int(get_lib().gf2_addmul_workspace_bytes(m, k, n))
    if ws is None or ws.numel() < nb:
        ws = workspace(nb, dev)
    _check(get_lib().gf2_addmul(ctx(dev.index), _mat(C, m, n), _mat(A, m, k), _mat(B, k, n), variant,
                          ws.data_ptr(), ws.numel(), _stream(stream)))
    return C


_prof_logs = {}


def prof_enable(slots: int = 1 << 16, device=None):
    """Time every Schur-product launch with HIP events (see gf2_prof_enable)."""
    dev = torch.cuda.current_device() if device is None else device
    log = torch.zeros(3 * slots, dtype=torch.int32, device=f"cuda:{dev}")
    _prof_logs[dev] = log
    _check(get_lib().gf2_prof_enable(ctx(dev), log.data_ptr(), slots))


def prof_disable(device=None):
    dev = torch.cuda.current_device() if device is None else device
    _check(get_lib().gf2_prof_enable(ctx(dev), None, 0))
    _prof_logs.pop(dev, None)


def prof_read(device=None) -> dict:
    """Launch count, summed event milliseconds and summed 2*M*N*K of the product
    launches recorded since the last read."""
    dev = torch.cuda.current_device() if device is None else device
    st = ProfStats()
    _check(get_lib().gf2_prof_read(ctx(dev), ctypes.byref(st)))
    return {"launches": int(st.launches), "ms": float(st.total_ms), "ops": float(st.total_ops)}


def prof_launches(max_count: int = 1 << 16, device=None) -> list[tuple]:
    """(ms, M, N, K) of each recorded product launch, in launch order."""
    dev = torch.cuda.current_device() if device is None else device
    arr = (ProfLaunch * max_count)()
    cnt = ctypes.c_int64()
    _check(get_lib().gf2_prof_read_launches(ctx(dev), arr, max_count, ctypes.byref(cnt)))
    return [(arr[i].ms, arr[i].m, arr[i].n, arr[i].k) for i in range(cnt.value)]
