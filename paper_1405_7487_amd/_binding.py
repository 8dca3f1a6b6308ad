"""Thin ctypes binding of libfmm_hip.so (the C ABI of include/fmm.h).

Argument marshalling only: every step of the evaluation runs in the HIP
library.  PyTorch supplies device memory (its caching allocator is handed to
the library as the plan allocator) and the current stream.  If the library
is not built, loading fails loudly; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfmm_hip.so")

FMM_OK, FMM_ERR_INVALID, FMM_ERR_NOMEM, FMM_ERR_DEVICE, FMM_ERR_UNSUPPORTED, FMM_ERR_NONFINITE = range(6)
FMM_F64, FMM_F32 = 0, 1
PREC = {"fp64": 0, "mixed": 1}

# Every symbol include/fmm.h declares.
EXPORTS = (
    "fmm_params_default", "fmm_build", "fmm_evaluate_plan", "fmm_evaluate", "fmm_adjoint",
    "fmm_plan_stats", "fmm_export_tree", "fmm_set_timing", "fmm_destroy", "fmm_last_error",
    "fmm_debug_mfma_layout", "fmm_list_digest", "fmm_count_body_pairs", "fmm_evaluate_noalloc",
    "fmm_let_evaluate",
)


class FMMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[fmm status {code}] {msg}")
        self.code = code


class _Params(C.Structure):
    _fields_ = [("p", C.c_int32), ("theta", C.c_double), ("ncrit", C.c_int32), ("precision", C.c_int32),
                ("coarse_fp64_levels", C.c_int32), ("kahan", C.c_int32), ("tight", C.c_int32),
                ("m2l_sparse", C.c_int32), ("m2l_rotation", C.c_int32), ("mutual", C.c_int32)]


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class _Allocator(C.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", C.c_void_p)]


class _Stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("ncell", C.c_int64), ("nleaf", C.c_int64), ("depth", C.c_int32),
                ("p", C.c_int32), ("n_m2l", C.c_int64), ("n_m2l_same", C.c_int64), ("n_m2l_cross", C.c_int64),
                ("n_p2p", C.c_int64), ("p2p_body_pairs", C.c_int64), ("m2l_stencil", C.c_int64),
                ("m2l_offsets", C.c_int64), ("m2l_slots", C.c_int64), ("device_bytes", C.c_int64),
                ("ms_build", C.c_double), ("ms_tree", C.c_double), ("ms_traverse", C.c_double),
                ("ms_ops", C.c_double),
                ("ms_p2m", C.c_double), ("ms_m2m", C.c_double), ("ms_m2l", C.c_double), ("ms_l2l", C.c_double),
                ("ms_l2p", C.c_double), ("ms_p2p", C.c_double), ("ms_evaluate", C.c_double),
                ("ms_adjoint", C.c_double), ("ms_m2l_cross", C.c_double),
                ("m2l_cross_keys", C.c_int64), ("m2l_cross_batched", C.c_int64),
                ("p2p_cut_leaves", C.c_int64), ("n_m2l_sparse", C.c_int64), ("m2l_rows", C.c_int64),
                ("p2p_mutual_pairs", C.c_int64)]


class _LetStats(C.Structure):
    _fields_ = [("nrank", C.c_int32), ("let_cells", C.c_int64), ("let_far", C.c_int64),
                ("let_body_leaves", C.c_int64), ("let_bodies", C.c_int64), ("let_bytes", C.c_int64),
                ("n_m2l_local", C.c_int64), ("n_p2p_local", C.c_int64), ("n_m2l_remote", C.c_int64),
                ("n_p2p_remote", C.c_int64), ("n_m2p_remote", C.c_int64), ("device_bytes", C.c_int64),
                ("ms_partition", C.c_double), ("ms_build", C.c_double), ("ms_let", C.c_double),
                ("ms_evaluate", C.c_double), ("ms_total", C.c_double)]


class _Export(C.Structure):
    _fields_ = [("keys", C.c_void_p), ("perm", C.c_void_p), ("level", C.c_void_p), ("cell_key", C.c_void_p),
                ("begin", C.c_void_p), ("end", C.c_void_p), ("parent", C.c_void_p), ("child_begin", C.c_void_p),
                ("nchild", C.c_void_p), ("centers", C.c_void_p), ("m2l", C.c_void_p), ("p2p", C.c_void_p)]


_LIB = None


def load():
    """Load the HIP library (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1405_7487_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    L.fmm_params_default.argtypes = [C.POINTER(_Params)]
    L.fmm_build.argtypes = [vp, C.c_int, C.c_int64, C.POINTER(_Params), C.POINTER(_Allocator), vp, C.POINTER(vp)]
    L.fmm_evaluate_plan.argtypes = [vp, vp, vp, vp, vp]
    L.fmm_evaluate.argtypes = [vp, vp, C.c_int, C.c_int64, C.c_int32, C.c_double, C.c_int32, C.c_int32,
                               C.POINTER(_Allocator), vp, vp, vp]
    L.fmm_adjoint.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.fmm_let_evaluate.argtypes = [vp, vp, C.c_int, C.c_int64, C.c_int32, vp, C.POINTER(_Params),
                                   C.POINTER(_Allocator), vp, vp, vp, vp, vp, vp, C.POINTER(_LetStats), vp]
    L.fmm_evaluate_noalloc.argtypes = [vp, vp, C.c_int, C.c_int64, C.c_int32, C.c_double, C.c_int32, C.c_int32,
                                       vp, vp, vp]
    L.fmm_plan_stats.argtypes = [vp, C.POINTER(_Stats)]
    L.fmm_export_tree.argtypes = [vp, C.POINTER(_Export)]
    L.fmm_set_timing.argtypes = [vp, C.c_int32]
    L.fmm_destroy.argtypes = [vp]
    L.fmm_destroy.restype = None
    L.fmm_last_error.restype = C.c_char_p
    L.fmm_debug_mfma_layout.argtypes = [C.c_int32, vp]
    L.fmm_list_digest.argtypes = [vp, C.POINTER(C.c_uint64)]
    L.fmm_count_body_pairs.argtypes = [vp, C.POINTER(C.c_int64)]
    for name in ("fmm_build", "fmm_evaluate_plan", "fmm_evaluate", "fmm_evaluate_noalloc", "fmm_let_evaluate",
                 "fmm_adjoint",
                 "fmm_plan_stats",
                 "fmm_export_tree", "fmm_set_timing", "fmm_debug_mfma_layout", "fmm_list_digest",
                 "fmm_count_body_pairs"):
        getattr(L, name).restype = C.c_int
    _LIB = L
    return L


def _check(code: int):
    if code != FMM_OK:
        msg = load().fmm_last_error().decode(errors="replace")
        raise FMMError(code, msg)


# ---- torch caching allocator as the plan allocator -----------------------
def _torch_alloc(nbytes, stream, ctx):
    try:
        return torch._C._cuda_cudaCachingAllocator_raw_alloc(int(nbytes), int(stream or 0))
    except Exception:  # out of memory: the library reports FMM_ERR_NOMEM
        return None


def _torch_free(ptr, stream, ctx):
    if ptr:
        torch._C._cuda_cudaCachingAllocator_raw_delete(int(ptr))


_ALLOC_CB = _ALLOC_FN(_torch_alloc)
_FREE_CB = _FREE_FN(_torch_free)
_TORCH_ALLOCATOR = _Allocator(_ALLOC_CB, _FREE_CB, None)


class CallbackAllocator:
    """A plan allocator from two Python callables: alloc(nbytes, stream) ->
    device address or None (the library then reports FMM_ERR_NOMEM) and
    free(address, stream).  Keeps the ctypes trampolines alive."""

    def __init__(self, alloc, free):
        def _a(nbytes, stream, ctx):
            try:
                return alloc(int(nbytes), stream)
            except Exception:
                return None

        def _f(ptr, stream, ctx):
            if ptr:
                free(int(ptr), stream)

        self._a = _ALLOC_FN(_a)
        self._f = _FREE_FN(_f)
        self.c = _Allocator(self._a, self._f, None)


def _stream_handle():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return FMM_F64
    if t.dtype == torch.float32:
        return FMM_F32
    raise TypeError(f"unsupported dtype {t.dtype}: use float64 or float32")


def _dev(t: torch.Tensor, name: str, shape=None, dtype=None, device=None):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if device is not None and t.device != device:
        raise ValueError(f"{name} must be on {device}, got {t.device}")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t.contiguous()


def _out(t: torch.Tensor, name: str, shape, dtype, device):
    """An output buffer the library writes into: it must already have the
    right device, dtype and shape and be contiguous (a copy would drop the
    results)."""
    t2 = _dev(t, name, shape, dtype, device)
    if t2.data_ptr() != t.data_ptr():
        raise ValueError(f"{name} must be contiguous")
    return t


def _coords(x: torch.Tensor):
    x = _dev(x, "x")
    if x.dim() != 2 or x.shape[1] != 3:
        raise ValueError(f"x must have shape (N, 3), got {tuple(x.shape)}")
    _dtype_code(x)
    return x


@dataclass
class Params:
    """Method parameters (the paper's P, theta, N_crit) and precision knobs."""
    p: int = 8
    theta: float = 0.4
    ncrit: int = 64
    precision: str = "mixed"          # "mixed" or "fp64"
    coarse_fp64_levels: int = 3
    kahan: bool = True
    tight: bool = False               # acceptance also by cell radii tight to the bodies
    m2l_sparse: int = -1              # same-level tile rows below this many sources per 64
                                      # targets run pair by pair (0: never; -1: 24 in plans
                                      # with at least 1024 tiles)
    m2l_rotation: bool = False        # every M2L pair by rotation, O(p^3), float64 vector units
    mutual: bool = False              # P2P: each unordered leaf pair once, both leaves updated

    def to_c(self) -> _Params:
        if self.precision not in PREC:
            raise ValueError("precision must be 'mixed' or 'fp64'")
        return _Params(int(self.p), float(self.theta), int(self.ncrit), PREC[self.precision],
                       int(self.coarse_fp64_levels), 1 if self.kahan else 0, 1 if self.tight else 0,
                       int(self.m2l_sparse), 1 if self.m2l_rotation else 0, 1 if self.mutual else 0)


class Plan:
    """Tree, lists and buffers for one set of coordinates (fmm_build)."""

    def __init__(self, x: torch.Tensor, params: Params | None = None, torch_allocator: bool = True,
                 timing: bool = False, allocator: CallbackAllocator | None = None):
        L = load()
        self.params = params or Params()
        x = _coords(x)
        self.n = int(x.shape[0])
        self.dtype = x.dtype
        self.device = x.device
        self._h = C.c_void_p()
        cp = self.params.to_c()
        self._allocator = allocator  # keeps the callbacks alive while the plan lives
        if allocator is not None:
            alloc = C.byref(allocator.c)
        else:
            alloc = C.byref(_TORCH_ALLOCATOR) if torch_allocator else None
        with torch.cuda.device(self.device):
            _check(L.fmm_build(C.c_void_p(x.data_ptr()), _dtype_code(x), self.n, C.byref(cp), alloc,
                               _stream_handle(), C.byref(self._h)))
            if timing:
                _check(L.fmm_set_timing(self._h, 1))

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            with torch.cuda.device(self.device):
                load().fmm_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def evaluate(self, q: torch.Tensor, field: bool = True, out=None):
        """Potential (N,) and field (N, 3) for charges q (fmm_evaluate_plan)."""
        q = _dev(q, "q", (self.n,), self.dtype, self.device)
        if out is None:
            phi = torch.empty(self.n, dtype=self.dtype, device=self.device)
            E = torch.empty((self.n, 3), dtype=self.dtype, device=self.device) if field else None
        else:
            phi, E = out
            phi = _out(phi, "phi", (self.n,), self.dtype, self.device)
            if E is not None:
                E = _out(E, "E", (self.n, 3), self.dtype, self.device)
        with torch.cuda.device(self.device):
            _check(load().fmm_evaluate_plan(self._h, C.c_void_p(q.data_ptr()), C.c_void_p(phi.data_ptr()),
                                            C.c_void_p(E.data_ptr()) if E is not None else None,
                                            _stream_handle()))
        return phi, E

    def adjoint(self, q: torch.Tensor, w: torch.Tensor, field_q: torch.Tensor | None = None, out=None):
        """(dL/dq, dL/dx) of L = sum_i w_i phi_i (fmm_adjoint)."""
        q = _dev(q, "q", (self.n,), self.dtype, self.device)
        w = _dev(w, "w", (self.n,), self.dtype, self.device)
        if field_q is not None:
            field_q = _dev(field_q, "field_q", (self.n, 3), self.dtype, self.device)
        if out is None:
            dq = torch.empty(self.n, dtype=self.dtype, device=self.device)
            dx = torch.empty((self.n, 3), dtype=self.dtype, device=self.device)
        else:
            dq, dx = out
            dq = _out(dq, "dq", (self.n,), self.dtype, self.device)
            dx = _out(dx, "dx", (self.n, 3), self.dtype, self.device)
        with torch.cuda.device(self.device):
            _check(load().fmm_adjoint(self._h, C.c_void_p(q.data_ptr()), C.c_void_p(w.data_ptr()),
                                      C.c_void_p(field_q.data_ptr()) if field_q is not None else None,
                                      C.c_void_p(dq.data_ptr()), C.c_void_p(dx.data_ptr()), _stream_handle()))
        return dq, dx

    def stats(self) -> dict:
        st = _Stats()
        _check(load().fmm_plan_stats(self._h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in _Stats._fields_}

    def list_digest(self) -> tuple:
        """(M2L digest, P2P digest) of the plan's lists (fmm_list_digest)."""
        out = (C.c_uint64 * 2)()
        with torch.cuda.device(self.device):
            _check(load().fmm_list_digest(self._h, out))
        return int(out[0]), int(out[1])

    def body_pairs(self) -> int:
        """Sum over P2P leaf pairs of |A| |B| (fmm_count_body_pairs)."""
        out = C.c_int64(0)
        with torch.cuda.device(self.device):
            _check(load().fmm_count_body_pairs(self._h, C.byref(out)))
        return int(out.value)

    def export_tree(self, lists: bool = True) -> dict:
        """Host copies of keys, permutation, cells and (optionally) lists."""
        import numpy as np
        st = self.stats()
        n, nc = self.n, st["ncell"]
        out = dict(keys=np.zeros(n, np.uint64), perm=np.zeros(n, np.int32), level=np.zeros(nc, np.int32),
                   ckey=np.zeros(nc, np.uint64), begin=np.zeros(nc, np.int32), end=np.zeros(nc, np.int32),
                   parent=np.zeros(nc, np.int32), child_begin=np.zeros(nc, np.int32),
                   nchild=np.zeros(nc, np.int32), centers=np.zeros((nc, 3)))
        if lists:
            out["m2l"] = np.zeros((st["n_m2l"], 2), np.int32)
            out["p2p"] = np.zeros((st["n_p2p"], 2), np.int32)
        ptr = lambda a: C.c_void_p(a.ctypes.data) if a is not None and a.size else None
        ex = _Export(ptr(out["keys"]), ptr(out["perm"]), ptr(out["level"]), ptr(out["ckey"]), ptr(out["begin"]),
                     ptr(out["end"]), ptr(out["parent"]), ptr(out["child_begin"]), ptr(out["nchild"]),
                     ptr(out["centers"]), ptr(out.get("m2l")), ptr(out.get("p2p")))
        with torch.cuda.device(self.device):
            _check(load().fmm_export_tree(self._h, C.byref(ex)))
        return out


def build(x: torch.Tensor, p: int = 8, theta: float = 0.4, ncrit: int = 64, precision: str = "mixed",
          **kw) -> Plan:
    return Plan(x, Params(p=p, theta=theta, ncrit=ncrit, precision=precision, **kw))


def evaluate(x: torch.Tensor, q: torch.Tensor, p: int = 8, theta: float = 0.4, ncrit: int = 64,
             precision: str = "mixed", field: bool = True):
    """One-shot evaluation (fmm_evaluate): returns (phi, E)."""
    L = load()
    x = _coords(x)
    n = int(x.shape[0])
    q = _dev(q, "q", (n,), x.dtype, x.device)
    phi = torch.empty(n, dtype=x.dtype, device=x.device)
    E = torch.empty((n, 3), dtype=x.dtype, device=x.device) if field else None
    with torch.cuda.device(x.device):
        _check(L.fmm_evaluate(C.c_void_p(x.data_ptr()), C.c_void_p(q.data_ptr()), _dtype_code(x), n, int(p),
                              float(theta), int(ncrit), PREC[precision], C.byref(_TORCH_ALLOCATOR),
                              C.c_void_p(phi.data_ptr()), C.c_void_p(E.data_ptr()) if E is not None else None,
                              _stream_handle()))
    return phi, E


def evaluate_noalloc(x: torch.Tensor, q: torch.Tensor, p: int = 8, theta: float = 0.4, ncrit: int = 64,
                     precision: str = "mixed", field: bool = True, out=None):
    """fmm_evaluate_noalloc: the one-shot evaluation with every device buffer
    in the library's static scratch (no device allocation by the library).
    out = (phi, E) writes into existing tensors (E may be None)."""
    L = load()
    x = _coords(x)
    n = int(x.shape[0])
    q = _dev(q, "q", (n,), x.dtype, x.device)
    if out is None:
        phi = torch.empty(n, dtype=x.dtype, device=x.device)
        E = torch.empty((n, 3), dtype=x.dtype, device=x.device) if field else None
    else:
        phi = _out(out[0], "phi", (n,), x.dtype, x.device)
        E = _out(out[1], "E", (n, 3), x.dtype, x.device) if out[1] is not None else None
    with torch.cuda.device(x.device):
        _check(L.fmm_evaluate_noalloc(C.c_void_p(x.data_ptr()), C.c_void_p(q.data_ptr()), _dtype_code(x), n,
                                      int(p), float(theta), int(ncrit), PREC[precision], C.c_void_p(phi.data_ptr()),
                                      C.c_void_p(E.data_ptr()) if E is not None else None, _stream_handle()))
    return phi, E


def let_evaluate(x: torch.Tensor, q: torch.Tensor, nrank: int, params: Params | None = None,
                 weights: torch.Tensor | None = None, field: bool = True, work: bool = False) -> dict:
    """fmm_let_evaluate: the evaluation over nrank virtual ranks (ORB
    partition weighted by `weights`, local trees, LETs, remote traversals).

    Returns a dict with phi, E (or None), rank (int32 per body), work_local
    and work_remote (int64 per body, when work=True), pair_stats (numpy,
    nrank x nrank x 11) and stats (dict of fmm_let_stats)."""
    import numpy as np
    L = load()
    params = params or Params()
    x = _coords(x)
    n = int(x.shape[0])
    q = _dev(q, "q", (n,), x.dtype, x.device)
    if weights is not None:
        weights = _dev(weights, "weights", (n,), torch.int64, x.device)
    phi = torch.empty(n, dtype=x.dtype, device=x.device)
    E = torch.empty((n, 3), dtype=x.dtype, device=x.device) if field else None
    rank = torch.empty(n, dtype=torch.int32, device=x.device)
    wl = torch.empty(n, dtype=torch.int64, device=x.device) if work else None
    wr = torch.empty(n, dtype=torch.int64, device=x.device) if work else None
    ps = np.zeros((nrank, nrank, 11), np.int64)
    st = _LetStats()
    cp = params.to_c()
    ptr = lambda t: C.c_void_p(t.data_ptr()) if t is not None else None
    with torch.cuda.device(x.device):
        _check(L.fmm_let_evaluate(ptr(x), ptr(q), _dtype_code(x), n, int(nrank), ptr(weights), C.byref(cp),
                                  C.byref(_TORCH_ALLOCATOR), ptr(phi), ptr(E), ptr(rank), ptr(wl), ptr(wr),
                                  C.c_void_p(ps.ctypes.data), C.byref(st), _stream_handle()))
    return dict(phi=phi, E=E, rank=rank, work_local=wl, work_remote=wr, pair_stats=ps,
                stats={k: getattr(st, k) for k, _ in _LetStats._fields_})


def mfma_layout(f64: bool, tail: bool = False) -> list:
    """Accumulator values of the MFMA lane-layout diagnostic (host list);
    tail=True probes the float32 4x4x1 blocks of the short last row tile."""
    import numpy as np
    out = np.zeros(256, np.float64 if (f64 and not tail) else np.float32)
    mode = 2 if tail else (1 if f64 else 0)
    _check(load().fmm_debug_mfma_layout(mode, C.c_void_p(out.ctypes.data)))
    return out


class FMMFunction(torch.autograd.Function):
    """phi, E = FMMFunction.apply(x, q, params); differentiable in x and q
    through L = sum_i w_i phi_i (w = grad of phi).  A gradient flowing into E
    would need second derivatives of 1/r and is not supported.

    params.recompute (attribute, default False): free the plan (tree, lists,
    operators and expansions) after the forward pass and rebuild it, with the
    same deterministic tree, in the backward.  The field E is an output of
    the forward pass anyway and is kept, so the backward is one rebuild plus
    one evaluation with charges w, as without recomputation."""

    @staticmethod
    def forward(ctx, x, q, params):
        ctx.set_materialize_grads(False)
        recompute = bool(getattr(params, "recompute", False))
        plan = Plan(x.detach(), params)
        phi, E = plan.evaluate(q.detach())
        ctx.params = params
        ctx.recompute = recompute
        if recompute:
            plan.close()
            ctx.plan = None
        else:
            ctx.plan = plan
        ctx.save_for_backward(x, q, E)
        ctx.mark_non_differentiable(E)
        return phi, E

    @staticmethod
    def backward(ctx, grad_phi, grad_E):
        if grad_E is not None and bool(torch.any(grad_E != 0)):
            raise NotImplementedError("gradient through the field E is not supported")
        if grad_phi is None:
            return None, None, None
        x, q, E = ctx.saved_tensors
        if ctx.recompute:
            plan = Plan(x.detach(), ctx.params)
            dq, dx = plan.adjoint(q.detach(), grad_phi.contiguous(), E)
            plan.close()
        else:
            if ctx.plan is None:
                raise RuntimeError("FMMFunction: the plan was released by an earlier backward; "
                                   "a second backward needs params.recompute = True")
            dq, dx = ctx.plan.adjoint(q.detach(), grad_phi.contiguous(), E)
            ctx.plan.close()
            ctx.plan = None
        return (dx if ctx.needs_input_grad[0] else None, dq if ctx.needs_input_grad[1] else None, None)
