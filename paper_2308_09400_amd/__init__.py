"""Python binding of libgipc (the GIPC barrier hot path on MI355X / gfx950).

Argument marshalling only: every step runs in the HIP kernels of
``libgipc.so``.  Tensors are torch tensors on the current HIP device and the
work goes on ``torch.cuda.current_stream()`` unless a stream is given.  The
names follow the C ABI in ``include/gipc.h`` without the ``gipc_`` prefix.
There is no CPU fallback: if the library cannot be loaded every call raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgipc.so")

OK, ERR_INVALID_ARG, ERR_INDEX, ERR_DEGENERATE, ERR_HIP, ERR_WORKSPACE, ERR_BREAKDOWN, ERR_STATE = 0, -1, -2, -3, -4, -5, -6, -7
WARN_NOT_CONVERGED, WARN_STALE = 1, 2
FLAG_FILTER, FLAG_MOLLIFY, FLAG_BARRIER_EQ12, FLAG_NO_MERGE = 0x1, 0x2, 0x4, 0x8
FLAGS_DEFAULT = FLAG_FILTER | FLAG_MOLLIFY
F64, F32 = 0, 1
SUBTYPES = {1: "PT", 2: "PE", 3: "PP", 4: "EE", 5: "EE_moll", 6: "PE_moll", 7: "PP_moll"}

EXPORTS = [
    "gipc_status_string", "gipc_ctx_create", "gipc_ctx_create_with_allocator", "gipc_ctx_destroy", "gipc_ctx_last_error", "gipc_pairs_build",
    "gipc_get_info", "gipc_bsr_pattern", "gipc_barrier_eval", "gipc_assemble_bsr", "gipc_eval_assemble",
    "gipc_bsr_spmv", "gipc_pcg", "gipc_pcg_delta", "gipc_pair_inspect", "gipc_copy", "gipc_get_tune", "gipc_set_tune",
    "gipc_autotune", "gipc_graph_create", "gipc_graph_launch", "gipc_graph_destroy", "gipc_mf_apply",
    "gipc_pcg_mf", "gipc_proxy_dense", "gipc_friction_lag", "gipc_friction_eval", "gipc_candidates",
    "gipc_read", "gipc_pairs_check", "gipc_pcg_static", "gipc_accd", "gipc_dense_apply", "gipc_pcg_dense",
]


class GipcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(msg)
        self.status = status


class BatchC(ctypes.Structure):
    _fields_ = [("S", ctypes.c_int32), ("vert_off", ctypes.c_void_p), ("dhat", ctypes.c_void_p),
                ("kappa", ctypes.c_void_p)]


class Params(ctypes.Structure):
    _fields_ = [("dhat", ctypes.c_double), ("kappa", ctypes.c_double), ("dthr_ratio", ctypes.c_double),
                ("epsx_ratio", ctypes.c_double), ("flags", ctypes.c_uint32), ("batch", ctypes.POINTER(BatchC))]


class Tune(ctypes.Structure):
    _fields_ = [("eval_waves", ctypes.c_int32), ("row_lanes", ctypes.c_int32), ("offdiag_waves", ctypes.c_int32),
                ("row_order", ctypes.c_int32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class Mesh(ctypes.Structure):
    _fields_ = [("V", ctypes.c_int32), ("x", ctypes.c_void_p), ("x_rest", ctypes.c_void_p)]


class Pairs(ctypes.Structure):
    _fields_ = [("P", ctypes.c_int64), ("tuples", ctypes.c_void_p)]


class Bsr(ctypes.Structure):
    _fields_ = [("nbrows", ctypes.c_int32), ("nnzb", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("val", ctypes.c_void_p), ("dtype", ctypes.c_int32),
                ("wave_head", ctypes.c_void_p), ("wave_row", ctypes.c_void_p)]


class Topology(ctypes.Structure):
    _fields_ = [("vobj", ctypes.c_void_p), ("tris", ctypes.c_void_p), ("F", ctypes.c_int64),
                ("edges", ctypes.c_void_p), ("E", ctypes.c_int64)]


class Friction(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_double), ("eps_v", ctypes.c_double), ("dt", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("n_candidates", ctypes.c_int64), ("n_active", ctypes.c_int64), ("n_by_type", ctypes.c_int64 * 8),
                ("n_staged", ctypes.c_int64), ("n_staged_by_type", ctypes.c_int64 * 8),
                ("n_degenerate", ctypes.c_int64), ("first_degenerate", ctypes.c_int64), ("nnzb", ctypes.c_int64),
                ("n_contrib", ctypes.c_int64), ("max_row_pairs", ctypes.c_int32),
                ("n_degenerate_prims", ctypes.c_int64), ("first_degenerate_prim", ctypes.c_int64)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f not in ("n_by_type", "n_staged_by_type")}
        d["n_by_type"] = {SUBTYPES[t]: int(self.n_by_type[t]) for t in range(1, 8)}
        d["n_staged_by_type"] = {SUBTYPES[t]: int(self.n_staged_by_type[t]) for t in range(1, 8)}
        return d


class Check(ctypes.Structure):
    _fields_ = [("n_entered", ctypes.c_int64), ("n_left", ctypes.c_int64), ("n_changed", ctypes.c_int64),
                ("n_degenerate", ctypes.c_int64), ("first", ctypes.c_int64)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class AccdInfo(ctypes.Structure):
    _fields_ = [("step", ctypes.c_double), ("n_capped", ctypes.c_int64), ("n_touching", ctypes.c_int64),
                ("max_steps", ctypes.c_int32)]


_lib = None


def lib():
    """The loaded libgipc.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing; build it with `python -m paper_2308_09400_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        st = ctypes.c_int
        sig = {
            "gipc_status_string": (ctypes.c_char_p, [ctypes.c_int]),
            "gipc_ctx_create": (st, [ctypes.POINTER(vp)]),
            "gipc_ctx_create_with_allocator": (st, [ctypes.POINTER(Allocator), ctypes.POINTER(vp)]),
            "gipc_ctx_destroy": (None, [vp]),
            "gipc_ctx_last_error": (ctypes.c_char_p, [vp]),
            "gipc_pairs_build": (st, [vp, ctypes.POINTER(Mesh), ctypes.POINTER(Pairs), ctypes.POINTER(Params), vp,
                                      ctypes.POINTER(Info)]),
            "gipc_get_info": (st, [vp, ctypes.POINTER(Info)]),
            "gipc_pairs_check": (st, [vp, ctypes.POINTER(Mesh), ctypes.POINTER(Pairs), ctypes.POINTER(Params),
                                      ctypes.POINTER(Check), vp]),
            "gipc_bsr_pattern": (st, [vp, ctypes.POINTER(Bsr)]),
            "gipc_barrier_eval": (st, [vp, ctypes.POINTER(Mesh), ctypes.POINTER(Params), vp, vp, vp]),
            "gipc_assemble_bsr": (st, [vp, vp, ctypes.POINTER(Bsr), vp]),
            "gipc_eval_assemble": (st, [vp, ctypes.POINTER(Mesh), ctypes.POINTER(Params), vp, vp, vp,
                                        ctypes.POINTER(Bsr), vp]),
            "gipc_bsr_spmv": (st, [ctypes.POINTER(Bsr), vp, vp, vp]),
            "gipc_pcg": (st, [vp, ctypes.POINTER(Bsr), vp, vp, d, i32, ctypes.POINTER(i32), ctypes.POINTER(d), vp]),
            "gipc_pcg_delta": (st, [vp, ctypes.POINTER(Bsr), vp, vp, d, i32, ctypes.POINTER(i32), ctypes.POINTER(d),
                                    vp]),
            "gipc_accd": (st, [vp, ctypes.POINTER(Mesh), vp, ctypes.POINTER(Pairs), d, d, i32, vp,
                               ctypes.POINTER(AccdInfo), vp]),
            "gipc_pcg_static": (st, [ctypes.POINTER(Bsr), vp, vp, d, i32, ctypes.POINTER(i32), ctypes.POINTER(d),
                                     vp]),
            "gipc_mf_apply": (st, [vp, vp, vp, vp, vp]),
            "gipc_dense_apply": (st, [vp, vp, i32, vp, vp, vp, vp]),
            "gipc_pcg_dense": (st, [vp, vp, i32, vp, vp, vp, d, i32, ctypes.POINTER(i32), ctypes.POINTER(d), vp]),
            "gipc_pcg_mf": (st, [vp, vp, vp, vp, d, i32, ctypes.POINTER(i32), ctypes.POINTER(d), vp]),
            "gipc_proxy_dense": (st, [vp, ctypes.POINTER(Mesh), ctypes.POINTER(Params), i32, vp, vp]),
            "gipc_friction_lag": (st, [vp, ctypes.POINTER(Mesh), ctypes.POINTER(Params), ctypes.POINTER(Friction),
                                       vp]),
            "gipc_friction_eval": (st, [vp, vp, vp, vp, ctypes.POINTER(Bsr), vp]),
            "gipc_candidates": (st, [vp, ctypes.POINTER(Mesh), ctypes.POINTER(Topology), d, vp, i64,
                                     ctypes.POINTER(i64), vp]),
            "gipc_pair_inspect": (st, [vp, ctypes.POINTER(Mesh), ctypes.POINTER(Params), vp, vp, vp, vp, vp, vp, vp,
                                       vp]),
            "gipc_copy": (st, [vp, vp, i64, vp]),
            "gipc_read": (st, [vp, i64, vp, vp]),
            "gipc_get_tune": (st, [vp, ctypes.POINTER(Tune)]),
            "gipc_set_tune": (st, [vp, ctypes.POINTER(Tune)]),
            "gipc_autotune": (st, [vp, ctypes.POINTER(Mesh), ctypes.POINTER(Params), vp, vp, vp, ctypes.POINTER(Bsr),
                                   i32, ctypes.POINTER(Tune), vp]),
            "gipc_graph_create": (st, [vp, ctypes.POINTER(Mesh), ctypes.POINTER(Params), vp, vp, vp,
                                       ctypes.POINTER(Bsr), ctypes.POINTER(vp)]),
            "gipc_graph_launch": (st, [vp, vp]),
            "gipc_graph_destroy": (None, [vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_string(s: int) -> str:
    return lib().gipc_status_string(int(s)).decode()


class Batch:
    """Independent scenes concatenated into one mesh: scene s owns the
    vertices [vert_off[s], vert_off[s+1]) and has its own dhat and kappa
    (device tensors int32 [S+1], float64 [S], float64 [S])."""

    def __init__(self, vert_off, dhat, kappa, device=None):
        dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.vert_off = torch.as_tensor(vert_off, dtype=torch.int32).to(dev).contiguous()
        self.dhat = torch.as_tensor(dhat, dtype=torch.float64).to(dev).contiguous()
        self.kappa = torch.as_tensor(kappa, dtype=torch.float64).to(dev).contiguous()
        self.S = int(self.dhat.numel())
        if self.vert_off.numel() != self.S + 1 or self.kappa.numel() != self.S:
            raise ValueError("vert_off must have S+1 entries, dhat and kappa S")
        self.c = BatchC(self.S, self.vert_off.data_ptr(), self.dhat.data_ptr(), self.kappa.data_ptr())
        self._scene_of_vertex = None

    def scene_of_vertex(self):
        """int64 [V] scene id of every vertex (for the autograd backward)."""
        if self._scene_of_vertex is None:
            counts = (self.vert_off[1:] - self.vert_off[:-1]).long()
            self._scene_of_vertex = torch.repeat_interleave(
                torch.arange(self.S, device=self.vert_off.device), counts)
        return self._scene_of_vertex


def params(dhat=1e-3, kappa=1e4, dthr_ratio=0.1, epsx_ratio=1e-3, flags=FLAGS_DEFAULT, batch: Batch | None = None
           ) -> Params:
    """Parameters; with ``batch`` its per-scene dhat and kappa replace dhat and kappa."""
    p = Params(float(dhat), float(kappa), float(dthr_ratio), float(epsx_ratio), int(flags),
               ctypes.pointer(batch.c) if batch is not None else None)
    p._batch = batch  # keeps the batch's tensors alive with the struct
    return p


def _energy_out(prm: Params, device):
    b = getattr(prm, "_batch", None)
    return torch.empty((b.S,) if b is not None else (), dtype=torch.float64, device=device)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _need(t, dtype, shape_last=None, name="tensor"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape_last is not None and (t.dim() < 1 or t.shape[-1] != shape_last):
        raise ValueError(f"{name} must have last dimension {shape_last}")


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("user", ctypes.c_void_p)]


def _torch_allocator() -> Allocator:
    """gipc_allocator callbacks over torch's caching allocator (blocks on the
    device's default stream)."""
    def alloc(user, nbytes, device):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device=int(device), stream=0)
        except Exception:
            return None

    def free(user, ptr, nbytes, device):
        torch.cuda.caching_allocator_delete(int(ptr))

    return Allocator(_ALLOC_FN(alloc), _FREE_FN(free), None)


class Context:
    """Owns a gipc_ctx (device workspace, staged pairs, pattern, factors)."""

    def __init__(self, allocator=None):
        """allocator=None: the library's own hipMalloc; "torch": every buffer
        of the context comes from torch's caching allocator."""
        h = ctypes.c_void_p()
        self._alloc = None
        if allocator is None:
            s = lib().gipc_ctx_create(ctypes.byref(h))
        elif allocator == "torch":
            self._alloc = _torch_allocator()
            s = lib().gipc_ctx_create_with_allocator(ctypes.byref(self._alloc), ctypes.byref(h))
        else:
            raise ValueError("allocator must be None or 'torch'")
        if s != OK:
            raise GipcError(s, f"gipc_ctx_create: {status_string(s)}")
        self.h = h
        self.V = 0
        self.info = None

    def close(self):
        if getattr(self, "h", None):
            lib().gipc_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, s, what):
        if s < 0:
            msg = lib().gipc_ctx_last_error(self.h).decode()
            raise GipcError(s, f"{what}: {status_string(s)}: {msg}")
        return s

    @staticmethod
    def _mesh(x, x_rest):
        _need(x, torch.float64, 3, "x")
        if x_rest is not None:
            _need(x_rest, torch.float64, 3, "x_rest")
            if x_rest.shape != x.shape:
                raise ValueError("x_rest must match x")
        return Mesh(int(x.shape[0]), x.data_ptr(), None if x_rest is None else x_rest.data_ptr())


def pairs_build(ctx: Context, x, tuples, prm: Params, x_rest=None, stream=None) -> dict:
    """Stage the tuples at positions x and build the BSR pattern (synchronises)."""
    _need(tuples, torch.int32, 4, "tuples")
    mesh = Context._mesh(x, x_rest)
    pairs = Pairs(int(tuples.shape[0]), tuples.data_ptr())
    info = Info()
    ctx._check(lib().gipc_pairs_build(ctx.h, ctypes.byref(mesh), ctypes.byref(pairs), ctypes.byref(prm),
                                      _stream(stream), ctypes.byref(info)), "gipc_pairs_build")
    ctx.V = int(x.shape[0])
    ctx.info = info.as_dict()
    return ctx.info


def pairs_check(ctx: Context, x, tuples, prm: Params, x_rest=None, stream=None):
    """Whether the last build still holds at positions x (synchronises):
    returns (stale, counts) with stale True when gipc_pairs_check answers
    GIPC_WARN_STALE (rebuild before evaluating at x)."""
    _need(tuples, torch.int32, 4, "tuples")
    mesh = Context._mesh(x, x_rest)
    pairs = Pairs(int(tuples.shape[0]), tuples.data_ptr())
    c = Check()
    s = lib().gipc_pairs_check(ctx.h, ctypes.byref(mesh), ctypes.byref(pairs), ctypes.byref(prm), ctypes.byref(c),
                               _stream(stream))
    if s < 0:
        ctx._check(s, "gipc_pairs_check")
    return s == WARN_STALE, c.as_dict()


def bsr_pattern(ctx: Context) -> Bsr:
    A = Bsr()
    ctx._check(lib().gipc_bsr_pattern(ctx.h, ctypes.byref(A)), "gipc_bsr_pattern")
    return A


def barrier_eval(ctx: Context, x, prm: Params, x_rest=None, energy=None, grad=None, stream=None):
    """Energy (device scalar tensor) and gradient [V][3] of the staged pairs."""
    mesh = Context._mesh(x, x_rest)
    energy = _energy_out(prm, x.device) if energy is None else energy
    grad = torch.empty_like(x) if grad is None else grad
    ctx._check(lib().gipc_barrier_eval(ctx.h, ctypes.byref(mesh), ctypes.byref(prm), _ptr(energy), _ptr(grad),
                                       _stream(stream)), "gipc_barrier_eval")
    return energy, grad


class BsrMatrix:
    """A BSR matrix on the context's pattern with caller-owned values [9][nnzb]."""

    def __init__(self, ctx: Context, dtype=F64, device=None):
        self.ctx = ctx
        self.desc = bsr_pattern(ctx)
        self.dtype = dtype
        tdt = torch.float64 if dtype == F64 else torch.float32
        dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.val = torch.empty((9, max(int(self.desc.nnzb), 1)), dtype=tdt, device=dev)
        self.desc.val = self.val.data_ptr()
        self.desc.dtype = dtype

    @property
    def nnzb(self):
        return int(self.desc.nnzb)

    @property
    def nbrows(self):
        return int(self.desc.nbrows)

    def row_ptr(self):
        return _wrap_i32(self.desc.row_ptr, self.nbrows + 1, self.val.device)

    def col_idx(self):
        return _wrap_i32(self.desc.col_idx, self.nnzb, self.val.device)

    def wave_map(self):
        """Copies of the row-start map: (head bits as int64 [ceil(nnzb/64)], first rows as int32)."""
        n = (self.nnzb + 63) // 64
        head = _wrap_i32(self.desc.wave_head, 2 * n, self.val.device).view(torch.int64)
        return head, _wrap_i32(self.desc.wave_row, n, self.val.device)

    def row_descriptor(self) -> Bsr:
        """A copy of the descriptor without the row-start map (products then run row by row)."""
        d = Bsr.from_buffer_copy(self.desc)
        d.wave_head = None
        d.wave_row = None
        return d

    def to_scipy(self):
        """Host scipy.sparse.bsr_matrix copy (test helper)."""
        import numpy as np
        import scipy.sparse as sps
        rp = self.row_ptr().cpu().numpy()
        ci = self.col_idx().cpu().numpy()
        v = self.val[:, :self.nnzb].double().cpu().numpy().T.reshape(-1, 3, 3)
        return sps.bsr_matrix((v, ci, rp), shape=(3 * self.nbrows, 3 * self.nbrows))


def _wrap_i32(ptr, n, device):
    """Copy n int32 from a library-owned device pointer into a new tensor."""
    out = torch.empty(max(n, 0), dtype=torch.int32, device=device)
    if n > 0:
        s = lib().gipc_copy(ctypes.c_void_p(ptr), ctypes.c_void_p(out.data_ptr()), 4 * n, _stream(None))
        if s != OK:
            raise GipcError(s, "gipc_copy failed")
    return out


def assemble_bsr(ctx: Context, A: BsrMatrix, diag=None, stream=None):
    if diag is not None:
        _need(diag, torch.float64, None, "diag")
    ctx._check(lib().gipc_assemble_bsr(ctx.h, _ptr(diag), ctypes.byref(A.desc), _stream(stream)), "gipc_assemble_bsr")
    return A


def eval_assemble(ctx: Context, x, prm: Params, A: BsrMatrix, diag=None, x_rest=None, energy=None, grad=None,
                  stream=None):
    mesh = Context._mesh(x, x_rest)
    if diag is not None:
        _need(diag, torch.float64, None, "diag")
    energy = _energy_out(prm, x.device) if energy is None else energy
    grad = torch.empty_like(x) if grad is None else grad
    ctx._check(lib().gipc_eval_assemble(ctx.h, ctypes.byref(mesh), ctypes.byref(prm), _ptr(energy), _ptr(grad),
                                        _ptr(diag), ctypes.byref(A.desc), _stream(stream)), "gipc_eval_assemble")
    return energy, grad


def bsr_spmv(A: BsrMatrix, x, y=None, stream=None, by_rows=False):
    """y = A x; by_rows=True drops the row-start map (row-by-row product)."""
    tdt = torch.float64 if A.dtype == F64 else torch.float32
    _need(x, tdt, 3, "x")
    y = torch.empty_like(x) if y is None else y
    desc = A.row_descriptor() if by_rows else A.desc
    s = lib().gipc_bsr_spmv(ctypes.byref(desc), _ptr(x), _ptr(y), _stream(stream))
    if s != OK:
        raise GipcError(s, f"gipc_bsr_spmv: {status_string(s)}")
    return y


def pcg(ctx: Context, A: BsrMatrix, b, x=None, rtol=1e-6, maxit=1000, stream=None, by_rows=False, stop="residual"):
    """Block-Jacobi PCG (synchronises).  Returns (x, iterations, relres, status).
    by_rows=True drops the row-start map (row-by-row products).  stop =
    "residual": ||r|| <= rtol ||b|| (gipc_pcg); "delta": the paper's
    termination r.z <= rtol r0.z0 (gipc_pcg_delta)."""
    _need(b, torch.float64, 3, "b")
    if stop not in ("residual", "delta"):
        raise ValueError("stop must be 'residual' or 'delta'")
    x = torch.zeros_like(b) if x is None else x
    it = ctypes.c_int32()
    rr = ctypes.c_double()
    desc = A.row_descriptor() if by_rows else A.desc
    f = lib().gipc_pcg_delta if stop == "delta" else lib().gipc_pcg
    s = f(ctx.h, ctypes.byref(desc), _ptr(b), _ptr(x), float(rtol), int(maxit), ctypes.byref(it), ctypes.byref(rr),
          _stream(stream))
    ctx._check(s, "gipc_pcg_delta" if stop == "delta" else "gipc_pcg")
    return x, int(it.value), float(rr.value), int(s)


def accd(ctx: Context, x, disp, tuples, s=0.1, tc=1.0, max_iter=1_000_000, toi=None, per_tuple=True, stream=None):
    """Additive-CCD step bound of a tuple list moving by disp (synchronises).
    Returns (toi [P] device tensor, or None with per_tuple=False; info dict
    with step, n_capped, n_touching, max_steps)."""
    _need(x, torch.float64, 3, "x")
    _need(disp, torch.float64, 3, "disp")
    _need(tuples, torch.int32, 4, "tuples")
    if disp.shape != x.shape:
        raise ValueError("disp must have the shape of x")
    P = int(tuples.shape[0])
    if toi is not None:
        _need(toi, torch.float64, None, "toi")
        if toi.numel() != P:
            raise ValueError("toi must hold one value per tuple")
    if per_tuple and toi is None:
        toi = torch.empty(P, dtype=torch.float64, device=x.device)
    if not per_tuple:
        toi = None
    mesh = Context._mesh(x, None)
    pairs = Pairs(P, tuples.data_ptr() if P else None)
    info = AccdInfo()
    ctx._check(lib().gipc_accd(ctx.h, ctypes.byref(mesh), _ptr(disp), ctypes.byref(pairs), float(s), float(tc),
                               int(max_iter), _ptr(toi), ctypes.byref(info), _stream(stream)), "gipc_accd")
    return toi, {f: getattr(info, f) for f, _ in AccdInfo._fields_}


def pcg_static(A: BsrMatrix, b, x=None, rtol=1e-6, maxit=1000, stream=None, counts=True):
    """gipc_pcg on the library's fixed work area (no context, no device
    allocation by the library).  Returns (x, iterations, relres, status);
    with rtol=0 and counts=False it only enqueues (capturable in a HIP
    graph) and returns (x, None, None, status)."""
    _need(b, torch.float64, 3, "b")
    x = torch.zeros_like(b) if x is None else x
    it = ctypes.c_int32()
    rr = ctypes.c_double()
    pit, prr = (ctypes.byref(it), ctypes.byref(rr)) if counts else (None, None)
    s = lib().gipc_pcg_static(ctypes.byref(A.desc), _ptr(b), _ptr(x), float(rtol), int(maxit), pit, prr,
                              _stream(stream))
    if s < 0:
        raise GipcError(s, f"gipc_pcg_static: {status_string(s)}")
    if not counts:
        return x, None, None, int(s)
    return x, int(it.value), float(rr.value), int(s)


def candidates(ctx: Context, x, vobj, tris, edges, dhat, stream=None):
    """Contact candidates (point-triangle, then edge-edge) of a surface mesh
    on the GPU: device int32 [P][4] in the sign encoding.

    The context remembers a capacity from its last call (the count plus a
    quarter); while the count stays under it, one library call counts and
    emits, and the result is the leading rows of a buffer of that capacity.
    Otherwise (and on a context's first call) a counting call sizes the
    output exactly and a second call emits."""
    mesh = Context._mesh(x, None)
    for t, name in ((vobj, "vobj"), (tris, "tris"), (edges, "edges")):
        _need(t, torch.int32, None, name)
    topo = Topology(_ptr(vobj), _ptr(tris), int(tris.numel() // 3), _ptr(edges), int(edges.numel() // 2))
    n = ctypes.c_int64()
    cap = getattr(ctx, "_cand_cap", 0)
    if cap > 0:
        out = torch.empty((cap, 4), dtype=torch.int32, device=x.device)
        st = lib().gipc_candidates(ctx.h, ctypes.byref(mesh), ctypes.byref(topo), float(dhat), _ptr(out), cap,
                                   ctypes.byref(n), _stream(stream))
        if st == OK:
            ctx._cand_cap = max(cap, int(n.value) + int(n.value) // 4)
            return out[: int(n.value)]
        if st != ERR_WORKSPACE:
            ctx._check(st, "gipc_candidates")
        del out
    else:
        ctx._check(lib().gipc_candidates(ctx.h, ctypes.byref(mesh), ctypes.byref(topo), float(dhat), None, 0,
                                         ctypes.byref(n), _stream(stream)), "gipc_candidates")
    out = torch.empty((max(int(n.value), 0), 4), dtype=torch.int32, device=x.device)
    if n.value > 0:
        ctx._check(lib().gipc_candidates(ctx.h, ctypes.byref(mesh), ctypes.byref(topo), float(dhat), _ptr(out),
                                         int(n.value), ctypes.byref(n), _stream(stream)), "gipc_candidates")
    ctx._cand_cap = int(n.value) + int(n.value) // 4 + 64
    return out


def friction_lag(ctx: Context, x_n, prm: Params, mu, eps_v, dt, x_rest=None, stream=None):
    """Lag the friction of the staged pairs at the previous positions x_n."""
    mesh = Context._mesh(x_n, x_rest)
    fr = Friction(float(mu), float(eps_v), float(dt))
    ctx._check(lib().gipc_friction_lag(ctx.h, ctypes.byref(mesh), ctypes.byref(prm), ctypes.byref(fr),
                                       _stream(stream)), "gipc_friction_lag")


def friction_eval(ctx: Context, x, prm: Params, A: "BsrMatrix | None" = None, energy=None, grad=None, stream=None):
    """Friction energy (per scene) and gradient at x; with A, its Hessian
    blocks are added to A.  Returns (energy, grad)."""
    _need(x, torch.float64, 3, "x")
    _need_rows(ctx, x, "x")
    energy = _energy_out(prm, x.device) if energy is None else energy
    grad = torch.empty_like(x) if grad is None else grad
    _need(grad, torch.float64, 3, "grad")
    _need_rows(ctx, grad, "grad")
    ctx._check(lib().gipc_friction_eval(ctx.h, _ptr(x), _ptr(energy), _ptr(grad),
                                        ctypes.byref(A.desc) if A is not None else None, _stream(stream)),
               "gipc_friction_eval")
    return energy, grad


PROJ_ANALYTIC, PROJ_NUMERIC, PROJ_EXACT = 0, 1, 2


def proxy_dense(ctx: Context, x, prm: Params, method=PROJ_ANALYTIC, x_rest=None, hess=None, stream=None):
    """Dense projected proxy Hessian [n_staged][12][12] of every staged pair,
    from the analytic eigensystems or by numeric Jacobi projection in x-space."""
    mesh = Context._mesh(x, x_rest)
    n = int(ctx.info["n_staged"]) if ctx.info else 0
    if hess is None:
        hess = torch.empty((n, 12, 12), dtype=torch.float64, device=x.device)
    _need(hess, torch.float64, 12, "hess")
    if hess.shape[0] < n:
        raise ValueError(f"hess must hold {n} pairs")
    ctx._check(lib().gipc_proxy_dense(ctx.h, ctypes.byref(mesh), ctypes.byref(prm), int(method), _ptr(hess),
                                      _stream(stream)), "gipc_proxy_dense")
    return hess


def _need_rows(ctx: Context, t, name):
    if t.shape[0] != ctx.V:
        raise ValueError(f"{name} must have {ctx.V} rows (the vertex count of the last build)")


def mf_apply(ctx: Context, x, y=None, diag=None, stream=None):
    """Matrix-free y = (diag (x) I3 + H) x over the factors of the last eval."""
    _need(x, torch.float64, 3, "x")
    _need_rows(ctx, x, "x")
    if diag is not None:
        _need(diag, torch.float64, None, "diag")
        _need_rows(ctx, diag, "diag")
    y = torch.empty_like(x) if y is None else y
    _need(y, torch.float64, 3, "y")
    _need_rows(ctx, y, "y")
    ctx._check(lib().gipc_mf_apply(ctx.h, _ptr(diag), _ptr(x), _ptr(y), _stream(stream)), "gipc_mf_apply")
    return y


def pcg_mf(ctx: Context, b, x=None, diag=None, rtol=1e-6, maxit=1000, stream=None):
    """Block-Jacobi PCG on the matrix-free operator (synchronises).
    Returns (x, iterations, relres, status)."""
    _need(b, torch.float64, 3, "b")
    _need_rows(ctx, b, "b")
    if diag is not None:
        _need(diag, torch.float64, None, "diag")
        _need_rows(ctx, diag, "diag")
    x = torch.zeros_like(b) if x is None else x
    _need(x, torch.float64, 3, "x")
    _need_rows(ctx, x, "x")
    it = ctypes.c_int32()
    rr = ctypes.c_double()
    s = lib().gipc_pcg_mf(ctx.h, _ptr(diag), _ptr(b), _ptr(x), float(rtol), int(maxit), ctypes.byref(it),
                          ctypes.byref(rr), _stream(stream))
    ctx._check(s, "gipc_pcg_mf")
    return x, int(it.value), float(rr.value), int(s)


DENSE_THREAD, DENSE_ENTRY = 0, 1


def _need_dense(ctx: Context, hess):
    _need(hess, torch.float64, 12, "hess")
    n = int(ctx.info["n_staged"]) if ctx.info else 0
    if hess.dim() != 3 or hess.shape[1] != 12 or hess.shape[0] < n:
        raise ValueError("hess must be [n_staged][12][12] (gipc_proxy_dense)")


def dense_apply(ctx: Context, hess, x, y=None, diag=None, scheme=DENSE_ENTRY, stream=None):
    """y = (diag (x) I3 + sum_k S_k^T H_k S_k) x from dense local Hessians
    (Table 2's two schemes; FP64 atomics, last bits vary)."""
    _need_dense(ctx, hess)
    _need(x, torch.float64, 3, "x")
    _need_rows(ctx, x, "x")
    if diag is not None:
        _need(diag, torch.float64, None, "diag")
        _need_rows(ctx, diag, "diag")
    y = torch.empty_like(x) if y is None else y
    _need(y, torch.float64, 3, "y")
    _need_rows(ctx, y, "y")
    ctx._check(lib().gipc_dense_apply(ctx.h, _ptr(hess), int(scheme), _ptr(diag), _ptr(x), _ptr(y),
                                      _stream(stream)), "gipc_dense_apply")
    return y


def pcg_dense(ctx: Context, hess, b, x=None, diag=None, scheme=DENSE_ENTRY, rtol=1e-6, maxit=1000, stream=None):
    """Block-Jacobi PCG on the dense-Hessian product (synchronises).
    Returns (x, iterations, relres, status)."""
    _need_dense(ctx, hess)
    _need(b, torch.float64, 3, "b")
    _need_rows(ctx, b, "b")
    if diag is not None:
        _need(diag, torch.float64, None, "diag")
        _need_rows(ctx, diag, "diag")
    x = torch.zeros_like(b) if x is None else x
    it = ctypes.c_int32()
    rr = ctypes.c_double()
    s = lib().gipc_pcg_dense(ctx.h, _ptr(hess), int(scheme), _ptr(diag), _ptr(b), _ptr(x), float(rtol), int(maxit),
                             ctypes.byref(it), ctypes.byref(rr), _stream(stream))
    ctx._check(s, "gipc_pcg_dense")
    return x, int(it.value), float(rr.value), int(s)


def pair_inspect(ctx: Context, x=None, prm: Params | None = None, x_rest=None, want=("src", "type", "vid"),
                 stream=None):
    """Per staged pair: src, type, vid, mult, energy, grad [12], hess [12,12]
    (device tensors; energy, grad and hess include the multiplicity)."""
    n = int(ctx.info["n_staged"]) if ctx.info else 0
    dev = torch.device("cuda", torch.cuda.current_device())
    out = {}
    alloc = {"src": ((n,), torch.int32), "type": ((n,), torch.int32), "vid": ((n, 4), torch.int32),
             "mult": ((n,), torch.int32),
             "energy": ((n,), torch.float64), "grad": ((n, 12), torch.float64), "hess": ((n, 12, 12), torch.float64)}
    for k in want:
        shp, dt = alloc[k]
        out[k] = torch.empty(shp, dtype=dt, device=dev)
    mesh = Context._mesh(x, x_rest) if x is not None else None
    ctx._check(lib().gipc_pair_inspect(ctx.h, ctypes.byref(mesh) if mesh else None,
                                       ctypes.byref(prm) if prm else None,
                                       *[_ptr(out.get(k)) for k in ("src", "type", "vid", "mult", "energy", "grad",
                                                                    "hess")],
                                       _stream(stream)), "gipc_pair_inspect")
    return out


def copy(src, dst, nbytes=None, stream=None):
    nbytes = src.numel() * src.element_size() if nbytes is None else nbytes
    s = lib().gipc_copy(_ptr(src), _ptr(dst), int(nbytes), _stream(stream))
    if s != OK:
        raise GipcError(s, "gipc_copy failed")
    return dst


def read(src, nbytes=None, sink=None, stream=None):
    """Streaming read of ``src`` with the library's read kernel (bandwidth
    reference); ``sink`` is a 4-byte device buffer it may write."""
    nbytes = src.numel() * src.element_size() if nbytes is None else nbytes
    if sink is None:
        sink = torch.empty(1, dtype=torch.int32, device=src.device)
    s = lib().gipc_read(_ptr(src), int(nbytes), _ptr(sink), _stream(stream))
    if s != OK:
        raise GipcError(s, "gipc_read failed")
    return sink


class BarrierEnergy(torch.autograd.Function):
    """Total barrier energy kappa * sum_k e_k b_k of the pairs staged in ``gctx``
    as a differentiable function of the positions (Eq. 3, 24, 29); with a
    batch, the vector of per-scene energies.

    ``forward`` runs the pair-evaluation and gradient kernels
    (``gipc_barrier_eval``) and keeps the gradient; ``backward`` returns
    ``grad_output * gradient`` -- no autograd graph is built through the
    kernels.  The pairs must have been staged with ``pairs_build`` (their
    sub-types stay fixed while x moves, as inside one Newton iteration).
    """

    @staticmethod
    def forward(ctx, x, gctx, prm, x_rest=None):
        E, g = barrier_eval(gctx, x.detach().contiguous(), prm, x_rest=x_rest)
        ctx.save_for_backward(g)
        ctx.batch = getattr(prm, "_batch", None)
        return E

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        if ctx.batch is not None:  # per-scene energies: each vertex takes its scene's weight
            return grad_out[ctx.batch.scene_of_vertex()].unsqueeze(1) * g, None, None, None
        return grad_out * g, None, None, None


def barrier_energy(x, gctx: Context, prm: Params, x_rest=None):
    """Differentiable total barrier energy (see BarrierEnergy)."""
    return BarrierEnergy.apply(x, gctx, prm, x_rest)


def hvp(gctx: Context, x, prm: Params, v, x_rest=None, A: BsrMatrix | None = None):
    """Product of the assembled proxy Hessian (Eq. 18-23, 32-36; no mass term)
    at positions x with a direction v [V][3]: eval + BSR assembly + BSR SpMV.
    Returns (Hv, A); pass A back in to reuse its value buffer."""
    A = BsrMatrix(gctx) if A is None else A
    eval_assemble(gctx, x, prm, A, diag=None, x_rest=x_rest)
    return bsr_spmv(A, v.contiguous()), A


def get_tune(ctx: Context) -> dict:
    t = Tune()
    ctx._check(lib().gipc_get_tune(ctx.h, ctypes.byref(t)), "gipc_get_tune")
    return t.as_dict()


def set_tune(ctx: Context, eval_waves=4, row_lanes=16, offdiag_waves=4, row_order=0):
    t = Tune(int(eval_waves), int(row_lanes), int(offdiag_waves), int(row_order))
    ctx._check(lib().gipc_set_tune(ctx.h, ctypes.byref(t)), "gipc_set_tune")


_LIB_DIGEST = None


def _lib_digest() -> str:
    """First 16 hex digits of the SHA-256 of the loaded library file."""
    global _LIB_DIGEST
    if _LIB_DIGEST is None:
        import hashlib
        with open(LIB_PATH, "rb") as f:
            _LIB_DIGEST = hashlib.sha256(f.read()).hexdigest()[:16]
    return _LIB_DIGEST


def autotune(ctx: Context, x, prm: Params, A: BsrMatrix, diag=None, x_rest=None, reps=5, cache=None, key=None,
             stream=None) -> dict:
    """Pick the fastest launch shapes of the eval / row / off-diagonal kernels
    for the current build (``gipc_autotune``, synchronises).  With ``cache``
    (a JSON file path), a stored choice is applied instead of timing, and a
    new one is stored.  The cache key is the device architecture, the tune
    fields and a digest of this library's binary (a rebuilt kernel is timed
    again), the build's mix of staged sub-types (rounded shares) and its size
    bucket (powers of two of staged pairs and vertices), plus ``key`` if
    given; an entry missing any tune field is timed again.
    Returns the shapes in force afterwards (``get_tune``)."""
    import json
    import math
    dkey = None
    if cache is not None:
        st = ctx.info["n_staged_by_type"]
        tot = max(sum(st.values()), 1)
        mix = ",".join(f"{k}:{round(10 * n / tot)}" for k, n in sorted(st.items()))
        bucket = f"P2^{int(math.log2(max(tot, 1)))},V2^{int(math.log2(max(int(x.shape[0]), 1)))}"
        arch = torch.cuda.get_device_properties(x.device).gcnArchName
        fields = ",".join(f for f, _ in Tune._fields_)
        dkey = f"{arch}|{fields}|{_lib_digest()}|{mix}|{bucket}|{key or ''}"
        try:
            with open(cache) as f:
                table = json.load(f)
        except (OSError, ValueError):
            table = {}
        entry = table.get(dkey)
        if isinstance(entry, dict) and all(f in entry for f, _ in Tune._fields_):
            set_tune(ctx, **{f: entry[f] for f, _ in Tune._fields_})
            return get_tune(ctx)
    mesh = Context._mesh(x, x_rest)
    if diag is not None:
        _need(diag, torch.float64, None, "diag")
    energy = _energy_out(prm, x.device)
    grad = torch.empty_like(x)
    t = Tune()
    ctx._check(lib().gipc_autotune(ctx.h, ctypes.byref(mesh), ctypes.byref(prm), _ptr(energy), _ptr(grad),
                                   _ptr(diag), ctypes.byref(A.desc), int(reps), ctypes.byref(t), _stream(stream)),
               "gipc_autotune")
    best = get_tune(ctx)
    if dkey is not None:
        try:
            with open(cache) as f:
                table = json.load(f)
        except (OSError, ValueError):
            table = {}
        table[dkey] = best
        with open(cache, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
    return best


class Graph:
    """``gipc_eval_assemble`` for fixed buffers, captured once into a HIP graph
    (``gipc_graph_create``); ``launch()`` replays it.  Write new positions
    into ``x`` in place between launches; ``energy`` and ``grad`` are the
    output tensors the graph writes."""

    def __init__(self, ctx: Context, x, prm: Params, A: BsrMatrix, diag=None, x_rest=None):
        mesh = Context._mesh(x, x_rest)
        if diag is not None:
            _need(diag, torch.float64, None, "diag")
        self.ctx, self.x, self.x_rest, self.prm, self.A, self.diag = ctx, x, x_rest, prm, A, diag
        self.energy = _energy_out(prm, x.device)
        self.grad = torch.empty_like(x)
        h = ctypes.c_void_p()
        ctx._check(lib().gipc_graph_create(ctx.h, ctypes.byref(mesh), ctypes.byref(prm), _ptr(self.energy),
                                           _ptr(self.grad), _ptr(diag), ctypes.byref(A.desc), ctypes.byref(h)),
                   "gipc_graph_create")
        self.h = h

    def launch(self, stream=None):
        self.ctx._check(lib().gipc_graph_launch(self.h, _stream(stream)), "gipc_graph_launch")
        return self.energy, self.grad

    def close(self):
        if getattr(self, "h", None):
            lib().gipc_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
