"""ctypes binding of the CPU FP64 oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP
library (``paper_2308_09400_amd``) and the product path never calls it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

INACTIVE, PT, PE, PP, EE, DEGENERATE = 0, 1, 2, 3, 4, 7


class Params(ctypes.Structure):
    _fields_ = [
        ("dhat", ctypes.c_double),
        ("kappa", ctypes.c_double),
        ("dthr_ratio", ctypes.c_double),
        ("epsx_ratio", ctypes.c_double),
        ("filter", ctypes.c_int),
        ("mollify", ctypes.c_int),
        ("eq12", ctypes.c_int),
    ]


def params(dhat=1e-3, kappa=1e4, dthr_ratio=0.1, epsx_ratio=1e-3, filter=True, mollify=True, eq12=False):
    return Params(dhat, kappa, dthr_ratio, epsx_ratio, int(filter), int(mollify), int(eq12))


class FParams(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_double), ("eps_v", ctypes.c_double), ("dt", ctypes.c_double)]


def fparams(mu=0.2, eps_v=1e-3, dt=1e-2):
    return FParams(mu, eps_v, dt)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fno-fast-math", "-shared", "-fPIC", "-o", tmp,
                               os.path.join(_HERE, "gipc_oracle.c"), "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _ptr(a):
    return None if a is None else a.ctypes.data


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        vp, d, i32, i64 = ctypes.c_void_p, ctypes.c_double, ctypes.c_int32, ctypes.c_int64
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_barrier.argtypes = [d, d, ctypes.c_int, dp, dp, dp]
        L.orc_barrier.restype = None
        L.orc_mollifier.argtypes = [d, d, dp, dp, dp]
        L.orc_mollifier.restype = None
        L.orc_jacobi_eig.argtypes = [ctypes.c_int, vp, vp, vp]
        L.orc_jacobi_eig.restype = ctypes.c_int
        L.orc_pair_local.argtypes = [vp, vp, vp, ctypes.POINTER(Params), dp, vp, vp,
                                     ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), dp,
                                     vp, vp, vp, ctypes.POINTER(ctypes.c_int)]
        L.orc_pair_local.restype = ctypes.c_int
        L.orc_pair_exact.argtypes = [vp, vp, vp, ctypes.POINTER(Params), vp, vp]
        L.orc_pair_exact.restype = ctypes.c_int
        L.orc_eval_exact.argtypes = [i32, vp, vp, i64, vp, ctypes.POINTER(Params), ctypes.c_int, vp, vp]
        L.orc_eval_exact.restype = ctypes.c_int
        L.orc_accd.argtypes = [vp, vp, vp, d, d, ctypes.c_int, dp, ctypes.POINTER(ctypes.c_int)]
        L.orc_accd.restype = ctypes.c_int
        L.orc_accd_scene.argtypes = [i32, vp, vp, i64, vp, d, d, ctypes.c_int, ctypes.c_int, vp]
        L.orc_accd_scene.restype = i64
        L.orc_num_threads.argtypes = []
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_stencil.argtypes = [vp, vp]
        L.orc_stencil.restype = ctypes.c_int
        L.orc_eval.argtypes = [i32, vp, vp, i64, vp, ctypes.POINTER(Params), ctypes.c_int, dp, vp, vp, vp, vp, vp, vp]
        L.orc_eval.restype = i64
        L.orc_friction_f.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, dp, dp]
        L.orc_friction_f.restype = None
        L.orc_friction_pair.argtypes = [vp, vp, vp, vp, ctypes.POINTER(Params), ctypes.POINTER(FParams), dp, vp, vp,
                                        vp]
        L.orc_friction_pair.restype = ctypes.c_int
        L.orc_friction_eval.argtypes = [i32, vp, vp, vp, i64, vp, ctypes.POINTER(Params), ctypes.POINTER(FParams),
                                        ctypes.c_int, dp, vp, vp, vp, vp]
        L.orc_friction_eval.restype = i64
        L.orc_candidates.argtypes = [i32, vp, vp, i64, vp, i64, vp, ctypes.c_double, vp, i64]
        L.orc_candidates.restype = i64
        L.orc_pair_xproj.argtypes = [vp, vp, vp, ctypes.POINTER(Params), vp, vp]
        L.orc_pair_xproj.restype = ctypes.c_int
        L.orc_eval_xproj.argtypes = [i32, vp, vp, i64, vp, ctypes.POINTER(Params), ctypes.c_int, vp]
        L.orc_eval_xproj.restype = ctypes.c_int
        L.orc_assemble.argtypes = [i32, i64, vp, vp, vp, vp, vp, vp, i64]
        L.orc_assemble.restype = i64
        L.orc_spmv.argtypes = [i32, i64, vp, vp, vp, vp, vp]
        L.orc_spmv.restype = None
        L.orc_matfree.argtypes = [i32, i64, vp, vp, vp, vp, vp]
        L.orc_matfree.restype = ctypes.c_int
        L.orc_pcg.argtypes = [i32, i64, vp, vp, vp, vp, vp, d, ctypes.c_int, dp]
        L.orc_pcg.restype = ctypes.c_int
        L.orc_pcg_delta.argtypes = [i32, i64, vp, vp, vp, vp, vp, d, ctypes.c_int, dp]
        L.orc_pcg_delta.restype = ctypes.c_int
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().orc_num_threads())


def barrier(g, dhat=1e-3, eq12=False):
    """(b, db/dg, d2b/dg2) of Eq. 24 (or Eq. 12)."""
    b, db, d2b = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib().orc_barrier(float(g), float(dhat), int(eq12), ctypes.byref(b), ctypes.byref(db), ctypes.byref(d2b))
    return b.value, db.value, d2b.value


def mollifier(c, epsx):
    e, de, d2e = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib().orc_mollifier(float(c), float(epsx), ctypes.byref(e), ctypes.byref(de), ctypes.byref(d2e))
    return e.value, de.value, d2e.value


def jacobi_eig(A):
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    lam = np.zeros(n)
    vec = np.zeros((n, n))
    lib().orc_jacobi_eig(n, A.ctypes.data, lam.ctypes.data, vec.ctypes.data)
    return lam, vec


def stencil(tuple4):
    t = np.ascontiguousarray(tuple4, dtype=np.int32)
    vid = np.zeros(4, dtype=np.int32)
    nv = lib().orc_stencil(t.ctypes.data, vid.ctypes.data)
    return nv, vid


def pair_local(tuple4, xs, xr=None, prm=None, debug=False):
    """One pair.  ``xs``/``xr``: stencil positions ``[4][3]`` (unused rows ignored).

    Returns a dict with E, grad (12,), hess (12, 12), subtype, mollified, d2
    and, with ``debug``, the inner Hessian before/after projection, vec(db/dJ)
    and the Jacobian dimension m.
    """
    prm = prm or params()
    t = np.ascontiguousarray(tuple4, dtype=np.int32)
    xs = np.zeros((4, 3)) + 0.0 if xs is None else np.ascontiguousarray(np.asarray(xs, np.float64).reshape(-1, 3))
    if xs.shape[0] < 4:
        xs = np.vstack([xs, np.zeros((4 - xs.shape[0], 3))])
    xr_a = None
    if xr is not None:
        xr_a = np.ascontiguousarray(np.asarray(xr, np.float64).reshape(-1, 3))
        if xr_a.shape[0] < 4:
            xr_a = np.vstack([xr_a, np.zeros((4 - xr_a.shape[0], 3))])
    E = ctypes.c_double()
    g = np.zeros(12)
    H = np.zeros(144)
    st, mo, m = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    d2 = ctypes.c_double()
    iH = np.zeros(81) if debug else None
    iHp = np.zeros(81) if debug else None
    bJ = np.zeros(9) if debug else None
    rc = lib().orc_pair_local(t.ctypes.data, xs.ctypes.data, _ptr(xr_a), ctypes.byref(prm), ctypes.byref(E),
                              g.ctypes.data, H.ctypes.data, ctypes.byref(st), ctypes.byref(mo), ctypes.byref(d2),
                              _ptr(iH), _ptr(iHp), _ptr(bJ), ctypes.byref(m))
    if rc < 0:
        raise ValueError("malformed tuple")
    out = dict(E=E.value, grad=g, hess=H.reshape(12, 12), subtype=st.value, mollified=bool(mo.value), d2=d2.value)
    if debug:
        M = m.value * m.value
        out.update(m=m.value, innerH=iH[:M * M].reshape(M, M), innerHp=iHp[:M * M].reshape(M, M), dbdJ=bJ[:M])
    return out


def pair_xproj(tuple4, xs, xr=None, prm=None):
    """The unprojected proxy Hessian kappa D^T H D [12][12] of one pair and its
    projection computed in x-space by Jacobi rotations (the traditional route)."""
    prm = prm or params()
    t = np.ascontiguousarray(tuple4, dtype=np.int32)
    xs = np.ascontiguousarray(np.asarray(xs, np.float64).reshape(-1, 3))
    if xs.shape[0] < 4:
        xs = np.vstack([xs, np.zeros((4 - xs.shape[0], 3))])
    xr_a = None
    if xr is not None:
        xr_a = np.ascontiguousarray(np.asarray(xr, np.float64).reshape(-1, 3))
        if xr_a.shape[0] < 4:
            xr_a = np.vstack([xr_a, np.zeros((4 - xr_a.shape[0], 3))])
    K = np.zeros(144)
    Px = np.zeros(144)
    if lib().orc_pair_xproj(t.ctypes.data, xs.ctypes.data, _ptr(xr_a), ctypes.byref(prm), K.ctypes.data,
                            Px.ctypes.data) < 0:
        raise ValueError("malformed tuple")
    return K.reshape(12, 12), Px.reshape(12, 12)


def eval_xproj(x, tuples, prm=None, x_rest=None, nthreads=0):
    """pair_xproj's projection for every tuple of a list, [P][12][12]."""
    prm = prm or params()
    x = np.ascontiguousarray(x, dtype=np.float64)
    t = np.ascontiguousarray(tuples, dtype=np.int32).reshape(-1, 4)
    xr = None if x_rest is None else np.ascontiguousarray(x_rest, dtype=np.float64)
    out = np.zeros((t.shape[0], 144))
    if lib().orc_eval_xproj(x.shape[0], x.ctypes.data, _ptr(xr), t.shape[0], t.ctypes.data, ctypes.byref(prm),
                            int(nthreads), out.ctypes.data) < 0:
        raise ValueError("malformed tuple or vertex index out of range")
    return out.reshape(-1, 12, 12)


def pair_exact(tuple4, xs, xr=None, prm=None):
    """Exact Hessian of one pair's energy and its numeric PSD projection
    (both [12][12]); the traditional route of Table 1."""
    prm = prm or params()
    t = np.ascontiguousarray(tuple4, dtype=np.int32)
    xs = _pad4(xs)
    xr_a = None if xr is None else _pad4(xr)
    H = np.zeros(144)
    Hp = np.zeros(144)
    if lib().orc_pair_exact(t.ctypes.data, xs.ctypes.data, _ptr(xr_a), ctypes.byref(prm), H.ctypes.data,
                            Hp.ctypes.data) < 0:
        raise ValueError("malformed tuple")
    return H.reshape(12, 12), Hp.reshape(12, 12)


def eval_exact(x, tuples, prm=None, x_rest=None, nthreads=0, want_exact=True, want_proj=True):
    """orc_pair_exact over a tuple list: (pairH or None, pairHp or None), [P][12][12]."""
    prm = prm or params()
    x = np.ascontiguousarray(x, dtype=np.float64)
    t = np.ascontiguousarray(tuples, dtype=np.int32).reshape(-1, 4)
    xr = None if x_rest is None else np.ascontiguousarray(x_rest, dtype=np.float64)
    P = t.shape[0]
    H = np.zeros((P, 12, 12)) if want_exact else None
    Hp = np.zeros((P, 12, 12)) if want_proj else None
    if lib().orc_eval_exact(int(x.shape[0]), x.ctypes.data, _ptr(xr), P, t.ctypes.data, ctypes.byref(prm),
                            int(nthreads), _ptr(H), _ptr(Hp)) < 0:
        raise ValueError("malformed tuple or vertex index out of range")
    return H, Hp


def accd(tuple4, xs, ps, s=0.1, tc=1.0, max_iter=1_000_000):
    """Additive CCD of one tuple moving by ps: (toi, trial steps; -1 if capped)."""
    t = np.ascontiguousarray(tuple4, dtype=np.int32)
    xs = _pad4(xs)
    ps = _pad4(ps)
    toi = ctypes.c_double()
    it = ctypes.c_int()
    rc = lib().orc_accd(t.ctypes.data, xs.ctypes.data, ps.ctypes.data, float(s), float(tc), int(max_iter),
                        ctypes.byref(toi), ctypes.byref(it))
    if rc == -2:
        raise ValueError("malformed tuple")
    return toi.value, it.value


def accd_scene(x, disp, tuples, s=0.1, tc=1.0, max_iter=1_000_000, nthreads=0):
    """orc_accd over a tuple list: (toi [P], number stopped by max_iter)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    d = np.ascontiguousarray(disp, dtype=np.float64)
    t = np.ascontiguousarray(tuples, dtype=np.int32).reshape(-1, 4)
    toi = np.zeros(t.shape[0])
    n = lib().orc_accd_scene(int(x.shape[0]), x.ctypes.data, d.ctypes.data, t.shape[0], t.ctypes.data, float(s),
                             float(tc), int(max_iter), int(nthreads), toi.ctypes.data)
    if n < 0:
        raise ValueError("malformed tuple or vertex index out of range")
    return toi, int(n)


def friction_f(y, eps_v, dt):
    f0, f1, df1 = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib().orc_friction_f(float(y), float(eps_v), float(dt), ctypes.byref(f0), ctypes.byref(f1), ctypes.byref(df1))
    return f0.value, f1.value, df1.value


def _pad4(a):
    a = np.ascontiguousarray(np.asarray(a, np.float64).reshape(-1, 3))
    if a.shape[0] < 4:
        a = np.vstack([a, np.zeros((4 - a.shape[0], 3))])
    return np.ascontiguousarray(a)


def friction_pair(tuple4, xs_n, xs, xr=None, prm=None, fp=None):
    """Lagged friction of one pair: dict with D, grad (12,), hess (12, 12),
    lam, normal (3,), coef (4,), u (2,)."""
    prm = prm or params()
    fp = fp or fparams()
    t = np.ascontiguousarray(tuple4, dtype=np.int32)
    xn, xc = _pad4(xs_n), _pad4(xs)
    xr_a = None if xr is None else _pad4(xr)
    D = ctypes.c_double()
    g = np.zeros(12)
    H = np.zeros(144)
    info = np.zeros(10)
    if lib().orc_friction_pair(t.ctypes.data, xn.ctypes.data, _ptr(xr_a), xc.ctypes.data, ctypes.byref(prm),
                               ctypes.byref(fp), ctypes.byref(D), g.ctypes.data, H.ctypes.data,
                               info.ctypes.data) < 0:
        raise ValueError("malformed tuple")
    return dict(D=D.value, grad=g, hess=H.reshape(12, 12), lam=info[0], normal=info[1:4], coef=info[4:8],
                u=info[8:10])


def friction_scene(x_n, x, tuples, prm=None, fp=None, x_rest=None, nthreads=0, per_pair=False):
    """Friction energy and gradient of a list (plus per-pair data on request)."""
    prm = prm or params()
    fp = fp or fparams()
    x_n = np.ascontiguousarray(x_n, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    t = np.ascontiguousarray(tuples, dtype=np.int32).reshape(-1, 4)
    xr = None if x_rest is None else np.ascontiguousarray(x_rest, dtype=np.float64)
    V, P = x.shape[0], t.shape[0]
    grad = np.zeros((V, 3))
    E = ctypes.c_double()
    pE = np.zeros(P) if per_pair else None
    pG = np.zeros((P, 12)) if per_pair else None
    pH = np.zeros((P, 144)) if per_pair else None
    rc = lib().orc_friction_eval(V, x_n.ctypes.data, x.ctypes.data, _ptr(xr), P, t.ctypes.data, ctypes.byref(prm),
                                 ctypes.byref(fp), int(nthreads), ctypes.byref(E), grad.ctypes.data, _ptr(pE),
                                 _ptr(pG), _ptr(pH))
    if rc < 0:
        raise ValueError("malformed tuple or vertex index out of range")
    out = dict(E=E.value, grad=grad)
    if per_pair:
        out.update(pairE=pE, pairG=pG, pairH=pH.reshape(P, 12, 12))
    return out


def candidates(x, vobj, tris, edges, dhat):
    """All contact candidates by brute force, int32 [P][4] (PT then EE)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    vobj = np.ascontiguousarray(vobj, dtype=np.int32)
    tris = np.ascontiguousarray(tris, dtype=np.int32).reshape(-1, 3)
    edges = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
    args = (x.shape[0], x.ctypes.data, vobj.ctypes.data, tris.shape[0], tris.ctypes.data, edges.shape[0],
            edges.ctypes.data, float(dhat))
    n = lib().orc_candidates(*args, None, 0)
    out = np.zeros((max(n, 1), 4), np.int32)
    lib().orc_candidates(*args, out.ctypes.data, n)
    return out[:n]


def eval_scene(x, tuples, prm=None, x_rest=None, nthreads=0, per_pair=False):
    """Energy and gradient of a whole pair list (plus per-pair data on request)."""
    prm = prm or params()
    x = np.ascontiguousarray(x, dtype=np.float64)
    t = np.ascontiguousarray(tuples, dtype=np.int32).reshape(-1, 4)
    xr = None if x_rest is None else np.ascontiguousarray(x_rest, dtype=np.float64)
    V, P = x.shape[0], t.shape[0]
    grad = np.zeros((V, 3))
    E = ctypes.c_double()
    pE = np.zeros(P) if per_pair else None
    pG = np.zeros((P, 12)) if per_pair else None
    pH = np.zeros((P, 144)) if per_pair else None
    st = np.zeros(P, np.int32)
    mo = np.zeros(P, np.int32)
    ndeg = lib().orc_eval(V, x.ctypes.data, _ptr(xr), P, t.ctypes.data, ctypes.byref(prm), int(nthreads),
                          ctypes.byref(E), grad.ctypes.data, _ptr(pE), _ptr(pG), _ptr(pH),
                          st.ctypes.data, mo.ctypes.data)
    if ndeg < 0:
        raise ValueError("malformed tuple or vertex index out of range")
    out = dict(E=E.value, grad=grad, subtype=st, mollified=mo.astype(bool), n_degenerate=int(ndeg))
    if per_pair:
        out.update(pairE=pE, pairG=pG, pairH=pH.reshape(P, 12, 12))
    return out


def assemble(V, tuples, pairH, diag=None):
    """Sorted block list (rows, cols, vals[nb,3,3]) of diag(d) I + sum_k S_k^T H_k S_k."""
    t = np.ascontiguousarray(tuples, dtype=np.int32).reshape(-1, 4)
    H = np.ascontiguousarray(pairH, dtype=np.float64).reshape(-1, 144)
    dg = None if diag is None else np.ascontiguousarray(diag, dtype=np.float64)
    L = lib()
    nb = L.orc_assemble(V, t.shape[0], t.ctypes.data, H.ctypes.data, _ptr(dg), None, None, None, 0)
    if nb < 0:
        raise ValueError("malformed tuple")
    rows = np.zeros(nb, np.int32)
    cols = np.zeros(nb, np.int32)
    vals = np.zeros((nb, 9))
    L.orc_assemble(V, t.shape[0], t.ctypes.data, H.ctypes.data, _ptr(dg), rows.ctypes.data, cols.ctypes.data,
                   vals.ctypes.data, nb)
    return rows, cols, vals.reshape(nb, 3, 3)


def spmv(V, rows, cols, vals, x):
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
    y = np.zeros(3 * V)
    vals = np.ascontiguousarray(vals, dtype=np.float64)
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    lib().orc_spmv(V, rows.shape[0], rows.ctypes.data, cols.ctypes.data, vals.ctypes.data, x.ctypes.data, y.ctypes.data)
    return y


def matfree(V, tuples, pairH, x, diag=None):
    """y = (diag (x) I3 + sum_k S_k^T H_k S_k) x by local mat-vecs, no global matrix."""
    t = np.ascontiguousarray(tuples, dtype=np.int32).reshape(-1, 4)
    H = np.ascontiguousarray(pairH, dtype=np.float64).reshape(-1, 144)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
    dg = None if diag is None else np.ascontiguousarray(diag, dtype=np.float64)
    y = np.zeros(3 * V)
    if lib().orc_matfree(V, t.shape[0], t.ctypes.data, H.ctypes.data, _ptr(dg), x.ctypes.data, y.ctypes.data) < 0:
        raise ValueError("malformed tuple")
    return y


def pcg(V, rows, cols, vals, b, x0=None, rtol=1e-6, maxit=1000, delta=False):
    """Block-Jacobi PCG on the COO block matrix; stops when ||r|| <= rtol ||b||,
    or with delta=True by the paper's termination r.z <= rtol r0.z0 (its
    PCG in the implementation section, tolerance 1e-4 there).  Returns (x,
    iterations, ||r||/||b||)."""
    b = np.ascontiguousarray(b, dtype=np.float64).reshape(-1)
    x = np.zeros(3 * V) if x0 is None else np.ascontiguousarray(x0, dtype=np.float64).reshape(-1).copy()
    vals = np.ascontiguousarray(vals, dtype=np.float64)
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    rr = ctypes.c_double()
    f = lib().orc_pcg_delta if delta else lib().orc_pcg
    it = f(V, rows.shape[0], rows.ctypes.data, cols.ctypes.data, vals.ctypes.data, b.ctypes.data,
           x.ctypes.data, float(rtol), int(maxit), ctypes.byref(rr))
    return x, it, rr.value
