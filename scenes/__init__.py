"""Seeded synthetic contact scenes (input generators only).

This module is shared by the oracle-side tests and the GPU path.  It builds
triangulated cloth sheets, picks contact candidates with an AABB broad phase
(``broadphase.c``) and returns plain numpy arrays.  It holds none of the
barrier method's arithmetic: no distances, no barrier values, no
classification.  Candidates use the paper's sign-encoded tuples
(Sec. 7.2, "Data structures"): point-triangle ``[-(p+1), t0, t1, t2]`` and
edge-edge ``[a0, a1, b0, b1]``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libbroadphase.so")
_lib = None


def build_broadphase(force: bool = True) -> str:
    """Compile the broad-phase helper with gcc (host code only)."""
    if force or not os.path.exists(_LIB_PATH):
        src = os.path.join(_HERE, "broadphase.c")
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_broadphase(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        lib.bp_candidates.restype = ctypes.c_int64
        lib.bp_candidates.argtypes = [
            ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
            ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
            ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.POINTER(ctypes.c_int32)),
        ]
        lib.bp_free.restype = None
        lib.bp_free.argtypes = [ctypes.POINTER(ctypes.c_int32)]
        _lib = lib
    return _lib


def broadphase(x, vobj, tris, edges, dhat, want_pt=True, want_ee=True) -> np.ndarray:
    """All cross-object PT and EE candidates whose boxes come within ``dhat``.

    Returns ``int32[P][4]`` sign-encoded tuples, sorted (PT first, then EE,
    each by decoded vertex ids).
    """
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    vobj = np.ascontiguousarray(vobj, dtype=np.int32)
    tris = np.ascontiguousarray(tris, dtype=np.int32).reshape(-1, 3)
    edges = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
    out = ctypes.POINTER(ctypes.c_int32)()
    n = lib.bp_candidates(int(x.shape[0]), x.ctypes.data, vobj.ctypes.data,
                          int(tris.shape[0]), tris.ctypes.data, int(edges.shape[0]), edges.ctypes.data,
                          float(dhat), int(bool(want_pt)), int(bool(want_ee)), ctypes.byref(out))
    if n == 0:
        if out:
            lib.bp_free(out)
        return np.zeros((0, 4), dtype=np.int32)
    arr = np.ctypeslib.as_array(out, shape=(n, 4)).copy()
    lib.bp_free(out)
    return arr


@dataclass
class Scene:
    """A synthetic contact scene.  Positions are AoS float64 ``[V][3]``."""

    name: str
    x: np.ndarray
    x_rest: np.ndarray
    tris: np.ndarray
    edges: np.ndarray
    vobj: np.ndarray
    dhat: float
    kappa: float
    tuples: np.ndarray
    diag: np.ndarray | None = None  # per-vertex mass / dt^2
    meta: dict = field(default_factory=dict)

    @property
    def V(self) -> int:
        return int(self.x.shape[0])

    @property
    def P(self) -> int:
        return int(self.tuples.shape[0])


def sheet_topology(n: int):
    """Triangles and edges of an ``n x n`` vertex grid.

    Vertex (i, j) (row i along y, column j along x) has index ``i*n + j``; each
    quad is split along its (i, j)-(i+1, j+1) diagonal.
    """
    i, j = np.meshgrid(np.arange(n - 1), np.arange(n - 1), indexing="ij")
    a = (i * n + j).ravel()
    b = (i * n + j + 1).ravel()
    c = ((i + 1) * n + j + 1).ravel()
    d = ((i + 1) * n + j).ravel()
    tris = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)]).astype(np.int32)
    ii, jj = np.meshgrid(np.arange(n), np.arange(n - 1), indexing="ij")
    horiz = np.stack([(ii * n + jj).ravel(), (ii * n + jj + 1).ravel()], 1)
    ii, jj = np.meshgrid(np.arange(n - 1), np.arange(n), indexing="ij")
    vert = np.stack([(ii * n + jj).ravel(), ((ii + 1) * n + jj).ravel()], 1)
    diag = np.stack([a, c], 1)
    edges = np.concatenate([horiz, vert, diag]).astype(np.int32)
    return tris, edges


def _sheet_xy(n: int):
    u = np.linspace(0.0, 1.0, n)
    yy, xx = np.meshgrid(u, u, indexing="ij")
    return xx.ravel(), yy.ravel()


def _stack(sheets_x, n):
    tris1, edges1 = sheet_topology(n)
    nv = n * n
    xs, tris, edges, vobj = [], [], [], []
    for k, xk in enumerate(sheets_x):
        xs.append(xk)
        tris.append(tris1 + k * nv)
        edges.append(edges1 + k * nv)
        vobj.append(np.full(nv, k, dtype=np.int32))
    return (np.concatenate(xs), np.concatenate(tris).astype(np.int32),
            np.concatenate(edges).astype(np.int32), np.concatenate(vobj))


def two_sheets(n: int = 16, dhat: float = 1e-3, kappa: float = 1e4, seed: int = 1,
               offset: float = 0.5, jitter: float = 0.2, with_pairs: bool = True) -> Scene:
    """Two ``n x n`` sheets over the unit square, the upper one at
    ``offset*dhat`` with per-vertex uniform z jitter of ``+-jitter*dhat``.

    The lower sheet is flat at z = 0.  ``x_rest`` is the un-jittered pair of
    sheets.
    """
    rng = np.random.default_rng(seed)
    xx, yy = _sheet_xy(n)
    nv = n * n
    jit = rng.uniform(-jitter, jitter, nv) * dhat
    lower = np.stack([xx, yy, np.zeros(nv)], 1)
    upper = np.stack([xx, yy, offset * dhat + jit], 1)
    upper_rest = np.stack([xx, yy, np.full(nv, offset * dhat)], 1)
    x, tris, edges, vobj = _stack([lower, upper], n)
    x_rest, _, _, _ = _stack([lower, upper_rest], n)
    tuples = broadphase(x, vobj, tris, edges, dhat) if with_pairs else np.zeros((0, 4), np.int32)
    return Scene(f"two_sheets_{n}", x, x_rest, tris, edges, vobj, dhat, kappa, tuples,
                 meta=dict(n=n, seed=seed, offset=offset, jitter=jitter))


def stacked_sheets(n_sheets: int = 10, n: int = 256, dhat: float = 1e-3, kappa: float = 1e4,
                   seed: int = 2, spacing: float = 0.6, jitter: float = 0.3,
                   shear_frac: float = 0.02, shear_deg: float = 1.0,
                   mass: float = 1e-3, dt: float = 1e-2, with_pairs: bool = True) -> Scene:
    """``n_sheets`` stacked ``n x n`` sheets over the unit square.

    Sheet k sits at ``z = spacing*k*dhat`` with per-vertex uniform jitter of
    ``+-jitter*dhat``.  ``max(1, round(shear_frac*n_sheets))`` sheets, chosen
    by the seed, are sheared: ``x <- x + tan(shear_deg) * (y - 0.5)``.
    ``x_rest`` is the flat, unsheared stack; ``diag`` is ``mass/dt^2`` per
    vertex.
    """
    rng = np.random.default_rng(seed)
    n_shear = max(1, int(round(shear_frac * n_sheets)))
    sheared = set(int(s) for s in rng.choice(n_sheets, size=n_shear, replace=False))
    jit = rng.uniform(-jitter, jitter, (n_sheets, n * n)) * dhat
    xx, yy = _sheet_xy(n)
    nv = n * n
    cur, rest = [], []
    t = np.tan(np.deg2rad(shear_deg))
    for k in range(n_sheets):
        z0 = spacing * k * dhat
        rest.append(np.stack([xx, yy, np.full(nv, z0)], 1))
        xk = xx + t * (yy - 0.5) if k in sheared else xx
        cur.append(np.stack([xk, yy, z0 + jit[k]], 1))
    x, tris, edges, vobj = _stack(cur, n)
    x_rest, _, _, _ = _stack(rest, n)
    tuples = broadphase(x, vobj, tris, edges, dhat) if with_pairs else np.zeros((0, 4), np.int32)
    diag = np.full(x.shape[0], mass / dt ** 2)
    return Scene(f"stacked_sheets_{n_sheets}x{n}", x, x_rest, tris, edges, vobj, dhat, kappa, tuples,
                 diag=diag, meta=dict(n_sheets=n_sheets, n=n, seed=seed, sheared=sorted(sheared)))


def decode_tuples(tuples: np.ndarray):
    """Split sign-encoded tuples into (kind, stencil) with kind 0 = point-first
    (PT/PE/PP), 1 = edge-edge; stencil holds decoded vertex ids (-1 unused)."""
    t = np.asarray(tuples, dtype=np.int64)
    kind = (t[:, 0] >= 0).astype(np.int32)
    st = t.copy()
    st[:, 0] = np.where(t[:, 0] < 0, -t[:, 0] - 1, t[:, 0])
    st[:, 1] = np.where(t[:, 1] < 0, -t[:, 1] - 1, t[:, 1])
    # close-to-parallel point-edge / point-point encodings: the first two
    # entries negative, then every negative entry is a vertex -(i+1)
    par = (t[:, 0] < 0) & (t[:, 1] < 0)
    for c in (2, 3):
        st[:, c] = np.where(par & (t[:, c] < 0), -t[:, c] - 1, st[:, c])
    return kind, st


def subsample(scene: Scene, n_pairs: int, seed: int = 0) -> np.ndarray:
    """A seeded random subset of ``n_pairs`` tuples (order preserved)."""
    rng = np.random.default_rng(seed)
    if n_pairs >= scene.P:
        return scene.tuples.copy()
    idx = np.sort(rng.choice(scene.P, size=n_pairs, replace=False))
    return scene.tuples[idx].copy()


def cube_surface_topology(n: int):
    """Boundary triangles and edges of an ``n x n x n`` vertex grid (vertex
    (i, j, k) -> index (i*n + j)*n + k); each boundary quad is split along a
    diagonal.  Interior vertices stay in the vertex set (they touch no
    boundary primitive)."""
    idx = np.arange(n ** 3).reshape(n, n, n)
    tris = []
    for axis in range(3):
        for side in (0, n - 1):
            face = np.take(idx, side, axis=axis)           # n x n grid of that face
            a = face[:-1, :-1].ravel(); b = face[:-1, 1:].ravel()
            c = face[1:, 1:].ravel(); d = face[1:, :-1].ravel()
            tris.append(np.stack([a, b, c], 1))
            tris.append(np.stack([a, c, d], 1))
    tris = np.concatenate(tris).astype(np.int32)
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
    e = np.sort(e, axis=1)
    edges = np.unique(e, axis=0).astype(np.int32)
    return tris, edges


def cube_lattice(m: int = 6, n: int = 10, dhat: float = 1e-3, kappa: float = 1e4, seed: int = 3,
                 gap_lo: float = 0.1, gap_hi: float = 0.9, with_pairs: bool = True) -> Scene:
    """An ``m x m x m`` lattice of unit cubes with ``n^3`` vertices each (spacing
    1/(n-1)).  The gap across each lattice plane (m-1 planes per axis) is drawn
    uniformly from ``(gap_lo, gap_hi) * dhat``, so facing faces are parallel and
    aligned.  ``x_rest`` = x (the gaps are part of the rest configuration)."""
    rng = np.random.default_rng(seed)
    gaps = rng.uniform(gap_lo, gap_hi, size=(3, m - 1)) * dhat
    offs = np.zeros((3, m))
    for ax in range(3):
        offs[ax, 1:] = np.arange(1, m) * 1.0 + np.cumsum(gaps[ax])
    u = np.linspace(0.0, 1.0, n)
    gx, gy, gz = np.meshgrid(u, u, u, indexing="ij")
    local = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], 1)
    tris1, edges1 = cube_surface_topology(n)
    nv = n ** 3
    xs, tris, edges, vobj = [], [], [], []
    c = 0
    for i in range(m):
        for j in range(m):
            for k in range(m):
                xs.append(local + np.array([offs[0, i], offs[1, j], offs[2, k]]))
                tris.append(tris1 + c * nv)
                edges.append(edges1 + c * nv)
                vobj.append(np.full(nv, c, dtype=np.int32))
                c += 1
    x = np.concatenate(xs)
    tris = np.concatenate(tris).astype(np.int32)
    edges = np.concatenate(edges).astype(np.int32)
    vobj = np.concatenate(vobj)
    tuples = broadphase(x, vobj, tris, edges, dhat) if with_pairs else np.zeros((0, 4), np.int32)
    return Scene(f"cube_lattice_{m}x{n}", x, x.copy(), tris, edges, vobj, dhat, kappa, tuples,
                 meta=dict(m=m, n=n, seed=seed, gaps=gaps))


@dataclass
class BatchScene:
    """Independent scenes concatenated into one vertex array and one tuple
    list: scene s owns vertices ``[vert_off[s], vert_off[s+1])`` and tuples
    ``[pair_off[s], pair_off[s+1])``, with its own dhat and kappa."""

    name: str
    x: np.ndarray
    x_rest: np.ndarray
    tuples: np.ndarray
    vert_off: np.ndarray
    pair_off: np.ndarray
    dhat: np.ndarray
    kappa: np.ndarray
    scenes: list
    meta: dict = field(default_factory=dict)

    @property
    def V(self) -> int:
        return int(self.x.shape[0])

    @property
    def P(self) -> int:
        return int(self.tuples.shape[0])

    @property
    def S(self) -> int:
        return len(self.scenes)


def offset_tuples(tuples: np.ndarray, off: int) -> np.ndarray:
    """Shift the vertex ids of sign-encoded tuples by ``off``: columns 0 and 1
    hold ids or -(id+1), columns 2 and 3 ids or -1 (unused)."""
    t = np.asarray(tuples, dtype=np.int64).copy()
    for c in (0, 1):
        t[:, c] = np.where(t[:, c] >= 0, t[:, c] + off, t[:, c] - off)
    for c in (2, 3):
        t[:, c] = np.where(t[:, c] >= 0, t[:, c] + off, t[:, c])
    return t.astype(np.int32)


def concat_scenes(scenes: list, name: str = "batch") -> BatchScene:
    """Concatenate scenes (each with its own dhat and kappa) into one batch."""
    vo, po = [0], [0]
    xs, xr, ts = [], [], []
    for sc in scenes:
        ts.append(offset_tuples(sc.tuples, vo[-1]))
        xs.append(sc.x)
        xr.append(sc.x_rest)
        vo.append(vo[-1] + sc.V)
        po.append(po[-1] + sc.P)
    tuples = np.concatenate(ts) if ts else np.zeros((0, 4), np.int32)
    return BatchScene(name, np.concatenate(xs), np.concatenate(xr), np.ascontiguousarray(tuples),
                      np.array(vo, np.int32), np.array(po, np.int64),
                      np.array([sc.dhat for sc in scenes]), np.array([sc.kappa for sc in scenes]), list(scenes))


def batch_two_sheets(S: int = 64, r_lo: int = 32, r_hi: int = 256, dhat_lo: float = 1e-4, dhat_hi: float = 1e-2,
                     kappa: float = 1e4, seed_base: int = 1000) -> BatchScene:
    """``S`` two-sheet scenes (the recipe of ``two_sheets``): scene s draws,
    from seed ``seed_base + s``, its resolution r uniform in ``r_lo..r_hi``
    vertices per side and dhat log-uniform in ``[dhat_lo, dhat_hi]``; the
    upper sheet sits at 0.5 dhat with +-0.2 dhat jitter."""
    scenes = []
    for s in range(S):
        rng = np.random.default_rng(seed_base + s)
        r = int(rng.integers(r_lo, r_hi + 1))
        dhat = float(10.0 ** rng.uniform(np.log10(dhat_lo), np.log10(dhat_hi)))
        scenes.append(two_sheets(n=r, dhat=dhat, kappa=kappa, seed=seed_base + s))
    b = concat_scenes(scenes, name=f"batch_two_sheets_{S}")
    b.meta = dict(S=S, r_lo=r_lo, r_hi=r_hi, dhat_lo=dhat_lo, dhat_hi=dhat_hi, seed_base=seed_base,
                  r=[sc.meta["n"] for sc in scenes])
    return b
