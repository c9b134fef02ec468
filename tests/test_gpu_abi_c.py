"""The C ABI from plain C (tests/abi_check.c, built by __graft_entry__.build):
context, pair build, pattern, eval + assembly, SpMV and PCG called from a C
program that links only the library and the HIP runtime, on the two-sheet
scene, against the oracle:

* every call returns OK;
* energy and gradient as the oracle's (1e-12 / 1e-10 relative);
* the assembled matrix as the oracle's assembly (1e-9 of its largest entry);
* y = A grad as the oracle's matrix times the program's gradient (1e-12);
* after 50 PCG iterations the solution's relative residual under the
  oracle's matrix equals the one the call reports (to 1e-6 of it) and is
  below 1e-6.
"""
import os
import struct
import subprocess

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

scipy_sparse = pytest.importorskip("scipy.sparse")

import oracle  # noqa: E402
import scenes  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "_build", "abi_check")


def _gpu():
    try:
        import torch
    except ImportError:
        return False
    return torch.cuda.is_available()


def _write(path, s, diag, maxit):
    V, P = s.V, s.tuples.shape[0]
    with open(path, "wb") as f:
        f.write(struct.pack("<iqddi", V, P, s.dhat, s.kappa, maxit))
        f.write(np.ascontiguousarray(s.x, np.float64).tobytes())
        f.write(np.ascontiguousarray(s.x_rest, np.float64).tobytes())
        f.write(np.ascontiguousarray(diag, np.float64).tobytes())
        f.write(np.ascontiguousarray(s.tuples, np.int32).tobytes())


def _read(path, V):
    b = open(path, "rb").read()
    o = 0

    def take(fmt_or_dtype, n=1):
        nonlocal o
        if isinstance(fmt_or_dtype, str):
            size = struct.calcsize(fmt_or_dtype)
            v = struct.unpack_from(fmt_or_dtype, b, o)
            o += size
            return v
        a = np.frombuffer(b, dtype=fmt_or_dtype, count=n, offset=o)
        o += a.nbytes
        return a

    st = take("<6i")
    (E,) = take("<d")
    (nnzb,) = take("<q")
    (iters,) = take("<i")
    (relres,) = take("<d")
    out = {"status": st, "E": E, "nnzb": nnzb, "iters": iters, "relres": relres}
    if o < len(b):
        out["grad"] = take(np.float64, 3 * V).reshape(V, 3)
        out["row_ptr"] = take(np.int32, V + 1)
        out["col_idx"] = take(np.int32, nnzb)
        out["val"] = take(np.float64, 9 * nnzb).reshape(9, nnzb)
        out["y"] = take(np.float64, 3 * V)
        out["sol"] = take(np.float64, 3 * V)
    return out


def _oracle_matrix(s, diag):
    r = oracle.eval_scene(s.x, s.tuples, oracle.params(dhat=s.dhat, kappa=s.kappa), x_rest=s.x_rest, per_pair=True)
    rows, cols, vals = oracle.assemble(s.V, s.tuples, r["pairH"], diag)
    b = vals.reshape(-1, 3, 3)
    ii = (3 * np.asarray(rows)[:, None, None] + np.arange(3)[None, :, None]).repeat(3, 2)
    jj = (3 * np.asarray(cols)[:, None, None] + np.arange(3)[None, None, :]).repeat(3, 1)
    G = scipy_sparse.coo_matrix((b.ravel(), (ii.ravel(), jj.ravel())), shape=(3 * s.V, 3 * s.V)).tocsr()
    return r, G


def test_c_program_drives_the_path(tmp_path):
    if not _gpu():
        pytest.skip("no GPU")
    if not os.path.exists(EXE):
        pytest.skip("tests/_build/abi_check not built (run __graft_entry__.build())")
    s = scenes.two_sheets(n=16, seed=1)
    diag = np.linspace(1.0, 2.0, s.V)
    maxit = 50
    fin, fout = tmp_path / "in.bin", tmp_path / "out.bin"
    _write(fin, s, diag, maxit)
    r = subprocess.run([EXE, str(fin), str(fout)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    out = _read(fout, s.V)
    assert out["status"] == (0, 0, 0, 0, 0, 0), out["status"]
    ref, G = _oracle_matrix(s, diag)
    assert abs(out["E"] - ref["E"]) <= 1e-12 * abs(ref["E"])
    g = out["grad"]
    assert np.abs(g - ref["grad"]).max() <= 1e-10 * np.abs(ref["grad"]).max()
    D = scipy_sparse.bsr_matrix((out["val"].T.reshape(-1, 3, 3), out["col_idx"], out["row_ptr"]),
                                shape=(3 * s.V, 3 * s.V)).tocsr()
    assert abs(D - G).max() <= 1e-9 * abs(G).max()
    yr = G @ g.ravel()
    assert np.abs(out["y"] - yr).max() <= 1e-12 * np.abs(yr).max()
    b = -g.ravel()
    res = np.linalg.norm(G @ out["sol"] - b) / np.linalg.norm(b)
    assert out["iters"] == maxit
    assert abs(res - out["relres"]) <= 1e-6 * out["relres"] + 1e-13 and res < 1e-6, (res, out["relres"])
