"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tolerances (FP64 path): energy and gradient within 1e-9 relative (the
gradient normwise in the max norm over all components, per pair relative to
that pair's own magnitude), proxy-Hessian blocks within 1e-9 of the largest
entry; FP32 blocks within 1e-5 relative Frobenius norm of the FP64 block.
Integer outputs (staged pair sets, pattern) are compared exactly, except
that a pair at distance within rounding of dhat may be active on one side
only (its contribution is zero to rounding there, which is checked).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import scenes  # noqa: E402

TOL = 1e-9


@pytest.fixture(scope="module")
def gp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2308_09400_amd as gp
    torch.cuda.set_device(0)
    return gp


def _prm_pair(gp, dhat, kappa, filter=True, mollify=True, eq12=False):
    flags = (gp.FLAG_FILTER if filter else 0) | (gp.FLAG_MOLLIFY if mollify else 0) | (gp.FLAG_BARRIER_EQ12 if eq12 else 0)
    return (gp.params(dhat=dhat, kappa=kappa, flags=flags),
            oracle.params(dhat=dhat, kappa=kappa, filter=filter, mollify=mollify, eq12=eq12))


def run_gpu(gp, x, xr, tuples, prm, diag=None, dtype=0, inspect=True):
    dev = torch.device("cuda", 0)
    X = torch.tensor(x, device=dev)
    XR = torch.tensor(xr, device=dev) if xr is not None else None
    T = torch.tensor(np.asarray(tuples, np.int32).reshape(-1, 4), device=dev)
    D = torch.tensor(diag, device=dev) if diag is not None else None
    ctx = gp.Context()
    info = gp.pairs_build(ctx, X, T, prm, x_rest=XR)
    A = gp.BsrMatrix(ctx, dtype=dtype)
    E, g = gp.eval_assemble(ctx, X, prm, A, diag=D, x_rest=XR)
    out = dict(ctx=ctx, info=info, A=A, E=E.item(), grad=g.cpu().numpy(), X=X, XR=XR)
    if inspect:
        pi = gp.pair_inspect(ctx, X, prm, x_rest=XR, want=("src", "type", "vid", "mult", "energy", "grad", "hess"))
        out["pairs"] = {k: v.cpu().numpy() for k, v in pi.items()}
    return out


def run_oracle(x, xr, tuples, prm, diag=None):
    r = oracle.eval_scene(x, tuples, prm, x_rest=xr, per_pair=True)
    rows, cols, vals = oracle.assemble(x.shape[0], tuples, r["pairH"], diag)
    r.update(rows=rows, cols=cols, vals=vals)
    return r


def blocks_of(A):
    """dict (row, col) -> 3x3 from a device BsrMatrix"""
    rp = A.row_ptr().cpu().numpy()
    ci = A.col_idx().cpu().numpy()
    v = A.val[:, :A.nnzb].double().cpu().numpy().T.reshape(-1, 3, 3)
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    return {(int(r), int(c)): B for r, c, B in zip(rows, ci, v)}, rp, ci


def compare_scene(gpu, ref, V, tol=TOL):
    assert gpu["E"] == pytest.approx(ref["E"], rel=tol, abs=1e-300)
    gs = np.abs(ref["grad"]).max()
    assert np.abs(gpu["grad"] - ref["grad"]).max() <= tol * max(gs, 1e-300)
    gb, rp, ci = blocks_of(gpu["A"])
    # pattern sanity: sorted columns, a diagonal block in every row
    for r in range(V):
        cols = ci[rp[r]:rp[r + 1]]
        assert (np.diff(cols) > 0).all() and r in cols
    ob = {(int(r), int(c)): B for r, c, B in zip(ref["rows"], ref["cols"], ref["vals"])}
    hs = max(np.abs(B).max() for B in ob.values())
    keys = set(gb) | set(ob)
    worst = max(np.abs(gb.get(k, 0.0) - ob.get(k, 0.0)).max() for k in keys)
    assert worst <= tol * hs, worst / hs


def compare_pairs(gpu, ref, tuples, x, xr, tol=TOL, whole_list=True):
    """Per staged pair: energy, local gradient and Hessian, keyed by vertex id.
    A staged pair of multiplicity m stands for m candidates with the same
    reduced constraint: it is compared with m times the oracle's values for
    its first tuple, and over a whole list the multiplicities add up to the
    oracle's active candidates."""
    pr = gpu["pairs"]
    src, typ, vid = pr["src"], pr["type"], pr["vid"]
    mult = pr["mult"] if "mult" in pr else np.ones(len(src), np.int32)
    st = ref["subtype"]
    active_o = set(np.nonzero((st > 0) & (st != oracle.DEGENERATE))[0].tolist())
    active_g = set(src.tolist())
    assert len(active_g) == len(src)                      # each tuple staged at most once
    assert (mult >= 1).all()
    Emax = np.abs(ref["pairE"]).max() if len(ref["pairE"]) else 0.0

    def boundary(p):                                       # d within rounding of dhat
        return abs(ref["pairE"][p]) <= 1e-12 * max(Emax, 1e-300)
    for p in active_g - active_o:
        assert boundary(p)
    if whole_list:
        nb = sum(1 for p in active_o if boundary(p))
        assert abs(int(mult.sum()) - len(active_o)) <= nb
    gmax = np.abs(ref["pairG"]).max()
    hmax = np.abs(ref["pairH"]).max()
    for k in range(len(src)):
        p = int(src[k])
        m = float(mult[k])
        nv, ov = oracle.stencil(tuples[p])
        og = {int(ov[i]): m * ref["pairG"][p][3 * i:3 * i + 3] for i in range(nv)}
        gg = {int(vid[k][i]): pr["grad"][k][3 * i:3 * i + 3] for i in range(4) if vid[k][i] >= 0}
        sc_e = m * max(abs(ref["pairE"][p]), 1e-6 * Emax)
        assert abs(pr["energy"][k] - m * ref["pairE"][p]) <= tol * sc_e + 1e-300
        sc_g = m * max(np.abs(ref["pairG"][p]).max(), 1e-6 * gmax)
        for v in set(og) | set(gg):
            assert np.abs(gg.get(v, 0.0) - og.get(v, 0.0)).max() <= tol * sc_g + 1e-300, (k, p, v)
        oh = {}
        for i in range(nv):
            for j in range(nv):
                oh[(int(ov[i]), int(ov[j]))] = m * ref["pairH"][p][3 * i:3 * i + 3, 3 * j:3 * j + 3]
        gh = {}
        for i in range(4):
            for j in range(4):
                if vid[k][i] >= 0 and vid[k][j] >= 0:
                    gh[(int(vid[k][i]), int(vid[k][j]))] = pr["hess"][k][3 * i:3 * i + 3, 3 * j:3 * j + 3]
        sc_h = m * max(np.abs(ref["pairH"][p]).max(), 1e-6 * hmax)
        for key in set(oh) | set(gh):
            assert np.abs(gh.get(key, 0.0) - oh.get(key, 0.0)).max() <= tol * sc_h + 1e-300, (k, p, key)
        # mollified kinds <-> oracle's mollifier decision (exact, away from c = eps_x)
        if typ[k] >= 5 or ref["mollified"][p]:
            t = tuples[p]
            a = x[t[1] if t[1] >= 0 else -t[1] - 1] - x[t[0]]
            b = x[t[3]] - x[t[2]]
            ar = xr[t[1] if t[1] >= 0 else -t[1] - 1] - xr[t[0]]
            br = xr[t[3]] - xr[t[2]]
            ratio = np.sum(np.cross(a, b) ** 2) / (1e-3 * (ar @ ar) * (br @ br))
            if abs(ratio - 1) > 1e-9:
                assert (typ[k] >= 5) == bool(ref["mollified"][p])


# ----------------------------------------------------------------- scenes


def _tiny_scene(seed=3):
    return scenes.two_sheets(n=6, dhat=0.15, kappa=10.0, seed=seed, offset=0.5, jitter=0.3)


@pytest.mark.parametrize("opts", [dict(), dict(filter=False), dict(mollify=False), dict(eq12=True)])
def test_two_sheet_scene(gp, opts):
    s = scenes.two_sheets(n=16, seed=1)
    pg, po = _prm_pair(gp, s.dhat, s.kappa, **opts)
    diag = np.full(s.V, 10.0)
    gpu = run_gpu(gp, s.x, s.x_rest, s.tuples, pg, diag)
    ref = run_oracle(s.x, s.x_rest, s.tuples, po, diag)
    compare_scene(gpu, ref, s.V)
    compare_pairs(gpu, ref, s.tuples, s.x, s.x_rest)
    info = gpu["info"]
    assert info["n_candidates"] == s.P and info["n_degenerate"] == 0
    assert sum(info["n_by_type"].values()) == info["n_active"]
    assert sum(info["n_staged_by_type"].values()) == info["n_staged"] < info["n_active"]
    if opts.get("mollify", True):
        assert info["n_by_type"]["EE_moll"] + info["n_by_type"]["PE_moll"] + info["n_by_type"]["PP_moll"] > 0
    gpu["ctx"].close()


@pytest.mark.parametrize("which", ["two_sheets", "tiny"])
def test_merged_duplicates_equal_the_unmerged_list(gp, which):
    # reading of Eq. 3: the candidate list equals its merged list of reduced
    # constraints weighted by integer multiplicities
    s = scenes.two_sheets(n=16, seed=1) if which == "two_sheets" else _tiny_scene(4)
    pm, po = _prm_pair(gp, s.dhat, s.kappa)
    pn = gp.params(dhat=s.dhat, kappa=s.kappa, flags=gp.FLAGS_DEFAULT | gp.FLAG_NO_MERGE)
    diag = np.full(s.V, 10.0)
    a = run_gpu(gp, s.x, s.x_rest, s.tuples, pm, diag)
    b = run_gpu(gp, s.x, s.x_rest, s.tuples, pn, diag)
    assert b["info"]["n_staged"] == b["info"]["n_active"] == a["info"]["n_active"]
    assert a["info"]["n_staged"] < a["info"]["n_active"]
    assert int(a["pairs"]["mult"].sum()) == a["info"]["n_active"] and (b["pairs"]["mult"] == 1).all()
    assert a["E"] == pytest.approx(b["E"], rel=1e-13)
    assert np.abs(a["grad"] - b["grad"]).max() <= 1e-13 * np.abs(b["grad"]).max()
    ga, _, _ = blocks_of(a["A"])
    gb, _, _ = blocks_of(b["A"])
    assert ga.keys() == gb.keys()
    hs = max(np.abs(B).max() for B in gb.values())
    assert max(np.abs(ga[k] - gb[k]).max() for k in gb) <= 1e-13 * hs
    ref = run_oracle(s.x, s.x_rest, s.tuples, po, diag)
    compare_scene(b, ref, s.V)
    compare_pairs(b, ref, s.tuples, s.x, s.x_rest)
    a["ctx"].close(); b["ctx"].close()


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_tiny_dense_contact_scene(gp, seed):
    # large dhat relative to the mesh: every sub-type, many pairs per vertex,
    # ragged pair count
    s = _tiny_scene(seed)
    pg, po = _prm_pair(gp, s.dhat, s.kappa)
    t = s.tuples[: s.P - 3]
    gpu = run_gpu(gp, s.x, s.x_rest, t, pg, np.linspace(1, 2, s.V))
    ref = run_oracle(s.x, s.x_rest, t, po, np.linspace(1, 2, s.V))
    compare_scene(gpu, ref, s.V)
    compare_pairs(gpu, ref, t, s.x, s.x_rest)
    gpu["ctx"].close()


def test_mollified_pair_with_scale_separated_inner_block(gp):
    # Edge pair taken from the 10-sheet scene (seed 2): nearly parallel edges
    # meeting at a point-point sub-case.  Its inner 2x2 block is about
    # [[-241, -1.2e-4], [-1.2e-4, 6.1e-10]]: the positive eigenvalue is tiny in
    # J-space yet dominates the x-space Hessian (grad f ~ 1/dhat), so it must
    # be formed without cancellation.
    x = np.array([[9.6078431372549022e-01, 7.7647058823529413e-01, 7.1354464226378522e-04],
                  [9.6078431372549022e-01, 7.8039215686274510e-01, 4.8911326628829979e-04],
                  [9.6078431372549022e-01, 7.7254901960784317e-01, 1.0145321285709062e-03],
                  [9.6078431372549022e-01, 7.7647058823529413e-01, 9.0001536707776629e-04]])
    xr = np.array([[9.607843137254902e-01, 7.764705882352941e-01, 5.999999999999999e-04],
                   [9.607843137254902e-01, 7.803921568627451e-01, 5.999999999999999e-04],
                   [9.607843137254902e-01, 7.725490196078432e-01, 1.200000000000000e-03],
                   [9.607843137254902e-01, 7.764705882352941e-01, 1.200000000000000e-03]])
    t = np.array([[0, 1, 2, 3]], np.int32)
    pg, po = _prm_pair(gp, 1e-3, 1e4)
    gpu = run_gpu(gp, x, xr, t, pg, np.full(4, 10.0))
    ref = run_oracle(x, xr, t, po, np.full(4, 10.0))
    assert ref["mollified"][0] and gpu["pairs"]["type"][0] == 7
    compare_scene(gpu, ref, 4)
    compare_pairs(gpu, ref, t, x, xr)
    gpu["ctx"].close()


def test_rounding_level_parallel_edges(gp):
    # Facing diagonals of a cube lattice: |a x b| = 4.9e-32 for the rounded
    # coordinates while the plain product formula gives 0.  The mollifier
    # term along grad sqrt(c) carries the whole proxy Hessian, so both sides
    # must take c from the input alone.
    x = np.array([[1.7779462971114925, 1.0, 1.1118521306832763],
                  [1.8890574082226037, 1.0, 1.2229632417943872],
                  [1.8890574082226037, 1.000289448405277, 1.2229632417943872],
                  [2.000168519333715, 1.000289448405277, 1.3340743529054984]])
    t = np.array([[0, 1, 2, 3], [1, 0, 3, 2]], np.int32)
    pg, po = _prm_pair(gp, 1e-3, 1e4)
    gpu = run_gpu(gp, x, x, t, pg, np.full(4, 10.0))
    ref = run_oracle(x, x, t, po, np.full(4, 10.0))
    assert ref["mollified"].all() and (gpu["pairs"]["type"] == 7).all()
    assert np.abs(ref["pairH"]).max() > 0
    compare_scene(gpu, ref, 4)
    compare_pairs(gpu, ref, t, x, x)
    gpu["ctx"].close()


def test_typed_point_edge_and_point_point_tuples(gp):
    rng = np.random.default_rng(11)
    V = 40
    x = rng.uniform(0, 0.2, size=(V, 3))
    tuples = []
    for _ in range(300):
        a, b, c = rng.choice(V, 3, replace=False)
        tuples.append([-(a + 1), b, c, -1] if rng.random() < 0.5 else [-(a + 1), b, -1, -1])
    tuples = np.array(tuples, np.int32)
    pg, po = _prm_pair(gp, 0.1, 5.0)
    gpu = run_gpu(gp, x, x, tuples, pg)
    ref = run_oracle(x, x, tuples, po)
    compare_scene(gpu, ref, V)
    compare_pairs(gpu, ref, tuples, x, x)
    gpu["ctx"].close()


# -------------------------------------------------------------- edge cases


def test_empty_pair_list(gp):
    s = scenes.two_sheets(n=4, seed=1, with_pairs=False)
    pg, _ = _prm_pair(gp, s.dhat, s.kappa)
    gpu = run_gpu(gp, s.x, s.x_rest, np.zeros((0, 4), np.int32), pg, np.full(s.V, 2.0), inspect=False)
    assert gpu["E"] == 0.0 and not gpu["grad"].any()
    assert gpu["info"]["n_active"] == 0 and gpu["A"].nnzb == s.V
    d = gpu["A"].to_scipy().toarray()
    assert np.array_equal(d, 2.0 * np.eye(3 * s.V))
    gpu["ctx"].close()


def test_all_candidates_inactive(gp):
    s = scenes.two_sheets(n=8, seed=1, offset=3.0, jitter=0.0, with_pairs=False)
    t = scenes.broadphase(s.x, s.vobj, s.tris, s.edges, 4 * s.dhat)   # candidates farther than dhat
    assert len(t) > 0
    pg, _ = _prm_pair(gp, s.dhat, s.kappa)
    gpu = run_gpu(gp, s.x, s.x_rest, t, pg, inspect=False)
    assert gpu["info"]["n_active"] == 0 and gpu["E"] == 0.0 and not gpu["grad"].any()
    gpu["ctx"].close()


@pytest.mark.parametrize("bad", [[0, 1, 2, 10 ** 6], [-1, 1, -1, 3], [0, 1, -1, 3], [-3, 1, 2, 2], [5, 5, 1, 2]])
def test_malformed_tuples_raise_index_error(gp, bad):
    s = _tiny_scene()
    t = s.tuples.copy()
    t[7] = bad
    pg, _ = _prm_pair(gp, s.dhat, s.kappa)
    with pytest.raises(gp.GipcError) as ei:
        run_gpu(gp, s.x, s.x_rest, t, pg, inspect=False)
    assert ei.value.status == gp.ERR_INDEX and "first at 7" in str(ei.value)


def test_degenerate_pair_is_counted_and_skipped(gp):
    # a point lying exactly on a triangle (d = 0) and a regular pair
    x = np.array([[0.2, 0.2, 0.0], [0, 0, 0], [1, 0, 0], [0, 1, 0], [0.3, 0.3, 0.05]], float)
    t = np.array([[-1, 1, 2, 3], [-5, 1, 2, 3]], np.int32)
    pg, po = _prm_pair(gp, 0.1, 1.0)
    gpu = run_gpu(gp, x, x, t, pg)
    assert gpu["info"]["n_degenerate"] == 1 and gpu["info"]["first_degenerate"] == 0
    assert gpu["info"]["n_active"] == 1
    ref = run_oracle(x, x, t, po)
    assert ref["n_degenerate"] == 1
    compare_scene(gpu, ref, 5)
    gpu["ctx"].close()


def test_call_order_and_argument_errors(gp):
    s = _tiny_scene()
    dev = torch.device("cuda", 0)
    ctx = gp.Context()
    pg, _ = _prm_pair(gp, s.dhat, s.kappa)
    X = torch.tensor(s.x, device=dev)
    with pytest.raises(gp.GipcError) as ei:
        gp.barrier_eval(ctx, X, pg)
    assert ei.value.status == gp.ERR_STATE
    bad = gp.params(dhat=-1.0)
    with pytest.raises(gp.GipcError) as ei:
        gp.pairs_build(ctx, X, torch.tensor(s.tuples, device=dev), bad)
    assert ei.value.status == gp.ERR_INVALID_ARG
    ctx.close()


# --------------------------------------------------- precision, SpMV, PCG


def test_fp32_blocks_and_spmv(gp):
    s = scenes.two_sheets(n=16, seed=1)
    pg, _ = _prm_pair(gp, s.dhat, s.kappa)
    diag = np.full(s.V, 10.0)
    g64 = run_gpu(gp, s.x, s.x_rest, s.tuples, pg, diag, dtype=gp.F64, inspect=False)
    g32 = run_gpu(gp, s.x, s.x_rest, s.tuples, pg, diag, dtype=gp.F32, inspect=False)
    b64, _, _ = blocks_of(g64["A"])
    b32, _, _ = blocks_of(g32["A"])
    assert set(b64) == set(b32)
    for k, B in b64.items():
        n = np.linalg.norm(B)
        if n > 0:
            assert np.linalg.norm(b32[k] - B) <= 1e-5 * n
    xv = torch.randn(s.V, 3, dtype=torch.float64, device="cuda")
    y64 = gp.bsr_spmv(g64["A"], xv).cpu().numpy()
    y32 = gp.bsr_spmv(g32["A"], xv.float()).double().cpu().numpy()
    assert np.abs(y32 - y64).max() <= 1e-5 * np.abs(y64).max()
    g64["ctx"].close(); g32["ctx"].close()


def test_fp32_pcg_against_fp64(gp):
    # FP32 blocks and FP32 SpMV; FP64 vectors, dots and preconditioner
    s = scenes.two_sheets(n=16, seed=1)
    pg, _ = _prm_pair(gp, s.dhat, s.kappa)
    diag = np.full(s.V, 10.0)
    g64 = run_gpu(gp, s.x, s.x_rest, s.tuples, pg, diag, dtype=gp.F64, inspect=False)
    g32 = run_gpu(gp, s.x, s.x_rest, s.tuples, pg, diag, dtype=gp.F32, inspect=False)
    b = torch.tensor(-g64["grad"], device="cuda")
    x64, it64, rr64, st64 = gp.pcg(g64["ctx"], g64["A"], b, rtol=1e-6, maxit=1000)
    x32, it32, rr32, st32 = gp.pcg(g32["ctx"], g32["A"], b, rtol=1e-6, maxit=1000)
    assert st64 == st32 == gp.OK and rr32 <= 1e-6
    assert abs(it32 - it64) <= 2
    # residual of the FP32 solution measured with the FP64 matrix
    r = b - gp.bsr_spmv(g64["A"], x32)
    assert float(torch.linalg.norm(r) / torch.linalg.norm(b)) <= 1e-5
    assert float(torch.linalg.norm(x32 - x64) / torch.linalg.norm(x64)) <= 1e-4
    # fixed iteration count with rtol = 0 on an FP32 matrix
    _, it, _, st = gp.pcg(g32["ctx"], g32["A"], b, rtol=0.0, maxit=7)
    assert it == 7 and st == gp.OK
    g64["ctx"].close(); g32["ctx"].close()


def test_spmv_matches_oracle(gp):
    s = _tiny_scene()
    pg, po = _prm_pair(gp, s.dhat, s.kappa)
    diag = np.linspace(1, 3, s.V)
    gpu = run_gpu(gp, s.x, s.x_rest, s.tuples, pg, diag, inspect=False)
    ref = run_oracle(s.x, s.x_rest, s.tuples, po, diag)
    xv = np.random.default_rng(0).normal(size=(s.V, 3))
    y = gp.bsr_spmv(gpu["A"], torch.tensor(xv, device="cuda")).cpu().numpy().reshape(-1)
    yo = oracle.spmv(s.V, ref["rows"], ref["cols"], ref["vals"], xv)
    assert np.abs(y - yo).max() <= 1e-12 * np.abs(yo).max()
    gpu["ctx"].close()


def test_pcg_matches_oracle_and_direct_solve(gp):
    s = scenes.two_sheets(n=16, seed=1)
    pg, po = _prm_pair(gp, s.dhat, s.kappa)
    diag = np.full(s.V, 10.0)
    gpu = run_gpu(gp, s.x, s.x_rest, s.tuples, pg, diag, inspect=False)
    ref = run_oracle(s.x, s.x_rest, s.tuples, po, diag)
    b = -ref["grad"].reshape(-1)
    bt = torch.tensor(-gpu["grad"], device="cuda")
    # a fixed number of iterations follows the oracle's iterates
    x10, it, rr, st = gp.pcg(gpu["ctx"], gpu["A"], bt, rtol=0.0, maxit=10)
    xo, ito, rro = oracle.pcg(s.V, ref["rows"], ref["cols"], ref["vals"], b, rtol=0.0, maxit=10)
    assert it == ito == 10 and st == gp.OK
    assert np.linalg.norm(x10.cpu().numpy().reshape(-1) - xo) <= 1e-8 * np.linalg.norm(xo)
    # to a tolerance: same iteration count, solution of the linear system
    xs, it, rr, st = gp.pcg(gpu["ctx"], gpu["A"], bt, rtol=1e-6, maxit=500)
    xo, ito, rro = oracle.pcg(s.V, ref["rows"], ref["cols"], ref["vals"], b, rtol=1e-6, maxit=500)
    assert st == gp.OK and rr <= 1e-6 and abs(it - ito) <= 1
    xs, it, rr, st = gp.pcg(gpu["ctx"], gpu["A"], bt, rtol=1e-11, maxit=2000)
    G = gpu["A"].to_scipy().toarray()
    ref_x = np.linalg.solve(G, b)
    assert np.linalg.norm(xs.cpu().numpy().reshape(-1) - ref_x) <= 1e-8 * np.linalg.norm(ref_x)
    # warm start at the solution: zero iterations
    x0 = torch.tensor(ref_x.reshape(-1, 3), device="cuda")
    _, it0, _, _ = gp.pcg(gpu["ctx"], gpu["A"], bt, x=x0, rtol=1e-6, maxit=10)
    assert it0 == 0
    # not converged within maxit -> warning status, not an error
    _, it1, rr1, st1 = gp.pcg(gpu["ctx"], gpu["A"], bt, rtol=1e-14, maxit=3)
    assert it1 == 3 and st1 == gp.WARN_NOT_CONVERGED
    gpu["ctx"].close()


def test_pcg_reports_breakdown_on_indefinite_matrix(gp):
    s = _tiny_scene()
    pg, _ = _prm_pair(gp, s.dhat, s.kappa)
    gpu = run_gpu(gp, s.x, s.x_rest, s.tuples, pg, np.full(s.V, -5.0), inspect=False)
    bt = torch.ones(s.V, 3, dtype=torch.float64, device="cuda")
    with pytest.raises(gp.GipcError) as ei:
        gp.pcg(gpu["ctx"], gpu["A"], bt, rtol=1e-8, maxit=50)
    assert ei.value.status == gp.ERR_BREAKDOWN
    gpu["ctx"].close()


def test_bsr_is_exactly_symmetric(gp):
    # every block above the diagonal is stored with its transpose below
    s = scenes.two_sheets(n=16, seed=1)
    pg, _ = _prm_pair(gp, s.dhat, s.kappa)
    for dtype in (gp.F64, gp.F32):
        g = run_gpu(gp, s.x, s.x_rest, s.tuples, pg, np.full(s.V, 10.0), dtype=dtype, inspect=False)
        blocks, _, _ = blocks_of(g["A"])
        for (r, c), B in blocks.items():
            assert np.array_equal(B, blocks[(c, r)].T), (r, c)
        g["ctx"].close()


def test_deterministic_bitwise(gp):
    s = scenes.two_sheets(n=16, seed=1)
    pg, _ = _prm_pair(gp, s.dhat, s.kappa)
    diag = np.full(s.V, 10.0)
    a = run_gpu(gp, s.x, s.x_rest, s.tuples, pg, diag, inspect=False)
    b = run_gpu(gp, s.x, s.x_rest, s.tuples, pg, diag, inspect=False)
    assert a["E"] == b["E"]
    assert np.array_equal(a["grad"], b["grad"])
    assert torch.equal(a["A"].val, b["A"].val)
    assert torch.equal(a["A"].col_idx(), b["A"].col_idx())
    a["ctx"].close(); b["ctx"].close()


# ------------------------------------------------------------ full scale


@pytest.fixture(scope="module")
def big(gp):
    s = scenes.stacked_sheets(n_sheets=10, n=256, seed=2)
    pg, po = _prm_pair(gp, s.dhat, s.kappa)
    gpu = run_gpu(gp, s.x, s.x_rest, s.tuples, pg, s.diag, inspect=False)
    yield s, pg, po, gpu
    gpu["ctx"].close()


def test_full_scale_energy_and_gradient(big):
    s, pg, po, gpu = big
    ref = oracle.eval_scene(s.x, s.tuples, po, x_rest=s.x_rest)
    assert gpu["E"] == pytest.approx(ref["E"], rel=TOL)
    assert np.abs(gpu["grad"] - ref["grad"]).max() <= TOL * np.abs(ref["grad"]).max()
    act = (ref["subtype"] > 0) & (ref["subtype"] != oracle.DEGENERATE)
    assert abs(gpu["info"]["n_active"] - int(act.sum())) <= 1e-6 * act.sum()


def test_full_scale_sampled_rows(big, gp):
    s, pg, po, gpu = big
    rng = np.random.default_rng(5)
    rows = rng.choice(s.V, 40, replace=False)
    kind, st = scenes.decode_tuples(s.tuples)
    touch = np.isin(st, rows).any(1)
    sub = s.tuples[touch]
    ref = run_oracle(s.x, s.x_rest, sub, po, s.diag)
    A = gpu["A"]
    rp = A.row_ptr().cpu().numpy()
    ci_all = A.col_idx()
    for r in rows:
        lo, hi = int(rp[r]), int(rp[r + 1])
        ci = ci_all[lo:hi].cpu().numpy()
        vals = A.val[:, lo:hi].cpu().numpy().T.reshape(-1, 3, 3)
        g = {int(c): B for c, B in zip(ci, vals)}
        sel = ref["rows"] == r
        o = {int(c): B for c, B in zip(ref["cols"][sel], ref["vals"][sel])}
        hs = max(np.abs(B).max() for B in o.values())
        for c in set(g) | set(o):
            assert np.abs(g.get(c, 0.0) - o.get(c, 0.0)).max() <= TOL * hs, (r, c)


def test_full_scale_sampled_pairs(big, gp):
    s, pg, po, gpu = big
    pi = gp.pair_inspect(gpu["ctx"], gpu["X"], pg, x_rest=gpu["XR"],
                         want=("src", "type", "vid", "mult", "energy", "grad", "hess"))
    n = pi["src"].shape[0]
    rng = np.random.default_rng(9)
    pick = np.sort(rng.choice(n, min(n, 4000), replace=False))
    idx = torch.tensor(pick, device="cuda")
    pairs = {k: v[idx].cpu().numpy() for k, v in pi.items()}
    src = pairs["src"]
    ref = oracle.eval_scene(s.x, s.tuples[src], po, x_rest=s.x_rest, per_pair=True)
    pairs["src"] = np.arange(len(src))
    compare_pairs(dict(pairs=pairs), ref, s.tuples[src], s.x, s.x_rest, whole_list=False)
