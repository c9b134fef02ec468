"""gipc_pcg_static (the PCG on the library's fixed work area, no device
allocation) against gipc_pcg on the same matrix and right-hand side.

Both run the same kernels in the same order, so the solutions agree to
rounding (checked to 1e-12 of the largest entry, iterations and residuals
equal).  Two calls in a row, the second on a smaller system, show that the
area keeps no state that the next call reads; FP32 blocks and a converging
solve (rtol > 0) run as well; a system beyond the area's capacity returns
WORKSPACE before anything is launched.  With rtol = 0 and no counts the
call only enqueues: recorded in a HIP graph and replayed three times, with
eager work and synchronisations in between, every replay gives gipc_pcg's
solution.
"""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import scenes  # noqa: E402


@pytest.fixture(scope="module")
def gp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2308_09400_amd as gp
    torch.cuda.set_device(0)
    return gp


def _system(gp, n, seed, dtype):
    s = scenes.two_sheets(n=n, seed=seed)
    dev = torch.device("cuda", 0)
    prm = gp.params(dhat=s.dhat, kappa=s.kappa)
    x = torch.tensor(s.x, device=dev)
    xr = torch.tensor(s.x_rest, device=dev)
    ctx = gp.Context()
    gp.pairs_build(ctx, x, torch.tensor(s.tuples, device=dev), prm, x_rest=xr)
    A = gp.BsrMatrix(ctx, dtype=dtype)
    diag = torch.full((s.V,), 10.0, dtype=torch.float64, device=dev)
    _, g = gp.eval_assemble(ctx, x, prm, A, diag=diag, x_rest=xr)
    return ctx, A, -g


def _compare(gp, ctx, A, b, rtol, maxit):
    x_ref, it_ref, rr_ref, st_ref = gp.pcg(ctx, A, b, rtol=rtol, maxit=maxit)
    xs, it, rr, st = gp.pcg_static(A, b, rtol=rtol, maxit=maxit)
    torch.cuda.synchronize()
    err = float((xs - x_ref).abs().max() / x_ref.abs().max())
    print(f"pcg_static V={A.nbrows} nnzb={A.nnzb} dtype={A.dtype} rtol={rtol}: iters {it} vs {it_ref}, "
          f"relres {rr:.3e} vs {rr_ref:.3e}, max rel diff {err:.2e}", flush=True)
    assert st == st_ref
    assert it == it_ref
    assert err <= 1e-12
    assert abs(rr - rr_ref) <= 1e-12 * max(rr_ref, 1e-300)


@pytest.mark.parametrize("dtype", [0, 1])
def test_two_calls_second_smaller(gp, dtype):
    big = _system(gp, 16, 1, dtype)
    small = _system(gp, 9, 4, dtype)
    assert small[1].nbrows < big[1].nbrows
    _compare(gp, big[0], big[1], big[2], 0.0, 25)
    _compare(gp, small[0], small[1], small[2], 0.0, 25)
    # and back to the larger one with a converging solve
    _compare(gp, big[0], big[1], big[2], 1e-8, 500)
    for c in (big[0], small[0]):
        c.close()


def test_capacity_rejected_before_launch(gp):
    ctx, A, b = _system(gp, 9, 4, 0)
    d = gp.Bsr.from_buffer_copy(A.desc)
    d.nbrows = 1 << 22  # beyond the fixed area: rejected on the host
    it = ctypes.c_int32(-1)
    st = gp.lib().gipc_pcg_static(ctypes.byref(d), ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                                  0.0, 5, ctypes.byref(it), None, None)
    assert st == gp.ERR_WORKSPACE
    assert it.value == -1
    # the area still works afterwards
    _compare(gp, ctx, A, b, 0.0, 10)
    ctx.close()


def test_recorded_in_a_graph(gp):
    ctx, A, b = _system(gp, 16, 1, 0)
    x_ref, it_ref, _, _ = gp.pcg(ctx, A, b, rtol=0.0, maxit=20)
    xbuf = torch.zeros_like(b)
    gp.pcg_static(A, b, x=xbuf, rtol=0.0, maxit=20, counts=False)  # eager once (device set-up)
    torch.cuda.synchronize()
    assert torch.equal(xbuf, x_ref)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            xbuf.zero_()
            gp.pcg_static(A, b, x=xbuf, rtol=0.0, maxit=20, counts=False)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        xbuf.fill_(float(rep + 1))  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        err = float((xbuf - x_ref).abs().max() / x_ref.abs().max())
        print(f"graph replay {rep}: max rel diff {err:.2e}", flush=True)
        assert err <= 1e-12
    del g
    ctx.close()
