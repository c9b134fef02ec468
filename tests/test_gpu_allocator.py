"""A context whose buffers come from the caller's allocator (torch's caching
allocator through gipc_ctx_create_with_allocator): the same bits as a
context on hipMalloc, its memory counted by torch while it lives and handed
back when it is destroyed; growing buffers across builds of different
sizes; a callback that fails turns into WORKSPACE."""
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


def _run(gp, ctx, s):
    dev = torch.device("cuda", 0)
    prm = gp.params(dhat=s.dhat, kappa=s.kappa)
    x = torch.tensor(s.x, device=dev)
    xr = torch.tensor(s.x_rest, device=dev)
    gp.pairs_build(ctx, x, torch.tensor(s.tuples, device=dev), prm, x_rest=xr)
    A = gp.BsrMatrix(ctx)
    diag = torch.full((s.V,), 10.0, dtype=torch.float64, device=dev)
    E, g = gp.eval_assemble(ctx, x, prm, A, diag=diag, x_rest=xr)
    d, it, rr, st = gp.pcg(ctx, A, -g, rtol=0.0, maxit=20)
    torch.cuda.synchronize()
    return E.clone(), g.clone(), A.val[:, :A.nnzb].clone(), d.clone()


def test_torch_allocator_same_bits(gp):
    small = scenes.two_sheets(n=9, dhat=0.2, kappa=10.0, seed=4, offset=0.5, jitter=0.3)
    big = scenes.two_sheets(n=16, seed=1)
    base = gp.Context()
    before = torch.cuda.memory_allocated()
    tc = gp.Context(allocator="torch")
    assert torch.cuda.memory_allocated() > before  # the counters block
    for s in (small, big, small):  # buffers grow, then are reused
        ref = _run(gp, base, s)
        got = _run(gp, tc, s)
        for a, b in zip(ref, got):
            assert torch.equal(a, b)
    held = torch.cuda.memory_allocated()
    tc.close()
    assert torch.cuda.memory_allocated() < held
    base.close()


def test_failing_allocator_is_workspace(gp):
    calls = {"n": 0}

    def alloc(user, nbytes, device):
        calls["n"] += 1
        return None if calls["n"] > 1 else torch.cuda.caching_allocator_alloc(int(nbytes), device=int(device),
                                                                              stream=0)

    def free(user, ptr, nbytes, device):
        torch.cuda.caching_allocator_delete(int(ptr))

    al = gp.Allocator(gp._ALLOC_FN(alloc), gp._FREE_FN(free), None)
    h = ctypes.c_void_p()
    assert gp.lib().gipc_ctx_create_with_allocator(ctypes.byref(al), ctypes.byref(h)) == gp.OK
    ctx = gp.Context.__new__(gp.Context)
    ctx.h, ctx.V, ctx.info, ctx._alloc = h, 0, None, al
    s = scenes.two_sheets(n=16, seed=1)
    x = torch.tensor(s.x, device="cuda")
    with pytest.raises(gp.GipcError) as e:
        gp.pairs_build(ctx, x, torch.tensor(s.tuples, device="cuda"), gp.params(dhat=s.dhat, kappa=s.kappa))
    assert e.value.status == gp.ERR_WORKSPACE
    ctx.close()
    bad = gp.Allocator(gp._ALLOC_FN(alloc), ctypes.cast(None, gp._FREE_FN), None)
    assert gp.lib().gipc_ctx_create_with_allocator(ctypes.byref(bad), ctypes.byref(h)) == gp.ERR_INVALID_ARG
    assert np.isfinite(calls["n"])
