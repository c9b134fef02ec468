"""Differentiation extension on the cube lattice (6 x 6 x 6 unit cubes of
10^3 vertices, per-plane gaps uniform in (0.1, 0.9) dhat, dhat = 1e-3,
kappa = 1e4): the barrier energy as a torch.autograd.Function whose backward
returns the gradient kernel's output, and the Hessian-vector product through
the assembled proxy Hessian and the BSR SpMV.

* gradient vs the oracle gradient: 1e-9 relative (max norm);
* gradient vs central finite differences of the energy, h = 1e-7 along 64
  unit random directions: per-pair energy differences (GPU, at x +- h v) are
  summed with math.fsum, to 1e-6 relative;
* HVP vs the oracle's proxy Hessian times v on sampled rows: 1e-9 of the
  largest entry.  (The proxy is not the exact Hessian, so the HVP is not
  checked against differences of the gradient.)
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import scenes  # noqa: E402


@pytest.fixture(scope="module")
def lattice():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2308_09400_amd as gp
    torch.cuda.set_device(0)
    s = scenes.cube_lattice(m=6, n=10, seed=3)
    dev = torch.device("cuda", 0)
    prm = gp.params(dhat=s.dhat, kappa=s.kappa)
    X = torch.tensor(s.x, device=dev)
    T = torch.tensor(s.tuples, device=dev)
    ctx = gp.Context()
    info = gp.pairs_build(ctx, X, T, prm)
    yield gp, s, prm, X, ctx, info
    ctx.close()


def test_autograd_gradient_matches_oracle(lattice):
    gp, s, prm, X, ctx, info = lattice
    x = X.clone().requires_grad_(True)
    E = gp.barrier_energy(x, ctx, prm)
    E.backward()
    ref = oracle.eval_scene(s.x, s.tuples, oracle.params(dhat=s.dhat, kappa=s.kappa))
    assert E.item() == pytest.approx(ref["E"], rel=1e-9)
    g = x.grad.cpu().numpy()
    assert np.abs(g - ref["grad"]).max() <= 1e-9 * np.abs(ref["grad"]).max()
    # the lattice has exactly parallel facing edges (c = 0): they are staged
    # as mollified pairs and contribute nothing
    assert info["n_active"] > 0 and ref["n_degenerate"] == 0


def test_gradient_vs_central_differences(lattice):
    gp, s, prm, X, ctx, info = lattice
    x = X.clone().requires_grad_(True)
    gp.barrier_energy(x, ctx, prm).backward()
    g = x.grad
    rng = np.random.default_rng(64)
    h = 1e-7
    for trial in range(64):
        v = torch.tensor(rng.normal(size=s.x.shape), device=X.device)
        v /= torch.linalg.norm(v)
        ep = gp.pair_inspect(ctx, (X + h * v).contiguous(), prm, want=("energy",))["energy"].cpu().numpy()
        em = gp.pair_inspect(ctx, (X - h * v).contiguous(), prm, want=("energy",))["energy"].cpu().numpy()
        fd = math.fsum((ep - em).tolist()) / (2 * h)
        an = math.fsum((g * v).reshape(-1).cpu().numpy().tolist())
        assert fd == pytest.approx(an, rel=1e-6, abs=1e-6 * float(torch.linalg.norm(g))), trial


def test_hvp_matches_oracle_proxy_hessian(lattice):
    gp, s, prm, X, ctx, info = lattice
    rng = np.random.default_rng(7)
    v = rng.normal(size=s.x.shape)
    Hv, A = gp.hvp(ctx, X, prm, torch.tensor(v, device=X.device))
    Hv = Hv.cpu().numpy()
    # rows touching active pairs
    kind, st = scenes.decode_tuples(s.tuples)
    rows = rng.choice(np.unique(st[:, :2].ravel()), 30, replace=False)
    touch = np.isin(st, rows).any(1)
    sub = s.tuples[touch]
    r = oracle.eval_scene(s.x, sub, oracle.params(dhat=s.dhat, kappa=s.kappa), per_pair=True)
    orows, ocols, ovals = oracle.assemble(s.V, sub, r["pairH"])
    for row in rows:
        sel = orows == row
        ref = np.zeros(3)
        for c, B in zip(ocols[sel], ovals[sel]):
            ref += B @ v[c]
        scale = max(np.abs(ovals[sel]).max() * np.abs(v).max(), 1e-300)
        assert np.abs(Hv[row] - ref).max() <= 1e-9 * scale, row
