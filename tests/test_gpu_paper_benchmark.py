"""The paper's strong-scaling benchmark shape (Sec. 8 and Sec. 6.3: 11
Gaussian bunches of 1e6 particles, sigma 1.5 / 5 / 5 mm, 4 cm apart, two
refined levels on the computation cube, homogeneous Dirichlet) at its real
particle count, in the launch configuration the bench times (mixed cycle,
brick Gauss-Seidel, deposit from the build's ordered copy, gather from it),
on a 288^3 base: the multigrid continues below level 0 on two geometric
levels (144^3, 72^3) before the direct solve.  Then one step of the
benchmark's particle motion on the kept hierarchy (amrmg_deposit of the
jittered particles, solve, E, amrmg_gather), checked the same way.

The oracle's full solve would take hours at this size, so the checks are
the ones that hold at any size and that the oracle evaluates in one pass:

  * box lists bit for bit (the oracle's own tagging and clustering);
  * the deposit element by element (<= 1e-12 relative per level);
  * the oracle's FP64 composite residual (Alg. 1) of the GPU's phi on every
    level at most the tolerance;
  * E against the oracle's -grad of the GPU's phi, and the gather against
    the oracle's interpolation of the GPU's E (round-off)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1812_03689_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def check_against_oracle(H, ctx, p, rho, phi, E, Exyz, tol, label):
    from paper_1812_03689_amd import amrmg as A  # noqa: F401
    nl = H.nlev
    orho = H.deposit_all(p)
    for l in range(nl):
        g = rho[l].cpu().numpy()
        err = np.linalg.norm(g - orho[l]) / np.linalg.norm(orho[l])
        assert err <= 1e-12, (label, "deposit", l, err)
    gphi = [t.cpu().numpy() for t in phi]
    r = H.residual(orho, gphi)
    b = H.residual(orho, H.zeros())
    rel = [float(np.linalg.norm(r[l]) / np.linalg.norm(b[l])) for l in range(nl)]
    print("  ", label, "oracle residual of the GPU phi", rel, flush=True)
    assert max(rel) <= 1.01 * tol, (label, rel)
    del r, b
    oE = H.efield(gphi)
    gE = [t.cpu().numpy() for t in E]
    for i, (g, o) in enumerate(zip(gE, oE)):
        assert np.abs(g - o).max() <= 1e-11 * np.abs(o).max(), (label, "E", i)
    del oE
    og = H.gather(p, gE)
    for d, (g, o) in enumerate(zip(Exyz, og)):
        assert np.abs(g.cpu().numpy() - o).max() <= 1e-12 * np.abs(o).max(), (label, "gather", d)


@pytest.mark.parametrize("n0", [288])
def test_paper_benchmark_shape(n0):
    from paper_1812_03689_amd import amrmg as A
    print("case chain11", n0, flush=True)
    w = W.config6(n0=n0)
    p = w.particles
    prm = A.make_params(w.n0, max_level=w.max_level, monopoles=w.monopoles, precision="mixed",
                        max_grid_size=w.max_grid_size, lo=w.lo, hi=w.hi)
    ctx = A.Context(prm)
    x, y, z, q = (torch.as_tensor(a, device="cuda") for a in (p.x, p.y, p.z, p.q))
    info = ctx.build_hierarchy(x, y, z, q, tag_rel=w.tag_rel)
    print("  ", info, flush=True)
    assert info["nlevels"] == 3
    rho, nout = ctx.deposit_built()
    assert nout == 0
    phi, E, st = ctx.solve(rho, tol=w.tol)
    print("  ", {k: st[k] for k in ("iters", "converged", "rel_residual", "dof")}, flush=True)
    assert st["converged"]
    Exyz = ctx.gather_built(E)
    torch.cuda.synchronize()

    H = O.hierarchy_from_workload(w)
    assert H.nlev == info["nlevels"]
    for l in range(H.nlev):
        gb, go = ctx.boxes(l)
        ob, oo = H.boxes(l)
        assert np.array_equal(gb, ob), l
        assert np.array_equal(go, oo), l
    check_against_oracle(H, ctx, p, rho, phi, E, Exyz, w.tol, "built")

    # one step of the benchmark's motion on the kept hierarchy
    gen = torch.Generator(device="cuda")
    gen.manual_seed(W.seed_for(6, 9))
    xj, yj, zj = W.jitter(x, y, z, w.lo, w.hi, 1e-3, gen)
    pj = W.Particles(xj.cpu().numpy(), yj.cpu().numpy(), zj.cpu().numpy(), p.q)
    nout_ref = int(np.sum(~((pj.x >= w.lo[0]) & (pj.x < w.hi[0]) & (pj.y >= w.lo[1]) & (pj.y < w.hi[1])
                            & (pj.z >= w.lo[2]) & (pj.z < w.hi[2]))))
    rho2, nout2 = ctx.deposit(xj, yj, zj, q)
    assert nout2 == nout_ref
    phi2, E2, st2 = ctx.solve(rho2, tol=w.tol)
    print("   jittered", {k: st2[k] for k in ("iters", "converged", "rel_residual")}, flush=True)
    assert st2["converged"]
    Exyz2 = ctx.gather(xj, yj, zj, E2)
    torch.cuda.synchronize()
    check_against_oracle(H, ctx, pj, rho2, phi2, E2, Exyz2, w.tol, "jittered")
