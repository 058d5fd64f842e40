"""Parity at the full sizes the bench times (1e6 Gaussian particles on 64^3 +
2 levels; nine bunches of 1e6 on 128^3 + 2; 1e7 FP32-position particles on
128^3 + 3), in the bench's launch configuration (mixed precision, brick
Gauss-Seidel, deposit from the build's ordered copy, solve from zero to
1e-8, E, gather).  The oracle's full solve would take minutes here, so the
checks are those that hold at any size and that the oracle evaluates in one
pass each:

  * box lists bit for bit (the oracle's own tagging and clustering);
  * the deposit, element by element, against the oracle's deposit;
  * the oracle's FP64 composite residual (Alg. 1) of the GPU's phi, per
    level relative to the right-hand side: at most the tolerance;
  * E against the oracle's E = -grad of the GPU's phi, and the gather against
    the oracle's interpolation of the GPU's E (both one pass of the same
    data, so to round-off); the gather from the build's ordered copy (the
    bench's) equal to it bit for bit."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1812_03689_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = {"gauss_64c_2lev": W.config2, "arc9_128c_2lev": W.config4, "gauss_128c_3lev_f32pos": W.config3}


@pytest.mark.parametrize("case", list(CASES))
def test_full_size_properties(case):
    from paper_1812_03689_amd import amrmg as A
    print("case", case, flush=True)
    w = CASES[case]()
    p = w.particles
    prm = A.make_params(w.n0, max_level=w.max_level, monopoles=w.monopoles, precision="mixed",
                        max_grid_size=w.max_grid_size, lo=w.lo, hi=w.hi)
    ctx = A.Context(prm)
    x, y, z, q = (torch.as_tensor(a, device="cuda") for a in (p.x, p.y, p.z, p.q))
    ctx.build_hierarchy(x, y, z, q, tag_rel=w.tag_rel, explicit_boxes=w.explicit_boxes)
    rho, nout = ctx.deposit_built()
    assert nout == 0
    phi, E, st = ctx.solve(rho, tol=w.tol)
    print("  ", {k: st[k] for k in ("iters", "converged", "rel_residual", "dof")}, flush=True)
    assert st["converged"]
    Ex, Ey, Ez = ctx.gather(x, y, z, E)
    # the bench's gather: from the build's ordered copy, equal bit for bit
    for u, v in zip((Ex, Ey, Ez), ctx.gather_built(E)):
        assert torch.equal(u, v)
    torch.cuda.synchronize()

    H = O.hierarchy_from_workload(w)
    assert ctx.info["nlevels"] == H.nlev
    for l in range(H.nlev):
        gb, go = ctx.boxes(l)
        ob, oo = H.boxes(l)
        assert np.array_equal(gb, ob), l
        assert np.array_equal(go, oo), l
    orho = H.deposit_all(p)
    for l in range(H.nlev):
        g = rho[l].cpu().numpy()
        assert np.linalg.norm(g - orho[l]) <= 1e-12 * np.linalg.norm(orho[l]), l
    gphi = [t.cpu().numpy() for t in phi]
    r = H.residual(orho, gphi)
    b = H.residual(orho, H.zeros())
    rel = [float(np.linalg.norm(r[l]) / np.linalg.norm(b[l])) for l in range(H.nlev)]
    print("   oracle residual of the GPU phi", rel, flush=True)
    # the GPU measures the same norms in its own FP64 kernels; the oracle's
    # rounding differs by far less than the margin
    assert max(rel) <= 1.01 * w.tol
    oE = H.efield(gphi)
    gE = [t.cpu().numpy() for t in E]
    for i, (g, o) in enumerate(zip(gE, oE)):
        assert np.abs(g - o).max() <= 1e-11 * np.abs(o).max(), i
    og = H.gather(p, gE)
    for g, o in zip((Ex, Ey, Ez), og):
        assert np.abs(g.cpu().numpy() - o).max() <= 1e-12 * np.abs(o).max()


@pytest.mark.timeout(900)
def test_error_at_the_metric_tolerance():
    """The bench workload (1e6 Gaussian particles, 64^3 + 2 levels) solved on
    the GPU from zero to the metric's 1e-8 relative residual, mixed and plain
    FP64, against the oracle's own solution (its solve to 1e-8 continued to
    1e-11): volume-weighted relative L2 of phi over the composite cells at
    most 1e-8 (mixed) and 1e-9 (FP64); E likewise within 20x that."""
    from paper_1812_03689_amd import amrmg as A
    print("case gauss_64c_2lev at tol 1e-8", flush=True)
    w = W.config2()
    p = w.particles
    x, y, z, q = (torch.as_tensor(a, device="cuda") for a in (p.x, p.y, p.z, p.q))
    sols = {}
    for prec in ("mixed", "fp64"):
        prm = A.make_params(w.n0, max_level=w.max_level, monopoles=w.monopoles, precision=prec,
                            max_grid_size=w.max_grid_size, lo=w.lo, hi=w.hi)
        ctx = A.Context(prm)
        ctx.build_hierarchy(x, y, z, q, tag_rel=w.tag_rel)
        rho, _ = ctx.deposit_built()
        phi, E, st = ctx.solve(rho, tol=w.tol)
        assert st["converged"], (prec, st)
        print("  ", prec, {k: st[k] for k in ("iters", "rel_residual")}, flush=True)
        sols[prec] = ([t.cpu().numpy() for t in phi], [t.cpu().numpy() for t in E])
        nu = (prm.nu1, prm.nu2)
    H = O.hierarchy_from_workload(w)
    orho = H.deposit_all(p)
    ophi, _, ost = H.solve(orho, tol=w.tol, max_iters=50, nu1=nu[0], nu2=nu[1], bottom_rtol=1e-12, want_E=False)
    print("   oracle at 1e-8", ost["iters"], flush=True)
    rphi, rE, rst = H.solve(orho, phi0=ophi, tol=1e-11, max_iters=50, nu1=nu[0], nu2=nu[1], bottom_rtol=1e-13)
    assert rst["converged"]
    print("   oracle continued to 1e-11", rst["iters"], "own error at 1e-8", H.composite_rel_l2(ophi, rphi),
          flush=True)
    for prec, gate in (("mixed", 1e-8), ("fp64", 1e-9)):
        gphi, gE = sols[prec]
        e_phi = H.composite_rel_l2(gphi, rphi)
        e_E = H.composite_rel_l2(gE, rE, ncomp=3)
        print("  ", prec, "phi", e_phi, "E", e_E, flush=True)
        assert e_phi <= gate, (prec, e_phi)
        assert e_E <= 20 * gate, (prec, e_E)
