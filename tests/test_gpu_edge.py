"""Degenerate inputs through the C ABI against the FP64 oracle: no particles
(with and without Dirichlet data), every particle outside the domain, one
particle (a hierarchy refined around a single charge), and particles on the
domain's faces and corners (stencil clamping)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1812_03689_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def amr():
    from paper_1812_03689_amd import amrmg
    return amrmg


def particles(x, y, z, q):
    return W.Particles(*(np.ascontiguousarray(np.asarray(a, dtype=np.float64)) for a in (x, y, z, q)))


def run(w, precision="fp64"):
    A = amr()
    prm = A.make_params(w.n0, max_level=w.max_level, monopoles=w.monopoles, precision=precision,
                        max_grid_size=w.max_grid_size, lo=w.lo, hi=w.hi)
    ctx = A.Context(prm)
    p = w.particles
    x, y, z, q = (torch.as_tensor(a, device="cuda") for a in (p.x, p.y, p.z, p.q))
    ctx.build_hierarchy(x, y, z, q, tag_rel=w.tag_rel, explicit_boxes=w.explicit_boxes)
    return ctx, (x, y, z, q)


def composite_err(H, a, b):
    """Volume-weighted relative L2 over the composite cells (absolute when
    the reference vanishes)."""
    return H.composite_rel_l2(a, b)


def test_no_particles_with_dirichlet_data():
    """The potential of the boundary data alone (a Laplace problem)."""
    e = np.zeros(0)
    w = W.Workload("empty", particles(e, e, e, e), (32, 32, 32), 2, [1e-3, 1e-3], [(1.0, 0.5, 0.5, 0.5)], 1e-10)
    ctx, (x, y, z, q) = run(w)
    assert ctx.info["nlevels"] == 1
    rho, nout = ctx.deposit(x, y, z, q)
    assert nout == 0 and float(rho[0].abs().max()) == 0.0
    rb, nb = ctx.deposit_built()
    assert nb == 0 and float(rb[0].abs().max()) == 0.0
    phi, E, st = ctx.solve(rho, tol=1e-10)
    assert st["converged"]
    H = O.hierarchy_from_workload(w)
    ophi, _, _ = H.solve(H.zeros(), tol=1e-13, max_iters=80, bottom_rtol=1e-14)
    assert composite_err(H, [t.cpu().numpy() for t in phi], ophi) <= 1e-9
    Ex, Ey, Ez = ctx.gather(x, y, z, E)
    assert Ex.numel() == 0


def test_no_particles_no_boundary_data():
    """b = 0 everywhere: the solve returns phi = 0 exactly and reports convergence."""
    e = np.zeros(0)
    w = W.Workload("zero", particles(e, e, e, e), (16, 16, 16), 1, [1e-3], [], 1e-8)
    for precision in ("fp64", "mixed"):
        ctx, (x, y, z, q) = run(w, precision)
        rho, _ = ctx.deposit(x, y, z, q)
        phi, E, st = ctx.solve(rho, tol=1e-8)
        assert st["converged"]
        assert float(phi[0].abs().max()) == 0.0 and float(E[0].abs().max()) == 0.0


def test_every_particle_outside():
    rng = np.random.default_rng(5)
    n = 1000
    x = np.where(rng.random(n) < 0.5, -0.1 - rng.random(n), 1.0 + rng.random(n))
    y, z = rng.random(n), rng.random(n)
    w = W.Workload("outside", particles(x, y, z, np.full(n, 1.0 / n)), (16, 16, 16), 1, [1e-3],
                   [(1.0, 0.5, 0.5, 0.5)], 1e-8)
    ctx, (xd, yd, zd, qd) = run(w)
    rho, nout = ctx.deposit(xd, yd, zd, qd)
    assert nout == n and float(rho[0].abs().max()) == 0.0
    rb, nb = ctx.deposit_built()
    assert nb == n and float(rb[0].abs().max()) == 0.0
    Ex, Ey, Ez = ctx.gather(xd, yd, zd, ctx.solve(rho)[1])
    for c in (Ex, Ey, Ez):  # particles outside the domain get no field
        assert float(c.abs().max()) == 0.0


def test_single_particle():
    """One charge: the hierarchy refines around it; deposit, boxes and solve
    equal the oracle's."""
    w = W.Workload("one", particles([0.4123], [0.5561], [0.3377], [1.0]), (32, 32, 32), 2, [1e-3, 1e-3],
                   [(1.0, 0.4123, 0.5561, 0.3377)], 1e-10)
    H = O.hierarchy_from_workload(w)
    ctx, (x, y, z, q) = run(w)
    assert ctx.info["nlevels"] == H.nlev
    for l in range(H.nlev):
        assert np.array_equal(ctx.boxes(l)[0], H.boxes(l)[0])
    rho, _ = ctx.deposit(x, y, z, q)
    orho = H.deposit_all(w.particles)
    for g, o in zip(rho, orho):
        assert np.linalg.norm(g.cpu().numpy() - o) <= 1e-12 * np.linalg.norm(o)
    phi, E, st = ctx.solve(rho, tol=1e-12)
    assert st["converged"]
    ophi, oE, _ = H.solve(orho, tol=1e-13, max_iters=80, bottom_rtol=1e-14)
    assert composite_err(H, [t.cpu().numpy() for t in phi], ophi) <= 1e-9
    g = np.array([c.cpu().numpy() for c in ctx.gather(x, y, z, E)])
    o = np.array(H.gather(w.particles, oE))
    assert np.linalg.norm(g - o) <= 1e-8 * np.linalg.norm(o)


def test_particles_on_faces_and_corners():
    """Positions at lo, just below hi and on the corners: the CIC stencil
    is clamped to the index space as the oracle does."""
    hi = np.nextafter(1.0, 0.0)
    pts = [(0.0, 0.0, 0.0), (hi, hi, hi), (0.0, 0.5, hi), (0.5, 0.0, 0.5), (hi, 0.25, 0.0), (0.999, 0.001, 0.5),
           (1.0 / 64, 1.0 / 32, 0.5)]
    x, y, z = (np.array([p[d] for p in pts]) for d in range(3))
    w = W.Workload("faces", particles(x, y, z, np.full(len(pts), 1.0 / len(pts))), (32, 32, 32), 1, [1e-3],
                   [(1.0, 0.5, 0.5, 0.5)], 1e-8, explicit_boxes=[(1, 0, 0, 0, 16, 16, 16)])
    H = O.hierarchy_from_workload(w)
    ctx, (xd, yd, zd, qd) = run(w)
    rho, nout = ctx.deposit(xd, yd, zd, qd)
    assert nout == 0
    orho = H.deposit_all(w.particles)
    for g, o in zip(rho, orho):
        g = g.cpu().numpy()
        assert np.abs(g - o).max() <= 1e-12 * np.abs(o).max()
    assert abs(float(sum(float(t.sum()) for t in rho[:1])) * (1.0 / 32) ** 3 - 1.0) <= 1e-12
