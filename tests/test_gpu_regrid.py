"""Regrids on one context, as a PIC run does them: a sequence of builds whose
hierarchies grow, shrink and move (two refined levels, none, a single one,
levels given explicitly, then tagged again, with particle counts up and
down; a threshold of 1 tags nothing under the strict comparison), each
checked against a fresh oracle hierarchy: boxes bit for bit, the deposit
from the build's ordered copy, and the oracle's residual of the solution.
Catches state that one build leaves to the next."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1812_03689_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def seq():
    g = lambda n, c, s, seed: W.gaussian_bunch(n, sigma=s, seed=W.seed_for(11, seed), centre=c)
    mono = [(1.0, 0.5, 0.5, 0.5)]
    yield W.Workload("a", g(40000, (0.5, 0.5, 0.5), (0.05, 0.05, 0.1), 1), (32, 32, 32), 2, [1e-3, 1e-3], mono, 1e-9)
    yield W.Workload("moved", g(60000, (0.4, 0.55, 0.6), (0.04, 0.06, 0.08), 2), (32, 32, 32), 2, [1e-3, 1e-3], mono,
                     1e-9)
    yield W.Workload("flat", W.uniform_ball(30000, radius=0.45, seed=W.seed_for(11, 3)), (32, 32, 32), 2,
                     [1.0, 1.0], mono, 1e-9)
    yield W.Workload("explicit", g(20000, (0.5, 0.5, 0.5), (0.08, 0.08, 0.08), 4), (32, 32, 32), 2, [1e-3, 1e-3],
                     mono, 1e-9, explicit_boxes=[(1, 16, 16, 16, 48, 48, 40)])
    yield W.Workload("one_level", g(80000, (0.6, 0.45, 0.5), (0.06, 0.06, 0.06), 5), (32, 32, 32), 2, [1e-2, 1.0],
                     mono, 1e-9)
    yield W.Workload("again", g(40000, (0.5, 0.5, 0.5), (0.05, 0.05, 0.1), 1), (32, 32, 32), 2, [1e-3, 1e-3], mono,
                     1e-9)


def test_regrid_sequence_matches_fresh_oracle_builds():
    from paper_1812_03689_amd import amrmg as A
    ctx = A.Context(A.make_params((32, 32, 32), max_level=2, monopoles=[(1.0, 0.5, 0.5, 0.5)], precision="mixed"))
    levels_seen = set()
    for w in seq():
        print("build", w.name, flush=True)
        p = w.particles
        x, y, z, q = (torch.as_tensor(a, device="cuda") for a in (p.x, p.y, p.z, p.q))
        ctx.build_hierarchy(x, y, z, q, tag_rel=w.tag_rel, explicit_boxes=w.explicit_boxes)
        H = O.hierarchy_from_workload(w)
        levels_seen.add(H.nlev)
        assert ctx.info["nlevels"] == H.nlev
        for l in range(H.nlev):
            assert np.array_equal(ctx.boxes(l)[0], H.boxes(l)[0]), (w.name, l)
        rho, nout = ctx.deposit_built()
        assert nout == 0
        orho = H.deposit_all(p)
        for l in range(H.nlev):
            assert np.linalg.norm(rho[l].cpu().numpy() - orho[l]) <= 1e-12 * np.linalg.norm(orho[l]), (w.name, l)
        phi, E, st = ctx.solve(rho, tol=w.tol)
        assert st["converged"], (w.name, st)
        r = H.residual(orho, [t.cpu().numpy() for t in phi])
        b = H.residual(orho, H.zeros())
        rel = [float(np.linalg.norm(r[l]) / np.linalg.norm(b[l])) for l in range(H.nlev)]
        assert max(rel) <= 1.01 * w.tol, (w.name, rel)
    assert levels_seen == {1, 2, 3}
