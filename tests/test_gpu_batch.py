"""amrmg_solve_batch (many independent small problems in one set of
launches) against the FP64 oracle: a mixed batch of base sizes and depths
element by element, and the full 64-instance batch of independent solves
through the oracle's composite residual (Alg. 1) of the GPU solution."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1812_03689_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def amr():
    from paper_1812_03689_amd import amrmg
    return amrmg


def contexts(ws, precision="mixed", **kw):
    A = amr()
    out = []
    for w in ws:
        prm = A.make_params(w.n0, max_level=w.max_level, monopoles=w.monopoles, precision=precision,
                            max_grid_size=w.max_grid_size, **kw)
        c = A.Context(prm)
        p = w.particles
        x, y, z, q = (torch.as_tensor(a, device="cuda") for a in (p.x, p.y, p.z, p.q))
        c.build_hierarchy(x, y, z, q, tag_rel=w.tag_rel, explicit_boxes=w.explicit_boxes)
        rho, nout = c.deposit(x, y, z, q)
        assert nout == 0
        out.append((c, rho, c.level_arrays()))
    return out


_oracle = {}


def oracle_phi(w):
    if w.name not in _oracle:
        H = O.hierarchy_from_workload(w)
        orho = H.deposit_all(w.particles)
        ophi, _, _ = H.solve(orho, tol=1e-13, max_iters=80, bottom_rtol=1e-13, want_E=False)
        _oracle[w.name] = (H, ophi)
    return _oracle[w.name]


def rel_l2_composite(H, a, b):
    """Volume-weighted relative L2 over the composite cells."""
    return H.composite_rel_l2(a, b)


@pytest.mark.parametrize("precision,tol_err", [("mixed", 1e-8), ("fp64", 1e-9)])
def test_batch_matches_oracle(precision, tol_err):
    """Six problems of different base size (16, 24, 32), depth (1 or 2
    refined levels) and coarsest grid (geometric levels below level 0 or not)
    solved together; each equals its own oracle solution."""
    A = amr()
    ws = [W.config5_instances(64)[i] for i in (1, 2, 4, 5, 10, 11)]
    print("batch", [w.name for w in ws], precision, flush=True)
    cs = contexts(ws, precision)
    st = A.amrmg_solve_batch([c.h for c, _, _ in cs], [r for _, r, _ in cs], [p for _, _, p in cs], 1e-12)
    for w, (c, rho, phi), s in zip(ws, cs, st):
        print(w.name, s["iters"], s["rel_residual"], flush=True)
        assert s["converged"], (w.name, s)
        H, ophi = oracle_phi(w)
        err = rel_l2_composite(H, [t.cpu().numpy() for t in phi], ophi)
        print("  rel L2", err, flush=True)
        assert err <= tol_err, w.name


def test_batch_same_as_single_solves():
    """The batch gives each problem what its own amrmg_solve gives (same
    cycle, same tolerance), up to the tolerance."""
    A = amr()
    ws = [W.config5_instances(64)[i] for i in (4, 3, 1)]
    cs = contexts(ws, "mixed")
    st = A.amrmg_solve_batch([c.h for c, _, _ in cs], [r for _, r, _ in cs], [p for _, _, p in cs], 1e-10)
    assert all(s["converged"] for s in st)
    for w, (c, rho, phi) in zip(ws, cs):
        phi1, _, s1 = c.solve(rho, tol=1e-10, want_E=False)
        a = np.concatenate([t.cpu().numpy() for t in phi])
        b = np.concatenate([t.cpu().numpy() for t in phi1])
        assert np.linalg.norm(a - b) <= 1e-8 * np.linalg.norm(b), w.name


def test_full_batch_residual_property():
    """All 64 instances (base 16-48, 1 or 2 refined levels, 1e4-1e5
    particles) in one batch to tol 1e-8: for every instance and level the
    oracle's composite residual of the GPU solution is within the tolerance
    of the oracle's right-hand-side norm (the stopping rule of Alg. 2)."""
    A = amr()
    ws = W.config5_instances(64)
    cs = contexts(ws, "mixed")
    st = A.amrmg_solve_batch([c.h for c, _, _ in cs], [r for _, r, _ in cs], [p for _, _, p in cs], 1e-8)
    worst = 0.0
    for w, (c, rho, phi), s in zip(ws, cs, st):
        assert s["converged"], (w.name, s)
        H = O.hierarchy_from_workload(w)
        orho = H.deposit_all(w.particles)
        r = H.residual(orho, [t.cpu().numpy() for t in phi])
        b = H.residual(orho, H.zeros())
        for l in range(H.nlev):
            rel = np.linalg.norm(r[l]) / np.linalg.norm(b[l])
            worst = max(worst, rel)
            assert rel <= 1.5e-8, (w.name, l, rel)
    print("worst oracle relative residual", worst, flush=True)


def test_batch_errors():
    A = amr()
    ws = [W.config5_instances(64)[i] for i in (4, 10)]
    cs = contexts(ws, "mixed")
    hs = [c.h for c, _, _ in cs]
    with pytest.raises(A.AmrmgError) as ei:
        A.amrmg_solve_batch([hs[0], hs[0]], [cs[0][1], cs[0][1]], [cs[0][2], cs[0][2]], 1e-8)
    assert ei.value.status == A.AMRMG_E_INVALID
    other = contexts(ws[:1], "fp64")[0]
    with pytest.raises(A.AmrmgError) as ei:
        A.amrmg_solve_batch([hs[0], other[0].h], [cs[0][1], other[1]], [cs[0][2], other[2]], 1e-8)
    assert ei.value.status == A.AMRMG_E_INVALID
