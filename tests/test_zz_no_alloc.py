"""amrmg_solve_noalloc (the solve for callers that cannot allocate device
memory; its workspace is the library's static device array) against
amrmg_solve through the C ABI: two calls in a row, the second on a smaller
hierarchy (and the other precision), each matching amrmg_solve's phi, E and
statistics (same iteration count, phi and E to 1e-12 relative, volume-
weighted over the composite cells), the smaller also against the oracle to
the mixed gate; then a hierarchy whose workspace exceeds the array is
refused with AMRMG_E_OOM and leaves phi untouched."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1812_03689_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def problem(A, n0, n_particles, levels, precision, seed):
    p = W.gaussian_bunch(n_particles, sigma=(0.06, 0.06, 0.1), seed=W.seed_for(2, seed))
    w = W.Workload("noalloc", p, (n0, n0, n0), levels, [1e-3] * levels, [(1.0, 0.5, 0.5, 0.5)], 1e-10)
    prm = A.make_params(w.n0, max_level=w.max_level, monopoles=w.monopoles, precision=precision)
    ctx = A.Context(prm)
    x, y, z, q = (torch.as_tensor(a, device="cuda") for a in (p.x, p.y, p.z, p.q))
    ctx.build_hierarchy(x, y, z, q, tag_rel=w.tag_rel)
    rho, _ = ctx.deposit(x, y, z, q)
    return w, ctx, rho


def test_solve_noalloc_matches_solve():
    from paper_1812_03689_amd import amrmg as A
    print("case noalloc: 64^3 + 2 mixed, then 32^3 + 1 fp64", flush=True)
    cases = [problem(A, 64, 200000, 2, "mixed", 31), problem(A, 32, 30000, 1, "fp64", 32)]
    assert cases[1][1].info["ndof"] < cases[0][1].info["ndof"]
    refs = []
    for w, ctx, rho in cases:
        assert A.amrmg_workspace_size(ctx.h) <= A.AMRMG_NOALLOC_SCRATCH_BYTES
        phi, E = ctx.level_arrays(), ctx.level_arrays(3)
        st = A.amrmg_solve(ctx.h, rho, phi, E, w.tol)
        assert st["converged"]
        refs.append(([t.cpu().numpy() for t in phi], [t.cpu().numpy() for t in E], st))
    outs = []
    for w, ctx, rho in cases:  # two calls in a row, the second smaller
        phi, E = ctx.level_arrays(), ctx.level_arrays(3)
        for t in phi + E:
            t.fill_(float("nan"))
        for t in phi:
            t.zero_()
        st = A.amrmg_solve_noalloc(ctx.h, rho, phi, E, w.tol)
        torch.cuda.synchronize()
        outs.append(([t.cpu().numpy() for t in phi], [t.cpu().numpy() for t in E], st))
    for (w, ctx, rho), (rphi, rE, rst), (gphi, gE, gst) in zip(cases, refs, outs):
        H = O.hierarchy_from_workload(w)
        print("  ", ctx.info["ncells"], gst["iters"], rst["iters"], flush=True)
        assert gst["status"] == A.AMRMG_OK and gst["converged"]
        assert gst["iters"] == rst["iters"] and gst["dof"] == rst["dof"]
        np.testing.assert_allclose(gst["rel_residual"], rst["rel_residual"], rtol=1e-6)
        assert H.composite_rel_l2(gphi, rphi) <= 1e-12
        assert H.composite_rel_l2(gE, rE, ncomp=3) <= 1e-12
        assert all(np.isfinite(a).all() for a in gE)
    # the smaller problem against the oracle
    w, ctx, rho = cases[1]
    H = O.hierarchy_from_workload(w)
    ophi, _, _ = H.solve(H.deposit_all(w.particles), tol=1e-13, max_iters=80, bottom_rtol=1e-14, want_E=False)
    assert H.composite_rel_l2(outs[1][0], ophi) <= 1e-8
    # the normal solve still works after the no-allocation one (own workspace)
    phi = ctx.level_arrays()
    st = A.amrmg_solve(ctx.h, rho, phi, None, w.tol)
    assert st["converged"] and H.composite_rel_l2([t.cpu().numpy() for t in phi], refs[1][0]) <= 1e-12


def test_solve_noalloc_refuses_a_larger_workspace():
    from paper_1812_03689_amd import amrmg as A
    print("case noalloc: 160^3 fp64 (workspace above the array)", flush=True)
    w, ctx, rho = problem(A, 160, 20000, 0, "fp64", 33)
    need = A.amrmg_workspace_size(ctx.h)
    assert need > A.AMRMG_NOALLOC_SCRATCH_BYTES
    phi = ctx.level_arrays()
    for t in phi:
        t.fill_(3.0)
    with pytest.raises(A.AmrmgError) as ei:
        A.amrmg_solve_noalloc(ctx.h, rho, phi, None, w.tol)
    assert ei.value.status == A.AMRMG_E_OOM
    assert "bytes of workspace" in str(ei.value)
    torch.cuda.synchronize()
    assert all(bool((t == 3.0).all()) for t in phi)
