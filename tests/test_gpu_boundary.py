"""Boundary contracts of the C ABI that the solve parity tests do not reach:

  * the caller-owned workspace (amrmg_workspace_size / amrmg_set_workspace):
    a solve in a torch uint8 buffer, filled with garbage first, gives phi and
    E bit-equal to the library-owned solve (the solve path has no floating-
    point atomics) and writes into that buffer; a buffer one byte short gives
    AMRMG_E_OOM, a misaligned one AMRMG_E_INVALID; NULL returns to library
    memory; a rebuild that needs more than the caller's buffer fails the next
    solve with AMRMG_E_OOM;
  * AMRMG_E_NOT_CONVERGED still writes phi, E and the statistics: E is the
    field of the phi returned (checked against the oracle's -grad of it)."""
import ctypes as C

import numpy as np
import pytest

from oracle import oracle as O
from paper_1812_03689_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def setup(w, precision):
    from paper_1812_03689_amd import amrmg as A
    prm = A.make_params(w.n0, max_level=w.max_level, monopoles=w.monopoles, precision=precision,
                        max_grid_size=w.max_grid_size, lo=w.lo, hi=w.hi)
    ctx = A.Context(prm)
    x, y, z, q = (torch.as_tensor(a, device="cuda") for a in (w.particles.x, w.particles.y, w.particles.z,
                                                              w.particles.q))
    ctx.build_hierarchy(x, y, z, q, tag_rel=w.tag_rel, explicit_boxes=w.explicit_boxes)
    return A, ctx, (x, y, z, q)


def aligned_buffer(nbytes, pad=0):
    """A uint8 device buffer of nbytes starting on a 256-byte boundary."""
    raw = torch.empty(nbytes + 512, dtype=torch.uint8, device="cuda")
    off = (-raw.data_ptr()) % 256 + pad
    return raw, raw[off:off + nbytes]


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_caller_workspace(precision):
    print("case workspace", precision, flush=True)
    p = W.gaussian_bunch(50000, sigma=(0.06, 0.06, 0.1), seed=W.seed_for(2, 21))
    w = W.Workload("ws", p, (32, 32, 32), 2, [1e-3, 1e-3], [(1.0, 0.5, 0.5, 0.5)], 1e-10)
    A, ctx, (x, y, z, q) = setup(w, precision)
    rho, _ = ctx.deposit(x, y, z, q)
    phi0, E0, st0 = ctx.solve(rho, tol=w.tol)
    assert st0["converged"]
    need = A.amrmg_workspace_size(ctx.h)
    assert need > 0
    raw, buf = aligned_buffer(need)
    buf.fill_(0xFF)  # NaN bit patterns in every float view
    A.amrmg_set_workspace(ctx.h, buf)
    phi1, E1, st1 = ctx.solve(rho, tol=w.tol)
    torch.cuda.synchronize()
    assert st1["iters"] == st0["iters"]
    for a, b in zip(phi0 + E0, phi1 + E1):
        assert torch.equal(a, b)
    assert int((buf != 0xFF).sum()) > need // 8  # the solve ran in the caller's buffer
    # a second solve reuses the same buffer (and its captured graph)
    phi2, E2, _ = ctx.solve(rho, tol=w.tol)
    for a, b in zip(phi0 + E0, phi2 + E2):
        assert torch.equal(a, b)
    # one byte short, misaligned
    L = A.lib()
    assert L.amrmg_set_workspace(ctx.h, C.c_void_p(buf.data_ptr()), need - 1) == A.AMRMG_E_OOM
    _, mis = aligned_buffer(need, pad=8)
    assert L.amrmg_set_workspace(ctx.h, C.c_void_p(mis.data_ptr()), need) == A.AMRMG_E_INVALID
    # back to library memory; the caller's buffer is no longer touched
    A.amrmg_set_workspace(ctx.h, None)
    buf.fill_(0x5A)
    phi3, E3, _ = ctx.solve(rho, tol=w.tol)
    torch.cuda.synchronize()
    for a, b in zip(phi0 + E0, phi3 + E3):
        assert torch.equal(a, b)
    assert bool((buf == 0x5A).all())
    # a caller buffer that a later, larger hierarchy outgrows
    A.amrmg_set_workspace(ctx.h, buf)
    pb = W.gaussian_bunch(50000, sigma=(0.2, 0.2, 0.2), seed=W.seed_for(2, 22))
    xb, yb, zb, qb = (torch.as_tensor(a, device="cuda") for a in (pb.x, pb.y, pb.z, pb.q))
    ctx.build_hierarchy(xb, yb, zb, qb, tag_rel=[1e-4, 1e-4])
    assert A.amrmg_workspace_size(ctx.h) > need
    rho_b, _ = ctx.deposit(xb, yb, zb, qb)
    with pytest.raises(A.AmrmgError) as ei:
        ctx.solve(rho_b, tol=w.tol)
    assert ei.value.status == A.AMRMG_E_OOM
    A.amrmg_set_workspace(ctx.h, None)
    _, _, st = ctx.solve(rho_b, tol=w.tol)
    assert st["converged"]


def test_not_converged_still_writes_phi_E_and_stats():
    print("case not converged", flush=True)
    w = W.config1(n_particles=5000)
    A, ctx, (x, y, z, q) = setup(w, "fp64")
    ctx2 = A.Context(A.make_params(w.n0, max_level=w.max_level, monopoles=w.monopoles, precision="fp64",
                                   max_iters=1))
    ctx2.build_hierarchy(x, y, z, q, explicit_boxes=w.explicit_boxes)
    rho, _ = ctx2.deposit(x, y, z, q)
    phi = ctx2.level_arrays()
    E = ctx2.level_arrays(3)
    for t in E:
        t.fill_(float("nan"))
    st = A.amrmg_solve(ctx2.h, rho, phi, E, 1e-12)
    torch.cuda.synchronize()
    assert st["status"] == A.AMRMG_E_NOT_CONVERGED
    assert st["iters"] == 1 and not st["converged"] and st["nlevels"] == 2
    assert st["dof"] == ctx2.info["ndof"] and st["time_ms"] > 0
    assert max(st["rel_residual"]) > 1e-12 and all(np.isfinite(st["rel_residual"]))
    gphi = [t.cpu().numpy() for t in phi]
    assert all(np.isfinite(a).all() and np.abs(a).max() > 0 for a in gphi)
    # the statistics and E belong to the phi returned
    H = O.hierarchy_from_workload(w)
    orho = H.deposit_all(w.particles)
    r = H.residual(orho, gphi)
    b = H.residual(orho, H.zeros())
    for l in range(H.nlev):
        rel = np.linalg.norm(r[l]) / np.linalg.norm(b[l])
        assert abs(rel - st["rel_residual"][l]) <= 1e-6 * rel, (l, rel, st["rel_residual"][l])
    oE = H.efield(gphi)
    for i, (g, o) in enumerate(zip([t.cpu().numpy() for t in E], oE)):
        assert np.isfinite(g).all()
        assert np.abs(g - o).max() <= 1e-11 * np.abs(o).max(), i
