"""amrmg_gather_built through the C ABI: E at the build's particles read from
the build's ordered copy equals amrmg_gather at the same positions bit for
bit (same arithmetic, same level choice), and the oracle's interpolation of
the same E to round-off; FP32 positions; the caller's arrays changed after
the build (the result stays that at the build's particles); a hierarchy of
no particles; the state errors."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1812_03689_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def workload():
    p = W.gaussian_bunch(100000, sigma=(0.05, 0.05, 0.1), seed=W.seed_for(2, 7))
    return W.Workload("gauss_32c_2lev", p, (32, 32, 32), 2, [1e-3, 1e-3], [(1.0, 0.5, 0.5, 0.5)], 1e-8)


def built(w, pos_dtype):
    from paper_1812_03689_amd import amrmg as A
    ctx = A.Context(A.make_params(w.n0, max_level=w.max_level, monopoles=w.monopoles, precision="mixed"))
    p = w.particles
    x, y, z = (torch.as_tensor(a, device="cuda").to(pos_dtype) for a in (p.x, p.y, p.z))
    q = torch.as_tensor(p.q, device="cuda")
    ctx.build_hierarchy(x, y, z, q, tag_rel=w.tag_rel)
    rho, _ = ctx.deposit_built()
    _, E, st = ctx.solve(rho, tol=1e-10)
    assert st["converged"]
    return ctx, (x, y, z), E


@pytest.mark.parametrize("pos_dtype", [torch.float64, torch.float32])
def test_gather_built_equals_gather_and_oracle(pos_dtype):
    print("gather_built", pos_dtype, flush=True)
    w = workload()
    ctx, (x, y, z), E = built(w, pos_dtype)
    a = ctx.gather(x, y, z, E)
    b = ctx.gather_built(E)
    torch.cuda.synchronize()
    for u, v in zip(a, b):
        assert torch.equal(u, v)
    H = O.hierarchy_from_workload(w)
    p = w.particles
    if pos_dtype == torch.float32:
        p = W.Particles(*(t.cpu().double().numpy() for t in (x, y, z)), p.q)
    og = H.gather(p, [t.cpu().numpy() for t in E])
    for g, o in zip(b, og):
        assert np.abs(g.cpu().numpy() - o).max() <= 1e-12 * np.abs(o).max()


def test_visiting_order_and_caller_order_agree_bit_for_bit():
    """The gather in the build's visiting order (E staged per particle, then
    written in the caller's order through the inverse order) and the single
    pass in the caller's order (taken for a particle count other than the
    build's) give the same E bit for bit on the particles they share."""
    w = workload()
    ctx, (x, y, z), E = built(w, torch.float32)
    a = ctx.gather_built(E)
    m = x.numel() - 1
    b = ctx.gather(x[:m], y[:m], z[:m], E)
    c = ctx.gather(x, y, z, E)
    torch.cuda.synchronize()
    for u, v, t in zip(a, b, c):
        assert torch.equal(u[:m], v)
        assert torch.equal(u, t)


def test_gather_built_after_the_arrays_change():
    w = workload()
    ctx, (x, y, z), E = built(w, torch.float64)
    ref = [t.clone() for t in ctx.gather(x, y, z, E)]
    for t in (x, y, z):
        t.mul_(0.5).add_(0.1)
    b = ctx.gather_built(E)
    torch.cuda.synchronize()
    for u, v in zip(ref, b):
        assert torch.equal(u, v)


def test_gather_built_without_particles_and_state_errors():
    from paper_1812_03689_amd import amrmg as A
    ctx = A.Context(A.make_params((16, 16, 16), max_level=1, monopoles=[(1.0, 0.5, 0.5, 0.5)]))
    E3 = [torch.zeros(16 ** 3, dtype=torch.float64, device="cuda") for _ in range(3)]
    e = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(A.AmrmgError) as ex:
        A.amrmg_gather_built(ctx.h, E3, e, e, e)
    assert ex.value.status == A.AMRMG_E_STATE
    empty = torch.zeros(0, dtype=torch.float64, device="cuda")
    ctx.build_hierarchy(empty, empty, empty, empty, tag_rel=[1e-3])
    rho, _ = ctx.deposit_built()
    _, E, st = ctx.solve(rho, tol=1e-10)
    assert st["converged"]
    Ex, Ey, Ez = ctx.gather_built(E)
    assert Ex.numel() == Ey.numel() == Ez.numel() == 0
