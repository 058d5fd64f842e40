"""The domain transform of Sec. 4.1 through the C ABI against the oracle
(oracle/transform.py): the scale s and the mapped coordinates bit for bit
(FP64 and FP32 positions, in place and out of place), the grid rescale bit
for bit, argument errors, and the whole space-charge workflow of the paper's
Fig. sc_workflow (transform, deposit, solve, rescale, gather) on a bunch
given in metres, against the oracle's same workflow and against a solve
done directly in particle space."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import transform as T
from paper_1812_03689_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def amr():
    from paper_1812_03689_amd import amrmg
    return amrmg


def ctx_for(n0=(16, 16, 16), **kw):
    A = amr()
    return A.Context(A.make_params(n0, **kw))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_scale_and_map_bit_exact(dtype):
    print("dtype", dtype, flush=True)
    rng = np.random.default_rng(21)
    n = 200003
    c, l = (0.3, -0.1, 2.0), (0.5, 0.25, 1.0)
    host = [rng.normal(c[d], 0.01 * (d + 1), n) for d in range(3)]
    host[1][777] = c[1] - 0.2  # the outermost particle, in y
    dev = [torch.as_tensor(a, device="cuda").to(dtype) for a in host]
    ref = [t.cpu().numpy() for t in dev]
    ctx = ctx_for()
    xs, ys, zs, s = ctx.transform_particles(*dev, c, l)
    os_ = T.domain_scale(*ref, c, l)
    assert s == os_
    ox = T.to_computation(*ref, c, os_)
    for g, o in zip((xs, ys, zs), ox):
        assert g.dtype == dtype
        assert np.array_equal(g.cpu().numpy(), o)
    # in place
    xi, yi, zi, si = ctx.transform_particles(*dev, c, l, out=dev)
    assert si == s and xi.data_ptr() == dev[0].data_ptr()
    for g, o in zip(dev, ox):
        assert np.array_equal(g.cpu().numpy(), o)


def test_transform_errors_and_empty():
    A = amr()
    ctx = ctx_for()
    e = torch.zeros(0, dtype=torch.float64, device="cuda")
    assert ctx.transform_particles(e, e, e, (0, 0, 0), (1, 1, 1))[3] == 0.0
    one = torch.full((5,), 2.0, dtype=torch.float64, device="cuda")
    with pytest.raises(A.AmrmgError) as ex:  # every particle at the centre
        ctx.transform_particles(one, one, one, (2.0, 2.0, 2.0), (1, 1, 1))
    assert ex.value.status == -1
    bad = one.clone()
    bad[3] = float("nan")
    with pytest.raises(A.AmrmgError):
        ctx.transform_particles(bad, one, one, (0, 0, 0), (1, 1, 1))
    with pytest.raises(A.AmrmgError):
        ctx.transform_particles(one, one, one, (0, 0, 0), (1, 0, 1))
    with pytest.raises(A.AmrmgError) as ex:  # rescale needs a hierarchy
        ctx.rescale_fields(2.0, [e])
    assert ex.value.status == -6


def test_rescale_bit_exact():
    w = W.config1()
    A = amr()
    ctx = A.Context(A.make_params(w.n0, max_level=w.max_level, monopoles=w.monopoles))
    p = w.particles
    x, y, z, q = (torch.as_tensor(a, device="cuda") for a in (p.x, p.y, p.z, p.q))
    ctx.build_hierarchy(x, y, z, q, tag_rel=w.tag_rel, explicit_boxes=w.explicit_boxes)
    g = torch.Generator(device="cpu").manual_seed(5)
    phi = [torch.randn(int(n), generator=g, dtype=torch.float64).cuda() for n in ctx.info["ncells"]]
    E = [torch.randn(int(n), generator=g, dtype=torch.float64).cuda() for n in ctx.info["ncells"] for _ in range(3)]
    hp, hE = [t.cpu().numpy() for t in phi], [t.cpu().numpy() for t in E]
    s = 0.0123456789
    ctx.rescale_fields(s, phi, E)
    op, oE = T.rescale(hp, hE, s)
    for a, b in zip(phi + E, op + oE):
        assert np.array_equal(a.cpu().numpy(), b)
    ctx.rescale_fields(3.0, None, E)  # phi may be omitted
    with pytest.raises(A.AmrmgError):
        ctx.rescale_fields(0.0, phi, E)


def bunch_in_metres():
    """A C2-shaped bunch 2 cm across around a reference position away from
    the origin, unit total charge."""
    p = W.gaussian_bunch(20000, sigma=(0.05, 0.05, 0.1), seed=W.seed_for(7, 2))
    c, scale = (0.3, -0.1, 2.0), 0.02
    X = [c[d] + scale * (a - 0.5) for d, a in enumerate((p.x, p.y, p.z))]
    return W.Particles(X[0], X[1], X[2], p.q.copy()), c


def composite_err(H, a, b):
    """Volume-weighted relative L2 over the composite cells."""
    return H.composite_rel_l2(a, b)


def test_space_charge_workflow_in_computation_space():
    """Transform (l = 1, margin 10 %), build, deposit, solve, rescale,
    gather on the GPU; the oracle runs the same workflow from its own
    transform."""
    A = amr()
    parts, c = bunch_in_metres()
    l, m = (1.0, 1.0, 1.0), 1.1
    dev = [torch.as_tensor(a, device="cuda") for a in (parts.x, parts.y, parts.z, parts.q)]
    probe = ctx_for()
    xs, ys, zs, s = probe.transform_particles(dev[0], dev[1], dev[2], c, l)
    n0, lo, hi = (32, 32, 32), (-m, -m, -m), (m, m, m)
    ctx = A.Context(A.make_params(n0, max_level=2, monopoles=[(1.0, 0.0, 0.0, 0.0)], precision="fp64", lo=lo,
                                  hi=hi))
    ctx.build_hierarchy(xs, ys, zs, dev[3], tag_rel=[1e-3, 1e-3])
    rho, nout = ctx.deposit_built()
    assert nout == 0
    phi, E, st = ctx.solve(rho, tol=1e-12)
    assert st["converged"]
    ctx.rescale_fields(s, phi, E)
    Ex, Ey, Ez = ctx.gather(xs, ys, zs, E)
    # the oracle's workflow
    os_ = T.domain_scale(parts.x, parts.y, parts.z, c, l)
    assert os_ == s
    ox = T.to_computation(parts.x, parts.y, parts.z, c, os_)
    wc = W.Workload("bunch_c", W.Particles(*ox, parts.q.copy()), n0, 2, [1e-3, 1e-3], [(1.0, 0.0, 0.0, 0.0)], 1e-12,
                    lo=lo, hi=hi)
    H = O.hierarchy_from_workload(wc)
    assert ctx.info["nlevels"] == H.nlev
    for lv in range(H.nlev):
        assert np.array_equal(ctx.boxes(lv)[0], H.boxes(lv)[0])
    ophi, oE, _ = H.solve(H.deposit_all(wc.particles), tol=1e-13, max_iters=80, bottom_rtol=1e-14)
    ophi, oE = T.rescale(ophi, oE, os_)
    assert composite_err(H, [t.cpu().numpy() for t in phi], ophi) <= 1e-9
    og = H.gather(wc.particles, oE)
    for g, o in zip((Ex, Ey, Ez), og):
        assert np.abs(g.cpu().numpy() - o).max() <= 2e-8 * np.abs(o).max()
    # the same cells solved directly in particle space (domain c + s * [lo, hi))
    lo_p = tuple(c[d] + s * lo[d] for d in range(3))
    hi_p = tuple(c[d] + s * hi[d] for d in range(3))
    direct = A.Context(A.make_params(n0, max_level=2, monopoles=[(1.0, *c)], precision="fp64", lo=lo_p, hi=hi_p))
    direct.build_hierarchy(*dev, tag_rel=[1e-3, 1e-3])
    for lv in range(H.nlev):
        assert np.array_equal(direct.boxes(lv)[0], H.boxes(lv)[0])
    rp, _ = direct.deposit_built()
    pp, Ep, st = direct.solve(rp, tol=1e-12)
    assert st["converged"]
    assert composite_err(H, [t.cpu().numpy() for t in pp], [t.cpu().numpy() for t in phi]) <= 1e-9
