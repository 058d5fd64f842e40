"""Parity of the HIP path (through the C ABI) with the FP64 oracle on the
same seeded inputs: hierarchy and pattern ids bit for bit, deposit to 1e-12,
the FP64 composite residual operator to round-off, and the solve to 1e-9
(FP64 cycle) / 1e-8 (mixed cycle) relative L2 over the composite cells, plus
E and the gather.  Sizes span several bricks, coarse-fine faces with shifted
windows, boundary-touching boxes, and multigrid levels below level 0."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1812_03689_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def amr():
    from paper_1812_03689_amd import amrmg
    return amrmg


def dev(p):
    return [torch.as_tensor(a, device="cuda") for a in (p.x, p.y, p.z, p.q)]


def np_list(ts):
    return [t.detach().cpu().numpy() for t in ts]


def rel_l2_composite(H, a, b):
    """Volume-weighted relative L2 over the composite cells."""
    return H.composite_rel_l2(a, b)


def make_ctx(w, precision="fp64", smoother="gsrb", **kw):
    A = amr()
    prm = A.make_params(w.n0, max_level=w.max_level, monopoles=w.monopoles, precision=precision,
                        smoother=smoother, max_grid_size=w.max_grid_size, lo=w.lo, hi=w.hi, **kw)
    ctx = A.Context(prm)
    x, y, z, q = dev(w.particles)
    ctx.build_hierarchy(x, y, z, q, tag_rel=w.tag_rel, explicit_boxes=w.explicit_boxes)
    return ctx, (x, y, z, q)


def small_c2(n=100000):
    """The C2 bunch shape (sigma 0.05, 0.05, 0.1, two levels at 1e-3 x max)
    on a 32^3 base so the oracle finishes in seconds."""
    p = W.gaussian_bunch(n, sigma=(0.05, 0.05, 0.1), seed=W.seed_for(2, 7))
    return W.Workload("gauss_32c_2lev", p, (32, 32, 32), 2, [1e-3, 1e-3], [(1.0, 0.5, 0.5, 0.5)], 1e-8)


_cache = {}


def oracle_solution(w, key):
    if key not in _cache:
        H = O.hierarchy_from_workload(w)
        rho = H.deposit_all(w.particles)
        phi, E, st = H.solve(rho, tol=1e-13, max_iters=80, bottom_rtol=1e-14)
        _cache[key] = (H, rho, phi, E, st)
    return _cache[key]


def small_chain():
    """The paper's benchmark shape (11 bunches 4 cm apart, sigma 1.5 / 5 / 5 mm,
    homogeneous Dirichlet on the computation cube around them, which is not
    the unit cube) with 2e3 particles per bunch on a 32^3 base: all charge
    lies on level 2, so levels 0 and 1 use the composite norm."""
    p = W.chain_bunches(2000, seed=W.seed_for(6, 1))
    lo, hi = W.isotropic_domain(p)
    return W.Workload("chain11_32c_2lev", p, (32, 32, 32), 2, [1e-3, 1e-3], [], 1e-8, lo=lo, hi=hi)


CASES = {"c1": lambda: W.config1(), "c2s": small_c2, "chain": small_chain}


@pytest.mark.parametrize("case", sorted(CASES))
def test_hierarchy_bit_exact(case):
    print("case", case, flush=True)
    w = CASES[case]()
    H = O.hierarchy_from_workload(w)
    ctx, _ = make_ctx(w)
    assert ctx.info["nlevels"] == H.nlev
    for l in range(H.nlev):
        gb, go = ctx.boxes(l)
        ob, oo = H.boxes(l)
        assert np.array_equal(gb, ob), l
        assert np.array_equal(go, oo), l
    for l in range(1, H.nlev):
        rows = ctx.cf_faces(l)
        assert rows.shape[0] > 0
        for r in rows[:: max(1, rows.shape[0] // 2000)]:
            op, _ = H.cf_pattern(l, *(int(v) for v in r[:5]))
            assert op == r[5]
    dof = sum(int((~H.covered_mask(l)).sum()) for l in range(H.nlev))
    assert ctx.info["ndof"] == dof


@pytest.mark.parametrize("case", sorted(CASES))
def test_deposit(case):
    print("case", case, flush=True)
    w = CASES[case]()
    H = O.hierarchy_from_workload(w)
    ctx, (x, y, z, q) = make_ctx(w)
    rho, nout = ctx.deposit(x, y, z, q)
    assert nout == 0
    orho = H.deposit_all(w.particles)
    for l, (g, o) in enumerate(zip(np_list(rho), orho)):
        assert np.linalg.norm(g - o) <= 1e-12 * np.linalg.norm(o), l


@pytest.mark.parametrize("case", sorted(CASES))
def test_deposit_built(case):
    """amrmg_deposit_built (levels kept from the build's tagging deposits,
    the rest deposited from its ordered copy) equals the oracle's deposit of
    the build's particles, also after the caller's arrays have changed."""
    print("case", case, flush=True)
    w = CASES[case]()
    H = O.hierarchy_from_workload(w)
    ctx, (x, y, z, q) = make_ctx(w)
    x.fill_(0.5)  # the caller reuses its arrays: the build's particles count
    q.mul_(3.0)
    rho, nout = ctx.deposit_built()
    assert nout == 0
    orho = H.deposit_all(w.particles)
    for l, (g, o) in enumerate(zip(np_list(rho), orho)):
        assert np.linalg.norm(g - o) <= 1e-12 * np.linalg.norm(o), l


def test_deposit_built_counts_outside_particles():
    """Particles outside [lo, hi) are skipped and counted as amrmg_deposit
    does, whether level 0 was deposited by the build (tagging) or not."""
    base = small_c2(20000)
    p = base.particles
    rng = np.random.default_rng(11)
    out = rng.choice(p.x.size, 37, replace=False)
    p.x[out[:20]] = 1.0 + 0.25 * rng.random(20)
    p.z[out[20:]] = -0.5 * rng.random(17)
    for w in (base, W.Workload("explicit", p, (32, 32, 32), 1, [], base.monopoles, 1e-8,
                               explicit_boxes=[(1, 16, 16, 16, 48, 48, 48)])):
        ctx, (x, y, z, q) = make_ctx(w)
        ref, nref = ctx.deposit(x, y, z, q)
        got, nout = ctx.deposit_built()
        assert nref == 37 and nout == 37, (w.name, nref, nout)
        for l, (g, o) in enumerate(zip(np_list(got), np_list(ref))):
            assert np.linalg.norm(g - o) <= 1e-12 * np.linalg.norm(o), (w.name, l)


@pytest.mark.parametrize("case", sorted(CASES))
def test_composite_residual_operator(case):
    """amrmg_residual (the FP64 outer-residual kernels) equals the oracle's
    Alg. 1 residual for arbitrary phi, element by element."""
    print("case", case, flush=True)
    w = CASES[case]()
    H = O.hierarchy_from_workload(w)
    ctx, _ = make_ctx(w)
    rng = np.random.default_rng(3)
    phi = [rng.standard_normal(H.ncells(l)) for l in range(H.nlev)]
    rho = [rng.standard_normal(H.ncells(l)) for l in range(H.nlev)]
    r_or = H.residual(rho, phi)
    r_gpu = np_list(ctx.residual([torch.as_tensor(a, device="cuda") for a in rho],
                                 [torch.as_tensor(a, device="cuda") for a in phi]))
    for l in range(H.nlev):
        scale = np.abs(r_or[l]).max()
        assert np.abs(r_gpu[l] - r_or[l]).max() <= 1e-13 * scale, l


@pytest.mark.parametrize("solve_tol", ["tight", "workload"])
@pytest.mark.parametrize("precision,tol_err", [("fp64", 1e-9), ("mixed", 1e-8)])
@pytest.mark.parametrize("case", sorted(CASES))
def test_solve_matches_oracle(case, precision, tol_err, solve_tol):
    """Solved to 1e-12, and to the workload's own tolerance (1e-8, or 1e-10
    for the sphere), which the error gates must also meet."""
    print("case", case, precision, solve_tol, flush=True)
    w = CASES[case]()
    H, orho, ophi, oE, ost = oracle_solution(w, case)
    ctx, (x, y, z, q) = make_ctx(w, precision=precision)
    rho, _ = ctx.deposit(x, y, z, q)
    phi, E, st = ctx.solve(rho, tol=1e-12 if solve_tol == "tight" else w.tol)
    print(st, flush=True)
    assert st["converged"]
    err = rel_l2_composite(H, np_list(phi), ophi)
    print("rel L2 phi", err, flush=True)
    assert err <= tol_err
    # E on every cell of every level, relative to the field's max
    gE = np_list(E)
    for l in range(H.nlev):
        for d in range(3):
            o = oE[3 * l + d]
            assert np.abs(gE[3 * l + d] - o).max() <= 20 * tol_err * np.abs(o).max(), (l, d)
    Ex, Ey, Ez = ctx.gather(x, y, z, E)
    oEx, oEy, oEz = H.gather(w.particles, oE)
    for g, o in zip((Ex, Ey, Ez), (oEx, oEy, oEz)):
        g = g.cpu().numpy()
        assert np.abs(g - o).max() <= 20 * tol_err * np.abs(o).max()


@pytest.mark.parametrize("smoother,nu", [("jacobi", 3), ("gsrb_global", 2), ("gsrb", 3), ("gsrb", 1)])
def test_other_smoothers_converge_to_same(smoother, nu):
    """Damped Jacobi, whole-level red-black and the brick-hybrid default with
    odd sweep counts all reach the same composite solution."""
    print("case", smoother, nu, flush=True)
    w = W.config1()
    H, orho, ophi, oE, ost = oracle_solution(w, "c1")
    ctx, (x, y, z, q) = make_ctx(w, precision="mixed", smoother=smoother, nu1=nu, nu2=nu, max_iters=200)
    rho, _ = ctx.deposit(x, y, z, q)
    phi, E, st = ctx.solve(rho, tol=1e-12)
    print(st, flush=True)
    assert st["converged"], st
    assert rel_l2_composite(H, np_list(phi), ophi) <= 1e-8


@pytest.mark.parametrize("n0,levels", [((16, 16, 16), []), ((24, 24, 24), [(1, 16, 16, 16, 32, 32, 32)]),
                                       ((16, 24, 32), [(1, 8, 16, 24, 24, 32, 40)]),
                                       ((8, 8, 8), [(1, 0, 0, 0, 8, 8, 8), (2, 0, 0, 0, 8, 8, 8)]),
                                       ((32, 32, 24), [(1, 8, 8, 8, 40, 40, 32)]),
                                       ((72, 72, 72), []), ((72, 120, 88), [])])
def test_small_and_ragged_hierarchies(n0, levels):
    """Single level; bases solved directly without multigrid levels below them
    (24^3, 32 x 32 x 24, and coarsest grids above 64 cells per edge whose
    transforms take several tiles per wavefront and several column chunks:
    72^3, 72 x 120 x 88); unequal edges (anisotropic spacing); a corner box
    touching the boundary on two refined levels over an 8^3 base.  Each with
    the automatic bottom solver (direct) and with CG forced."""
    print("case", n0, levels, flush=True)
    p = W.gaussian_bunch(20000, centre=(0.45, 0.5, 0.55), sigma=(0.12, 0.1, 0.15), seed=77)
    w = W.Workload("edge", p, n0, len(set(b[0] for b in levels)), [], [(1.0, 0.3, 0.6, 0.5)], 1e-10,
                   explicit_boxes=levels or None)
    H, orho, ophi, oE, ost = oracle_solution(w, ("edge", n0, tuple(levels)))
    for precision in ("fp64", "mixed"):
        for bottom in ("auto", "cg"):
            print("  ", precision, bottom, flush=True)
            ctx, (x, y, z, q) = make_ctx(w, precision=precision, bottom=bottom)
            rho, _ = ctx.deposit(x, y, z, q)
            for l, (g, o) in enumerate(zip(np_list(rho), orho)):
                assert np.linalg.norm(g - o) <= 1e-12 * np.linalg.norm(o)
            phi, E, st = ctx.solve(rho, tol=1e-12)
            assert st["converged"], st
            assert rel_l2_composite(H, np_list(phi), ophi) <= (1e-9 if precision == "fp64" else 1e-8)


def test_status_codes():
    A = amr()
    w = W.config1(n_particles=2000)
    ctx, (x, y, z, q) = make_ctx(w, precision="fp64", max_iters=1)
    rho, _ = ctx.deposit(x, y, z, q)
    phi, E, st = ctx.solve(rho, tol=1e-12)
    assert st["status"] == A.AMRMG_E_NOT_CONVERGED and st["iters"] == 1 and not st["converged"]
    # explicit box not properly nested: a level-2 box touching level 1's edge
    prm = A.make_params(w.n0, max_level=2, monopoles=w.monopoles)
    c2 = A.Context(prm)
    with pytest.raises(A.AmrmgError) as ei:
        c2.build_hierarchy(x, y, z, q, explicit_boxes=[(1, 16, 16, 16, 48, 48, 48), (2, 32, 32, 32, 48, 48, 48)])
    assert ei.value.status == A.AMRMG_E_NESTING
    fresh = A.Context(prm)
    with pytest.raises(A.AmrmgError) as ei:
        A.amrmg_solve(fresh.h, [rho[0]], [phi[0]], None, 1e-8)
    assert ei.value.status == A.AMRMG_E_STATE
    with pytest.raises(A.AmrmgError) as ei:
        A.amrmg_deposit_built(fresh.h, [rho[0]])
    assert ei.value.status == A.AMRMG_E_STATE
    # particles outside the domain are counted and skipped
    xo = x.clone()
    xo[:5] = 1.5
    _, nout = ctx.deposit(xo, y, z, q)
    assert nout == 5
