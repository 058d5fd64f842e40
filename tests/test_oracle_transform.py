"""Pins of the domain-transform oracle (oracle/transform.py, Sec. 4.1 of the
paper) on the CPU: a hand-worked example of Gamma and s, the outermost
particle landing on the boundary of the computation space, and the physics
the transform must preserve: one problem solved by the composite oracle in
particle space and again in computation space gives the same potential after
phi = phi*/s and the same field after E = E*/s^2 (the exponents follow from
the scaling of the Laplacian, the charge density and the Dirichlet data; a
wrong exponent is off by a factor s)."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import transform as T
from paper_1812_03689_amd import workloads as W


def test_gamma_and_scale_by_hand():
    c, l = (1.0, -2.0, 0.5), (0.1, 1.0, 2.0)
    x = np.array([1.3, 1.0, 1.0, 0.95])
    y = np.array([-2.0, -2.5, -2.0, -2.0])
    z = np.array([0.5, 0.5, 5.5, 0.5])
    # |0.3|/0.1 = 3, |-0.5|/1 = 0.5, |5|/2 = 2.5, |-0.05|/0.1 = 0.5
    assert np.allclose(T.gamma(x, y, z, c, l), [3.0, 0.5, 2.5, 0.5], rtol=1e-15)
    s = T.domain_scale(x, y, z, c, l)
    assert abs(s - 3.0) <= 4e-16 * 3
    xs, ys, zs = T.to_computation(x, y, z, c, s)
    assert np.allclose(xs, [0.1, 0.0, 0.0, -0.05 / 3], rtol=1e-14, atol=1e-17)
    assert np.allclose(zs, [0.0, 0.0, 5.0 / 3, 0.0], rtol=1e-14)
    assert T.domain_scale(x[:0], y[:0], z[:0], c, l) == 0.0


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_outermost_particle_on_the_boundary(dtype):
    rng = np.random.default_rng(3)
    n = 5000
    c, l = (0.3, -0.1, 2.0), (0.5, 0.25, 1.0)
    x, y, z = (rng.normal(c[d], 0.01 * (d + 1), n).astype(dtype) for d in range(3))
    s = T.domain_scale(x, y, z, c, l)
    xs, ys, zs = T.to_computation(x, y, z, c, s)
    assert xs.dtype == dtype
    g = T.gamma(xs, ys, zs, (0, 0, 0), l)
    eps = 8 * np.finfo(dtype).eps
    assert g.max() <= 1 + eps and g.max() >= 1 - eps
    assert np.all(g <= 1 + eps)


def _bunch_problem(scale, centre, lo, hi, mono_at):
    p = W.gaussian_bunch(3000, sigma=(0.05, 0.05, 0.1), seed=W.seed_for(7, 1))
    X = [centre[d] + scale * (a - 0.5) for d, a in enumerate((p.x, p.y, p.z))]
    parts = W.Particles(X[0], X[1], X[2], p.q.copy())
    return W.Workload("bunch", parts, (16, 16, 16), 1, [1e-2], [(1.0, *mono_at)], 1e-10, lo=lo, hi=hi)


def test_solution_invariant_under_the_transform():
    """Same discrete problem in S_p (domain centre +- scale/2, metres) and in
    S_c (the same cells after x* = (x - c)/s): phi_p = phi*/s, E_p = E*/s^2."""
    centre, scale = (0.3, -0.1, 2.0), 0.02
    lo_p = tuple(centre[d] - scale / 2 for d in range(3))
    hi_p = tuple(centre[d] + scale / 2 for d in range(3))
    wp = _bunch_problem(scale, centre, lo_p, hi_p, centre)
    p = wp.particles
    s = T.domain_scale(p.x, p.y, p.z, centre, (1.0, 1.0, 1.0))
    assert 0 < s < scale  # a real change of scale
    xs, ys, zs = T.to_computation(p.x, p.y, p.z, centre, s)
    lo_c = tuple((lo_p[d] - centre[d]) / s for d in range(3))
    hi_c = tuple((hi_p[d] - centre[d]) / s for d in range(3))
    wc = W.Workload("bunch_c", W.Particles(xs, ys, zs, p.q.copy()), wp.n0, 1, [1e-2], [(1.0, 0.0, 0.0, 0.0)], 1e-10,
                    lo=lo_c, hi=hi_c)
    Hp, Hc = O.hierarchy_from_workload(wp), O.hierarchy_from_workload(wc)
    assert Hp.nlev == Hc.nlev == 2
    for l in range(Hp.nlev):
        assert np.array_equal(Hp.boxes(l)[0], Hc.boxes(l)[0])
    php, Ep, _ = Hp.solve(Hp.deposit_all(wp.particles), tol=1e-13, max_iters=80, bottom_rtol=1e-14)
    phc, Ec, _ = Hc.solve(Hc.deposit_all(wc.particles), tol=1e-13, max_iters=80, bottom_rtol=1e-14)
    phr, Er = T.rescale(phc, Ec, s)
    for a, b in zip(phr, php):
        assert np.linalg.norm(a - b) <= 1e-10 * np.linalg.norm(b)
    for a, b in zip(Er, Ep):
        assert np.abs(a - b).max() <= 1e-9 * np.abs(b).max()
    # the gather at the transformed positions gives the particle-space field
    gp = np.array(Hp.gather(wp.particles, Ep))
    gc = np.array(Hc.gather(wc.particles, Er))
    assert np.abs(gc - gp).max() <= 1e-9 * np.abs(gp).max()
