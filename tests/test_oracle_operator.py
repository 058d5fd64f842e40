"""Pins of the oracle's composite operator (arXiv:1812.03689 Sec. 5.1, Eqs.
lap_flux_differencing, coarse_fluxes, flux_differencing; Sec. 5.3 composite
domain) by properties the mathematics fixes:
  * exactness on quadratics away from the physical boundary (flux matching
    plus second-order ghosts);
  * covered coarse values are never read;
  * conservation: interior and coarse-fine fluxes telescope to the
    boundary flux;
  * the single-level operator is symmetric;
  * central-difference fields are exact on quadratics.
"""
import numpy as np
import pytest

HIERS = {
    "centred": ((16, 16, 16), [[(8, 8, 8, 24, 24, 24)]]),
    "lshape_3lev": ((32, 32, 32), [[(16, 16, 16, 40, 32, 48), (16, 32, 16, 32, 48, 32), (40, 16, 24, 48, 24, 40)],
                                   [(40, 40, 40, 56, 56, 56), (56, 40, 40, 64, 48, 48)]]),
    "touch_boundary": ((16, 16, 16), [[(0, 8, 8, 16, 24, 16), (16, 8, 8, 24, 16, 24)]]),
    "aniso_base": ((16, 24, 32), [[(8, 16, 16, 24, 32, 48)]]),
}


def make(O, name):
    n0, levels = HIERS[name]
    H = O.OracleHierarchy(n0)
    for l, boxes in enumerate(levels):
        H.set_level(l + 1, boxes)
    return H


def quad(a):
    def f(x, y, z):
        return (a[0] + a[1] * x + a[2] * y + a[3] * z + a[4] * x * x + a[5] * y * y + a[6] * z * z
                + a[7] * x * y + a[8] * y * z + a[9] * x * z)
    return f


@pytest.mark.parametrize("name", sorted(HIERS))
def test_quadratic_exactness(oracle_lib, name):
    O = oracle_lib
    H = make(O, name)
    rng = np.random.default_rng(11)
    a = rng.standard_normal(10)
    f = quad(a)
    phi = [f(*H.cell_centres(l)) for l in range(H.nlev)]
    A = H.apply_composite(phi)
    exact = -2 * (a[4] + a[5] + a[6])
    for l in range(H.nlev):
        ijk = H.cell_indices(l)
        n = np.asarray(H.n0) * 2 ** l
        inner = np.all((ijk > 0) & (ijk < n - 1), axis=1) & ~H.covered_mask(l)
        assert inner.sum() > 0
        scale = 1.0 / H.spacing(l).min() ** 2
        assert np.abs(A[l][inner] - exact).max() < 1e-14 * scale * 10, (name, l)


def test_quadratic_pin_is_sensitive(oracle_lib):
    """The exactness pin reacts to a small error in the coarse data the
    fine-side ghosts read: a bump of 1e-3 on one uncovered coarse cell next
    to the fine box moves the fine operator by O(1e-3 / h^2)."""
    O = oracle_lib
    H = make(O, "centred")
    a = np.random.default_rng(3).standard_normal(10)
    f = quad(a)
    phi = [f(*H.cell_centres(l)) for l in range(H.nlev)]
    ph2 = [p.copy() for p in phi]
    c = H.cell_index(0, 3, 8, 8)  # fine box covers coarse [4, 12)^3
    ph2[0][c] += 1e-3
    A = H.apply_composite(ph2)
    exact = -2 * (a[4] + a[5] + a[6])
    assert np.abs(A[1] - exact).max() > 0.1  # 8/15 * (15/16)^2 * 1e-3 / h_f^2 = 0.48


def test_covered_values_never_read(oracle_lib):
    O = oracle_lib
    H = make(O, "lshape_3lev")
    rng = np.random.default_rng(2)
    phi = [rng.standard_normal(H.ncells(l)) for l in range(H.nlev)]
    A1 = H.apply_composite(phi, inhom=False)
    phi2 = [p.copy() for p in phi]
    for l in range(H.nlev):
        cm = H.covered_mask(l)
        phi2[l][cm] = 1e3 * rng.standard_normal(cm.sum())
    A2 = H.apply_composite(phi2, inhom=False)
    for x, y in zip(A1, A2):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("name", ["centred", "lshape_3lev", "touch_boundary"])
def test_conservation(oracle_lib, name):
    """sum over uncovered cells of vol * (A u) equals the flux through the
    physical boundary, sum of area * 2 u_c / h (homogeneous Dirichlet ghost):
    all same-level and coarse-fine fluxes cancel."""
    O = oracle_lib
    H = make(O, name)
    rng = np.random.default_rng(4)
    u = [rng.standard_normal(H.ncells(l)) for l in range(H.nlev)]
    A = H.apply_composite(u, inhom=False)
    S, B = 0.0, 0.0
    for l in range(H.nlev):
        h = H.spacing(l)
        vol = h.prod()
        unc = ~H.covered_mask(l)
        S += vol * A[l][unc].sum()
        ijk = H.cell_indices(l)
        n = np.asarray(H.n0) * 2 ** l
        for d in range(3):
            area = vol / h[d]
            for side in (ijk[:, d] == 0, ijk[:, d] == n[d] - 1):
                m = side & unc
                B += area * 2.0 * u[l][m].sum() / h[d]
    assert abs(S - B) < 1e-12 * max(1.0, abs(B)) * 1e3


def test_single_level_operator_symmetric(oracle_lib):
    O = oracle_lib
    H = O.OracleHierarchy((8, 8, 8))
    n = H.ncells(0)
    A = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        A[:, j] = H.apply_nf(0, e)
    assert np.abs(A - A.T).max() <= 1e-15 * np.abs(A).max()
    assert np.all(np.linalg.eigvalsh(0.5 * (A + A.T)) > 0)


@pytest.mark.parametrize("name", ["centred", "lshape_3lev"])
def test_efield_exact_on_quadratics(oracle_lib, name):
    O = oracle_lib
    H = make(O, name)
    a = np.random.default_rng(8).standard_normal(10)
    f = quad(a)
    phi = [f(*H.cell_centres(l)) for l in range(H.nlev)]
    E = H.efield(phi)
    for l in range(H.nlev):
        x, y, z = H.cell_centres(l)
        grad = [a[1] + 2 * a[4] * x + a[7] * y + a[9] * z,
                a[2] + 2 * a[5] * y + a[7] * x + a[8] * z,
                a[3] + 2 * a[6] * z + a[8] * y + a[9] * x]
        ijk = H.cell_indices(l)
        n = np.asarray(H.n0) * 2 ** l
        inner = np.all((ijk > 0) & (ijk < n - 1), axis=1)
        for d in range(3):
            assert np.abs(E[3 * l + d][inner] + grad[d][inner]).max() < 1e-11


def test_average_down_is_child_mean(oracle_lib):
    O = oracle_lib
    H = make(O, "lshape_3lev")
    rng = np.random.default_rng(1)
    phi = [rng.standard_normal(H.ncells(l)) for l in range(H.nlev)]
    out = H.average_down(phi)
    # a covered cell of level 1 becomes the mean of its 8 children
    ijk = H.cell_indices(1)
    cm = H.covered_mask(1)
    t = np.flatnonzero(cm)[7]
    i, j, k = ijk[t]
    kids = [out[2][H.cell_index(2, 2 * i + a, 2 * j + b, 2 * k + c)]
            for a in (0, 1) for b in (0, 1) for c in (0, 1)]
    assert out[1][t] == pytest.approx(np.mean(kids), rel=1e-15)
    assert np.array_equal(out[1][~cm], phi[1][~cm])
    const = [np.full(H.ncells(l), 2.5) for l in range(H.nlev)]
    for v in H.average_down(const):
        assert np.all(v == 2.5)
