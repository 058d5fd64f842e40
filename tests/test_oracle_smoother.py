"""Pin of the oracle's smoother (Sec. 5.3, the Gauss-Seidel smoothing of
Alg. 3) on the CPU: one update of one cell, every other value fixed, must
leave that cell's residual of the no-finer-level operator (homogeneous
boundary data, zero coarse data) at zero.  The residual is evaluated by the
operator itself, so a wrong diagonal term of any kind of face -- interior,
coarse-fine, Dirichlet or Robin boundary -- leaves a residual of the order
of the one before the update.  Cells checked: every boundary cell (faces,
edges, corners) and every coarse-fine cell of a fine box that touches the
physical boundary, on anisotropic spacings, for Dirichlet and for the Robin
condition with several distances."""
import numpy as np
import pytest

from oracle import oracle as O


def hier(robin):
    # level 0 anisotropic (h = 1/16, 1.2/24, 0.6/8); level 1 box touches x = lo and z = hi
    H = O.OracleHierarchy((16, 24, 8), lo=(0.0, -0.2, 0.4), hi=(1.0, 1.0, 1.0), robin=robin)
    H.set_level(1, [(0, 8, 0, 16, 32, 16), (16, 8, 8, 24, 16, 16)])
    return H


def selected_cells(H, l):
    ijk = H.cell_indices(l)
    n = np.asarray(H.n0) * 2 ** l
    bnd = np.any((ijk == 0) | (ijk == n - 1), axis=1)
    sel = bnd.copy()
    if l > 0:
        # cells with a face on the coarse-fine interface
        for d in range(3):
            for s in (-1, 1):
                p = ijk.copy()
                p[:, d] += s
                inside = (p[:, d] >= 0) & (p[:, d] < n[d])
                cf = np.array([ok and H.cell_index(l, *q) < 0 for ok, q in zip(inside, p)])
                sel |= cf
    return ijk[sel], bnd


@pytest.mark.parametrize("robin", [0.0, 0.05, 1.7, 30.0])
@pytest.mark.parametrize("level", [0, 1])
def test_one_update_zeroes_the_cell_residual(robin, level):
    H = hier(robin)
    rng = np.random.default_rng(17 + level)
    n = H.ncells(level)
    e = rng.standard_normal(n)
    r = rng.standard_normal(n) * 1e3
    cells, _ = selected_cells(H, level)
    assert len(cells) > 50
    before, after = [], []
    for (i, j, k) in cells[:: max(1, len(cells) // 400)]:
        c = H.cell_index(level, i, j, k)
        e2 = H.relax_point(level, i, j, k, e, r)
        changed = np.flatnonzero(e2 != e)
        assert set(changed.tolist()) <= {c}
        res0 = r[c] - H.apply_nf(level, e)[c]
        res1 = r[c] - H.apply_nf(level, e2)[c]
        before.append(abs(res0))
        after.append(abs(res1))
    scale = np.max(before)
    assert scale > 1.0
    assert np.max(after) <= 1e-12 * scale, (robin, level, np.max(after), scale)


def test_robin_and_dirichlet_updates_differ_on_boundary_cells():
    """The same cell, data and neighbours give different updates under the
    two boundary conditions (the pin above sees the boundary term)."""
    Hd, Hr = hier(0.0), hier(1.7)
    rng = np.random.default_rng(3)
    n = Hd.ncells(0)
    e = rng.standard_normal(n)
    r = rng.standard_normal(n)
    a = Hd.relax_point(0, 0, 5, 3, e, r)
    b = Hr.relax_point(0, 0, 5, 3, e, r)
    c = Hd.cell_index(0, 0, 5, 3)
    assert abs(a[c] - b[c]) > 1e-3 * abs(a[c] - e[c])
    # an interior cell away from every boundary updates identically
    a = Hd.relax_point(0, 5, 5, 3, e, r)
    b = Hr.relax_point(0, 5, 5, 3, e, r)
    assert np.array_equal(a, b)
