"""Pins of the oracle front end's composite-cell bookkeeping, used by every
parity comparison (Sec. 5.3: the composite domain is the uncovered part of
each level):

  * covered_mask agrees with a brute-force lookup of each cell's first child
    in the next level (hierarchies with several boxes, three levels, boxes
    touching the boundary);
  * composite_rel_l2 weights a cell by its volume (a level-1 cell counts 1/8
    of a level-0 cell), ignores covered cells, and is relative to the
    reference's own weighted norm."""
import numpy as np
import pytest

from oracle import oracle as O

HIERS = {
    "lshape_3lev": ((32, 32, 32), [[(16, 16, 16, 40, 32, 48), (16, 32, 16, 32, 48, 32), (40, 16, 24, 48, 24, 40)],
                                   [(40, 40, 40, 56, 56, 56), (56, 40, 40, 64, 48, 48)]]),
    "touch_boundary": ((16, 24, 16), [[(0, 8, 8, 16, 24, 16), (16, 8, 8, 24, 16, 24), (24, 40, 0, 32, 48, 8)]]),
}


def make(name):
    n0, levels = HIERS[name]
    H = O.OracleHierarchy(n0)
    for l, boxes in enumerate(levels):
        H.set_level(l + 1, boxes)
    return H


@pytest.mark.parametrize("name", sorted(HIERS))
def test_covered_mask_brute_force(name):
    H = make(name)
    for l in range(H.nlev):
        ijk = H.cell_indices(l)
        if l + 1 < H.nlev:
            ref = np.array([H.cell_index(l + 1, 2 * i, 2 * j, 2 * k) >= 0 for i, j, k in ijk])
        else:
            ref = np.zeros(len(ijk), dtype=bool)
        got = H.covered_mask(l)
        assert got.dtype == bool and got.shape == ref.shape
        assert np.array_equal(got, ref), (name, l)
        if l + 1 < H.nlev:
            assert 0 < ref.sum() < len(ref)


def test_composite_rel_l2_weights():
    H = O.OracleHierarchy((16, 16, 16))
    H.set_level(1, [(8, 8, 8, 24, 24, 24)])
    ref = [np.ones(H.ncells(0)), np.ones(H.ncells(1))]
    cov = H.covered_mask(0)
    unc0, unc1 = np.flatnonzero(~cov), np.arange(H.ncells(1))
    v0, v1 = 1.0 / 16 ** 3, 1.0 / 32 ** 3
    den = np.sqrt(v0 * len(unc0) + v1 * len(unc1))
    # a unit error on one uncovered level-0 cell vs one level-1 cell: ratio sqrt(8)
    a = [r.copy() for r in ref]
    a[0][unc0[5]] += 1.0
    e0 = H.composite_rel_l2(a, ref)
    b = [r.copy() for r in ref]
    b[1][unc1[7]] += 1.0
    e1 = H.composite_rel_l2(b, ref)
    assert abs(e0 - np.sqrt(v0) / den) <= 1e-15 * e0
    assert abs(e1 - np.sqrt(v1) / den) <= 1e-15 * e1
    assert abs(e0 / e1 - np.sqrt(8.0)) <= 1e-12
    # covered cells do not count
    c = [r.copy() for r in ref]
    c[0][np.flatnonzero(cov)] += 100.0
    assert H.composite_rel_l2(c, ref) == 0.0
    # per-component arrays (E[3 l + d])
    E = [np.ones(H.ncells(l)) for l in range(2) for _ in range(3)]
    F = [e.copy() for e in E]
    F[3 * 1 + 2][unc1[0]] += 1.0
    assert abs(H.composite_rel_l2(F, E, ncomp=3) - np.sqrt(v1) / (np.sqrt(3) * den)) <= 1e-15
