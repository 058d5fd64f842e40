"""Pins of the oracle's potential and electric-field refinement criteria
(Sec. 4.2; ``oracle.field_tags``) on the CPU, against the closed-form fields
of a uniformly charged ball (charge Q, radius R, Dirichlet data from the
exact exterior potential):

    phi(r) = Q (3R^2 - r^2) / (8 pi R^3) inside,  Q / (4 pi r) outside;
    E(x)   = Q (x - c) / (4 pi R^3) inside,       Q (x - c) / (4 pi r^3) outside.

With lambda = 1/2 the potential criterion tags exactly the cells with
r < 4R/3 (where phi falls to half its central value), and the field
criterion tags a cell when some component |E_w| exceeds half of that
component's maximum over the level; per component, not the magnitude: at
45 degrees in a coordinate plane the two differ between r = 2^(1/4) R and
sqrt(2) R.  Cells within a band around each decision surface (the discrete
solution carries O(h^2) error and particle noise) are not compared; the band
is a few percent, far smaller than the gaps that a wrong exponent, a
magnitude instead of components, or a missing absolute value would open.
The criteria are also invariant under the sign and size of the charge."""
import functools

import numpy as np
import pytest

from oracle import oracle as O
from paper_1812_03689_amd import workloads as W

R = 0.2
N0 = 48


@functools.lru_cache(maxsize=None)
def tags_of(Q, policy):
    p = W.uniform_ball(200000, radius=R, seed=W.seed_for(9, 1), total_charge=Q)
    H = O.OracleHierarchy((N0, N0, N0), monopoles=[(Q, 0.5, 0.5, 0.5)])
    return O.field_tags(H, 0, p, policy, 0.5)


def centres():
    i = (np.arange(N0) + 0.5) / N0 - 0.5
    z, y, x = np.meshgrid(i, i, i, indexing="ij")  # x fastest in the flat layout
    return x.ravel(), y.ravel(), z.ravel()


@pytest.mark.parametrize("Q", [1.0, -2.0])
def test_potential_criterion_is_the_ball_of_radius_4R_over_3(Q):
    tags = tags_of(Q, "potential")
    x, y, z = centres()
    r = np.sqrt(x * x + y * y + z * z)
    h = 1.0 / N0
    inner, outer = r < 4 * R / 3 - 0.5 * h, r > 4 * R / 3 + 0.5 * h
    assert inner.sum() > 500 and outer.sum() > 20000
    assert np.all(tags[inner] == 1)
    assert np.all(tags[outer] == 0)


@pytest.mark.parametrize("Q", [1.0, -2.0])
def test_field_criterion_per_component(Q):
    tags = tags_of(Q, "efield")
    x, y, z = centres()
    r = np.sqrt(x * x + y * y + z * z)
    scale = np.where(r <= R, 1.0 / R ** 3, 1.0 / np.maximum(r, 1e-300) ** 3)
    comp = np.abs(np.stack([x, y, z])) * scale  # |E_w| up to the common factor |Q| / (4 pi)
    ratio = (comp / comp.max(axis=1, keepdims=True)).max(axis=0) / 0.5
    sure_in, sure_out = ratio > 1.1, ratio < 0.9
    assert sure_in.sum() > 300 and sure_out.sum() > 20000
    assert np.all(tags[sure_in] == 1)
    assert np.all(tags[sure_out] == 0)
    # where the magnitude criterion and the per-component one disagree, the
    # components decide: cells near 45 degrees in a coordinate plane with
    # r near 1.3 R (component ratio below 0.9 there, magnitude ratio above 1.1)
    mag = np.sqrt((comp ** 2).sum(axis=0))
    mag_ratio = mag / mag.max() / 0.5
    split = sure_out & (mag_ratio > 1.1)
    assert split.sum() > 0
    assert np.all(tags[split] == 0)


@pytest.mark.parametrize("policy", ["potential", "efield"])
def test_field_tags_of_a_scaled_problem_are_unchanged(policy):
    assert np.array_equal(tags_of(1.0, policy), tags_of(-2.0, policy))
