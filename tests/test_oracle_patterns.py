"""Pins of the coarse-fine interpolation patterns (arXiv:1812.03689 Sec. 5.1,
Eq. 2d_lagrange, Fig. of the nine quadratic configurations, Tab. bit_pattern
and the bilinear table) against what the paper prints and what Lagrange
interpolation fixes."""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.filterwarnings("ignore")

GOLD = os.path.join(os.path.dirname(__file__), "golden", "cf_patterns.json")


def _gold():
    with open(GOLD) as f:
        return json.load(f)


def _window_int(ent, side):
    v = 0
    for j in range(ent["j"][0], ent["j"][1] + 1):
        for i in range(ent["i"][0], ent["i"][1] + 1):
            v |= 1 << (i + side * j)
    return v


def test_printed_integers_are_the_drawn_windows():
    g = _gold()
    for ent in g["quadratic"]:
        assert _window_int(ent, 5) == ent["value"], ent
    for ent in g["linear"]:
        assert _window_int(ent, 3) == ent["value"], ent
    # the bit strings of the table, most significant bit first
    bs = g["bit_strings_msb_first"]
    assert int(bs["0"], 2) == g["quadratic"][0]["value"]
    assert int(bs["1"], 2) == g["quadratic"][1]["value"]
    assert int(bs["8"], 2) == g["quadratic"][8]["value"]
    assert int(bs["linear0"], 2) == g["linear"][0]["value"]


def test_selection_follows_printed_order(oracle_lib):
    O = oracle_lib
    g = _gold()
    full = (1 << 25) - 1
    assert O.select_pattern(full) == 0
    for ent in g["quadratic"]:
        assert O.select_pattern(ent["value"]) == ent["case"]
    # a fine region on the +v side (rows j = 3, 4 covered) -> shift towards -v
    m = full
    for i in range(5):
        for j in (3, 4):
            m &= ~(1 << (i + 5 * j))
    assert O.select_pattern(m) == 1
    # covered quadrant (+u, +v) of the inner 3x3: centred window fails, the
    # first listed window that fits is the -v shift
    m = full & ~(1 << (3 + 5 * 3)) & ~(1 << (4 + 5 * 3)) & ~(1 << (3 + 5 * 4)) & ~(1 << (4 + 5 * 4))
    assert O.select_pattern(m) == 1
    # bilinear fallback: only the (-u,-v) 2x2 block of the inner layer
    lin0 = (1 << (1 + 5 * 1)) | (1 << (2 + 5 * 1)) | (1 << (1 + 5 * 2)) | (1 << (2 + 5 * 2))
    assert O.select_pattern(lin0) == 9
    lin2 = (1 << (2 + 5 * 2)) | (1 << (3 + 5 * 2)) | (1 << (2 + 5 * 3)) | (1 << (3 + 5 * 3))
    assert O.select_pattern(lin2) == 11
    # paper order ignores the quadrant: with both (-u,+v) and (+u,+v) blocks
    # available, the earlier listed one wins
    both = lin2 | (1 << (1 + 5 * 2)) | (1 << (1 + 5 * 3))
    assert O.select_pattern(both) == 10
    assert O.select_pattern(1 << 12) == 13


def _layer(fun):
    L = np.zeros((5, 5))
    for j in range(5):
        for i in range(5):
            L[j, i] = fun(i - 2, j - 2)
    return L


@pytest.mark.parametrize("tu,tv", [(-0.25, -0.25), (0.25, -0.25), (-0.25, 0.25), (0.25, 0.25)])
def test_step1_exact_on_polynomials(oracle_lib, tu, tv):
    O = oracle_lib
    g = _gold()
    rng = np.random.default_rng(5)
    for ent in g["quadratic"]:
        c = rng.standard_normal((3, 3))
        f = lambda u, v: sum(c[a, b] * u ** a * v ** b for a in range(3) for b in range(3))
        val, pat = O.step1_layer(ent["value"], _layer(f), tu, tv)
        assert pat == ent["case"]
        assert abs(val - f(tu, tv)) < 1e-13 * (1 + abs(f(tu, tv)))
    for ent in g["linear"]:
        c = rng.standard_normal((2, 2))
        f = lambda u, v: sum(c[a, b] * u ** a * v ** b for a in range(2) for b in range(2))
        m5 = 0
        for j in range(3):
            for i in range(3):
                if ent["value"] & (1 << (i + 3 * j)):
                    m5 |= 1 << ((i + 1) + 5 * (j + 1))
        val, pat = O.step1_layer(m5, _layer(f), tu, tv)
        assert pat == 9 + ent["case"]
        assert abs(val - f(tu, tv)) < 1e-13 * (1 + abs(f(tu, tv)))
    val, pat = O.step1_layer(1 << 12, _layer(lambda u, v: 3.25), tu, tv)
    assert pat == 13 and val == 3.25


def test_step1_closed_form_weights(oracle_lib):
    """Centred nodes {-1,0,1} at +1/4: (-3/32, 15/16, 5/32); nodes {0,1,2} at
    +1/4: (21/32, 7/16, -3/32)."""
    O = oracle_lib
    full = (1 << 25) - 1
    wc = {-1: -3 / 32, 0: 15 / 16, 1: 5 / 32}
    for a in (-1, 0, 1):
        for b in (-1, 0, 1):
            lay = _layer(lambda u, v: 1.0 if (u, v) == (a, b) else 0.0)
            val, _ = O.step1_layer(full, lay, 0.25, 0.25)
            assert val == pytest.approx(wc[a] * wc[b], abs=1e-15)
    ws = {0: 21 / 32, 1: 7 / 16, 2: -3 / 32}
    p4 = 947072  # +u shift: u nodes {0,1,2}, v nodes {-1,0,1}
    for a in (0, 1, 2):
        lay = _layer(lambda u, v: 1.0 if (u, v) == (a, 0) else 0.0)
        val, pat = O.step1_layer(p4, lay, 0.25, 0.25)
        assert pat == 4
        assert val == pytest.approx(ws[a] * wc[0], abs=1e-15)


def test_step2_weights_through_operator(oracle_lib):
    """Along the normal, nodes at -3/2 h, -1/2 h (fine) and +h (coarse centre)
    evaluated at +h/2 give (-1/5, 2/3, 8/15).  Read through the fine operator
    at a cell on the face of a fine box: the CF face adds (1 - 2/3)/h^2 to the
    diagonal, +1/5 / h^2 to the inner neighbour's -1/h^2, and -8/15 times the
    step-1 weight to the coarse centre."""
    O = oracle_lib
    H = O.OracleHierarchy((16, 16, 16))
    H.set_level(1, [(8, 8, 8, 24, 24, 24)])
    h = H.spacing(1)[0]
    # fine cell on the -x face of the fine box, away from edges
    i, j, k = 8, 13, 14
    c = H.cell_index(1, i, j, k)
    cin = H.cell_index(1, i + 1, j, k)
    n1 = H.ncells(1)
    u = np.zeros(n1)
    u[c] = 1.0
    A = H.apply_nf(1, u)
    assert A[c] * h * h == pytest.approx(5 + 1 / 3, rel=1e-14)
    u = np.zeros(n1)
    u[cin] = 1.0
    A = H.apply_nf(1, u)
    assert A[c] * h * h == pytest.approx(-1 + 1 / 5, rel=1e-14)
    # coarse centre of the ghost's layer: ghost at fine (7, 13, 14) -> coarse (3, 6, 7)
    uc = np.zeros(H.ncells(0))
    uc[H.cell_index(0, 3, 6, 7)] = 1.0
    A = H.apply_nf(1, np.zeros(n1), uc)
    # transverse offsets of fine (13, 14) in coarse (6, 7): +1/4 along y, -1/4 along z
    assert A[c] * h * h == pytest.approx(-(8 / 15) * (15 / 16) * (15 / 16), rel=1e-14)
    pat, _ = H.cf_pattern(1, i, j, k, 0, -1)
    assert pat == 0
