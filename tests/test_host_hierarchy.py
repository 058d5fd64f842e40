"""The product's host-side hierarchy code (box generation and coarse-fine
pattern selection, C++ in paper_1812_03689_amd/csrc/amrmg_hier.cpp) against
the oracle: box lists and pattern ids must agree bit for bit.  Runs on the
CPU through a g++-built shim that links only product code."""
import ctypes as C
import json
import os
import subprocess

import numpy as np
import pytest

from paper_1812_03689_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1812_03689_amd", "csrc")


@pytest.fixture(scope="module")
def shim(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("shim") / "libhier_shim.so")
    subprocess.check_call(["g++", "-std=c++17", "-O2", "-fPIC", "-shared", "-I" + CSRC,
                           os.path.join(ROOT, "tests", "native", "hier_shim.cpp"),
                           os.path.join(CSRC, "amrmg_hier.cpp"), "-o", out])
    L = C.CDLL(out)
    L.hs_generate_boxes.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int,
                                    C.c_int, C.c_void_p, C.c_int]
    L.hs_cf_patterns.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_long]
    L.hs_cf_patterns.restype = C.c_long
    L.hs_merge_block_bits.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_int]
    L.hs_tables.argtypes = [C.c_void_p, C.c_void_p]
    L.hs_direct_tables.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_long]
    L.hs_direct_tables.restype = C.c_long
    return L


def product_boxes(shim, H, l, tags, mgs=32):
    b, _ = H.boxes(l)
    b = np.ascontiguousarray(b, dtype=np.int32)
    n = np.asarray(H.n0, dtype=np.int32) * 2 ** l
    out = np.zeros((1 << 16, 6), dtype=np.int32)
    t = np.ascontiguousarray(tags, dtype=np.uint8)
    nb = shim.hs_generate_boxes(n.ctypes.data, b.shape[0], b.ctypes.data, t.ctypes.data, 1, 2, 8, mgs,
                                out.ctypes.data, out.shape[0])
    assert nb >= 0
    return out[:nb]


def product_patterns(shim, H, level):
    n0 = np.asarray(H.n0, dtype=np.int32)
    nbox = np.asarray([H.boxes(l)[0].shape[0] for l in range(H.nlev)], dtype=np.int32)
    boxes = np.ascontiguousarray(np.concatenate([H.boxes(l)[0] for l in range(H.nlev)]), dtype=np.int32)
    cap = 1 << 22
    out = np.zeros((cap, 6), dtype=np.int32)
    k = shim.hs_cf_patterns(n0.ctypes.data, H.nlev, nbox.ctypes.data, boxes.ctypes.data, level,
                            out.ctypes.data, cap)
    return out[:k]


def test_tables_match_printed_integers(shim):
    w = np.zeros(14 * 4 * 9)
    q = np.zeros(9, dtype=np.uint32)
    shim.hs_tables(w.ctypes.data, q.ctypes.data)
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "cf_patterns.json")))
    assert [int(v) for v in q] == [e["value"] for e in gold["quadratic"]]
    W4 = w.reshape(14, 4, 9)
    # each window's weights sum to 8/15 (interpolation of constants)
    assert np.allclose(W4.sum(axis=2), 8 / 15, atol=1e-15)
    # centred window at (+1/4, +1/4): (8/15) (-3/32, 15/16, 5/32)^2 tensor
    c = np.array([-3 / 32, 15 / 16, 5 / 32])
    assert np.allclose(W4[0, 3].reshape(3, 3), (8 / 15) * np.outer(c, c), atol=1e-15)


@pytest.mark.parametrize("cfg", [2, 4])
def test_box_generation_matches_oracle(oracle_lib, shim, cfg):
    O = oracle_lib
    w = W.CONFIGS[cfg]() if cfg != 4 else W.config4(n_per=50000)
    if cfg == 2:
        w = W.config2(n_particles=200000)
    H = O.OracleHierarchy(w.n0, monopoles=w.monopoles)
    for l in range(w.max_level):
        rho, _ = H.deposit(l, w.particles)
        tags = H.tag(l, rho, w.tag_rel[l])
        ob = H.cluster(l, tags, mgs=w.max_grid_size)
        pb = product_boxes(shim, H, l, tags, w.max_grid_size)
        assert np.array_equal(ob, pb), (cfg, l)
        if ob.shape[0] == 0:
            break
        H.set_level(l + 1, ob)
    assert H.nlev == w.max_level + 1


def test_box_generation_random_tags(oracle_lib, shim):
    O = oracle_lib
    rng = np.random.default_rng(12)
    H = O.OracleHierarchy((32, 32, 32))
    H.set_level(1, [(16, 16, 16, 48, 40, 48), (16, 40, 16, 40, 48, 40)])
    for trial in range(5):
        tags = (rng.random(H.ncells(1)) < 0.002 * (trial + 1)).astype(np.uint8)
        assert np.array_equal(H.cluster(1, tags), product_boxes(shim, H, 1, tags))
    for mgs in (8, 16, 24, 32, 64):
        tags = (rng.random(H.ncells(0)) < 0.001).astype(np.uint8)
        assert np.array_equal(H.cluster(0, tags, mgs=mgs), product_boxes(shim, H, 0, tags, mgs))


HIERS = {
    "lshape_3lev": ((32, 32, 32), [[(16, 16, 16, 40, 32, 48), (16, 32, 16, 32, 48, 32), (40, 16, 24, 48, 24, 40)],
                                   [(40, 40, 40, 56, 56, 56), (56, 40, 40, 64, 48, 48)]]),
    "touch_boundary": ((16, 16, 16), [[(0, 8, 8, 16, 24, 16), (16, 8, 8, 24, 16, 24)]]),
    "corner_blocks": ((32, 32, 32), [[(16, 16, 16, 32, 32, 32), (32, 32, 16, 48, 48, 32), (32, 16, 32, 48, 32, 48)]]),
}


def greedy_merge_reference(mask, g, maxb):
    """The greedy merge written out on a byte mask: blocks in linear order (x
    fastest); an available block starts a box that grows along x, then y,
    then z while whole rows (slabs) are available, at most maxb blocks per
    axis; its blocks are then taken."""
    m = mask.reshape(g[2], g[1], g[0]).copy()
    boxes = []
    for z in range(g[2]):
        for y in range(g[1]):
            for x in range(g[0]):
                if m[z, y, x] != 1:
                    continue
                ex = 1
                while x + ex < g[0] and ex < maxb and m[z, y, x + ex] == 1:
                    ex += 1
                ey = 1
                while y + ey < g[1] and ey < maxb and (m[z, y + ey, x:x + ex] == 1).all():
                    ey += 1
                ez = 1
                while z + ez < g[2] and ez < maxb and (m[z + ez, y:y + ey, x:x + ex] == 1).all():
                    ez += 1
                m[z:z + ez, y:y + ey, x:x + ex] = 2
                boxes.append((x, y, z, x + ex, y + ey, z + ez))
    return np.asarray(boxes, dtype=np.int32).reshape(-1, 6)


@pytest.mark.parametrize("g,maxb,fill", [((70, 5, 4), 4, 0.7), ((13, 9, 7), 3, 0.5), ((130, 3, 3), 100, 0.95),
                                          ((64, 4, 2), 64, 1.0), ((1, 1, 1), 4, 1.0), ((33, 17, 5), 8, 0.0)])
def test_bit_array_merge_matches_byte_greedy(shim, g, maxb, fill):
    """The product's greedy merge on a bit array (rows straddling 64-bit
    words, runs longer than a word, ragged and empty masks) against the byte
    greedy written out above."""
    rng = np.random.default_rng(1812 + g[0])
    mask = (rng.random(g[0] * g[1] * g[2]) < fill).astype(np.uint8)
    gg = np.asarray(g, dtype=np.int32)
    out = np.zeros((mask.size + 1, 6), dtype=np.int32)
    nb = shim.hs_merge_block_bits(gg.ctypes.data, mask.ctypes.data, maxb, out.ctypes.data, out.shape[0])
    assert nb >= 0
    ref = greedy_merge_reference(mask, g, maxb)
    assert np.array_equal(out[:nb], ref)
    cover = np.zeros(mask.size, dtype=np.int32)
    for x0, y0, z0, x1, y1, z1 in out[:nb]:
        for z in range(z0, z1):
            for y in range(y0, y1):
                cover[x0 + g[0] * (y + g[1] * z):x1 + g[0] * (y + g[1] * z)] += 1
    assert np.array_equal(cover, mask.astype(np.int32))


@pytest.mark.parametrize("name", sorted(HIERS))
def test_cf_patterns_match_oracle(oracle_lib, shim, name):
    O = oracle_lib
    n0, levels = HIERS[name]
    H = O.OracleHierarchy(n0)
    for l, b in enumerate(levels):
        H.set_level(l + 1, b)
    seen = set()
    for l in range(1, H.nlev):
        rows = product_patterns(shim, H, l)
        assert rows.shape[0] > 0
        for (i, j, k, d, s, pat) in rows:
            op, _ = H.cf_pattern(l, int(i), int(j), int(k), int(d), int(s))
            assert op == pat, (name, l, i, j, k, d, s)
            seen.add(int(pat))
        # every coarse-fine face of the oracle appears exactly once
        count = 0
        for (i, j, k) in H.cell_indices(l):
            for d in range(3):
                for s in (-1, 1):
                    if H.cf_pattern(l, int(i), int(j), int(k), d, s)[0] >= 0:
                        count += 1
        assert count == rows.shape[0]
    assert seen


def dirichlet_laplacian_dense(n, h, abnd=(-1.0, -1.0, -1.0)):
    """-L_h of the 7-point cell-centred Laplacian on one box with homogeneous
    boundary ghosts (ghost = abnd_d u of the boundary cell: -1 is Dirichlet),
    x fastest."""
    nx, ny, nz = n
    N = nx * ny * nz
    A = np.zeros((N, N))
    idx = lambda i, j, k: i + nx * (j + ny * k)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                r = idx(i, j, k)
                for d, (m, hd) in enumerate(zip(n, h)):
                    for s in (-1, 1):
                        c = [i, j, k]
                        c[d] += s
                        A[r, r] += 1.0 / hd ** 2
                        if 0 <= c[d] < m:
                            A[r, idx(*c)] -= 1.0 / hd ** 2
                        else:
                            A[r, r] -= abnd[d] / hd ** 2
    return A


@pytest.mark.parametrize("robin", [None, 1.7, 0.03])
@pytest.mark.parametrize("n,h", [((8, 8, 8), (1 / 8, 1 / 8, 1 / 8)), ((8, 16, 24), (0.1, 0.05, 0.02))])
def test_direct_tables_diagonalise_the_laplacian(shim, n, h, robin):
    """The coarsest-grid direct solve, Dirichlet (sine tables) or Robin
    (Jacobi eigenvectors; ghost (2d - h)/(2d + h) u, Eq. robin_bc by central
    difference): Q diag(lambda) Q^T reproduces the dense operator and Q is
    orthonormal, so Q diag(1/lambda) Q^T r = A^-1 r."""
    n32 = np.asarray(n, dtype=np.int32)
    hh = np.asarray(h, dtype=np.float64)
    ab = np.array([-1.0] * 3 if robin is None else [(2 * robin - hd) / (2 * robin + hd) for hd in h])
    out = np.zeros(1 << 16)
    k = shim.hs_direct_tables(n32.ctypes.data, hh.ctypes.data, ab.ctypes.data, out.ctypes.data, out.size)
    assert k == 2 * sum(m * m for m in n) + sum(n)
    off, F, B = 0, [], []
    for m in n:
        F.append(out[off:off + m * m].reshape(m, m))
        B.append(out[off + m * m:off + 2 * m * m].reshape(m, m))
        off += 2 * m * m
    mu = [out[off:off + n[0]], out[off + n[0]:off + n[0] + n[1]], out[off + n[0] + n[1]:off + sum(n)]]
    for d in range(3):
        np.testing.assert_allclose(F[d] @ F[d].T, np.eye(n[d]), atol=1e-13)
        np.testing.assert_array_equal(B[d], F[d].T)
    # Q = kron over axes with x fastest: index i + nx (j + ny k)
    Q = np.kron(B[2], np.kron(B[1], B[0]))
    lam = (mu[2][:, None, None] + mu[1][None, :, None] + mu[0][None, None, :]).ravel()
    A = dirichlet_laplacian_dense(n, h, ab)
    np.testing.assert_allclose(Q @ np.diag(lam) @ Q.T, A, atol=1e-9 * np.abs(A).max())
    rng = np.random.default_rng(3)
    r = rng.standard_normal(A.shape[0])
    np.testing.assert_allclose(Q @ ((Q.T @ r) / lam), np.linalg.solve(A, r), rtol=1e-10, atol=1e-14)
