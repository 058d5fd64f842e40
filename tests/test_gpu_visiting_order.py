"""amrmg_visiting_order through the C ABI: the build's visiting order is the
stable sort of the particles by the Morton code of their cell on the sort
grid (the level-0 grid refined towards four particles per cell, at most to
the finest level, merged 2^3 at a time beyond 1024 cells per axis), checked
element by element against the same keys computed here and NumPy's stable
argsort, on ragged counts (one particle, one short of a radix tile, several
tiles and a tail, above 4M keys where the tiles are four times longer), FP64 and FP32 positions, particles outside the domain
(nearest cell), a refined sort grid, one above 1024 cells per axis, digit
widths from 6 to 10 bits, and a domain other than the unit cube.  Also the inverse order through the gather's write-back
(bit-equal E) and the state errors."""
import numpy as np
import pytest

from paper_1812_03689_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def morton_keys(x, y, z, lo, hi, n0, levels):
    """Key of every particle on the sort grid: the level-0 grid refined while
    it has fewer than a quarter as many cells as particles, at most levels
    times; cell = floor((x - lo) * cells / (hi - lo)) clamped to the grid,
    merged while the grid exceeds 1024 per axis, bits of x, y, z interleaved
    (bit i of axis d at bit 3 i + d)."""
    n = len(x)
    m0 = max(n0)
    r = 0
    while r < levels and float(m0 << r) ** 3 < n / 4.0:
        r += 1
    nf = [n0[d] << r for d in range(3)]
    b = int(np.ceil(np.log2(max(nf)))) if max(nf) > 1 else 0
    shift = max(0, b - 10)
    key = np.zeros(n, dtype=np.uint64)
    for d, v in enumerate((x, y, z)):
        s = (np.asarray(v, dtype=np.float64) - lo[d]) * (float(nf[d]) / (hi[d] - lo[d]))
        c = np.fmin(np.fmax(s, 0.0), float(nf[d] - 1)).astype(np.uint64) >> np.uint64(shift)
        for i in range(10):
            key |= ((c >> np.uint64(i)) & np.uint64(1)) << np.uint64(3 * i + d)
    return key


def build(p, n0, levels, lo=(0, 0, 0), hi=(1, 1, 1), pos_dtype=torch.float64, tag=1e-3):
    from paper_1812_03689_amd import amrmg as A
    ctx = A.Context(A.make_params(n0, max_level=levels, monopoles=[(1.0, 0.5, 0.5, 0.5)], lo=lo, hi=hi))
    x, y, z = (torch.as_tensor(a, device="cuda").to(pos_dtype) for a in (p.x, p.y, p.z))
    q = torch.as_tensor(p.q, device="cuda")
    ctx.build_hierarchy(x, y, z, q, tag_rel=[tag] * levels)
    return ctx, (x, y, z)


CASES = {
    "one": (1, (16, 16, 16), 1, torch.float64),
    "tile_minus_one": (4095, (32, 32, 32), 2, torch.float64),
    "tiles_and_tail": (3 * 4096 + 17, (32, 32, 32), 2, torch.float32),
    "gauss_fp32": (200000, (64, 64, 64), 2, torch.float32),
    "refined_once": (100000, (16, 16, 16), 2, torch.float64),
    "merged_cells": (50000, (2048, 16, 16), 1, torch.float64),
    "digit7": (20000, (128, 128, 128), 1, torch.float32),
    "large_tiles": (4300000, (64, 64, 64), 1, torch.float32),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_order_is_the_stable_morton_sort(name):
    n, n0, levels, dt = CASES[name]
    print("visiting order", name, flush=True)
    p = W.gaussian_bunch(n, sigma=(0.05, 0.05, 0.1), seed=W.seed_for(2, 40 + n % 97))
    if n > 10:  # a few particles outside the domain take the nearest cell
        for a, v in ((p.x, -0.25), (p.y, 1.5), (p.z, 1.0)):
            a[3] = v
    ctx, (x, y, z) = build(p, n0, levels, pos_dtype=dt)
    perm = ctx.visiting_order().cpu().numpy()
    keys = morton_keys(*(t.cpu().double().numpy() for t in (x, y, z)), (0, 0, 0), (1, 1, 1), n0, levels)
    assert np.array_equal(perm, np.argsort(keys, kind="stable"))


def test_order_on_a_shifted_domain():
    lo, hi = (-0.3, 0.1, 2.0), (0.7, 1.1, 3.0)
    p = W.gaussian_bunch(50000, sigma=(0.05, 0.05, 0.1), seed=W.seed_for(2, 41))  # in the unit cube
    p = W.Particles(p.x + lo[0], p.y + lo[1], p.z + lo[2], p.q)
    ctx, (x, y, z) = build(p, (32, 32, 32), 2, lo=lo, hi=hi)
    perm = ctx.visiting_order().cpu().numpy()
    keys = morton_keys(p.x, p.y, p.z, lo, hi, (32, 32, 32), 2)
    assert np.array_equal(perm, np.argsort(keys, kind="stable"))


def test_gather_write_back_uses_the_inverse_order():
    """E written in the caller's order through the inverse of the visiting
    order equals E gathered in the caller's order directly (the single pass
    a particle count other than the build's takes)."""
    p = W.gaussian_bunch(3 * 4096 + 17, sigma=(0.05, 0.05, 0.1), seed=W.seed_for(2, 42))
    ctx, (x, y, z) = build(p, (32, 32, 32), 2)
    rho, _ = ctx.deposit_built()
    _, E, st = ctx.solve(rho, tol=1e-10)
    a = ctx.gather_built(E)
    m = x.numel() - 5
    b = ctx.gather(x[:m], y[:m], z[:m], E)
    torch.cuda.synchronize()
    for u, v in zip(a, b):
        assert torch.equal(u[:m], v)


def test_state_errors():
    from paper_1812_03689_amd import amrmg as A
    ctx = A.Context(A.make_params((16, 16, 16), max_level=1, monopoles=[(1.0, 0.5, 0.5, 0.5)]))
    perm = torch.zeros(4, dtype=torch.int32, device="cuda")
    with pytest.raises(A.AmrmgError) as ex:
        A.amrmg_visiting_order(ctx.h, perm, 4)
    assert ex.value.status == A.AMRMG_E_STATE
    p = W.gaussian_bunch(1000, seed=W.seed_for(2, 43))
    ctx, _ = build(p, (16, 16, 16), 1)
    with pytest.raises(A.AmrmgError) as ex:
        A.amrmg_visiting_order(ctx.h, perm, 4)
    assert ex.value.status == A.AMRMG_E_INVALID
    empty = torch.zeros(0, dtype=torch.float64, device="cuda")
    ctx.build_hierarchy(empty, empty, empty, empty, tag_rel=[1e-3])
    with pytest.raises(A.AmrmgError) as ex:
        A.amrmg_visiting_order(ctx.h, perm, 0)
    assert ex.value.status == A.AMRMG_E_STATE
