"""Seeded synthetic inputs for the composite AMR Poisson path.

This module only draws particles and states workload sizes.  It holds none of
the method's arithmetic (no deposition, tagging, operator or solver code), so
that the FP64 oracle and the HIP path can both take their inputs from here
without sharing any part of the computation.

Workloads follow the paper's own synthetic test problems: a uniformly charged
sphere (Sec. 6.2, "Uniformly Charged Sphere in Free Space") and Gaussian
bunches, alone or placed side by side (Sec. 6.3 and Sec. 7, neighbouring
bunches in a cyclotron), and the paper's benchmark chain of 11 bunches.  The
domain is the unit cube (the chain: a computation cube around the
particles), eps0 = 1, and the total charge is 1 split evenly over the macro
particles.

Random numbers: NumPy PCG64 seeded with ``1812000 + 100*config + instance``.
Particles that fall outside [0, 1)^3 are redrawn.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

SEED_BASE = 1812000


def seed_for(config: int, instance: int = 0) -> int:
    return SEED_BASE + 100 * config + instance


@dataclasses.dataclass
class Particles:
    """Structure-of-arrays macro particles.

    ``x, y, z`` are float64 or float32 arrays (float32 is the stored truth when
    the workload says so), ``q`` is float64.
    """

    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    q: np.ndarray

    @property
    def n(self) -> int:
        return int(self.q.shape[0])

    @property
    def pos_dtype(self):
        return self.x.dtype


def _redraw_outside(rng, draw, n):
    """Draw ``n`` points with ``draw(rng, m) -> (m,3)``, redrawing any that
    fall outside the half-open unit cube."""
    out = np.empty((n, 3), dtype=np.float64)
    filled = 0
    while filled < n:
        pts = draw(rng, n - filled)
        ok = np.all((pts >= 0.0) & (pts < 1.0), axis=1)
        pts = pts[ok]
        out[filled:filled + pts.shape[0]] = pts
        filled += pts.shape[0]
    return out


def uniform_ball(n: int, centre=(0.5, 0.5, 0.5), radius: float = 0.2,
                 seed: int = seed_for(1), total_charge: float = 1.0,
                 pos_dtype=np.float64) -> Particles:
    """Points uniform in a ball: direction from a normalised Gaussian,
    radius ``R * U**(1/3)``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = np.asarray(centre, dtype=np.float64)

    def draw(rng, m):
        d = rng.standard_normal((m, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        r = radius * rng.random(m) ** (1.0 / 3.0)
        return c + d * r[:, None]

    p = _redraw_outside(rng, draw, n)
    p = p.astype(pos_dtype)
    q = np.full(n, total_charge / n, dtype=np.float64)
    return Particles(np.ascontiguousarray(p[:, 0]), np.ascontiguousarray(p[:, 1]),
                     np.ascontiguousarray(p[:, 2]), q)


def gaussian_bunch(n: int, centre=(0.5, 0.5, 0.5), sigma=(0.05, 0.05, 0.1),
                   seed: int = seed_for(2), total_charge: float = 1.0,
                   pos_dtype=np.float64, rng=None) -> Particles:
    """Independent normal coordinates around ``centre`` with per-axis sigma."""
    if rng is None:
        rng = np.random.Generator(np.random.PCG64(seed))
    c = np.asarray(centre, dtype=np.float64)
    s = np.asarray(sigma, dtype=np.float64)

    def draw(rng, m):
        return c + rng.standard_normal((m, 3)) * s

    p = _redraw_outside(rng, draw, n).astype(pos_dtype)
    q = np.full(n, total_charge / n, dtype=np.float64)
    return Particles(np.ascontiguousarray(p[:, 0]), np.ascontiguousarray(p[:, 1]),
                     np.ascontiguousarray(p[:, 2]), q)


def concat(parts: Sequence[Particles]) -> Particles:
    return Particles(np.concatenate([p.x for p in parts]),
                     np.concatenate([p.y for p in parts]),
                     np.concatenate([p.z for p in parts]),
                     np.concatenate([p.q for p in parts]))


def arc_centres(nb: int = 9, radius: float = 0.35, centre=(0.5, 0.5, 0.5)):
    """Bunch centres on a circular arc in the z = centre plane,
    theta_k = -pi/2 + k*pi/8."""
    out = []
    for k in range(nb):
        th = -math.pi / 2 + k * math.pi / 8
        out.append((centre[0] + radius * math.cos(th),
                    centre[1] + radius * math.sin(th), centre[2]))
    return out


def arc_bunches(n_per: int = 10**6, nb: int = 9, sigma: float = 0.02,
                seed: int = seed_for(4)) -> Tuple[Particles, List[Tuple[float, float, float, float]]]:
    rng = np.random.Generator(np.random.PCG64(seed))
    cs = arc_centres(nb)
    parts = [gaussian_bunch(n_per, c, (sigma, sigma, sigma), rng=rng,
                            total_charge=1.0 / nb) for c in cs]
    monopoles = [(1.0 / nb, c[0], c[1], c[2]) for c in cs]
    return concat(parts), monopoles


@dataclasses.dataclass
class Workload:
    """One solve: particles, base grid, refinement and solver settings."""

    name: str
    particles: Particles
    n0: Tuple[int, int, int]
    max_level: int
    tag_rel: List[float]                 # one threshold per refined level
    monopoles: List[Tuple[float, float, float, float]]   # (q, x, y, z)
    tol: float
    explicit_boxes: Optional[List[Tuple[int, int, int, int, int, int, int]]] = None
    max_grid_size: int = 32
    blocking_factor: int = 8
    precision: str = "mixed"
    lo: Tuple[float, float, float] = (0.0, 0.0, 0.0)   # the domain [lo, hi)
    hi: Tuple[float, float, float] = (1.0, 1.0, 1.0)
    tag_policy: str = "charge"                          # "charge", "potential" or "efield"
    robin: float = 0.0                                  # > 0: Robin open boundary with this distance


def config1(n_particles: int = 10**4) -> Workload:
    """Uniform ball (radius 0.2, unit charge) on 32^3 with one fixed fine box
    over the central 16^3 base cells; Dirichlet data from the exact sphere
    potential, which outside the ball equals a unit monopole."""
    p = uniform_ball(n_particles, seed=seed_for(1))
    return Workload("sphere_32c_1lev", p, (32, 32, 32), 1, [],
                    [(1.0, 0.5, 0.5, 0.5)], 1e-10,
                    explicit_boxes=[(1, 16, 16, 16, 48, 48, 48)], precision="fp64")


def config2(n_particles: int = 10**6) -> Workload:
    p = gaussian_bunch(n_particles, sigma=(0.05, 0.05, 0.1), seed=seed_for(2))
    return Workload("gauss_64c_2lev", p, (64, 64, 64), 2, [1e-3, 1e-3],
                    [(1.0, 0.5, 0.5, 0.5)], 1e-8)


def config3(n_particles: int = 10**7) -> Workload:
    p = gaussian_bunch(n_particles, sigma=(0.03, 0.03, 0.08), seed=seed_for(3),
                       pos_dtype=np.float32)
    return Workload("gauss_128c_3lev_f32pos", p, (128, 128, 128), 3,
                    [1e-4, 1e-4, 1e-4], [(1.0, 0.5, 0.5, 0.5)], 1e-8)


def config4(n_per: int = 10**6) -> Workload:
    p, mono = arc_bunches(n_per, seed=seed_for(4))
    return Workload("arc9_128c_2lev", p, (128, 128, 128), 2, [1e-3, 1e-3],
                    mono, 1e-8, max_grid_size=32)


def config5_instances(count: int = 64, scale: float = 1.0) -> List[Workload]:
    """Independent small solves: base edge from {16, 24, 32, 48}, 1 or 2 refined
    levels, 1e4..1e5 particles (times ``scale``), centre in [0.3, 0.7]^3,
    isotropic sigma in [0.02, 0.08]."""
    out = []
    for i in range(count):
        rng = np.random.Generator(np.random.PCG64(seed_for(5, i)))
        n0 = int(rng.choice([16, 24, 32, 48]))
        levels = int(rng.choice([1, 2]))
        npart = max(16, int(int(rng.integers(10**4, 10**5 + 1)) * scale))
        c = tuple(float(v) for v in rng.uniform(0.3, 0.7, 3))
        s = float(rng.uniform(0.02, 0.08))
        p = gaussian_bunch(npart, c, (s, s, s), rng=rng)
        out.append(Workload(f"batch{i}_{n0}c_{levels}lev", p, (n0, n0, n0), levels,
                            [1e-3] * levels, [(1.0,) + c], 1e-8))
    return out


def chain_bunches(n_per: int = 10**6, nb: int = 11, sigma=(1.5e-3, 5e-3, 5e-3), spacing: float = 0.04,
                  seed: int = seed_for(6)) -> Particles:
    """The paper's benchmark source (Sec. 6.3 and the strong-scaling test of
    Sec. 8): ``nb`` Gaussian bunches of ``n_per`` particles in metres, sigma
    (1.5 mm, 5 mm, 5 mm), centres 4 cm apart along x around the origin.  Unit
    total charge split evenly (the paper's 0.1 fC per particle only scales
    phi)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    s = np.asarray(sigma, dtype=np.float64)
    pts = []
    for k in range(nb):
        c = np.array([(k - (nb - 1) / 2.0) * spacing, 0.0, 0.0])
        pts.append(c + rng.standard_normal((n_per, 3)) * s)
    p = np.concatenate(pts)
    q = np.full(p.shape[0], 1.0 / p.shape[0], dtype=np.float64)
    return Particles(np.ascontiguousarray(p[:, 0]), np.ascontiguousarray(p[:, 1]),
                     np.ascontiguousarray(p[:, 2]), q)


def isotropic_domain(p: Particles, margin: float = 0.1):
    """The computation cube around the particles (the paper's S_c with a
    box increment delta = 10 %): centred on their bounding box, edge
    (1 + margin) times its longest side, so that cells are cubes."""
    lo = np.array([p.x.min(), p.y.min(), p.z.min()], dtype=np.float64)
    hi = np.array([p.x.max(), p.y.max(), p.z.max()], dtype=np.float64)
    c, hw = 0.5 * (lo + hi), 0.5 * (1.0 + margin) * float(np.max(hi - lo))
    return tuple(float(v) for v in c - hw), tuple(float(v) for v in c + hw)


def config6(n_per: int = 10**6, n0: int = 576, lam: float = 1e-3, nb: int = 11) -> Workload:
    """The paper's strong-scaling benchmark on one GPU: 11 Gaussian bunches of
    1e6 particles, 576^3 base cells on the computation cube, 2 refined levels
    tagged at lam x max|rho| (the paper does not state its threshold),
    homogeneous Dirichlet boundary, tol 1e-8."""
    p = chain_bunches(n_per, nb)
    lo, hi = isotropic_domain(p)
    return Workload(f"chain{nb}_{n0}c_2lev", p, (n0, n0, n0), 2, [lam, lam], [], 1e-8, max_grid_size=32,
                    lo=lo, hi=hi)


def jitter(x, y, z, lo, hi, amp: float = 1e-3, gen=None):
    """One step of the benchmark's particle motion: every coordinate moves by a
    uniform random amount in [-amp, amp] times the half-edge of the
    computation cube (the paper's displacement within [-1e-3, 1e-3] in
    computation-space units).  Works on torch tensors (any device); gen is a
    torch.Generator of that device."""
    import torch
    out = []
    for a, l, h in zip((x, y, z), lo, hi):
        d = torch.rand(a.shape, generator=gen, device=a.device, dtype=torch.float64) * 2.0 - 1.0
        out.append(a + (d * (amp * 0.5 * (h - l))).to(a.dtype))
    return out


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 6: config6}
