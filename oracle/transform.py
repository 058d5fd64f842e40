"""FP64 oracle of the domain transform of arXiv:1812.03689, Sec. 4.1.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``.  Plain NumPy, no code
shared with the product library.

Particles in particle space S_p are mapped into the computation space
S_c = [-l0, l0] x [-l1, l1] x [-l2, l2] around a reference position c by
x* = (x - c) / s, where s is the largest Gamma(x_i, l) = max_d |x_id - c_d| /
l_d over the particles (subsection "Particle Coordinate"; the printed
definition of s is garbled, and the reading taken is the scale that puts the
outermost particle on the boundary of S_c).  After a solve in S_c the
potential and field on the grid are rescaled by phi = phi* / s (Eq.
potential_transform) and E = E* / s^2 (Eq. efield_transform), the
three-dimensional case of the paper's derivation.
"""
from __future__ import annotations

from typing import List, Optional, Sequence, Tuple

import numpy as np


def gamma(x, y, z, center, l) -> np.ndarray:
    """Gamma(x, l) of every particle (positions promoted to FP64)."""
    g = [np.abs(np.asarray(a, dtype=np.float64) - float(center[d])) / float(l[d]) for d, a in enumerate((x, y, z))]
    return np.maximum(np.maximum(g[0], g[1]), g[2])


def domain_scale(x, y, z, center, l) -> float:
    """s = max_i Gamma(x_i, l); 0 for no particles."""
    g = gamma(x, y, z, center, l)
    return float(g.max()) if g.size else 0.0


def to_computation(x, y, z, center, s) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """x* = (x - c) / s in FP64, returned in the positions' own type."""
    out = []
    for d, a in enumerate((x, y, z)):
        a = np.asarray(a)
        out.append(((a.astype(np.float64) - float(center[d])) / float(s)).astype(a.dtype))
    return out[0], out[1], out[2]


def rescale(phi: Sequence[np.ndarray], E: Optional[Sequence[np.ndarray]], s: float):
    """phi / s and E / s^2 per level array (Eqs. potential_transform, efield_transform)."""
    s2 = float(s) * float(s)
    p = [np.asarray(a, dtype=np.float64) / float(s) for a in phi]
    e: Optional[List[np.ndarray]] = None if E is None else [np.asarray(a, dtype=np.float64) / s2 for a in E]
    return p, e
