"""Python front end of the FP64 CPU oracle (``amrmg_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``.  The product library never imports
it, and it imports nothing from the product except the seeded input
generators (``paper_1812_03689_amd.workloads``), which hold none of the
method's arithmetic.

Each wrapper names the passage of arXiv:1812.03689 that the C function
follows; the C source restates the definitions.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "amrmg_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
MAXL = 10

_lib = None


def build_oracle(force: bool = True) -> str:
    """Compile the oracle: single-threaded, -O2, no contraction of a*b+c into
    FMAs and no fast-math, so that it rounds like the plain C it is."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class OStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("bottom_iters", C.c_int), ("converged", C.c_int),
                ("rel", C.c_double * MAXL)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build_oracle(force=True)
        L = C.CDLL(LIB)
        vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.or_new.restype = vp
        L.or_new.argtypes = [vp, vp, vp, dbl, C.c_int, vp]
        L.or_free.argtypes = [vp]
        L.or_set_robin.argtypes = [vp, dbl]
        L.or_set_robin.restype = None
        L.or_set_level.argtypes = [vp, C.c_int, C.c_int, vp]
        L.or_nlev.argtypes = [vp]
        L.or_nboxes.argtypes = [vp, C.c_int]
        L.or_ncells.argtypes = [vp, C.c_int]
        L.or_ncells.restype = i64
        L.or_get_boxes.argtypes = [vp, C.c_int, vp, vp]
        L.or_cell_index.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int]
        L.or_cell_index.restype = i64
        L.or_cf_pattern.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, vp]
        L.or_select_pattern.argtypes = [C.c_uint32]
        L.or_step1_layer.argtypes = [C.c_uint32, vp, dbl, dbl, vp]
        L.or_step1_layer.restype = dbl
        L.or_apply_composite.argtypes = [vp, vp, vp, C.c_int]
        L.or_apply_nf.argtypes = [vp, C.c_int, vp, vp, vp, C.c_int]
        L.or_average_down.argtypes = [vp, vp]
        L.or_efield.argtypes = [vp, vp, vp]
        L.or_solve.argtypes = [vp, vp, vp, vp, dbl, C.c_int, C.c_int, C.c_int, C.c_int, dbl,
                               C.POINTER(OStats)]
        L.or_residual.argtypes = [vp, vp, vp, vp]
        L.or_relax_point.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int, vp, vp]
        L.or_relax_point.restype = None
        L.or_deposit.argtypes = [vp, C.c_int, i64, vp, vp, vp, vp, vp]
        L.or_deposit.restype = i64
        L.or_gather.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp]
        L.or_gather.restype = i64
        L.or_tag.argtypes = [vp, C.c_int, vp, dbl, vp]
        L.or_cluster.argtypes = [vp, C.c_int, vp, C.c_int, C.c_int, C.c_int, C.c_int, vp, C.c_int]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _ptrs(arrs: Sequence[Optional[np.ndarray]]):
    P = (C.c_void_p * max(1, len(arrs)))()
    for i, a in enumerate(arrs):
        P[i] = None if a is None else a.ctypes.data
    return P


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleHierarchy:
    """A box-list hierarchy held by the oracle (Sec. 3, the level / grid
    relations under Eq. mesh_spacing; refinement ratio 2)."""

    def __init__(self, n0, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), eps0: float = 1.0,
                 monopoles: Sequence[Sequence[float]] = (), robin: float = 0.0):
        self.n0 = tuple(int(v) for v in n0)
        self.lo = np.asarray(lo, dtype=np.float64)
        self.hi = np.asarray(hi, dtype=np.float64)
        self.eps0 = float(eps0)
        mono = np.asarray(monopoles, dtype=np.float64).reshape(-1, 4)
        self._mono = np.ascontiguousarray(mono)
        n0a = np.asarray(self.n0, dtype=np.int32)
        self.h = lib().or_new(_ptr(self.lo), _ptr(self.hi), _ptr(n0a), self.eps0,
                              int(mono.shape[0]), _ptr(self._mono))
        self.set_level(0, [(0, 0, 0) + self.n0])
        # open boundary d phi/dn + phi/robin = 0 (Sec. 5.2, Eq. robin_bc) instead of Dirichlet data
        self.robin = float(robin)
        lib().or_set_robin(self.h, self.robin)

    def __del__(self):
        try:
            if self.h:
                lib().or_free(self.h)
                self.h = None
        except Exception:
            pass

    # -- structure ---------------------------------------------------------
    def set_level(self, l: int, boxes) -> None:
        b = np.ascontiguousarray(np.asarray(boxes, dtype=np.int32).reshape(-1, 6))
        rc = lib().or_set_level(self.h, l, int(b.shape[0]), _ptr(b))
        if rc != 0:
            raise ValueError(f"or_set_level(level {l}) failed with {rc}")

    @property
    def nlev(self) -> int:
        return lib().or_nlev(self.h)

    def ncells(self, l: int) -> int:
        return int(lib().or_ncells(self.h, l))

    def boxes(self, l: int):
        nb = lib().or_nboxes(self.h, l)
        b = np.zeros((nb, 6), dtype=np.int32)
        off = np.zeros(nb + 1, dtype=np.int64)
        lib().or_get_boxes(self.h, l, _ptr(b), _ptr(off))
        return b, off

    def cell_index(self, l, i, j, k) -> int:
        return int(lib().or_cell_index(self.h, l, i, j, k))

    def spacing(self, l: int) -> np.ndarray:
        return (self.hi - self.lo) / (np.asarray(self.n0) * 2 ** l)

    def cell_centres(self, l: int):
        """(x, y, z) centres of every cell of level l in arena order."""
        b, _ = self.boxes(l)
        h = self.spacing(l)
        xs, ys, zs = [], [], []
        for B in b:
            k, j, i = np.meshgrid(np.arange(B[2], B[5]), np.arange(B[1], B[4]),
                                  np.arange(B[0], B[3]), indexing="ij")
            xs.append(self.lo[0] + (i.ravel() + 0.5) * h[0])
            ys.append(self.lo[1] + (j.ravel() + 0.5) * h[1])
            zs.append(self.lo[2] + (k.ravel() + 0.5) * h[2])
        return np.concatenate(xs), np.concatenate(ys), np.concatenate(zs)

    def cell_indices(self, l: int):
        b, _ = self.boxes(l)
        out = []
        for B in b:
            k, j, i = np.meshgrid(np.arange(B[2], B[5]), np.arange(B[1], B[4]),
                                  np.arange(B[0], B[3]), indexing="ij")
            out.append(np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1))
        return np.concatenate(out).astype(np.int64)

    def covered_mask(self, l: int) -> np.ndarray:
        """True on cells of level l whose children are in level l+1: per box
        of level l, the coarse footprints [lo/2, hi/2) of the level-(l+1)
        boxes that meet it (fine boxes are whole blocks, so even-aligned)."""
        n = self.ncells(l)
        m = np.zeros(n, dtype=bool)
        if l + 1 >= self.nlev:
            return m
        cb, coff = self.boxes(l)
        fb, _ = self.boxes(l + 1)
        flo, fhi = fb[:, :3] // 2, fb[:, 3:] // 2
        for bi, B in enumerate(cb):
            lo = np.maximum(flo, B[:3])
            hi = np.minimum(fhi, B[3:])
            hit = np.all(hi > lo, axis=1)
            if not hit.any():
                continue
            ext = B[3:] - B[:3]
            blk = np.zeros((ext[2], ext[1], ext[0]), dtype=bool)
            for a, b in zip(lo[hit] - B[:3], hi[hit] - B[:3]):
                blk[a[2]:b[2], a[1]:b[1], a[0]:b[0]] = True
            m[coff[bi]:coff[bi + 1]] = blk.ravel()
        return m

    def composite_rel_l2(self, a: Sequence[np.ndarray], b: Sequence[np.ndarray], ncomp: int = 1) -> float:
        """Relative L2 difference of a from the reference b over the composite
        cells (the uncovered cells of every level, Sec. 5.3), each cell
        weighted by its volume h_x h_y h_z.  With ncomp > 1 the arrays are
        per level and component (E[ncomp * l + d]) and the components are
        summed."""
        num = den = 0.0
        for l in range(self.nlev):
            unc = ~self.covered_mask(l)
            vol = float(np.prod(self.spacing(l)))
            for d in range(ncomp):
                x = np.asarray(a[ncomp * l + d])[unc]
                y = np.asarray(b[ncomp * l + d])[unc]
                num += vol * float(np.sum((x - y) ** 2))
                den += vol * float(np.sum(y ** 2))
        return float(np.sqrt(num / den)) if den > 0 else float(np.sqrt(num))

    def zeros(self) -> List[np.ndarray]:
        return [np.zeros(self.ncells(l)) for l in range(self.nlev)]

    # -- particles (CIC, Hockney & Eastwood; Fig. 2 workflow) -------------
    def deposit(self, l: int, particles) -> tuple:
        x, y, z = _f64(particles.x), _f64(particles.y), _f64(particles.z)
        q = _f64(particles.q)
        rho = np.zeros(self.ncells(l))
        nout = lib().or_deposit(self.h, l, int(q.shape[0]), _ptr(x), _ptr(y), _ptr(z), _ptr(q), _ptr(rho))
        return rho, int(nout)

    def deposit_all(self, particles) -> List[np.ndarray]:
        return [self.deposit(l, particles)[0] for l in range(self.nlev)]

    def gather(self, particles, E: Sequence[np.ndarray]):
        x, y, z = _f64(particles.x), _f64(particles.y), _f64(particles.z)
        n = x.shape[0]
        Ex, Ey, Ez = np.zeros(n), np.zeros(n), np.zeros(n)
        Es = [_f64(e) for e in E]
        lib().or_gather(self.h, n, _ptr(x), _ptr(y), _ptr(z), _ptrs(Es), _ptr(Ex), _ptr(Ey), _ptr(Ez))
        return Ex, Ey, Ez

    # -- tagging and box generation (Sec. 4.2; box generation see C) ------
    def tag(self, l: int, rho: np.ndarray, lam: float) -> np.ndarray:
        tags = np.zeros(self.ncells(l), dtype=np.uint8)
        lib().or_tag(self.h, l, _ptr(_f64(rho)), float(lam), _ptr(tags))
        return tags

    def cluster(self, l: int, tags: np.ndarray, n_buffer=1, n_proper=2, bf=8, mgs=32) -> np.ndarray:
        cap = 1 << 20
        out = np.zeros((cap, 6), dtype=np.int32)
        t = np.ascontiguousarray(tags, dtype=np.uint8)
        nb = lib().or_cluster(self.h, l, _ptr(t), n_buffer, n_proper, bf, mgs, _ptr(out), cap)
        if nb < 0:
            raise RuntimeError("too many boxes")
        return out[:nb].copy()

    # -- coarse-fine interpolation patterns (Tab. bit_pattern) -------------
    def cf_pattern(self, l, i, j, k, d, s):
        m = C.c_uint32(0)
        p = lib().or_cf_pattern(self.h, l, i, j, k, d, s, C.byref(m))
        return int(p), int(m.value)

    # -- operators (Sec. 5.1) and Alg. 1-3 ---------------------------------
    def apply_composite(self, phi: Sequence[np.ndarray], inhom: bool = False) -> List[np.ndarray]:
        ph = [_f64(p) for p in phi]
        out = self.zeros()
        lib().or_apply_composite(self.h, _ptrs(ph), _ptrs(out), int(inhom))
        return out

    def apply_nf(self, l: int, u: np.ndarray, ucoarse: Optional[np.ndarray] = None,
                 inhom: bool = False) -> np.ndarray:
        arrs = [None] * self.nlev
        arrs[l] = _f64(u)
        uc = None if ucoarse is None else _f64(ucoarse)
        out = np.zeros(self.ncells(l))
        lib().or_apply_nf(self.h, l, _ptrs(arrs), None if uc is None else _ptr(uc), _ptr(out), int(inhom))
        return out

    def relax_point(self, l: int, i: int, j: int, k: int, e: np.ndarray, r: np.ndarray) -> np.ndarray:
        """One Gauss-Seidel update (the smoother of Alg. 3, Sec. 5.3) of cell
        (i, j, k) of level l for A_nf e = r with zero coarse data and
        homogeneous boundary data; returns the updated copy of e."""
        out = np.array(e, dtype=np.float64, copy=True)
        lib().or_relax_point(self.h, l, i, j, k, _ptr(out), _ptr(_f64(r)))
        return out

    def residual(self, rho: Sequence[np.ndarray], phi: Sequence[np.ndarray]) -> List[np.ndarray]:
        rr = [_f64(r) for r in rho]
        ph = [_f64(p) for p in phi]
        out = self.zeros()
        lib().or_residual(self.h, _ptrs(rr), _ptrs(ph), _ptrs(out))
        return out

    def average_down(self, phi: Sequence[np.ndarray]) -> List[np.ndarray]:
        ph = [np.array(p, dtype=np.float64, copy=True) for p in phi]
        lib().or_average_down(self.h, _ptrs(ph))
        return ph

    def efield(self, phi: Sequence[np.ndarray]) -> List[np.ndarray]:
        ph = [_f64(p) for p in phi]
        E = [np.zeros(self.ncells(l)) for l in range(self.nlev) for _ in range(3)]
        lib().or_efield(self.h, _ptrs(ph), _ptrs(E))
        return E

    def solve(self, rho: Sequence[np.ndarray], phi0: Optional[Sequence[np.ndarray]] = None,
              tol: float = 1e-10, max_iters: int = 50, nu1: int = 2, nu2: int = 2, norm_p: int = 2,
              bottom_rtol: float = 1e-12, want_E: bool = True):
        """Alg. 2 with the V-cycle of Alg. 3 (GSRB smoothing, CG on level 0).
        Returns (phi, E or None, stats dict)."""
        rr = [_f64(r) for r in rho]
        phi = [np.array(p, dtype=np.float64, copy=True) for p in phi0] if phi0 is not None else self.zeros()
        E = [np.zeros(self.ncells(l)) for l in range(self.nlev) for _ in range(3)] if want_E else None
        st = OStats()
        lib().or_solve(self.h, _ptrs(rr), _ptrs(phi), _ptrs(E) if E is not None else None, float(tol),
                       int(max_iters), int(nu1), int(nu2), int(norm_p), float(bottom_rtol), C.byref(st))
        stats = dict(iters=st.iters, bottom_iters=st.bottom_iters, converged=bool(st.converged),
                     rel=[st.rel[l] for l in range(self.nlev)])
        return phi, E, stats


def select_pattern(mask5: int) -> int:
    """Pattern id chosen for a 5x5 availability mask (Tab. bit_pattern order,
    then the bilinear table): 0..8 quadratic, 9..12 bilinear, 13 centre only."""
    return int(lib().or_select_pattern(int(mask5)))


def step1_layer(mask5: int, layer: np.ndarray, tu: float, tv: float):
    """Step 1 of the ghost interpolation (Eq. 2d_lagrange) on a 5x5 coarse
    layer ``layer[jv, iu]`` (centre (2,2)); returns (value, pattern id)."""
    lay = np.ascontiguousarray(np.asarray(layer, dtype=np.float64).reshape(25))
    pat = C.c_int(0)
    v = lib().or_step1_layer(int(mask5), _ptr(lay), float(tu), float(tv), C.byref(pat))
    return float(v), int(pat.value)


TAG_SOLVE_TOL = 1e-13


def field_tags(H: OracleHierarchy, l: int, particles, policy: str, lam: float) -> np.ndarray:
    """Tags of level l, the finest level of H, by the potential or the
    electric field (Sec. 4.2): the composite problem on H's levels is solved
    with every particle deposited, then a cell is tagged when |phi| exceeds
    lam times the level's max |phi| ("potential"), or when some component
    |E_w| exceeds lam times that component's max over the level ("efield")."""
    assert H.nlev == l + 1
    phi, E, st = H.solve(H.deposit_all(particles), tol=TAG_SOLVE_TOL, max_iters=80, bottom_rtol=1e-14)
    if policy == "potential":
        return H.tag(l, phi[l], lam)
    if policy == "efield":
        tags = np.zeros(H.ncells(l), dtype=np.uint8)
        for d in range(3):
            tags |= H.tag(l, E[3 * l + d], lam)
        return tags
    raise ValueError(policy)


def build_hierarchy(n0, particles, max_level: int, tag_rel: Sequence[float],
                    monopoles=(), explicit_boxes=None, n_buffer=1, n_proper=2, bf=8, mgs=32,
                    lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), eps0=1.0, tag_policy="charge",
                    robin=0.0) -> OracleHierarchy:
    """Regrid loop: tag level l (by its own deposit, or by the potential or
    field of a solve on levels 0..l), generate level l+1 boxes; explicit
    boxes ``(level, lo3, hi3)`` replace the tagging for their level."""
    H = OracleHierarchy(n0, lo, hi, eps0, monopoles, robin)
    explicit = {}
    for e in (explicit_boxes or []):
        explicit.setdefault(int(e[0]), []).append(tuple(int(v) for v in e[1:7]))
    for l in range(max_level):
        if (l + 1) in explicit:
            boxes = np.asarray(explicit[l + 1], dtype=np.int32)
        else:
            if tag_policy == "charge":
                rho, _ = H.deposit(l, particles)
                tags = H.tag(l, rho, tag_rel[l])
            else:
                tags = field_tags(H, l, particles, tag_policy, tag_rel[l])
            boxes = H.cluster(l, tags, n_buffer, n_proper, bf, mgs)
        if boxes.shape[0] == 0:
            break
        H.set_level(l + 1, boxes)
    return H


def hierarchy_from_workload(w) -> OracleHierarchy:
    return build_hierarchy(w.n0, w.particles, w.max_level, w.tag_rel, w.monopoles,
                           w.explicit_boxes, mgs=w.max_grid_size, bf=w.blocking_factor,
                           lo=getattr(w, "lo", (0.0, 0.0, 0.0)), hi=getattr(w, "hi", (1.0, 1.0, 1.0)),
                           tag_policy=getattr(w, "tag_policy", "charge"), robin=getattr(w, "robin", 0.0))
