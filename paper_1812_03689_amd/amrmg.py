"""Python binding of libamrmg (include/amrmg.h).

Argument marshalling only: every step of the path runs in the HIP kernels of
the shared library.  Functions carry the C names; ``Context`` bundles them for
convenience.  PyTorch provides the device memory (tensors) and the HIP stream.
If the library is not built, importing works but every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libamrmg.so")

AMRMG_OK = 0
AMRMG_E_INVALID = -1
AMRMG_E_HIP = -2
AMRMG_E_NOT_CONVERGED = -3
AMRMG_E_NESTING = -4
AMRMG_E_OOM = -5
AMRMG_E_STATE = -6
AMRMG_E_NOT_IMPLEMENTED = -7
STATUS_NAMES = {0: "OK", -1: "E_INVALID", -2: "E_HIP", -3: "E_NOT_CONVERGED", -4: "E_NESTING",
                -5: "E_OOM", -6: "E_STATE", -7: "E_NOT_IMPLEMENTED"}
AMRMG_POS_F64, AMRMG_POS_F32 = 0, 1
AMRMG_FP64, AMRMG_MIXED = 0, 1
AMRMG_GSRB, AMRMG_JACOBI, AMRMG_GSRB_GLOBAL = 0, 1, 2
AMRMG_BOTTOM_AUTO, AMRMG_BOTTOM_CG = 0, 1
AMRMG_TAG_CHARGE, AMRMG_TAG_POTENTIAL, AMRMG_TAG_EFIELD = 0, 1, 2
TAG_POLICIES = {"charge": AMRMG_TAG_CHARGE, "potential": AMRMG_TAG_POTENTIAL, "efield": AMRMG_TAG_EFIELD}
AMRMG_MAX_LEVELS = 8
AMRMG_NOALLOC_SCRATCH_BYTES = 128 << 20

EXPORTED = ["amrmg_default_params", "amrmg_create", "amrmg_destroy", "amrmg_last_error",
            "amrmg_build_hierarchy", "amrmg_hierarchy_info", "amrmg_get_boxes", "amrmg_cf_faces", "amrmg_brick_tables",
            "amrmg_workspace_size", "amrmg_set_workspace", "amrmg_deposit", "amrmg_deposit_built", "amrmg_solve",
            "amrmg_solve_noalloc",
            "amrmg_gather", "amrmg_gather_built", "amrmg_visiting_order", "amrmg_residual", "amrmg_solve_batch", "amrmg_profile_enable",
            "amrmg_profile_read", "amrmg_profile_launches", "amrmg_transform_particles", "amrmg_rescale_fields"]
KCLASS = ["gsrb", "jacobi", "restrict", "prolong", "reflux", "cpart", "residual", "phi_update", "bottom",
          "efield", "avgdown", "deposit", "gather"]


class amrmg_params(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("hi", C.c_double * 3), ("n0", C.c_int32 * 3),
                ("max_level", C.c_int32), ("ref_ratio", C.c_int32), ("blocking_factor", C.c_int32),
                ("max_grid_size", C.c_int32), ("n_buffer", C.c_int32), ("n_proper", C.c_int32),
                ("eps0", C.c_double), ("n_monopoles", C.c_int32), ("monopoles", C.POINTER(C.c_double)),
                ("precision", C.c_int32), ("smoother", C.c_int32), ("nu1", C.c_int32), ("nu2", C.c_int32),
                ("omega", C.c_double), ("norm_p", C.c_int32), ("max_iters", C.c_int32),
                ("bottom_rtol", C.c_double), ("bottom", C.c_int32), ("tag_policy", C.c_int32),
                ("robin_d", C.c_double)]


class amrmg_solve_stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("nlevels", C.c_int32),
                ("bottom_iters_max", C.c_int32), ("rel_residual", C.c_double * AMRMG_MAX_LEVELS),
                ("time_ms", C.c_double), ("dof", C.c_int64)]

    def as_dict(self):
        return dict(iters=self.iters, converged=bool(self.converged), nlevels=self.nlevels,
                    bottom_iters_max=self.bottom_iters_max,
                    rel_residual=[self.rel_residual[i] for i in range(self.nlevels)],
                    time_ms=self.time_ms, dof=self.dof)


class AmrmgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    """The loaded shared library; raises when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libamrmg.so not built ({LIB_PATH}); run paper_1812_03689_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.amrmg_default_params.argtypes = [C.POINTER(amrmg_params)]
        L.amrmg_default_params.restype = None
        L.amrmg_create.argtypes = [C.POINTER(amrmg_params), vp, C.POINTER(vp)]
        L.amrmg_destroy.argtypes = [vp]
        L.amrmg_destroy.restype = None
        L.amrmg_last_error.restype = C.c_char_p
        L.amrmg_build_hierarchy.argtypes = [vp, C.c_int, vp, vp, vp, vp, i64, vp, vp, i32]
        L.amrmg_hierarchy_info.argtypes = [vp, vp, vp, vp, vp]
        L.amrmg_get_boxes.argtypes = [vp, i32, vp, vp]
        L.amrmg_cf_faces.argtypes = [vp, i32, vp, i64, vp]
        L.amrmg_brick_tables.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.amrmg_workspace_size.argtypes = [vp, C.POINTER(C.c_size_t)]
        L.amrmg_set_workspace.argtypes = [vp, vp, C.c_size_t]
        L.amrmg_deposit.argtypes = [vp, C.c_int, vp, vp, vp, vp, i64, vp, vp]
        L.amrmg_deposit_built.argtypes = [vp, vp, vp]
        L.amrmg_solve.argtypes = [vp, vp, vp, vp, dbl, C.POINTER(amrmg_solve_stats)]
        L.amrmg_solve_noalloc.argtypes = [vp, vp, vp, vp, dbl, C.POINTER(amrmg_solve_stats)]
        L.amrmg_gather.argtypes = [vp, C.c_int, vp, vp, vp, i64, vp, vp, vp, vp]
        L.amrmg_gather_built.argtypes = [vp, vp, vp, vp, vp]
        L.amrmg_visiting_order.argtypes = [vp, vp, C.c_int64]
        L.amrmg_residual.argtypes = [vp, vp, vp, vp]
        L.amrmg_solve_batch.argtypes = [vp, i32, vp, vp, dbl, C.POINTER(amrmg_solve_stats)]
        L.amrmg_profile_enable.argtypes = [vp, C.c_uint32]
        L.amrmg_profile_read.argtypes = [vp, i32, vp, vp, vp]
        L.amrmg_profile_launches.argtypes = [vp, i32, vp, vp, i64, vp]
        L.amrmg_transform_particles.argtypes = [vp, C.c_int, vp, vp, vp, i64, vp, vp, vp, vp, vp, vp]
        L.amrmg_rescale_fields.argtypes = [vp, dbl, vp, vp]
        _lib = L
    return _lib


def _check(rc, allow=()):
    if rc != AMRMG_OK and rc not in allow:
        raise AmrmgError(rc, lib().amrmg_last_error().decode())
    return rc


def _ptrs(tensors):
    P = (C.c_void_p * max(1, len(tensors)))()
    for i, t in enumerate(tensors):
        P[i] = None if t is None else t.data_ptr()
    return P


def _pos_dtype(t):
    import torch
    if t.dtype == torch.float64:
        return AMRMG_POS_F64
    if t.dtype == torch.float32:
        return AMRMG_POS_F32
    raise TypeError("positions must be float32 or float64")


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


# --- C-named entry points ---------------------------------------------------

def amrmg_default_params() -> amrmg_params:
    p = amrmg_params()
    lib().amrmg_default_params(C.byref(p))
    return p


def amrmg_create(params: amrmg_params, stream=None) -> C.c_void_p:
    h = C.c_void_p()
    _check(lib().amrmg_create(C.byref(params), _stream_handle(stream), C.byref(h)))
    return h


def amrmg_destroy(h) -> None:
    lib().amrmg_destroy(h)


def amrmg_build_hierarchy(h, x, y, z, q, tag_rel=None, explicit_boxes=None) -> None:
    n = int(q.numel())
    tr = None
    if tag_rel is not None and len(tag_rel):
        tr = (C.c_double * len(tag_rel))(*tag_rel)
    eb, ne = None, 0
    if explicit_boxes:
        flat = [int(v) for b in explicit_boxes for v in b]
        eb = (C.c_int32 * len(flat))(*flat)
        ne = len(explicit_boxes)
    _check(lib().amrmg_build_hierarchy(h, _pos_dtype(x), x.data_ptr(), y.data_ptr(), z.data_ptr(), q.data_ptr(),
                                       n, tr, eb, ne))


def amrmg_hierarchy_info(h):
    nl = C.c_int32()
    nb = (C.c_int32 * AMRMG_MAX_LEVELS)()
    nc = (C.c_int64 * AMRMG_MAX_LEVELS)()
    dof = C.c_int64()
    _check(lib().amrmg_hierarchy_info(h, C.byref(nl), nb, nc, C.byref(dof)))
    L = nl.value
    return dict(nlevels=L, nboxes=[nb[i] for i in range(L)], ncells=[nc[i] for i in range(L)], ndof=dof.value)


def amrmg_get_boxes(h, level: int):
    import numpy as np
    info = amrmg_hierarchy_info(h)
    nb = info["nboxes"][level]
    boxes = np.zeros((nb, 6), dtype=np.int32)
    off = np.zeros(nb + 1, dtype=np.int64)
    _check(lib().amrmg_get_boxes(h, level, boxes.ctypes.data, off.ctypes.data))
    return boxes, off


def amrmg_cf_faces(h, level: int):
    import numpy as np
    cnt = C.c_int64()
    _check(lib().amrmg_cf_faces(h, level, None, 0, C.byref(cnt)))
    out = np.zeros((max(1, cnt.value), 6), dtype=np.int32)
    _check(lib().amrmg_cf_faces(h, level, out.ctypes.data, cnt.value, C.byref(cnt)))
    return out[:cnt.value]


def amrmg_brick_tables(h) -> dict:
    """Host copies of the brick tables (include/amrmg.h, amrmg_brick_tables)."""
    import numpy as np
    cnt = np.zeros(4, dtype=np.int64)
    _check(lib().amrmg_brick_tables(h, cnt.ctypes.data, *([None] * 9)))
    nb, nbc, ncf, nup = (int(v) for v in cnt)
    t = {"org": np.zeros((nb, 4), np.int32), "nbr": np.zeros((nb, 6), np.int32), "child": np.zeros((nb, 8), np.int32),
         "parent": np.zeros(nb, np.int32), "cmask": np.zeros(nb, np.uint8), "ubase": np.zeros(nb, np.int64),
         "ustr": np.zeros((nb, 2), np.int32), "owner": np.zeros(nbc + ncf, np.int32),
         "update": np.zeros(nup, np.int32)}
    keys = ["org", "nbr", "child", "parent", "cmask", "ubase", "ustr", "owner", "update"]
    _check(lib().amrmg_brick_tables(h, cnt.ctypes.data, *[t[k].ctypes.data if t[k].size else None for k in keys]))
    t.update(nbrick=nb, nbc=nbc, ncf=ncf)
    return t


def amrmg_workspace_size(h) -> int:
    s = C.c_size_t()
    _check(lib().amrmg_workspace_size(h, C.byref(s)))
    return s.value


def amrmg_set_workspace(h, buf) -> None:
    if buf is None:
        _check(lib().amrmg_set_workspace(h, None, 0))
    else:
        _check(lib().amrmg_set_workspace(h, buf.data_ptr(), buf.numel() * buf.element_size()))


def amrmg_deposit(h, x, y, z, q, rho: Sequence, count_outside: bool = True) -> Optional[int]:
    """count_outside: return the number of particles outside the domain
    (the call then waits for the deposit); else None and no wait."""
    nout = C.c_int64()
    _check(lib().amrmg_deposit(h, _pos_dtype(x), x.data_ptr(), y.data_ptr(), z.data_ptr(), q.data_ptr(),
                               int(q.numel()), _ptrs(rho), C.byref(nout) if count_outside else None))
    return nout.value if count_outside else None


def amrmg_deposit_built(h, rho: Sequence, count_outside: bool = True) -> Optional[int]:
    """count_outside as in amrmg_deposit."""
    nout = C.c_int64()
    _check(lib().amrmg_deposit_built(h, _ptrs(rho), C.byref(nout) if count_outside else None))
    return nout.value if count_outside else None


def amrmg_solve(h, rho: Sequence, phi: Sequence, E: Optional[Sequence], tol: float, allow_not_converged=True):
    st = amrmg_solve_stats()
    allow = (AMRMG_E_NOT_CONVERGED,) if allow_not_converged else ()
    rc = _check(lib().amrmg_solve(h, _ptrs(rho), _ptrs(phi), _ptrs(E) if E is not None else None, float(tol),
                                  C.byref(st)), allow)
    d = st.as_dict()
    d["status"] = rc
    return d


def amrmg_solve_noalloc(h, rho: Sequence, phi: Sequence, E: Optional[Sequence], tol: float,
                        allow_not_converged=True):
    """amrmg_solve with its workspace in the library's static device array
    (no device allocation)."""
    st = amrmg_solve_stats()
    allow = (AMRMG_E_NOT_CONVERGED,) if allow_not_converged else ()
    rc = _check(lib().amrmg_solve_noalloc(h, _ptrs(rho), _ptrs(phi), _ptrs(E) if E is not None else None,
                                          float(tol), C.byref(st)), allow)
    d = st.as_dict()
    d["status"] = rc
    return d


def amrmg_gather(h, x, y, z, E: Sequence, Ex, Ey, Ez) -> None:
    _check(lib().amrmg_gather(h, _pos_dtype(x), x.data_ptr(), y.data_ptr(), z.data_ptr(), int(x.numel()),
                              _ptrs(E), Ex.data_ptr(), Ey.data_ptr(), Ez.data_ptr()))


def amrmg_gather_built(h, E: Sequence, Ex, Ey, Ez) -> None:
    _check(lib().amrmg_gather_built(h, _ptrs(E), Ex.data_ptr(), Ey.data_ptr(), Ez.data_ptr()))


def amrmg_visiting_order(h, perm, n: int) -> None:
    _check(lib().amrmg_visiting_order(h, perm.data_ptr() if n > 0 else None, int(n)))


def amrmg_residual(h, rho: Sequence, phi: Sequence, r: Sequence) -> None:
    _check(lib().amrmg_residual(h, _ptrs(rho), _ptrs(phi), _ptrs(r)))


def amrmg_solve_batch(handles: Sequence, rho: Sequence[Sequence], phi: Sequence[Sequence], tol: float):
    nb = len(handles)
    H = (C.c_void_p * nb)(*[h.value for h in handles])
    rp = [_ptrs(r) for r in rho]
    pp = [_ptrs(p) for p in phi]
    R = (C.c_void_p * nb)(*[C.cast(x, C.c_void_p).value for x in rp])
    P = (C.c_void_p * nb)(*[C.cast(x, C.c_void_p).value for x in pp])
    st = (amrmg_solve_stats * nb)()
    rc = _check(lib().amrmg_solve_batch(H, nb, R, P, float(tol), st), (AMRMG_E_NOT_CONVERGED,))
    out = [s.as_dict() for s in st]
    for d in out:
        d["status"] = rc
    return out


def amrmg_transform_particles(h, x, y, z, center, l, xs, ys, zs) -> float:
    c = (C.c_double * 3)(*[float(v) for v in center])
    ll = (C.c_double * 3)(*[float(v) for v in l])
    s = C.c_double()
    _check(lib().amrmg_transform_particles(h, _pos_dtype(x), x.data_ptr(), y.data_ptr(), z.data_ptr(),
                                           int(x.numel()), c, ll, xs.data_ptr(), ys.data_ptr(), zs.data_ptr(),
                                           C.byref(s)))
    return s.value


def amrmg_rescale_fields(h, s: float, phi: Optional[Sequence], E: Optional[Sequence]) -> None:
    _check(lib().amrmg_rescale_fields(h, float(s), _ptrs(phi) if phi is not None else None,
                                      _ptrs(E) if E is not None else None))


def amrmg_profile_enable(h, classes) -> None:
    mask = 0
    for c in classes:
        mask |= 1 << (KCLASS.index(c) if isinstance(c, str) else int(c))
    _check(lib().amrmg_profile_enable(h, mask))


def amrmg_profile_read(h, kclass):
    k = KCLASS.index(kclass) if isinstance(kclass, str) else int(kclass)
    ms, n, b = C.c_double(), C.c_int64(), C.c_double()
    _check(lib().amrmg_profile_read(h, k, C.byref(ms), C.byref(n), C.byref(b)))
    return dict(ms=ms.value, launches=n.value, bytes=b.value)


def amrmg_profile_launches(h, kclass):
    """Per-launch (ms, bytes) lists of one kernel class since the last enable."""
    import numpy as np
    k = KCLASS.index(kclass) if isinstance(kclass, str) else int(kclass)
    cnt = C.c_int64()
    _check(lib().amrmg_profile_launches(h, k, None, None, 0, C.byref(cnt)))
    ms = np.zeros(max(1, cnt.value))
    by = np.zeros(max(1, cnt.value))
    _check(lib().amrmg_profile_launches(h, k, ms.ctypes.data, by.ctypes.data, cnt.value, C.byref(cnt)))
    return ms[:cnt.value], by[:cnt.value]


# --- convenience wrapper ----------------------------------------------------

def make_params(n0, max_level=2, monopoles=(), precision="mixed", smoother="gsrb", nu1=2, nu2=4,
                max_grid_size=32, max_iters=50, norm_p=2, bottom_rtol=1e-2, lo=(0, 0, 0), hi=(1, 1, 1),
                eps0=1.0, n_buffer=1, n_proper=2, omega=6.0 / 7.0, bottom="auto", tag_policy="charge",
                robin_d=0.0):
    p = amrmg_default_params()
    for d in range(3):
        p.lo[d], p.hi[d], p.n0[d] = float(lo[d]), float(hi[d]), int(n0[d])
    p.max_level = int(max_level)
    p.max_grid_size = int(max_grid_size)
    p.n_buffer, p.n_proper = int(n_buffer), int(n_proper)
    p.eps0 = float(eps0)
    mono = [float(v) for m in monopoles for v in m]
    p._mono_keep = (C.c_double * max(1, len(mono)))(*mono)
    p.n_monopoles = len(monopoles)
    p.monopoles = C.cast(p._mono_keep, C.POINTER(C.c_double)) if mono else None
    p.precision = {"fp64": AMRMG_FP64, "mixed": AMRMG_MIXED}[precision]
    p.smoother = {"gsrb": AMRMG_GSRB, "jacobi": AMRMG_JACOBI, "gsrb_global": AMRMG_GSRB_GLOBAL}[smoother]
    p.nu1, p.nu2 = int(nu1), int(nu2)
    p.omega = float(omega)
    p.norm_p = int(norm_p)
    p.max_iters = int(max_iters)
    p.bottom_rtol = float(bottom_rtol)
    p.bottom = {"auto": AMRMG_BOTTOM_AUTO, "cg": AMRMG_BOTTOM_CG}[bottom]
    p.tag_policy = TAG_POLICIES[tag_policy]
    p.robin_d = float(robin_d)
    return p


class Context:
    """One problem: hierarchy, deposit, solve, gather (owns the C context)."""

    def __init__(self, params: amrmg_params, stream=None):
        self.params = params
        self.h = amrmg_create(params, stream)

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            amrmg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def build_hierarchy(self, x, y, z, q, tag_rel=None, explicit_boxes=None):
        amrmg_build_hierarchy(self.h, x, y, z, q, tag_rel, explicit_boxes)
        self.built_n = x.numel()
        self.info = amrmg_hierarchy_info(self.h)
        return self.info

    def boxes(self, level):
        return amrmg_get_boxes(self.h, level)

    def cf_faces(self, level):
        return amrmg_cf_faces(self.h, level)

    def brick_tables(self):
        return amrmg_brick_tables(self.h)

    def level_arrays(self, ncomp=1):
        import torch
        return [torch.zeros(n, dtype=torch.float64, device="cuda") for n in self.info["ncells"]
                for _ in range(ncomp)]

    def deposit(self, x, y, z, q, rho=None):
        rho = rho if rho is not None else self.level_arrays()
        nout = amrmg_deposit(self.h, x, y, z, q, rho)
        return rho, nout

    def deposit_built(self, rho=None):
        """Charge of the particles of the last build_hierarchy (amrmg_deposit_built)."""
        rho = rho if rho is not None else self.level_arrays()
        nout = amrmg_deposit_built(self.h, rho)
        return rho, nout

    def solve(self, rho, phi=None, E=None, tol=1e-8, want_E=True):
        phi = phi if phi is not None else self.level_arrays()
        if E is None and want_E:
            E = self.level_arrays(3)
        st = amrmg_solve(self.h, rho, phi, E, tol)
        return phi, E, st

    def residual(self, rho, phi):
        r = self.level_arrays()
        amrmg_residual(self.h, rho, phi, r)
        return r

    def gather(self, x, y, z, E):
        import torch
        n = x.numel()
        Ex, Ey, Ez = (torch.empty(n, dtype=torch.float64, device=x.device) for _ in range(3))
        amrmg_gather(self.h, x, y, z, E, Ex, Ey, Ez)
        return Ex, Ey, Ez

    def visiting_order(self):
        """The build's visiting order as an int64 tensor (amrmg_visiting_order)."""
        import torch
        perm = torch.empty(max(self.built_n, 0), dtype=torch.int32, device="cuda")
        amrmg_visiting_order(self.h, perm, self.built_n)
        return perm.to(torch.int64) & 0xFFFFFFFF

    def gather_built(self, E):
        """E at the particles of the last build_hierarchy, in their order
        (amrmg_gather_built)."""
        import torch
        Ex, Ey, Ez = (torch.empty(self.built_n, dtype=torch.float64, device="cuda") for _ in range(3))
        amrmg_gather_built(self.h, E, Ex, Ey, Ez)
        return Ex, Ey, Ez

    def transform_particles(self, x, y, z, center, l, out=None):
        """Map particles into computation space (amrmg_transform_particles):
        returns (xs, ys, zs, s); out=(x, y, z) transforms in place."""
        import torch
        xs, ys, zs = out if out is not None else (torch.empty_like(x), torch.empty_like(y), torch.empty_like(z))
        s = amrmg_transform_particles(self.h, x, y, z, center, l, xs, ys, zs)
        return xs, ys, zs, s

    def rescale_fields(self, s, phi=None, E=None):
        amrmg_rescale_fields(self.h, s, phi, E)
