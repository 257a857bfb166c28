"""ctypes binding of libpbdsbi.so (include/pbsolve.h): argument marshalling only.

Every step of the path runs in the HIP library; this module converts numpy
arrays / torch device tensors to the C structs and pointers of the ABI and
turns negative status codes into :class:`PbError`.  There is no fallback:
when the library is not built, loading raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpbdsbi.so")

PB_OK = 0
PB_NOT_CONVERGED = 1
PB_ERR_ARG = -1
PB_ERR_GEOMETRY = -2
PB_ERR_CHARGE = -3
PB_ERR_HIP = -4
PB_ERR_OOM = -5
PB_FP64 = 0
PB_FP32_IR = 1
PB_SWEEP_PAIRWISE = 8   # pb_set_sweep_config kind: each unordered pair once
PB_SWEEP_BANDED = 16    # FP32: pairwise with four target tiles per workgroup, banded items
PB_KERNEL_PAIRS_FP64 = 0
PB_KERNEL_PAIRS_FP32 = 1
PB_KERNEL_PAIRS_FP64_T = 2
PB_KERNEL_PAIRS_FP32_T = 3
PB_KERNEL_SOURCE = 4
PB_KERNEL_CHARGE = 5
PB_KERNEL_TREE = 6
PB_PROBE_FMA_F32 = 0    # pb_probe_valu kinds
PB_PROBE_FMA_F64 = 1
PB_PROBE_EXP_F32 = 2
PB_PAIR_MATH_MAX = 1 << 24   # pb_eval_pair_math limits
PB_PAIR_MATH_XMAX = 1e12
PB_PAIR_MATH_YMIN = 1e-30
PB_PAIR_MATH_YMAX = 1e30

# Every function the header declares, with its C prototype in ctypes terms.
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_int = ctypes.c_int
_dbl = ctypes.c_double


class _Surface(ctypes.Structure):
    _fields_ = [("n_vert", _i64), ("n_tri", _i64), ("vert", _vp), ("tri", _vp)]


class _Charges(ctypes.Structure):
    _fields_ = [("n", _i64), ("pos", _vp), ("q", _vp)]


class _Params(ctypes.Structure):
    _fields_ = [("eps_in", _dbl), ("eps_out", _dbl), ("kappa", _dbl), ("tol", _dbl),
                ("restart", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("max_refine", ctypes.c_int32),
                ("inner_tol", _dbl), ("precond_leaf", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("e_solv", _dbl), ("rel_residual", _dbl), ("seconds", _dbl),
                ("iters", ctypes.c_int32), ("matvecs_fp64", ctypes.c_int32),
                ("matvecs_fp32", ctypes.c_int32), ("refinements", ctypes.c_int32),
                ("status", ctypes.c_int32), ("adjoint_iters", ctypes.c_int32)]


_PROTOS = {
    "pb_abi_version": (_int, []),
    "pb_create": (_int, [_int, _vp, ctypes.POINTER(_vp)]),
    "pb_destroy": (None, [_vp]),
    "pb_last_error": (ctypes.c_char_p, [_vp]),
    "pb_geometry": (_int, [_vp, ctypes.POINTER(_Surface), _vp, _vp, _vp]),
    "pb_source": (_int, [_vp, ctypes.POINTER(_Surface), ctypes.POINTER(_Charges),
                         ctypes.POINTER(_Params), _vp]),
    "pb_matvec": (_int, [_vp, ctypes.POINTER(_Surface), ctypes.POINTER(_Params), _vp, _vp,
                         _int, _int]),
    "pb_matvec_tree": (_int, [_vp, ctypes.POINTER(_Surface), ctypes.POINTER(_Params), _dbl,
                              _int, _int, _vp, _vp, _vp]),
    "pb_solve_tree": (_int, [_vp, ctypes.POINTER(_Surface), ctypes.POINTER(_Charges),
                             ctypes.POINTER(_Params), _dbl, _int, _int, _vp, _vp,
                             ctypes.POINTER(_Info)]),
    "pb_energy": (_int, [_vp, ctypes.POINTER(_Surface), ctypes.POINTER(_Charges),
                         ctypes.POINTER(_Params), _vp, _vp, ctypes.POINTER(_dbl)]),
    "pb_solve": (_int, [_vp, ctypes.POINTER(_Surface), ctypes.POINTER(_Charges),
                        ctypes.POINTER(_Params), _vp, _vp, ctypes.POINTER(_Info)]),
    "pb_matvec_dev": (_int, [_vp, _i64, _i64, _vp, _vp, ctypes.POINTER(_Params), _vp, _vp,
                             _int, _int]),
    "pb_matvec_dev_noalloc": (_int, [_vp, _i64, _i64, _vp, _vp, ctypes.POINTER(_Params), _vp,
                                     _vp, _int, _int]),
    "pb_solve_dev": (_int, [_vp, _i64, _i64, _vp, _vp, _i64, _vp, _vp,
                            ctypes.POINTER(_Params), _vp, _vp, ctypes.POINTER(_Info)]),
    "pb_source_dev": (_int, [_vp, _i64, _i64, _vp, _vp, _i64, _vp, _vp,
                             ctypes.POINTER(_Params), _vp]),
    "pb_energy_dev": (_int, [_vp, _i64, _i64, _vp, _vp, _i64, _vp, _vp,
                             ctypes.POINTER(_Params), _vp, _vp, ctypes.POINTER(_dbl)]),
    "pb_solve_batch_dev": (_int, [_vp, ctypes.c_int32, ctypes.POINTER(_Surface),
                                  ctypes.POINTER(_Charges), ctypes.POINTER(_Params), _vp, _vp,
                                  _vp, ctypes.POINTER(_Info)]),
    "pb_forces": (_int, [_vp, ctypes.POINTER(_Surface), ctypes.POINTER(_Charges),
                         ctypes.POINTER(_Params), _vp, _vp, ctypes.POINTER(_Info)]),
    "pb_forces_dev": (_int, [_vp, _i64, _i64, _vp, _vp, _i64, _vp, _vp,
                             ctypes.POINTER(_Params), _vp, _vp, ctypes.POINTER(_Info)]),
    "pb_solve_batch": (_int, [_vp, ctypes.c_int32, ctypes.POINTER(_Surface),
                              ctypes.POINTER(_Charges), ctypes.POINTER(_Params), _vp, _vp, _vp,
                              ctypes.POINTER(_Info)]),
    "pb_potential": (_int, [_vp, ctypes.POINTER(_Surface), ctypes.POINTER(_Charges),
                            ctypes.POINTER(_Params), _vp, _vp, _i64, _vp, _vp, _vp]),
    "pb_coulomb_energy": (_int, [_vp, ctypes.POINTER(_Charges), ctypes.POINTER(_Params),
                                 ctypes.POINTER(_dbl)]),
    "pb_precond_leaves": (_int, [_vp, ctypes.POINTER(_Surface), _int, _vp, _vp,
                                 ctypes.POINTER(_i64)]),
    "pb_precond_apply": (_int, [_vp, ctypes.POINTER(_Surface), ctypes.POINTER(_Params), _vp, _vp,
                                _int]),
    "pb_set_sweep_config": (_int, [_vp, _int, _int]),
    "pb_set_fp64_sweep": (_int, [_vp, _int]),
    "pb_get_fp64_sweep": (_int, [_vp, ctypes.POINTER(_int)]),
    "pb_get_sweep_config": (_int, [_vp, ctypes.POINTER(_int), ctypes.POINTER(_int)]),
    "pb_autotune": (_int, [_vp, ctypes.POINTER(_Surface), ctypes.POINTER(_Params),
                           ctypes.POINTER(_int), ctypes.POINTER(_int)]),
    "pb_autotune_batch": (_int, [_vp, ctypes.c_int32, ctypes.POINTER(_Surface),
                                 ctypes.POINTER(_Charges), ctypes.POINTER(_Params),
                                 ctypes.POINTER(_int), ctypes.POINTER(_int)]),
    "pb_set_batch_tiles": (_int, [_vp, _int]),
    "pb_get_batch_tiles": (_int, [_vp, ctypes.POINTER(_int)]),
    "pb_set_memory_limit": (_int, [_vp, _i64]),
    "pb_get_memory_used": (_int, [_vp, ctypes.POINTER(_i64)]),
    "pb_profile_enable": (_int, [_vp, _int]),
    "pb_profile_reset": (_int, [_vp]),
    "pb_probe_valu": (_int, [_vp, _int, ctypes.POINTER(_i64)]),
    "pb_eval_pair_math": (_int, [_vp, _i64, _vp, _vp, _vp, _vp]),
    "pb_profile_read": (_int, [_vp, _int, ctypes.POINTER(_i64), ctypes.POINTER(_dbl),
                               ctypes.POINTER(_dbl)]),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libpbdsbi.so and attach prototypes.  Raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"HIP library {path} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(path)
        for name, (res, args) in _PROTOS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_PROTOS)


class PbError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"status {status}: {message}")
        self.status = status
        self.message = message


@dataclass
class Params:
    eps_in: float = 1.0
    eps_out: float = 80.0
    kappa: float = 0.1257
    tol: float = 1e-6
    restart: int = 10
    max_iter: int = 1000
    precision: int = PB_FP64
    max_refine: int = 20
    inner_tol: float = 1e-4
    precond_leaf: int = 0

    def c(self) -> _Params:
        return _Params(float(self.eps_in), float(self.eps_out), float(self.kappa), float(self.tol),
                       int(self.restart), int(self.max_iter), int(self.precision),
                       int(self.max_refine), float(self.inner_tol), int(self.precond_leaf), 0)


@dataclass
class Info:
    e_solv: float
    rel_residual: float
    seconds: float
    iters: int
    matvecs_fp64: int
    matvecs_fp32: int
    refinements: int
    status: int
    adjoint_iters: int = 0

    @staticmethod
    def of(ci: _Info) -> "Info":
        return Info(ci.e_solv, ci.rel_residual, ci.seconds, ci.iters, ci.matvecs_fp64,
                    ci.matvecs_fp32, ci.refinements, ci.status, ci.adjoint_iters)


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, _vp(a.ctypes.data)


def _dev(t, dtype_name: str):
    """Pointer of a contiguous torch device tensor of the given dtype."""
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous() or str(t.dtype) != "torch." + dtype_name:
        raise PbError(PB_ERR_ARG, f"expected a contiguous {dtype_name} device tensor")
    return _vp(t.data_ptr())


class Context:
    """One pb_ctx: a device, a stream and the device scratch reused across calls."""

    def __init__(self, device: int = 0, stream=None):
        L = load_library()
        h = _vp()
        s = None
        if stream is not None:
            s = _vp(stream if isinstance(stream, int) else int(stream.cuda_stream))
        st = L.pb_create(int(device), s, ctypes.byref(h))
        if st != PB_OK or not h.value:
            raise PbError(st, f"pb_create(device={device}) failed")
        self._h = h
        self._L = L

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._L.pb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, st: int) -> int:
        if st < 0:
            raise PbError(st, self._L.pb_last_error(self._h).decode())
        return st

    @staticmethod
    def _surface(verts, tris):
        v, pv = _host(verts, np.float64)
        t, pt = _host(tris, np.int32)
        return _Surface(v.shape[0], t.shape[0], pv, pt), (v, t)

    @staticmethod
    def _charges(pos, q):
        p, pp = _host(pos, np.float64)
        qq, pq = _host(q, np.float64)
        return _Charges(qq.shape[0], pp, pq), (p, qq)

    # -- host-pointer entry points ------------------------------------------
    def pb_geometry(self, verts, tris):
        s, keep = self._surface(verts, tris)
        n = s.n_tri
        cen = np.empty((n, 3))
        nrm = np.empty((n, 3))
        area = np.empty(n)
        self._check(self._L.pb_geometry(self._h, ctypes.byref(s), _vp(cen.ctypes.data),
                                        _vp(nrm.ctypes.data), _vp(area.ctypes.data)))
        return cen, nrm, area

    def pb_source(self, verts, tris, pos, q, params: Params):
        s, k1 = self._surface(verts, tris)
        c, k2 = self._charges(pos, q)
        b = np.empty(2 * s.n_tri)
        p = params.c()
        self._check(self._L.pb_source(self._h, ctypes.byref(s), ctypes.byref(c), ctypes.byref(p),
                                      _vp(b.ctypes.data)))
        return b

    def pb_matvec(self, verts, tris, x, params: Params, transpose=False, precision=PB_FP64):
        s, k1 = self._surface(verts, tris)
        xx, px = _host(x, np.float64)
        y = np.empty_like(xx)
        p = params.c()
        self._check(self._L.pb_matvec(self._h, ctypes.byref(s), ctypes.byref(p), px,
                                      _vp(y.ctypes.data), int(bool(transpose)), int(precision)))
        return y

    def pb_matvec_tree(self, verts, tris, x, params: Params, theta=0.8, order=3, leaf_size=100,
                       with_counts=False):
        """Treecode matvec; returns y, or (y, (n_far, n_pairs, n_nodes))."""
        s, k1 = self._surface(verts, tris)
        xx, px = _host(x, np.float64)
        y = np.empty_like(xx)
        p = params.c()
        cnt = np.zeros(3, dtype=np.int64)
        self._check(self._L.pb_matvec_tree(self._h, ctypes.byref(s), ctypes.byref(p),
                                           float(theta), int(order), int(leaf_size), px,
                                           _vp(y.ctypes.data),
                                           _vp(cnt.ctypes.data) if with_counts else None))
        return (y, tuple(int(v) for v in cnt)) if with_counts else y

    def pb_energy(self, verts, tris, pos, q, phi, dphi, params: Params) -> float:
        s, k1 = self._surface(verts, tris)
        c, k2 = self._charges(pos, q)
        a, pa = _host(phi, np.float64)
        b, pb = _host(dphi, np.float64)
        e = _dbl()
        p = params.c()
        self._check(self._L.pb_energy(self._h, ctypes.byref(s), ctypes.byref(c), ctypes.byref(p),
                                      pa, pb, ctypes.byref(e)))
        return float(e.value)

    def pb_solve(self, verts, tris, pos, q, params: Params):
        """Returns (info, phi, dphi); info.status is PB_OK or PB_NOT_CONVERGED."""
        s, k1 = self._surface(verts, tris)
        c, k2 = self._charges(pos, q)
        phi = np.empty(s.n_tri)
        dphi = np.empty(s.n_tri)
        info = _Info()
        p = params.c()
        self._check(self._L.pb_solve(self._h, ctypes.byref(s), ctypes.byref(c), ctypes.byref(p),
                                     _vp(phi.ctypes.data), _vp(dphi.ctypes.data),
                                     ctypes.byref(info)))
        return Info.of(info), phi, dphi

    def pb_solve_tree(self, verts, tris, pos, q, params: Params, theta=0.8, order=3,
                      leaf_size=100):
        """pb_solve with the treecode matvec; returns (info, phi, dphi)."""
        s, k1 = self._surface(verts, tris)
        c, k2 = self._charges(pos, q)
        phi = np.empty(s.n_tri)
        dphi = np.empty(s.n_tri)
        info = _Info()
        p = params.c()
        self._check(self._L.pb_solve_tree(self._h, ctypes.byref(s), ctypes.byref(c),
                                          ctypes.byref(p), float(theta), int(order),
                                          int(leaf_size), _vp(phi.ctypes.data),
                                          _vp(dphi.ctypes.data), ctypes.byref(info)))
        return Info.of(info), phi, dphi

    def pb_forces(self, verts, tris, pos, q, params: Params):
        """Returns (info, dE_dpos [Nc,3], dE_dq [Nc]) for a fixed surface."""
        s, k1 = self._surface(verts, tris)
        c, k2 = self._charges(pos, q)
        gpos = np.empty((c.n, 3))
        gq = np.empty(c.n)
        info = _Info()
        p = params.c()
        self._check(self._L.pb_forces(self._h, ctypes.byref(s), ctypes.byref(c), ctypes.byref(p),
                                      _vp(gpos.ctypes.data), _vp(gq.ctypes.data),
                                      ctypes.byref(info)))
        return Info.of(info), gpos, gq

    def _batch_args(self, systems):
        n = len(systems)
        surfs = (_Surface * n)()
        chgs = (_Charges * n)()
        keep = []
        nct = 0
        for b, (v, t, pos, q) in enumerate(systems):
            s, k1 = self._surface(v, t)
            c, k2 = self._charges(pos, q)
            surfs[b] = s
            chgs[b] = c
            keep += [k1, k2]
            nct += c.n
        return n, surfs, chgs, keep, nct

    def pb_autotune_batch(self, systems, params: Params):
        """Time the batched FP32 sweep configurations on this batch and keep
        the fastest; returns (sweep kind, source tiles per work item)."""
        n, surfs, chgs, keep, _nct = self._batch_args(systems)
        p = params.c()
        kind, tiles = _int(0), _int(0)
        self._check(self._L.pb_autotune_batch(self._h, n, surfs, chgs, ctypes.byref(p),
                                              ctypes.byref(kind), ctypes.byref(tiles)))
        return int(kind.value), int(tiles.value)

    def set_batch_tiles(self, tiles: int = 0):
        """Source tiles per pairwise work item of the batched sweeps; 0 keeps it."""
        self._check(self._L.pb_set_batch_tiles(self._h, int(tiles)))

    def get_batch_tiles(self) -> int:
        t = _int(0)
        self._check(self._L.pb_get_batch_tiles(self._h, ctypes.byref(t)))
        return int(t.value)

    def pb_solve_batch(self, systems, params: Params, forces: bool = False):
        """systems: list of (verts, tris, pos, q).  Returns (e [n_sys], infos,
        dE_dpos [sum n_b, 3] or None, dE_dq [sum n_b] or None)."""
        n, surfs, chgs, keep, nct = self._batch_args(systems)
        e = np.empty(n)
        infos = (_Info * n)()
        gpos = np.empty((nct, 3)) if forces else None
        gq = np.empty(nct) if forces else None
        p = params.c()
        self._check(self._L.pb_solve_batch(self._h, n, surfs, chgs, ctypes.byref(p),
                                           _vp(e.ctypes.data),
                                           _vp(gpos.ctypes.data) if forces else None,
                                           _vp(gq.ctypes.data) if forces else None, infos))
        return e, [Info.of(infos[b]) for b in range(n)], gpos, gq

    # -- device-pointer entry points (torch tensors) --------------------------
    def pb_matvec_dev(self, verts, tris, x, y, params: Params, transpose=False,
                      precision=PB_FP64):
        p = params.c()
        self._check(self._L.pb_matvec_dev(self._h, verts.shape[0], tris.shape[0],
                                          _dev(verts, "float64"), _dev(tris, "int32"), ctypes.byref(p),
                                          _dev(x, "float64"), _dev(y, "float64"),
                                          int(bool(transpose)), int(precision)))
        return y

    def pb_matvec_dev_noalloc(self, verts, tris, x, y, params: Params, transpose=False,
                              precision=PB_FP64):
        """pb_matvec_dev without device allocation (fixed library scratch)."""
        p = params.c()
        self._check(self._L.pb_matvec_dev_noalloc(self._h, verts.shape[0], tris.shape[0],
                                                  _dev(verts, "float64"), _dev(tris, "int32"),
                                                  ctypes.byref(p), _dev(x, "float64"),
                                                  _dev(y, "float64"), int(bool(transpose)),
                                                  int(precision)))
        return y

    def pb_solve_dev(self, verts, tris, pos, q, params: Params, phi=None, dphi=None) -> Info:
        p = params.c()
        info = _Info()
        self._check(self._L.pb_solve_dev(self._h, verts.shape[0], tris.shape[0],
                                         _dev(verts, "float64"), _dev(tris, "int32"), q.shape[0],
                                         _dev(pos, "float64"), _dev(q, "float64"), ctypes.byref(p),
                                         _dev(phi, "float64"), _dev(dphi, "float64"),
                                         ctypes.byref(info)))
        return Info.of(info)

    def pb_forces_dev(self, verts, tris, pos, q, params: Params, dE_dpos, dE_dq) -> Info:
        p = params.c()
        info = _Info()
        self._check(self._L.pb_forces_dev(self._h, verts.shape[0], tris.shape[0],
                                          _dev(verts, "float64"), _dev(tris, "int32"), q.shape[0],
                                          _dev(pos, "float64"), _dev(q, "float64"), ctypes.byref(p),
                                          _dev(dE_dpos, "float64"), _dev(dE_dq, "float64"),
                                          ctypes.byref(info)))
        return Info.of(info)

    def pb_source_dev(self, verts, tris, pos, q, params: Params, b):
        """b [2 n_tri] <- [S1; S2] on device tensors."""
        p = params.c()
        self._check(self._L.pb_source_dev(self._h, verts.shape[0], tris.shape[0],
                                          _dev(verts, "float64"), _dev(tris, "int32"), q.shape[0],
                                          _dev(pos, "float64"), _dev(q, "float64"),
                                          ctypes.byref(p), _dev(b, "float64")))
        return b

    def pb_energy_dev(self, verts, tris, pos, q, phi, dphi, params: Params) -> float:
        p = params.c()
        e = _dbl()
        self._check(self._L.pb_energy_dev(self._h, verts.shape[0], tris.shape[0],
                                          _dev(verts, "float64"), _dev(tris, "int32"), q.shape[0],
                                          _dev(pos, "float64"), _dev(q, "float64"),
                                          ctypes.byref(p), _dev(phi, "float64"),
                                          _dev(dphi, "float64"), ctypes.byref(e)))
        return float(e.value)

    def pb_solve_batch_dev(self, systems, params: Params, dE_dpos=None, dE_dq=None):
        """systems: list of (verts, tris, pos, q) device tensors (float64, int32,
        float64, float64).  Returns (e [n_sys], infos); gradients, when wanted,
        go to the device tensors dE_dpos [sum n_b, 3] and dE_dq [sum n_b]."""
        n = len(systems)
        surfs = (_Surface * n)()
        chgs = (_Charges * n)()
        for b, (v, t, pos, q) in enumerate(systems):
            surfs[b] = _Surface(v.shape[0], t.shape[0], _dev(v, "float64"), _dev(t, "int32"))
            chgs[b] = _Charges(q.shape[0], _dev(pos, "float64"), _dev(q, "float64"))
        e = np.empty(n)
        infos = (_Info * n)()
        p = params.c()
        self._check(self._L.pb_solve_batch_dev(self._h, n, surfs, chgs, ctypes.byref(p),
                                               _vp(e.ctypes.data), _dev(dE_dpos, "float64"),
                                               _dev(dE_dq, "float64"), infos))
        return e, [Info.of(infos[b]) for b in range(n)]

    def pb_potential(self, verts, tris, pos, q, phi, dphi, points, params: Params):
        """(reaction, total) potential at interior points (BIE units)."""
        s, k1 = self._surface(verts, tris)
        c, k2 = self._charges(pos, q)
        a, pa = _host(phi, np.float64)
        b, pb = _host(dphi, np.float64)
        pts, pp = _host(points, np.float64)
        npts = pts.shape[0]
        reac = np.empty(npts)
        tot = np.empty(npts)
        p = params.c()
        self._check(self._L.pb_potential(self._h, ctypes.byref(s), ctypes.byref(c), ctypes.byref(p),
                                         pa, pb, npts, pp, _vp(reac.ctypes.data),
                                         _vp(tot.ctypes.data)))
        return reac, tot

    def pb_coulomb_energy(self, pos, q, params: Params) -> float:
        c, k = self._charges(pos, q)
        e = _dbl()
        p = params.c()
        self._check(self._L.pb_coulomb_energy(self._h, ctypes.byref(c), ctypes.byref(p),
                                              ctypes.byref(e)))
        return float(e.value)

    # -- preconditioner hooks ----------------------------------------------------
    def pb_precond_leaves(self, verts, tris, leaf: int):
        """Octree leaves of the preconditioner: list of index arrays."""
        s, keep = self._surface(verts, tris)
        perm = np.empty(s.n_tri, dtype=np.int32)
        start = np.empty(s.n_tri + 1, dtype=np.int32)
        nl = _i64()
        self._check(self._L.pb_precond_leaves(self._h, ctypes.byref(s), int(leaf),
                                              _vp(perm.ctypes.data), _vp(start.ctypes.data),
                                              ctypes.byref(nl)))
        L = int(nl.value)
        return [perm[start[k]:start[k + 1]].astype(np.int64) for k in range(L)]

    def pb_precond_apply(self, verts, tris, x, params: Params, transpose=False):
        s, keep = self._surface(verts, tris)
        xx, px = _host(x, np.float64)
        y = np.empty_like(xx)
        p = params.c()
        self._check(self._L.pb_precond_apply(self._h, ctypes.byref(s), ctypes.byref(p), px,
                                             _vp(y.ctypes.data), int(bool(transpose))))
        return y

    # -- launch configuration --------------------------------------------------
    def set_fp64_sweep(self, kind: int = 0):
        """FP64 sweep kind: 1 (per target) or PB_SWEEP_PAIRWISE; 0 keeps it."""
        self._check(self._L.pb_set_fp64_sweep(self._h, int(kind)))

    def get_fp64_sweep(self) -> int:
        k = _int(0)
        self._check(self._L.pb_get_fp64_sweep(self._h, ctypes.byref(k)))
        return int(k.value)

    def set_sweep_config(self, targets_per_thread: int = 0, target_waves: int = 0):
        self._check(self._L.pb_set_sweep_config(self._h, int(targets_per_thread),
                                                int(target_waves)))

    def get_sweep_config(self):
        a, b = _int(), _int()
        self._check(self._L.pb_get_sweep_config(self._h, ctypes.byref(a), ctypes.byref(b)))
        return int(a.value), int(b.value)

    def pb_autotune(self, verts, tris, params: Params):
        s, keep = self._surface(verts, tris)
        a, b = _int(), _int()
        p = params.c()
        self._check(self._L.pb_autotune(self._h, ctypes.byref(s), ctypes.byref(p),
                                        ctypes.byref(a), ctypes.byref(b)))
        return int(a.value), int(b.value)

    # -- device memory -------------------------------------------------------------
    def set_memory_limit(self, nbytes: int):
        """Cap on the context's device scratch (0: none); past it calls fail
        with PB_ERR_OOM before allocating."""
        self._check(self._L.pb_set_memory_limit(self._h, int(nbytes)))

    def memory_used(self) -> int:
        v = _i64()
        self._check(self._L.pb_get_memory_used(self._h, ctypes.byref(v)))
        return int(v.value)

    # -- kernel timing hook ------------------------------------------------------
    def profile_enable(self, on: bool = True):
        self._check(self._L.pb_profile_enable(self._h, int(bool(on))))

    def profile_reset(self):
        self._check(self._L.pb_profile_reset(self._h))

    def probe_valu(self, kind: int) -> int:
        """One launch of the counter-calibration probe; returns its exact
        operation count (lane-level)."""
        n = _i64()
        self._check(self._L.pb_probe_valu(self._h, int(kind), ctypes.byref(n)))
        return int(n.value)

    def eval_pair_math(self, x, y):
        """(exp(-x), 1/sqrt(y)) by the FP64 pair sweeps' device functions."""
        xx, px = _host(x, np.float64)
        yy, py = _host(y, np.float64)
        if xx.shape != yy.shape or xx.ndim != 1:
            raise PbError(PB_ERR_ARG, "x and y must be 1-d arrays of one length")
        ex = np.empty_like(xx)
        rq = np.empty_like(yy)
        self._check(self._L.pb_eval_pair_math(self._h, int(xx.size), px, py,
                                              _vp(ex.ctypes.data), _vp(rq.ctypes.data)))
        return ex, rq

    def profile_read(self, kernel: int):
        """(launches, total_ms, algorithmic pairs) accumulated for one kernel id."""
        n = _i64()
        ms = _dbl()
        pr = _dbl()
        self._check(self._L.pb_profile_read(self._h, int(kernel), ctypes.byref(n),
                                            ctypes.byref(ms), ctypes.byref(pr)))
        return int(n.value), float(ms.value), float(pr.value)
