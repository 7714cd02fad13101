"""FP64 CPU oracle for inverse ray-shooting near a critical curve.

TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the
CPU-baseline leg of ``bench.py`` may import this package; the product path
(``paper_2308_14278_amd``) never does, and the two share no code.  The only
module both sides use is the seeded input generator
``paper_2308_14278_amd.inputs``, which holds none of the method's arithmetic.

``lensoracle.c`` holds the arithmetic (see its header for the equations and the
paper passages they follow); this module compiles it with gcc and wraps it with
ctypes.  ``geometry.py`` derives the ray lattice and grid sizes from the paper's
rules, independently of the library's own derivation.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .geometry import OracleGeometry, derive_fold_geometry, derive_geometry  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lensoracle.c")
_LIB = os.path.join(_HERE, "liblensoracle.so")

SCHEME_DIRECT = 0
SCHEME_INTERP = 1


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2 -fopenmp).  Returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("src_x0", ctypes.c_double), ("src_y0", ctypes.c_double),
        ("src_dx", ctypes.c_double), ("src_dy", ctypes.c_double),
        ("src_nx", ctypes.c_int64), ("src_ny", ctypes.c_int64),
        ("ray_x0", ctypes.c_double), ("ray_y0", ctypes.c_double),
        ("ray_dx", ctypes.c_double), ("ray_dy", ctypes.c_double),
        ("ray_nx", ctypes.c_int64), ("ray_ny", ctypes.c_int64),
        ("kappa", ctypes.c_double), ("gamma", ctypes.c_double),
        ("kappa_star", ctypes.c_double),
        ("scheme", ctypes.c_int64), ("coarse", ctypes.c_int64),
        ("l1_kx", ctypes.c_int64), ("l1_ky", ctypes.c_int64),
        ("halo", ctypes.c_int64), ("terms", ctypes.c_int64),
        ("macro", ctypes.c_int64), ("d_x", ctypes.c_double), ("d_y", ctypes.c_double),
        ("far_order", ctypes.c_int64),
        ("sheet", ctypes.c_int64), ("sx0", ctypes.c_double), ("sx1", ctypes.c_double),
        ("sy0", ctypes.c_double), ("sy1", ctypes.c_double),
    ]


_lib = None
_P = ctypes.POINTER
_d = _P(ctypes.c_double)
_i64 = _P(ctypes.c_int64)
_u64 = _P(ctypes.c_uint64)


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        pp = _P(_Params)
        lib.lmo_deflect_direct.argtypes = [_d, _d, _d, ctypes.c_int64, _d, ctypes.c_int64, _d]
        lib.lmo_coeffs.argtypes = [pp, _d, _d, _d, ctypes.c_int64, ctypes.c_int64,
                                   ctypes.c_int64, _d]
        lib.lmo_near_mask.argtypes = [pp, _d, _d, ctypes.c_int64, ctypes.c_int64,
                                      ctypes.c_int64, _P(ctypes.c_uint8)]
        lib.lmo_deflect.argtypes = [pp, _d, _d, _d, ctypes.c_int64, _d, ctypes.c_int64, _d]
        lib.lmo_trace.argtypes = [pp, _d, _d, _d, ctypes.c_int64, _i64, _i64, ctypes.c_int64,
                                  _d, _i64]
        lib.lmo_shoot.argtypes = [pp, _d, _d, _d, ctypes.c_int64, ctypes.c_int64,
                                  ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _u64, _u64,
                                  ctypes.c_int]
        lib.lmo_shoot_window.argtypes = [pp, _d, _d, _d, ctypes.c_int64, ctypes.c_int64,
                                         ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                         ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                         ctypes.c_int64, _u64, _u64, ctypes.c_int]
        lib.lmo_shoot_window.restype = ctypes.c_int
        lib.lmo_mu_factor.argtypes = [pp]
        lib.lmo_mu_factor.restype = ctypes.c_double
        lib.lmo_num_threads.restype = ctypes.c_int
        lib.lmo_sheet.argtypes = [pp, _d, ctypes.c_int64, _d]
        lib.lmo_sheet.restype = ctypes.c_int
        for f in (lib.lmo_deflect_direct, lib.lmo_coeffs, lib.lmo_near_mask, lib.lmo_deflect,
                  lib.lmo_trace, lib.lmo_shoot):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(_d)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Oracle:
    """One problem instance: geometry + macro model + lenses.

    ``geom`` is an :class:`OracleGeometry` (or anything with the same fields).
    Lenses are copied to contiguous float64 arrays.
    """

    def __init__(self, geom, kappa, gamma, kappa_star, lx, ly, lm, fold=None, sheet=None):
        """fold=(kappa_0, d_x, d_y) selects the fold macro model of Eq. 5/6
        (d in 1/theta_E); kappa and gamma are then ignored.  sheet=(x0, x1, y0,
        y1): the -kappa_star sheet covers that rectangle (the region of the
        lenses); None: an infinite sheet about the origin."""
        self.geom = geom
        self.kappa, self.gamma, self.kappa_star = float(kappa), float(gamma), float(kappa_star)
        macro, dx, dy = 0, 0.0, 0.0
        if fold is not None:
            macro = 1
            self.kappa, dx, dy = float(fold[0]), float(fold[1]), float(fold[2])
            self.gamma = 0.0
        self.lx, self.ly, self.lm = _f64(lx), _f64(ly), _f64(lm)
        if not (self.lx.shape == self.ly.shape == self.lm.shape) or self.lx.ndim != 1:
            raise ValueError("lens arrays must be 1-D and of equal length")
        g = geom
        self._p = _Params(
            g.src_x0, g.src_y0, g.src_dx, g.src_dy, g.src_nx, g.src_ny,
            g.ray_x0, g.ray_y0, g.ray_dx, g.ray_dy, g.ray_nx, g.ray_ny,
            self.kappa, self.gamma, self.kappa_star,
            g.scheme, g.coarse, g.l1_kx, g.l1_ky, g.halo, g.terms, macro, dx, dy,
            getattr(g, "far_order", 0), 0 if sheet is None else 1,
            *(float(v) for v in (sheet if sheet is not None else (0.0, 0.0, 0.0, 0.0))))

    @property
    def n(self):
        return int(self.lx.shape[0])

    def _lens(self):
        return _dp(self.lx), _dp(self.ly), _dp(self.lm), self.n

    def deflect(self, theta):
        """Deflection of the configured scheme at positions theta[n,2] (FP64)."""
        th = _f64(theta).reshape(-1, 2)
        out = np.empty_like(th)
        rc = _load().lmo_deflect(ctypes.byref(self._p), *self._lens(), _dp(th), th.shape[0],
                                 _dp(out))
        if rc:
            raise RuntimeError("lmo_deflect failed (%d)" % rc)
        return out

    def sheet(self, theta):
        """The sheet term s(theta) of the lens equation at positions theta[n,2]."""
        th = _f64(theta).reshape(-1, 2)
        out = np.empty_like(th)
        rc = _load().lmo_sheet(ctypes.byref(self._p), _dp(th), th.shape[0], _dp(out))
        if rc:
            raise RuntimeError("lmo_sheet failed (%d)" % rc)
        return out

    def deflect_direct(self, theta):
        """Direct-sum deflection over all lenses at theta[n,2]."""
        th = _f64(theta).reshape(-1, 2)
        out = np.empty_like(th)
        _load().lmo_deflect_direct(*self._lens()[:3], self.n, _dp(th), th.shape[0], _dp(out))
        return out

    def coeffs(self, ci, cj):
        """Complex Taylor coefficients a_0..a_{P-1} of level-2 cell (ci, cj)."""
        a = np.empty(2 * self.geom.terms)
        rc = _load().lmo_coeffs(ctypes.byref(self._p), *self._lens(), int(ci), int(cj), _dp(a))
        if rc:
            raise RuntimeError("lmo_coeffs failed (%d)" % rc)
        return a[0::2] + 1j * a[1::2]

    def near_mask(self, ci, cj):
        m = np.zeros(self.n, dtype=np.uint8)
        rc = _load().lmo_near_mask(ctypes.byref(self._p), _dp(self.lx), _dp(self.ly), self.n,
                                   int(ci), int(cj), m.ctypes.data_as(_P(ctypes.c_uint8)))
        if rc:
            raise RuntimeError("lmo_near_mask failed (%d)" % rc)
        return m.astype(bool)

    def trace(self, ii, jj):
        """Source positions beta[n,2] and pixel index (q*nx+p, -1 outside) of rays (i,j)."""
        ii = np.ascontiguousarray(ii, dtype=np.int64)
        jj = np.ascontiguousarray(jj, dtype=np.int64)
        beta = np.empty((ii.shape[0], 2))
        pix = np.empty(ii.shape[0], dtype=np.int64)
        rc = _load().lmo_trace(ctypes.byref(self._p), *self._lens(), ii.ctypes.data_as(_i64),
                               jj.ctypes.data_as(_i64), ii.shape[0], _dp(beta),
                               pix.ctypes.data_as(_i64))
        if rc:
            raise RuntimeError("lmo_trace failed (%d)" % rc)
        return beta, pix

    def shoot(self, i0=0, j0=0, ni=None, nj=None, counts=None, nthreads=0):
        """Shoot a lattice sub-rectangle; returns (counts[ny,nx] uint64, n_out)."""
        g = self.geom
        ni = g.ray_nx - i0 if ni is None else ni
        nj = g.ray_ny - j0 if nj is None else nj
        if counts is None:
            counts = np.zeros((g.src_ny, g.src_nx), dtype=np.uint64)
        nout = ctypes.c_uint64(0)
        rc = _load().lmo_shoot(ctypes.byref(self._p), *self._lens(), int(i0), int(j0), int(ni),
                               int(nj), counts.ctypes.data_as(_u64), ctypes.byref(nout),
                               int(nthreads))
        if rc:
            raise RuntimeError("lmo_shoot failed (%d)" % rc)
        return counts, int(nout.value)

    def shoot_window(self, i0, j0, ni, nj, p0, q0, np_, nq, nthreads=0):
        """Counts of the pixel window [p0, p0+np_) x [q0, q0+nq) (uint64 [nq, np_])
        from the lattice sub-rectangle; returns (counts, rays outside the window)."""
        counts = np.zeros((nq, np_), dtype=np.uint64)
        nout = ctypes.c_uint64(0)
        rc = _load().lmo_shoot_window(ctypes.byref(self._p), *self._lens(), int(i0), int(j0),
                                      int(ni), int(nj), int(p0), int(q0), int(np_), int(nq),
                                      counts.ctypes.data_as(_u64), ctypes.byref(nout),
                                      int(nthreads))
        if rc:
            raise RuntimeError("lmo_shoot_window failed (%d)" % rc)
        return counts, int(nout.value)

    def mu_factor(self):
        """S_I / S_S of Eq. 12: magnification per ray count."""
        return float(_load().lmo_mu_factor(ctypes.byref(self._p)))


def num_threads() -> int:
    return int(_load().lmo_num_threads())
