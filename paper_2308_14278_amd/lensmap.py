"""ctypes binding of liblensmap (include/lensmap.h): the same entry points,
argument marshalling only.  Every step of the hot path runs in the library's
HIP kernels; there is no Python or CPU fallback, and importing this module
fails if the built library is missing.

PyTorch is used for streams only: a ``stream`` argument may be a
``torch.cuda.Stream``, a raw ``hipStream_t`` integer, or None (the current
torch stream if torch has a GPU, else the default stream).
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblensmap.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "lensmap.h")

LM_OK = 0
LM_EINVAL = -1
LM_ENOMEM = -2
LM_EDEVICE = -3
LM_ESTATE = -4
LM_ERANGE = -5
LM_EUNSUPPORTED = -6
LM_SCHEME_DIRECT = 0
LM_SCHEME_INTERP = 1
LM_PREC_MIXED = 0
LM_PREC_FP32 = 1
LM_PREC_MIXED_FP64 = 2
LM_PREC_AUTO = 3
LM_PREC_MIXED_CENTRED = 4
LM_MAX_TERMS = 7

_STATUS_NAMES = {0: "LM_OK", -1: "LM_EINVAL", -2: "LM_ENOMEM", -3: "LM_EDEVICE", -4: "LM_ESTATE",
                 -5: "LM_ERANGE", -6: "LM_EUNSUPPORTED"}


class LensmapError(RuntimeError):
    def __init__(self, status, func, msg):
        self.status = status
        super().__init__("%s -> %s: %s" % (func, _STATUS_NAMES.get(status, status), msg))


class lm_geometry(ctypes.Structure):
    _fields_ = [
        ("src_x0", ctypes.c_double), ("src_y0", ctypes.c_double),
        ("src_dx", ctypes.c_double), ("src_dy", ctypes.c_double),
        ("src_nx", ctypes.c_int32), ("src_ny", ctypes.c_int32),
        ("ray_x0", ctypes.c_double), ("ray_y0", ctypes.c_double),
        ("ray_dx", ctypes.c_double), ("ray_dy", ctypes.c_double),
        ("ray_nx", ctypes.c_int64), ("ray_ny", ctypes.c_int64),
        ("scheme", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("coarse", ctypes.c_int32), ("l1_kx", ctypes.c_int32), ("l1_ky", ctypes.c_int32),
        ("near_halo", ctypes.c_int32), ("taylor_terms", ctypes.c_int32),
        ("far_order", ctypes.c_int32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}

    @property
    def n_rays(self):
        return int(self.ray_nx) * int(self.ray_ny)


class lm_fold_scales_t(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("kappa_c", "sin_a", "s_w", "c_star", "s_f", "n_cf", "mu_peak0")]


class lm_tune_result(ctypes.Structure):
    _fields_ = [("rays_per_lane", ctypes.c_int32), ("tile_scale", ctypes.c_int32),
                ("wg_per_cu", ctypes.c_int32), ("lds_layout", ctypes.c_int32),
                ("rays", ctypes.c_int64), ("seconds", ctypes.c_double)]


class lm_stats(ctypes.Structure):
    _fields_ = [("rays", ctypes.c_int64), ("near_pairs", ctypes.c_double),
                ("cells", ctypes.c_int64), ("far_pairs", ctypes.c_double)]


_P = ctypes.POINTER
_vp = ctypes.c_void_p
_d = _P(ctypes.c_double)
_i64 = _P(ctypes.c_int64)
_i32 = _P(ctypes.c_int32)
_u64 = _P(ctypes.c_uint64)

_SIGS = {
    "lm_geometry_derive": [_P(lm_geometry), ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                           ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                           ctypes.c_double, ctypes.c_double, ctypes.c_int64, ctypes.c_int64,
                           ctypes.c_int32, ctypes.c_int32, ctypes.c_double],
    "lm_geometry_derive_fold": [_P(lm_geometry), ctypes.c_double, ctypes.c_double,
                                ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                ctypes.c_int32, ctypes.c_double],
    "lm_set_fold": [_vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double],
    "lm_set_sheet": [_vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double],
    "lm_read_counts_region": [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                              _u64],
    "lm_create": [_P(lm_geometry), _P(_vp)],
    "lm_set_macro": [_vp, ctypes.c_double, ctypes.c_double, ctypes.c_double],
    "lm_set_lenses": [_vp, _d, _d, _d, ctypes.c_int64],
    "lm_bind_counts": [_vp, _vp],
    "lm_prepare": [_vp, _vp],
    "lm_shoot": [_vp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _vp],
    "lm_sync": [_vp],
    "lm_read_counts": [_vp, _u64, _u64, _u64],
    "lm_mu_factor": [_vp, _d],
    "lm_read_mu": [_vp, _d],
    "lm_reset_counts": [_vp, _vp],
    "lm_deflect": [_vp, _d, ctypes.c_int64, _d],
    "lm_trace": [_vp, _i64, _i64, ctypes.c_int64, _i32, _i32],
    "lm_trace_beta": [_vp, _i64, _i64, ctypes.c_int64, _d],
    "lm_precision_info": [_vp, _i32, _d],
    "lm_batch_tune_results": [_vp, _P(lm_tune_result), ctypes.c_int32, _i32],
    "lm_tune_sample": [_P(lm_geometry), ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                       ctypes.c_int64, ctypes.c_double, ctypes.c_int32, _i64, _i64],
    "lm_batch_create": [_P(_vp), ctypes.c_int32, _P(_vp)],
    "lm_batch_set_rect": [_vp, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                          ctypes.c_int64],
    "lm_batch_tune": [_vp, ctypes.c_char_p],
    "lm_batch_shoot": [_vp, _vp],
    "lm_batch_params": [_vp, _i32, _i32, _i32, _i32],
    "lm_batch_set_params": [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                            ctypes.c_int32],
    "lm_shot_stats": [_vp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                      _P(lm_stats)],
    "lm_batch_timing": [_vp, _P(ctypes.c_float), _P(ctypes.c_float)],
    "lm_measure_valu_peak": [_d, _d],
    "lm_read_coeffs": [_vp, ctypes.c_int64, ctypes.c_int64, _d],
    "lm_sum_counts": [_vp, _P(ctypes.c_uint64)],
    "lm_geometry_far_order": [_P(lm_geometry)],
    "lm_measure_issue_rates": [_d, ctypes.c_int32],
    "lm_find_peaks": [_vp, _i32, ctypes.c_int32, ctypes.c_int32, _P(ctypes.c_uint8)],
    "lm_fold_scales": [ctypes.c_double] * 7 + [_P(lm_fold_scales_t)],
    "lm_peak_stats": [_vp, _i32, ctypes.c_int32, ctypes.c_int32, _d, ctypes.c_int32, _u64, _u64,
                      _u64],
    "lm_peak_stats_noalloc": [_vp, _i32, ctypes.c_int32, ctypes.c_int32, _d, ctypes.c_int32,
                              _u64, _u64, _u64],
}

_lib = None


def load(path: str = LIB_PATH):
    """Load liblensmap.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError("liblensmap.so is not built (run __graft_entry__.build() or "
                              "python -m paper_2308_14278_amd.build_lib): " + path)
        lib = ctypes.CDLL(path)
        for name, args in _SIGS.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = ctypes.c_int32
        lib.lm_destroy.argtypes = [_vp]
        lib.lm_destroy.restype = None
        lib.lm_batch_destroy.argtypes = [_vp]
        lib.lm_batch_destroy.restype = None
        lib.lm_last_error.restype = ctypes.c_char_p
        lib.lm_version.restype = ctypes.c_char_p
        _lib = lib
    return _lib


def header_symbols(path: str = HEADER):
    """Function names declared in include/lensmap.h."""
    txt = open(path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lm_[a-z_]+)\s*\(", txt)))


def _check(status, func):
    if status != LM_OK:
        raise LensmapError(status, func, lm_last_error())


def _stream_ptr(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        except ImportError:
            pass
        return ctypes.c_void_p(0)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ------------------------------------------------------------ entry points


def lm_last_error() -> str:
    return load().lm_last_error().decode()


def lm_version() -> str:
    return load().lm_version().decode()


def lm_geometry_derive(src_lx, src_ly, src_nx, src_ny, kappa, gamma, kappa_star, protect=-1.0,
                       n_rays=0.0, ray_nx=0, ray_ny=0, scheme=LM_SCHEME_INTERP, coarse=0,
                       mean_mass=1.0) -> lm_geometry:
    g = lm_geometry()
    p = -1.0 if protect is None else float(protect)
    _check(load().lm_geometry_derive(ctypes.byref(g), src_lx, src_ly, src_nx, src_ny, kappa, gamma,
                                     kappa_star, p, float(n_rays or 0.0), int(ray_nx or 0),
                                     int(ray_ny or 0), scheme, coarse, mean_mass),
           "lm_geometry_derive")
    return g


def lm_geometry_derive_fold(src_lx, src_ly, src_nx, src_ny, kappa0, d_x, kappa_star,
                            margin=-1.0, n_rays=1.0, scheme=LM_SCHEME_INTERP, coarse=0,
                            mean_mass=1.0) -> lm_geometry:
    g = lm_geometry()
    _check(load().lm_geometry_derive_fold(ctypes.byref(g), src_lx, src_ly, src_nx, src_ny, kappa0,
                                          d_x, kappa_star, -1.0 if margin is None else margin,
                                          float(n_rays), scheme, coarse, mean_mass),
           "lm_geometry_derive_fold")
    return g


def lm_set_fold(m, kappa0, d_x, d_y, kappa_star):
    _check(load().lm_set_fold(m, kappa0, d_x, d_y, kappa_star), "lm_set_fold")


def lm_set_sheet(m, x0, x1, y0, y1):
    _check(load().lm_set_sheet(m, float(x0), float(x1), float(y0), float(y1)), "lm_set_sheet")


def lm_read_counts_region(m, p0, q0, np_, nq):
    out = np.empty((nq, np_), dtype=np.uint64)
    _check(load().lm_read_counts_region(m, int(p0), int(q0), int(np_), int(nq),
                                        out.ctypes.data_as(_u64)), "lm_read_counts_region")
    return out


def lm_create(g: lm_geometry):
    h = ctypes.c_void_p()
    _check(load().lm_create(ctypes.byref(g), ctypes.byref(h)), "lm_create")
    return h


def lm_destroy(m):
    if m:
        load().lm_destroy(m)


def lm_set_macro(m, kappa, gamma, kappa_star):
    _check(load().lm_set_macro(m, kappa, gamma, kappa_star), "lm_set_macro")


def lm_set_lenses(m, x, y, mass):
    x, y, mass = _f64(x), _f64(y), _f64(mass)
    n = x.shape[0]
    if y.shape[0] != n or mass.shape[0] != n:
        raise ValueError("lens arrays differ in length")
    _check(load().lm_set_lenses(m, x.ctypes.data_as(_d), y.ctypes.data_as(_d),
                                mass.ctypes.data_as(_d), n), "lm_set_lenses")


def lm_bind_counts(m, device_ptr):
    """Bind a caller-owned device buffer (int address, e.g. tensor.data_ptr()) or None."""
    _check(load().lm_bind_counts(m, ctypes.c_void_p(device_ptr or 0)), "lm_bind_counts")


def lm_prepare(m, stream=None):
    _check(load().lm_prepare(m, _stream_ptr(stream)), "lm_prepare")


def lm_shoot(m, i0, j0, ni, nj, stream=None):
    _check(load().lm_shoot(m, int(i0), int(j0), int(ni), int(nj), _stream_ptr(stream)), "lm_shoot")


def lm_sync(m):
    _check(load().lm_sync(m), "lm_sync")


def lm_read_counts(m, g: lm_geometry, with_counts=True):
    """Returns (counts[src_ny, src_nx] uint64 or None, n_out, n_shot)."""
    counts = np.empty((g.src_ny, g.src_nx), dtype=np.uint64) if with_counts else None
    nout = ctypes.c_uint64()
    nshot = ctypes.c_uint64()
    ptr = counts.ctypes.data_as(_u64) if with_counts else None
    _check(load().lm_read_counts(m, ptr, ctypes.byref(nout), ctypes.byref(nshot)),
           "lm_read_counts")
    return counts, int(nout.value), int(nshot.value)


def lm_mu_factor(m) -> float:
    f = ctypes.c_double()
    _check(load().lm_mu_factor(m, ctypes.byref(f)), "lm_mu_factor")
    return f.value


def lm_read_mu(m, g: lm_geometry):
    mu = np.empty((g.src_ny, g.src_nx), dtype=np.float64)
    _check(load().lm_read_mu(m, mu.ctypes.data_as(_d)), "lm_read_mu")
    return mu


def lm_reset_counts(m, stream=None):
    _check(load().lm_reset_counts(m, _stream_ptr(stream)), "lm_reset_counts")


def lm_deflect(m, theta):
    th = _f64(theta).reshape(-1, 2)
    out = np.empty_like(th)
    _check(load().lm_deflect(m, th.ctypes.data_as(_d), th.shape[0], out.ctypes.data_as(_d)),
           "lm_deflect")
    return out


def lm_trace(m, i, j):
    i = np.ascontiguousarray(i, dtype=np.int64)
    j = np.ascontiguousarray(j, dtype=np.int64)
    p = np.empty(i.shape[0], dtype=np.int32)
    q = np.empty(i.shape[0], dtype=np.int32)
    _check(load().lm_trace(m, i.ctypes.data_as(_i64), j.ctypes.data_as(_i64), i.shape[0],
                           p.ctypes.data_as(_i32), q.ctypes.data_as(_i32)), "lm_trace")
    return p, q


def lm_trace_beta(m, i, j):
    """Source positions beta[n, 2] (theta_E) of lattice rays, as the kernel bins them."""
    i = np.ascontiguousarray(i, dtype=np.int64)
    j = np.ascontiguousarray(j, dtype=np.int64)
    out = np.empty((i.shape[0], 2), dtype=np.float64)
    _check(load().lm_trace_beta(m, i.ctypes.data_as(_i64), j.ctypes.data_as(_i64), i.shape[0],
                                out.ctypes.data_as(_d)), "lm_trace_beta")
    return out


def lm_precision_info(m):
    """(precision the kernels run in, estimated bin mismatch of plain FP32 near sums,
    of centred FP32 near sums); estimates are -1 for a fixed precision."""
    p = ctypes.c_int32()
    e = (ctypes.c_double * 2)()
    _check(load().lm_precision_info(m, ctypes.byref(p), e), "lm_precision_info")
    return int(p.value), float(e[0]), float(e[1])


def lm_batch_tune_results(b):
    """Candidates timed by the last lm_batch_tune: list of dicts with rays/s."""
    n = ctypes.c_int32()
    _check(load().lm_batch_tune_results(b, None, 0, ctypes.byref(n)), "lm_batch_tune_results")
    arr = (lm_tune_result * max(1, n.value))()
    _check(load().lm_batch_tune_results(b, arr, n.value, ctypes.byref(n)),
           "lm_batch_tune_results")
    out = []
    for r in arr[:n.value]:
        d = {f: getattr(r, f) for f, _ in r._fields_}
        d["rays_per_s"] = r.rays / r.seconds if r.seconds > 0 else 0.0
        out.append(d)
    return out


def lm_tune_sample(g, i0, j0, ni, nj, fraction, tile_scale=1):
    """(rect (i0, j0, ni, nj), workgroup tiles) of the tuning sample of one map."""
    rect = (ctypes.c_int64 * 4)()
    tiles = ctypes.c_int64()
    _check(load().lm_tune_sample(ctypes.byref(g), int(i0), int(j0), int(ni), int(nj),
                                 float(fraction), int(tile_scale), rect, ctypes.byref(tiles)),
           "lm_tune_sample")
    return tuple(int(v) for v in rect), int(tiles.value)


def lm_batch_create(maps):
    arr = (ctypes.c_void_p * len(maps))(*[m.value if isinstance(m, ctypes.c_void_p) else m
                                          for m in maps])
    h = ctypes.c_void_p()
    _check(load().lm_batch_create(arr, len(maps), ctypes.byref(h)), "lm_batch_create")
    return h


def lm_batch_set_rect(b, index, i0, j0, ni, nj):
    _check(load().lm_batch_set_rect(b, index, int(i0), int(j0), int(ni), int(nj)),
           "lm_batch_set_rect")


def lm_batch_tune(b, cache_path=None):
    _check(load().lm_batch_tune(b, cache_path.encode() if cache_path else None), "lm_batch_tune")


def lm_batch_shoot(b, stream=None):
    _check(load().lm_batch_shoot(b, _stream_ptr(stream)), "lm_batch_shoot")


def lm_batch_params(b):
    """(rays per lane, tile scale, workgroups per CU, LDS layout)."""
    a, c, d, e = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(load().lm_batch_params(b, ctypes.byref(a), ctypes.byref(c), ctypes.byref(d),
                                  ctypes.byref(e)), "lm_batch_params")
    return int(a.value), int(c.value), int(d.value), int(e.value)


def lm_batch_set_params(b, rays_per_lane, tile_cells, wg_per_cu, lds_layout=0):
    _check(load().lm_batch_set_params(b, int(rays_per_lane), int(tile_cells), int(wg_per_cu),
                                      int(lds_layout)), "lm_batch_set_params")


def lm_fold_scales(theta_e_arcsec, d_x, d_y, kappa0, kappa_star, n_star, ds_over_r=0.0):
    out = lm_fold_scales_t()
    _check(load().lm_fold_scales(theta_e_arcsec, d_x, d_y, kappa0, kappa_star, n_star, ds_over_r,
                                 ctypes.byref(out)), "lm_fold_scales")
    return {n: getattr(out, n) for n, _ in out._fields_}


PEAK_CANDIDATE = 1
PEAK_TRUE = 2


def lm_find_peaks(m, g: lm_geometry, tracks, k=5):
    """Peak flags (bit 0 candidate, bit 1 true peak) of the listed map rows:
    uint8 array [len(tracks), src_nx]."""
    tr = np.ascontiguousarray(tracks, dtype=np.int32)
    flags = np.empty((tr.shape[0], g.src_nx), dtype=np.uint8)
    _check(load().lm_find_peaks(m, tr.ctypes.data_as(_i32), tr.shape[0], int(k),
                                flags.ctypes.data_as(_P(ctypes.c_uint8))), "lm_find_peaks")
    return flags


def _peak_stats(name, m, tracks, beta_edges, k):
    tr = np.ascontiguousarray(tracks, dtype=np.int32)
    ed = np.ascontiguousarray(beta_edges, dtype=np.float64)
    nb = ed.shape[0] - 1
    out = [np.zeros(max(nb, 0), dtype=np.uint64) for _ in range(3)]
    _check(getattr(load(), name)(m, tr.ctypes.data_as(_i32), tr.shape[0], int(k),
                                 ed.ctypes.data_as(_d), nb,
                                 *[o.ctypes.data_as(_u64) for o in out]), name)
    return tuple(out)


def lm_peak_stats(m, tracks, beta_edges, k=5):
    """(peaks, heights, pixels) per distance bin, uint64 arrays of len(edges) - 1."""
    return _peak_stats("lm_peak_stats", m, tracks, beta_edges, k)


def lm_peak_stats_noalloc(m, tracks, beta_edges, k=5):
    """lm_peak_stats on the library's per-device scratch memory (no allocation)."""
    return _peak_stats("lm_peak_stats_noalloc", m, tracks, beta_edges, k)


def lm_shot_stats(m, i0, j0, ni, nj) -> lm_stats:
    st = lm_stats()
    _check(load().lm_shot_stats(m, int(i0), int(j0), int(ni), int(nj), ctypes.byref(st)),
           "lm_shot_stats")
    return st


def lm_batch_timing(b):
    """(coefficient ms, shooting-kernel ms) of the last lm_batch_shoot."""
    a, c = ctypes.c_float(), ctypes.c_float()
    _check(load().lm_batch_timing(b, ctypes.byref(a), ctypes.byref(c)), "lm_batch_timing")
    return float(a.value), float(c.value)


def lm_sum_counts(m):
    """Sum of the map's counts, reduced on the device."""
    t = ctypes.c_uint64()
    _check(load().lm_sum_counts(m, ctypes.byref(t)), "lm_sum_counts")
    return int(t.value)


def lm_geometry_far_order(g):
    """Opt g into the hierarchical far field (smallest adequate series order);
    returns the order, or 0 (g unchanged apart from far_order = 0) when the
    geometry does not allow it."""
    rc = load().lm_geometry_far_order(ctypes.byref(g))
    if rc == LM_EUNSUPPORTED:
        return 0
    _check(rc, "lm_geometry_far_order")
    return int(g.far_order)


def lm_read_coeffs(m, ci, cj, terms):
    """Complex far-field coefficients a_0..a_{terms-1} of level-2 cell (ci, cj)."""
    import numpy as np
    a = np.zeros(2 * terms, dtype=np.float64)
    _check(load().lm_read_coeffs(m, int(ci), int(cj), a.ctypes.data_as(_d)), "lm_read_coeffs")
    return a[0::2] + 1j * a[1::2]


def lm_measure_issue_rates():
    """Measured issue rates on the current device: dict of lane instructions/s
    for VOP2 mul, VOP2 fmac, VOP3 fma (scalar operand), rcp, FP64 fma, and near
    pairs/s of the shooting kernel's shared-reciprocal pattern."""
    r = (ctypes.c_double * 6)()
    _check(load().lm_measure_issue_rates(r, 6), "lm_measure_issue_rates")
    return {"v_mul_f32": r[0], "v_fmac_f32": r[1], "v_fma_f32_sgpr": r[2], "v_rcp_f32": r[3],
            "pair2_pairs": r[4], "v_fma_f64": r[5]}


def lm_measure_valu_peak():
    """(unpacked FP32 FMA TFLOP/s, 1e9 ray-lens pairs/s) measured on the current device."""
    a, c = ctypes.c_double(), ctypes.c_double()
    _check(load().lm_measure_valu_peak(ctypes.byref(a), ctypes.byref(c)), "lm_measure_valu_peak")
    return float(a.value), float(c.value)


def lm_batch_destroy(b):
    if b:
        load().lm_batch_destroy(b)


# ------------------------------------------------------------ convenience


class Map:
    """Owning wrapper: geometry + macro + lenses, with the ABI's calls as methods."""

    def __init__(self, g: lm_geometry, kappa=0.0, gamma=0.0, kappa_star=0.0, lenses=None,
                 fold=None, sheet=None):
        """fold=(kappa0, d_x, d_y) selects the fold macro model (kappa, gamma
        ignored); sheet=(x0, x1, y0, y1) puts the -kappa_star sheet on that
        rectangle (None: an infinite sheet)."""
        self.g = g
        self.h = lm_create(g)
        if fold is None:
            lm_set_macro(self.h, kappa, gamma, kappa_star)
        else:
            lm_set_fold(self.h, fold[0], fold[1], fold[2], kappa_star)
        if sheet is not None:
            lm_set_sheet(self.h, *sheet)
        if lenses is not None:
            lm_set_lenses(self.h, *lenses)

    def shoot(self, i0=0, j0=0, ni=None, nj=None, stream=None):
        ni = self.g.ray_nx - i0 if ni is None else ni
        nj = self.g.ray_ny - j0 if nj is None else nj
        lm_shoot(self.h, i0, j0, ni, nj, stream)

    def counts(self):
        return lm_read_counts(self.h, self.g)

    def reset(self, stream=None):
        lm_reset_counts(self.h, stream)

    def trace(self, i, j):
        return lm_trace(self.h, i, j)

    def deflect(self, theta):
        return lm_deflect(self.h, theta)

    def trace_beta(self, i, j):
        return lm_trace_beta(self.h, i, j)

    def precision(self):
        return lm_precision_info(self.h)

    def mu_factor(self):
        return lm_mu_factor(self.h)

    def close(self):
        if self.h:
            lm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
