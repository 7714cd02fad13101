#!/usr/bin/env python3
"""Throughput of inverse ray-shooting on one MI355X, paper-scale workload.

One step = the whole hot path for one magnification map of the paper-scale
workload (13000 Salpeter microlenses, lambda_t = 0.005, lambda_r = 0.3,
kappa_star = 0.01, 1e13 rays, 5000 x 5000 uint64 map): counts reset, far-field
Taylor coefficients of every level-2 cell, the persistent shooting kernel
(one HIP-graph launch of the batched executor, autotuned), read-back of the
counts and the magnification map.  Inputs (lenses, partition) are resident on
the device before the timed region.

Printed: one JSON line with the whole-job rays/s, the shooting kernel's
roofline figures (algorithmic FP32 FLOPs from the exact near-lens pair count,
over its event-timed duration, against the 157.3 TFLOP/s FP32 vector peak),
the plain per-map FP32 comparison path, and the FP64 CPU oracle timed on a
bounded sample of the same workload with the map errors of both GPU paths.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "rays/s at 13k lenses; batched mixed vs plain per-map at stated map error vs FP64"
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_shoot_batch_paper_scale.json")


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def algorithmic_flops(stats, terms):
    """FP32 FLOPs the method needs per shot: 11 per near ray-lens pair (2 sub,
    r^2 3, rcp 1, m*w 1, 2 FMA 4), 8 per Taylor term after a_0, 8 for the
    map and pixel (rcp = 1, FMA = 2)."""
    return 11.0 * stats.near_pairs + (8.0 * (terms - 1) + 8.0) * stats.rays


def load_traffic(launch_rays):
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    # the counters hold for the machine code of the kernel they were taken on
    from paper_2308_14278_amd import codeobj
    sym = t.get("kernel_symbol")
    if not sym or t.get("kernel_code_sha") != codeobj.kernel_code_sha(sym):
        return None
    return t["bytes_per_ray"] * launch_rays


def make_map(lm, w, g, lenses, precision):
    g2 = type(g)()
    for k, _ in g._fields_:
        setattr(g2, k, getattr(g, k))
    g2.precision = precision
    return lm.Map(g2, w.kappa, w.gamma, w.kappa_star, lenses, sheet=w.sheet()), g2


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _timed_shoot(orc, rect, nthreads):
    t0 = time.perf_counter()
    out = orc.shoot(*rect, nthreads=nthreads)
    return time.perf_counter() - t0, out


def cpu_baseline_leg(lm, w, g, lenses, mp_mixed, mp_fp32, budget_s):
    """The FP64 oracle on a bounded sample of the workload (median of three
    runs on all host threads, and of three on one thread), and the errors of
    the batched GPU path and the plain-FP32 per-map path against it."""
    import numpy as np

    import oracle
    from oracle.geometry import OracleGeometry
    oracle.build()
    og = OracleGeometry(**{k: getattr(g, k) for k in
                           ("src_x0", "src_y0", "src_dx", "src_dy", "src_nx", "src_ny", "ray_x0",
                            "ray_y0", "ray_dx", "ray_dy", "ray_nx", "ray_ny", "scheme", "coarse",
                            "l1_kx", "l1_ky")}, halo=g.near_halo, terms=g.taylor_terms)
    orc = oracle.Oracle(og, w.kappa, w.gamma, w.kappa_star, *lenses, sheet=w.sheet())
    cores = oracle.num_threads()
    # calibrate on growing blocks until one takes a second, then size the
    # all-thread sample so that three runs fit the time budget
    nj = g.coarse
    i0, j0 = g.ray_nx // 2, g.ray_ny // 2 - nj // 2
    ni = g.coarse
    while True:
        dt0, _ = _timed_shoot(orc, (i0, j0, ni, nj), 0)
        if dt0 > 1.0 or ni >= g.ray_nx // 4:
            break
        ni *= 4
    rate0 = ni * nj / dt0
    ni = int(max(g.coarse, min(g.ray_nx // 2, rate0 * budget_s / 3 / nj)))
    ni -= ni % g.coarse
    runs = [_timed_shoot(orc, (i0, j0, ni, nj), 0) for _ in range(3)]
    ref, ref_out = runs[0][1]
    times = sorted(r[0] for r in runs)
    dt = times[1]
    rays = ni * nj
    log("oracle: %d rays in %.1f s (median of %s) on %d threads" %
        (rays, dt, ", ".join("%.1f" % t for t in times), cores))
    # one thread: a sample with about the same run time per thread count ratio
    ni1 = max(g.coarse, (ni // max(1, cores)) // g.coarse * g.coarse)
    runs1 = sorted(_timed_shoot(orc, (i0, j0, ni1, nj), 1)[0] for _ in range(3))
    rate1 = ni1 * nj / runs1[1]
    log("oracle: %d rays in %.1f s (median of 3) on 1 thread" % (ni1 * nj, runs1[1]))
    errors = {}
    rng = np.random.default_rng(2308)
    ii = rng.integers(0, g.ray_nx, 4000)
    jj = rng.integers(0, g.ray_ny, 4000)
    _, pix = orc.trace(ii, jj)
    for name, mp in (("batched_mixed", mp_mixed), ("plain_fp32", mp_fp32)):
        mp.reset()
        if name == "batched_mixed":
            # the timed path: the oracle's rectangle through the batch kernel
            bb = lm.lm_batch_create([mp.h])
            lm.lm_batch_set_rect(bb, 0, i0, j0, ni, nj)
            lm.lm_batch_shoot(bb)
            lm.lm_batch_destroy(bb)
        else:
            mp.shoot(i0, j0, ni, nj)
        c, o, _ = mp.counts()
        d = np.abs(c.astype(np.int64) - ref.astype(np.int64))
        big = ref >= 10000
        per_pix = float((d[big] / ref[big]).max()) if big.any() else 0.0
        p, q = mp.trace(ii, jj)
        gp = np.where(p >= 0, q.astype(np.int64) * g.src_nx + p, -1)
        errors[name] = {"bin_mismatch": 0.5 * float(d.sum()) / rays,
                        "max_pixel_rel_err_counts_ge_1e4": per_pix,
                        "n_out_diff": int(o) - int(ref_out),
                        "sampled_full_lattice_rays": int(ii.shape[0]),
                        "sampled_pixel_flips": int((gp != pix).sum())}
        mp.reset()
    return {"value": rays / dt, "unit": "rays/s", "cores": cores, "kind": "oracle",
            "sample": "FP64 oracle, interpolated scheme, %d x %d-ray sub-rectangle (%.3g rays) "
                      "of the paper-scale lattice at i0=%d, j0=%d; median of 3 runs" %
                      (ni, nj, rays, i0, j0),
            "seconds": dt, "run_seconds": times, "cpu_model": cpu_model(),
            "one_core": {"value": rate1, "unit": "rays/s", "cores": 1,
                         "sample": "%d x %d rays, same origin; median of 3 runs" % (ni1, nj),
                         "run_seconds": runs1}}, errors


def precision_stress_leg(lm, inputs):
    """Precision stress (lambda_t = 0.001, 20000 lenses, 4e12-ray lattice,
    4000^2 map): the mixed path (FP64 along the critical direction) and the
    plain FP32 path against the FP64 oracle on a 1e9-ray sub-region at the
    centre of the lattice."""
    import numpy as np

    import oracle
    from oracle.geometry import OracleGeometry
    w = inputs.precision_stress()
    lenses = w.lenses()
    out = {}
    ref = None
    for name, prec in (("mixed", lm.LM_PREC_MIXED), ("plain_fp32", lm.LM_PREC_FP32)):
        g = lm.lm_geometry_derive(w.src_side, w.src_side, w.src_pixels, w.src_pixels, w.kappa,
                                  w.gamma, w.kappa_star, protect=w.protect, n_rays=w.n_rays,
                                  scheme=w.scheme, coarse=w.coarse, mean_mass=w.mean_mass)
        g.precision = prec
        nj = 8 * g.coarse
        ni = int(1e9 // nj)
        i0, j0 = g.ray_nx // 2 - ni // 2, g.ray_ny // 2 - nj // 2
        mp = lm.Map(g, w.kappa, w.gamma, w.kappa_star, lenses, sheet=w.sheet())
        mp.shoot(i0, j0, ni, nj)
        c, o, _ = mp.counts()
        mp.close()
        if ref is None:
            og = OracleGeometry(**{k: getattr(g, k) for k in
                                   ("src_x0", "src_y0", "src_dx", "src_dy", "src_nx", "src_ny",
                                    "ray_x0", "ray_y0", "ray_dx", "ray_dy", "ray_nx", "ray_ny",
                                    "scheme", "coarse", "l1_kx", "l1_ky")},
                                halo=g.near_halo, terms=g.taylor_terms)
            t0 = time.perf_counter()
            ref, ref_out = oracle.Oracle(og, w.kappa, w.gamma, w.kappa_star, *lenses,
                                         sheet=w.sheet()).shoot(
                i0, j0, ni, nj)
            log("precision stress: oracle %d rays in %.1f s" % (ni * nj, time.perf_counter() - t0))
        d = np.abs(c.astype(np.int64) - ref.astype(np.int64))
        big = ref >= 10000
        out[name] = {"bin_mismatch": 0.5 * float(d.sum()) / (ni * nj),
                     "max_pixel_rel_err_counts_ge_1e4":
                         float((d[big] / ref[big]).max()) if big.any() else 0.0,
                     "n_out_diff": int(o) - int(ref_out)}
        log("precision stress %s: mismatch %.3g" % (name, out[name]["bin_mismatch"]))
    out["sample"] = "%d x %d rays at the centre of the 4e12-ray lattice" % (ni, nj)
    return out


def table1_window_leg(lm, inputs, precisions):
    """The paper's Table 1 map against the FP64 oracle on an 8e8-ray window of
    its lattice near the critical line (400000 x 2000 rays): the bin mismatch
    of every near-sum precision the Table 1 leg shot, the library's default
    (LM_PREC_AUTO) included."""
    import numpy as np

    import oracle
    from oracle.geometry import OracleGeometry
    w = inputs.paper_table1()
    k0, dx, _ = w.fold
    out = {}
    win = None
    for prec in precisions:
        g = lm.lm_geometry_derive_fold(w.src_side, w.extra["src_ly"], w.src_pixels,
                                       w.extra["src_ny"], k0, dx, w.kappa_star, n_rays=w.n_rays)
        g.precision = prec
        half = (g.ray_nx * g.ray_dx / 2, g.ray_ny * g.ray_dy / 2)
        lenses, rect = w.lenses(rect=half), w.sheet(rect=half)
        ni, nj = 400_000, 2000
        i0, j0 = g.ray_nx // 2 + 1000, g.ray_ny // 2
        if win is None:
            og = OracleGeometry(**{k: getattr(g, k) for k in
                                   ("src_x0", "src_y0", "src_dx", "src_dy", "src_nx", "src_ny",
                                    "ray_x0", "ray_y0", "ray_dx", "ray_dy", "ray_nx", "ray_ny",
                                    "scheme", "coarse", "l1_kx", "l1_ky")},
                                halo=g.near_halo, terms=g.taylor_terms, far_order=g.far_order)
            orc = oracle.Oracle(og, 0.0, 0.0, w.kappa_star, *lenses, fold=w.fold, sheet=rect)
            _, pix = orc.trace(np.array([i0, i0 + ni - 1, i0, i0 + ni - 1]),
                               np.array([j0, j0, j0 + nj - 1, j0 + nj - 1]))
            ps = [int(v % g.src_nx) for v in pix if v >= 0]
            qs = [int(v // g.src_nx) for v in pix if v >= 0]
            p0, q0 = max(0, min(ps) - 400), max(0, min(qs) - 400)
            np_ = min(g.src_nx - p0, max(ps) - p0 + 400)
            nq = min(g.src_ny - q0, max(qs) - q0 + 400)
            t0 = time.perf_counter()
            ref, _ = orc.shoot_window(i0, j0, ni, nj, p0, q0, np_, nq)
            log("Table 1 window: oracle %d rays in %.1f s" % (ni * nj, time.perf_counter() - t0))
            win = (p0, q0, np_, nq)
        mp = lm.Map(g, kappa_star=w.kappa_star, lenses=lenses, fold=w.fold, sheet=rect)
        used, est, est_c = mp.precision()
        mp.shoot(i0, j0, ni, nj)
        total = lm.lm_sum_counts(mp.h)
        got = lm.lm_read_counts_region(mp.h, *win)
        mp.close()
        name = {lm.LM_PREC_MIXED_FP64: "fp64-near", lm.LM_PREC_MIXED: "mixed",
                lm.LM_PREC_MIXED_CENTRED: "centred", lm.LM_PREC_AUTO: "auto"}[prec]
        # the window holds at most the rays counted in the whole map
        if int(got.sum(dtype=np.uint64)) > total or int(got.max()) > total:
            out[name] = {"precision_used": used, "error": "window read-back exceeds the map's "
                         "%d counted rays" % total}
            log("Table 1 window %s: inconsistent read-back" % name)
            continue
        mis = 0.5 * float(np.abs(got.astype(np.int64) - ref.astype(np.int64)).sum()) / (ni * nj)
        out[name] = {"precision_used": used, "bin_mismatch": mis,
                     "fp32_mismatch_estimate": est, "centred_fp32_mismatch_estimate": est_c}
        log("Table 1 window %s (precision %d): mismatch %.3g" % (name, used, mis))
    out["sample"] = "%d x %d rays of the 2.69e13-ray lattice beside the critical line" % (ni, nj)
    return out


def batched_study(lm, inputs, torch, scale, hierarchical=False):
    """The 80-map study at a fraction of its rays: one batch (coefficients of
    every map, one persistent shooting kernel over all maps' tiles), then ten
    light curves per map through the peak finder.  hierarchical: maps whose
    level-1 cells allow it take their far-field coefficients from level-1
    series (lm_geometry_far_order), the others sum them directly."""
    import numpy as np
    ws = inputs.batched_study(80, scale)
    maps, geoms = [], []
    n_hier = 0
    for w in ws:
        g = lm.lm_geometry_derive(w.src_side, w.src_side, w.src_pixels, w.src_pixels, w.kappa,
                                  w.gamma, w.kappa_star, n_rays=w.n_rays, scheme=w.scheme,
                                  coarse=w.coarse, mean_mass=w.mean_mass)
        if hierarchical and lm.lm_geometry_far_order(g) > 0:
            n_hier += 1
        maps.append(lm.Map(g, w.kappa, w.gamma, w.kappa_star, w.lenses(), sheet=w.sheet()))
        geoms.append(g)
    rays = sum(g.n_rays for g in geoms)
    flops = sum(algorithmic_flops(lm.lm_shot_stats(m.h, 0, 0, g.ray_nx, g.ray_ny),
                                  g.taylor_terms) for m, g in zip(maps, geoms))
    b = lm.lm_batch_create([m.h for m in maps])
    lm.lm_batch_tune(b, None)
    stream = torch.cuda.current_stream()
    lm.lm_batch_shoot(b, stream)  # warm-up (graph build)
    torch.cuda.synchronize()
    for m in maps:
        m.reset(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lm.lm_batch_shoot(b, stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    c_ms, s_ms = lm.lm_batch_timing(b)
    precisions = {}
    for m in maps:
        used = m.precision()[0]
        precisions[str(used)] = precisions.get(str(used), 0) + 1
    t1 = time.perf_counter()
    n_cand = n_true = 0
    for m, g in zip(maps, geoms):
        tracks = np.linspace(g.src_ny // 10, g.src_ny - g.src_ny // 10, 10).astype(np.int32)
        f = lm.lm_find_peaks(m.h, g, tracks)
        n_cand += int((f & 1).sum())
        n_true += int((f >> 1).sum())
    dt_peaks = time.perf_counter() - t1
    for m in maps:
        counts, n_out, n_shot = m.counts()
        assert int(counts.sum()) + n_out == n_shot
    lm.lm_batch_destroy(b)
    for m in maps:
        m.close()
    shoot_tflops = flops / (s_ms * 1e-3) / 1e12
    log("batched study%s: 80 maps, %.4g rays in %.2f s (%.4g rays/s, coefficients %.0f ms, "
        "shoot %.0f ms = %.1f TFLOP/s algorithmic); 800 light curves: %d candidates, "
        "%d true peaks in %.2f s" %
        (" (hierarchical far field)" if hierarchical else "", rays, dt, rays / dt, c_ms, s_ms,
         shoot_tflops, n_cand, n_true, dt_peaks))
    return {"maps": 80, "rays": rays, "seconds": dt, "rays_per_s": rays / dt,
            "coefficients_ms": c_ms, "shoot_kernel_ms": s_ms,
            "shoot_algorithmic_tflops": shoot_tflops,
            "shoot_frac_of_fp32_peak": shoot_tflops / PEAK_FP32_TFLOPS,
            "rays_scale": scale, "maps_per_precision": precisions,
            "light_curves": 800, "candidate_peaks": n_cand,
            "true_peaks": n_true, "peak_finding_s": dt_peaks,
            "far_field": ("hierarchical for %d maps, direct for %d" % (n_hier, 80 - n_hier)
                          if hierarchical else "direct (Sec. 3.2.2) for all maps")}


def other_workloads_leg(lm, inputs, torch):
    """The other single-map workloads (plain-small: direct sum; near-fold: 1e11
    rays at R = 64; precision stress: 4e12 rays, lambda_t = 0.001), each shot
    whole through the batched path (tuned, graphs built by one shot, then one
    timed shot: the shooting launch event-timed, the whole batch from the host),
    with direct far-field coefficients and, where its series converges, the
    hierarchical far field."""
    out = {}
    for name, make in (("plain_small", inputs.plain_small), ("near_fold", inputs.near_fold),
                       ("precision_stress", inputs.precision_stress)):
        w = make()
        res = {}
        for hier in (False, True):
            g = lm.lm_geometry_derive(w.src_side, w.src_side, w.src_pixels, w.src_pixels, w.kappa,
                                      w.gamma, w.kappa_star, protect=w.protect,
                                      n_rays=w.n_rays or 0.0, ray_nx=w.ray_nx or 0,
                                      ray_ny=w.ray_ny or 0, scheme=w.scheme, coarse=w.coarse,
                                      mean_mass=w.mean_mass)
            if hier and (w.scheme != lm.LM_SCHEME_INTERP or lm.lm_geometry_far_order(g) <= 0):
                continue
            mp = lm.Map(g, w.kappa, w.gamma, w.kappa_star, w.lenses(), sheet=w.sheet())
            stats = lm.lm_shot_stats(mp.h, 0, 0, g.ray_nx, g.ray_ny)
            flops = algorithmic_flops(stats, g.taylor_terms)
            b = lm.lm_batch_create([mp.h])
            lm.lm_batch_tune(b, None)
            stream = torch.cuda.current_stream()
            lm.lm_batch_shoot(b, stream)
            torch.cuda.synchronize()
            mp.reset(stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lm.lm_batch_shoot(b, stream)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            c_ms, s_ms = lm.lm_batch_timing(b)
            counts, n_out, n_shot = mp.counts()
            assert n_shot == g.n_rays and int(counts.sum()) + n_out == n_shot
            used = mp.precision()[0]
            lm.lm_batch_destroy(b)
            mp.close()
            r = {"rays": g.n_rays, "near_pairs_per_ray": stats.near_pairs / stats.rays,
                 "precision_used": used, "shoot_kernel_ms": s_ms,
                 "shoot_rays_per_s": g.n_rays / (s_ms * 1e-3),
                 "shoot_algorithmic_tflops": flops / (s_ms * 1e-3) / 1e12,
                 "coefficients_ms": c_ms, "batch_seconds": dt}
            if hier:
                r["far_order"] = g.far_order
            res["hierarchical" if hier else "direct"] = r
            log("%s%s: %.3g rays, %.2f near pairs per ray, shoot %.1f ms (%.3g rays/s, %.1f TFLOP/s "
                "algorithmic), coefficients %.1f ms, whole batch %.1f ms" %
                (name, " (hierarchical, Q = %d)" % g.far_order if hier else "", g.n_rays,
                 stats.near_pairs / stats.rays, s_ms, g.n_rays / (s_ms * 1e-3),
                 flops / (s_ms * 1e-3) / 1e12, c_ms, dt * 1e3))
        out[name] = res
    return out


TABLE1_THETA_E_ARCSEC = 1e-6
TABLE1_D_ARCMIN = (3.62, -3.41)
TABLE1_N_STAR = 13745


def fold_study_leg(lm, inputs, torch, n_maps=80):
    """The statistics of Sec. 4.2 (Figs. 4 and 5) on n_maps independent fold
    maps with the physics of Table 1 (inputs.fold_study: 40 theta_E across the
    caustic and 40 along it, 0.011 theta_E pixels, 1000 rays per pixel): one
    batch shoots every map (far field from the hierarchical series, which
    converges for these elongated level-1 cells through their near-square
    boxes), then ten light curves per map cross the caustic
    (map rows) and the library finds their true peaks and bins them by
    distance to the caustic on the GPU.  Reported: the true-peak number density
    per unit length of light curve, in units of s_f and divided by N_cf of
    Eq. 14, against beta_x / s_f; and the mean peak magnification divided by
    the prefactor of Eq. 15 against beta_x / s_w.  The prefactor takes the
    source radius as half a pixel (D_s / R = 2 / (pixel theta_E), theta_E in
    radians)."""
    import math

    import numpy as np
    ws = inputs.fold_study(n_maps)
    maps, geoms = [], []
    t_setup = time.perf_counter()
    for w in ws:
        k0, dx, _ = w.fold
        g = lm.lm_geometry_derive_fold(w.src_side, w.extra["src_ly"], w.src_pixels,
                                       w.extra["src_ny"], k0, dx, w.kappa_star, n_rays=w.n_rays)
        lm.lm_geometry_far_order(g)  # hierarchical far field where it converges
        half = (g.ray_nx * g.ray_dx / 2, g.ray_ny * g.ray_dy / 2)
        maps.append(lm.Map(g, kappa_star=w.kappa_star, lenses=w.lenses(rect=half), fold=w.fold,
                           sheet=w.sheet(rect=half)))
        geoms.append(g)
    rays = sum(g.n_rays for g in geoms)
    b = lm.lm_batch_create([m.h for m in maps])
    lm.lm_batch_tune(b, None)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    t0 = time.perf_counter()
    lm.lm_batch_shoot(b, stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    c_ms, s_ms = lm.lm_batch_timing(b)
    g0 = geoms[0]
    th_rad = TABLE1_THETA_E_ARCSEC / 3600.0 * math.pi / 180.0
    dsr = 2.0 / (g0.src_dx * th_rad)
    sc = lm.lm_fold_scales(TABLE1_THETA_E_ARCSEC, *TABLE1_D_ARCMIN, 0.83, 0.001, TABLE1_N_STAR,
                           dsr)
    sf, sw = sc["s_f"], sc["s_w"]
    e_sf = np.arange(-8, 49) * sf
    e_sw = sw * np.logspace(-3.0, math.log10(1.2), 26)
    acc = {"sf": [np.zeros(len(e_sf) - 1, dtype=np.uint64) for _ in range(3)],
           "sw": [np.zeros(len(e_sw) - 1, dtype=np.uint64) for _ in range(3)]}
    t1 = time.perf_counter()
    for m, g in zip(maps, geoms):
        tracks = np.linspace(g.src_ny // 10, g.src_ny - g.src_ny // 10, 10).astype(np.int32)
        for key, edges in (("sf", e_sf), ("sw", e_sw)):
            for a, v in zip(acc[key], lm.lm_peak_stats(m.h, tracks, edges)):
                a += v
    dt_stats = time.perf_counter() - t1
    factor = maps[0].mu_factor()
    lm.lm_batch_destroy(b)
    for m in maps:
        m.close()
    pk, _, px = acc["sf"]
    length = px.astype(np.float64) * g0.src_dx  # theta_E of light curve per bin
    density = np.where(length > 0, pk / np.maximum(length, 1e-300), 0.0) * sf / sc["n_cf"]
    pk2, ht2, _ = acc["sw"]
    mu_red = np.where(pk2 > 0, ht2.astype(np.float64) / np.maximum(pk2, 1) * factor, 0.0) / \
        sc["mu_peak0"]
    log("fold study: %d maps, %.4g rays in %.2f s (%.4g rays/s, shoot %.0f ms, coefficients "
        "%.0f ms); %d light curves, %d true peaks, statistics in %.2f s" %
        (len(maps), rays, dt, rays / dt, s_ms, c_ms, 10 * len(maps), int(pk.sum()), dt_stats))
    return {"maps": len(maps), "rays": rays, "seconds": dt, "rays_per_s": rays / dt,
            "shoot_kernel_ms": s_ms, "coefficients_ms": c_ms, "setup_s": t_setup,
            "light_curves": 10 * len(maps), "true_peaks": int(pk.sum()),
            "far_field_orders": sorted({int(g.far_order) for g in geoms}),
            "scales": {"s_f": sf, "s_w": sw, "n_cf": sc["n_cf"], "mu_peak0": sc["mu_peak0"],
                       "kappa_c": sc["kappa_c"], "ds_over_r": dsr},
            "density_vs_beta_over_s_f": {
                "bin_centres": [round(0.5 * (a + c) / sf, 3) for a, c in zip(e_sf, e_sf[1:])],
                "true_peaks": [int(v) for v in pk],
                "density_per_s_f_over_n_cf": [round(float(v), 5) for v in density]},
            "mean_peak_mu_vs_beta_over_s_w": {
                "bin_centres": [round(math.sqrt(a * c) / sw, 5) for a, c in zip(e_sw, e_sw[1:])],
                "true_peaks": [int(v) for v in pk2],
                "mu_peak_over_prefactor": [round(float(v), 5) for v in mu_red]}}


def paper_table1_leg(lm, inputs, torch, precision):
    """The paper's own map (Table 1, Sec. 4.1): fold model, 13745 unit lenses,
    2.69e13 rays into a 73877 x 363635 uint64 map (215 GB, resident in HBM).
    One step as in the headline (reset, coefficients, persistent shoot), then
    a device-side check that every ray was counted."""
    w = inputs.paper_table1()
    k0, dx, dy = w.fold
    g = lm.lm_geometry_derive_fold(w.src_side, w.extra["src_ly"], w.src_pixels, w.extra["src_ny"],
                                   k0, dx, w.kappa_star, n_rays=w.n_rays)
    g.precision = precision
    half = (g.ray_nx * g.ray_dx / 2, g.ray_ny * g.ray_dy / 2)
    mp = lm.Map(g, kappa_star=w.kappa_star, lenses=w.lenses(rect=half), fold=w.fold,
                sheet=w.sheet(rect=half))
    used, est, est_c = mp.precision()
    flops = algorithmic_flops(lm.lm_shot_stats(mp.h, 0, 0, g.ray_nx, g.ray_ny), g.taylor_terms)
    b = lm.lm_batch_create([mp.h])
    lm.lm_batch_tune(b, None)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lm.lm_reset_counts(mp.h, stream)
    lm.lm_batch_shoot(b, stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    c_ms, s_ms = lm.lm_batch_timing(b)
    total = lm.lm_sum_counts(mp.h)
    _, n_out, n_shot = lm.lm_read_counts(mp.h, g, with_counts=False)
    assert total + n_out == n_shot == g.n_rays, "ray count not conserved"
    params = list(lm.lm_batch_params(b))
    lm.lm_batch_destroy(b)
    mp.close()
    name = {lm.LM_PREC_MIXED_FP64: "fp64-near", lm.LM_PREC_MIXED: "mixed",
            lm.LM_PREC_MIXED_CENTRED: "centred", lm.LM_PREC_AUTO: "auto"}[precision]
    # near pairs in FP64 are priced against the FP64 vector peak
    peak = PEAK_FP64_TFLOPS if used == lm.LM_PREC_MIXED_FP64 else PEAK_FP32_TFLOPS
    tflops = flops / (s_ms * 1e-3) / 1e12
    log("paper Table 1 map (%s): %d x %d rays (%.4g), R=%d: %.1f s (shoot %.1f s = %.1f TFLOP/s "
        "algorithmic, %.2f of peak; coefficients %.0f ms), %.4g rays/s; %d rays in the map" %
        (name, g.ray_nx, g.ray_ny, g.n_rays, g.coarse, dt, s_ms / 1e3, tflops, tflops / peak,
         c_ms, g.n_rays / dt, total))
    return {"precision": name, "precision_used": used, "fp32_mismatch_estimate": est,
            "centred_fp32_mismatch_estimate": est_c,
            "exec_params": params,
            "rays": g.n_rays, "seconds": dt, "rays_per_s": g.n_rays / dt,
            "shoot_algorithmic_tflops": tflops, "shoot_frac_of_peak": tflops / peak,
            "near_pairs_per_ray": (flops / g.n_rays - 8.0 * g.taylor_terms) / 11.0,
            "shoot_kernel_ms": s_ms, "coefficients_ms": c_ms, "rays_in_map": total,
            "map_pixels": [g.src_nx, g.src_ny], "coarse": g.coarse,
            "paper_seconds_context": 7000.0}


def copy_calibration():
    """A plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters give the
    scale from counter units to bytes."""
    import torch
    n = 1 << 28  # float32 elements = 1 GiB
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="time budget of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--plain-rays", type=float, default=5e11,
                    help="rays of the per-map comparison runs")
    ap.add_argument("--rays", type=float, default=1e13,
                    help="rays per map (1e13 is the workload; smaller values are for profiling)")
    ap.add_argument("--study-scale", type=float, default=0.25,
                    help="fraction of the batched 80-map study's rays for its side measurement "
                         "(0 skips it)")
    ap.add_argument("--fold-maps", type=int, default=80,
                    help="fold maps of the peak-statistics side measurement (Sec. 4.2; 0 skips "
                         "it)")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default execution parameters (16 rays per lane, tile scale 1, "
                         "all workgroups that fit), which the tuner picks on MI355X")
    ap.add_argument("--no-comparison", action="store_true",
                    help="skip the per-map comparison runs (profiling)")
    ap.add_argument("--paper-map", choices=("none", "auto", "mixed", "centred", "fp64", "both",
                                            "all"),
                    default="none",
                    help="also shoot the paper's own Table 1 map (2.69e13 rays, 215 GB map) once "
                         "per chosen precision (auto: the library's choice; both: FP32 and FP64 "
                         "near sums; all: the library's choice and the three forms; side "
                         "measurement, about a minute each), and with the CPU baseline compare "
                         "an 8e8-ray window of it with the oracle")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the plain-small, near-fold and precision-stress workloads")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (reference for the HBM "
                         "byte counters) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2308_14278_amd.lensmap as lm
    from paper_2308_14278_amd import inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    lm.load()
    w = inputs.paper_scale()
    g = lm.lm_geometry_derive(w.src_side, w.src_side, w.src_pixels, w.src_pixels, w.kappa,
                              w.gamma, w.kappa_star, protect=w.protect, n_rays=args.rays,
                              scheme=w.scheme, coarse=w.coarse, mean_mass=w.mean_mass)
    lenses = w.lenses()
    log("geometry: %d x %d rays (%.4g), R=%d, K=%dx%d, %d lenses" %
        (g.ray_nx, g.ray_ny, g.n_rays, g.coarse, g.l1_kx, g.l1_ky, w.n_lenses))
    mp, _ = make_map(lm, w, g, lenses, g.precision)  # the library's default (LM_PREC_AUTO)
    prec_used, prec_est, prec_est_c = mp.precision()
    log("precision: %d (near-sum mismatch estimates: plain FP32 %.2e, centred FP32 %.2e)" %
        (prec_used, prec_est, prec_est_c))
    stats = lm.lm_shot_stats(mp.h, 0, 0, g.ray_nx, g.ray_ny)
    flops = algorithmic_flops(stats, g.taylor_terms)
    log("near pairs per ray %.3f, FLOP per ray %.1f" % (stats.near_pairs / stats.rays,
                                                         flops / stats.rays))
    b = lm.lm_batch_create([mp.h])
    stream = torch.cuda.current_stream()
    if not args.no_tune:
        t0 = time.perf_counter()
        lm.lm_batch_tune(b, os.environ.get("LENSMAP_TUNE_CACHE"))
        log("tuned %s in %.1f s" % (lm.lm_batch_params(b), time.perf_counter() - t0))
    tune_results = lm.lm_batch_tune_results(b)
    for r in tune_results:
        log("  candidate rays/lane %d, tile scale %d, WG/CU %d, LDS layout %d: %.4g rays/s on "
            "%.3g rays" % (r["rays_per_lane"], r["tile_scale"], r["wg_per_cu"], r["lds_layout"],
                           r["rays_per_s"], r["rays"]))

    def step():
        lm.lm_reset_counts(mp.h, stream)
        lm.lm_batch_shoot(b, stream)
        mu = lm.lm_read_mu(mp.h, g)
        return mu

    for k in range(args.warmup):
        t0 = time.perf_counter()
        step()
        log("warmup %d: %.2f s" % (k, time.perf_counter() - t0))
    torch.cuda.synchronize()
    shoot_ms, coeff_ms = [], []
    t0 = time.perf_counter()
    for k in range(args.steps):
        mu = step()
        c_ms, s_ms = lm.lm_batch_timing(b)
        coeff_ms.append(c_ms)
        shoot_ms.append(s_ms)
        log("step %d: shoot kernel %.1f ms, coefficients %.1f ms" % (k, s_ms, c_ms))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    counts, n_out, n_shot = lm.lm_read_counts(mp.h, g)
    assert int(counts.sum()) + n_out == g.n_rays, "ray count not conserved"
    assert abs(float(mu.mean()) - float(counts.mean()) * mp.mu_factor()) <= 1e-9 * float(mu.mean())
    value = g.n_rays * args.steps / elapsed
    avg_shoot_s = float(np.mean(shoot_ms)) / 1e3
    achieved = flops / avg_shoot_s / 1e12
    traffic = load_traffic(g.n_rays)
    issue = lm.lm_measure_issue_rates()
    pair_bound = issue["pair2_pairs"] / (stats.near_pairs / stats.rays)
    log("value %.4g rays/s; shoot kernel %.2f s -> %.1f TFLOP/s" % (value, avg_shoot_s, achieved))

    # plain per-map FP32 path and the mixed per-map path on the same band
    nj = min(g.ray_ny, 4 * g.coarse)
    ni = min(g.ray_nx, int(args.plain_rays / nj) // 64 * 64)
    i0 = (g.ray_nx - ni) // 2
    j0 = (g.ray_ny - nj) // 2
    mp32, _ = make_map(lm, w, g, lenses, lm.LM_PREC_FP32)
    per_map = {}
    for name, m in (() if args.no_comparison else
                    (("plain_fp32_per_map", mp32), ("mixed_per_map", mp))):
        m.reset(stream)
        m.shoot(i0, j0, ni, nj, stream)  # coefficients + warm-up
        torch.cuda.synchronize()
        m.reset(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        m.shoot(i0, j0, ni, nj, stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        per_map[name] = {"value": ni * nj / dt, "unit": "rays/s",
                         "sample": "%d x %d-ray band of the paper-scale lattice" % (ni, nj)}
        log("%s: %.4g rays/s" % (name, ni * nj / dt))

    study = None
    if args.study_scale > 0:
        study = batched_study(lm, inputs, torch, args.study_scale)
        study["hierarchical_far_field"] = batched_study(lm, inputs, torch, args.study_scale,
                                                        hierarchical=True)

    line = {
        "metric": METRIC, "value": value, "unit": "rays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "paper-scale: 13000 Salpeter lenses (0.08-1.5), lambda_t=0.005, "
                               "lambda_r=0.3, kappa_star=0.01, %.4g rays, 5000x5000 uint64 map "
                               "over 24x24 theta_E, interpolated scheme (P=4, R=%d, K=%dx%d), "
                               "compensating sheet on the lenses' rectangle, batched "
                               "mixed-precision path" %
                               (g.n_rays, g.coarse, g.l1_kx, g.l1_ky),
                   "rays": g.n_rays, "lenses": w.n_lenses, "map_pixels": [g.src_nx, g.src_ny],
                   "precision": "FP32 lens sums on rebased offsets in pixel units, FP64 cell "
                                "and row pixel bases, FP64 Taylor coefficients",
                   "precision_choice": {"requested": "LM_PREC_AUTO", "used": prec_used,
                                        "fp32_mismatch_estimate": prec_est,
                                        "centred_fp32_mismatch_estimate": prec_est_c},
                   "exec_params": list(lm.lm_batch_params(b)),
                   "tuner_candidates": [{"params": [r["rays_per_lane"], r["tile_scale"],
                                                    r["wg_per_cu"], r["lds_layout"]],
                                         "rays_per_s": r["rays_per_s"], "rays": r["rays"]}
                                        for r in tune_results]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": traffic, "kernel": "k_shoot_batch",
                     "flops_per_launch": flops, "avg_launch_s": avg_shoot_s,
                     "flop_per_ray": flops / stats.rays,
                     "near_pairs_per_ray": stats.near_pairs / stats.rays,
                     "issue_rates": issue,
                     "pair_issue_bound_rays_per_s": pair_bound,
                     "frac_of_pair_issue_bound": g.n_rays / avg_shoot_s / pair_bound},
        "coefficients_ms": float(np.mean(coeff_ms)),
        "comparison": per_map,
    }
    if study is not None:
        line["batched_study"] = study
    if args.fold_maps > 0:
        line["fold_peak_statistics"] = fold_study_leg(lm, inputs, torch, args.fold_maps)
    if not args.no_workloads:
        line["other_workloads"] = other_workloads_leg(lm, inputs, torch)
    precs = []
    if args.paper_map != "none":
        precs = {"auto": [lm.LM_PREC_AUTO], "mixed": [lm.LM_PREC_MIXED],
                 "centred": [lm.LM_PREC_MIXED_CENTRED], "fp64": [lm.LM_PREC_MIXED_FP64],
                 "both": [lm.LM_PREC_MIXED, lm.LM_PREC_MIXED_FP64],
                 "all": [lm.LM_PREC_AUTO, lm.LM_PREC_MIXED, lm.LM_PREC_MIXED_CENTRED,
                         lm.LM_PREC_MIXED_FP64]}[args.paper_map]
        line["paper_table1_map"] = [paper_table1_leg(lm, inputs, torch, pr) for pr in precs]
    if not args.no_cpu_baseline:
        cb, errors = cpu_baseline_leg(lm, w, g, lenses, mp, mp32, args.cpu_seconds)
        line["cpu_baseline"] = cb
        errors["precision_stress"] = precision_stress_leg(lm, inputs)
        if precs:
            errors["paper_table1_window"] = table1_window_leg(lm, inputs, precs)
        line["map_error_vs_fp64"] = errors
    lm.lm_batch_destroy(b)
    mp.close()
    mp32.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
