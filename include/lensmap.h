/*
 * lensmap.h -- C ABI of liblensmap: inverse ray-shooting of microlensing
 * magnification maps near a critical curve on AMD Instinct MI355X (gfx950).
 *
 * The problem (Sec. 2 and Sec. 3 of the paper): a regular lattice of
 * image-plane rays is mapped to the source plane by the lens equation with a
 * constant macro Jacobian diag(1-kappa-gamma, 1-kappa+gamma) (Eq. 1), point-mass
 * microlenses and a compensating negative mass sheet of density kappa_star
 * (Eq. 6):
 *     beta = (diag(1-kappa-gamma, 1-kappa+gamma) + kappa_star) theta - alpha(theta),
 *     alpha(theta) = sum_k m_k (theta - theta_k) / |theta - theta_k|^2 .
 * The sheet is infinite and uniform about the origin of the coordinates.  Each
 * ray is counted into the source-plane pixel it lands in; mu_pq = N_pq S_I/S_S
 * (Eq. 12).  The deflection is either the direct sum over all lenses or the
 * paper's interpolated scheme (Eq. 9, Sec. 3.2.1-3.2.3): lenses in the 3x3
 * block of level-1 cells around the ray's level-1 cell are summed directly,
 * all others enter through P complex Taylor coefficients of the ray's level-2
 * cell (P = 4: the eight real coefficients of Sec. 3.2.2).
 *
 * All lengths are in Einstein radii of a unit mass (Eq. 7).
 *
 * Conventions shared by every call:
 *  - every call returns an lm_status and never aborts or throws; on failure
 *    lm_last_error() describes the cause (thread-local, valid until the next
 *    call on the same thread);
 *  - input arrays are copied before the call returns; the caller keeps
 *    ownership of every buffer it passes;
 *  - a map lives on the HIP device that was current when it was created and
 *    uses it for every later call;
 *  - "stream" arguments are hipStream_t passed as void*; NULL is the default
 *    stream.  Calls that take a stream are asynchronous on it; calls that do
 *    not are synchronous;
 *  - calls on one map must not overlap from several threads.
 */
#ifndef LENSMAP_H
#define LENSMAP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lm_status;
#define LM_OK 0
#define LM_EINVAL (-1)        /* bad argument (NaN/Inf, non-positive size, ...) */
#define LM_ENOMEM (-2)        /* host or device allocation failed */
#define LM_EDEVICE (-3)       /* a HIP call failed */
#define LM_ESTATE (-4)        /* call not allowed in the current state */
#define LM_ERANGE (-5)        /* index range outside the lattice or map */
#define LM_EUNSUPPORTED (-6)  /* valid request the library does not handle */

#define LM_SCHEME_DIRECT 0    /* every lens summed for every ray */
#define LM_SCHEME_INTERP 1    /* near lenses direct, far lenses by Taylor coefficients */

#define LM_PREC_MIXED 0       /* rebased FP32 lens sums, FP64 bases and binning */
#define LM_PREC_FP32 1        /* plain FP32 in global coordinates (comparison path) */
#define LM_PREC_MIXED_FP64 2  /* as LM_PREC_MIXED with FP64 near-lens sums (interpolated
                                 scheme only; for pixels much finer than 1e-3 theta_E) */
#define LM_PREC_AUTO 3        /* LM_PREC_MIXED, LM_PREC_MIXED_CENTRED or LM_PREC_MIXED_FP64,
                                 chosen by the library for the map's current lenses and
                                 macro model: the first whose estimated bin mismatch is at
                                 most 5e-6 while near lists are short, else FP64 (see
                                 lm_precision_info); the direct scheme keeps
                                 LM_PREC_MIXED */
#define LM_PREC_MIXED_CENTRED 4 /* as LM_PREC_MIXED, but the FP32 near sums hold only each
                                 near lens's change of deflection from the level-2 cell
                                 centre, whose near deflection is summed in FP64 once per
                                 cell (interpolated scheme only): errors several times
                                 smaller for about a third more work per near pair; cells
                                 with a near lens within twice their half-diagonal of the
                                 centre sum plainly */

#define LM_MAX_TERMS 7        /* largest supported P */

/*
 * Geometry of one map (Sec. 3.2: the level-3 ray lattice, level-2 and level-1
 * cells; Sec. 3.2.3: the source-plane pixels).  Source pixel (p, q) covers
 *   [src_x0 + p src_dx, src_x0 + (p+1) src_dx) x [src_y0 + q src_dy, src_y0 + (q+1) src_dy);
 * ray (i, j), 0 <= i < ray_nx, 0 <= j < ray_ny, sits at the centre of
 * level-3 pixel (i, j): (ray_x0 + (i+1/2) ray_dx, ray_y0 + (j+1/2) ray_dy)
 * (Sec. 3.2.3).  A level-2 cell is a coarse x coarse block of rays (coarse a
 * multiple of 64); a level-1 cell is l1_kx x l1_ky level-2 cells; near lenses
 * lie within near_halo level-1 cells of the ray's level-1 cell (1: the 3x3
 * block).  A lens belongs to level-1 cell
 *   (floor((x - ray_x0) / (ray_dx * coarse * l1_kx)),
 *    floor((y - ray_y0) / (ray_dy * coarse * l1_ky))).
 * For the direct scheme `coarse` is the size of the blocks of rays that share
 * one FP64 origin for their FP32 arithmetic; l1_*, near_halo, taylor_terms are
 * ignored.
 */
typedef struct lm_geometry {
    double src_x0, src_y0, src_dx, src_dy;
    int32_t src_nx, src_ny;
    double ray_x0, ray_y0, ray_dx, ray_dy;
    int64_t ray_nx, ray_ny;
    int32_t scheme;        /* LM_SCHEME_* */
    int32_t precision;     /* LM_PREC_* */
    int32_t coarse;        /* R: rays per level-2 cell side, multiple of 64 */
    int32_t l1_kx, l1_ky;  /* level-2 cells per level-1 cell side */
    int32_t near_halo;     /* H */
    int32_t taylor_terms;  /* P, 1..LM_MAX_TERMS (interpolated scheme) */
    int32_t far_order;     /* 0: each level-2 cell's coefficients summed over its far
                              lenses (Sec. 3.2.2); Q in [P, 64]: from one Q-term series
                              of the same far lenses per level-1 cell, re-expanded about
                              each level-2 centre (hierarchical far field; not with
                              LM_PREC_FP32) */
} lm_geometry;

/*
 * Derive a geometry from the paper's rules (Sec. 3.1, Sec. 3.2, Eq. 8, 10, 11).
 * The paper states the problem by lambda_t = 1-kappa-gamma and lambda_r =
 * 1-kappa+gamma (Eq. 1); this call takes kappa and gamma, which fix both, and
 * the mean lens mass <m>, which turns the unit-mass N_star of Sec. 3.1 into a
 * mass function's.  Rules:
 *  - the source square s = [-src_lx/2, src_lx/2] x [-src_ly/2, src_ly/2] is
 *    split into src_nx x src_ny pixels;
 *  - the protection zone widens s by `protect` on every side (protect < 0:
 *    10 sqrt(kappa_star), Sec. 3.1);
 *  - the shooting region is the preimage of the widened region under
 *    diag(1-kappa-gamma, 1-kappa+gamma), centred on the origin;
 *  - if ray_nx > 0 and ray_ny > 0 they are used as given, otherwise
 *    L3 = sqrt(L_ix L_iy / n_rays) (Eq. 11), ray_nx = round(L_ix / L3),
 *    ray_ny = round(L_iy / L3); the spacings are then L_ix/ray_nx, L_iy/ray_ny;
 *  - level-1 sides min(L0, L_ix/10) and min(L0, L_iy/10) with
 *    L0 = sqrt(pi <m> / kappa_star) (Eq. 10, N_star of Sec. 3.1 with mean mass <m>);
 *  - coarse = R given (> 0), or 64 * max(1, round(min(L1x/L3x, L1y/L3y)/20/64))
 *    (level-2 = level-1/20, Sec. 3.2.2);
 *    l1_kx = max(1, round(L1x / (R L3x))), l1_ky likewise;
 *  - near_halo = 1, taylor_terms = 4, far_order = 0; precision = LM_PREC_AUTO
 *    for the interpolated scheme, LM_PREC_MIXED for the direct one.
 * Rounding is half away from zero.  Returns LM_EINVAL for non-finite or
 * non-positive inputs or a singular macro map.
 */
lm_status lm_geometry_derive(lm_geometry* g, double src_lx, double src_ly, int32_t src_nx,
                             int32_t src_ny, double kappa, double gamma, double kappa_star,
                             double protect, double n_rays, int64_t ray_nx, int64_t ray_ny,
                             int32_t scheme, int32_t coarse, double mean_mass);

/*
 * Geometry of a map next to a fold caustic (Sec. 2 Eq. 5, Sec. 3.1, Sec. 4.1):
 * the source window spans beta_x in [-margin, src_lx] across the caustic (the
 * margin lies on the side without macro images and is part of the map;
 * margin < 0: 20 sqrt(kappa_star)) and beta_y in [-src_ly/2, src_ly/2] along it,
 * in src_nx x src_ny pixels.  The shooting region is the rectangle
 * L_ix = 2 sqrt(2 (src_lx + margin) / d_x), L_iy = src_ly / (2 (1 - kappa0)),
 * centred on the origin (with Table 1 it holds N_star = 13745 lenses); rays and
 * grid levels follow lm_geometry_derive (n_rays rays, Eq. 10, 11, level-2 =
 * level-1 / 20 unless coarse > 0; precision as lm_geometry_derive).  d_x in
 * 1/theta_E, d_x > 0.
 */
lm_status lm_geometry_derive_fold(lm_geometry* g, double src_lx, double src_ly, int32_t src_nx,
                                  int32_t src_ny, double kappa0, double d_x, double kappa_star,
                                  double margin, double n_rays, int32_t scheme, int32_t coarse,
                                  double mean_mass);

/*
 * Opt a geometry into the hierarchical far field (an extension of the level-2
 * Taylor coefficients of Sec. 3.2.2): set g->far_order to the smallest Q in
 * [taylor_terms, 64] for which the series meets its truncation bound on this
 * geometry (rho^Q / (1 - rho) <= 1e-9, rho the largest ratio of a level-2
 * centre's and a far lens's distances from the series centre).  The series of
 * a level-1 cell is taken about the centre of the cell, or, when its sides
 * differ, about the centres of near-square boxes that cut it along its longer
 * side (round(long / short) boxes of ceil(K / boxes) level-2 cells), so that
 * elongated cells converge too.  LM_EUNSUPPORTED, far_order left at 0, when no
 * Q does, or for the direct scheme or LM_PREC_FP32.
 */
lm_status lm_geometry_far_order(lm_geometry* g);

typedef struct lm_map lm_map;
typedef struct lm_batch lm_batch;

/* Create a map with the given geometry on the current HIP device (Sec. 3.2: the
 * ray lattice and its cells; Sec. 3.2.3: one count per source pixel).  Counts
 * start at zero; the macro model is kappa = gamma = kappa_star = 0 and there
 * are no lenses until set.  The map owns its device buffers.  LM_EINVAL for an invalid geometry (non-positive
 * sizes, coarse not a positive multiple of 64, more than 2^31 rays per
 * workgroup tile, P outside 1..LM_MAX_TERMS, src_nx or src_ny above 2^30,
 * src_nx*src_ny >= 2^40). */
lm_status lm_create(const lm_geometry* g, lm_map** out);

/* Release every resource of the map (NULL is ignored).  Waits for the map's
 * outstanding work first.  (Resource management: no passage of the paper.) */
void lm_destroy(lm_map* m);

/* Macro convergence kappa, shear gamma and star convergence kappa_star of the
 * compensating sheet (Eq. 1, Eq. 6): the constant-Jacobian macro model.
 * LM_ESTATE if the map has counts. */
lm_status lm_set_macro(lm_map* m, double kappa, double gamma, double kappa_star);

/* The fold macro model of Eq. 5/6 instead:
 *   beta_x = (d_x theta_x / 2 + d_y theta_y) theta_x + kappa_star theta_x - alpha_x,
 *   beta_y = (2 (1 - kappa0) + kappa_star) theta_y - alpha_y,
 * with d = -(grad kappa)_0 - (grad gamma)_0 in 1/theta_E (Table 1 gives d in
 * arcmin^-1: multiply by theta_E in arcmin).  LM_ESTATE if the map has counts. */
lm_status lm_set_fold(lm_map* m, double kappa0, double d_x, double d_y, double kappa_star);

/* Where the compensating sheet of density -kappa_star lies (Sec. 2, Eq. 6).
 * Sec. 2 subtracts the microlenses' mean density so that the total density
 * stays the smooth model's; the sheet therefore belongs where the microlenses
 * are.  By default (and after a call with x0 = x1 = y0 = y1 = 0) it is infinite
 * about the origin, with the term kappa_star theta written in the macro
 * models above, which is exact inside a disk of lenses centred there.  For
 * lenses spread over a rectangle, pass it as [x0, x1] x [y0, y1] (theta_E):
 * the term becomes that rectangle's deflection, kappa_star theta plus a part
 * that is holomorphic inside the rectangle, which enters every level-2 cell's
 * Taylor coefficients with the far field (lm_read_coeffs includes it).  Its
 * series about a cell converges within the distance to the rectangle's
 * nearest corner, so cells next to a corner carry a truncation error of order
 * (kappa_star / pi) d rho^P, d that distance and rho the cell's half-diagonal
 * over d.  The rectangle must hold the ray lattice; interpolated scheme only
 * (LM_EUNSUPPORTED for the direct scheme).  LM_EINVAL for a non-finite or
 * empty rectangle or one that does not hold the lattice, LM_ESTATE if the map
 * has counts. */
lm_status lm_set_sheet(lm_map* m, double x0, double x1, double y0, double y1);

/* Copy n point-mass microlenses (Sec. 2, Eq. 6): positions (x[k], y[k]) in
 * theta_E and masses mass[k] > 0 in units of the unit mass of theta_E.  n may
 * be 0.  Sorts them by level-1 cell (Sec. 3.2.1) on the host and uploads them;
 * the arrays stay the caller's.  LM_EINVAL for NULL arrays with n > 0,
 * non-finite values or non-positive masses, LM_ESTATE if the map has counts. */
lm_status lm_set_lenses(lm_map* m, const double* x, const double* y, const double* mass,
                        int64_t n);

/* Use a caller-owned device buffer of src_nx*src_ny uint64 counts (row-major,
 * index q*src_nx + p; the count array of Sec. 3.2.3) instead of the map's own;
 * the buffer must outlive the map or the next lm_bind_counts.  Its contents are
 * taken as the current counts (the caller clears it).  NULL returns to the
 * map's own buffer.  Never fails for a non-NULL map (LM_EINVAL for NULL). */
lm_status lm_bind_counts(lm_map* m, uint64_t* device_counts);

/* Compute the level-2 Taylor coefficients of the far lenses (Sec. 3.2.2) for
 * every level-2 cell of the lattice.  lm_shoot does this on its own when the
 * coefficients are stale; this call forces a recomputation. No-op for the
 * direct scheme. Asynchronous on `stream`. */
lm_status lm_prepare(lm_map* m, void* stream);

/* Shoot the rays of the lattice sub-rectangle [i0, i0+ni) x [j0, j0+nj) and add
 * them to the counts (Sec. 3.2.3; deflection by Eq. 9, lens equation Eq. 6):
 * rays landing outside the map are added to n_out.  ni or nj = 0 is a no-op.
 * LM_ERANGE if the rectangle leaves the lattice.  Asynchronous on `stream`,
 * except that with LM_PREC_AUTO the first shot after new lenses or a new macro
 * model waits for the precision probe (a few milliseconds). */
lm_status lm_shoot(lm_map* m, int64_t i0, int64_t j0, int64_t ni, int64_t nj, void* stream);

/* Wait for all work issued on the map (Sec. 3.2.3: the counts are complete
 * before they are transferred). */
lm_status lm_sync(lm_map* m);

/* Copy the counts (src_nx*src_ny uint64, may be NULL), the number of rays that
 * left the map and the number of rays shot so far (either may be NULL) to the
 * host (Sec. 3.2.3: counts transferred to the CPU).  Synchronous. */
lm_status lm_read_counts(lm_map* m, uint64_t* host_counts, uint64_t* n_out, uint64_t* n_shot);

/* Sum of all counts, reduced on the device (Sec. 3.2.3; for maps too large to
 * copy back: with n_out it checks that every shot ray was counted).
 * Synchronous.  LM_EINVAL for NULL arguments. */
lm_status lm_sum_counts(lm_map* m, uint64_t* total);

/* Copy the counts of the pixel window [p0, p0+np) x [q0, q0+nq) to host
 * memory (nq rows of np uint64, caller-owned; Sec. 3.2.3, and Sec. 4.1 shows
 * such a window of the paper's map).  LM_ERANGE if the window leaves the map,
 * LM_ENOMEM if the device cannot hold a packed copy of the window (np * nq * 8
 * bytes, allocated and freed per call).  Synchronous. */
lm_status lm_read_counts_region(lm_map* m, int32_t p0, int32_t q0, int32_t np, int32_t nq,
                                uint64_t* host_counts);

/* Magnification of one ray count: (ray_dx ray_dy) / (src_dx src_dy) (Eq. 12). */
lm_status lm_mu_factor(const lm_map* m, double* factor);

/* Magnification map mu[q*src_nx + p] = counts * factor (Eq. 12), on the host.
 * Synchronous. */
lm_status lm_read_mu(lm_map* m, double* host_mu);

/* Zero the counts, n_out and the number of rays shot (Sec. 3.2.3: a fresh
 * count array).  Asynchronous on `stream`. */
lm_status lm_reset_counts(lm_map* m, void* stream);

/* Far-field coefficients a_0..a_{P-1} of level-2 cell (ci, cj) as the shooting
 * kernel reads them (Sec. 3.2.2; with a sheet rectangle, less the Taylor
 * coefficients of its holomorphic part): a[2n] = Re a_n, a[2n+1] = Im a_n, a_0 in FP64,
 * a_1.. stored in FP32 and widened.  Computes the coefficients first if the
 * lenses or the macro model changed.  Synchronous.  LM_ERANGE outside the
 * lattice's level-2 cells; LM_EUNSUPPORTED for the direct scheme. */
lm_status lm_read_coeffs(lm_map* m, int64_t ci, int64_t cj, double* a);

/* Deflection alpha(theta) of the map's scheme and precision (Eq. 9: near lenses
 * summed directly, far lenses through the Taylor coefficients) at n arbitrary
 * positions theta_xy[2t], theta_xy[2t+1] (FP64, host), written to alpha_xy
 * (host).  theta is rebased on the level-2 cell that contains it and the near
 * lenses are summed in the shooting kernel's order and precision (with
 * weights in theta_E where the kernel keeps its FP32 sums in pixels), but one
 * reciprocal per lens (the kernel shares one between two lattice columns) and
 * the Taylor series by Horner (the kernel re-expands it per ray row), so its
 * rounding differs slightly from the kernel's; lm_trace_beta gives the
 * kernel's own values for lattice rays.  Synchronous; a test probe. */
lm_status lm_deflect(lm_map* m, const double* theta_xy, int64_t n, double* alpha_xy);

/* Pixels of listed lattice rays (i[t], j[t]): p[t], q[t] as the shooting
 * kernel computes them (Sec. 3.2.3), -1 in both for rays that land outside the
 * map.  Synchronous; a test probe.  LM_ERANGE for a ray outside the lattice. */
lm_status lm_trace(lm_map* m, const int64_t* i, const int64_t* j, int64_t n, int32_t* p,
                   int32_t* q);

/* Source-plane positions beta (Eq. 6) of listed lattice rays (i[t], j[t]),
 * beta_xy[2t], beta_xy[2t+1] in theta_E (host, caller-owned), from the values
 * the shooting kernel takes the floor of when it bins the ray: the kernel's
 * arithmetic, ray for ray, including the shared reciprocals and the per-row
 * Taylor re-expansion.  With the macro map, beta gives the deflection the
 * kernel used.  Synchronous; a test probe.  LM_ERANGE for a ray outside the
 * lattice. */
lm_status lm_trace_beta(lm_map* m, const int64_t* i, const int64_t* j, int64_t n,
                        double* beta_xy);

/* The precision the map's kernels run in (LM_PREC_*; never LM_PREC_AUTO) and,
 * for an LM_PREC_AUTO geometry of the interpolated scheme, the estimated bin
 * mismatches that chose it, mismatch_estimates[0] for plain FP32 near sums and
 * [1] for centred ones (host, 2 doubles, may be NULL): the mean of |du| + |dv|,
 * the distance in pixels between a ray's image with those sums and with FP64
 * near sums -- the chance that rounding moves the image across a pixel edge --
 * over the rays of a fixed sample of 65536 lattice rays (every ray of smaller
 * lattices) whose images lie in the map.  The first form (plain, centred)
 * whose estimate is at most 5e-6 is chosen while the mean near list over the
 * lattice holds at most 32 lenses (FP32 rounding of a running sum grows with
 * its length, and with long lists varies strongly from region to region);
 * otherwise FP64.  The estimates are -1 when no choice was made (a fixed
 * precision) and 0 for a map without lenses.  The paper states no precision;
 * this is the library's reading of the accuracy the maps need.  Synchronous
 * (runs the probe if the lenses or the macro model changed). */
lm_status lm_precision_info(lm_map* m, int32_t* precision, double* mismatch_estimates);

/* Light-curve peak identification (Sec. 4.2) on the map's current counts.
 * A light curve is row i of the map (counts[i*src_nx + j], i along the
 * caustic direction of the map's y axis, j across it).  For each listed row
 * tracks[t] (0 <= tracks[t] < src_ny) and each j, flags[t*src_nx + j] gets
 * bit 0 if (i, j) is a candidate peak (N_ij greater than both neighbours in j
 * and N_ij - <N> > k sqrt(<N>), <N> the mean of the three counts; decided
 * exactly in integers) and bit 1 if it is a true peak (also a candidate among
 * (i-1, j-1..j+1) and among (i+1, j-1..j+1)).  End pixels of a row are never
 * candidates; the first and last rows keep no true peaks.  k = 5 in the
 * paper; 1 <= k <= 1000.  flags is host memory of n_tracks*src_nx bytes.
 * Synchronous. */
lm_status lm_find_peaks(lm_map* m, const int32_t* tracks, int32_t n_tracks, int32_t k,
                        uint8_t* flags);

/* Statistics of the true peaks of Sec. 4.2 (Figs. 4 and 5) by distance to the
 * caustic, on the map's current counts.  Light curves are the listed rows
 * tracks[t] as in lm_find_peaks (peak test with threshold k); distance bin b
 * covers beta_x in [beta_edges[b], beta_edges[b+1]) (n_bins + 1 increasing
 * edges in theta_E, host), and pixel column p belongs to the bin holding its
 * centre src_x0 + (p + 1/2) src_dx (evaluated in FP64 in that order).  For
 * each bin, written to host arrays of n_bins entries: peaks[b] the true peaks
 * of the listed rows in the bin, heights[b] the sum of their counts (times
 * lm_mu_factor: their summed magnification), pixels[b] the light-curve pixels
 * in the bin (n_tracks x its columns: the length the peaks were found on).
 * Exact integers.  LM_EINVAL for bad arguments (1 <= n_bins <= 65536,
 * 1 <= k <= 1000, edges finite and increasing), LM_ERANGE for a row outside
 * the map.  Synchronous. */
lm_status lm_peak_stats(lm_map* m, const int32_t* tracks, int32_t n_tracks, int32_t k,
                        const double* beta_edges, int32_t n_bins, uint64_t* peaks,
                        uint64_t* heights, uint64_t* pixels);

/* lm_peak_stats without any device allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and errors as
 * lm_peak_stats; its device staging (the rows, the bin of every pixel column,
 * the bin edges and the two histograms, 4.2 MB) lives in a scratch array that
 * the library holds on each device it runs on until the process ends, which
 * limits a call to at most 8192 rows, maps of at most 2^20 columns and at most
 * 4096 bins (LM_EINVAL beyond).  Every call on one device shares that array,
 * so calls that overlap on one device (from several threads) race; the
 * histograms are cleared at the start of each call.  Synchronous. */
lm_status lm_peak_stats_noalloc(lm_map* m, const int32_t* tracks, int32_t n_tracks, int32_t k,
                                const double* beta_edges, int32_t n_bins, uint64_t* peaks,
                                uint64_t* heights, uint64_t* pixels);

/* Analysis scales near a fold caustic (Sec. 4): kappa_c = (theta_E |d|)^(2/3),
 * |sin a| with tan a = d_x/d_y, the micro-caustic band width s_w (Eq. 13),
 * C_star and s_f = C_star theta_E kappa_star^(1/2), the micro-caustic count
 * N_cf (Eq. 14), and the prefactor of the peak magnification of Eq. 15,
 * mu_peak(|beta|) = mu_peak0 x (1 if |beta| < s_w else (s_w/|beta|)^(3/8)).
 * theta_E in arcsec, d in arcmin^-1 (Table 1 units), ds_over_r = D_s / R
 * (0 leaves mu_peak0 at 0); s_w and s_f in theta_E.  Host only. */
typedef struct lm_fold_scales_t {
    double kappa_c, sin_a, s_w, c_star, s_f, n_cf, mu_peak0;
} lm_fold_scales_t;
lm_status lm_fold_scales(double theta_e_arcsec, double d_x, double d_y, double kappa0,
                         double kappa_star, double n_star, double ds_over_r,
                         lm_fold_scales_t* out);

/* Work of one shot, for throughput accounting (Sec. 3.2: direct shooting costs
 * N_star x rays; the near/far split of Eq. 9): rays, ray-lens pairs of the
 * directly summed (near) lenses, and for the interpolated scheme the level-2
 * cells of the lattice and the (cell, far lens) pairs their Taylor
 * coefficients need (Sec. 3.2.2).  Host-only, from the lens partition.
 * LM_ERANGE for a rectangle outside the lattice. */
typedef struct lm_stats {
    int64_t rays;
    double near_pairs;
    int64_t cells;
    double far_pairs;
} lm_stats;
lm_status lm_shot_stats(const lm_map* m, int64_t i0, int64_t j0, int64_t ni, int64_t nj,
                        lm_stats* out);

/* Batched execution (the study of 80 maps, Sec. 4.2): the maps (same scheme
 * and taylor_terms, same device) are shot together by persistent kernels fed
 * from work queues -- one kernel per precision the maps run in -- preceded by
 * their coefficient kernels; both phases are captured as HIP graphs and
 * replayed.  Each map's shot rectangle is the one given by lm_batch_set_rect
 * (default: its whole lattice).  The batch keeps pointers to the maps, which
 * must outlive it.  A member map changed after the graphs were captured (new
 * lenses, macro model or bound counts) is picked up by the next
 * lm_batch_shoot, which captures the graphs again.  LM_EUNSUPPORTED for maps
 * that differ in scheme, terms or device. */
lm_status lm_batch_create(lm_map* const* maps, int32_t n, lm_batch** out);
/* Shot rectangle of map `index` of the batch: [i0, i0+ni) x [j0, j0+nj) of its
 * lattice (Sec. 3.2.3).  LM_ERANGE outside the lattice or for a bad index. */
lm_status lm_batch_set_rect(lm_batch* b, int32_t index, int64_t i0, int64_t j0, int64_t ni,
                            int64_t nj);

/* Pick execution parameters (rays per lane, workgroup tile size, workgroups
 * per CU, LDS layout) for the study of Sec. 4.2 by timing every candidate on one fixed
 * sample of the batch's rays (lm_tune_sample of each map with the fraction
 * that makes about 2e10 rays in all, or the whole batch if smaller): the
 * fastest in rays/s wins.  Results never depend on the choice.  Unless the
 * cache holds the choice, the maps must have no counts (LM_ESTATE); they are
 * zero again afterwards.  The choice is
 * cached at cache_path (NULL: no cache), a text file of lines "key
 * rays_per_lane tile_scale wg_per_cu lds_layout" keyed by device and batch
 * shape.
 * Synchronous. */
lm_status lm_batch_tune(lm_batch* b, const char* cache_path);

/* One candidate timed by lm_batch_tune: its parameters, the rays of the
 * tuning sample (the same for every candidate of a run) and the device time
 * of one shooting launch over them. */
typedef struct lm_tune_result {
    int32_t rays_per_lane, tile_scale, wg_per_cu, lds_layout;
    int64_t rays;
    double seconds;
} lm_tune_result;
/* Candidates of the last lm_batch_tune that timed (none after a cache hit):
 * *n gets their number, out[0 .. min(max, *n)) the records (host, caller-owned).
 * LM_EINVAL for NULL b or n, max < 0, or out NULL with max > 0. */
lm_status lm_batch_tune_results(const lm_batch* b, lm_tune_result* out, int32_t max, int32_t* n);

/* The tuning sample of one map (host only, no device needed): the
 * sub-rectangle of its shot rectangle [i0, i0+ni) x [j0, j0+nj) centred in it,
 * each side scaled by sqrt(fraction) and rounded up to whole level-2 cells (at
 * most the side), written to rect[0..4) as (i0, j0, ni, nj).  It depends on
 * the geometry, the rectangle and the fraction only, so every candidate of a
 * tuning run shoots the same rays; *tiles (may be NULL) gets the number of
 * workgroup tiles the sample spans with the given tile scale (1..8), which
 * does depend on the candidate.  LM_EINVAL for a bad geometry, fraction
 * outside (0, 1] or tile scale outside 1..8; LM_ERANGE for a rectangle outside
 * the lattice. */
lm_status lm_tune_sample(const lm_geometry* g, int64_t i0, int64_t j0, int64_t ni, int64_t nj,
                         double fraction, int32_t tile_scale, int64_t* rect, int64_t* tiles);

/* Shoot every map's rectangle once (Sec. 3.2.3 for each map of the study of
 * Sec. 4.2): two graph launches, coefficients then shooting.  Asynchronous on
 * `stream` (capturing the graphs again first when needed, which waits for the
 * precision probes of LM_PREC_AUTO maps).  LM_EUNSUPPORTED if a map's
 * rectangle needs 2^31 or more workgroup tiles (only the direct scheme on an
 * extreme lattice can). */
lm_status lm_batch_shoot(lm_batch* b, void* stream);

/* Device time of the last lm_batch_shoot, from events recorded on its stream
 * around its two graph launches: all coefficient kernels (with the queue
 * reset), and the shooting kernels alone (ms, either pointer may be NULL).
 * Waits for that launch to finish.  LM_ESTATE before the first shot.
 * (Measurement: no passage of the paper.) */
lm_status lm_batch_timing(lm_batch* b, float* coeff_ms, float* shoot_ms);

/* Execution parameters in use: rays per lane, tile scale (multiplier of the
 * default level-2 cells per workgroup tile side), workgroups per CU (0: as many
 * as fit), LDS layout of the maps that run with FP32 near sums (0..3: lenses
 * per block of the wave-shared LDS table / uint32 bins of the workgroup's LDS
 * window / near lenses staged per block = 16/7040/64, 8/8064/64, 32/5000/64,
 * 16/7552/32; each fits 40 KiB per workgroup).  Any pointer may be NULL.
 * (Execution shape: no passage.) */
lm_status lm_batch_params(const lm_batch* b, int32_t* rays_per_lane, int32_t* tile_cells,
                          int32_t* wg_per_cu, int32_t* lds_layout);
/* Set the execution parameters by hand instead of lm_batch_tune: rays per
 * lane 4, 8 or 16, tile scale 1..8, workgroups per CU 0..8 (0: as many as
 * fit), LDS layout 0..3.  Results never depend on them.  LM_EINVAL outside
 * those ranges; LM_EUNSUPPORTED for layouts 1..3 except with the interpolated
 * scheme, 4 Taylor terms and 8 or 16 rays per lane. */
lm_status lm_batch_set_params(lm_batch* b, int32_t rays_per_lane, int32_t tile_cells,
                              int32_t wg_per_cu, int32_t lds_layout);
void lm_batch_destroy(lm_batch* b);

/* Device micro-benchmarks on the current device (diagnostics for the
 * roofline; no passage of the paper): the issue rate of independent unpacked FP32 FMAs in TFLOP/s, and
 * the rate of the near-lens pair instruction mix in 1e9 ray-lens pairs/s.
 * Either pointer may be NULL.  Synchronous; takes well under a second. */
lm_status lm_measure_valu_peak(double* fma_tflops, double* pair_gpairs);
/* Issue rates of single instruction kinds on the current device, in lane
 * instructions per second: rates[0] v_mul_f32 (two-source VOP2), rates[1]
 * v_fmac_f32 (VOP2), rates[2] v_fma_f32 with a scalar operand (VOP3), rates[3]
 * v_rcp_f32; rates[4] the shooting kernel's near-pair pattern (two columns
 * sharing one reciprocal) in pairs per second; rates[5] v_fma_f64.  The first
 * min(n, 6) entries are written.  Synchronous, well under a second.  LM_EINVAL
 * for rates NULL or n < 0. */
lm_status lm_measure_issue_rates(double* rates, int32_t n);

/* Description of the last failure on this thread ("" if none); owned by the
 * library, valid until the next call on the thread. */
const char* lm_last_error(void);

/* Library version string (static storage). */
const char* lm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LENSMAP_H */
