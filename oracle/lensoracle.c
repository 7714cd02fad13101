/*
 * lensoracle.c -- plain, slow FP64 CPU oracle for inverse ray-shooting of a
 * microlensing magnification map with the near/far (Taylor) deflection scheme.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the CPU-baseline leg of the benchmark may load or call this library.  The
 * product path (liblensmap) never links or calls it, and the two share no
 * source, header, table or helper.
 *
 * What is computed (all lengths in Einstein radii, all arithmetic in FP64):
 *
 *  Lens equation with point-mass microlenses and a compensating negative mass
 *  sheet (Sec. 2, Eq. 6), with either macro model:
 *   linear (Eq. 1): beta = diag(1-kappa-gamma, 1-kappa+gamma) theta
 *                          + s(theta) - alpha(theta);
 *   fold (Eq. 5, 6): beta_x = (d_x theta_x / 2 + d_y theta_y) theta_x
 *                            + s_x(theta) - alpha_x,
 *                    beta_y = 2 (1 - kappa_0) theta_y + s_y(theta) - alpha_y,
 *  alpha(theta) = sum_k m_k (theta - theta_k) / |theta - theta_k|^2.
 *  The sheet of density -kappa_star subtracts the microlenses' mean density
 *  where they are (Sec. 2: the total density stays that of the smooth model),
 *  so it covers the region of the microlenses.  Its term (sheet = 1) is the
 *  deflection of a uniform density kappa_star on the rectangle
 *  [sx0, sx1] x [sy0, sy1] that holds them,
 *    s(theta) = (kappa_star / pi) int int (theta - t) / |theta - t|^2 d^2 t,
 *  in closed form (rect_sheet below); for a region that is large and round
 *  about theta this tends to kappa_star * theta, which is the term of an
 *  infinite sheet about the coordinate origin (sheet = 0, also exact inside a
 *  disk of lenses centred there).  In fold mode the kappa field holds kappa_0
 *  and d = (d_x, d_y) is in units of 1/theta_E.
 *
 *  Ray lattice (Sec. 3.2, level-3 grid, Eq. 11): ray (i,j) sits at the centre
 *  of level-3 pixel (i,j): theta = (X0 + (i+1/2) L3x, Y0 + (j+1/2) L3y).
 *
 *  Direct scheme (Sec. 3.2, the direct deflection sum): every lens enters the
 *  sum.  A term whose ray coincides exactly with its lens is skipped.
 *
 *  Interpolated scheme (Sec. 3.2, Eq. 9, levels 1-2):
 *   - level-2 cell (ci,cj) = (floor(i/R), floor(j/R)): a block of R x R rays
 *     with centre z_c = (X0 + (ci+1/2) R L3x, Y0 + (cj+1/2) R L3y);
 *   - level-1 cell (I,J) = (floor(ci/Kx), floor(cj/Ky)); a lens belongs to
 *     level-1 cell (floor((x-X0)/(Kx R L3x)), floor((y-Y0)/(Ky R L3y)));
 *   - near lenses of a ray: those whose level-1 cell lies within H cells of the
 *     ray's level-1 cell in both directions (the 3x3 block for H = 1);
 *   - far lenses enter through P complex Taylor coefficients of the level-2
 *     cell (P = 4 gives the eight real coefficients of Sec. 3.2.2):
 *       conj(alpha_far)(z) = sum_{n<P} a_n (z - z_c)^n,
 *       a_n = - sum_{k far} m_k / (z_k - z_c)^{n+1},
 *     which is the power series of sum_k m_k / (z - z_k) about z_c;
 *   - alpha = alpha_near (direct sum over near lenses) + alpha_far.
 *
 *  Binning and magnification (Sec. 3.2, Eq. 12): pixel (p,q) covers
 *  [Bx0 + p dx, Bx0 + (p+1) dx) x [By0 + q dy, By0 + (q+1) dy); a ray outside
 *  every pixel is counted in n_out; mu_pq = N_pq * (L3x L3y) / (dx dy).
 *
 *  Hierarchical far field (optional, far_order = Q > 0): the coefficients of
 *  a level-2 cell come from a Q-term series of the same far lenses about the
 *  centre of its level-1 cell, re-expanded about z_c (see far_coeffs_hier).
 *
 * Sums of many terms use Neumaier's compensated summation.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define LMO_PI 3.14159265358979323846

typedef struct {
    /* source map */
    double src_x0, src_y0, src_dx, src_dy;
    int64_t src_nx, src_ny;
    /* ray lattice */
    double ray_x0, ray_y0, ray_dx, ray_dy;
    int64_t ray_nx, ray_ny;
    /* macro model */
    double kappa, gamma, kappa_star;
    /* scheme: 0 direct, 1 interpolated */
    int64_t scheme, coarse, l1_kx, l1_ky, halo, terms;
    /* macro model: 0 linear (kappa, gamma), 1 fold (kappa = kappa_0, d_x, d_y) */
    int64_t macro;
    double d_x, d_y;
    /* far field: 0 direct per level-2 cell; Q > 0 through a Q-term expansion
     * per level-1 cell (hierarchical far field) */
    int64_t far_order;
    /* the -kappa_star sheet: 0 infinite about the origin, 1 the rectangle
     * [sx0, sx1] x [sy0, sy1] */
    int64_t sheet;
    double sx0, sx1, sy0, sy1;
} lmo_params;

typedef struct {
    const double *x, *y, *m;
    int64_t n;
} lmo_lenses;

/* ---- compensated summation (Neumaier) ---------------------------------- */
typedef struct { double s, c; } nsum;

static inline void nsum_add(nsum *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v))
        a->c += (a->s - t) + v;
    else
        a->c += (v - t) + a->s;
    a->s = t;
}
static inline double nsum_get(const nsum *a) { return a->s + a->c; }

/* ---- lens equation pieces ---------------------------------------------- */

/* Direct deflection of a lens subset: alpha = sum m_k (theta-theta_k)/|.|^2.
 * idx (may be NULL for all lenses) lists the lenses that enter, in lens order. */
static void direct_sum(const lmo_lenses *L, const int64_t *idx, int64_t nidx,
                       double tx, double ty, double *ax, double *ay)
{
    nsum sx = {0, 0}, sy = {0, 0};
    int64_t cnt = idx ? nidx : L->n;
    for (int64_t t = 0; t < cnt; ++t) {
        int64_t k = idx ? idx[t] : t;
        double dx = tx - L->x[k], dy = ty - L->y[k];
        double r2 = dx * dx + dy * dy;
        if (r2 == 0.0) continue; /* ray on the lens: term skipped */
        nsum_add(&sx, L->m[k] * dx / r2);
        nsum_add(&sy, L->m[k] * dy / r2);
    }
    *ax = nsum_get(&sx);
    *ay = nsum_get(&sy);
}

/* indices of the lenses flagged near, in lens order; returns their number */
static int64_t near_list(const unsigned char *near, int64_t n, int64_t *idx)
{
    int64_t c = 0;
    for (int64_t k = 0; k < n; ++k)
        if (near[k]) idx[c++] = k;
    return c;
}

static int64_t floor_div_i64(int64_t a, int64_t b)
{
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
    return q;
}

/* level-1 cell of a lens (Sec. 3.2.1) */
static void lens_l1(const lmo_params *p, double x, double y, int64_t *I, int64_t *J)
{
    double wx = p->ray_dx * (double)(p->coarse * p->l1_kx);
    double wy = p->ray_dy * (double)(p->coarse * p->l1_ky);
    double fi = floor((x - p->ray_x0) / wx);
    double fj = floor((y - p->ray_y0) / wy);
    /* clamp far-away lenses: they stay far from every ray cell */
    double lim = 4.0e15;
    if (fi > lim) fi = lim;
    if (fi < -lim) fi = -lim;
    if (fj > lim) fj = lim;
    if (fj < -lim) fj = -lim;
    *I = (int64_t)fi;
    *J = (int64_t)fj;
}

/* near mask of level-2 cell (ci,cj): 1 where the lens is near */
static void near_mask(const lmo_params *p, const lmo_lenses *L, int64_t ci, int64_t cj,
                      unsigned char *near)
{
    int64_t I = floor_div_i64(ci, p->l1_kx), J = floor_div_i64(cj, p->l1_ky);
    for (int64_t k = 0; k < L->n; ++k) {
        int64_t Ik, Jk;
        lens_l1(p, L->x[k], L->y[k], &Ik, &Jk);
        int64_t di = Ik - I, dj = Jk - J;
        near[k] = (di >= -p->halo && di <= p->halo && dj >= -p->halo && dj <= p->halo);
    }
}

static void cell_centre(const lmo_params *p, int64_t ci, int64_t cj, double *zx, double *zy)
{
    *zx = p->ray_x0 + ((double)ci + 0.5) * (double)p->coarse * p->ray_dx;
    *zy = p->ray_y0 + ((double)cj + 0.5) * (double)p->coarse * p->ray_dy;
}

/* Taylor coefficients a_n, n < P, of the far lenses about z_c (Sec. 3.2.2).
 * a[2n] = Re a_n, a[2n+1] = Im a_n. */
static void far_coeffs(const lmo_params *p, const lmo_lenses *L, const unsigned char *near,
                       double zx, double zy, double *a)
{
    int64_t P = p->terms;
    nsum *re = (nsum *)calloc((size_t)P, sizeof(nsum));
    nsum *im = (nsum *)calloc((size_t)P, sizeof(nsum));
    for (int64_t k = 0; k < L->n; ++k) {
        if (near[k]) continue;
        /* u = 1 / (z_k - z_c) */
        double wx = L->x[k] - zx, wy = L->y[k] - zy;
        double w2 = wx * wx + wy * wy;
        double ux = wx / w2, uy = -wy / w2;
        /* t = m u^{n+1}, accumulated as -t */
        double tx = L->m[k] * ux, ty = L->m[k] * uy;
        for (int64_t n = 0; n < P; ++n) {
            nsum_add(&re[n], -tx);
            nsum_add(&im[n], -ty);
            double nx = tx * ux - ty * uy;
            double ny = tx * uy + ty * ux;
            tx = nx;
            ty = ny;
        }
    }
    for (int64_t n = 0; n < P; ++n) {
        a[2 * n] = nsum_get(&re[n]);
        a[2 * n + 1] = nsum_get(&im[n]);
    }
    free(re);
    free(im);
}

/* Centre Z of the hierarchical expansion that serves level-2 cell (ci,cj).
 * Normally the centre of its level-1 cell (I,J).  A level-1 cell whose sides
 * L1x = Kx R L3x and L1y = Ky R L3y differ is cut along its longer side into
 * n = round(long / short) boxes of b = ceil(K / n) level-2 cells (the last one
 * may be narrower), and Z is the centre of the box holding the level-2 cell:
 * a single series about the centre of an elongated cell would not converge
 * at the cell's far ends, while a near-square box keeps the convergence ratio
 * of a square cell.  The far set stays that of the level-1 cell. */
static void far_centre(const lmo_params *p, int64_t ci, int64_t cj, double *Zx, double *Zy)
{
    int64_t Kx = p->l1_kx, Ky = p->l1_ky;
    int64_t I = floor_div_i64(ci, Kx), J = floor_div_i64(cj, Ky);
    double l1x = (double)(Kx * p->coarse) * p->ray_dx, l1y = (double)(Ky * p->coarse) * p->ray_dy;
    int64_t nx = 1, ny = 1;
    if (l1x > l1y) nx = (int64_t)floor(l1x / l1y + 0.5);
    if (l1y > l1x) ny = (int64_t)floor(l1y / l1x + 0.5);
    if (nx < 1) nx = 1;
    if (ny < 1) ny = 1;
    if (nx == 1) {
        *Zx = p->ray_x0 + ((double)I + 0.5) * (double)(Kx * p->coarse) * p->ray_dx;
    } else {
        int64_t b = (Kx + nx - 1) / nx;
        int64_t c0 = I * Kx + ((ci - I * Kx) / b) * b;
        int64_t c1 = c0 + b < (I + 1) * Kx ? c0 + b : (I + 1) * Kx;
        *Zx = p->ray_x0 + 0.5 * (double)(c0 + c1) * (double)p->coarse * p->ray_dx;
    }
    if (ny == 1) {
        *Zy = p->ray_y0 + ((double)J + 0.5) * (double)(Ky * p->coarse) * p->ray_dy;
    } else {
        int64_t b = (Ky + ny - 1) / ny;
        int64_t r0 = J * Ky + ((cj - J * Ky) / b) * b;
        int64_t r1 = r0 + b < (J + 1) * Ky ? r0 + b : (J + 1) * Ky;
        *Zy = p->ray_y0 + 0.5 * (double)(r0 + r1) * (double)p->coarse * p->ray_dy;
    }
}

/* Hierarchical far field: the far set of level-2 cell (ci,cj) is the far set
 * of its level-1 cell (I,J) (Sec. 3.2.1), so its Taylor series about the
 * level-2 centre z_c (Sec. 3.2.2) can be obtained from one series about a
 * centre Z of the level-1 cell (far_centre), truncated after Q terms:
 *   A_n = - sum_{k far} m_k / (z_k - Z)^{n+1},                n < Q,
 *   a_p = sum_{n=p}^{Q-1} C(n,p) A_n (z_c - Z)^{n-p},           p < P,
 * which is the re-expansion of sum_n A_n (z - Z)^n about z_c.  Far lenses lie
 * outside the (2H+1)^2 block of level-1 cells, so |z_c - Z| / |z_k - Z| stays
 * below about 0.47 for square level-1 cells and square boxes of elongated ones,
 * and the truncation error falls geometrically with Q. */
static void far_coeffs_hier(const lmo_params *p, const lmo_lenses *L, const unsigned char *near,
                            int64_t ci, int64_t cj, double *a)
{
    int64_t Q = p->far_order, P = p->terms;
    double Zx, Zy;
    far_centre(p, ci, cj, &Zx, &Zy);
    double zx, zy;
    cell_centre(p, ci, cj, &zx, &zy);
    /* level-1 expansion */
    nsum *re = (nsum *)calloc((size_t)Q, sizeof(nsum));
    nsum *im = (nsum *)calloc((size_t)Q, sizeof(nsum));
    for (int64_t k = 0; k < L->n; ++k) {
        if (near[k]) continue;
        double wx = L->x[k] - Zx, wy = L->y[k] - Zy;
        double w2 = wx * wx + wy * wy;
        double ux = wx / w2, uy = -wy / w2;
        double tx = L->m[k] * ux, ty = L->m[k] * uy;
        for (int64_t n = 0; n < Q; ++n) {
            nsum_add(&re[n], -tx);
            nsum_add(&im[n], -ty);
            double nx = tx * ux - ty * uy;
            double ny = tx * uy + ty * ux;
            tx = nx;
            ty = ny;
        }
    }
    /* re-expansion about z_c */
    double sx = zx - Zx, sy = zy - Zy;
    for (int64_t q = 0; q < P; ++q) {
        nsum ar = {0.0, 0.0}, ai = {0.0, 0.0};
        double px = 1.0, py = 0.0; /* (z_c - Z)^(n-q) */
        double binom = 1.0;        /* C(n, q) */
        for (int64_t n = q; n < Q; ++n) {
            double Ax = nsum_get(&re[n]), Ay = nsum_get(&im[n]);
            nsum_add(&ar, binom * (Ax * px - Ay * py));
            nsum_add(&ai, binom * (Ax * py + Ay * px));
            double nx = px * sx - py * sy;
            double ny = px * sy + py * sx;
            px = nx;
            py = ny;
            binom = binom * (double)(n + 1) / (double)(n + 1 - q);
        }
        a[2 * q] = nsum_get(&ar);
        a[2 * q + 1] = nsum_get(&ai);
    }
    free(re);
    free(im);
}

/* Coefficients of level-2 cell (ci,cj) by the configured far-field method. */
static void sheet_coeffs(const lmo_params *p, int64_t ci, int64_t cj, double *c);

static void cell_coeffs(const lmo_params *p, const lmo_lenses *L, const unsigned char *near,
                        int64_t ci, int64_t cj, double *a)
{
    if (p->far_order > 0) {
        far_coeffs_hier(p, L, near, ci, cj, a);
    } else {
        double zx, zy;
        cell_centre(p, ci, cj, &zx, &zy);
        far_coeffs(p, L, near, zx, zy, a);
    }
    if (p->sheet == 1) {
        /* the rectangle sheet's holomorphic part rides with the far field:
         * the far term is subtracted in the lens equation and the sheet's is
         * added */
        double c[32];
        sheet_coeffs(p, ci, cj, c);
        for (int64_t n = 0; n < 2 * p->terms; ++n) a[n] -= c[n];
    }
}

/* alpha_far = conj( sum_n a_n d^n ), d = z - z_c, evaluated by Horner */
static void far_eval(int64_t P, const double *a, double dx, double dy, double *ax, double *ay)
{
    double fx = a[2 * (P - 1)], fy = a[2 * (P - 1) + 1];
    for (int64_t n = P - 2; n >= 0; --n) {
        double gx = fx * dx - fy * dy + a[2 * n];
        double gy = fx * dy + fy * dx + a[2 * n + 1];
        fx = gx;
        fy = gy;
    }
    *ax = fx;
    *ay = -fy;
}

/* F(u, v) = u atan(v / u) + (v / 2) ln(u^2 + v^2), whose mixed derivative
 * d2F / du dv is u / (u^2 + v^2); F -> 0 as u -> 0 in its first term and as
 * (u, v) -> 0 in its second. */
static double rect_prim(double u, double v)
{
    double r2 = u * u + v * v;
    double a = (u != 0.0) ? u * atan(v / u) : 0.0;
    double b = (r2 > 0.0) ? 0.5 * v * log(r2) : 0.0;
    return a + b;
}

/* Deflection of a uniform density kappa on the rectangle [x0, x1] x [y0, y1]
 * at theta = (tx, ty):
 *   s_x = (kappa / pi) int_{x0}^{x1} int_{y0}^{y1} (tx - x) / ((tx - x)^2 + (ty - y)^2) dy dx,
 * with u = tx - x, v = ty - y the double integral of u / (u^2 + v^2) over
 * u in [tx - x1, tx - x0], v in [ty - y1, ty - y0], i.e. the double difference
 * of F over the corners; s_y likewise with the roles of u and v exchanged. */
static void rect_sheet(double kappa, double x0, double x1, double y0, double y1, double tx,
                       double ty, double *sx, double *sy)
{
    double ua = tx - x1, ub = tx - x0, va = ty - y1, vb = ty - y0;
    double fx = rect_prim(ub, vb) - rect_prim(ua, vb) - rect_prim(ub, va) + rect_prim(ua, va);
    double fy = rect_prim(vb, ub) - rect_prim(va, ub) - rect_prim(vb, ua) + rect_prim(va, ua);
    *sx = kappa / LMO_PI * fx;
    *sy = kappa / LMO_PI * fy;
}

/* the sheet term s(theta) of the lens equation */
static void sheet_term(const lmo_params *p, double tx, double ty, double *sx, double *sy)
{
    if (p->sheet == 1) {
        rect_sheet(p->kappa_star, p->sx0, p->sx1, p->sy0, p->sy1, tx, ty, sx, sy);
    } else {
        *sx = p->kappa_star * tx;
        *sy = p->kappa_star * ty;
    }
}

/* Interpolated scheme with the rectangle sheet.  Inside the rectangle,
 * s(theta) = kappa_star theta + h(theta) where conj(h) is holomorphic (the
 * density is uniform, so s - kappa_star theta has no divergence and no curl);
 * that part is carried by P Taylor coefficients per level-2 cell, like the far
 * lenses.  The expansion point z_e is the centre of the part of the cell that
 * lies in the ray lattice (the cell centre itself except in a partial last
 * column or row).  About z_e the coefficients are
 *   e_n = (1 / 2 pi i) oint conj(h)(z_e + w) w^-(n+1) dw
 * on the circle |w| = r, r half the distance from z_e to the nearest edge of
 * the rectangle (so the circle stays where the closed form is conj(h)); the
 * trapezoid rule over M equally spaced points,
 *   e_n = (1/M) sum_j conj(h)(z_e + w_j) w_j^-n,
 * is exact to rounding for a function analytic on a larger disk.  The
 * polynomial is then written about the cell centre z_c: with t = z_c - z_e,
 * c_k = sum_{n>=k} C(n,k) e_n t^(n-k).  c holds (re, im) of c_0 .. c_{P-1}. */
static void sheet_coeffs(const lmo_params *p, int64_t ci, int64_t cj, double *c)
{
    const int64_t P = p->terms;
    const int M = 64;
    double zx, zy;
    cell_centre(p, ci, cj, &zx, &zy);
    int64_t i1 = (ci + 1) * p->coarse, j1 = (cj + 1) * p->coarse;
    if (i1 > p->ray_nx) i1 = p->ray_nx;
    if (j1 > p->ray_ny) j1 = p->ray_ny;
    double ex = p->ray_x0 + 0.5 * ((double)(ci * p->coarse) + (double)i1) * p->ray_dx;
    double ey = p->ray_y0 + 0.5 * ((double)(cj * p->coarse) + (double)j1) * p->ray_dy;
    double dist = fmin(fmin(ex - p->sx0, p->sx1 - ex), fmin(ey - p->sy0, p->sy1 - ey));
    double r = 0.5 * dist;
    double e[32];
    for (int64_t n = 0; n < 2 * P; ++n) e[n] = 0.0;
    for (int j = 0; j < M; ++j) {
        double phi = 2.0 * LMO_PI * (double)j / (double)M;
        double tx = ex + r * cos(phi), ty = ey + r * sin(phi);
        double sx, sy;
        rect_sheet(p->kappa_star, p->sx0, p->sx1, p->sy0, p->sy1, tx, ty, &sx, &sy);
        /* conj(h) = conj(s) - kappa_star conj(theta) */
        double hr = sx - p->kappa_star * tx, hi = -(sy - p->kappa_star * ty);
        for (int64_t n = 0; n < P; ++n) {
            /* w^-n = r^-n e^(-i n phi) */
            double rn = pow(r, -(double)n), cn = cos((double)n * phi), sn = sin((double)n * phi);
            e[2 * n] += (hr * cn + hi * sn) * rn / (double)M;
            e[2 * n + 1] += (hi * cn - hr * sn) * rn / (double)M;
        }
    }
    double t_x = zx - ex, t_y = zy - ey;
    for (int64_t k = 0; k < P; ++k) {
        double sr = 0.0, si = 0.0;
        double pr = 1.0, pi = 0.0;  /* t^(n-k) */
        double binom = 1.0;         /* C(n, k) */
        for (int64_t n = k; n < P; ++n) {
            sr += binom * (e[2 * n] * pr - e[2 * n + 1] * pi);
            si += binom * (e[2 * n] * pi + e[2 * n + 1] * pr);
            double npr = pr * t_x - pi * t_y, npi = pr * t_y + pi * t_x;
            pr = npr;
            pi = npi;
            binom = binom * (double)(n + 1) / (double)(n + 1 - k);
        }
        c[2 * k] = sr;
        c[2 * k + 1] = si;
    }
}

/* source-plane position (Eq. 6 with the constant Jacobian of Eq. 1, or the
 * fold mapping of Eq. 5) */
static void lens_map(const lmo_params *p, double tx, double ty, double ax, double ay,
                     double *bx, double *by)
{
    double sx, sy;
    if (p->scheme == 1) {
        /* interpolated: the rectangle's holomorphic part is in alpha (far) */
        sx = p->kappa_star * tx;
        sy = p->kappa_star * ty;
    } else {
        sheet_term(p, tx, ty, &sx, &sy);
    }
    if (p->macro == 1) {
        *bx = (0.5 * p->d_x * tx + p->d_y * ty) * tx + sx - ax;
        *by = 2.0 * (1.0 - p->kappa) * ty + sy - ay;
        return;
    }
    double lt = 1.0 - p->kappa - p->gamma, lr = 1.0 - p->kappa + p->gamma;
    *bx = lt * tx + sx - ax;
    *by = lr * ty + sy - ay;
}

/* pixel index q*nx + p of a source position, or -1 outside the map */
static int64_t bin_of(const lmo_params *p, double bx, double by)
{
    double u = floor((bx - p->src_x0) / p->src_dx);
    double v = floor((by - p->src_y0) / p->src_dy);
    if (!(u >= 0.0 && u < (double)p->src_nx && v >= 0.0 && v < (double)p->src_ny)) return -1;
    return (int64_t)v * p->src_nx + (int64_t)u;
}

static int check_params(const lmo_params *p)
{
    if (p->macro != 0 && p->macro != 1) return -1;
    if (p->sheet != 0 && p->sheet != 1) return -1;
    if (p->sheet == 1) {
        /* the rectangle holds the ray lattice (up to rounding of its ends) */
        double lx1 = p->ray_x0 + (double)p->ray_nx * p->ray_dx;
        double ly1 = p->ray_y0 + (double)p->ray_ny * p->ray_dy;
        double tol = 1e-9 * (fabs(p->ray_x0) + fabs(lx1) + fabs(p->ray_y0) + fabs(ly1));
        if (!(p->sx1 > p->sx0 && p->sy1 > p->sy0)) return -1;
        if (p->scheme == 1 && p->terms > 16) return -1;
        if (p->scheme == 1 && (p->ray_x0 < p->sx0 - tol || lx1 > p->sx1 + tol ||
                               p->ray_y0 < p->sy0 - tol || ly1 > p->sy1 + tol))
            return -1;
    }
    if (!(p->src_dx > 0 && p->src_dy > 0 && p->ray_dx > 0 && p->ray_dy > 0)) return -1;
    if (p->src_nx <= 0 || p->src_ny <= 0 || p->ray_nx < 0 || p->ray_ny < 0) return -1;
    if (p->scheme == 1) {
        if (p->coarse <= 0 || p->l1_kx <= 0 || p->l1_ky <= 0 || p->halo < 0) return -1;
        if (p->terms <= 0 || p->terms > 16) return -1;
        if (p->far_order < 0 || (p->far_order > 0 && p->far_order < p->terms)) return -1;
    } else if (p->scheme != 0) {
        return -1;
    }
    return 0;
}

/* ---- exported entry points ---------------------------------------------- */

/* The sheet term s(theta) of the configured map at arbitrary positions. */
int lmo_sheet(const lmo_params *p, const double *theta, int64_t nth, double *s)
{
    if (check_params(p)) return -1;
    for (int64_t t = 0; t < nth; ++t)
        sheet_term(p, theta[2 * t], theta[2 * t + 1], &s[2 * t], &s[2 * t + 1]);
    return 0;
}

/* Direct deflection at arbitrary positions (Sec. 3.2, direct sum). */
int lmo_deflect_direct(const double *lx, const double *ly, const double *lm, int64_t n,
                       const double *theta, int64_t nth, double *alpha)
{
    lmo_lenses L = {lx, ly, lm, n};
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < nth; ++t)
        direct_sum(&L, NULL, 0, theta[2 * t], theta[2 * t + 1], &alpha[2 * t], &alpha[2 * t + 1]);
    return 0;
}

/* Taylor coefficients of level-2 cell (ci,cj); a has 2*terms doubles. */
int lmo_coeffs(const lmo_params *p, const double *lx, const double *ly, const double *lm,
               int64_t n, int64_t ci, int64_t cj, double *a)
{
    if (check_params(p) || p->scheme != 1) return -1;
    lmo_lenses L = {lx, ly, lm, n};
    unsigned char *near = (unsigned char *)malloc((size_t)(n > 0 ? n : 1));
    near_mask(p, &L, ci, cj, near);
    cell_coeffs(p, &L, near, ci, cj, a);
    free(near);
    return 0;
}

/* Near mask of level-2 cell (ci,cj) as bytes (1 = near). */
int lmo_near_mask(const lmo_params *p, const double *lx, const double *ly, int64_t n,
                  int64_t ci, int64_t cj, unsigned char *near)
{
    if (check_params(p) || p->scheme != 1) return -1;
    lmo_lenses L = {lx, ly, NULL, n};
    near_mask(p, &L, ci, cj, near);
    return 0;
}

/* Deflection of the configured scheme at arbitrary positions.  For the
 * interpolated scheme the level-2 cell is the one containing theta. */
int lmo_deflect(const lmo_params *p, const double *lx, const double *ly, const double *lm,
                int64_t n, const double *theta, int64_t nth, double *alpha)
{
    if (check_params(p)) return -1;
    if (p->scheme == 0) return lmo_deflect_direct(lx, ly, lm, n, theta, nth, alpha);
    lmo_lenses L = {lx, ly, lm, n};
    int64_t P = p->terms;
    int err = 0;
#pragma omp parallel
    {
        unsigned char *near = (unsigned char *)malloc((size_t)(n > 0 ? n : 1));
        int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
        double *a = (double *)malloc(sizeof(double) * 2 * (size_t)P);
        if (!near || !idx || !a) {
#pragma omp atomic write
            err = -2;
        } else {
#pragma omp for schedule(dynamic, 16)
            for (int64_t t = 0; t < nth; ++t) {
                double tx = theta[2 * t], ty = theta[2 * t + 1];
                int64_t ci = (int64_t)floor((tx - p->ray_x0) / ((double)p->coarse * p->ray_dx));
                int64_t cj = (int64_t)floor((ty - p->ray_y0) / ((double)p->coarse * p->ray_dy));
                double zx, zy, nx, ny, fx, fy;
                near_mask(p, &L, ci, cj, near);
                cell_centre(p, ci, cj, &zx, &zy);
                cell_coeffs(p, &L, near, ci, cj, a);
                int64_t nn = near_list(near, n, idx);
                direct_sum(&L, idx, nn, tx, ty, &nx, &ny);
                far_eval(P, a, tx - zx, ty - zy, &fx, &fy);
                alpha[2 * t] = nx + fx;
                alpha[2 * t + 1] = ny + fy;
            }
        }
        free(near);
        free(idx);
        free(a);
    }
    return err;
}

/* Source positions and pixel indices of listed lattice rays (i[t], j[t]). */
int lmo_trace(const lmo_params *p, const double *lx, const double *ly, const double *lm,
              int64_t n, const int64_t *ii, const int64_t *jj, int64_t nr, double *beta,
              int64_t *pix)
{
    if (check_params(p)) return -1;
    double *th = (double *)calloc(2 * (size_t)(nr > 0 ? nr : 1), sizeof(double));
    double *al = (double *)malloc(sizeof(double) * 2 * (size_t)(nr > 0 ? nr : 1));
    if (!th || !al) {
        free(th);
        free(al);
        return -2;
    }
    for (int64_t t = 0; t < nr; ++t) {
        th[2 * t] = p->ray_x0 + ((double)ii[t] + 0.5) * p->ray_dx;
        th[2 * t + 1] = p->ray_y0 + ((double)jj[t] + 0.5) * p->ray_dy;
    }
    int rc = lmo_deflect(p, lx, ly, lm, n, th, nr, al);
    if (rc == 0) {
        for (int64_t t = 0; t < nr; ++t) {
            double bx, by;
            lens_map(p, th[2 * t], th[2 * t + 1], al[2 * t], al[2 * t + 1], &bx, &by);
            beta[2 * t] = bx;
            beta[2 * t + 1] = by;
            pix[t] = bin_of(p, bx, by);
        }
    }
    free(th);
    free(al);
    return rc;
}

/* Shoot the rays of the lattice sub-rectangle [i0,i0+ni) x [j0,j0+nj) and add
 * those landing in the pixel window [wp0, wp0+wnp) x [wq0, wq0+wnq) of the map
 * to counts[wnq*wnp] (row-major); every other ray (outside the map or outside
 * the window) is added to *n_out.  nthreads <= 0 uses the OpenMP default. */
int lmo_shoot_window(const lmo_params *p, const double *lx, const double *ly, const double *lm,
                     int64_t n, int64_t i0, int64_t j0, int64_t ni, int64_t nj, int64_t wp0,
                     int64_t wq0, int64_t wnp, int64_t wnq, uint64_t *counts, uint64_t *n_out,
                     int nthreads);

/* Shoot into the whole map: counts[src_ny*src_nx] (row-major, q*src_nx + p). */
int lmo_shoot(const lmo_params *p, const double *lx, const double *ly, const double *lm,
              int64_t n, int64_t i0, int64_t j0, int64_t ni, int64_t nj, uint64_t *counts,
              uint64_t *n_out, int nthreads)
{
    return lmo_shoot_window(p, lx, ly, lm, n, i0, j0, ni, nj, 0, 0, p->src_nx, p->src_ny, counts,
                            n_out, nthreads);
}

/* index of a map pixel in the window, or -1 */
static int64_t window_of(int64_t b, const lmo_params *p, int64_t wp0, int64_t wq0, int64_t wnp,
                         int64_t wnq)
{
    if (b < 0) return -1;
    int64_t q = b / p->src_nx, pp = b % p->src_nx;
    if (pp < wp0 || pp >= wp0 + wnp || q < wq0 || q >= wq0 + wnq) return -1;
    return (q - wq0) * wnp + (pp - wp0);
}

int lmo_shoot_window(const lmo_params *p, const double *lx, const double *ly, const double *lm,
                     int64_t n, int64_t i0, int64_t j0, int64_t ni, int64_t nj, int64_t wp0,
                     int64_t wq0, int64_t wnp, int64_t wnq, uint64_t *counts, uint64_t *n_out,
                     int nthreads)
{
    if (check_params(p)) return -1;
    if (wnp <= 0 || wnq <= 0) return -1;
    if (ni < 0 || nj < 0 || i0 < 0 || j0 < 0 || i0 + ni > p->ray_nx || j0 + nj > p->ray_ny)
        return -1;
    if (ni == 0 || nj == 0) return 0;
    /* thread count of this call only: a num_threads clause, not
     * omp_set_num_threads, which would stay in force for later calls */
#ifdef _OPENMP
    const int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    const int nt = 1;
    (void)nthreads;
#endif
    lmo_lenses L = {lx, ly, lm, n};
    uint64_t outs = 0;
    int err = 0;
    if (p->scheme == 0) {
        /* direct: one row of rays per task */
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : outs) num_threads(nt)
        for (int64_t j = j0; j < j0 + nj; ++j) {
            double ty = p->ray_y0 + ((double)j + 0.5) * p->ray_dy;
            for (int64_t i = i0; i < i0 + ni; ++i) {
                double tx = p->ray_x0 + ((double)i + 0.5) * p->ray_dx;
                double ax, ay, bx, by;
                direct_sum(&L, NULL, 0, tx, ty, &ax, &ay);
                lens_map(p, tx, ty, ax, ay, &bx, &by);
                int64_t b = window_of(bin_of(p, bx, by), p, wp0, wq0, wnp, wnq);
                if (b < 0) {
                    ++outs;
                } else {
#pragma omp atomic update
                    counts[b] += 1;
                }
            }
        }
    } else {
        /* interpolated: one level-2 cell per task; its coefficients and near
         * set are found once and used for all of its rays */
        int64_t R = p->coarse, P = p->terms;
        int64_t ci0 = i0 / R, ci1 = (i0 + ni - 1) / R, cj0 = j0 / R, cj1 = (j0 + nj - 1) / R;
        int64_t ncx = ci1 - ci0 + 1, ncells = ncx * (cj1 - cj0 + 1);
#pragma omp parallel reduction(+ : outs) num_threads(nt)
        {
            unsigned char *near = (unsigned char *)malloc((size_t)(n > 0 ? n : 1));
            int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
            double *a = (double *)malloc(sizeof(double) * 2 * (size_t)P);
            if (!near || !idx || !a) {
#pragma omp atomic write
                err = -2;
            } else {
#pragma omp for schedule(dynamic, 1)
                for (int64_t c = 0; c < ncells; ++c) {
                    int64_t ci = ci0 + c % ncx, cj = cj0 + c / ncx;
                    double zx, zy;
                    near_mask(p, &L, ci, cj, near);
                    cell_centre(p, ci, cj, &zx, &zy);
                    cell_coeffs(p, &L, near, ci, cj, a);
                    int64_t nn = near_list(near, n, idx);
                    int64_t ia = ci * R > i0 ? ci * R : i0;
                    int64_t ib = (ci + 1) * R < i0 + ni ? (ci + 1) * R : i0 + ni;
                    int64_t ja = cj * R > j0 ? cj * R : j0;
                    int64_t jb = (cj + 1) * R < j0 + nj ? (cj + 1) * R : j0 + nj;
                    for (int64_t j = ja; j < jb; ++j) {
                        double ty = p->ray_y0 + ((double)j + 0.5) * p->ray_dy;
                        for (int64_t i = ia; i < ib; ++i) {
                            double tx = p->ray_x0 + ((double)i + 0.5) * p->ray_dx;
                            double nx, ny, fx, fy, bx, by;
                            direct_sum(&L, idx, nn, tx, ty, &nx, &ny);
                            far_eval(P, a, tx - zx, ty - zy, &fx, &fy);
                            lens_map(p, tx, ty, nx + fx, ny + fy, &bx, &by);
                            int64_t b = window_of(bin_of(p, bx, by), p, wp0, wq0, wnp, wnq);
                            if (b < 0) {
                                ++outs;
                            } else {
#pragma omp atomic update
                                counts[b] += 1;
                            }
                        }
                    }
                }
            }
            free(near);
            free(idx);
            free(a);
        }
    }
    *n_out += outs;
    return err;
}

/* Magnification of a pixel from its count (Eq. 12). */
double lmo_mu_factor(const lmo_params *p)
{
    return (p->ray_dx * p->ray_dy) / (p->src_dx * p->src_dy);
}

int lmo_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
