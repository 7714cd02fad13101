// lm_api.cpp -- host side of liblensmap: C ABI, geometry rules, lens
// partition into level-1 cells, device buffers, launches, batching and the
// execution-parameter tuner.  The kernels live in lm_kernels.hip.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <new>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/lensmap.h"
#include "lm_internal.h"

namespace {

thread_local std::string g_err;

lm_status fail(lm_status code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

lm_status ok()
{
    g_err.clear();
    return LM_OK;
}

#define HIP_TRY(call)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(LM_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));     \
    } while (0)

#define LAUNCH_TRY(expr)                                                                 \
    do {                                                                                 \
        int e_ = (expr);                                                                 \
        if (e_ != 0)                                                                     \
            return fail(LM_EDEVICE, "%s failed: %s", #expr,                             \
                        hipGetErrorString((hipError_t)e_));                              \
    } while (0)

bool isfin(double v) { return std::isfinite(v); }

int64_t round_half_away(double x) { return x >= 0 ? (int64_t)std::floor(x + 0.5) : -(int64_t)std::floor(-x + 0.5); }

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Device buffer owned by a map or batch.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    ~DevBuf() { release(); }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    hipError_t ensure(size_t n)
    {
        if (n <= bytes && p) return hipSuccess;
        release();
        if (n == 0) return hipSuccess;
        hipError_t e = hipMalloc(&p, n);
        if (e == hipSuccess) bytes = n;
        return e;
    }
    template <class T>
    T* as() const { return static_cast<T*>(p); }
};

// Boxes of the hierarchical far field: a level-1 cell whose sides differ is
// cut along its longer side into n = round(long / short) near-square boxes of
// b = ceil(K / n) level-2 cells (the last one may be narrower), each with its
// own series about its centre; a square-ish cell is one box.
struct FarBoxes {
    int nx = 1, ny = 1, bx = 1, by = 1;
};

FarBoxes far_boxes(const lm_geometry& g)
{
    FarBoxes f;
    const double l1x = (double)((int64_t)g.l1_kx * g.coarse) * g.ray_dx;
    const double l1y = (double)((int64_t)g.l1_ky * g.coarse) * g.ray_dy;
    if (l1x > l1y) f.nx = (int)std::max<int64_t>(1, round_half_away(l1x / l1y));
    if (l1y > l1x) f.ny = (int)std::max<int64_t>(1, round_half_away(l1y / l1x));
    f.nx = std::min(f.nx, g.l1_kx);
    f.ny = std::min(f.ny, g.l1_ky);
    f.bx = (int)ceil_div(g.l1_kx, f.nx);
    f.by = (int)ceil_div(g.l1_ky, f.ny);
    return f;
}

// Largest ratio |z_c - Z| / |z_k - Z| of the hierarchical far field: level-2
// centres lie within ((b-1)/2 L2x, (b'-1)/2 L2y) of their box centre Z, far
// lenses outside the (2H+1)^2 block of level-1 cells, at least H L1 + b L2 / 2
// from Z along each axis; the largest over full and narrower last boxes.
double far_ratio(const lm_geometry& g)
{
    const double l2x = (double)g.coarse * g.ray_dx, l2y = (double)g.coarse * g.ray_dy;
    const double l1x = g.l1_kx * l2x, l1y = g.l1_ky * l2y;
    const FarBoxes f = far_boxes(g);
    const int lastx = g.l1_kx - (f.nx - 1) * f.bx, lasty = g.l1_ky - (f.ny - 1) * f.by;
    double rho = 0.0;
    for (int wx : {f.bx, lastx})
        for (int wy : {f.by, lasty}) {
            if (wx < 1 || wy < 1) continue;
            const double hx = 0.5 * (wx - 1) * l2x, hy = 0.5 * (wy - 1) * l2y;
            const double umin = std::min(g.near_halo * l1x + 0.5 * wx * l2x,
                                         g.near_halo * l1y + 0.5 * wy * l2y);
            rho = std::max(rho, std::sqrt(hx * hx + hy * hy) / umin);
        }
    return rho;
}

lm_status validate_geometry(const lm_geometry* g)
{
    if (!g) return fail(LM_EINVAL, "geometry is NULL");
    const double v[] = {g->src_x0, g->src_y0, g->src_dx, g->src_dy,
                        g->ray_x0, g->ray_y0, g->ray_dx, g->ray_dy};
    for (double x : v)
        if (!isfin(x)) return fail(LM_EINVAL, "geometry has a non-finite value");
    if (!(g->src_dx > 0 && g->src_dy > 0 && g->ray_dx > 0 && g->ray_dy > 0))
        return fail(LM_EINVAL, "pixel and ray spacings must be positive");
    if (g->src_nx <= 0 || g->src_ny <= 0) return fail(LM_EINVAL, "source map must have pixels");
    if (g->src_nx > (1 << 30) || g->src_ny > (1 << 30))
        return fail(LM_EINVAL, "a source map side must be at most 2^30 pixels");
    if ((int64_t)g->src_nx * g->src_ny >= (int64_t(1) << 40))
        return fail(LM_EINVAL, "source map too large (src_nx*src_ny must be < 2^40)");
    if (g->ray_nx <= 0 || g->ray_ny <= 0) return fail(LM_EINVAL, "ray lattice must be non-empty");
    if (g->scheme != LM_SCHEME_DIRECT && g->scheme != LM_SCHEME_INTERP)
        return fail(LM_EINVAL, "unknown scheme %d", g->scheme);
    if (g->precision != LM_PREC_MIXED && g->precision != LM_PREC_FP32 &&
        g->precision != LM_PREC_MIXED_FP64 && g->precision != LM_PREC_AUTO &&
        g->precision != LM_PREC_MIXED_CENTRED)
        return fail(LM_EINVAL, "unknown precision %d", g->precision);
    if ((g->precision == LM_PREC_MIXED_FP64 || g->precision == LM_PREC_MIXED_CENTRED) &&
        g->scheme != LM_SCHEME_INTERP)
        return fail(LM_EUNSUPPORTED, "precision %d is built for the interpolated scheme only",
                    g->precision);
    if (g->far_order != 0) {
        if (g->scheme != LM_SCHEME_INTERP)
            return fail(LM_EINVAL, "far_order needs the interpolated scheme");
        if (g->precision == LM_PREC_FP32)
            return fail(LM_EUNSUPPORTED, "far_order is built for the FP64-coefficient precisions");
        if (g->far_order < g->taylor_terms || g->far_order > 64)
            return fail(LM_EINVAL, "far_order must be 0 or in [taylor_terms, 64], got %d",
                        g->far_order);
        // truncation: |z_c - Z| / |z_k - Z| <= rho for every level-2 centre z_c
        // of a level-1 cell and every far lens z_k; the series must reach
        // rho^Q / (1 - rho) <= 1e-9
        const double rho = far_ratio(*g);
        if (!(rho < 1.0) || std::pow(rho, g->far_order) / (1.0 - rho) > 1e-9)
            return fail(LM_EINVAL,
                        "far_order %d is too small for this geometry (convergence ratio %.3f)",
                        g->far_order, rho);
    }
    if (g->coarse <= 0 || g->coarse % 64 != 0 || g->coarse > (1 << 15))
        return fail(LM_EINVAL, "coarse must be a positive multiple of 64 (at most 32768), got %d",
                    g->coarse);
    if (g->scheme == LM_SCHEME_INTERP) {
        if (g->l1_kx <= 0 || g->l1_ky <= 0) return fail(LM_EINVAL, "l1_kx, l1_ky must be positive");
        if (g->near_halo < 0 || g->near_halo > 64) return fail(LM_EINVAL, "near_halo must be in 0..64");
        if (g->taylor_terms < 1 || g->taylor_terms > LM_MAX_TERMS)
            return fail(LM_EINVAL, "taylor_terms must be in 1..%d", LM_MAX_TERMS);
    }
    const int64_t ncx = ceil_div(g->ray_nx, g->coarse), ncy = ceil_div(g->ray_ny, g->coarse);
    if (ncx > (int64_t(1) << 40) / std::max<int64_t>(ncy, 1))
        return fail(LM_EINVAL, "lattice too large");
    return LM_OK;
}

}  // namespace

// ====================================================================== map

struct lm_map {
    lm_geometry g{};
    int device = 0;
    double kappa = 0, gamma = 0, kappa_star = 0;
    bool fold = false;
    double fold_dx = 0, fold_dy = 0;  // 1/theta_E
    // the -kappa_star sheet: infinite about the origin, or on a rectangle
    bool sheet = false;
    double sheet_x0 = 0, sheet_x1 = 0, sheet_y0 = 0, sheet_y1 = 0;
    int64_t nlens = 0;
    // derived
    int64_t ncx = 0, ncy = 0, n1x = 0, n1y = 0;
    int nl1x = 0, nl1y = 0;
    // device buffers
    DevBuf lx, ly, lmd, lxf, lyf, lmf, lI, lJ, cell_start, coef, counts_own, n_out, ptab, l1exp;
    std::vector<int32_t> h_start;  // host copy of the level-1 CSR
    uint64_t* counts = nullptr;  // own or bound
    bool bound = false;
    bool coef_valid = false;
    bool has_counts = false;
    uint64_t n_shot = 0;
    hipStream_t last = nullptr;
    int rays_per_lane = 16;
    // bumped by every call that changes what a batch's captured launches read
    // (lens buffers and count, macro model, counts buffer)
    uint64_t gen = 0;
    uint64_t model_gen = 0;  // bumped by changes of the lenses or the macro model
    // precision the kernels run in: the geometry's, or for LM_PREC_AUTO the
    // one chosen for the current lenses and macro model (prec_gen == gen)
    int prec = LM_PREC_MIXED;
    uint64_t prec_gen = ~0ull;
    double prec_est = -1.0;  // LM_PREC_AUTO: estimated FP32 near-sum bin mismatch
    double prec_est_centred = -1.0;  // ... and of the centred FP32 near sums
};

namespace {

lm_status use_device(const lm_map* m)
{
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != m->device) HIP_TRY(hipSetDevice(m->device));
    return LM_OK;
}

// Work decomposition of a tile: cells per side, column chunks, window.
struct Exec {
    int G = 1, ncc = 1, cw = 64, wx = 64, wy = 64;
};

// Level-2 cells per side of a workgroup tile: about 512 rays per side times the
// tile scale, fewer if a rectangle of ncells_x x ncells_y cells would then give
// fewer than 4096 tiles (too few to fill the device) or a tile would hold 1e9
// rays or more.
int tile_cells(int R, int64_t ncells_x, int64_t ncells_y, int g_scale)
{
    int G = std::max(1, 512 / R) * std::max(1, g_scale);
    while (G > 1 && ceil_div(ncells_x, G) * ceil_div(ncells_y, G) < 4096) G /= 2;
    while (G > 1 && (double)G * G * R * R > 1.0e9) G /= 2;
    return G;
}

// Level-2 cells of the rectangle i0 + [0, ni) x j0 + [0, nj) per side.
void rect_cells(int R, int64_t i0, int64_t j0, int64_t ni, int64_t nj, int64_t& cx, int64_t& cy)
{
    cx = ni > 0 ? (i0 + ni - 1) / R - i0 / R + 1 : 1;
    cy = nj > 0 ? (j0 + nj - 1) / R - j0 / R + 1 : 1;
}

// win_max: uint32 bins the kernel's LDS window holds (its layout's).
// Rays per lane a kernel of precision prec runs when nr are asked for (the
// centred sums run at most 8).
int lanes_nr(int prec, int nr) { return prec == LM_PREC_MIXED_CENTRED && nr > 8 ? 8 : nr; }

Exec choose_exec(const lm_map* m, int64_t ncells_x, int64_t ncells_y, int g_scale,
                 int win_max = kLayWin[0])
{
    const lm_geometry& g = m->g;
    Exec e;
    const int R = g.coarse;
    const int G = tile_cells(R, ncells_x, ncells_y, g_scale);
    e.G = G;
    const int nrb = R / 64;
    int ncc = 1;
    while ((G * G * nrb * ncc) % LM_WAVES != 0) ncc *= 2;
    e.ncc = ncc;
    e.cw = (int)ceil_div(R, ncc);
    double mx = std::fabs(1.0 - m->kappa - m->gamma + m->kappa_star);
    double my = std::fabs(1.0 - m->kappa + m->gamma + m->kappa_star);
    if (m->fold) {
        // largest Jacobian entries over the lattice
        const double hx = 0.5 * g.ray_nx * g.ray_dx, hy = 0.5 * g.ray_ny * g.ray_dy;
        mx = std::fabs(m->kappa_star) + std::fabs(m->fold_dx) * hx + 2.0 * std::fabs(m->fold_dy) * hx +
             std::fabs(m->fold_dy) * hy;
        my = std::fabs(2.0 * (1.0 - m->kappa) + m->kappa_star);
    }
    // pixels spanned by the tile's smooth image, plus a margin of 0.1 theta_E
    // (at least 8 pixels) on each side for the variation of the near-lens
    // deflection across the tile
    const double ext_x = (double)G * R * g.ray_dx * mx / g.src_dx + 2.0 * std::max(8.0, 0.1 / g.src_dx);
    const double ext_y = (double)G * R * g.ray_dy * my / g.src_dy + 2.0 * std::max(8.0, 0.1 / g.src_dy);
    // use the whole LDS window in the extents' aspect ratio (sides multiples
    // of 8): more rays counted in LDS, fewer global atomics
    const double fill = std::sqrt((double)win_max / (ext_x * ext_y));
    int wx = std::max(8, std::min(win_max / 8, (int)(ext_x * fill) / 8 * 8));
    int wy = std::max(8, std::min(win_max / 8, (int)(ext_y * fill) / 8 * 8));
    while (wx * wy > win_max) {
        if (wy <= 8 || (wx > 8 && wx / ext_x > wy / ext_y))
            wx -= 8;
        else
            wy -= 8;
    }
    e.wx = wx;
    e.wy = wy;
    return e;
}

void split_ff(double v, float& hi, float& lo)
{
    hi = (float)v;
    lo = (float)(v - (double)hi);
}

LmDesc make_desc(const lm_map* m, int64_t i0, int64_t j0, int64_t i1, int64_t j1, const Exec& e)
{
    const lm_geometry& g = m->g;
    LmDesc d;
    std::memset(&d, 0, sizeof d);
    d.x0 = g.ray_x0;
    d.y0 = g.ray_y0;
    d.dx = g.ray_dx;
    d.dy = g.ray_dy;
    d.sheet = m->sheet ? 1 : 0;
    d.sx0 = m->sheet_x0;
    d.sx1 = m->sheet_x1;
    d.sy0 = m->sheet_y0;
    d.sy1 = m->sheet_y1;
    d.kappa_star = m->kappa_star;
    if (m->fold) {
        d.fold = 1;
        d.mx = m->kappa_star;
        d.my = 2.0 * (1.0 - m->kappa) + m->kappa_star;
        d.qx = 0.5 * m->fold_dx;
        d.qy = m->fold_dy;
    } else {
        d.mx = 1.0 - m->kappa - m->gamma + m->kappa_star;
        d.my = 1.0 - m->kappa + m->gamma + m->kappa_star;
    }
    d.bx0 = g.src_x0;
    d.by0 = g.src_y0;
    d.inv_sdx = 1.0 / g.src_dx;
    d.inv_sdy = 1.0 / g.src_dy;
    split_ff(0.5 * g.ray_dx, d.hxh, d.hxl);
    split_ff(0.5 * g.ray_dy, d.hyh, d.hyl);
    d.x0f = (float)g.ray_x0;
    d.y0f = (float)g.ray_y0;
    d.dxf = (float)g.ray_dx;
    d.dyf = (float)g.ray_dy;
    d.mxf = (float)d.mx;
    d.myf = (float)d.my;
    d.bx0f = (float)g.src_x0;
    d.by0f = (float)g.src_y0;
    d.inv_sdxf = (float)d.inv_sdx;
    d.inv_sdyf = (float)d.inv_sdy;
    d.snx = g.src_nx;
    d.sny = g.src_ny;
    d.R = g.coarse;
    d.Kx = g.scheme == LM_SCHEME_INTERP ? g.l1_kx : 1;
    d.Ky = g.scheme == LM_SCHEME_INTERP ? g.l1_ky : 1;
    d.H = g.scheme == LM_SCHEME_INTERP ? g.near_halo : 0;
    d.G = e.G;
    d.ncc = e.ncc;
    d.cw = e.cw;
    d.nrb = g.coarse / 64;
    d.wx = e.wx;
    d.wy = e.wy;
    d.nl1x = m->nl1x;
    d.nl1y = m->nl1y;
    d.nx = g.ray_nx;
    d.ny = g.ray_ny;
    d.i0 = i0;
    d.j0 = j0;
    d.i1 = i1;
    d.j1 = j1;
    d.ncx = m->ncx;
    d.ncy = m->ncy;
    if (i1 > i0 && j1 > j0) {
        const int64_t ci_lo = i0 / g.coarse, ci_hi = (i1 - 1) / g.coarse;
        const int64_t cj_lo = j0 / g.coarse, cj_hi = (j1 - 1) / g.coarse;
        d.tcx0 = ci_lo / e.G;
        d.tcy0 = cj_lo / e.G;
        d.ntx = ci_hi / e.G - d.tcx0 + 1;
        d.nty = cj_hi / e.G - d.tcy0 + 1;
        d.ntiles = d.ntx * d.nty;
    }
    d.nlens = m->nlens;
    d.lx = m->lx.as<double>();
    d.ly = m->ly.as<double>();
    d.lmd = m->lmd.as<double>();
    d.lxf = m->lxf.as<float>();
    d.lyf = m->lyf.as<float>();
    d.lmf = m->lmf.as<float>();
    d.lI = m->lI.as<int32_t>();
    d.lJ = m->lJ.as<int32_t>();
    d.cell_start = m->cell_start.as<int32_t>();
    d.coef = m->coef.as<LmCoef>();
    d.ptab = m->ptab.as<float>();
    d.Q = g.scheme == LM_SCHEME_INTERP ? g.far_order : 0;
    d.n1x = m->n1x;
    {
        const FarBoxes f = far_boxes(g);
        d.nbx = f.nx;
        d.nby = f.ny;
        d.bx = f.bx;
        d.by = f.by;
    }
    d.n1y = m->n1y;
    d.l1exp = m->l1exp.as<double>();
    d.counts = reinterpret_cast<unsigned long long*>(m->counts);
    d.n_out = m->n_out.as<unsigned long long>();
    return d;
}

lm_status ensure_coef(lm_map* m)
{
    if (m->g.scheme != LM_SCHEME_INTERP) return LM_OK;
    if (m->coef.ensure((size_t)(m->ncx * m->ncy) * sizeof(LmCoef)) != hipSuccess)
        return fail(LM_ENOMEM, "cannot allocate %lld level-2 coefficient records",
                    (long long)(m->ncx * m->ncy));
    if (m->g.far_order > 0 &&
        m->l1exp.ensure((size_t)(m->n1x * m->n1y) * far_boxes(m->g).nx * far_boxes(m->g).ny *
                        m->g.far_order * 16) != hipSuccess)
        return fail(LM_ENOMEM, "cannot allocate the level-1 series");
    return LM_OK;
}

// Coefficients of every level-2 cell of a map (direct, or hierarchical), and
// the near-lens deflection of every cell centre (for the centred near sums).
int launch_coefficients(const lm_map* m, const LmDesc& d, hipStream_t s)
{
    int e = m->g.far_order > 0
                ? lm_launch_coeffs_hier(d, m->g.taylor_terms, m->coef.as<LmCoef>(), s)
                : lm_launch_coeffs(d, m->g.precision, m->g.taylor_terms, 0, 0, m->ncx, m->ncy,
                                   m->coef.as<LmCoef>(), s);
    if (e == 0 && m->sheet) e = lm_launch_sheet(d, m->g.taylor_terms, m->coef.as<LmCoef>(), s);
    if (e == 0) e = lm_launch_near_centre(d, m->coef.as<LmCoef>(), s);
    return e;
}

lm_status prepare(lm_map* m, hipStream_t s)
{
    if (m->g.scheme != LM_SCHEME_INTERP) return LM_OK;
    if (m->ncx * m->ncy >= (int64_t(1) << 30))
        return fail(LM_EUNSUPPORTED, "more than 2^30 level-2 cells");
    lm_status st = ensure_coef(m);
    if (st) return st;
    LmDesc d = make_desc(m, 0, 0, 0, 0, Exec{});
    LAUNCH_TRY(launch_coefficients(m, d, s));
    m->coef_valid = true;
    m->last = s;
    return LM_OK;
}

uint64_t splitmix64(uint64_t x)
{
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}

constexpr int64_t kPrecSample = 65536;   // rays probed to choose the near-sum precision
constexpr double kPrecFp32Max = 5e-6;    // largest estimated FP32 mismatch kept in FP32
constexpr double kPrecFp32MaxNear = 32;  // longest mean near list kept in FP32

// Near lenses of level-1 cell (I, J): its 2H+1 rows of the padded CSR.
int64_t near_count(const lm_map* m, int64_t I, int64_t J)
{
    const int H = m->g.near_halo;
    int64_t n = 0;
    for (int r = 0; r <= 2 * H; ++r) {
        const int64_t base = (J + r) * m->nl1x + I;
        n += m->h_start[base + 2 * H + 1] - m->h_start[base];
    }
    return n;
}

// Mean near-list length over the rays of the whole lattice.
double mean_near(const lm_map* m)
{
    const lm_geometry& g = m->g;
    const int64_t sx = (int64_t)g.coarse * g.l1_kx, sy = (int64_t)g.coarse * g.l1_ky;
    double pairs = 0.0;
    for (int64_t J = 0; J < m->n1y; ++J) {
        const double ry = (double)(std::min(g.ray_ny, (J + 1) * sy) - J * sy);
        for (int64_t I = 0; I < m->n1x; ++I) {
            const double rx = (double)(std::min(g.ray_nx, (I + 1) * sx) - I * sx);
            pairs += rx * ry * (double)near_count(m, I, J);
        }
    }
    return pairs / ((double)g.ray_nx * (double)g.ray_ny);
}

// LM_PREC_AUTO: the near-sum precision for the current lenses and macro model.
// A ray changes pixel when rounding moves its image across a pixel edge; for
// images spread evenly over their pixels that happens with probability
// |du| + |dv|, the move in pixel units.  The bin mismatch of FP32 near sums,
// plain and centred, is estimated as the mean of that move against FP64 near
// sums over the rays of a fixed lattice sample (all rays of small lattices)
// whose images lie in the map.  The cheapest form whose estimate is at most
// kPrecFp32Max, half the 1e-5 bar, is taken -- plain FP32, then centred FP32
// (about a third more work per near pair) -- while the mean near list holds at
// most kPrecFp32MaxNear lenses; otherwise the near pairs are summed in FP64.  The
// second condition covers what a lattice mean misses: the rounding of an FP32
// running sum grows with the number of its terms and, with long lists, varies
// strongly from one region to the next (with ~110 near lenses a lattice mean of
// 3.4e-6 came with 1.8e-5 in a 2e6-ray region).  The paper's level-1 size
// gives about 9 near lenses; lists of 32 and more arise only when a caller
// enlarges the level-1 cells.  The direct scheme has no FP64 near-sum mode and keeps
// LM_PREC_MIXED (its FP32 sums are compensated per 256-lens block).
lm_status resolve_precision(lm_map* m, hipStream_t s)
{
    if (m->g.precision != LM_PREC_AUTO) {
        m->prec = m->g.precision;
        return LM_OK;
    }
    if (m->prec_gen == m->model_gen) return LM_OK;
    if (m->g.scheme != LM_SCHEME_INTERP || m->nlens == 0) {
        m->prec = LM_PREC_MIXED;
        m->prec_est = 0.0;
        m->prec_est_centred = 0.0;
        m->prec_gen = m->model_gen;
        return LM_OK;
    }
    lm_status st;
    if (!m->coef_valid) {
        st = prepare(m, s);
        if (st) return st;
    }
    const lm_geometry& g = m->g;
    const int64_t nrays = g.ray_nx * g.ray_ny;
    const int64_t n = std::min<int64_t>(kPrecSample, nrays);
    std::vector<int64_t> hi(n), hj(n);
    for (int64_t t = 0; t < n; ++t) {
        if (n == nrays) {
            hi[t] = t % g.ray_nx;
            hj[t] = t / g.ray_nx;
        } else {
            hi[t] = (int64_t)(splitmix64(2 * (uint64_t)t) % (uint64_t)g.ray_nx);
            hj[t] = (int64_t)(splitmix64(2 * (uint64_t)t + 1) % (uint64_t)g.ray_ny);
        }
    }
    DevBuf di, dj, dp, dq, u32, uct, u64;
    if (di.ensure(n * 8) || dj.ensure(n * 8) || dp.ensure(n * 4) || dq.ensure(n * 4) ||
        u32.ensure(n * 16) || uct.ensure(n * 16) || u64.ensure(n * 16))
        return fail(LM_ENOMEM, "cannot allocate the precision probe");
    HIP_TRY(hipMemcpyAsync(di.p, hi.data(), n * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(dj.p, hj.data(), n * 8, hipMemcpyHostToDevice, s));
    const LmDesc d = make_desc(m, 0, 0, 0, 0, Exec{});
    LAUNCH_TRY(lm_launch_trace(d, g.scheme, LM_PREC_MIXED, g.taylor_terms, di.as<int64_t>(),
                               dj.as<int64_t>(), n, dp.as<int32_t>(), dq.as<int32_t>(),
                               u32.as<double>(), s));
    LAUNCH_TRY(lm_launch_trace(d, g.scheme, LM_PREC_MIXED_CENTRED, g.taylor_terms,
                               di.as<int64_t>(), dj.as<int64_t>(), n, dp.as<int32_t>(),
                               dq.as<int32_t>(), uct.as<double>(), s));
    LAUNCH_TRY(lm_launch_trace(d, g.scheme, LM_PREC_MIXED_FP64, g.taylor_terms, di.as<int64_t>(),
                               dj.as<int64_t>(), n, dp.as<int32_t>(), dq.as<int32_t>(),
                               u64.as<double>(), s));
    std::vector<double> a(2 * n), c(2 * n), b(2 * n);
    HIP_TRY(hipMemcpyAsync(a.data(), u32.p, n * 16, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(c.data(), uct.p, n * 16, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(b.data(), u64.p, n * 16, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    double acc = 0.0, acc_c = 0.0;
    int64_t n_in = 0;
    auto move = [](double du, double dv) {
        const double mv = std::fabs(du) + std::fabs(dv);
        return std::isfinite(mv) ? std::min(1.0, mv) : 1.0;
    };
    for (int64_t t = 0; t < n; ++t) {
        const double u = b[2 * t], v = b[2 * t + 1];
        if (!(u >= 0.0 && u < g.src_nx && v >= 0.0 && v < g.src_ny)) continue;
        ++n_in;
        acc += move(a[2 * t] - u, a[2 * t + 1] - v);
        acc_c += move(c[2 * t] - u, c[2 * t + 1] - v);
    }
    // per ray imaged into the map: a shot region that lands inside the map
    // sees this rate, however few of the lattice's rays reach the map
    m->prec_est = n_in > 0 ? acc / (double)n_in : 0.0;
    m->prec_est_centred = n_in > 0 ? acc_c / (double)n_in : 0.0;
    const bool short_lists = mean_near(m) <= kPrecFp32MaxNear;
    if (short_lists && m->prec_est <= kPrecFp32Max)
        m->prec = LM_PREC_MIXED;
    else if (short_lists && m->prec_est_centred <= kPrecFp32Max)
        m->prec = LM_PREC_MIXED_CENTRED;
    else
        m->prec = LM_PREC_MIXED_FP64;
    m->prec_gen = m->model_gen;
    m->last = s;
    return LM_OK;
}

}  // namespace

extern "C" {

const char* lm_last_error(void) { return g_err.c_str(); }

const char* lm_version(void) { return "lensmap 0.1 (gfx950)"; }

lm_status lm_geometry_derive(lm_geometry* g, double src_lx, double src_ly, int32_t src_nx,
                             int32_t src_ny, double kappa, double gamma, double kappa_star,
                             double protect, double n_rays, int64_t ray_nx, int64_t ray_ny,
                             int32_t scheme, int32_t coarse, double mean_mass)
{
    if (!g) return fail(LM_EINVAL, "g is NULL");
    if (!(isfin(src_lx) && isfin(src_ly) && isfin(kappa) && isfin(gamma) &&
          isfin(kappa_star) && isfin(protect) && isfin(mean_mass)))
        return fail(LM_EINVAL, "non-finite input");
    if (!(src_lx > 0 && src_ly > 0) || src_nx <= 0 || src_ny <= 0)
        return fail(LM_EINVAL, "source region and pixels must be positive");
    if (kappa_star < 0 || !(mean_mass > 0)) return fail(LM_EINVAL, "bad kappa_star or mean mass");
    if (scheme != LM_SCHEME_DIRECT && scheme != LM_SCHEME_INTERP)
        return fail(LM_EINVAL, "unknown scheme %d", scheme);
    const double lt = 1.0 - kappa - gamma, lr = 1.0 - kappa + gamma;
    if (lt == 0.0 || lr == 0.0) return fail(LM_EINVAL, "the mean macro map is singular");
    // protection zone (Sec. 3.1) and its preimage (the shooting region)
    const double w = protect < 0 ? 10.0 * std::sqrt(kappa_star) : protect;
    const double lix = (src_lx + 2.0 * w) / std::fabs(lt);
    const double liy = (src_ly + 2.0 * w) / std::fabs(lr);
    if (ray_nx <= 0 || ray_ny <= 0) {
        if (!(isfin(n_rays) && n_rays >= 1.0)) return fail(LM_EINVAL, "n_rays must be >= 1");
        const double l3 = std::sqrt(lix * liy / n_rays);  // Eq. 11
        ray_nx = std::max<int64_t>(1, round_half_away(lix / l3));
        ray_ny = std::max<int64_t>(1, round_half_away(liy / l3));
    }
    std::memset(g, 0, sizeof *g);
    g->src_x0 = -0.5 * src_lx;
    g->src_y0 = -0.5 * src_ly;
    g->src_dx = src_lx / src_nx;
    g->src_dy = src_ly / src_ny;
    g->src_nx = src_nx;
    g->src_ny = src_ny;
    g->ray_x0 = -0.5 * lix;
    g->ray_y0 = -0.5 * liy;
    g->ray_dx = lix / (double)ray_nx;
    g->ray_dy = liy / (double)ray_ny;
    g->ray_nx = ray_nx;
    g->ray_ny = ray_ny;
    g->scheme = scheme;
    g->precision = scheme == LM_SCHEME_INTERP ? LM_PREC_AUTO : LM_PREC_MIXED;
    g->near_halo = 1;
    g->taylor_terms = 4;
    g->l1_kx = 1;
    g->l1_ky = 1;
    int64_t R = coarse;
    if (scheme == LM_SCHEME_INTERP) {
        // level-1 sides (Eq. 10), with N_star = L_ix L_iy kappa_star / (pi <m>)
        const double l0 = kappa_star > 0 ? std::sqrt(M_PI * mean_mass / kappa_star) : INFINITY;
        const double l1x = std::min(l0, lix / 10.0), l1y = std::min(l0, liy / 10.0);
        if (R <= 0) {  // level-2 = level-1 / 20 (Sec. 3.2.2)
            const double l2 = std::min(l1x / 20.0 / g->ray_dx, l1y / 20.0 / g->ray_dy);
            R = 64 * std::max<int64_t>(1, round_half_away(l2 / 64.0));
        }
        g->l1_kx = (int32_t)std::max<int64_t>(1, round_half_away(l1x / ((double)R * g->ray_dx)));
        g->l1_ky = (int32_t)std::max<int64_t>(1, round_half_away(l1y / ((double)R * g->ray_dy)));
    } else if (R <= 0) {
        R = 64;
    }
    if (R > (1 << 15)) return fail(LM_EINVAL, "level-2 cells of %lld rays are too large", (long long)R);
    g->coarse = (int32_t)R;
    return ok();
}

lm_status lm_geometry_derive_fold(lm_geometry* g, double src_lx, double src_ly, int32_t src_nx,
                                  int32_t src_ny, double kappa0, double d_x, double kappa_star,
                                  double margin, double n_rays, int32_t scheme, int32_t coarse,
                                  double mean_mass)
{
    if (!g) return fail(LM_EINVAL, "g is NULL");
    if (!(isfin(src_lx) && isfin(src_ly) && isfin(kappa0) && isfin(d_x) && isfin(kappa_star) &&
          isfin(margin) && isfin(mean_mass) && isfin(n_rays)))
        return fail(LM_EINVAL, "non-finite input");
    if (!(src_lx > 0 && src_ly > 0) || src_nx <= 0 || src_ny <= 0 || !(d_x > 0) ||
        kappa0 == 1.0 || kappa_star < 0 || !(mean_mass > 0) || !(n_rays >= 1.0))
        return fail(LM_EINVAL, "out-of-domain input");
    if (scheme != LM_SCHEME_DIRECT && scheme != LM_SCHEME_INTERP)
        return fail(LM_EINVAL, "unknown scheme %d", scheme);
    // source window [-w, src_lx] x [-src_ly/2, src_ly/2]; the preimage rectangle
    // of both fold images (Sec. 3.1, Eq. 5)
    const double w = margin < 0 ? 20.0 * std::sqrt(kappa_star) : margin;
    const double lsx = src_lx + w;
    const double lix = 2.0 * std::sqrt(2.0 * lsx / d_x);
    const double liy = src_ly / std::fabs(2.0 * (1.0 - kappa0));
    const double l3 = std::sqrt(lix * liy / n_rays);  // Eq. 11
    const int64_t ray_nx = std::max<int64_t>(1, round_half_away(lix / l3));
    const int64_t ray_ny = std::max<int64_t>(1, round_half_away(liy / l3));
    std::memset(g, 0, sizeof *g);
    g->src_x0 = -w;
    g->src_y0 = -0.5 * src_ly;
    g->src_dx = lsx / src_nx;
    g->src_dy = src_ly / src_ny;
    g->src_nx = src_nx;
    g->src_ny = src_ny;
    g->ray_x0 = -0.5 * lix;
    g->ray_y0 = -0.5 * liy;
    g->ray_dx = lix / (double)ray_nx;
    g->ray_dy = liy / (double)ray_ny;
    g->ray_nx = ray_nx;
    g->ray_ny = ray_ny;
    g->scheme = scheme;
    g->precision = scheme == LM_SCHEME_INTERP ? LM_PREC_AUTO : LM_PREC_MIXED;
    g->near_halo = 1;
    g->taylor_terms = 4;
    g->l1_kx = 1;
    g->l1_ky = 1;
    int64_t R = coarse;
    if (scheme == LM_SCHEME_INTERP) {
        const double l0 = kappa_star > 0 ? std::sqrt(M_PI * mean_mass / kappa_star) : INFINITY;
        const double l1x = std::min(l0, lix / 10.0), l1y = std::min(l0, liy / 10.0);
        if (R <= 0) {
            const double l2 = std::min(l1x / 20.0 / g->ray_dx, l1y / 20.0 / g->ray_dy);
            R = 64 * std::max<int64_t>(1, round_half_away(l2 / 64.0));
        }
        g->l1_kx = (int32_t)std::max<int64_t>(1, round_half_away(l1x / ((double)R * g->ray_dx)));
        g->l1_ky = (int32_t)std::max<int64_t>(1, round_half_away(l1y / ((double)R * g->ray_dy)));
    } else if (R <= 0) {
        R = 64;
    }
    if (R > (1 << 15)) return fail(LM_EINVAL, "level-2 cells of %lld rays are too large", (long long)R);
    g->coarse = (int32_t)R;
    return ok();
}

lm_status lm_geometry_far_order(lm_geometry* g)
{
    if (!g) return fail(LM_EINVAL, "g is NULL");
    g->far_order = 0;
    if (g->scheme != LM_SCHEME_INTERP || g->precision == LM_PREC_FP32)
        return fail(LM_EUNSUPPORTED, "the hierarchical far field needs the interpolated scheme "
                                     "and FP64 coefficients");
    const double rho = far_ratio(*g);
    if (!(rho < 1.0)) return fail(LM_EUNSUPPORTED, "level-1 cells too elongated (ratio %.3f)", rho);
    for (int q = std::max(1, g->taylor_terms); q <= 64; ++q)
        if (std::pow(rho, q) / (1.0 - rho) <= 1e-9) {
            g->far_order = q;
            return ok();
        }
    return fail(LM_EUNSUPPORTED, "no series order up to 64 converges (ratio %.3f)", rho);
}

lm_status lm_create(const lm_geometry* g, lm_map** out)
{
    if (!out) return fail(LM_EINVAL, "out is NULL");
    *out = nullptr;
    lm_status st = validate_geometry(g);
    if (st) return st;
    std::unique_ptr<lm_map> m(new (std::nothrow) lm_map);
    if (!m) return fail(LM_ENOMEM, "out of host memory");
    m->g = *g;
    HIP_TRY(hipGetDevice(&m->device));
    m->ncx = ceil_div(g->ray_nx, g->coarse);
    m->ncy = ceil_div(g->ray_ny, g->coarse);
    if (g->scheme == LM_SCHEME_INTERP) {
        m->n1x = ceil_div(m->ncx, g->l1_kx);
        m->n1y = ceil_div(m->ncy, g->l1_ky);
        if (m->n1x + 2 * g->near_halo > (1 << 20) || m->n1y + 2 * g->near_halo > (1 << 20) ||
            (m->n1x + 2 * g->near_halo) * (m->n1y + 2 * g->near_halo) > (int64_t(1) << 28))
            return fail(LM_EINVAL, "level-1 grid too large");
        m->nl1x = (int)(m->n1x + 2 * g->near_halo);
        m->nl1y = (int)(m->n1y + 2 * g->near_halo);
    }
    const size_t npix = (size_t)g->src_nx * g->src_ny;
    if (m->counts_own.ensure(npix * sizeof(uint64_t)) != hipSuccess)
        return fail(LM_ENOMEM, "cannot allocate %zu counts", npix);
    if (m->n_out.ensure(sizeof(uint64_t)) != hipSuccess) return fail(LM_ENOMEM, "cannot allocate n_out");
    m->counts = m->counts_own.as<uint64_t>();
    LAUNCH_TRY(lm_launch_fill_u64((unsigned long long*)m->counts, (int64_t)npix, 0ull, nullptr));
    LAUNCH_TRY(lm_launch_fill_u64(m->n_out.as<unsigned long long>(), 1, 0ull, nullptr));
    // column offsets of a level-2 cell and their powers, read by the shooting kernels
    const int nptab = g->coarse + LM_PTAB_PAD;
    if (m->ptab.ensure((size_t)LM_PTAB_ROWS * nptab * sizeof(float)) != hipSuccess)
        return fail(LM_ENOMEM, "cannot allocate the column-offset table");
    LAUNCH_TRY(lm_launch_ptab(make_desc(m.get(), 0, 0, 0, 0, Exec{}), m->ptab.as<float>(), nptab,
                              nullptr));
    HIP_TRY(hipStreamSynchronize(nullptr));
    // empty lens set
    st = lm_set_lenses(m.get(), nullptr, nullptr, nullptr, 0);
    if (st) return st;
    *out = m.release();
    return ok();
}

void lm_destroy(lm_map* m)
{
    if (!m) return;
    (void)use_device(m);
    if (m->last) (void)hipStreamSynchronize(m->last);
    (void)hipDeviceSynchronize();
    delete m;
}

lm_status lm_set_macro(lm_map* m, double kappa, double gamma, double kappa_star)
{
    if (!m) return fail(LM_EINVAL, "map is NULL");
    if (!(isfin(kappa) && isfin(gamma) && isfin(kappa_star)))
        return fail(LM_EINVAL, "non-finite macro parameter");
    if (m->has_counts) return fail(LM_ESTATE, "map has counts; call lm_reset_counts first");
    m->kappa = kappa;
    m->gamma = gamma;
    m->kappa_star = kappa_star;
    m->fold = false;
    m->fold_dx = m->fold_dy = 0.0;
    ++m->gen;
    ++m->model_gen;
    if (m->sheet) m->coef_valid = false;  // the sheet's coefficients scale with kappa_star
    return ok();
}

lm_status lm_set_fold(lm_map* m, double kappa0, double d_x, double d_y, double kappa_star)
{
    if (!m) return fail(LM_EINVAL, "map is NULL");
    if (!(isfin(kappa0) && isfin(d_x) && isfin(d_y) && isfin(kappa_star)))
        return fail(LM_EINVAL, "non-finite fold parameter");
    if (m->has_counts) return fail(LM_ESTATE, "map has counts; call lm_reset_counts first");
    m->kappa = kappa0;
    m->gamma = 0.0;
    m->kappa_star = kappa_star;
    m->fold = true;
    m->fold_dx = d_x;
    m->fold_dy = d_y;
    ++m->gen;
    ++m->model_gen;
    if (m->sheet) m->coef_valid = false;  // the sheet's coefficients scale with kappa_star
    return ok();
}

lm_status lm_set_sheet(lm_map* m, double x0, double x1, double y0, double y1)
{
    if (!m) return fail(LM_EINVAL, "map is NULL");
    if (!(isfin(x0) && isfin(x1) && isfin(y0) && isfin(y1)))
        return fail(LM_EINVAL, "non-finite sheet rectangle");
    if (m->has_counts) return fail(LM_ESTATE, "map has counts; call lm_reset_counts first");
    const bool on = !(x0 == 0.0 && x1 == 0.0 && y0 == 0.0 && y1 == 0.0);
    if (on) {
        const lm_geometry& g = m->g;
        if (g.scheme != LM_SCHEME_INTERP)
            return fail(LM_EUNSUPPORTED, "a sheet rectangle needs the interpolated scheme");
        if (!(x1 > x0 && y1 > y0)) return fail(LM_EINVAL, "empty sheet rectangle");
        const double lx1 = g.ray_x0 + (double)g.ray_nx * g.ray_dx;
        const double ly1 = g.ray_y0 + (double)g.ray_ny * g.ray_dy;
        const double tol =
            1e-9 * (std::fabs(g.ray_x0) + std::fabs(lx1) + std::fabs(g.ray_y0) + std::fabs(ly1));
        if (g.ray_x0 < x0 - tol || lx1 > x1 + tol || g.ray_y0 < y0 - tol || ly1 > y1 + tol)
            return fail(LM_EINVAL, "the sheet rectangle must hold the ray lattice");
    }
    m->sheet = on;
    m->sheet_x0 = on ? x0 : 0.0;
    m->sheet_x1 = on ? x1 : 0.0;
    m->sheet_y0 = on ? y0 : 0.0;
    m->sheet_y1 = on ? y1 : 0.0;
    m->coef_valid = false;
    ++m->gen;
    ++m->model_gen;
    return ok();
}

lm_status lm_set_lenses(lm_map* m, const double* x, const double* y, const double* mass, int64_t n)
{
    if (!m) return fail(LM_EINVAL, "map is NULL");
    if (n < 0) return fail(LM_EINVAL, "negative lens count");
    if (n > 0 && (!x || !y || !mass)) return fail(LM_EINVAL, "lens arrays are NULL");
    if (n > (int64_t(1) << 28)) return fail(LM_EINVAL, "too many lenses");
    if (m->has_counts) return fail(LM_ESTATE, "map has counts; call lm_reset_counts first");
    for (int64_t k = 0; k < n; ++k)
        if (!(isfin(x[k]) && isfin(y[k]) && isfin(mass[k]) && mass[k] > 0))
            return fail(LM_EINVAL, "lens %lld has a non-finite position or a non-positive mass",
                        (long long)k);
    lm_status st = use_device(m);
    if (st) return st;
    const lm_geometry& g = m->g;
    std::vector<int64_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::vector<int32_t> I(n, 0), J(n, 0);
    std::vector<int32_t> start;
    if (g.scheme == LM_SCHEME_INTERP) {
        // level-1 cell of each lens (Sec. 3.2.1), same FP64 expression as the
        // lattice definition in lensmap.h
        const int H = g.near_halo;
        const double wx = g.ray_dx * (double)((int64_t)g.coarse * g.l1_kx);
        const double wy = g.ray_dy * (double)((int64_t)g.coarse * g.l1_ky);
        const double lox = -2.0 * H - 2.0, hix = (double)m->n1x + 2.0 * H + 1.0;
        const double loy = -2.0 * H - 2.0, hiy = (double)m->n1y + 2.0 * H + 1.0;
        const int ncell = m->nl1x * m->nl1y;
        std::vector<int64_t> key(n);
        std::vector<int64_t> hist((size_t)ncell + 2, 0);
        for (int64_t k = 0; k < n; ++k) {
            double fi = std::floor((x[k] - g.ray_x0) / wx);
            double fj = std::floor((y[k] - g.ray_y0) / wy);
            fi = std::min(std::max(fi, lox), hix);
            fj = std::min(std::max(fj, loy), hiy);
            I[k] = (int32_t)fi;
            J[k] = (int32_t)fj;
            const bool in = I[k] >= -H && I[k] < m->n1x + H && J[k] >= -H && J[k] < m->n1y + H;
            key[k] = in ? (int64_t)(J[k] + H) * m->nl1x + (I[k] + H) : ncell;
            ++hist[key[k] + 1];
        }
        for (int c = 0; c <= ncell; ++c) hist[c + 1] += hist[c];
        start.assign(hist.begin(), hist.begin() + ncell + 1);
        std::vector<int64_t> pos(hist.begin(), hist.end());
        for (int64_t k = 0; k < n; ++k) order[pos[key[k]]++] = k;  // stable counting sort
    }
    std::vector<double> sx(n), sy(n), sm(n);
    std::vector<float> fx(n), fy(n), fm(n);
    std::vector<int32_t> sI(n), sJ(n);
    for (int64_t t = 0; t < n; ++t) {
        const int64_t k = order[t];
        sx[t] = x[k];
        sy[t] = y[k];
        sm[t] = mass[k];
        fx[t] = (float)x[k];
        fy[t] = (float)y[k];
        fm[t] = (float)mass[k];
        sI[t] = I[k];
        sJ[t] = J[k];
    }
    const size_t nn = (size_t)std::max<int64_t>(n, 1);
    if (m->lx.ensure(nn * 8) || m->ly.ensure(nn * 8) || m->lmd.ensure(nn * 8) ||
        m->lxf.ensure(nn * 4) || m->lyf.ensure(nn * 4) || m->lmf.ensure(nn * 4) ||
        m->lI.ensure(nn * 4) || m->lJ.ensure(nn * 4))
        return fail(LM_ENOMEM, "cannot allocate lens arrays");
    if (n > 0) {
        HIP_TRY(hipMemcpy(m->lx.p, sx.data(), n * 8, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(m->ly.p, sy.data(), n * 8, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(m->lmd.p, sm.data(), n * 8, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(m->lxf.p, fx.data(), n * 4, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(m->lyf.p, fy.data(), n * 4, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(m->lmf.p, fm.data(), n * 4, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(m->lI.p, sI.data(), n * 4, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(m->lJ.p, sJ.data(), n * 4, hipMemcpyHostToDevice));
    }
    if (g.scheme == LM_SCHEME_INTERP) {
        if (m->cell_start.ensure(start.size() * 4))
            return fail(LM_ENOMEM, "cannot allocate the level-1 index");
        HIP_TRY(hipMemcpy(m->cell_start.p, start.data(), start.size() * 4, hipMemcpyHostToDevice));
    }
    m->h_start.swap(start);
    m->nlens = n;
    m->coef_valid = false;
    ++m->gen;
    ++m->model_gen;
    return ok();
}

lm_status lm_bind_counts(lm_map* m, uint64_t* device_counts)
{
    if (!m) return fail(LM_EINVAL, "map is NULL");
    if (device_counts) {
        m->counts = device_counts;
        m->bound = true;
    } else {
        m->counts = m->counts_own.as<uint64_t>();
        m->bound = false;
    }
    m->has_counts = true;  // contents are the caller's
    ++m->gen;
    return ok();
}

lm_status lm_prepare(lm_map* m, void* stream)
{
    if (!m) return fail(LM_EINVAL, "map is NULL");
    lm_status st = use_device(m);
    if (st) return st;
    st = prepare(m, (hipStream_t)stream);
    if (st) return st;
    return ok();
}

lm_status lm_shoot(lm_map* m, int64_t i0, int64_t j0, int64_t ni, int64_t nj, void* stream)
{
    if (!m) return fail(LM_EINVAL, "map is NULL");
    if (ni < 0 || nj < 0 || i0 < 0 || j0 < 0 || i0 > m->g.ray_nx - ni || j0 > m->g.ray_ny - nj)
        return fail(LM_ERANGE, "rectangle [%lld,+%lld) x [%lld,+%lld) leaves the %lld x %lld lattice",
                    (long long)i0, (long long)ni, (long long)j0, (long long)nj,
                    (long long)m->g.ray_nx, (long long)m->g.ray_ny);
    if (ni == 0 || nj == 0) return ok();
    lm_status st = use_device(m);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    if (!m->coef_valid) {
        st = prepare(m, s);
        if (st) return st;
    }
    st = resolve_precision(m, s);
    if (st) return st;
    const int64_t R = m->g.coarse;
    const Exec e = choose_exec(m, (i0 + ni - 1) / R - i0 / R + 1, (j0 + nj - 1) / R - j0 / R + 1, 1,
                               window_bins(m->prec, 0, lanes_nr(m->prec, m->rays_per_lane)));
    LmDesc d = make_desc(m, i0, j0, i0 + ni, j0 + nj, e);
    if (d.ntiles > 0x7fffffffLL) return fail(LM_EUNSUPPORTED, "too many workgroup tiles");
    LAUNCH_TRY(lm_launch_shoot_map(d, m->g.scheme, m->prec, m->g.taylor_terms,
                                   m->rays_per_lane, s));
    m->n_shot += (uint64_t)ni * (uint64_t)nj;
    m->has_counts = true;
    m->last = s;
    return ok();
}

lm_status lm_sync(lm_map* m)
{
    if (!m) return fail(LM_EINVAL, "map is NULL");
    lm_status st = use_device(m);
    if (st) return st;
    HIP_TRY(hipStreamSynchronize(m->last));
    return ok();
}

lm_status lm_read_counts(lm_map* m, uint64_t* host_counts, uint64_t* n_out, uint64_t* n_shot)
{
    if (!m) return fail(LM_EINVAL, "map is NULL");
    lm_status st = use_device(m);
    if (st) return st;
    HIP_TRY(hipStreamSynchronize(m->last));
    HIP_TRY(hipDeviceSynchronize());
    if (host_counts)
        HIP_TRY(hipMemcpy(host_counts, m->counts, (size_t)m->g.src_nx * m->g.src_ny * 8,
                          hipMemcpyDeviceToHost));
    if (n_out) HIP_TRY(hipMemcpy(n_out, m->n_out.p, 8, hipMemcpyDeviceToHost));
    if (n_shot) *n_shot = m->n_shot;
    return ok();
}

lm_status lm_sum_counts(lm_map* m, uint64_t* total)
{
    if (!m || !total) return fail(LM_EINVAL, "map or output is NULL");
    lm_status st = use_device(m);
    if (st) return st;
    HIP_TRY(hipStreamSynchronize(m->last));
    HIP_TRY(hipDeviceSynchronize());
    DevBuf acc;
    if (acc.ensure(8) != hipSuccess) return fail(LM_ENOMEM, "cannot allocate the sum");
    LAUNCH_TRY(lm_launch_fill_u64(acc.as<unsigned long long>(), 1, 0ull, nullptr));
    LAUNCH_TRY(lm_launch_sum_u64(reinterpret_cast<const unsigned long long*>(m->counts),
                                 (int64_t)m->g.src_nx * m->g.src_ny, acc.as<unsigned long long>(),
                                 nullptr));
    HIP_TRY(hipMemcpy(total, acc.p, 8, hipMemcpyDeviceToHost));
    return ok();
}

lm_status lm_read_counts_region(lm_map* m, int32_t p0, int32_t q0, int32_t np, int32_t nq,
                                uint64_t* host_counts)
{
    if (!m) return fail(LM_EINVAL, "map is NULL");
    if (np < 0 || nq < 0 || (np > 0 && nq > 0 && !host_counts)) return fail(LM_EINVAL, "bad arguments");
    if (p0 < 0 || q0 < 0 || p0 > m->g.src_nx - np || q0 > m->g.src_ny - nq)
        return fail(LM_ERANGE, "window leaves the map");
    if (np == 0 || nq == 0) return ok();
    lm_status st = use_device(m);
    if (st) return st;
    // packed on the device, then one contiguous copy
    DevBuf tmp;
    if (tmp.ensure((size_t)np * nq * 8)) return fail(LM_ENOMEM, "cannot allocate the window");
    HIP_TRY(hipStreamSynchronize(m->last));
    HIP_TRY(hipDeviceSynchronize());
    LAUNCH_TRY(lm_launch_copy_region_u64(reinterpret_cast<const unsigned long long*>(m->counts),
                                         m->g.src_nx, p0, q0, np, nq,
                                         tmp.as<unsigned long long>(), nullptr));
    HIP_TRY(hipStreamSynchronize(nullptr));
    HIP_TRY(hipMemcpy(host_counts, tmp.p, (size_t)np * nq * 8, hipMemcpyDeviceToHost));
    return ok();
}

lm_status lm_mu_factor(const lm_map* m, double* factor)
{
    if (!m || !factor) return fail(LM_EINVAL, "NULL argument");
    *factor = (m->g.ray_dx * m->g.ray_dy) / (m->g.src_dx * m->g.src_dy);
    return ok();
}

lm_status lm_read_mu(lm_map* m, double* host_mu)
{
    if (!m || !host_mu) return fail(LM_EINVAL, "NULL argument");
    const size_t npix = (size_t)m->g.src_nx * m->g.src_ny;
    std::vector<uint64_t> c;
    try {
        c.resize(npix);
    } catch (const std::bad_alloc&) {
        return fail(LM_ENOMEM, "cannot allocate %zu host counts", npix);
    }
    lm_status st = lm_read_counts(m, c.data(), nullptr, nullptr);
    if (st) return st;
    double f;
    lm_mu_factor(m, &f);
    for (size_t k = 0; k < npix; ++k) host_mu[k] = (double)c[k] * f;
    return ok();
}

lm_status lm_reset_counts(lm_map* m, void* stream)
{
    if (!m) return fail(LM_EINVAL, "map is NULL");
    lm_status st = use_device(m);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    LAUNCH_TRY(lm_launch_fill_u64((unsigned long long*)m->counts,
                                  (int64_t)m->g.src_nx * m->g.src_ny, 0ull, s));
    LAUNCH_TRY(lm_launch_fill_u64(m->n_out.as<unsigned long long>(), 1, 0ull, s));
    m->n_shot = 0;
    m->has_counts = false;
    m->last = s;
    return ok();
}

lm_status lm_read_coeffs(lm_map* m, int64_t ci, int64_t cj, double* a)
{
    if (!m || !a) return fail(LM_EINVAL, "map or output is NULL");
    if (m->g.scheme != LM_SCHEME_INTERP)
        return fail(LM_EUNSUPPORTED, "the direct scheme has no far-field coefficients");
    if (ci < 0 || cj < 0 || ci >= m->ncx || cj >= m->ncy)
        return fail(LM_ERANGE, "level-2 cell (%lld, %lld) outside the lattice", (long long)ci,
                    (long long)cj);
    lm_status st = use_device(m);
    if (st) return st;
    if (!m->coef_valid) {
        st = prepare(m, nullptr);
        if (st) return st;
    }
    if (m->last) HIP_TRY(hipStreamSynchronize(m->last));
    HIP_TRY(hipDeviceSynchronize());
    LmCoef c;
    HIP_TRY(hipMemcpy(&c, m->coef.as<LmCoef>() + (cj * m->ncx + ci), sizeof c,
                      hipMemcpyDeviceToHost));
    a[0] = c.a0r;
    a[1] = c.a0i;
    for (int n = 1; n < m->g.taylor_terms; ++n) {
        a[2 * n] = (double)c.a[2 * (n - 1)];
        a[2 * n + 1] = (double)c.a[2 * (n - 1) + 1];
    }
    return ok();
}

lm_status lm_deflect(lm_map* m, const double* theta_xy, int64_t n, double* alpha_xy)
{
    if (!m) return fail(LM_EINVAL, "map is NULL");
    if (n < 0 || (n > 0 && (!theta_xy || !alpha_xy))) return fail(LM_EINVAL, "bad arrays");
    if (n >= (int64_t(1) << 30)) return fail(LM_EUNSUPPORTED, "too many probe positions");
    if (n == 0) return ok();
    const lm_geometry& g = m->g;
    const double wx = (double)g.coarse * g.ray_dx * (double)m->ncx;
    const double wy = (double)g.coarse * g.ray_dy * (double)m->ncy;
    for (int64_t t = 0; t < n; ++t) {
        const double tx = theta_xy[2 * t], ty = theta_xy[2 * t + 1];
        if (!(isfin(tx) && isfin(ty))) return fail(LM_EINVAL, "non-finite position %lld", (long long)t);
        if (g.scheme == LM_SCHEME_INTERP &&
            !(tx >= g.ray_x0 && tx < g.ray_x0 + wx && ty >= g.ray_y0 && ty < g.ray_y0 + wy))
            return fail(LM_ERANGE, "position %lld lies outside the level-2 grid", (long long)t);
    }
    lm_status st = use_device(m);
    if (st) return st;
    if (!m->coef_valid) {
        st = prepare(m, nullptr);
        if (st) return st;
    }
    st = resolve_precision(m, nullptr);
    if (st) return st;
    DevBuf dth, dal;
    if (dth.ensure((size_t)n * 16) || dal.ensure((size_t)n * 16))
        return fail(LM_ENOMEM, "cannot allocate probe buffers");
    HIP_TRY(hipStreamSynchronize(m->last));
    HIP_TRY(hipMemcpy(dth.p, theta_xy, (size_t)n * 16, hipMemcpyHostToDevice));
    LmDesc d = make_desc(m, 0, 0, 0, 0, Exec{});
    LAUNCH_TRY(lm_launch_deflect(d, g.scheme, m->prec, g.taylor_terms, dth.as<double>(), n,
                                 dal.as<double>(), nullptr));
    HIP_TRY(hipStreamSynchronize(nullptr));
    HIP_TRY(hipMemcpy(alpha_xy, dal.p, (size_t)n * 16, hipMemcpyDeviceToHost));
    return ok();
}

}  // extern "C"

namespace {

// Pixels (p, q; either may be null) and source positions (beta, 2 per ray, may
// be null) of listed lattice rays, with the shooting kernel's arithmetic.
lm_status trace_rays(lm_map* m, const int64_t* i, const int64_t* j, int64_t n, int32_t* p,
                     int32_t* q, double* beta)
{
    if (!m) return fail(LM_EINVAL, "map is NULL");
    if (n < 0 || (n > 0 && (!i || !j))) return fail(LM_EINVAL, "bad arrays");
    if (n >= (int64_t(1) << 30)) return fail(LM_EUNSUPPORTED, "too many probe rays");
    if (n == 0) return ok();
    for (int64_t t = 0; t < n; ++t)
        if (i[t] < 0 || i[t] >= m->g.ray_nx || j[t] < 0 || j[t] >= m->g.ray_ny)
            return fail(LM_ERANGE, "ray %lld (%lld, %lld) is outside the lattice", (long long)t,
                        (long long)i[t], (long long)j[t]);
    lm_status st = use_device(m);
    if (st) return st;
    if (!m->coef_valid) {
        st = prepare(m, nullptr);
        if (st) return st;
    }
    st = resolve_precision(m, nullptr);
    if (st) return st;
    DevBuf di, dj, dp, dq, duv;
    if (di.ensure((size_t)n * 8) || dj.ensure((size_t)n * 8) || dp.ensure((size_t)n * 4) ||
        dq.ensure((size_t)n * 4) || (beta && duv.ensure((size_t)n * 16)))
        return fail(LM_ENOMEM, "cannot allocate probe buffers");
    HIP_TRY(hipStreamSynchronize(m->last));
    HIP_TRY(hipMemcpy(di.p, i, (size_t)n * 8, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(dj.p, j, (size_t)n * 8, hipMemcpyHostToDevice));
    LmDesc d = make_desc(m, 0, 0, 0, 0, Exec{});
    LAUNCH_TRY(lm_launch_trace(d, m->g.scheme, m->prec, m->g.taylor_terms, di.as<int64_t>(),
                               dj.as<int64_t>(), n, dp.as<int32_t>(), dq.as<int32_t>(),
                               beta ? duv.as<double>() : nullptr, nullptr));
    HIP_TRY(hipStreamSynchronize(nullptr));
    if (p) HIP_TRY(hipMemcpy(p, dp.p, (size_t)n * 4, hipMemcpyDeviceToHost));
    if (q) HIP_TRY(hipMemcpy(q, dq.p, (size_t)n * 4, hipMemcpyDeviceToHost));
    if (beta) {
        HIP_TRY(hipMemcpy(beta, duv.p, (size_t)n * 16, hipMemcpyDeviceToHost));
        // pixel coordinates -> source-plane position (pixel (p, q) starts at
        // src_x0 + p src_dx, src_y0 + q src_dy)
        for (int64_t t = 0; t < n; ++t) {
            beta[2 * t] = m->g.src_x0 + beta[2 * t] * m->g.src_dx;
            beta[2 * t + 1] = m->g.src_y0 + beta[2 * t + 1] * m->g.src_dy;
        }
    }
    return ok();
}

}  // namespace

extern "C" {

lm_status lm_trace(lm_map* m, const int64_t* i, const int64_t* j, int64_t n, int32_t* p, int32_t* q)
{
    if (n > 0 && (!p || !q)) return fail(LM_EINVAL, "bad arrays");
    return trace_rays(m, i, j, n, p, q, nullptr);
}

lm_status lm_trace_beta(lm_map* m, const int64_t* i, const int64_t* j, int64_t n, double* beta_xy)
{
    if (n > 0 && !beta_xy) return fail(LM_EINVAL, "bad arrays");
    return trace_rays(m, i, j, n, nullptr, nullptr, beta_xy);
}

lm_status lm_precision_info(lm_map* m, int32_t* precision, double* mismatch_estimates)
{
    if (!m) return fail(LM_EINVAL, "map is NULL");
    lm_status st = use_device(m);
    if (st) return st;
    st = resolve_precision(m, nullptr);
    if (st) return st;
    if (precision) *precision = m->prec;
    if (mismatch_estimates) {
        mismatch_estimates[0] = m->prec_est;
        mismatch_estimates[1] = m->prec_est_centred;
    }
    return ok();
}

lm_status lm_find_peaks(lm_map* m, const int32_t* tracks, int32_t n_tracks, int32_t k,
                        uint8_t* flags)
{
    if (!m) return fail(LM_EINVAL, "map is NULL");
    if (n_tracks < 0 || (n_tracks > 0 && (!tracks || !flags))) return fail(LM_EINVAL, "bad arrays");
    if (k < 1 || k > 1000) return fail(LM_EINVAL, "k must be in 1..1000");
    if (n_tracks == 0) return ok();
    for (int32_t t = 0; t < n_tracks; ++t)
        if (tracks[t] < 0 || tracks[t] >= m->g.src_ny)
            return fail(LM_ERANGE, "track %d (row %d) is outside the map", t, tracks[t]);
    if ((int64_t)n_tracks * m->g.src_nx >= (int64_t(1) << 31))
        return fail(LM_EUNSUPPORTED, "too many track pixels");
    lm_status st = use_device(m);
    if (st) return st;
    DevBuf dt, df;
    const size_t nf = (size_t)n_tracks * m->g.src_nx;
    if (dt.ensure((size_t)n_tracks * 4) || df.ensure(nf)) return fail(LM_ENOMEM, "cannot allocate");
    HIP_TRY(hipStreamSynchronize(m->last));
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(dt.p, tracks, (size_t)n_tracks * 4, hipMemcpyHostToDevice));
    LAUNCH_TRY(lm_launch_peaks(reinterpret_cast<const unsigned long long*>(m->counts), m->g.src_nx,
                               m->g.src_ny, dt.as<int32_t>(), n_tracks, k, df.as<uint8_t>(),
                               nullptr));
    HIP_TRY(hipStreamSynchronize(nullptr));
    HIP_TRY(hipMemcpy(flags, df.p, nf, hipMemcpyDeviceToHost));
    return ok();
}

}  // extern "C"

namespace {

// Device buffers of one peak-statistics call: tracks (n_tracks int32), the bin
// of every pixel column (src_nx int32), the bin edges (n_bins + 1 doubles) and
// the two histograms (2 n_bins uint64).
struct PeakScratch {
    int32_t* tracks;
    int32_t* bin_of;
    double* edges;
    unsigned long long* hist;
};

lm_status peak_stats_check(lm_map* m, const int32_t* tracks, int32_t n_tracks, int32_t k,
                           const double* beta_edges, int32_t n_bins, const uint64_t* peaks,
                           const uint64_t* heights, const uint64_t* pixels)
{
    if (!m) return fail(LM_EINVAL, "map is NULL");
    if (n_tracks < 0 || n_bins < 1 || n_bins > (1 << 16) || !beta_edges || !peaks || !heights ||
        !pixels || (n_tracks > 0 && !tracks))
        return fail(LM_EINVAL, "bad arguments");
    if (k < 1 || k > 1000) return fail(LM_EINVAL, "k must be in 1..1000");
    for (int32_t b = 0; b <= n_bins; ++b)
        if (!isfin(beta_edges[b]) || (b > 0 && !(beta_edges[b] > beta_edges[b - 1])))
            return fail(LM_EINVAL, "bin edges must be finite and increasing");
    for (int32_t t = 0; t < n_tracks; ++t)
        if (tracks[t] < 0 || tracks[t] >= m->g.src_ny)
            return fail(LM_ERANGE, "track %d (row %d) is outside the map", t, tracks[t]);
    if ((int64_t)n_tracks * m->g.src_nx >= (int64_t(1) << 31))
        return fail(LM_EUNSUPPORTED, "too many track pixels");
    return LM_OK;
}

// The statistics proper, on device buffers the caller provides.  Light-curve
// pixels per bin are counted on the host with the same column centres the
// device bins by; the device does the peak test and the histograms.
lm_status peak_stats_run(lm_map* m, const int32_t* tracks, int32_t n_tracks, int32_t k,
                         const double* beta_edges, int32_t n_bins, uint64_t* peaks,
                         uint64_t* heights, uint64_t* pixels, const PeakScratch& d)
{
    const int64_t nx = m->g.src_nx;
    std::fill(pixels, pixels + n_bins, 0);
    for (int64_t p = 0; p < nx; ++p) {
        const double bc = m->g.src_x0 + ((double)p + 0.5) * m->g.src_dx;
        if (bc >= beta_edges[0] && bc < beta_edges[n_bins]) {
            const int64_t b =
                (std::upper_bound(beta_edges, beta_edges + n_bins + 1, bc) - beta_edges) - 1;
            pixels[b] += (uint64_t)n_tracks;
        }
    }
    std::fill(peaks, peaks + n_bins, 0);
    std::fill(heights, heights + n_bins, 0);
    if (n_tracks == 0) return ok();
    lm_status st = use_device(m);
    if (st) return st;
    HIP_TRY(hipStreamSynchronize(m->last));
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(d.tracks, tracks, (size_t)n_tracks * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(d.edges, beta_edges, (size_t)(n_bins + 1) * 8, hipMemcpyHostToDevice));
    LAUNCH_TRY(lm_launch_column_bins(m->g.src_x0, m->g.src_dx, nx, d.edges, n_bins, d.bin_of,
                                     nullptr));
    LAUNCH_TRY(lm_launch_fill_u64(d.hist, 2 * (int64_t)n_bins, 0ull, nullptr));
    LAUNCH_TRY(lm_launch_peak_bins(reinterpret_cast<const unsigned long long*>(m->counts), nx,
                                   m->g.src_ny, d.tracks, n_tracks, k, d.bin_of, d.hist,
                                   d.hist + n_bins, nullptr));
    HIP_TRY(hipStreamSynchronize(nullptr));
    HIP_TRY(hipMemcpy(peaks, d.hist, (size_t)n_bins * 8, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(heights, d.hist + n_bins, (size_t)n_bins * 8, hipMemcpyDeviceToHost));
    return ok();
}

}  // namespace

extern "C" {

lm_status lm_peak_stats(lm_map* m, const int32_t* tracks, int32_t n_tracks, int32_t k,
                        const double* beta_edges, int32_t n_bins, uint64_t* peaks,
                        uint64_t* heights, uint64_t* pixels)
{
    lm_status st = peak_stats_check(m, tracks, n_tracks, k, beta_edges, n_bins, peaks, heights,
                                    pixels);
    if (st) return st;
    st = use_device(m);
    if (st) return st;
    DevBuf dt, db, de, dh;
    if (dt.ensure((size_t)std::max(n_tracks, 1) * 4) || db.ensure((size_t)m->g.src_nx * 4) ||
        de.ensure((size_t)(n_bins + 1) * 8) || dh.ensure((size_t)n_bins * 16))
        return fail(LM_ENOMEM, "cannot allocate");
    return peak_stats_run(m, tracks, n_tracks, k, beta_edges, n_bins, peaks, heights, pixels,
                          PeakScratch{dt.as<int32_t>(), db.as<int32_t>(), de.as<double>(),
                                      dh.as<unsigned long long>()});
}

lm_status lm_peak_stats_noalloc(lm_map* m, const int32_t* tracks, int32_t n_tracks, int32_t k,
                                const double* beta_edges, int32_t n_bins, uint64_t* peaks,
                                uint64_t* heights, uint64_t* pixels)
{
    lm_status st = peak_stats_check(m, tracks, n_tracks, k, beta_edges, n_bins, peaks, heights,
                                    pixels);
    if (st) return st;
    if (n_tracks > LM_SCRATCH_TRACKS || m->g.src_nx > LM_SCRATCH_COLS || n_bins > LM_SCRATCH_BINS)
        return fail(LM_EINVAL,
                    "lm_peak_stats_noalloc takes at most %d rows, maps of at most %d columns and "
                    "%d bins (got %d rows, %d columns, %d bins)",
                    LM_SCRATCH_TRACKS, LM_SCRATCH_COLS, LM_SCRATCH_BINS, n_tracks, m->g.src_nx,
                    n_bins);
    st = use_device(m);
    if (st) return st;
    void* base = nullptr;
    LAUNCH_TRY(lm_scratch_address(&base));
    unsigned char* s = static_cast<unsigned char*>(base);
    return peak_stats_run(m, tracks, n_tracks, k, beta_edges, n_bins, peaks, heights, pixels,
                          PeakScratch{reinterpret_cast<int32_t*>(s),
                                      reinterpret_cast<int32_t*>(s + LM_SCRATCH_OFF_BINOF),
                                      reinterpret_cast<double*>(s + LM_SCRATCH_OFF_EDGES),
                                      reinterpret_cast<unsigned long long*>(
                                          s + LM_SCRATCH_OFF_HIST)});
}

lm_status lm_fold_scales(double theta_e_arcsec, double d_x, double d_y, double kappa0,
                         double kappa_star, double n_star, double ds_over_r,
                         lm_fold_scales_t* out)
{
    if (!out) return fail(LM_EINVAL, "out is NULL");
    const double in[] = {theta_e_arcsec, d_x, d_y, kappa0, kappa_star, n_star, ds_over_r};
    for (double v : in)
        if (!isfin(v)) return fail(LM_EINVAL, "non-finite input");
    const double dn = std::hypot(d_x, d_y);
    if (!(theta_e_arcsec > 0) || !(dn > 0) || d_x == 0 || !(kappa_star > 0) || !(n_star > 0) ||
        ds_over_r < 0 || kappa0 == 1.0)
        return fail(LM_EINVAL, "out-of-domain input");
    // theta_E |d| is dimensionless once theta_E is in arcmin (d is per arcmin)
    const double kc = std::pow(theta_e_arcsec / 60.0 * dn, 2.0 / 3.0);
    const double sin_a = std::fabs(d_x) / dn;  // tan a = d_x / d_y
    const double r = kappa_star / kc;
    const double cs = std::sqrt(std::log(3.05 * std::sqrt(n_star)));
    out->kappa_c = kc;
    out->sin_a = sin_a;
    out->s_w = 2.0 / sin_a * std::sqrt(kc) * r * r;
    out->c_star = cs;
    out->s_f = cs * std::sqrt(kappa_star);
    out->n_cf = std::sqrt(2.0 * cs / sin_a) * std::pow(r, 0.75);
    const double d_per_rad = dn * (180.0 * 60.0 / M_PI);
    out->mu_peak0 = ds_over_r > 0 ? 1.0 / std::fabs(1.0 - kappa0) *
                                        std::sqrt(ds_over_r / d_per_rad) * std::pow(1.0 / r, 0.75)
                                  : 0.0;
    return ok();
}

lm_status lm_shot_stats(const lm_map* m, int64_t i0, int64_t j0, int64_t ni, int64_t nj,
                        lm_stats* out)
{
    if (!m || !out) return fail(LM_EINVAL, "NULL argument");
    if (ni < 0 || nj < 0 || i0 < 0 || j0 < 0 || i0 > m->g.ray_nx - ni || j0 > m->g.ray_ny - nj)
        return fail(LM_ERANGE, "rectangle leaves the lattice");
    std::memset(out, 0, sizeof *out);
    out->rays = ni * nj;
    if (m->g.scheme != LM_SCHEME_INTERP) {
        out->near_pairs = (double)out->rays * (double)m->nlens;
        return ok();
    }
    const lm_geometry& g = m->g;
    const int64_t sx = (int64_t)g.coarse * g.l1_kx, sy = (int64_t)g.coarse * g.l1_ky;
    double pairs = 0;
    if (ni > 0 && nj > 0)
        for (int64_t J = j0 / sy; J <= (j0 + nj - 1) / sy; ++J) {
            const int64_t ry = std::min(j0 + nj, (J + 1) * sy) - std::max(j0, J * sy);
            for (int64_t I = i0 / sx; I <= (i0 + ni - 1) / sx; ++I) {
                const int64_t rx = std::min(i0 + ni, (I + 1) * sx) - std::max(i0, I * sx);
                pairs += (double)rx * (double)ry * (double)near_count(m, I, J);
            }
        }
    out->near_pairs = pairs;
    out->cells = m->ncx * m->ncy;
    double far = 0;
    for (int64_t J = 0; J < m->n1y; ++J) {
        const int64_t cy = std::min(m->ncy, (J + 1) * (int64_t)g.l1_ky) - J * g.l1_ky;
        for (int64_t I = 0; I < m->n1x; ++I) {
            const int64_t cx = std::min(m->ncx, (I + 1) * (int64_t)g.l1_kx) - I * g.l1_kx;
            far += (double)cx * (double)cy * (double)(m->nlens - near_count(m, I, J));
        }
    }
    out->far_pairs = far;
    return ok();
}

}  // extern "C"

// ==================================================================== batch

// Precision groups of a batch: indexed by the LM_PREC_* value a map's kernels
// run in (LM_PREC_AUTO, 3, is resolved before and never one).
constexpr int kGroups = 5;

// Maps of a batch whose kernels run in one precision (LM_PREC_*): one
// persistent shooting launch over their tiles, fed from its own work counter.
struct BatchGroup {
    int nmaps = 0;
    DevBuf offs, order;
    int64_t total = 0;  // tiles in the queue
    int grid = 0;
};

struct lm_batch {
    std::vector<lm_map*> maps;
    std::vector<int64_t> rect;  // 4 per map: i0, j0, ni, nj
    std::vector<uint64_t> gens; // each map's generation when the graphs were built
    int scheme = 0, terms = 4, device = 0;
    int rays_per_lane = 16, g_scale = 1, wg_per_cu = 0;
    int layout = 0;             // LDS layout of the LM_PREC_MIXED group (others use 0)
    DevBuf descs;               // one LmDesc per map
    BatchGroup grp[kGroups];    // indexed by precision
    DevBuf queue;               // one counter per group
    hipStream_t cap = nullptr;
    // two graphs: every map's coefficients + queue reset, then the persistent
    // shooting kernels; events on the caller's stream bracket both
    hipGraphExec_t exec = nullptr, exec_pre = nullptr;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};  // start, coefficients done, shoot done
    bool launched = false;
    bool dirty = true;
    std::vector<lm_tune_result> tuned;  // candidates timed by the last tuning run
    ~lm_batch()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (exec_pre) (void)hipGraphExecDestroy(exec_pre);
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

namespace {

// LDS layout of the maps that run in precision `prec`: the batch's for the
// FP32 rebased path, layout 0 for the others.
int group_layout(const lm_batch* b, int prec) { return prec == LM_PREC_MIXED ? b->layout : 0; }

// Layouts with instances for this batch's MIXED group at rays_per_lane nr.
bool layout_built(const lm_batch* b, int nr, int layout)
{
    return layout == 0 ||
           (layout > 0 && layout < LM_LAYOUTS && b->scheme == LM_SCHEME_INTERP && b->terms == 4 &&
            (nr == 8 || nr == 16));
}

int device_cus(int dev)
{
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) n = 256;
    return n > 0 ? n : 256;
}

// Build descriptors, cost order and queue offsets of every precision group and
// upload them.  work: the rectangles to shoot (4 per map; the batch's own, or
// a tuning sample); tile sizes always follow the batch's own rectangles, so a
// sample runs with the tiles of the real shot.
lm_status batch_build(lm_batch* b, const std::vector<int64_t>& work)
{
    const int n = (int)b->maps.size();
    for (lm_map* m : b->maps) {
        lm_status st = resolve_precision(m, b->cap);
        if (st) return st;
    }
    std::vector<LmDesc> ds(n);
    std::vector<double> cost(n);
    for (int k = 0; k < n; ++k) {
        lm_map* m = b->maps[k];
        const int64_t* r = &work[4 * k];
        const int64_t* own = &b->rect[4 * k];
        int64_t cx, cy;
        rect_cells(m->g.coarse, own[0], own[1], own[2], own[3], cx, cy);
        const Exec e = choose_exec(
            m, cx, cy, b->g_scale,
            window_bins(m->prec, group_layout(b, m->prec), lanes_nr(m->prec, b->rays_per_lane)));
        ds[k] = make_desc(m, r[0], r[1], r[0] + r[2], r[1] + r[3], e);
        if (r[2] == 0 || r[3] == 0) ds[k].ntiles = 0;
        if (ds[k].ntiles > 0x7fffffffLL)
            return fail(LM_EUNSUPPORTED, "map %d: too many workgroup tiles", k);
        const double lenses = m->g.scheme == LM_SCHEME_INTERP
                                  ? 9.0 * std::max(1.0, (double)m->nlens / std::max<int64_t>(1, m->n1x * m->n1y))
                                  : (double)m->nlens;
        cost[k] = (double)r[2] * (double)r[3] * (20.0 + 6.0 * lenses);
    }
    if (b->descs.ensure(n * sizeof(LmDesc)) || b->queue.ensure(kGroups * 8))
        return fail(LM_ENOMEM, "cannot allocate batch tables");
    HIP_TRY(hipMemcpy(b->descs.p, ds.data(), n * sizeof(LmDesc), hipMemcpyHostToDevice));
    for (int pr = 0; pr < kGroups; ++pr) {
        BatchGroup& G = b->grp[pr];
        std::vector<int32_t> order;
        for (int k = 0; k < n; ++k)
            if (b->maps[k]->prec == pr) order.push_back(k);
        std::stable_sort(order.begin(), order.end(),
                         [&](int a, int c) { return cost[a] > cost[c]; });
        G.nmaps = (int)order.size();
        G.total = 0;
        if (G.nmaps == 0) continue;
        std::vector<int64_t> offs(G.nmaps + 1, 0);
        for (int k = 0; k < G.nmaps; ++k) offs[k + 1] = offs[k] + ds[order[k]].ntiles;
        G.total = offs[G.nmaps];
        if (G.offs.ensure((G.nmaps + 1) * 8) || G.order.ensure(G.nmaps * 4))
            return fail(LM_ENOMEM, "cannot allocate batch tables");
        HIP_TRY(hipMemcpy(G.offs.p, offs.data(), (G.nmaps + 1) * 8, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(G.order.p, order.data(), G.nmaps * 4, hipMemcpyHostToDevice));
        int occ = 0;
        LAUNCH_TRY(lm_shoot_occupancy(b->scheme, pr, b->terms, b->rays_per_lane,
                                      group_layout(b, pr), &occ));
        if (occ <= 0) occ = 1;
        const int wg = b->wg_per_cu > 0 ? std::min(b->wg_per_cu, occ) : occ;
        G.grid = device_cus(b->device) * wg;
    }
    return LM_OK;
}

// Enqueue phase 1 (coefficients of every map when asked, queue reset) and/or
// phase 2 (the persistent shoot of every precision group).
lm_status batch_enqueue(lm_batch* b, hipStream_t s, bool with_coeffs, bool pre = true,
                        bool shoot = true)
{
    const int n = (int)b->maps.size();
    if (pre && with_coeffs)
        for (int k = 0; k < n; ++k) {
            lm_map* m = b->maps[k];
            if (m->g.scheme != LM_SCHEME_INTERP) continue;
            LmDesc d = make_desc(m, 0, 0, 0, 0, Exec{});
            LAUNCH_TRY(launch_coefficients(m, d, s));
        }
    if (pre) LAUNCH_TRY(lm_launch_fill_u64(b->queue.as<unsigned long long>(), kGroups, 0ull, s));
    if (shoot)
        for (int pr = 0; pr < kGroups; ++pr) {
            const BatchGroup& G = b->grp[pr];
            if (G.total <= 0) continue;
            LAUNCH_TRY(lm_launch_shoot_batch(b->descs.as<LmDesc>(), G.offs.as<int64_t>(),
                                             G.order.as<int32_t>(), G.nmaps,
                                             b->queue.as<unsigned long long>() + pr, b->scheme,
                                             pr, b->terms, b->rays_per_lane, group_layout(b, pr),
                                             G.grid, s));
        }
    return LM_OK;
}

lm_status capture(lm_batch* b, bool pre, bool shoot, hipGraphExec_t* out)
{
    hipGraph_t graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    lm_status st = batch_enqueue(b, b->cap, true, pre, shoot);
    hipError_t e = hipStreamEndCapture(b->cap, &graph);
    if (st) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return fail(LM_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(LM_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
    return LM_OK;
}

lm_status batch_graph(lm_batch* b)
{
    for (hipGraphExec_t* e : {&b->exec, &b->exec_pre})
        if (*e) {
            (void)hipGraphExecDestroy(*e);
            *e = nullptr;
        }
    // coefficients (and the precision choice) before the capture: nothing in
    // the capture may synchronise
    for (lm_map* m : b->maps) {
        lm_status st = resolve_precision(m, b->cap);
        if (st) return st;
    }
    HIP_TRY(hipStreamSynchronize(b->cap));
    lm_status st = batch_build(b, b->rect);
    if (st) return st;
    for (hipEvent_t& e : b->ev)
        if (!e) HIP_TRY(hipEventCreate(&e));
    st = capture(b, true, false, &b->exec_pre);
    if (st) return st;
    st = capture(b, false, true, &b->exec);
    if (st) return st;
    b->gens.resize(b->maps.size());
    for (size_t k = 0; k < b->maps.size(); ++k) b->gens[k] = b->maps[k]->gen;
    b->dirty = false;
    return LM_OK;
}

std::string batch_key(const lm_batch* b)
{
    hipDeviceProp_t prop;
    std::string dev = "unknown";
    if (hipGetDeviceProperties(&prop, b->device) == hipSuccess) dev = prop.gcnArchName;
    std::ostringstream k;
    k << dev << "|s" << b->scheme << "t" << b->terms << "|n" << b->maps.size();
    uint64_t h = 1469598103934665603ull;
    for (size_t i = 0; i < b->maps.size(); ++i) {
        const lm_map* m = b->maps[i];
        const int64_t vals[] = {m->g.coarse, m->g.l1_kx, m->g.l1_ky, m->nlens, b->rect[4 * i + 2],
                                b->rect[4 * i + 3], m->g.src_nx, m->g.src_ny, m->prec};
        for (int64_t v : vals) {
            h ^= (uint64_t)v;
            h *= 1099511628211ull;
        }
    }
    k << "|h" << std::hex << h;
    return k.str();
}

// Tuning cache: a text file of "key rays_per_lane tile_scale wg_per_cu
// layout" lines.
bool cache_lookup(const char* path, const std::string& key, int& nr, int& gs, int& wg, int& lay)
{
    if (!path) return false;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string k;
        int a, c, d, e;
        if (is >> k >> a >> c >> d >> e && k == key && lm_supported_rays_per_lane(a) && c >= 1 &&
            d >= 0 && e >= 0 && e < LM_LAYOUTS) {
            nr = a;
            gs = c;
            wg = d;
            lay = e;
            return true;
        }
    }
    return false;
}

void cache_store(const char* path, const std::string& key, int nr, int gs, int wg, int lay)
{
    if (!path) return;
    std::vector<std::string> keep;
    {
        std::ifstream f(path);
        std::string line;
        while (std::getline(f, line))
            if (line.compare(0, key.size() + 1, key + " ") != 0 && !line.empty()) keep.push_back(line);
    }
    std::ofstream f(path, std::ios::trunc);
    for (auto& l : keep) f << l << "\n";
    f << key << " " << nr << " " << gs << " " << wg << " " << lay << "\n";
}

// Rays the tuner times each candidate on: about 2e10 (25 ms at 8e11 rays/s),
// or the whole batch if it is smaller.
constexpr double kTuneRays = 2.0e10;

// The tuning sample of one map: the sub-rectangle of its shot rectangle
// (i0, j0, ni, nj) centred in it, each side scaled by sqrt(fraction) and
// rounded to whole level-2 cells (at least one, at most the side).  It depends
// on nothing but the geometry, the rectangle and the fraction, so every
// candidate of a tuning run shoots the same rays.
void sample_rect(int R, const int64_t* r, double fraction, int64_t* out)
{
    const double f = std::sqrt(std::min(1.0, std::max(0.0, fraction)));
    auto side = [&](int64_t lo, int64_t n, int64_t& slo, int64_t& sn) {
        if (n <= 0) {
            slo = lo;
            sn = 0;
            return;
        }
        int64_t want = (int64_t)std::ceil((double)n * f);
        want = std::max<int64_t>(R, (want + R - 1) / R * R);
        if (want >= n) {
            slo = lo;
            sn = n;
            return;
        }
        // start on a cell boundary near the centre, inside the rectangle
        int64_t s0 = lo + (n - want) / 2;
        s0 = s0 / R * R;
        if (s0 < lo) s0 += R;
        if (s0 + want > lo + n) s0 = lo + n - want;
        slo = s0;
        sn = want;
    };
    side(r[0], r[2], out[0], out[2]);
    side(r[1], r[3], out[1], out[3]);
}

}  // namespace

extern "C" {

lm_status lm_tune_sample(const lm_geometry* g, int64_t i0, int64_t j0, int64_t ni, int64_t nj,
                         double fraction, int32_t tile_scale, int64_t* rect, int64_t* tiles)
{
    lm_status st = validate_geometry(g);
    if (st) return st;
    if (!rect) return fail(LM_EINVAL, "rect is NULL");
    if (!(fraction > 0.0 && fraction <= 1.0)) return fail(LM_EINVAL, "fraction must be in (0, 1]");
    if (tile_scale < 1 || tile_scale > 8) return fail(LM_EINVAL, "tile_scale must be in 1..8");
    if (ni < 0 || nj < 0 || i0 < 0 || j0 < 0 || i0 > g->ray_nx - ni || j0 > g->ray_ny - nj)
        return fail(LM_ERANGE, "rectangle leaves the lattice");
    const int64_t r[4] = {i0, j0, ni, nj};
    sample_rect(g->coarse, r, fraction, rect);
    if (tiles) {
        int64_t cx, cy;
        rect_cells(g->coarse, i0, j0, ni, nj, cx, cy);
        const int G = tile_cells(g->coarse, cx, cy, tile_scale);
        *tiles = 0;
        if (rect[2] > 0 && rect[3] > 0) {
            const int64_t R = g->coarse;
            const int64_t tx = (rect[0] + rect[2] - 1) / R / G - rect[0] / R / G + 1;
            const int64_t ty = (rect[1] + rect[3] - 1) / R / G - rect[1] / R / G + 1;
            *tiles = tx * ty;
        }
    }
    return ok();
}

lm_status lm_batch_create(lm_map* const* maps, int32_t n, lm_batch** out)
{
    if (!out) return fail(LM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!maps || n <= 0) return fail(LM_EINVAL, "a batch needs at least one map");
    std::unique_ptr<lm_batch> b(new (std::nothrow) lm_batch);
    if (!b) return fail(LM_ENOMEM, "out of host memory");
    for (int k = 0; k < n; ++k) {
        lm_map* m = maps[k];
        if (!m) return fail(LM_EINVAL, "map %d is NULL", k);
        if (k == 0) {
            b->scheme = m->g.scheme;
            b->terms = m->g.scheme == LM_SCHEME_INTERP ? m->g.taylor_terms : 1;
            b->device = m->device;
        } else if (m->g.scheme != b->scheme ||
                   (b->scheme == LM_SCHEME_INTERP && m->g.taylor_terms != b->terms) ||
                   m->device != b->device) {
            return fail(LM_EUNSUPPORTED, "map %d differs in scheme, terms or device", k);
        }
        b->maps.push_back(m);
        const int64_t r[4] = {0, 0, m->g.ray_nx, m->g.ray_ny};
        b->rect.insert(b->rect.end(), r, r + 4);
    }
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != b->device) HIP_TRY(hipSetDevice(b->device));
    for (lm_map* m : b->maps) {
        lm_status st = ensure_coef(m);
        if (st) return st;
    }
    HIP_TRY(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    *out = b.release();
    return ok();
}

lm_status lm_batch_set_rect(lm_batch* b, int32_t index, int64_t i0, int64_t j0, int64_t ni, int64_t nj)
{
    if (!b) return fail(LM_EINVAL, "batch is NULL");
    if (index < 0 || index >= (int)b->maps.size()) return fail(LM_ERANGE, "no map %d", index);
    const lm_map* m = b->maps[index];
    if (ni < 0 || nj < 0 || i0 < 0 || j0 < 0 || i0 > m->g.ray_nx - ni || j0 > m->g.ray_ny - nj)
        return fail(LM_ERANGE, "rectangle leaves the lattice of map %d", index);
    int64_t* r = &b->rect[4 * index];
    r[0] = i0;
    r[1] = j0;
    r[2] = ni;
    r[3] = nj;
    b->dirty = true;
    return ok();
}

lm_status lm_batch_shoot(lm_batch* b, void* stream)
{
    if (!b) return fail(LM_EINVAL, "batch is NULL");
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != b->device) HIP_TRY(hipSetDevice(b->device));
    // a member map changed since the graphs were captured: its lens buffers,
    // macro constants or counts pointer in the captured launches are stale
    bool stale = b->gens.size() != b->maps.size();
    for (size_t k = 0; !stale && k < b->maps.size(); ++k) stale = b->gens[k] != b->maps[k]->gen;
    if (b->dirty || !b->exec || stale) {
        lm_status st = batch_graph(b);
        if (st) return st;
    }
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipEventRecord(b->ev[0], s));
    HIP_TRY(hipGraphLaunch(b->exec_pre, s));
    HIP_TRY(hipEventRecord(b->ev[1], s));
    HIP_TRY(hipGraphLaunch(b->exec, s));
    HIP_TRY(hipEventRecord(b->ev[2], s));
    b->launched = true;
    for (size_t k = 0; k < b->maps.size(); ++k) {
        lm_map* m = b->maps[k];
        m->n_shot += (uint64_t)b->rect[4 * k + 2] * (uint64_t)b->rect[4 * k + 3];
        if (b->rect[4 * k + 2] && b->rect[4 * k + 3]) m->has_counts = true;
        m->coef_valid = true;
        m->last = (hipStream_t)stream;
    }
    return ok();
}

lm_status lm_batch_tune(lm_batch* b, const char* cache_path)
{
    if (!b) return fail(LM_EINVAL, "batch is NULL");
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != b->device) HIP_TRY(hipSetDevice(b->device));
    for (lm_map* m : b->maps) {
        lm_status st = resolve_precision(m, b->cap);
        if (st) return st;
    }
    const std::string key = batch_key(b);
    int nr = 0, gs = 0, wg = 0, lay = 0;
    if (!cache_lookup(cache_path, key, nr, gs, wg, lay)) {
        for (lm_map* m : b->maps)
            if (m->has_counts) return fail(LM_ESTATE, "tuning shoots: the maps must have no counts");
        // coefficients once, then every candidate on the same sample of rays
        for (lm_map* m : b->maps) {
            lm_status st = prepare(m, b->cap);
            if (st) return st;
        }
        HIP_TRY(hipStreamSynchronize(b->cap));
        double total = 0.0;
        for (size_t k = 0; k < b->maps.size(); ++k)
            total += (double)b->rect[4 * k + 2] * (double)b->rect[4 * k + 3];
        const double frac = total > kTuneRays ? kTuneRays / total : 1.0;
        std::vector<int64_t> sample(b->rect.size());
        int64_t rays = 0;
        for (size_t k = 0; k < b->maps.size(); ++k) {
            sample_rect(b->maps[k]->g.coarse, &b->rect[4 * k], frac, &sample[4 * k]);
            rays += sample[4 * k + 2] * sample[4 * k + 3];
        }
        hipEvent_t e0, e1;
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        b->tuned.clear();
        double best = 1e300;
        const int nrs[] = {4, 8, 16};
        const int gss[] = {1, 2};
        lm_status st = LM_OK;
        for (int clay = 0; clay < LM_LAYOUTS && !st; ++clay)
            for (int cnr : nrs)
                for (int cgs : gss)
                    for (int cwg : {0, 2}) {
                        if (st || !layout_built(b, cnr, clay)) continue;
                        b->rays_per_lane = cnr;
                        b->g_scale = cgs;
                        b->wg_per_cu = cwg;
                        b->layout = clay;
                        st = batch_build(b, sample);
                        if (!st) st = batch_enqueue(b, b->cap, false);  // warm-up
                        if (st) break;
                        HIP_TRY(hipEventRecord(e0, b->cap));
                        st = batch_enqueue(b, b->cap, false);
                        if (st) break;
                        HIP_TRY(hipEventRecord(e1, b->cap));
                        HIP_TRY(hipEventSynchronize(e1));
                        float ms = 0;
                        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                        lm_tune_result r{cnr, cgs, cwg, clay, rays, ms * 1e-3};
                        b->tuned.push_back(r);
                        if (r.seconds < best) {
                            best = r.seconds;
                            nr = cnr;
                            gs = cgs;
                            wg = cwg;
                            lay = clay;
                        }
                    }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (st) return st;
        cache_store(cache_path, key, nr, gs, wg, lay);
        for (lm_map* m : b->maps) {
            st = lm_reset_counts(m, b->cap);
            if (st) return st;
        }
        HIP_TRY(hipStreamSynchronize(b->cap));
    }
    b->rays_per_lane = nr;
    b->g_scale = gs;
    b->wg_per_cu = wg;
    b->layout = lay;
    b->dirty = true;
    return ok();
}

lm_status lm_batch_tune_results(const lm_batch* b, lm_tune_result* out, int32_t max, int32_t* n)
{
    if (!b || !n || max < 0 || (max > 0 && !out)) return fail(LM_EINVAL, "bad arguments");
    *n = (int32_t)b->tuned.size();
    for (int32_t k = 0; k < std::min<int32_t>(max, *n); ++k) out[k] = b->tuned[k];
    return ok();
}

lm_status lm_batch_timing(lm_batch* b, float* coeff_ms, float* shoot_ms)
{
    if (!b) return fail(LM_EINVAL, "batch is NULL");
    if (!b->launched) return fail(LM_ESTATE, "the batch has not been shot");
    HIP_TRY(hipEventSynchronize(b->ev[2]));
    float a = 0, c = 0;
    HIP_TRY(hipEventElapsedTime(&a, b->ev[0], b->ev[1]));
    HIP_TRY(hipEventElapsedTime(&c, b->ev[1], b->ev[2]));
    if (coeff_ms) *coeff_ms = a;
    if (shoot_ms) *shoot_ms = c;
    return ok();
}

lm_status lm_batch_params(const lm_batch* b, int32_t* rays_per_lane, int32_t* tile_cells,
                          int32_t* wg_per_cu, int32_t* lds_layout)
{
    if (!b) return fail(LM_EINVAL, "batch is NULL");
    if (rays_per_lane) *rays_per_lane = b->rays_per_lane;
    if (tile_cells) *tile_cells = b->g_scale;
    if (wg_per_cu) *wg_per_cu = b->wg_per_cu;
    if (lds_layout) *lds_layout = b->layout;
    return ok();
}

lm_status lm_batch_set_params(lm_batch* b, int32_t rays_per_lane, int32_t tile_cells,
                              int32_t wg_per_cu, int32_t lds_layout)
{
    if (!b) return fail(LM_EINVAL, "batch is NULL");
    if (!lm_supported_rays_per_lane(rays_per_lane))
        return fail(LM_EINVAL, "rays_per_lane must be 4, 8 or 16, got %d", rays_per_lane);
    if (tile_cells < 1 || tile_cells > 8) return fail(LM_EINVAL, "tile_cells must be in 1..8");
    if (wg_per_cu < 0 || wg_per_cu > 8) return fail(LM_EINVAL, "wg_per_cu must be in 0..8");
    if (lds_layout < 0 || lds_layout >= LM_LAYOUTS)
        return fail(LM_EINVAL, "lds_layout must be in 0..%d", LM_LAYOUTS - 1);
    if (!layout_built(b, rays_per_lane, lds_layout))
        return fail(LM_EUNSUPPORTED,
                    "LDS layout %d is built for the interpolated scheme with 4 Taylor terms and 8 "
                    "or 16 rays per lane only",
                    lds_layout);
    b->rays_per_lane = rays_per_lane;
    b->g_scale = tile_cells;
    b->wg_per_cu = wg_per_cu;
    b->layout = lds_layout;
    b->dirty = true;
    return ok();
}

void lm_batch_destroy(lm_batch* b)
{
    if (!b) return;
    int cur = 0;
    if (hipGetDevice(&cur) == hipSuccess && cur != b->device) (void)hipSetDevice(b->device);
    if (b->cap) (void)hipStreamSynchronize(b->cap);
    (void)hipDeviceSynchronize();
    delete b;
}

}  // extern "C"
