// lm_device.h -- device code shared by the gfx950 kernels of liblensmap:
// the per-ray arithmetic of the shooting kernels (k_shoot_map, k_shoot_batch),
// the probes that repeat it ray by ray (k_trace, k_deflect), and the templates
// that launch them.  lm_shoot_inst.hip instantiates them for one (scheme,
// precision) pair per compilation; lm_kernels.hip holds the coefficient
// kernels and the entry points that pick the pair.
//
// Layout of work inside a tile: a wave owns "units" of 64 consecutive rows
// (one ray row per lane) by a run of columns of one level-2 cell; the lane
// walks its row NR columns at a time.  Every ray of a unit shares the cell's
// near-lens list, which the wave stages once in its own LDS slice, so the
// lens loop is uniform and reads lenses as LDS broadcasts.  Quantities that
// are the same for all 64 rows -- the column offsets and their powers (scalar
// loads), and per column and lens dx^2 and m dx (an LDS table the wave fills
// 64 entries at a time) -- are computed once per wave, and the rays of columns
// 2m and 2m+1 share one reciprocal per lens.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "lm_internal.h"

namespace {


constexpr int kWG = LM_WG;

// Lenses staged per wave per block: the direct sum sums 256-lens blocks (the
// compensated blocks); a near list rarely exceeds a few tens of lenses.
template <int SCHEME, int LAY>
struct Cap {
    static constexpr int value = SCHEME == 0 ? LM_LENS_CAP : kLayNear[LAY];
};

// Arithmetic of the ray-lens pairs: FP32 (rebased or plain global) or FP64
// (rebased), and the staged lens record of each.
template <int PREC>
struct Prec {
    using T = float;
    using L = float4;
};
template <>
struct Prec<2> {
    using T = double;
    using L = double4;
};

// The interpolated scheme shares the column-lens differences of a wave through
// an LDS table (kLayTab[LAY] lenses at a time), in every precision: rebased
// FP32 or FP64 offsets, and the plain path's global FP32 coordinates.
template <int SCHEME, int PREC>
struct UseTab {
    static constexpr bool value = SCHEME == 1;
};

// Waves per SIMD the shooting kernels must keep: the FP32 table paths are
// issue-bound and needs 4 (at most 128 VGPRs with 256-thread workgroups, 4 per
// CU).  The per-map kernel, whose descriptor arrives by value, would otherwise
// allocate a few registers more than that and drop to 3; the hint holds it at
// 128 (spilling per-unit values to scratch if it must).  The batch kernel
// carries the same hint, with which the register allocator also schedules
// the plain FP32 form a little tighter.
template <int SCHEME, int PREC>
struct MinWaves {
    static constexpr int value = (SCHEME == 1 && PREC != 2) ? 4 : 1;
};

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int64_t uniform_i64(int64_t v)
{
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(uint64_t)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ unsigned wave_sum_u32(unsigned v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Map constants the per-ray code reads, copied into registers once per unit so
// that the global atomics of the counting step do not force reloads.
struct Hot {
    double inv_sdx, inv_sdy;
    float mxf, myf, bx0f, by0f, inv_sdxf, inv_sdyf, snxf, snyf;
    float qxf, qyf;  // fold: d_x/2, d_y
    int snx, sny, wx, wy;
    unsigned long long* counts;
};

__device__ __forceinline__ Hot make_hot(const LmDesc& d)
{
    Hot h;
    h.inv_sdx = d.inv_sdx;
    h.inv_sdy = d.inv_sdy;
    h.mxf = d.mxf;
    h.myf = d.myf;
    h.qxf = (float)d.qx;
    h.qyf = (float)d.qy;
    h.bx0f = d.bx0f;
    h.by0f = d.by0f;
    h.inv_sdxf = d.inv_sdxf;
    h.inv_sdyf = d.inv_sdyf;
    h.snxf = (float)d.snx;
    h.snyf = (float)d.sny;
    h.snx = d.snx;
    h.sny = d.sny;
    h.wx = d.wx;
    h.wy = d.wy;
    h.counts = d.counts;
    return h;
}

// ---------------------------------------------------------------- cell data

__device__ __forceinline__ double cell_cx(const LmDesc& d, int64_t ci)
{
    return d.x0 + ((double)ci + 0.5) * (double)d.R * d.dx;
}
__device__ __forceinline__ double cell_cy(const LmDesc& d, int64_t cj)
{
    return d.y0 + ((double)cj + 0.5) * (double)d.R * d.dy;
}
__device__ __forceinline__ float cell_cxf(const LmDesc& d, int64_t ci)
{
    return d.x0f + ((float)ci + 0.5f) * (float)d.R * d.dxf;
}
__device__ __forceinline__ float cell_cyf(const LmDesc& d, int64_t cj)
{
    return d.y0f + ((float)cj + 0.5f) * (float)d.R * d.dyf;
}

// FP64 pixel coordinates of the cell centre's image (includes a_0).
template <int SCHEME>
__device__ __forceinline__ void cell_base(const LmDesc& d, int64_t ci, int64_t cj, double& ubx,
                                          double& uby)
{
    const double zx = cell_cx(d, ci), zy = cell_cy(d, cj);
    double bx = d.mx * zx;
    double by = d.my * zy;
    if (d.fold) bx += (d.qx * zx + d.qy * zy) * zx;
    if (SCHEME == 1) {
        const LmCoef& c = d.coef[cj * d.ncx + ci];
        bx -= c.a0r;
        by += c.a0i;
    }
    ubx = (bx - d.bx0) * d.inv_sdx;
    uby = (by - d.by0) * d.inv_sdy;
}

// ----------------------------------------------------------- per-ray pieces

// Every r^2 of the near sums is at least 2^-62 theta_E^2, added to its dx^2
// (in the wave-shared table, once per lens and column) or, without the table,
// to its dy^2: with it the product of two r^2 that two columns share stays a
// normal FP32 number and every FP32 near sum stays finite, whatever the lens
// positions.  It changes r^2 only for rays within ~1e-6 theta_E of a lens's
// column or row, by at most a few ulps, and only rays within ~5e-10 theta_E of
// a lens, deflected far out of any map, materially.
constexpr float kR2Floor = 0x1p-62f;

template <class T>
__device__ __forceinline__ T sq_floor(T v)
{
    return fma(v, v, T(kR2Floor));
}

// One ray-lens pair: accumulates (mx dx, my dy) / r^2 with dx = px - lx, from
// the row's dy^2 and my dy (the weights mx, my differ where the sums are kept
// in pixel units).
__device__ __forceinline__ void pair(float px, float dy2, float mdy, float lxv, float lmx,
                                     float& ax, float& ay)
{
    float dx = px - lxv;
    float r2 = __builtin_fmaf(dx, dx, dy2);
    float w = __builtin_amdgcn_rcpf(r2);
    ax = __builtin_fmaf(dx, lmx * w, ax);
    ay = __builtin_fmaf(mdy, w, ay);
}


// Pair from the wave-shared dx^2 and m dx, dx = px - lx (one per column and
// lens, the same for every row), and the row's dy^2 and m dy.  Every operation
// but the reciprocal is a two-source VOP2 instruction.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }

// FP64 reciprocal: hardware estimate refined by one Newton step.
__device__ __forceinline__ double recip(double x)
{
    const double r0 = __builtin_amdgcn_rcp(x);
    return __builtin_fma(r0, __builtin_fma(-x, r0, 1.0), r0);
}

// FP64 reciprocal to within an ulp or two: two Newton steps from the hardware
// estimate (5 instructions instead of the ~11 of a correctly rounded division).
__device__ __forceinline__ double recip_nr2(double x)
{
    const double r1 = recip(x);
    return __builtin_fma(r1, __builtin_fma(-x, r1, 1.0), r1);
}
__device__ __forceinline__ float recip_nr2(float x) { return 1.0f / x; }

template <class T>
__device__ __forceinline__ void pair_tab(T dx2, T mdx, T dy2, T mdy, T& ax, T& ay)
{
    const T r2 = dx2 + dy2;
    const T w = recip(r2);
    ax = fma(mdx, w, ax);
    ay = fma(mdy, w, ay);
}

// Two pairs of one lens and the row's rays in columns a = 2m and b = 2m + 1
// sharing one reciprocal: 1/r2a = r2b / (r2a r2b) and 1/r2b = r2a / (r2a r2b)
// (the reciprocal is the expensive instruction of a pair).  The product stays a
// normal FP32 number while both r2 exceed 1.1e-19 theta_E^2, which the floor
// kR2Floor on every r2 guarantees, and stay below 1e19.
template <class T>
__device__ __forceinline__ void pair2(T dx2a, T dx2b, T mdxa, T mdxb, T dy2, T mdy, T& axa,
                                      T& aya, T& axb, T& ayb)
{
    const T r2a = dx2a + dy2, r2b = dx2b + dy2;
    const T r = recip(r2a * r2b);
    const T wa = r * r2b, wb = r * r2a;
    axa = fma(mdxa, wa, axa);
    aya = fma(mdy, wa, aya);
    axb = fma(mdxb, wb, axb);
    ayb = fma(mdy, wb, ayb);
}

template <class T>
__device__ __forceinline__ void kahan_add(T& s, T& c, T v)
{
    T y = v - c;
    T t = s + y;
    c = (t - s) - y;
    s = t;
}

// f = sum_{n=1}^{P-1} a_n d^n by Horner, FP32.
template <int P>
__device__ __forceinline__ void taylor(const float* ar, const float* ai, float dx, float dy,
                                       float& fr, float& fi)
{
    if (P <= 1) {
        fr = 0.f;
        fi = 0.f;
        return;
    }
    float gr = ar[P - 1], gi = ai[P - 1];
#pragma unroll
    for (int n = P - 2; n >= 1; --n) {
        float tr = __builtin_fmaf(gr, dx, __builtin_fmaf(-gi, dy, ar[n]));
        float ti = __builtin_fmaf(gr, dy, __builtin_fmaf(gi, dx, ai[n]));
        gr = tr;
        gi = ti;
    }
    fr = __builtin_fmaf(gr, dx, -(gi * dy));
    fi = __builtin_fmaf(gr, dy, gi * dx);
}

// Macro mapping of offsets (dx, dy) from a level-2 cell centre z: the
// constant Jacobian diag(mx, my), or for the fold model the Jacobian at z,
// [[mx + d_x z_x + d_y z_y, d_y z_x], [0, my]], plus the quadratic remainder
// (d_x dx / 2 + d_y dy) dx.  FP32 constants formed in FP64 per cell.
struct CellMap {
    float cxx, cxy, qx, qy;
};

__device__ __forceinline__ CellMap cell_map(const LmDesc& d, double zx, double zy)
{
    CellMap c;
    if (d.fold) {
        c.cxx = (float)(d.mx + 2.0 * d.qx * zx + d.qy * zy);
        c.cxy = (float)(d.qy * zx);
    } else {
        c.cxx = d.mxf;
        c.cxy = 0.f;
    }
    c.qx = (float)d.qx;
    c.qy = (float)d.qy;
    return c;
}

// FP64 pixel y coordinate of the image of a ray row before deflection: the
// cell base plus the macro term of the row's offset l * (L3y / 2) from the cell
// centre, l = 2 (j - cj R) - (R - 1).  Exact offsets here keep the rounding of
// the FP32 offset out of the large macro term.
__device__ __forceinline__ double row_base(const LmDesc& d, double uby, int l)
{
    return __builtin_fma(d.my * ((double)l * (0.5 * d.dy)), d.inv_sdy, uby);
}

// Pixel indices are biased by kBias and converted with saturation (NaN and
// negative values give 0), so the per-ray code needs no range test: index
// p - kBias outside [0, size) means "outside the map", which the count step
// tests once per run of equal pixels.
constexpr unsigned kBias = 1u << 22;
constexpr double kBiasD = 4194304.0;

// Saturating FP64 -> u32 conversion (negative and NaN give 0).
__device__ __forceinline__ unsigned cvt_u32_sat(double v)
{
    unsigned r;
    asm("v_cvt_u32_f64 %0, %1" : "=v"(r) : "v"(v));
    return r;
}

// floor(v) as a 32-bit integer, saturated at the ends of the int32 range (the
// pixel step of the FP32 rebased path, whose sums are finite: see kR2Floor).
__device__ __forceinline__ int cvt_floor_i32_sat(float v)
{
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(v));
    return r;
}

// Degree of the per-row polynomial in the column offset.
template <int P, bool FOLD>
struct Deg {
    static constexpr int value = (P - 1) > (FOLD ? 2 : 1) ? (P - 1) : (FOLD ? 2 : 1);
};

// Far field and macro map of one ray row as polynomials in the column offset dx
// (Sec. 3.2.2 and Eq. 6).  With delta = dx + i dy and f = sum_{n>=1} a_n delta^n,
// gx(dx) = Re f - (macro x displacement) and gy(dx) = -Im f: the x displacement
// of a ray's image is then -(gx + near_x) and its y deflection gy + near_y, so
// the near sums start from gx and gy.  The coefficients come from a Taylor
// shift of f by i dy (synthetic division), once per row.  The constant terms
// gx[0], gy[0] go into the row's FP64 pixel bases (row_setup); per ray the
// rest is summed from the wave-uniform powers of dx (ray_start).  Macro
// constants: Jacobian diag(cxx, .) at the cell centre, cxy = d_y z_x and the
// fold's quadratic remainder (qx dx + qy dy) dx.
template <int P, bool FOLD, class T>
__device__ __forceinline__ void row_poly(const float* ar, const float* ai, T dy, T cxx, T cxy,
                                         T qx, T qy, T* gx, T* gy)
{
    constexpr int D = Deg<P, FOLD>::value;
    T cr[D + 1], cim[D + 1];
#pragma unroll
    for (int k = 0; k <= D; ++k) {
        cr[k] = (k >= 1 && k < P) ? (T)ar[k < P ? k : 0] : T(0);
        cim[k] = (k >= 1 && k < P) ? (T)ai[k < P ? k : 0] : T(0);
    }
    // c_j += (i dy) c_{j+1}, j = N-1 .. k, for k = 0 .. N-1 (N = P - 1)
#pragma unroll
    for (int k = 0; k < P - 1; ++k) {
#pragma unroll
        for (int jj = P - 2; jj >= k; --jj) {
            cr[jj] = fma(-cim[jj + 1], dy, cr[jj]);
            cim[jj] = fma(cr[jj + 1], dy, cim[jj]);
        }
    }
#pragma unroll
    for (int k = 0; k <= D; ++k) {
        gx[k] = cr[k];
        gy[k] = -cim[k];
    }
    if (FOLD) {
        gx[0] = fma(-cxy, dy, gx[0]);
        gx[1] = gx[1] - fma(qy, dy, cxx);
        gx[2] = gx[2] - qx;
    } else {
        gx[1] = gx[1] - cxx;
    }
}

// Powers dx, dx^2, .., dx^D of a column offset, in this order of products
// (the per-cell column table holds the same values).
template <int D, class T>
__device__ __forceinline__ void col_powers(T x, T* pw)
{
    pw[0] = x;
#pragma unroll
    for (int k = 1; k < D; ++k) pw[k] = pw[k - 1] * x;
}

// Biased pixel of one ray of the rebased paths from its sums sx = gx - gx[0] +
// near_x, sy = gy - gy[0] + near_y; ubxb and ubyb are the biased FP64 pixel
// coordinates of the cell centre's image (x) and of the row (y, row_base), each
// with its row polynomial's constant term.
template <class T>
__device__ __forceinline__ void bin_rebased(double inv_sdx, double inv_sdy, double ubxb,
                                            double ubyb, T sx, T sy, unsigned& p, unsigned& q)
{
    const double u = __builtin_fma(-(double)sx, inv_sdx, ubxb);
    const double v = __builtin_fma(-(double)sy, inv_sdy, ubyb);
    p = cvt_u32_sat(u);
    q = cvt_u32_sat(v);
}

// Continuous pixel coordinates (u, v) of one ray in the plain FP32 path
// (global coordinates).
template <int P, bool FOLD>
__device__ __forceinline__ void coords_fp32(const Hot& h, const float* ar, const float* ai,
                                            float a0r, float a0i, float zcx, float zcy, float tx,
                                            float ty, float ax, float ay, float& u, float& v)
{
    float fr, fi;
    float dx = tx - zcx, dy = ty - zcy;
    taylor<P>(ar, ai, dx, dy, fr, fi);
    float alx = ax + (a0r + fr);
    float aly = ay - (a0i + fi);
    float mx = h.mxf;
    if (FOLD) mx = __builtin_fmaf(h.qxf, tx, __builtin_fmaf(h.qyf, ty, mx));
    float bx = __builtin_fmaf(mx, tx, -alx);
    float by = __builtin_fmaf(h.myf, ty, -aly);
    u = (bx - h.bx0f) * h.inv_sdxf;
    v = (by - h.by0f) * h.inv_sdyf;
}

// Pixel of one ray in the plain FP32 path.
template <int P, bool FOLD>
__device__ __forceinline__ void bin_fp32(const Hot& h, const float* ar, const float* ai,
                                         float a0r, float a0i, float zcx, float zcy, float tx,
                                         float ty, float ax, float ay, int& p, int& q)
{
    float u, v;
    coords_fp32<P, FOLD>(h, ar, ai, a0r, a0i, zcx, zcy, tx, ty, ax, ay, u, v);
    bool in = (u >= 0.f) & (u < h.snxf) & (v >= 0.f) & (v < h.snyf);
    p = in ? (int)u : -1;
    q = in ? (int)v : -1;
}

// Offset of lattice index k from the centre of its level-2 cell, as
// (2 (k - c R) - (R - 1)) * (spacing / 2) with the half spacing in float-float.
__device__ __forceinline__ int local_index(int64_t k, int64_t c, int R)
{
    return 2 * (int)(k - c * (int64_t)R) - (R - 1);
}

__device__ __forceinline__ float local_offset(int64_t k, int64_t c, int R, float hh, float hl)
{
    float fl = (float)local_index(k, c, R);
    return __builtin_fmaf(fl, hl, fl * hh);
}

// ------------------------------------------------------------ lens lists

// Level-1 cell (I, J) of level-2 cell (ci, cj).  The interpolated scheme keeps
// fewer than 2^30 level-2 cells, so 32-bit division does (a 64-bit division
// is a long scalar sequence, and this runs once per unit of 64 x R rays).
struct L1Cell {
    int I, J;
};

__device__ __forceinline__ L1Cell l1_of(const LmDesc& d, int64_t ci, int64_t cj)
{
    return L1Cell{(int)ci / d.Kx, (int)cj / d.Ky};
}

// Near-lens rows of level-1 cell c: row r in [0, 2H] is the contiguous sorted
// range [start, end) of level-1 cells (I-H..I+H, J-H+r).
__device__ __forceinline__ void near_row(const LmDesc& d, L1Cell c, int r, int& s, int& e)
{
    int row = c.J + r;  // padded row of J - H + r is (J - H + r) + H
    int base = row * d.nl1x + c.I;  // padded column of I - H is I
    s = d.cell_start[base];
    e = d.cell_start[base + 2 * d.H + 1];
}

template <int SCHEME>
__device__ __forceinline__ int list_count(const LmDesc& d, int64_t ci, int64_t cj)
{
    if (SCHEME == 0) return (int)d.nlens;
    const L1Cell c = l1_of(d, ci, cj);
    int n = 0;
    for (int r = 0; r <= 2 * d.H; ++r) {
        int s, e;
        near_row(d, c, r, s, e);
        n += e - s;
    }
    return n;
}

// Lens value as the per-ray loop sees it: position (x, y) and the weights of
// the x sums (z) and the y sums (w) -- the mass, or with PIX the mass in pixels
// per theta_E of each axis (the rebased FP32 sums then come out in pixels).
// Centred sums: (z, w) = c_k = m_k / delta_k, with PIX in x pixels per theta_E.
template <int PREC, bool PIX = PREC == 0 || PREC == kPrecCentred>
__device__ __forceinline__ typename Prec<PREC>::L lens_value(const LmDesc& d, int idx, double zcx,
                                                            double zcy)
{
    if constexpr (PREC == 2) {
        return make_double4(d.lx[idx] - zcx, d.ly[idx] - zcy, d.lmd[idx], d.lmd[idx]);
    } else if constexpr (PREC == kPrecCentred) {
        // offset delta_k and c_k = m / delta_k (complex) of the centred sums
        const double ox = d.lx[idx] - zcx, oy = d.ly[idx] - zcy;
        const double q = d.lmd[idx] / (ox * ox + oy * oy) * (PIX ? d.inv_sdx : 1.0);
        return make_float4((float)ox, (float)oy, (float)(q * ox), (float)(-(q * oy)));
    } else if constexpr (PREC == 0) {
        const float ox = (float)(d.lx[idx] - zcx), oy = (float)(d.ly[idx] - zcy);
        if constexpr (PIX)
            return make_float4(ox, oy, (float)(d.lmd[idx] * d.inv_sdx),
                               (float)(d.lmd[idx] * d.inv_sdy));
        else
            return make_float4(ox, oy, d.lmf[idx], d.lmf[idx]);
    } else {
        return make_float4(d.lxf[idx], d.lyf[idx], d.lmf[idx], d.lmf[idx]);
    }
}

// Stage list positions [b0, b0+nb) of the cell's lens list into this wave's LDS slice.
template <int SCHEME, int PREC>
__device__ void stage(const LmDesc& d, int64_t ci, int64_t cj, int b0, int nb, double zcx,
                      double zcy, typename Prec<PREC>::L* lb, int lane)
{
    if (SCHEME == 0) {
        for (int s = lane; s < nb; s += 64) lb[s] = lens_value<PREC>(d, b0 + s, zcx, zcy);
    } else {
        const L1Cell c = l1_of(d, ci, cj);
        int off = 0;
        for (int r = 0; r <= 2 * d.H; ++r) {
            int s, e;
            near_row(d, c, r, s, e);
            int lo = max(off, b0), hi = min(off + (e - s), b0 + nb);
            for (int k = lo + lane; k < hi; k += 64)
                lb[k - b0] = lens_value<PREC>(d, s + (k - off), zcx, zcy);
            off += e - s;
        }
    }
    wave_sync_lds();
}

// Global-memory walk over the same list in the same order (probes).
template <int SCHEME>
__device__ __forceinline__ int list_index(const LmDesc& d, int64_t ci, int64_t cj, int pos)
{
    if (SCHEME == 0) return pos;
    const L1Cell c = l1_of(d, ci, cj);
    int off = 0;
    for (int r = 0; r <= 2 * d.H; ++r) {
        int s, e;
        near_row(d, c, r, s, e);
        if (pos < off + (e - s)) return s + (pos - off);
        off += e - s;
    }
    return -1;
}

template <int P>
__device__ __forceinline__ void load_taylor(const LmDesc& d, int64_t ci, int64_t cj, float* ar,
                                            float* ai, float& a0r, float& a0i)
{
    const LmCoef& c = d.coef[cj * d.ncx + ci];
    a0r = (float)c.a0r;
    a0i = (float)c.a0i;
    ar[0] = 0.f;
    ai[0] = 0.f;
#pragma unroll
    for (int n = 1; n < P; ++n) {
        ar[n] = c.a[2 * (n - 1)];
        ai[n] = c.a[2 * (n - 1) + 1];
    }
}

// ------------------------------------------------------------- counting

// A lane's pending run: biased pixel (p, q) as one 64-bit key (one compare per
// ray) and the unit-local column of its first ray; its length is only formed
// when the run is emitted.
struct Run {
    unsigned long long key;  // p | q << 32
    int start;
};

__device__ __forceinline__ unsigned long long run_key(unsigned p, unsigned q)
{
    return (unsigned long long)p | ((unsigned long long)q << 32);
}

// A workgroup's LDS window on the map: biased origin (axb, ayb) and the
// extent (wxe, wye) of its part inside the map (the origin lies in the map).
struct Win {
    unsigned axb, ayb, wxe, wye;
};

// Add n rays at biased pixel (p, q): inside the window's part of the map ->
// LDS, outside the map -> n_out, else a global atomic.
__device__ __forceinline__ void emit(const Hot& h, unsigned p, unsigned q, unsigned n,
                                     const Win& w, unsigned* win, unsigned& nout)
{
    const unsigned wxi = p - w.axb, wyi = q - w.ayb;
    if ((wxi < w.wxe) & (wyi < w.wye)) {
        atomicAdd(&win[__umul24(wyi, (unsigned)h.wx) + wxi], n);
        return;
    }
    const unsigned pm = p - kBias, qm = q - kBias;
    if ((pm >= (unsigned)h.snx) | (qm >= (unsigned)h.sny))
        nout += n;
    else
        atomicAdd(&h.counts[(int64_t)qm * h.snx + pm], (unsigned long long)n);
}

// Lanes whose row lies outside the shot rectangle (row_ok false) keep runs like
// every lane but never emit them, so the per-ray path needs no lane mask.  col
// is the unit-local column of the ray (rays are pushed column by column).
// (p, q) is the pixel less the lane's row base (bx, by), which is the same for
// all of the lane's rays, so runs compare the offsets and a run adds the base
// only when it is emitted.
__device__ __forceinline__ void run_push(const Hot& h, Run& r, unsigned p, unsigned q, int col,
                                         unsigned bx, unsigned by, const Win& w, unsigned* win,
                                         unsigned& nout, bool row_ok)
{
    // (a unit starts with an empty run at an arbitrary key; a run of length 0
    // is never emitted, and one whose rays match that key names their pixel)
    const unsigned long long key = run_key(p, q);
    if (key != r.key) {
        // one divergent region for every lane whose run ends
        const unsigned n = row_ok ? (unsigned)(col - r.start) : 0u;
        if (n) emit(h, (unsigned)r.key + bx, (unsigned)(r.key >> 32) + by, n, w, win, nout);
        r.key = key;
        r.start = col;
    }
}

// End of a unit (col_end = unit-local column after its last ray): lanes whose
// pending runs all name one pixel add it once.
__device__ __forceinline__ void run_flush(const Hot& h, const Run& r, int col_end, unsigned bx,
                                          unsigned by, const Win& w, unsigned* win,
                                          unsigned& nout, int lane, bool row_ok)
{
    const unsigned n = (unsigned)(col_end - r.start);
    const unsigned rp = (unsigned)r.key + bx, rq = (unsigned)(r.key >> 32) + by;
    bool act = row_ok && n > 0;
    unsigned long long am = __ballot(act);
    if (am) {
        int first = __builtin_ctzll(am);
        unsigned p0 = __shfl(rp, first, 64), q0 = __shfl(rq, first, 64);
        unsigned long long diff = __ballot(act && (rp != p0 || rq != q0));
        if (diff == 0) {
            unsigned tot = wave_sum_u32(act ? n : 0u);
            if (lane == first) emit(h, p0, q0, tot, w, win, nout);
        } else if (act) {
            emit(h, rp, rq, n, w, win, nout);
        }
    }
}

// Everything one ray row needs before its rays: the row offset, the biased
// FP64 bases and (rebased paths) the row polynomials.  The rebased FP32 paths
// (plain and centred sums) keep their sums in pixel units: the polynomials
// are scaled to pixels, and each base is split into an integer part (bxi,
// byi: biased pixel indices, as 32-bit integers) and the fraction below it
// (fx, fy), which the sums start from; a ray's pixel is then the integer part
// plus the floor of its FP32 sum, added as integers.
template <int PREC, int P, bool FOLD>
struct Row {
    using T = typename Prec<PREC>::T;
    static constexpr int D = Deg<P, FOLD>::value;
    T py;
    double ubxb, ubyb;
    T gx[D + 1], gy[D + 1];
    unsigned bxi, byi;
    float fx, fy;
    T pyr;  // centred sums: the row offset times sdx / sdy
};

// sdx / sdy in FP32: converts the centred sums' y change from x pixels (the
// unit of their lens weights) to y pixels; one value for the kernels, the
// column table and the probes.
__device__ __forceinline__ float pix_ratio(const LmDesc& d)
{
    return (float)(d.inv_sdy / d.inv_sdx);
}

// Integer part of a biased FP64 pixel coordinate for the integer pixel step,
// and the remainder against it.  The integer part is held within 2^26 pixels
// of any map (maps hold at most 2^30 pixels a side): a row whose base lies
// farther out sends every ray outside the map, since an FP32 sum of more than
// 2^26 pixels has no pixel resolution left.  Within those bounds the base
// plus a floor saturated at the int32 limits stays below 2^32 or, when
// negative, wraps to at least 2^31 - 2^26 + kBias, beyond every map, so no
// result that is not truly in the map lands in it.
__device__ __forceinline__ void split_base(double ub, unsigned& bi, float& f)
{
    constexpr double lo = kBiasD - 67108864.0, hi = kBiasD + 1073741824.0 + 67108864.0;
    const double b = fmin(fmax(floor(ub), lo), hi);
    bi = (unsigned)(int64_t)b;
    f = (float)(ub - b);
}

// Row polynomials to pixel units and the bases split (rebased FP32 paths;
// the centred sums call it after the centre's near deflection is in the
// bases).
template <int PREC, int P, bool FOLD>
__device__ __forceinline__ void row_pixels(const LmDesc& d, Row<PREC, P, FOLD>& rw)
{
    constexpr int D = Row<PREC, P, FOLD>::D;
#pragma unroll
    for (int k = 1; k <= D; ++k) {
        rw.gx[k] = rw.gx[k] * d.inv_sdxf;
        rw.gy[k] = rw.gy[k] * d.inv_sdyf;
    }
    split_base(rw.ubxb, rw.bxi, rw.fx);
    split_base(rw.ubyb, rw.byi, rw.fy);
    if constexpr (PREC == kPrecCentred) rw.pyr = pix_ratio(d) * rw.py;
}

template <int PREC, int P, bool FOLD>
__device__ __forceinline__ void row_setup(const LmDesc& d, int64_t cj, int64_t j, double zcx,
                                          double zcy, double ubx, double uby, const float* ar,
                                          const float* ai, Row<PREC, P, FOLD>& rw)
{
    using T = typename Prec<PREC>::T;
    const int R = d.R;
    if constexpr (PREC == 1) {
        rw.py = __builtin_fmaf((float)j + 0.5f, d.dyf, d.y0f);
        rw.ubxb = 0.0;
        rw.ubyb = 0.0;
    } else {
        const int l = local_index(j, cj, R);
        rw.ubxb = ubx + kBiasD;
        rw.ubyb = row_base(d, uby + kBiasD, l);
        T cxx, cxy, qx, qy;
        if constexpr (PREC == 2) {
            rw.py = (double)l * (0.5 * d.dy);
            cxx = d.fold ? d.mx + 2.0 * d.qx * zcx + d.qy * zcy : d.mx;
            cxy = d.fold ? d.qy * zcx : 0.0;
            qx = d.qx;
            qy = d.qy;
        } else {
            rw.py = local_offset(j, cj, R, d.hyh, d.hyl);
            const CellMap cm = cell_map(d, zcx, zcy);
            cxx = cm.cxx;
            cxy = cm.cxy;
            qx = cm.qx;
            qy = cm.qy;
        }
        row_poly<P, FOLD, T>(ar, ai, rw.py, cxx, cxy, qx, qy, rw.gx, rw.gy);
        rw.ubxb = __builtin_fma(-(double)rw.gx[0], d.inv_sdx, rw.ubxb);
        rw.ubyb = __builtin_fma(-(double)rw.gy[0], d.inv_sdy, rw.ubyb);
        if constexpr (PREC == 0) row_pixels(d, rw);
    }
}

// Column offset of lattice column k in level-2 cell ci (plain path: global).
template <int PREC>
__device__ __forceinline__ typename Prec<PREC>::T column_offset(const LmDesc& d, int64_t k,
                                                                int64_t ci)
{
    if constexpr (PREC == 2)
        return (double)local_index(k, ci, d.R) * (0.5 * d.dx);
    else if constexpr (PREC == 0 || PREC == kPrecCentred)
        return local_offset(k, ci, d.R, d.hxh, d.hxl);
    else
        return __builtin_fmaf((float)k + 0.5f, d.dxf, d.x0f);
}

// Start values of one ray's near sums (rebased paths): the row polynomials
// without their constant terms, g1 dx + g2 dx^2 + .., from the column's powers
// pw[k] = dx^(k+1) (one multiply or FMA and D - 1 FMAs per axis with
// wave-uniform powers); in pixel units (PREC 0) less the bases' fractions
// (the centred sums start with centred_first instead).
// (NEGX, NEGY: ax, ay are the negated sums; every step is an exact negation
// of the plain one, and the negated coefficients need no sign modifier)
template <bool NEGX, bool NEGY, int PREC, int P, bool FOLD>
__device__ __forceinline__ void ray_start_first(const Row<PREC, P, FOLD>& rw,
                                                typename Prec<PREC>::T p1,
                                                typename Prec<PREC>::T& ax,
                                                typename Prec<PREC>::T& ay)
{
    if constexpr (PREC == 0) {
        ax = fma(p1, NEGX ? -rw.gx[1] : rw.gx[1], NEGX ? rw.fx : -rw.fx);
        ay = fma(p1, NEGY ? -rw.gy[1] : rw.gy[1], NEGY ? rw.fy : -rw.fy);
    } else {
        ax = p1 * (NEGX ? -rw.gx[1] : rw.gx[1]);
        ay = p1 * (NEGY ? -rw.gy[1] : rw.gy[1]);
    }
}

// term k + 1 (k >= 1) with pk = dx^(k+1)
template <bool NEGX, bool NEGY, int PREC, int P, bool FOLD>
__device__ __forceinline__ void ray_start_next(const Row<PREC, P, FOLD>& rw, int k,
                                               typename Prec<PREC>::T pk,
                                               typename Prec<PREC>::T& ax,
                                               typename Prec<PREC>::T& ay)
{
    ax = fma(pk, NEGX ? -rw.gx[k + 1] : rw.gx[k + 1], ax);
    ay = fma(pk, NEGY ? -rw.gy[k + 1] : rw.gy[k + 1], ay);
}

template <int PREC, int P, bool FOLD>
__device__ __forceinline__ void ray_start(const Row<PREC, P, FOLD>& rw,
                                          const typename Prec<PREC>::T* pw,
                                          typename Prec<PREC>::T& ax, typename Prec<PREC>::T& ay)
{
    if constexpr (PREC == 1) {
        ax = 0.f;
        ay = 0.f;
    } else {
        constexpr int D = Row<PREC, P, FOLD>::D;
        ray_start_first<false, false, PREC, P, FOLD>(rw, pw[0], ax, ay);
#pragma unroll
        for (int k = 1; k < D; ++k)
            ray_start_next<false, false, PREC, P, FOLD>(rw, k, pw[k], ax, ay);
    }
}

template <int PREC, int P, bool FOLD>
__device__ __forceinline__ void ray_bin(const Hot& h, const Row<PREC, P, FOLD>& rw,
                                        const float* ar, const float* ai, float a0r, float a0i,
                                        float zcxf, float zcyf, typename Prec<PREC>::T px,
                                        typename Prec<PREC>::T ax, typename Prec<PREC>::T ay,
                                        unsigned& p, unsigned& q)
{
    if constexpr (PREC == 1) {
        int pi, qi;
        bin_fp32<P, FOLD>(h, ar, ai, a0r, a0i, zcxf, zcyf, px, rw.py, ax, ay, pi, qi);
        p = pi < 0 ? 0u : (unsigned)pi + kBias;
        q = qi < 0 ? 0u : (unsigned)qi + kBias;
    } else if constexpr (PREC == 0 || PREC == kPrecCentred) {
        // pixel sums (ax, ay) = (image offset less base fraction): the pixel is
        // the base's integer part (row_base_px) plus floor(-sum), added modulo
        // 2^32 (the clamped base and the saturated floor keep every result
        // that is not truly in the map out of it: split_base); here only the
        // floor, the offset from the base
        p = (unsigned)cvt_floor_i32_sat(-ax);
        q = (unsigned)cvt_floor_i32_sat(-ay);
    } else {
        bin_rebased(h.inv_sdx, h.inv_sdy, rw.ubxb, rw.ubyb, ax, ay, p, q);
    }
}

// The row's pixel base that ray_bin's results are offsets from (zero where
// they are the pixels themselves).
template <int PREC, int P, bool FOLD>
__device__ __forceinline__ void row_base_px(const Row<PREC, P, FOLD>& rw, unsigned& bx,
                                            unsigned& by)
{
    if constexpr (PREC == 0 || PREC == kPrecCentred) {
        bx = rw.bxi;
        by = rw.byi;
    } else {
        bx = 0u;
        by = 0u;
    }
}

// --------------------------------------------------------------- units

// Scalar (SMEM) loads of wave-uniform table entries.
typedef const __attribute__((address_space(4))) float* ConstF;

// One lens (row offset dy, mass m; called with dy = y_k - y, so that by holds
// negated y sums) against the NR rays of a lane from its
// table row (dx^2 and m dx per column): pair2 for all columns, staged so that
// the reciprocals issue back to back instead of each right before its use.
template <int NR, class T>
__device__ __forceinline__ void lens_pairs(const T* row, T dy, T m, T* bx, T* by)
{
    const T dy2 = dy * dy;
    const T mdy = m * dy;
    T r2[NR], md[NR], rr[NR / 2];
#pragma unroll
    for (int c = 0; c < NR; ++c) {
        r2[c] = row[c] + dy2;
        md[c] = row[NR + c];
    }
#pragma unroll
    for (int c = 0; c < NR; c += 2) rr[c / 2] = r2[c] * r2[c + 1];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int c = 0; c < NR / 2; ++c) rr[c] = recip(rr[c]);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int c = 0; c < NR; c += 2) {
        const T wa = rr[c / 2] * r2[c + 1], wb = rr[c / 2] * r2[c];
        bx[c] = fma(md[c], wa, bx[c]);
        by[c] = fma(mdy, wa, by[c]);
        bx[c + 1] = fma(md[c + 1], wb, bx[c + 1]);
        by[c + 1] = fma(mdy, wb, by[c + 1]);
    }
}

// Centred near sums.  With delta the ray's offset from the level-2 cell centre
// and delta_k a near lens's, the lens deflects the ray by m (delta - delta_k) /
// |delta - delta_k|^2; as complex numbers its change from the cell centre is
//   conj(that - at the centre) = delta c_k / d_k,  c_k = m / delta_k,
//   d_k = delta - delta_k,
// so the near lenses change the deflection by conj(delta S), S = sum_k c_k /
// d_k = sum_k c_k conj(d_k) / |d_k|^2, while the deflection of the centre
// itself is summed once per cell in FP64 (k_near_centre).  Every FP32 term is
// then small (of order m |delta| / |delta_k|^2 instead of m / |delta_k|), so
// its rounding is too.  One lens (e = y_k - y; the row holds dx^2, c_r dx and
// c_i dx per column) against the NR rays of a lane, two columns sharing one
// reciprocal as in lens_pairs:
//   S_r += (c_r dx - c_i e) w,  S_i += (c_i dx + c_r e) w,  w = 1 / |d|^2.
template <int NR, class T>
__device__ __forceinline__ void lens_pairs_c(const T* row, T e, T cr, T ci, T* sr, T* si)
{
    const T e2 = e * e;
    const T cie = ci * e, cre = cr * e;
    T r2[NR], rr[NR / 2];
#pragma unroll
    for (int c = 0; c < NR; ++c) r2[c] = row[c] + e2;
#pragma unroll
    for (int c = 0; c < NR; c += 2) rr[c / 2] = r2[c] * r2[c + 1];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int c = 0; c < NR / 2; ++c) rr[c] = recip(rr[c]);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int c = 0; c < NR; c += 2) {
        const T wa = rr[c / 2] * r2[c + 1], wb = rr[c / 2] * r2[c];
        sr[c] = fma(row[NR + c] - cie, wa, sr[c]);
        si[c] = fma(row[2 * NR + c] + cre, wa, si[c]);
        sr[c + 1] = fma(row[NR + c + 1] - cie, wb, sr[c + 1]);
        si[c + 1] = fma(row[2 * NR + c + 1] + cre, wb, si[c + 1]);
    }
}

// One centred pair of the probes: the ray's column a, its partner column b
// (the kernel's shared reciprocal) or, unpaired, a reciprocal of its own.
template <bool PAIRED, class T>
__device__ __forceinline__ void pair_c(T dxa, T dxb, T e, T cr, T ci, T& sr, T& si)
{
    const T e2 = e * e;
    const T cie = ci * e, cre = cr * e;
    const T r2a = sq_floor(dxa) + e2;
    T w;
    if constexpr (PAIRED) {
        const T r2b = sq_floor(dxb) + e2;
        w = recip(r2a * r2b) * r2b;
    } else {
        w = recip(r2a);
    }
    sr = fma(cr * dxa - cie, w, sr);
    si = fma(ci * dxa + cre, w, si);
}

// The change conj(delta S) of a ray's near deflection from S (sr, si) at
// column offset px and row offset py: x change dx = Re(delta S), and the
// negated y change dyn = Im(delta S) (the table path's y sums are negated).
template <class T>
__device__ __forceinline__ void centred_change(T px, T py, T sr, T si, T& dx, T& dyn)
{
    dx = fma(px, sr, -(py * si));
    dyn = fma(px, si, py * sr);
}

// First start values of a ray of the centred sums, both negated and in pixel
// units: the change conj(delta S) of the near deflection (S in x pixels; the y
// change converted with px_r = px sdx/sdy and the row's pyr), less the bases'
// fractions, plus the first row-polynomial term.  x: -(Re(delta S) - fx +
// gx1 px); y: Im(delta S) sdx/sdy + fy - gy1 px (the negated y change is
// Im(delta S)).
template <int P, bool FOLD>
__device__ __forceinline__ void centred_first(const Row<kPrecCentred, P, FOLD>& rw, float px,
                                              float pxr, float sr, float si, float& axn,
                                              float& ayn)
{
    const float ndx = fma(-px, sr, fma(rw.py, si, rw.fx));
    const float dyn = fma(pxr, si, fma(rw.pyr, sr, rw.fy));
    axn = fma(px, -rw.gx[1], ndx);
    ayn = fma(px, -rw.gy[1], dyn);
}

// The cell centre's near-lens deflection into a row's FP64 pixel bases.
template <int PREC, int P, bool FOLD>
__device__ __forceinline__ void centre_bases(const LmDesc& d, const LmCoef& cf,
                                             Row<PREC, P, FOLD>& rw)
{
    rw.ubxb = __builtin_fma(-cf.n0x, d.inv_sdx, rw.ubxb);
    rw.ubyb = __builtin_fma(-cf.n0y, d.inv_sdy, rw.ubyb);
}

// Row-polynomial start values of the NR rays of a lane from the wave-uniform
// column powers (scalar loads), one power at a time so that only NR of them
// are live in scalar registers; px gets the column offsets (first powers).
// CENT: ax, ay hold the centred sums S on entry, and the start is added on top
// of their change conj(delta S) (centred_first; the table's row LM_PTAB_POW
// holds the column offsets times sdx / sdy).
template <bool NEGX, bool NEGY, int PREC, int P, bool FOLD, int NR, bool CENT = false>
__device__ __forceinline__ void table_start(ConstF tab, int R, const Row<PREC, P, FOLD>& rw,
                                            typename Prec<PREC>::T* px,
                                            typename Prec<PREC>::T* ax,
                                            typename Prec<PREC>::T* ay)
{
    using T = typename Prec<PREC>::T;
    constexpr int D = Row<PREC, P, FOLD>::D;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int c = 0; c < NR; ++c) {
            const T pk = tab[k * (R + LM_PTAB_PAD) + c];
            if (k == 0) {
                px[c] = pk;
                if constexpr (CENT) {
                    // the centred sums S on entry (ax = S_r, ay = S_i)
                    const T pkr = tab[LM_PTAB_POW * (R + LM_PTAB_PAD) + c];
                    centred_first<P, FOLD>(rw, pk, pkr, ax[c], ay[c], ax[c], ay[c]);
                } else {
                    ray_start_first<NEGX, NEGY, PREC, P, FOLD>(rw, pk, ax[c], ay[c]);
                }
            } else {
                ray_start_next<NEGX, NEGY, PREC, P, FOLD>(rw, k, pk, ax[c], ay[c]);
            }
        }
    }
    __builtin_amdgcn_sched_barrier(0);
}

// Columns [c_lo, c_hi) of cell ci are computed (c_lo even, so columns 2m and
// 2m + 1 share a group); rays of columns >= c_beg are counted.  LAY: the LDS
// layout (near-list block, table block).
template <int SCHEME, int PREC, int NR, int P, bool FOLD, int LAY>
__device__ void process_unit(const LmDesc& d, int64_t ci, int64_t cj, int64_t c_lo, int64_t c_beg,
                             int64_t c_hi, int64_t j, bool row_ok, const Win& w,
                             unsigned* win, typename Prec<PREC>::L* lb,
                             typename Prec<PREC>::T* tb, int lane, unsigned& nout)
{
    using T = typename Prec<PREC>::T;
    constexpr bool CENT = PREC == kPrecCentred;
    const int R = d.R;
    const Hot h = make_hot(d);
    const double zcx = cell_cx(d, ci), zcy = cell_cy(d, cj);
    double ubx, uby;
    cell_base<SCHEME>(d, ci, cj, ubx, uby);
    float ar[P > 1 ? P : 1], ai[P > 1 ? P : 1], a0r = 0.f, a0i = 0.f;
    if (SCHEME == 1) load_taylor<P>(d, ci, cj, ar, ai, a0r, a0i);
    const float zcxf = cell_cxf(d, ci), zcyf = cell_cyf(d, cj);
    const float h_hxh = d.hxh, h_hxl = d.hxl;

    // the lane's ray row
    Row<PREC, P, FOLD> rw;
    row_setup<PREC, P, FOLD>(d, cj, j, zcx, zcy, ubx, uby, ar, ai, rw);
    if constexpr (CENT) {
        centre_bases(d, d.coef[cj * d.ncx + ci], rw);
        row_pixels(d, rw);
    }
    const T py = rw.py;

    constexpr int kCap = Cap<SCHEME, LAY>::value;
    constexpr int kTabCh = kLayTab[LAY];
    const int count = __builtin_amdgcn_readfirstlane(list_count<SCHEME>(d, ci, cj));
    const int nblk = (count + kCap - 1) / kCap;
    if (nblk == 1) stage<SCHEME, PREC>(d, ci, cj, 0, count, zcx, zcy, lb, lane);

    Run run{run_key(kBias - 2, kBias - 2), (int)(c_beg - c_lo)};
    unsigned bxr, byr;
    row_base_px(rw, bxr, byr);
    for (int64_t c0 = c_lo; c0 < c_hi; c0 += NR) {
        constexpr int D = Row<PREC, P, FOLD>::D;
        static_assert(D <= LM_PTAB_POW, "column table holds too few powers");
        // the table path carries the y sums negated (lens offsets y_k - y):
        // the row coefficients -gy and the FP64 binning take the sign for free
        constexpr bool NEGY = UseTab<SCHEME, PREC>::value;
        // and the x sums too; the table of the plain sums holds -m dx for it
        // (the centred sums negate theirs when the start is added)
        constexpr bool NEGX = NEGY;
        constexpr int TW = tab_width(PREC);
        T px[NR], ax[NR], ay[NR], kx[NR], ky[NR];
        if constexpr (CENT) {
            // the sums S start at zero; the row-polynomial start is added after
            // the lenses (table_start on the sums' change)
#pragma unroll
            for (int c = 0; c < NR; ++c) {
                ax[c] = 0;
                ay[c] = 0;
            }
        } else if constexpr (PREC == 0) {
            // wave-uniform column offsets and their powers from the map's table
            table_start<NEGX, NEGY, PREC, P, FOLD, NR>((ConstF)(d.ptab + (c0 - ci * (int64_t)R)),
                                                       R, rw, px, ax, ay);
        } else {
#pragma unroll
            for (int c = 0; c < NR; ++c) {
                T pw[D];
                px[c] = column_offset<PREC>(d, c0 + c, ci);
                col_powers<D>(px[c], pw);
                ray_start<PREC, P, FOLD>(rw, pw, ax[c], ay[c]);
                if (NEGX) ax[c] = -ax[c];
                if (NEGY) ay[c] = -ay[c];
            }
        }
#pragma unroll
        for (int c = 0; c < NR; ++c) {
            kx[c] = 0;
            ky[c] = 0;
        }
        for (int b = 0; b < nblk; ++b) {
            const int nb = __builtin_amdgcn_readfirstlane(min(kCap, count - b * kCap));
            if (nblk > 1) stage<SCHEME, PREC>(d, ci, cj, b * kCap, nb, zcx, zcy, lb, lane);
            T bx[NR], by[NR];
#pragma unroll
            for (int c = 0; c < NR; ++c) {
                bx[c] = SCHEME == 0 ? T(0) : ax[c];
                by[c] = SCHEME == 0 ? T(0) : ay[c];
            }
            if constexpr (UseTab<SCHEME, PREC>::value) {
                // this lane's column in the table build: NR divides 64
                T pxl;
                if constexpr (PREC == 0 || CENT)
                    pxl = local_offset(c0 + (lane & (NR - 1)), ci, R, h_hxh, h_hxl);
                else
                    pxl = column_offset<PREC>(d, c0 + (lane & (NR - 1)), ci);
                for (int k0 = 0; k0 < nb; k0 += kTabCh) {
                    // wave-uniform count: scalar loop control
                    const int nk = __builtin_amdgcn_readfirstlane(min(kTabCh, nb - k0));
                    // tb[k][0..NR) = dx^2, tb[k][NR..2NR) = m dx (centred: c_r dx,
                    // and c_i dx in tb[k][2NR..3NR)), for lenses k0 .. k0+nk
                    for (int e = lane; e < nk * NR; e += 64) {
                        const int k = e / NR, c = e & (NR - 1);
                        const auto L = lb[k0 + k];
                        const T dx = (NEGX && !CENT) ? L.x - pxl : pxl - L.x;
                        tb[k * TW * NR + c] = sq_floor(dx);
                        tb[k * TW * NR + NR + c] = L.z * dx;
                        if constexpr (CENT) tb[k * TW * NR + 2 * NR + c] = L.w * dx;
                    }
                    wave_sync_lds();
                    // two lenses per step: their LDS reads share base addresses
                    int k = 0;
                    for (; k + 2 <= nk; k += 2) {
                        const auto L0 = lb[k0 + k], L1 = lb[k0 + k + 1];
                        if constexpr (CENT) {
                            lens_pairs_c<NR>(tb + k * TW * NR, L0.y - py, L0.z, L0.w, bx, by);
                            lens_pairs_c<NR>(tb + (k + 1) * TW * NR, L1.y - py, L1.z, L1.w, bx,
                                             by);
                        } else {
                            lens_pairs<NR>(tb + k * TW * NR, L0.y - py, L0.w, bx, by);
                            lens_pairs<NR>(tb + (k + 1) * TW * NR, L1.y - py, L1.w, bx, by);
                        }
                    }
                    if (k < nk) {
                        const auto L = lb[k0 + k];
                        if constexpr (CENT)
                            lens_pairs_c<NR>(tb + k * TW * NR, L.y - py, L.z, L.w, bx, by);
                        else
                            lens_pairs<NR>(tb + k * TW * NR, L.y - py, L.w, bx, by);
                    }
                    wave_sync_lds();
                }
            } else {
#pragma unroll 2
                for (int k = 0; k < nb; ++k) {
                    const auto L = lb[k];
                    const T dy = py - L.y;
                    const T dy2 = sq_floor(dy), mdy = L.w * dy;
#pragma unroll
                    for (int c = 0; c < NR; ++c) pair(px[c], dy2, mdy, L.x, L.z, bx[c], by[c]);
                }
            }
#pragma unroll
            for (int c = 0; c < NR; ++c) {
                if (SCHEME == 0) {
                    kahan_add(ax[c], kx[c], bx[c]);
                    kahan_add(ay[c], ky[c], by[c]);
                } else {
                    ax[c] = bx[c];
                    ay[c] = by[c];
                }
            }
            if (nblk > 1) wave_sync_lds();
        }
        if constexpr (CENT) {
            // the change conj(delta S) of the near deflection, then the
            // row-polynomial start on top of it (and the column offsets)
            table_start<NEGX, NEGY, PREC, P, FOLD, NR, true>(
                (ConstF)(d.ptab + (c0 - ci * (int64_t)R)), R, rw, px, ax, ay);
        }
        const int ncol = (int)min((int64_t)NR, c_hi - c0);
        const int cfirst = (int)max((int64_t)0, c_beg - c0);
        const int col0 = (int)(c0 - c_lo);
        if (cfirst == 0 && ncol == NR) {
            // a whole group (every group but a unit's first and last)
#pragma unroll
            for (int c = 0; c < NR; ++c) {
                unsigned p, q;
                ray_bin<PREC, P, FOLD>(h, rw, ar, ai, a0r, a0i, zcxf, zcyf, px[c],
                                       NEGX ? -ax[c] : ax[c], NEGY ? -ay[c] : ay[c], p, q);
                run_push(h, run, p, q, col0 + c, bxr, byr, w, win, nout, row_ok);
            }
        } else {
#pragma unroll
            for (int c = 0; c < NR; ++c) {
                if (c >= cfirst && c < ncol) {
                    unsigned p, q;
                    ray_bin<PREC, P, FOLD>(h, rw, ar, ai, a0r, a0i, zcxf, zcyf, px[c],
                                           NEGX ? -ax[c] : ax[c], NEGY ? -ay[c] : ay[c], p,
                                           q);
                    run_push(h, run, p, q, col0 + c, bxr, byr, w, win, nout, row_ok);
                }
            }
        }
    }
    run_flush(h, run, (int)(c_hi - c_lo), bxr, byr, w, win, nout, lane, row_ok);
}

// Window origin of a tile: the pixel of the image of its centre cell's centre
// (macro map, far field and near lenses, FP64), less half the window, moved
// into the map as far as the window allows (no window bin outside the map is
// ever written, and none of its area is spent outside the map where the
// map allows).
template <int SCHEME>
__device__ __forceinline__ void tile_anchor(const LmDesc& d, int64_t cib, int64_t cjb, int& ax0,
                                            int& ay0)
{
    int64_t cic = min(cib + d.G / 2, d.ncx - 1), cjc = min(cjb + d.G / 2, d.ncy - 1);
    double ubx, uby;
    cell_base<SCHEME>(d, cic, cjc, ubx, uby);
    const double zcx = cell_cx(d, cic), zcy = cell_cy(d, cjc);
    double sx = 0.0, sy = 0.0;
    auto add = [&](int idx) {
        const double dx = zcx - d.lx[idx], dy = zcy - d.ly[idx];
        const double r2 = dx * dx + dy * dy;
        if (r2 > 0.0) {
            const double w = d.lmd[idx] / r2;
            sx += dx * w;
            sy += dy * w;
        }
    };
    // the cell's lens list in list order
    if (SCHEME == 0) {
        for (int k = 0; k < (int)d.nlens; ++k) add(k);
    } else {
        const L1Cell c = l1_of(d, cic, cjc);
        for (int r = 0; r <= 2 * d.H; ++r) {
            int s, e;
            near_row(d, c, r, s, e);
            for (int idx = s; idx < e; ++idx) add(idx);
        }
    }
    ubx -= sx * d.inv_sdx;
    uby -= sy * d.inv_sdy;
    double fx = floor(ubx) - (double)(d.wx / 2), fy = floor(uby) - (double)(d.wy / 2);
    if (fx != fx) fx = 0.0;
    if (fy != fy) fy = 0.0;
    fx = fmin(fmax(fx, 0.0), (double)max(d.snx - d.wx, 0));
    fy = fmin(fmax(fy, 0.0), (double)max(d.sny - d.wy, 0));
    ax0 = (int)fx;
    ay0 = (int)fy;
}

template <int SCHEME, int PREC, int NR, int P, int LAY>
__device__ void process_tile(const LmDesc& d, int64_t t, int ax0, int ay0, unsigned* win,
                             typename Prec<PREC>::L* lb, typename Prec<PREC>::T* tb, int wave,
                             int lane)
{
    const Win w{(unsigned)ax0 + kBias, (unsigned)ay0 + kBias,
                (unsigned)min(d.wx, d.snx - ax0), (unsigned)min(d.wy, d.sny - ay0)};
    // fewer than 2^31 tiles per launch (checked on the host)
    const int ntx = (int)d.ntx;
    const int64_t tx = (int)t % ntx, ty = (int)t / ntx;
    const int64_t cib = (d.tcx0 + tx) * d.G, cjb = (d.tcy0 + ty) * d.G;
    const int per_cell = d.nrb * d.ncc;
    const int U = d.G * d.G * per_cell;
    unsigned nout = 0;
    for (int u = wave; u < U; u += LM_WAVES) {
        const int cu = u / per_cell, rem = u - cu * per_cell;
        const int rb = rem / d.ncc, cc = rem - rb * d.ncc;
        const int64_t ci = cib + cu % d.G, cj = cjb + cu / d.G;
        if (ci >= d.ncx || cj >= d.ncy) continue;
        const int64_t cell_lo = ci * d.R, cell_hi = cell_lo + d.R;
        const int64_t c_beg = max(cell_lo + (int64_t)cc * d.cw, d.i0);
        const int64_t c_hi = min(min(cell_lo + (int64_t)(cc + 1) * d.cw, cell_hi), d.i1);
        const int64_t r_lo = cj * d.R + (int64_t)rb * 64;
        if (c_beg >= c_hi || r_lo + 64 <= d.j0 || r_lo >= d.j1) continue;
        // cells start at even columns (R is a multiple of 64), so c_lo stays in the cell
        const int64_t c_lo = c_beg & ~(int64_t)1;
        const int64_t j = r_lo + lane;
        const bool row_ok = j >= d.j0 && j < d.j1;
        // centred sums: a cell with a near lens close to its centre (n0 NaN,
        // wave-uniform) sums its near lenses plainly
        constexpr int PU = PREC == kPrecCentred ? 0 : PREC;
        if (PREC == kPrecCentred && !__builtin_isnan(d.coef[cj * d.ncx + ci].n0x)) {
            if (d.fold)
                process_unit<SCHEME, PREC, NR, P, true, LAY>(d, ci, cj, c_lo, c_beg, c_hi, j,
                                                             row_ok, w, win, lb, tb, lane, nout);
            else
                process_unit<SCHEME, PREC, NR, P, false, LAY>(d, ci, cj, c_lo, c_beg, c_hi, j,
                                                              row_ok, w, win, lb, tb, lane, nout);
        } else if (d.fold) {
            process_unit<SCHEME, PU, NR, P, true, LAY>(d, ci, cj, c_lo, c_beg, c_hi, j, row_ok, w,
                                                       win, lb, tb, lane, nout);
        } else {
            process_unit<SCHEME, PU, NR, P, false, LAY>(d, ci, cj, c_lo, c_beg, c_hi, j, row_ok, w,
                                                        win, lb, tb, lane, nout);
        }
    }
    unsigned tot = wave_sum_u32(nout);
    if (lane == 0 && tot) atomicAdd(d.n_out, (unsigned long long)tot);
}

__device__ __forceinline__ void flush_window(const LmDesc& d, unsigned* win, int ax0, int ay0,
                                             int tid)
{
    const int n = d.wx * d.wy;
    for (int b = tid; b < n; b += kWG) {
        unsigned v = win[b];
        if (v) {
            int64_t p = (int64_t)ax0 + b % d.wx, q = (int64_t)ay0 + b / d.wx;
            atomicAdd(&d.counts[q * d.snx + p], (unsigned long long)v);
            win[b] = 0u;
        }
    }
}

// ------------------------------------------------------------- kernels

template <int SCHEME, int PREC, int NR, int P>
__global__ __launch_bounds__(kWG)
__attribute__((amdgpu_waves_per_eu(MinWaves<SCHEME, PREC>::value))) void k_shoot_map(LmDesc d)
{
    __shared__ unsigned win[window_bins(PREC, 0, NR)];
    __shared__ typename Prec<PREC>::L lens[LM_WAVES][Cap<SCHEME, 0>::value];
    __shared__ __align__(16) typename Prec<PREC>::T
        tab[LM_WAVES][UseTab<SCHEME, PREC>::value ? kLayTab[0] * tab_width(PREC) * NR : 1];
    const int tid = threadIdx.x, lane = tid & 63;
    // wave index as a scalar: everything derived from it stays uniform
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t t = d.tile0 + blockIdx.x;
    for (int b = tid; b < d.wx * d.wy; b += kWG) win[b] = 0u;
    // fewer than 2^31 tiles per map (checked on the host)
    const int64_t tx = (int)t % (int)d.ntx, ty = (int)t / (int)d.ntx;
    int ax0, ay0;
    tile_anchor<SCHEME>(d, (d.tcx0 + tx) * d.G, (d.tcy0 + ty) * d.G, ax0, ay0);
    __syncthreads();
    process_tile<SCHEME, PREC, NR, P, 0>(d, t, ax0, ay0, win, lens[wave], tab[wave], wave, lane);
    __syncthreads();
    flush_window(d, win, ax0, ay0, tid);
}

template <int SCHEME, int PREC, int NR, int P, int LAY>
__global__ __launch_bounds__(kWG)
__attribute__((amdgpu_waves_per_eu(MinWaves<SCHEME, PREC>::value))) void k_shoot_batch(const LmDesc* __restrict__ descs,
                                                     const int64_t* __restrict__ offs,
                                                     const int32_t* __restrict__ order, int nmaps,
                                                     unsigned long long* queue)
{
    __shared__ unsigned win[window_bins(PREC, LAY, NR)];
    __shared__ typename Prec<PREC>::L lens[LM_WAVES][Cap<SCHEME, LAY>::value];
    __shared__ __align__(16) typename Prec<PREC>::T
        tab[LM_WAVES][UseTab<SCHEME, PREC>::value ? kLayTab[LAY] * tab_width(PREC) * NR : 1];
    __shared__ long long s_item;
    const int tid = threadIdx.x, lane = tid & 63;
    // wave index as a scalar: everything derived from it stays uniform
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    for (int b = tid; b < window_bins(PREC, LAY, NR); b += kWG) win[b] = 0u;
    const int64_t total = offs[nmaps];
    for (;;) {
        if (tid == 0) s_item = (long long)atomicAdd(queue, 1ull);
        __syncthreads();
        const int64_t item = uniform_i64(s_item);
        __syncthreads();
        if (item >= total) break;
        int lo = 0, hi = nmaps - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (offs[mid] <= item)
                lo = mid;
            else
                hi = mid - 1;
        }
        const LmDesc& d = descs[order[lo]];
        const int64_t t = item - offs[lo];
        // fewer than 2^31 tiles per map (checked on the host)
        const int64_t tx = (int)t % (int)d.ntx, ty = (int)t / (int)d.ntx;
        int ax0, ay0;
        tile_anchor<SCHEME>(d, (d.tcx0 + tx) * d.G, (d.tcy0 + ty) * d.G, ax0, ay0);
        process_tile<SCHEME, PREC, NR, P, LAY>(d, t, ax0, ay0, win, lens[wave], tab[wave], wave,
                                               lane);
        __syncthreads();
        flush_window(d, win, ax0, ay0, tid);
        __syncthreads();
    }
}

// Near-field sum of one position (lens for lens as in the shooting kernel),
// added to the start values ax, ay.
// PAIRED: the shooting kernel's two-column reciprocal, pxp = offset of the
// partner column (column index ^ 1).  PIX: weights in pixel units, as the
// rebased FP32 shooting path sums (else in theta_E).
template <int SCHEME, int PREC, bool PAIRED = false,
          bool PIX = PREC == 0 || PREC == kPrecCentred>
__device__ void near_sum(const LmDesc& d, int64_t ci, int64_t cj, double zcx, double zcy,
                         typename Prec<PREC>::T px, typename Prec<PREC>::T py,
                         typename Prec<PREC>::T& ax, typename Prec<PREC>::T& ay,
                         typename Prec<PREC>::T pxp = 0)
{
    using T = typename Prec<PREC>::T;
    constexpr int kCap = Cap<SCHEME, 0>::value;
    const int count = list_count<SCHEME>(d, ci, cj);
    if constexpr (PREC == kPrecCentred) {
        // the centred sums S over the list in list order (ax, ay get S)
        T sr = 0, si = 0;
        for (int k = 0; k < count; ++k) {
            const auto L = lens_value<PREC, PIX>(d, list_index<SCHEME>(d, ci, cj, k), zcx, zcy);
            pair_c<PAIRED>(px - L.x, pxp - L.x, L.y - py, L.z, L.w, sr, si);
        }
        ax = sr;
        ay = si;
        return;
    }
    T kx = 0, ky = 0;
    for (int b0 = 0; b0 < count; b0 += kCap) {
        const int nb = min(kCap, count - b0);
        T bx = SCHEME == 0 ? T(0) : ax, by = SCHEME == 0 ? T(0) : ay;
        for (int k = 0; k < nb; ++k) {
            const auto L =
                lens_value<PREC, PIX>(d, list_index<SCHEME>(d, ci, cj, b0 + k), zcx, zcy);
            const T dy = py - L.y;
            if constexpr (UseTab<SCHEME, PREC>::value && PAIRED) {
                const T dx = px - L.x, dxp = pxp - L.x;
                T ayp = 0, axp = 0;
                pair2(sq_floor(dx), sq_floor(dxp), L.z * dx, L.z * dxp, dy * dy, L.w * dy, bx, by,
                      axp, ayp);
            } else if constexpr (UseTab<SCHEME, PREC>::value) {
                const T dx = px - L.x;
                pair_tab(sq_floor(dx), L.z * dx, dy * dy, L.w * dy, bx, by);
            } else {
                pair(px, sq_floor(dy), L.w * dy, L.x, L.z, bx, by);
            }
        }
        if (SCHEME == 0) {
            kahan_add(ax, kx, bx);
            kahan_add(ay, ky, by);
        } else {
            ax = bx;
            ay = by;
        }
    }
}

// Per-ray pixels with the shooting kernel's arithmetic, lens for lens, and the
// continuous pixel coordinates (u, v) the pixel is the floor of (uv non-null).
template <int SCHEME, int PREC, int P, bool FOLD>
__device__ void trace_one(const LmDesc& d, int64_t i, int64_t j, int32_t& po, int32_t& qo,
                          double* uv)
{
    using T = typename Prec<PREC>::T;
    const int R = d.R;
    const int64_t ci = i / R, cj = j / R;
    if constexpr (PREC == kPrecCentred) {
        if (__builtin_isnan(d.coef[cj * d.ncx + ci].n0x)) {  // as the kernel: plain sums
            trace_one<SCHEME, 0, P, FOLD>(d, i, j, po, qo, uv);
            return;
        }
    }
    const double zcx = cell_cx(d, ci), zcy = cell_cy(d, cj);
    double ubx, uby;
    cell_base<SCHEME>(d, ci, cj, ubx, uby);
    float ar[P > 1 ? P : 1], ai[P > 1 ? P : 1], a0r = 0.f, a0i = 0.f;
    if (SCHEME == 1) load_taylor<P>(d, ci, cj, ar, ai, a0r, a0i);
    Row<PREC, P, FOLD> rw;
    row_setup<PREC, P, FOLD>(d, cj, j, zcx, zcy, ubx, uby, ar, ai, rw);
    if constexpr (PREC == kPrecCentred) {
        centre_bases(d, d.coef[cj * d.ncx + ci], rw);
        row_pixels(d, rw);
    }
    const T px = column_offset<PREC>(d, i, ci);
    constexpr int D = Row<PREC, P, FOLD>::D;
    T pw[D], ax, ay;
    col_powers<D>(px, pw);
    if constexpr (PREC == kPrecCentred) {
        // as the kernel: S, then the start on its change, both sums negated
        T sr, si;
        near_sum<SCHEME, PREC, true>(d, ci, cj, zcx, zcy, px, rw.py, sr, si,
                                     column_offset<PREC>(d, i ^ 1, ci));
        centred_first<P, FOLD>(rw, px, pix_ratio(d) * px, sr, si, ax, ay);
#pragma unroll
        for (int k = 1; k < D; ++k)
            ray_start_next<true, true, PREC, P, FOLD>(rw, k, pw[k], ax, ay);
        ax = -ax;
        ay = -ay;
    } else {
        ray_start<PREC, P, FOLD>(rw, pw, ax, ay);
        near_sum<SCHEME, PREC, true>(d, ci, cj, zcx, zcy, px, rw.py, ax, ay,
                                     column_offset<PREC>(d, i ^ 1, ci));
    }
    const Hot h = make_hot(d);
    unsigned p, q;
    ray_bin<PREC, P, FOLD>(h, rw, ar, ai, a0r, a0i, cell_cxf(d, ci), cell_cyf(d, cj), px, ax, ay, p,
                           q);
    unsigned bxr, byr;
    row_base_px(rw, bxr, byr);
    p += bxr;
    q += byr;
    const unsigned pm = p - kBias, qm = q - kBias;
    const bool in = (pm < (unsigned)d.snx) & (qm < (unsigned)d.sny);
    po = in ? (int32_t)pm : -1;
    qo = in ? (int32_t)qm : -1;
    if (uv) {
        if constexpr (PREC == 1) {
            float u, v;
            coords_fp32<P, FOLD>(h, ar, ai, a0r, a0i, cell_cxf(d, ci), cell_cyf(d, cj), px, rw.py,
                                 ax, ay, u, v);
            uv[0] = u;
            uv[1] = v;
        } else if constexpr (PREC == 0 || PREC == kPrecCentred) {
            // the values whose floors ray_bin forms, less the bias
            uv[0] = ((double)(int)rw.bxi - kBiasD) - (double)ax;
            uv[1] = ((double)(int)rw.byi - kBiasD) - (double)ay;
        } else {
            // the FP64 values bin_rebased floors, less the bias
            uv[0] = __builtin_fma(-(double)ax, h.inv_sdx, rw.ubxb) - kBiasD;
            uv[1] = __builtin_fma(-(double)ay, h.inv_sdy, rw.ubyb) - kBiasD;
        }
    }
}

template <int SCHEME, int PREC, int P>
__global__ __launch_bounds__(kWG) void k_trace(LmDesc d, const int64_t* __restrict__ ii,
                                               const int64_t* __restrict__ jj, int64_t n,
                                               int32_t* __restrict__ po, int32_t* __restrict__ qo,
                                               double* __restrict__ uv)
{
    const int64_t t = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (t >= n) return;
    double* u = uv ? uv + 2 * t : nullptr;
    if (d.fold)
        trace_one<SCHEME, PREC, P, true>(d, ii[t], jj[t], po[t], qo[t], u);
    else
        trace_one<SCHEME, PREC, P, false>(d, ii[t], jj[t], po[t], qo[t], u);
}

// Deflection at an arbitrary position, rebased on the level-2 cell holding it.
template <int SCHEME, int PREC, int P>
__device__ void deflect_one(const LmDesc& d, double tx, double ty, double& outx, double& outy)
{
    using T = typename Prec<PREC>::T;
    const int64_t ci = (int64_t)floor((tx - d.x0) / ((double)d.R * d.dx));
    const int64_t cj = (int64_t)floor((ty - d.y0) / ((double)d.R * d.dy));
    if constexpr (PREC == kPrecCentred) {
        if (__builtin_isnan(d.coef[cj * d.ncx + ci].n0x)) {  // plain sums for this cell
            deflect_one<SCHEME, 0, P>(d, tx, ty, outx, outy);
            return;
        }
    }
    const double zcx = cell_cx(d, ci), zcy = cell_cy(d, cj);
    float ar[P > 1 ? P : 1], ai[P > 1 ? P : 1], a0r = 0.f, a0i = 0.f;
    if (SCHEME == 1) load_taylor<P>(d, ci, cj, ar, ai, a0r, a0i);
    T px, py;
    if (PREC != 1) {
        px = (T)(tx - zcx);
        py = (T)(ty - zcy);
    } else {
        px = (float)tx;
        py = (float)ty;
    }
    T ax = 0, ay = 0;
    near_sum<SCHEME, PREC, false, false>(d, ci, cj, zcx, zcy, px, py, ax, ay);
    if constexpr (PREC == kPrecCentred) {
        T dx, dyn;
        centred_change(px, py, ax, ay, dx, dyn);
        ax = dx;
        ay = -dyn;
    }
    outx = ax;
    outy = ay;
    if (SCHEME == 1) {
        float fr, fi, dx, dy;
        if (PREC != 1) {
            dx = (float)px;
            dy = (float)py;
        } else {
            dx = (float)px - cell_cxf(d, ci);
            dy = (float)py - cell_cyf(d, cj);
        }
        taylor<P>(ar, ai, dx, dy, fr, fi);
        if (PREC != 1) {
            const LmCoef& c = d.coef[cj * d.ncx + ci];
            outx = (double)ax + (double)fr + c.a0r;
            outy = (double)ay - (double)fi - c.a0i;
            if constexpr (PREC == kPrecCentred) {
                // the centred sums hold the change from the centre's near deflection
                outx += c.n0x;
                outy += c.n0y;
            }
        } else {
            outx = (double)(ax + (a0r + fr));
            outy = (double)(ay - (a0i + fi));
        }
    }
}

template <int SCHEME, int PREC, int P>
__global__ __launch_bounds__(kWG) void k_deflect(LmDesc d, const double* __restrict__ th,
                                                 int64_t n, double* __restrict__ al)
{
    const int64_t t = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (t >= n) return;
    deflect_one<SCHEME, PREC, P>(d, th[2 * t], th[2 * t + 1], al[2 * t], al[2 * t + 1]);
}

// ------------------------------------------------------------ dispatch

// Grids stay below 2^22 workgroups (2^30 work-items) per launch.
constexpr int64_t kMaxGrid = int64_t(1) << 22;

template <int S, int PR, int NR, int P>
int launch_map_t(const LmDesc& d0, hipStream_t s)
{
    LmDesc d = d0;
    for (int64_t t0 = 0; t0 < d0.ntiles; t0 += kMaxGrid) {
        d.tile0 = t0;
        const int64_t n = d0.ntiles - t0 < kMaxGrid ? d0.ntiles - t0 : kMaxGrid;
        hipLaunchKernelGGL((k_shoot_map<S, PR, NR, P>), dim3((unsigned)n), dim3(kWG), 0, s, d);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return (int)e;
    }
    return 0;
}

template <int S, int PR, int NR, int P, int LAY>
int launch_batch_t(const LmDesc* descs, const int64_t* offs, const int32_t* order, int nmaps,
                   unsigned long long* queue, int grid, hipStream_t s)
{
    hipLaunchKernelGGL((k_shoot_batch<S, PR, NR, P, LAY>), dim3(grid), dim3(kWG), 0, s, descs,
                       offs, order, nmaps, queue);
    return (int)hipGetLastError();
}

template <int S, int PR, int NR, int P, int LAY>
const void* kernel_ptr_t()
{
    return (const void*)&k_shoot_batch<S, PR, NR, P, LAY>;
}

// The LDS layouts built for (S, PR, NR, P): every one for the FP32 rebased
// path with P = 4 and 8 or 16 rays per lane, layout 0 for the rest.
template <int S, int PR, int NR, int P>
struct HasLayouts {
    static constexpr bool value = S == 1 && PR == 0 && P == 4 && (NR == 8 || NR == 16);
};

// f.template with<S, PR, NR, P, LAY>() for a runtime layout.
template <int S, int PR, int NR, int P, class F>
int dispatch_layout(int layout, F& f)
{
    if (layout == 0) return f.template with<S, PR, NR, P, 0>();
    if constexpr (HasLayouts<S, PR, NR, P>::value) {
        switch (layout) {
        case 1: return f.template with<S, PR, NR, P, 1>();
        case 2: return f.template with<S, PR, NR, P, 2>();
        case 3: return f.template with<S, PR, NR, P, 3>();
        default: break;
        }
    }
    return (int)hipErrorInvalidValue;
}

// Visit the instantiation for runtime (scheme, precision, NR, P).  The direct
// scheme has no Taylor terms and is instantiated with P = 1 only.
template <int S, int PR, int NR, class F>
int dispatch_p(int terms, F& f)
{
    if constexpr (S == 0) {
        return f.template go<S, PR, NR, 1>();
    } else {
        switch (terms) {
        case 1: return f.template go<S, PR, NR, 1>();
        case 2: return f.template go<S, PR, NR, 2>();
        case 3: return f.template go<S, PR, NR, 3>();
        case 4: return f.template go<S, PR, NR, 4>();
        case 5: return f.template go<S, PR, NR, 5>();
        case 6: return f.template go<S, PR, NR, 6>();
        case 7: return f.template go<S, PR, NR, 7>();
        default: return (int)hipErrorInvalidValue;
        }
    }
}

// The centred sums run at most 8 rays per lane: with 16, their wider table
// rows and the change of deflection need more than the 128 VGPRs of four waves
// per SIMD.
template <int S, int PR, class F>
int dispatch_nr(int nr, int terms, F& f)
{
    switch (nr) {
    case 4: return dispatch_p<S, PR, 4>(terms, f);
    case 8: return dispatch_p<S, PR, 8>(terms, f);
    case 16:
        // the centred sums need more registers per ray: 16 rays per lane would
        // spill at 4 waves per SIMD, so they run 8
        if constexpr (PR == kPrecCentred)
            return dispatch_p<S, PR, 8>(terms, f);
        else
            return dispatch_p<S, PR, 16>(terms, f);
    default: return (int)hipErrorInvalidValue;
    }
}

struct MapLauncher {
    const LmDesc& d;
    hipStream_t s;
    template <int S, int PR, int NR, int P>
    int go() { return launch_map_t<S, PR, NR, P>(d, s); }
};

struct BatchLauncher {
    const LmDesc* descs;
    const int64_t* offs;
    const int32_t* order;
    int nmaps;
    unsigned long long* queue;
    int layout;
    int grid;
    hipStream_t s;
    template <int S, int PR, int NR, int P, int LAY>
    int with()
    {
        return launch_batch_t<S, PR, NR, P, LAY>(descs, offs, order, nmaps, queue, grid, s);
    }
    template <int S, int PR, int NR, int P>
    int go() { return dispatch_layout<S, PR, NR, P>(layout, *this); }
};

struct Occupancy {
    int layout;
    int* out;
    template <int S, int PR, int NR, int P, int LAY>
    int with()
    {
        return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(
            out, kernel_ptr_t<S, PR, NR, P, LAY>(), kWG, 0);
    }
    template <int S, int PR, int NR, int P>
    int go() { return dispatch_layout<S, PR, NR, P>(layout, *this); }
};
struct TraceLauncher {
    const LmDesc& d;
    const int64_t* ii;
    const int64_t* jj;
    int64_t n;
    int32_t* p;
    int32_t* q;
    double* uv;
    hipStream_t s;
    template <int S, int PR, int NR, int P>
    int go()
    {
        hipLaunchKernelGGL((k_trace<S, PR, P>), dim3((unsigned)((n + kWG - 1) / kWG)), dim3(kWG),
                           0, s, d, ii, jj, n, p, q, uv);
        return (int)hipGetLastError();
    }
};
struct DeflectLauncher {
    const LmDesc& d;
    const double* th;
    int64_t n;
    double* al;
    hipStream_t s;
    template <int S, int PR, int NR, int P>
    int go()
    {
        hipLaunchKernelGGL((k_deflect<S, PR, P>), dim3((unsigned)((n + kWG - 1) / kWG)), dim3(kWG),
                           0, s, d, th, n, al);
        return (int)hipGetLastError();
    }
};

}  // namespace
