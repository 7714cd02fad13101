// lm_internal.h -- layouts shared by the host code and the gfx950 kernels of
// liblensmap (not part of the public ABI).
#pragma once
#include <stdint.h>

#define LM_WG 256          // threads per workgroup: 4 waves of 64
#define LM_WAVES 4
#define LM_LENS_CAP 256    // direct sum: lenses staged per wave per block (the summation block)
// Kernel value of LM_PREC_MIXED_CENTRED: FP32 near sums of each near lens's
// deflection change from the level-2 cell centre, whose near-lens deflection
// is taken in FP64 (n0 below).
constexpr int kPrecCentred = 4;

// LDS layouts of the interpolated-scheme shooting kernels, the tuner's third
// axis besides rays per lane and tile size: lenses per LDS table block (the
// wave-shared dx^2, m dx table), uint32 bins of the workgroup's LDS window
// (the histogram tile), near lenses staged per wave per block.  With 16 rays
// per lane and FP32 sums each fits 40 KiB per workgroup (four per CU).  Layout
// 0 serves every kernel; the others are built for the FP32 rebased path with
// P = 4 and 8 or 16 rays per lane.  Results never depend on the layout.
#define LM_LAYOUTS 4
static constexpr int kLayTab[LM_LAYOUTS] = {16, 8, 32, 16};
static constexpr int kLayWin[LM_LAYOUTS] = {7040, 8064, 5000, 7552};
static constexpr int kLayNear[LM_LAYOUTS] = {64, 64, 64, 32};

// Table entries per (column, lens) of a precision's wave-shared LDS table: dx^2
// and m dx, or for the centred sums dx^2, c_r dx and c_i dx.
constexpr int tab_width(int prec) { return prec == kPrecCentred ? 3 : 2; }

// Window bins of a shooting kernel: the layout's, less what the wider table of
// the centred sums takes (rays_per_lane columns per lens and wave), so that
// the workgroup keeps to the layout's LDS budget.
constexpr int window_bins(int prec, int layout, int rays_per_lane)
{
    return kLayWin[layout] -
           (prec == kPrecCentred ? LM_WAVES * kLayTab[layout] * rays_per_lane : 0);
}
#define LM_PTAB_PAD 64     // column-offset table entries past R (last column group)
#define LM_PTAB_POW 6      // powers dx .. dx^6 per column (row polynomials, P <= 7)
#define LM_PTAB_ROWS 7     // and a row of dx sdx / sdy (the centred sums' y change)

// Allocation-free peak statistics: limits and layout of the per-device scratch
// array (tracks, column bins, two histograms; each part 256-byte aligned).
#define LM_SCRATCH_TRACKS 8192
#define LM_SCRATCH_COLS (1 << 20)
#define LM_SCRATCH_BINS 4096
#define LM_SCRATCH_OFF_BINOF (4 * LM_SCRATCH_TRACKS)
#define LM_SCRATCH_OFF_EDGES (LM_SCRATCH_OFF_BINOF + 4 * LM_SCRATCH_COLS)
#define LM_SCRATCH_OFF_HIST (LM_SCRATCH_OFF_EDGES + (8 * (LM_SCRATCH_BINS + 1) + 255) / 256 * 256)
#define LM_SCRATCH_BYTES (LM_SCRATCH_OFF_HIST + 16 * LM_SCRATCH_BINS)
#define LM_MAX_DEVICES 64

// Taylor coefficients of one level-2 cell: a_0 in FP64 (it carries the large
// far-field deflection of the cell centre), a_1..a_6 in FP32 (they multiply
// offsets of at most half a cell); and for the centred near sums the
// deflection of the cell centre by its near lenses, FP64, NaN when a near lens
// lies within twice the cell's half-diagonal of the centre.  80 bytes per cell.
struct LmCoef {
    double a0r, a0i;
    double n0x, n0y;
    float a[12];  // (re, im) of a_1 .. a_6
};

// Everything a kernel needs about one map and one shot rectangle.
struct LmDesc {
    // ray lattice and macro mapping (FP64)
    double x0, y0, dx, dy;
    double mx, my;                 // linear: 1-kappa-gamma+kappa_star, 1-kappa+gamma+kappa_star;
                                   // fold: kappa_star, 2(1-kappa0)+kappa_star
    double qx, qy;                 // fold: d_x/2, d_y (beta_x gains (qx theta_x + qy theta_y) theta_x)
    double bx0, by0, inv_sdx, inv_sdy;
    double sx0, sx1, sy0, sy1;     // rectangle of the -kappa_star sheet (sheet = 1)
    double kappa_star;
    // FP32 copies: half ray spacing as float-float (rebased arithmetic) and
    // plain values (the global-FP32 comparison path)
    float hxh, hxl, hyh, hyl;
    float x0f, y0f, dxf, dyf;
    float mxf, myf, bx0f, by0f;
    float inv_sdxf, inv_sdyf;
    int32_t snx, sny;
    int32_t fold;                  // 1: fold macro model
    int32_t sheet;                 // 1: the sheet covers [sx0, sx1] x [sy0, sy1]
    int32_t Q;                     // terms of the level-1 series (0: direct coefficients)
    int32_t nbx, nby;              // boxes of the level-1 series per level-1 cell side
    int32_t bx, by;                // level-2 cells per box side (the last box may be narrower)
    // scheme and work decomposition
    int32_t R, Kx, Ky, H;
    int32_t G;                     // level-2 cells per workgroup-tile side
    int32_t ncc;                   // column chunks per level-2 cell
    int32_t cw;                    // columns per chunk
    int32_t nrb;                   // 64-row blocks per level-2 cell (R / 64)
    int32_t wx, wy;                // LDS window (pixels)
    int32_t nl1x, nl1y;            // padded level-1 grid (N1 + 2H per side)
    int64_t n1x, n1y;              // level-1 cells holding level-2 cells of the lattice
    int64_t nx, ny;                // lattice
    int64_t i0, j0, i1, j1;        // shot rectangle [i0,i1) x [j0,j1)
    int64_t ncx, ncy;              // level-2 cells of the lattice
    int64_t tcx0, tcy0, ntx, nty;  // workgroup tiles covering the rectangle
    int64_t ntiles;
    int64_t tile0;                 // first tile of a k_shoot_map launch
    int64_t nlens;
    // lenses: sorted by level-1 cell for the interpolated scheme
    const double* lx;
    const double* ly;
    const double* lmd;
    const float* lxf;
    const float* lyf;
    const float* lmf;
    const int32_t* lI;             // level-1 cell of each lens (clamped)
    const int32_t* lJ;
    const int32_t* cell_start;     // CSR over the padded level-1 grid
    const LmCoef* coef;            // [ncy][ncx]
    const float* ptab;             // [LM_PTAB_ROWS][R + LM_PTAB_PAD] column offsets of a
                                   // level-2 cell and their powers
    double* l1exp;                 // [n1y nby][n1x nbx][Q] level-1 series per box, complex
    unsigned long long* counts;    // [sny][snx]
    unsigned long long* n_out;
};

// Launchers implemented in lm_kernels.hip (return hipError_t as int).
// The rectangle sheet's holomorphic part added to every level-2 cell's
// coefficients (after the far-field kernels).
int lm_launch_sheet(const LmDesc& d, int terms, LmCoef* coef, void* stream);
int lm_launch_ptab(const LmDesc& d, float* out, int n, void* stream);
int lm_launch_coeffs(const LmDesc& d, int precision, int terms, int64_t ci0, int64_t cj0,
                     int64_t nci, int64_t ncj, LmCoef* out, void* stream);
// Hierarchical far field: level-1 series (d.Q terms) into d.l1exp, then the
// coefficients of every level-2 cell.
int lm_launch_coeffs_hier(const LmDesc& d, int terms, LmCoef* out, void* stream);
// Near-lens deflection of every level-2 cell centre (LmCoef::n0x, n0y) for the
// centred near sums; the rest of each record is left as it is.
int lm_launch_near_centre(const LmDesc& d, LmCoef* out, void* stream);
int lm_launch_shoot_map(const LmDesc& d, int scheme, int precision, int terms, int rays_per_lane,
                        void* stream);
// layout: an LDS layout (above); LM_LAYOUTS pairs it is not built for give
// hipErrorInvalidValue
int lm_launch_shoot_batch(const LmDesc* descs, const int64_t* offsets, const int32_t* order,
                          int nmaps, unsigned long long* queue, int scheme, int precision,
                          int terms, int rays_per_lane, int layout, int grid, void* stream);
int lm_launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, void* stream);
int lm_launch_copy_region_u64(const unsigned long long* map, int64_t snx, int64_t p0, int64_t q0,
                              int64_t np, int64_t nq, unsigned long long* out, void* stream);
// *total (zeroed by the caller) += sum of p[0..n)
int lm_launch_sum_u64(const unsigned long long* p, int64_t n, unsigned long long* total,
                      void* stream);
// p, q: pixels (-1 outside the map); uv (may be null): continuous pixel
// coordinates, 2 per ray, that the pixels are the floor of
int lm_launch_trace(const LmDesc& d, int scheme, int precision, int terms, const int64_t* ii,
                    const int64_t* jj, int64_t n, int32_t* p, int32_t* q, double* uv,
                    void* stream);
int lm_launch_deflect(const LmDesc& d, int scheme, int precision, int terms, const double* th,
                      int64_t n, double* alpha, void* stream);
int lm_launch_peaks(const unsigned long long* counts, int64_t nx, int64_t ny,
                    const int32_t* tracks, int64_t nt, int k, uint8_t* flags, void* stream);
// bin_of[p] = b with edges[b] <= x0 + (p + 1/2) dx < edges[b+1] (FP64, multiply
// and add each rounded to nearest), -1 outside [edges[0], edges[nb])
int lm_launch_column_bins(double x0, double dx, int64_t nx, const double* edges, int nb,
                          int32_t* bin_of, void* stream);
// peaks[b] += true peaks of the listed rows in pixels j with bin_of[j] == b,
// heights[b] += their counts (bin_of[j] < 0: no bin)
int lm_launch_peak_bins(const unsigned long long* counts, int64_t nx, int64_t ny,
                        const int32_t* tracks, int64_t nt, int k, const int32_t* bin_of,
                        unsigned long long* peaks, unsigned long long* heights, void* stream);
int lm_shoot_occupancy(int scheme, int precision, int terms, int rays_per_lane, int layout,
                       int* wg_per_cu);
// Device address of the current device's scratch array (resolved once per
// device); returns a hipError_t.
int lm_scratch_address(void** out);
bool lm_supported_rays_per_lane(int r);

// Per-pair instances of the shooting kernels, probes and their launchers
// (lm_shoot_inst.hip, compiled once per (scheme, precision) pair).
#define LM_INST_CAT2(base, s, p) base##_s##s##_p##p
#define LM_INST_CAT(base, s, p) LM_INST_CAT2(base, s, p)
#define LM_INST_DECLARE(S, PR)                                                                \
    int LM_INST_CAT(lm_inst_shoot_map, S, PR)(const LmDesc& d, int nr, int terms, void* stream); \
    int LM_INST_CAT(lm_inst_shoot_batch, S, PR)(const LmDesc* descs, const int64_t* offs,     \
                                                const int32_t* order, int nmaps,              \
                                                unsigned long long* queue, int nr, int terms, \
                                                int layout, int grid, void* stream);          \
    int LM_INST_CAT(lm_inst_occupancy, S, PR)(int nr, int terms, int layout, int* wg_per_cu); \
    int LM_INST_CAT(lm_inst_trace, S, PR)(const LmDesc& d, int terms, const int64_t* ii,      \
                                          const int64_t* jj, int64_t n, int32_t* p,           \
                                          int32_t* q, double* uv, void* stream);              \
    int LM_INST_CAT(lm_inst_deflect, S, PR)(const LmDesc& d, int terms, const double* th,     \
                                            int64_t n, double* alpha, void* stream);
LM_INST_DECLARE(0, 0)
LM_INST_DECLARE(0, 1)
LM_INST_DECLARE(1, 0)
LM_INST_DECLARE(1, 1)
LM_INST_DECLARE(1, 2)
LM_INST_DECLARE(1, 4)
